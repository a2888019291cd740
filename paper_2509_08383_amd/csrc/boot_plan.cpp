// Host-side plan of the CKKS bootstrap (see boot_plan.h for the factorisation).
#include "boot_plan.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>

namespace he {

namespace {

uint64_t pow_mod(uint64_t b, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    b %= m;
    for (; e; e >>= 1, b = (b * b) % m)
        if (e & 1) r = (r * b) % m;
    return r;
}

// xi_j of a block of length ln: e^{2 pi i (5^j mod 4 ln) / (4 ln)}
cplx xi(int j, int ln) {
    const uint64_t M = 4ull * (uint64_t)ln;
    const double ang = 2.0 * M_PI * (double)pow_mod(5, (uint64_t)j, M) / (double)M;
    return cplx(std::cos(ang), std::sin(ang));
}

void put(Diag &D, int s, int d, int t, cplx v) {
    const int k = ((d % s) + s) % s;
    auto it = D.find(k);
    if (it == D.end()) it = D.emplace(k, std::vector<cplx>(s, cplx(0.0, 0.0))).first;
    it->second[t] += v;
}

}  // namespace

Diag bt_stage(int s, int lenh, bool inverse) {
    const int ln = 2 * lenh;
    Diag D;
    for (int t = 0; t < s; ++t) {
        const int jj = t % ln;
        if (jj < lenh) {
            // out[t] = u + xi v  (inverse: (a + b) / 2)
            if (inverse) {
                put(D, s, 0, t, 0.5);
                put(D, s, lenh, t, 0.5);
            } else {
                put(D, s, 0, t, 1.0);
                put(D, s, lenh, t, xi(jj, ln));
            }
        } else {
            // out[t] = u - xi v  (inverse: conj(xi) (a - b) / 2, a at t - lenh)
            const cplx x = xi(jj - lenh, ln);
            if (inverse) {
                put(D, s, 0, t, -std::conj(x) * 0.5);
                put(D, s, -lenh, t, std::conj(x) * 0.5);
            } else {
                put(D, s, 0, t, -x);
                put(D, s, -lenh, t, 1.0);
            }
        }
    }
    return D;
}

Diag bt_compose(const Diag &A, const Diag &B, int s) {
    // (A B) v = sum_{e,f} A_e * rot_e(B_f) * rot_{e+f}(v)
    Diag out;
    for (const auto &ea : A)
        for (const auto &fb : B) {
            const int d = (ea.first + fb.first) % s;
            auto it = out.find(d);
            if (it == out.end()) it = out.emplace(d, std::vector<cplx>(s, cplx(0.0, 0.0))).first;
            std::vector<cplx> &o = it->second;
            const std::vector<cplx> &a = ea.second, &b = fb.second;
            for (int t = 0; t < s; ++t) o[t] += a[t] * b[(t + ea.first) % s];
        }
    return out;
}

std::vector<Diag> bt_groups(int s, int n, bool inverse) {
    int lg = 0;
    while ((1 << lg) < s) ++lg;
    if (n < 1 || n > lg) throw std::invalid_argument("bootstrap: group count must lie in [1, log2(slots)]");
    std::vector<int> lenh(lg);
    for (int i = 0; i < lg; ++i) lenh[i] = inverse ? s >> (i + 1) : 1 << i;
    std::vector<Diag> groups;
    int i = 0;
    for (int g = 0; g < n; ++g) {
        const int size = lg / n + (g < lg % n ? 1 : 0);
        Diag M;
        for (int k = 0; k < size; ++k, ++i) {
            Diag S = bt_stage(s, lenh[i], inverse);
            M = k == 0 ? std::move(S) : bt_compose(S, M, s);
        }
        groups.push_back(std::move(M));
    }
    return groups;
}

std::vector<int> Bsgs::babies() const {
    std::vector<int> b;
    for (const auto &a : terms)
        for (const auto &t : a.second)
            if (t.first) b.push_back(t.first);
    std::sort(b.begin(), b.end());
    b.erase(std::unique(b.begin(), b.end()), b.end());
    return b;
}

std::vector<int> Bsgs::rotations(int s) const {
    std::vector<int> r;
    for (int b : babies()) r.push_back((int)(((long long)b * h0) % s));
    for (const auto &a : terms)
        if (a.first) r.push_back((int)(((long long)a.first * B * h0) % s));
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    return r;
}

Bsgs bsgs_plan(const Diag &D, int s) {
    Bsgs P;
    int h0 = s;
    for (const auto &e : D)
        if (e.first) h0 = std::gcd(h0, e.first);
    P.h0 = h0;
    const int n = (int)D.size();
    int B = 1;
    while (B * B < n) B *= 2;
    P.B = B;
    for (const auto &e : D) {
        const int q = e.first / h0;
        P.terms[q / B].push_back({q % B, e.first});
    }
    return P;
}

void encode_cplx(const std::vector<cplx> &z, int N, double scale, int64_t *m) {
    // E[n] = value at zeta^{2n+1}; m_k = (1/N) zeta^{-k} sum_n E[n] e^{-2 pi i n k / N}
    const int s = N / 2;
    if ((int)z.size() != s) throw std::invalid_argument("encode: need N/2 slot values");
    std::vector<cplx> E(N, cplx(0.0, 0.0));
    const uint64_t M = 2ull * (uint64_t)N;
    uint64_t t = 1;
    for (int j = 0; j < s; ++j) {
        const cplx v = z[j] * scale;
        E[(t - 1) / 2] = v;
        E[(M - t - 1) / 2] = std::conj(v);
        t = (t * 5) % M;
    }
    // iterative radix-2 forward DFT (bit reversal, then butterflies)
    int lg = 0;
    while ((1 << lg) < N) ++lg;
    for (int i = 0; i < N; ++i) {
        int r = 0;
        for (int b = 0; b < lg; ++b)
            if ((i >> b) & 1) r |= 1 << (lg - 1 - b);
        if (r > i) std::swap(E[i], E[r]);
    }
    std::vector<cplx> w(N / 2);
    for (int k = 0; k < N / 2; ++k) {
        const double a = -2.0 * M_PI * (double)k / (double)N;
        w[k] = cplx(std::cos(a), std::sin(a));
    }
    for (int len = 2; len <= N; len <<= 1) {
        const int half = len / 2, step = N / len;
        for (int b = 0; b < N; b += len)
            for (int k = 0; k < half; ++k) {
                const cplx u = E[b + k], v = E[b + k + half] * w[k * step];
                E[b + k] = u + v;
                E[b + k + half] = u - v;
            }
    }
    for (int k = 0; k < N; ++k) {
        const double a = -M_PI * (double)k / (double)N;
        const double v = (E[k] * cplx(std::cos(a), std::sin(a))).real() / (double)N;
        if (!(std::fabs(v) < 4.611686018427387904e18)) throw std::range_error("plaintext does not fit 64 bits");
        m[k] = std::llround(v);
    }
}

std::vector<double> cheb_interp(const std::function<double(double)> &f, int deg) {
    const int n = deg + 1;
    std::vector<double> fx(n), c(n, 0.0);
    for (int k = 0; k < n; ++k) fx[k] = f(std::cos(M_PI * (k + 0.5) / n));
    for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += fx[k] * std::cos(j * M_PI * (k + 0.5) / n);
        c[j] = acc * (j == 0 ? 1.0 : 2.0) / n;
    }
    return c;
}

}  // namespace he
