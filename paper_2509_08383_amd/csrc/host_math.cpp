// Host-side number theory and encoding for the MI355X CKKS library.
#include <algorithm>
#include <cmath>
#include <complex>
#include <stdexcept>
#include <vector>

#include "he_internal.h"

namespace he {

using u128 = unsigned __int128;

uint64_t mulmod_u(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

uint64_t powmod_u(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod_u(r, a, q);
        a = mulmod_u(a, a, q);
        e >>= 1;
    }
    return r;
}

uint64_t invmod_u(uint64_t a, uint64_t q) { return powmod_u(a % q, q - 2, q); }

uint64_t red_i64(int64_t v, uint64_t q) {
    int64_t r = v % (int64_t)q;
    if (r < 0) r += (int64_t)q;
    return (uint64_t)r;
}

bool miller_rabin(uint64_t n) {
    static const uint64_t W[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (uint64_t w : W) {
        if (n == w) return true;
        if (n % w == 0) return false;
    }
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) { d >>= 1; ++s; }
    for (uint64_t w : W) {
        uint64_t x = powmod_u(w, d, n);
        if (x == 1 || x == n - 1) continue;
        bool composite = true;
        for (int i = 1; i < s && composite; ++i) {
            x = mulmod_u(x, x, n);
            if (x == n - 1) composite = false;
        }
        if (composite) return false;
    }
    return true;
}

// Primes 2^b - k*2N + 1 (k = 1, 2, ...), first unused prime per slot, in the
// order q0, q1..q_{n_q-1}, p0..p_{alpha-1}.
std::vector<uint64_t> gen_primes(int logN, int n_q, int q0_bits, int q_bits, int p_bits, int alpha, int n_hi,
                                 int hi_bits) {
    const uint64_t M = 2ull << logN;
    std::vector<uint64_t> out;
    auto next = [&](int bits) {
        for (uint64_t k = 1;; ++k) {
            const uint64_t c = (1ull << bits) - k * M + 1;
            if (c < (1ull << (bits - 1))) throw std::runtime_error("prime search exhausted");
            bool used = false;
            for (uint64_t u : out) used |= (u == c);
            if (!used && miller_rabin(c)) return c;
        }
    };
    out.push_back(next(q0_bits));
    // the top n_hi Q primes (the levels a bootstrap consumes first) have hi_bits bits
    for (int i = 1; i < n_q; ++i) out.push_back(next(i >= n_q - n_hi ? hi_bits : q_bits));
    for (int i = 0; i < alpha; ++i) out.push_back(next(p_bits));
    return out;
}

// a primitive 2N-th root of unity: g^((q-1)/2N) for the smallest g >= 2 whose
// power has order exactly 2N (psi^N = -1)
uint64_t find_psi(uint64_t q, int N) {
    const uint64_t M = 2ull * N;
    for (uint64_t g = 2;; ++g) {
        const uint64_t psi = powmod_u(g, (q - 1) / M, q);
        if (powmod_u(psi, (uint64_t)N, q) == q - 1) return psi;
    }
}

int64_t llround_d(double x) { return std::llround(x); }

// Philox4x32-10 (Salmon et al., SC 2011) on the host; the same counter layout as the
// device sampler: (i, prime, obj, attempt), key (seed low, seed high)
void philox_host(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed, uint32_t out[4]) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        const uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// sparse ternary secret with exactly hw nonzero coefficients: the i-th is placed at
// word 0 mod N of draw (i, 0, obj, attempt), attempt = 0, 1, .. until that position
// is still free; its sign is - when word 1 is odd
std::vector<int> sparse_secret(int N, int hw, uint64_t seed, uint32_t obj) {
    if (hw < 0 || hw > N) throw std::invalid_argument("secret weight out of range");
    std::vector<int> s(N, 0);
    for (int i = 0; i < hw; ++i)
        for (uint32_t att = 0;; ++att) {
            uint32_t o[4];
            philox_host((uint32_t)i, 0u, obj, att, seed, o);
            const int pos = (int)(o[0] & (uint32_t)(N - 1));
            if (s[pos]) continue;
            s[pos] = (o[1] & 1u) ? -1 : 1;
            break;
        }
    return s;
}

// ------------------------------------------------------------------ encoding
// Slot j <-> zeta^(t_j), t_j = 5^j mod 2N, zeta = e^{i pi / N}.  The N odd
// powers zeta^(2k+1) are reached by a length-N DFT of (m_i zeta^i); encoding
// inverts it with the conjugate slots filled in (real messages).
namespace {
using cd = std::complex<double>;

void fft_inplace(std::vector<cd> &a, bool invert) {
    const int n = (int)a.size();
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (int len = 2; len <= n; len <<= 1) {
        const double ang = 2.0 * M_PI / len * (invert ? -1.0 : 1.0);
        std::vector<cd> w(len / 2);
        for (int k = 0; k < len / 2; ++k) w[k] = cd(std::cos(ang * k), std::sin(ang * k));
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < len / 2; ++k) {
                const cd u = a[i + k], v = a[i + k + len / 2] * w[k];
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
    }
}
}  // namespace

void encode_slots(const double *z, int N, double scale, int64_t *m) {
    std::vector<cd> E(N, cd(0, 0));
    uint64_t t = 1;
    const uint64_t M = 2ull * N;
    for (int j = 0; j < N / 2; ++j) {
        const double v = z[j] * scale;
        E[(t - 1) / 2] = cd(v, 0);
        E[(M - t - 1) / 2] = cd(v, 0);
        t = (t * 5) % M;
    }
    // m_i zeta^i = (1/N) sum_k E_k omega^(-ik)
    fft_inplace(E, true);
    for (int i = 0; i < N; ++i) {
        const double ang = -M_PI * i / N;
        const cd v = E[i] / (double)N * cd(std::cos(ang), std::sin(ang));
        m[i] = std::llround(v.real());
    }
}

void decode_slots(const double *m, int N, double scale, double *z) {
    std::vector<cd> a(N);
    for (int i = 0; i < N; ++i) {
        const double ang = M_PI * i / N;
        a[i] = m[i] * cd(std::cos(ang), std::sin(ang));
    }
    fft_inplace(a, false);  // a_k = m(zeta^(2k+1))
    uint64_t t = 1;
    const uint64_t M = 2ull * N;
    for (int j = 0; j < N / 2; ++j) {
        z[j] = a[(t - 1) / 2].real() / scale;
        t = (t * 5) % M;
    }
}

// Power-basis coefficients of the polynomial interpolating u^(-1/2) at the
// degree+1 Chebyshev nodes of the first kind on [u_lo, 1] (Gaussian
// elimination with partial pivoting on the Vandermonde system).
void chebyshev_invsqrt_fit(double u_lo, int degree, double *coef) {
    const int n = degree + 1;
    std::vector<double> A(n * n), b(n);
    for (int k = 0; k < n; ++k) {
        const double t = std::cos(M_PI * (k + 0.5) / n);
        const double u = 0.5 * (1.0 + u_lo) + 0.5 * (1.0 - u_lo) * t;
        double pw = 1.0;
        for (int j = 0; j < n; ++j) { A[k * n + j] = pw; pw *= u; }
        b[k] = 1.0 / std::sqrt(u);
    }
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (piv != c) {
            for (int j = 0; j < n; ++j) std::swap(A[c * n + j], A[piv * n + j]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = A[r * n + c] / A[c * n + c];
            for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
            b[r] -= f * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double s = b[c];
        for (int j = c + 1; j < n; ++j) s -= A[c * n + j] * coef[j];
        coef[c] = s / A[c * n + c];
    }
}

// Wide-domain inverse square root on [u_lo, 1]: the Chebyshev guess, the range of
// x = g(u) sqrt(u) over a geometric grid (widened by 1e-3 relative; the range only picks
// the refinement constants and the bootstrap bounds), then K refinements
// x <- x (a - b x^2), each the cubic that maps the range [l, h] it receives onto
// [1 - e, 1 + e] touching both ends and its maximum: a = b s, s = h^2 + h l + l^2,
// b = 2 / (l h (h + l) + 2 (s / 3)^(3/2)), e = 1 - b l h (h + l).
// Returns false when the guess is not positive on the domain.
bool invsqrt_scaled_plan(double u_lo, int degree, int K, double *coef, double *steps, double *ranges) {
    chebyshev_invsqrt_fit(u_lo, degree, coef);
    const int pts = 20001;
    double lo = 1e300, hi = -1e300;
    const double r = std::log(1.0 / u_lo);
    for (int i = 0; i < pts; ++i) {
        const double u = i == pts - 1 ? 1.0 : u_lo * std::exp(r * i / (pts - 1));
        double y = 0.0;
        for (int k = degree; k >= 0; --k) y = y * u + coef[k];
        const double x = y * std::sqrt(u);
        lo = std::min(lo, x);
        hi = std::max(hi, x);
    }
    if (!(lo > 0.0)) return false;
    lo *= 1.0 - 1e-3;
    hi *= 1.0 + 1e-3;
    ranges[0] = lo;
    ranges[1] = hi;
    for (int k = 0; k < K; ++k) {
        const double s2 = hi * hi + hi * lo + lo * lo;
        const double b = 2.0 / (lo * hi * (hi + lo) + 2.0 * std::pow(s2 / 3.0, 1.5));
        const double a = b * s2;
        const double e = 1.0 - b * lo * hi * (hi + lo);
        steps[2 * k] = a;
        steps[2 * k + 1] = b;
        lo = 1.0 - e;
        hi = 1.0 + e;
        ranges[2 * k + 2] = lo;
        ranges[2 * k + 3] = hi;
    }
    return true;
}

}  // namespace he
