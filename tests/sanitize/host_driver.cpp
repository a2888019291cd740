// Drives the library's host-side math (csrc/host_math.cpp: prime chain, Philox, secret,
// slot encoding, inverse-square-root guess and scaled plan; csrc/boot_plan.cpp: the
// bootstrap's butterfly diagonals, their grouping, baby-step giant-step split, complex
// encoding and Chebyshev interpolation; csrc/mlp_file.cpp: the learned guess's collapse
// and file form), built with AddressSanitizer and
// UndefinedBehaviorSanitizer (LeakSanitizer at exit) by tests/test_sanitizers.py.
// Cheap identities are checked on the way; a sanitizer report or a failed check gives a
// non-zero status.
#include <cmath>
#include <complex>
#include <cstdio>
#include <stdexcept>
#include <vector>

#include "boot_plan.h"
#include "he_internal.h"
#include "mlp_file.h"

static int fails = 0;
#define CHECK(c, msg) do { if (!(c)) { std::fprintf(stderr, "check failed: %s\n", msg); ++fails; } } while (0)

int main() {
    using namespace he;
    // modular helpers and the prime chain (secure-size shape: 30 Q primes, 10 P primes)
    for (int logN : {12, 16}) {
        const int n_q = logN == 16 ? 30 : 8, alpha = (n_q + 2) / 3;
        std::vector<uint64_t> P = gen_primes(logN, n_q, 48, 40, 48, alpha);
        CHECK((int)P.size() == n_q + alpha, "prime count");
        for (uint64_t p : P) {
            CHECK(miller_rabin(p), "prime");
            CHECK(p % (2ull << logN) == 1, "NTT-friendly");
            const uint64_t psi = find_psi(p, 1 << logN);
            CHECK(powmod_u(psi, 1ull << logN, p) == p - 1, "psi^N = -1");
            CHECK(mulmod_u(invmod_u(psi, p), psi, p) == 1, "inverse");
            CHECK(red_i64(-1, p) == p - 1 && red_i64(INT64_MIN, p) < p, "signed reduction");
        }
    }
    std::vector<uint64_t> H = gen_primes(12, 10, 48, 40, 48, 4, 3, 44);
    CHECK(H.size() == 14, "chain with wider top primes");
    uint32_t o[4];
    philox_host(0, 0, 0, 0, 0, o);
    philox_host(0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu, ~0ull, o);
    std::vector<int> s = sparse_secret(1 << 12, 64, 11, 7);
    int nz = 0;
    for (int v : s) nz += v != 0;
    CHECK(nz == 64, "sparse secret weight");
    // slot encoding round trip at N = 2^12
    const int N = 1 << 12;
    std::vector<double> z(N / 2), back(N / 2), md(N);
    for (int i = 0; i < N / 2; ++i) z[i] = std::sin(0.37 * i) * 3.0;
    std::vector<int64_t> m(N);
    encode_slots(z.data(), N, std::ldexp(1.0, 40), m.data());
    for (int i = 0; i < N; ++i) md[i] = (double)m[i];
    decode_slots(md.data(), N, std::ldexp(1.0, 40), back.data());
    double e = 0;
    for (int i = 0; i < N / 2; ++i) e = std::fmax(e, std::fabs(back[i] - z[i]));
    CHECK(e < 1e-9, "encode/decode");
    CHECK(llround_d(-2.5) == -3 && llround_d(2.5) == 3, "rounding half away from zero");
    // inverse square root guess and the scaled plan, over degrees and step counts
    for (int d = 1; d <= 4; ++d) {
        double c[5];
        chebyshev_invsqrt_fit(0.05, d, c);
        double g = 0;
        for (int k = d; k >= 0; --k) g = g * 0.5 + c[k];
        CHECK(std::fabs(g * std::sqrt(0.5) - 1.0) < 0.3, "guess near u^(-1/2)");
        for (int K : {0, 1, 7, 16}) {
            double cf[5], st[32], rg[34];
            CHECK(invsqrt_scaled_plan(2.5e-6, d, K, cf, st, rg), "scaled plan");
            CHECK(rg[2 * K] > 0 && rg[2 * K] <= rg[2 * K + 1] && rg[2 * K + 1] < 2.0, "plan range");
        }
    }
    // bootstrap planning at 2^10 slots: three groups each way, their BSGS split, the
    // complex encoding of a diagonal, and EvalMod's interpolant
    const int slots = 1 << 10, NN = 2 * slots;
    for (bool inv : {false, true}) {
        std::vector<Diag> G = bt_groups(slots, 3, inv);
        CHECK(G.size() == 3, "groups");
        for (const Diag &D : G) {
            Bsgs B = bsgs_plan(D, slots);
            CHECK(!B.rotations(slots).empty() || D.size() == 1, "rotations");
            std::vector<int64_t> pm(NN);
            encode_cplx(D.begin()->second, NN, std::ldexp(1.0, 30), pm.data());
        }
    }
    Diag A = bt_stage(slots, 4, false), Ai = bt_stage(slots, 4, true);
    Diag I = bt_compose(Ai, A, slots);
    double off = 0;
    for (auto &kv : I)
        for (size_t t = 0; t < kv.second.size(); ++t)
            off = std::fmax(off, std::abs(kv.second[t] - (kv.first == 0 ? cplx(1.0, 0.0) : cplx(0.0, 0.0))));
    CHECK(off < 1e-12, "stage^-1 stage = identity");
    std::vector<double> ch = cheb_interp([](double x) { return std::sin(6.0 * x); }, 31);
    CHECK(ch.size() == 32, "interpolant length");
    bool threw = false;
    try {
        std::vector<cplx> big(slots, cplx(1e30, 0.0));
        std::vector<int64_t> pm(NN);
        encode_cplx(big, NN, 1.0, pm.data());
    } catch (const std::exception &) {
        threw = true;
    }
    CHECK(threw, "oversized encoding throws");
    // learned-guess file: write, read back, refuse a corrupted copy and a missing file
    {
        std::vector<float> th(kMlpParams);
        for (int i = 0; i < kMlpParams; ++i) th[i] = 0.1f * (float)std::sin(1.3 * i);
        const char *path = "host_driver_mlp.bin";
        std::string err;
        CHECK(mlp_file_write(path, th.data(), 0.4f, 0.3f, &err) == 0, "mlp file write");
        std::vector<float> back(kMlpParams);
        float mean = 0, sd = 0;
        double poly[5], want[5];
        CHECK(mlp_file_read(path, back.data(), &mean, &sd, poly, &err) == 0, "mlp file read");
        mlp_poly(th.data(), 0.4f, 0.3f, want);
        bool same = mean == 0.4f && sd == 0.3f;
        for (int i = 0; i < kMlpParams; ++i) same = same && back[i] == th[i];
        for (int d = 0; d < 5; ++d) same = same && poly[d] == want[d];
        CHECK(same, "mlp file round trip");
        FILE *f = std::fopen(path, "r+b");
        if (f) {
            std::fseek(f, 100, SEEK_SET);
            std::fputc(0x5a, f);
            std::fclose(f);
        }
        CHECK(mlp_file_read(path, nullptr, nullptr, nullptr, poly, &err) != 0, "corrupted file refused");
        std::remove(path);
        CHECK(mlp_file_read(path, nullptr, nullptr, nullptr, poly, &err) != 0, "missing file refused");
    }
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("host driver: ok\n");
    return 0;
}
