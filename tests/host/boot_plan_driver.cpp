// Prints the library's host-side bootstrap plan (butterfly groups as diagonals, the
// baby-step giant-step split, the complex encoder, the Chebyshev interpolant) for a
// CPU test that compares it with the oracle's independent Python plan.
// Usage: boot_plan_driver <slots> <groups> <inverse 0|1>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "../../paper_2509_08383_amd/csrc/boot_plan.h"

using namespace he;

int main(int argc, char **argv) {
    if (argc != 4) return 2;
    const int s = std::atoi(argv[1]), n = std::atoi(argv[2]), inv = std::atoi(argv[3]);
    const auto G = bt_groups(s, n, inv != 0);
    for (size_t g = 0; g < G.size(); ++g) {
        const auto P = bsgs_plan(G[g], s);
        std::printf("G %zu %zu %d %d\n", g, G[g].size(), P.h0, P.B);
        for (const auto &e : G[g]) {
            std::printf("D %d", e.first);
            for (int t = 0; t < s; ++t) std::printf(" %.17g %.17g", e.second[t].real(), e.second[t].imag());
            std::printf("\n");
        }
        std::printf("R");
        for (int r : P.rotations(s)) std::printf(" %d", r);
        std::printf("\n");
    }
    const int N = 2 * s;
    std::vector<cplx> z(s);
    for (int i = 0; i < s; ++i) z[i] = cplx(std::sin(i * 0.37), std::cos(i * 1.3));
    std::vector<int64_t> m(N);
    encode_cplx(z, N, 1099511627776.0, m.data());
    std::printf("M");
    for (auto v : m) std::printf(" %lld", (long long)v);
    std::printf("\n");
    const auto c = cheb_interp([](double x) { return std::cos(3 * std::sqrt(std::max(0.0, (1 + x) / 2))); }, 31);
    std::printf("C");
    for (double v : c) std::printf(" %.17g", v);
    std::printf("\n");
    return 0;
}
