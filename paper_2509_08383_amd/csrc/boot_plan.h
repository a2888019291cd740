// Host-side plan of the CKKS bootstrap: the slot decoding map as butterfly
// stages in the rotation-diagonal basis, their grouping into a few levels, the
// baby-step giant-step split of each group, the encoding of complex slot vectors
// and the Chebyshev interpolant of EvalMod.  Host math only (no HIP).
//
// Decoding map (CKKS canonical embedding): slot j of m holds m(zeta^{t_j}),
// t_j = 5^j mod 2N, zeta = e^{i pi / N}.  With w_k = m_k + i m_{k + N/2} (k < s =
// N/2) the slots are U w, U[j][k] = zeta^{t_j k}, and U = S_s ... S_4 S_2 P (P the
// bit reversal) where S_len acts on blocks of `len` slots: for j < len/2,
// (u_j, u_{j+len/2}) -> (u + xi_j v, u - xi_j v), xi_j = e^{2 pi i (5^j mod 4 len) / (4 len)}.
// A matrix M is held by its diagonals: M v = sum_d D_d * rot_d(v),
// rot_d(v)[t] = v[(t + d) mod s].
#pragma once

#include <complex>
#include <cstdint>
#include <functional>
#include <map>
#include <utility>
#include <vector>

namespace he {

using cplx = std::complex<double>;
using Diag = std::map<int, std::vector<cplx>>;  // offset (mod s) -> s entries

// one butterfly stage of half-length lenh (forward), or its inverse
Diag bt_stage(int s, int lenh, bool inverse);
// diagonals of A B (B applied first)
Diag bt_compose(const Diag &A, const Diag &B, int s);
// the log2(s) stages merged into n groups in application order: inverse (slots to
// coefficients, CoeffToSlot) S_s^-1 first .. S_2^-1 last; forward S_2 first .. S_s last
std::vector<Diag> bt_groups(int s, int n, bool inverse);

// offset d = (a B + b) h0, 0 <= b < B: sum_d D_d rot_d(v) =
// sum_a rot_{a B h0}( sum_b rot_{-a B h0}(D_d) * rot_{b h0}(v) )
struct Bsgs {
    int h0 = 1, B = 1;
    std::map<int, std::vector<std::pair<int, int>>> terms;  // giant a -> [(baby b, offset d)]
    std::vector<int> babies() const;                        // nonzero b, ascending
    std::vector<int> rotations(int s) const;                // amounts (mod s) used, ascending
};
Bsgs bsgs_plan(const Diag &D, int s);

// integer plaintext m (N coefficients) with m(zeta^{t_j}) ~ scale z_j and the
// conjugate at 2N - t_j; rounding half away from zero.  Throws if a coefficient
// reaches 2^62.
void encode_cplx(const std::vector<cplx> &z, int N, double scale, int64_t *m);

// Chebyshev interpolant of f on [-1, 1] at the deg + 1 Chebyshev points of the
// first kind: c_j = (2 / (deg + 1)) sum_k f(x_k) T_j(x_k), c_0 halved
std::vector<double> cheb_interp(const std::function<double(double)> &f, int deg);

}  // namespace he
