"""CKKS bootstrapping on the CPU oracle -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg may
import this module.  It shares no code with the HIP path.

The paper runs its deeper CutMax schedules (T = 4, p up to 16, its Sec. 4 and
Table 2) with bootstrapping between iterations and counts the levels that the
inverse square root and inverse consume because depth decides how often a
bootstrap is needed (App. B.1).  A bootstrap takes a ciphertext whose levels are
spent back to a high level; here it is the standard CKKS procedure, written from
its definition:

  1. ModRaise: the level-0 residues mod q_0, centred and reduced modulo the whole
     chain, decrypt to m + q_0 I for a small integer polynomial I.
  2. CoeffToSlot: the inverse of the slot decoding map, as the stages of the
     special FFT (below), so that the slots hold the coefficients of m + q_0 I
     (divided by q_0 B, B the bound of I plus one half); one conjugation splits the
     complex slots w_k = c_k + i c_{k + N/2} into two real ciphertexts.
  3. EvalMod: x -> sin(2 pi x) / (2 pi), which removes the integer part and keeps
     m / q_0 (m / q_0 is small), evaluated as cos(2 pi (x - 1/4) / 2^r) by a
     Chebyshev interpolant followed by r double-angle steps cos 2t = 2 cos^2 t - 1.
  4. SlotToCoeff: the decoding map again, which puts the (scaled) coefficients back.

Decoding map: slot j of a plaintext m holds m(zeta^{t_j}), t_j = 5^j mod 2N,
zeta = exp(i pi / N).  Because zeta^{t_j N/2} = i, the slots are U w with
w_k = m_k + i m_{k + N/2} (k < s = N/2) and U[j][k] = zeta^{t_j k}.  U factors as
U = S_s ... S_4 S_2 P with P the bit reversal and S_len a butterfly stage: for a
block of `len` entries and j < len/2, (u, v) -> (u + xi_j v, u - xi_j v) with
xi_j = exp(2 pi i (5^j mod 4 len) / (4 len)).  A stage is three diagonals in the
rotation basis (M v = sum_d D_d * rot_d(v), rot_d(v)[t] = v[t + d]), so a group
of consecutive stages costs few rotations, found baby-step giant-step.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

from . import ckks

Diag = Dict[int, np.ndarray]


# ----------------------------------------------------------------------------
# the decoding map and its butterfly factorisation
# ----------------------------------------------------------------------------
def decode_matrix(N: int) -> np.ndarray:
    """U[j][k] = zeta^{t_j k}: slots of m from w_k = m_k + i m_{k+N/2} (small N)."""
    s = N // 2
    t = ckks.slot_exponents(N)
    k = np.arange(s)
    return np.exp(1j * np.pi * (np.outer(t, k) % (2 * N)) / N)


def bitrev_perm(s: int) -> np.ndarray:
    lg = s.bit_length() - 1
    out = np.zeros(s, dtype=np.int64)
    for i in range(s):
        r = 0
        for b in range(lg):
            if (i >> b) & 1:
                r |= 1 << (lg - 1 - b)
        out[i] = r
    return out


def stage(s: int, lenh: int, inverse: bool) -> Diag:
    """Diagonals of the butterfly stage of half-length lenh (or of its inverse)."""
    ln = 2 * lenh
    D: Diag = {}

    def put(d, t, v):
        D.setdefault(d % s, np.zeros(s, dtype=np.complex128))[t] += v

    for t in range(s):
        jj = t % ln
        if jj < lenh:
            xi = np.exp(2j * np.pi * pow(5, jj, 4 * ln) / (4 * ln))
            if inverse:
                put(0, t, 0.5)
                put(lenh, t, 0.5)
            else:
                put(0, t, 1.0)
                put(lenh, t, xi)
        else:
            xi = np.exp(2j * np.pi * pow(5, jj - lenh, 4 * ln) / (4 * ln))
            if inverse:
                put(0, t, -np.conj(xi) / 2)
                put(-lenh, t, np.conj(xi) / 2)
            else:
                put(0, t, -xi)
                put(-lenh, t, 1.0)
    return D


def compose(A: Diag, B: Diag, s: int) -> Diag:
    """Diagonals of A B (B applied first): (AB)_{e+f}[t] += A_e[t] B_f[t + e]."""
    out: Diag = {}
    for e, a in A.items():
        for f, b in B.items():
            d = (e + f) % s
            out[d] = out.get(d, 0) + a * np.roll(b, -e)
    return out


def apply_diag(D: Diag, v: np.ndarray) -> np.ndarray:
    """M v = sum_d D_d * rot_d(v) on a plain vector (pins and plaintext checks)."""
    out = np.zeros(v.size, dtype=np.complex128)
    for d, a in D.items():
        out += a * np.roll(v, -d)
    return out


def group_sizes(lg: int, n: int) -> List[int]:
    return [lg // n + (1 if i < lg % n else 0) for i in range(n)]


def stage_groups(s: int, n: int, inverse: bool) -> List[Diag]:
    """CoeffToSlot (inverse): stages S_s^-1 first .. S_2^-1 last; SlotToCoeff: S_2
    first .. S_s last; consecutive stages merged into n groups, in application order."""
    lg = s.bit_length() - 1
    lenhs = [s >> (i + 1) for i in range(lg)] if inverse else [1 << i for i in range(lg)]
    groups, i = [], 0
    for size in group_sizes(lg, n):
        M = None
        for lenh in lenhs[i:i + size]:
            S = stage(s, lenh, inverse)
            M = S if M is None else compose(S, M, s)
        groups.append(M)
        i += size
    return groups


# ----------------------------------------------------------------------------
# baby-step giant-step plan of one group
# ----------------------------------------------------------------------------
@dataclass
class Bsgs:
    h0: int                       # every offset is a multiple of h0
    B: int                        # baby steps 0 .. B-1 (times h0)
    terms: Dict[int, List[Tuple[int, int]]]   # giant a -> [(b, offset d)]

    @property
    def babies(self) -> List[int]:
        return sorted({b for ts in self.terms.values() for b, _ in ts if b})

    def rotations(self, s: int) -> List[int]:
        """rotation amounts (mod s) the group uses"""
        amts = {(b * self.h0) % s for b in self.babies}
        amts |= {(a * self.B * self.h0) % s for a in self.terms if a}
        return sorted(amts)


def bsgs_plan(D: Diag, s: int) -> Bsgs:
    """Offset d = (a B + b) h0 with 0 <= b < B: sum_d D_d rot_d(v) =
    sum_a rot_{a B h0}( sum_b rot_{-a B h0}(D_d) * rot_{b h0}(v) ).  h0 is the
    largest power of two dividing every offset (and s); B is the smallest power of
    two with B^2 >= the number of offsets."""
    offs = sorted(D)
    h0 = s
    for d in offs:
        if d:
            h0 = math.gcd(h0, d)
    n = len(offs)
    B = 1
    while B * B < n:
        B *= 2
    terms: Dict[int, List[Tuple[int, int]]] = {}
    for d in offs:
        e = d // h0
        terms.setdefault(e // B, []).append((e % B, d))
    return Bsgs(h0, B, terms)


@dataclass(frozen=True)
class BootCfg:
    n_cts: int = 3         # CoeffToSlot levels
    n_stc: int = 3         # SlotToCoeff levels
    K: int = 0             # bound of |I|; 0: ceil(6 sqrt(h / 12))
    ratio_bits: int = 12   # the message enters at scale q_0 2^-ratio_bits / bound
    cheb_deg: int = 31     # degree of the interpolant in z = 2 y^2 - 1 (62 in y)
    r: int = 3             # double-angle steps
    s_eval: float = 2.0 ** 48  # scale of the EvalMod ciphertexts

    def k_bound(self, h: int) -> int:
        return self.K if self.K > 0 else int(math.ceil(6.0 * math.sqrt(h / 12.0)))


def levels_used(cfg: BootCfg) -> int:
    """levels a bootstrap consumes above the output: CoeffToSlot, EvalMod (1 for
    z, ceil(log2(deg + 1)) for the Chebyshev basis, 1 for its coefficients, r
    double angles), SlotToCoeff"""
    return cfg.n_cts + 1 + int(math.ceil(math.log2(cfg.cheb_deg + 1))) + 1 + cfg.r + cfg.n_stc


def boot_rotations(s: int, cfg: BootCfg) -> List[int]:
    """every rotation amount (mod s) of the two linear transforms, ascending"""
    amts = set()
    for inverse, n in ((True, cfg.n_cts), (False, cfg.n_stc)):
        for D in stage_groups(s, n, inverse):
            amts |= set(bsgs_plan(D, s).rotations(s))
    amts.discard(0)
    return sorted(amts)


def boot_keys(O: "ckks.Oracle", cfg: BootCfg) -> Dict[int, int]:
    """Key index of every Galois element a bootstrap needs: rotation amounts that
    already have a CutMax key keep it; the others follow in ascending order from the
    first free index, and the conjugation (Galois 2N - 1) comes last."""
    s, M = O.slots, 2 * O.N
    have = ckks.rotation_keys(s, O.prm.hoist) if O.prm.hoist >= 1 else \
        {1 << e: 1 + e for e in range(int(math.log2(s)))}
    nxt = max(have.values()) + 1
    gal = {}
    for a in boot_rotations(s, cfg):
        if a in have:
            gal[pow(5, a, M)] = have[a]
        else:
            gal[pow(5, a, M)] = nxt
            nxt += 1
    gal[M - 1] = nxt
    return gal


def keygen_boot(O: "ckks.Oracle", cfg: BootCfg) -> Dict[int, int]:
    keys = boot_keys(O, cfg)
    for g, k in keys.items():
        O.keygen_galois(k, g)
    return keys


# ----------------------------------------------------------------------------
# encoding of complex slot vectors
# ----------------------------------------------------------------------------
def round_half_away(x: np.ndarray) -> np.ndarray:
    return np.where(x >= 0, np.floor(x + 0.5), np.ceil(x - 0.5))


def encode_complex(z: np.ndarray, N: int, scale: float) -> np.ndarray:
    """integer m with m(zeta^{t_j}) ~ scale z_j (and the conjugate at -t_j)"""
    t = ckks.slot_exponents(N)
    E = np.zeros(N, dtype=np.complex128)
    zz = np.asarray(z, dtype=np.complex128) * scale
    E[(t - 1) // 2] = zz
    E[(2 * N - t - 1) // 2] = np.conj(zz)
    i = np.arange(N)
    v = (np.fft.fft(E) / N * np.exp(-1j * np.pi * i / N)).real
    if np.abs(v).max() >= 2.0 ** 62:
        raise ckks.SchedError("plaintext does not fit 64 bits")
    return round_half_away(v).astype(np.int64)


def decode_complex(m: np.ndarray, N: int, scale: float) -> np.ndarray:
    ev = ckks._eval_all_odd(m, N)
    t = ckks.slot_exponents(N)
    return ev[(t - 1) // 2] / scale


# ----------------------------------------------------------------------------
# homomorphic pieces
# ----------------------------------------------------------------------------
def linear_transform(O: "ckks.Oracle", ct: "ckks.Ct", D: Diag, rho: float, keys: Dict[int, int]) -> "ckks.Ct":
    """sum_d D_d * rot_d(ct), baby-step giant-step, the diagonals encoded at scale
    rho q_l (l the ciphertext's level), one rescale: output scale = scale * rho."""
    s, M = O.slots, 2 * O.N
    plan = bsgs_plan(D, s)
    l = ct.level
    pscale = rho * float(O.q[l])
    baby = {0: ct}
    for b in plan.babies:
        a = (b * plan.h0) % s
        baby[b] = O.rotate_gal(ct, keys[pow(5, a, M)], pow(5, a, M))
    acc = None
    for a in sorted(plan.terms):
        shift = (a * plan.B * plan.h0) % s
        inner = None
        for b, d in plan.terms[a]:
            pt = encode_complex(np.roll(D[d], shift), O.N, pscale)
            t = O.mul_plain(baby[b], pt, pscale)
            inner = t if inner is None else O.add(inner, t)
        if shift:
            inner = O.rotate_gal(inner, keys[pow(5, shift, M)], pow(5, shift, M))
        acc = inner if acc is None else O.add(acc, inner)
    return O.rescale(acc)


def monomial(N: int, k: int, sign: int = 1) -> np.ndarray:
    m = np.zeros(N, dtype=np.int64)
    m[k] = sign
    return m


def cheb_coeffs(f, deg: int) -> np.ndarray:
    """Chebyshev interpolant of f on [-1, 1] at the deg + 1 Chebyshev points"""
    return np.polynomial.chebyshev.chebinterpolate(f, deg)


def eval_mod_coeffs(cfg: BootCfg, Bk: float) -> np.ndarray:
    """g(z) = cos(2 pi Bk y / 2^r) with y^2 = (1 + z) / 2"""
    a = 2.0 * math.pi * Bk / 2.0 ** cfg.r
    return cheb_coeffs(lambda z: np.cos(a * np.sqrt(np.maximum(0.0, (1.0 + z) / 2.0))), cfg.cheb_deg)


def match(O: "ckks.Oracle", x: "ckks.Ct", level: int, scale: float) -> "ckks.Ct":
    """x brought to `level` and (declared) `scale` through one constant product"""
    y = O.cm_target(x, 1.0, scale)
    return O.drop(y, level)


def chebyshev_sum(O: "ckks.Oracle", z: "ckks.Ct", c: np.ndarray, s_out: float) -> "ckks.Ct":
    """sum_k c_k T_k(z): T_{2k} = 2 T_k^2 - 1, T_{m+n} = 2 T_m T_n - T_{m-n} (m the
    largest power of two below the index); each term c_k T_k through a constant
    product at scale s_out, all dropped to the level a degree len(c) - 1 sum
    reaches; c_0 added last.  Coefficients below 2^-40 in magnitude (terms under
    the noise of the scale) are left out, and the basis stops at the last one kept."""
    lv = z.level - int(math.ceil(math.log2(len(c)))) - 1
    keep = [k for k in range(1, len(c)) if abs(c[k]) >= 2.0 ** -40]
    d = max(keep)
    T = {1: z}
    for k in range(2, d + 1):
        m = 1 << (k.bit_length() - 1)
        if m == k:
            h = T[k // 2]
            P = O.mul_int(O.mul(h, h), 2)
            T[k] = O.add_const(P, -1.0)
        else:
            n = k - m
            lm = min(T[m].level, T[n].level)
            P = O.mul_int(O.mul(O.drop(T[m], lm), O.drop(T[n], lm)), 2)
            T[k] = O.sub(P, match(O, T[m - n], P.level, P.scale))
    acc = None
    for k in keep:
        t = O.drop(O.cm_target(T[k], float(c[k]), s_out), lv)
        acc = t if acc is None else O.add(acc, t)
    return O.add_const(acc, float(c[0]))


def eval_mod(O: "ckks.Oracle", y: "ckks.Ct", cfg: BootCfg, Bk: float) -> "ckks.Ct":
    """y = (x - 1/4) / Bk  ->  sin(2 pi x): z = 2 y^2 - 1, Chebyshev sum of
    cos(2 pi (x - 1/4) / 2^r), r double angles"""
    c = eval_mod_coeffs(cfg, Bk)
    z = O.add_const(O.mul_int(O.mul(y, y), 2), -1.0)
    v = chebyshev_sum(O, z, c, cfg.s_eval)
    for _ in range(cfg.r):
        v = O.add_const(O.mul_int(O.mul(v, v), 2), -1.0)
    return v


def bootstrap(O: "ckks.Oracle", ct: "ckks.Ct", bound: float, cfg: BootCfg, keys: Dict[int, int],
              s_out: float = None) -> "ckks.Ct":
    """A ciphertext at level >= 1 whose real slot values satisfy |v| <= bound, back
    at level L - levels_used(cfg) with the same values at scale s_out (Delta)."""
    N, s, L = O.N, O.slots, O.L
    s_out = O.Delta if s_out is None else s_out
    q0 = float(O.q[0])
    Bk = cfg.k_bound(O.prm.secret_hw or N) + 0.5
    s_in = q0 * 2.0 ** -cfg.ratio_bits / bound
    # to level 0 at scale s_in; the raised plaintext m + q_0 I read at scale q_0 Bk
    c0 = O.cm_target(O.drop(ct, 1), 1.0, s_in)
    R = O.modraise(c0, L, q0 * Bk)
    # CoeffToSlot: the slots of U become (w / (q_0 Bk)) / 2 in bit-reversed order
    groups = stage_groups(s, cfg.n_cts, True)
    groups[-1] = {d: v * 0.5 for d, v in groups[-1].items()}
    rho = (cfg.s_eval / R.scale) ** (1.0 / cfg.n_cts)
    U = R
    for D in groups:
        U = linear_transform(O, U, D, rho, keys)
    conj = keys[2 * N - 1]
    V = O.rotate_gal(U, conj, 2 * N - 1)
    re = O.add(U, V)
    im = O.mul_plain(O.sub(U, V), monomial(N, N // 2, -1), 1.0)   # times -i
    shift = -0.25 / Bk
    Sre = eval_mod(O, O.add_const(re, shift), cfg, Bk)
    Sim = eval_mod(O, O.add_const(im, shift), cfg, Bk)
    Z = O.add(Sre, O.mul_plain(Sim, monomial(N, N // 2, 1), 1.0))  # + i sin(2 pi x_hi)
    # SlotToCoeff, with kappa = q_0 / (2 pi s_in) turning sin(2 pi x) into m / s_in
    kappa = q0 / (2.0 * math.pi * s_in)
    groups = stage_groups(s, cfg.n_stc, False)
    groups[0] = {d: v * kappa for d, v in groups[0].items()}
    rho = (s_out / Z.scale) ** (1.0 / cfg.n_stc)
    out = Z
    for D in groups:
        out = linear_transform(O, out, D, rho, keys)
    return out
