"""Python side of the O2 CPU RNS-CKKS oracle -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
leg may import this module.  It loads ``oracle/libckks_oracle.so`` (plain C,
built from ``oracle/ckks_oracle.c``) for the ring arithmetic and keeps the
scale bookkeeping, the constant encodings and the CutMax schedule here, in
float64 Python, written from the CKKS conventions (scale rules, constant
encodings) and the encrypted CutMax schedule stated in this module.  It shares
no code with the HIP path.

Paper anchors: CKKS correctness and homomorphic properties (Sec. 2.1);
SIMD slots, rotations and rotate-and-sum (Sec. 3.2, App. D); the encrypted
CutMax (Alg. 2) and its Goldschmidt inverse (App. B.1); the nucleus sampler
(Alg. 3).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_oracle.c")
_LIB = os.path.join(_HERE, "libckks_oracle.so")

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)
dblp = ctypes.POINTER(ctypes.c_double)


def build_oracle(force: bool = False) -> str:
    """Compile the C oracle (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build_oracle())
        V = ctypes.c_void_p
        L.oc_ctx_create.restype = V
        L.oc_ctx_create.argtypes = [ctypes.c_int] * 6 + [ctypes.c_uint64]
        L.oc_ctx_create_ex.restype = V
        L.oc_ctx_create_ex.argtypes = [ctypes.c_int] * 6 + [ctypes.c_uint64] + [ctypes.c_int] * 3
        L.oc_ctx_free.argtypes = [V]
        L.oc_ctx_info.argtypes = [V] + [ctypes.POINTER(ctypes.c_int)] * 4
        L.oc_ctx_primes.argtypes = [V, u64p]
        L.oc_ctx_secret.argtypes = [V, ctypes.POINTER(ctypes.c_int8)]
        L.oc_set_nonce.argtypes = [V, ctypes.c_uint32]
        L.oc_get_nonce.restype = ctypes.c_uint32
        L.oc_get_nonce.argtypes = [V]
        L.oc_keygen.argtypes = [V, ctypes.c_int]
        L.oc_keygen_galois.argtypes = [V, ctypes.c_int, ctypes.c_uint64]
        L.oc_rotsum_step.restype = V
        L.oc_rotsum_step.argtypes = [V, V, ctypes.c_int, ctypes.POINTER(ctypes.c_int), u64p]
        L.oc_rotsum_carried.restype = V
        L.oc_rotsum_carried.argtypes = [V, V, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int), u64p]
        L.oc_ct_free.argtypes = [V]
        L.oc_ct_level.argtypes = [V]
        L.oc_ct_export.argtypes = [V, V, u64p]
        L.oc_ct_import.restype = V
        L.oc_ct_import.argtypes = [V, u64p, ctypes.c_int]
        L.oc_encrypt.restype = V
        L.oc_encrypt.argtypes = [V, i64p]
        L.oc_decrypt.argtypes = [V, V, dblp]
        for name in ("oc_add", "oc_sub", "oc_mul", "oc_mul_norescale"):
            getattr(L, name).restype = V
            getattr(L, name).argtypes = [V, V, V]
        for name in ("oc_mul_int", "oc_add_const_int", "oc_mul_int_rescale"):
            getattr(L, name).restype = V
            getattr(L, name).argtypes = [V, V, ctypes.c_int64]
        L.oc_drop.restype = V
        L.oc_drop.argtypes = [V, V, ctypes.c_int]
        L.oc_rescale.restype = V
        L.oc_rescale.argtypes = [V, V]
        L.oc_rotate.restype = V
        L.oc_rotate.argtypes = [V, V, ctypes.c_int]
        L.oc_automorph.restype = V
        L.oc_automorph.argtypes = [V, V, ctypes.c_uint64]
        L.oc_rotate_gal.restype = V
        L.oc_rotate_gal.argtypes = [V, V, ctypes.c_int, ctypes.c_uint64]
        L.oc_mul_plain.restype = V
        L.oc_mul_plain.argtypes = [V, V, i64p]
        L.oc_modraise.restype = V
        L.oc_modraise.argtypes = [V, V, ctypes.c_int]
        L.oc_keyswitch.argtypes = [V, u64p, ctypes.c_int, ctypes.c_int, u64p, u64p]
        L.oc_schoolbook.argtypes = [u64p, u64p, u64p, ctypes.c_int, ctypes.c_uint64]
        L.oc_ring_mul.argtypes = [V, ctypes.c_int, u64p, u64p, u64p]
        L.oc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.oc_num_threads.restype = ctypes.c_int
        L.oc_set_num_threads.argtypes = [ctypes.c_int]
        L.oc_set_num_threads.restype = None
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().oc_philox4x32_10(c, k, o)
    return list(o)


def llround(x: float) -> int:
    """C llround: nearest integer, halves away from zero."""
    f = math.floor(x)
    d = x - f
    if d > 0.5 or (d == 0.5 and x > 0):
        return int(f) + 1
    return int(f)


# ----------------------------------------------------------------------------
# parameters
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Params:
    log_n: int
    n_q: int          # number of Q primes (q_0 .. q_L), L = n_q - 1
    q0_bits: int
    q_bits: int
    p_bits: int
    dnum: int
    log2_scale: float
    seed: int = 1
    hoist: int = 0    # rotate-and-sum: 0 one rotation at a time, h >= 1 hoisted radix-2^h steps
    n_hi: int = 0     # the top n_hi Q primes have hi_bits bits (levels a bootstrap uses first)
    hi_bits: int = 0
    secret_hw: int = 0  # 0: dense ternary secret; h > 0: sparse ternary with h nonzeros

    @property
    def N(self):
        return 1 << self.log_n

    @property
    def slots(self):
        return self.N // 2


# ----------------------------------------------------------------------------
# encoding (canonical embedding, slot j <-> zeta^(5^j mod 2N), zeta = e^{i pi/N})
# ----------------------------------------------------------------------------
def slot_exponents(N: int) -> np.ndarray:
    t = np.empty(N // 2, dtype=np.int64)
    v = 1
    for j in range(N // 2):
        t[j] = v
        v = (v * 5) % (2 * N)
    return t


def encode_direct(z: np.ndarray, N: int, scale: float) -> np.ndarray:
    """m_k = round((2 scale / N) sum_j z_j cos(pi t_j k / N)), real slots z (small N)."""
    t = slot_exponents(N)
    k = np.arange(N)
    ang = np.pi * np.outer(t, k).astype(np.float64) / N % (2 * np.pi)
    m = (2.0 * scale / N) * (np.asarray(z, dtype=np.float64) @ np.cos(ang))
    return np.array([llround(v) for v in m], dtype=np.int64)


def decode_direct(m: np.ndarray, N: int, scale: float) -> np.ndarray:
    """z_j = Re m(zeta^{t_j}) / scale, by direct evaluation (small N)."""
    t = slot_exponents(N)
    k = np.arange(N)
    ang = np.pi * np.outer(t, k).astype(np.float64) / N % (2 * np.pi)
    return (np.cos(ang) @ np.asarray(m, dtype=np.float64)) / scale


def _eval_all_odd(m: np.ndarray, N: int) -> np.ndarray:
    """m(zeta^(2k+1)) for k < N as a twisted DFT: sum_i (m_i zeta^i) omega^(ik)."""
    i = np.arange(N)
    tw = np.exp(1j * np.pi * i / N)
    return np.fft.ifft(np.asarray(m, dtype=np.float64) * tw) * N


def decode_fft(m: np.ndarray, N: int, scale: float) -> np.ndarray:
    ev = _eval_all_odd(m, N)
    t = slot_exponents(N)
    return ev[(t - 1) // 2].real / scale


def encode_fft(z: np.ndarray, N: int, scale: float) -> np.ndarray:
    t = slot_exponents(N)
    E = np.zeros(N, dtype=np.complex128)
    zz = np.asarray(z, dtype=np.float64) * scale
    E[(t - 1) // 2] = zz
    E[(2 * N - t - 1) // 2] = zz          # conjugate slots (real input)
    i = np.arange(N)
    v = np.fft.fft(E) / N * np.exp(-1j * np.pi * i / N)
    return np.array([llround(x) for x in v.real], dtype=np.int64)


def encode(z, N, scale):
    return encode_direct(z, N, scale) if N <= 4096 else encode_fft(z, N, scale)


def decode(m, N, scale):
    return decode_direct(m, N, scale) if N <= 4096 else decode_fft(m, N, scale)


# ----------------------------------------------------------------------------
# ciphertext handle with scale bookkeeping
# ----------------------------------------------------------------------------
class Ct:
    __slots__ = ("h", "level", "scale", "ctx")

    def __init__(self, ctx, h, scale):
        if not h:
            raise RuntimeError("oracle op failed")
        self.ctx, self.h, self.scale = ctx, h, float(scale)
        self.level = lib().oc_ct_level(h)

    def __del__(self):
        try:
            if self.h:
                lib().oc_ct_free(self.h)
        except Exception:
            pass

    def export(self) -> np.ndarray:
        N = self.ctx.N
        out = np.empty((2, self.level + 1, N), dtype=np.uint64)
        lib().oc_ct_export(self.ctx.h, self.h, _p(out, u64p))
        return out


class SchedError(RuntimeError):
    pass


def hoist_steps(slots: int, h: int) -> List[List[int]]:
    """Rotation amounts of each step of the hoisted rotate-and-sum with radix 2^h over
    log2(slots) bits: step b covers bits [b, b + hb), hb = min(h, bits left), and
    rotates by r 2^b for r = 1 .. 2^hb - 1."""
    lg = int(math.log2(slots))
    out, b = [], 0
    while b < lg:
        hb = min(h, lg - b)
        out.append([r << b for r in range(1, 1 << hb)])
        b += hb
    return out


def rotation_keys(slots: int, h: int) -> dict:
    """Key index of every rotation amount the hoisted rotate-and-sum uses: a power of
    two 2^e has key 1 + e (the single-rotation keys); the other amounts follow, in
    step order, from 1 + log2(slots)."""
    lg = int(math.log2(slots))
    keys = {1 << e: 1 + e for e in range(lg)}
    nxt = 1 + lg
    for step in hoist_steps(slots, h):
        for a in step:
            if a not in keys:
                keys[a] = nxt
                nxt += 1
    return keys


class Oracle:
    """CPU RNS-CKKS context: primes, secret, keys, and the evaluator ops."""

    def __init__(self, prm: Params):
        self.prm = prm
        self.h = lib().oc_ctx_create_ex(prm.log_n, prm.n_q, prm.q0_bits, prm.q_bits, prm.p_bits,
                                        prm.dnum, ctypes.c_uint64(prm.seed), prm.n_hi, prm.hi_bits,
                                        prm.secret_hw)
        if not self.h:
            raise ValueError("bad parameters")
        N, L, A, npr = (ctypes.c_int() for _ in range(4))
        lib().oc_ctx_info(self.h, ctypes.byref(N), ctypes.byref(L), ctypes.byref(A), ctypes.byref(npr))
        self.N, self.L, self.alpha, self.np = N.value, L.value, A.value, npr.value
        self.primes = np.empty(self.np, dtype=np.uint64)
        lib().oc_ctx_primes(self.h, _p(self.primes, u64p))
        self.q = [int(v) for v in self.primes]
        self.Delta = 2.0 ** prm.log2_scale
        self.slots = self.N // 2
        # plain form of the two kernel-shaped steps: with plain=True, rotsum runs the
        # log2(slots) single rotations of Sec. 3.2 and mul relinearises (ModDown by P)
        # and then rescales (by q_l) instead of one ModDown by P q_l
        self.plain = False

    def __del__(self):
        try:
            lib().oc_ctx_free(self.h)
        except Exception:
            pass

    # keys --------------------------------------------------------------
    def keygen(self, relin=True, rot_logs: Sequence[int] = ()):
        if relin:
            lib().oc_keygen(self.h, 0)
        for r in rot_logs:
            lib().oc_keygen(self.h, 1 + int(r))

    def keygen_cutmax(self):
        self.keygen(True, range(int(math.log2(self.slots))))
        if self.prm.hoist >= 1:
            for amount, k in rotation_keys(self.slots, self.prm.hoist).items():
                lib().oc_keygen_galois(self.h, k, pow(5, amount, 2 * self.N))

    def secret(self) -> np.ndarray:
        s = np.empty(self.N, dtype=np.int8)
        lib().oc_ctx_secret(self.h, _p(s, ctypes.POINTER(ctypes.c_int8)))
        return s

    @property
    def nonce(self):
        return lib().oc_get_nonce(self.h)

    @nonce.setter
    def nonce(self, v):
        lib().oc_set_nonce(self.h, v)

    # encryption --------------------------------------------------------
    def encrypt_coeffs(self, m: np.ndarray, scale: float) -> Ct:
        m = np.ascontiguousarray(m, dtype=np.int64)
        assert m.size == self.N
        return Ct(self, lib().oc_encrypt(self.h, _p(m, i64p)), scale)

    def encrypt(self, z: np.ndarray, scale: Optional[float] = None) -> Ct:
        scale = self.Delta if scale is None else scale
        return self.encrypt_coeffs(encode(z, self.N, scale), scale)

    def decrypt_coeffs(self, ct: Ct) -> np.ndarray:
        out = np.empty(self.N, dtype=np.float64)
        lib().oc_decrypt(self.h, ct.h, _p(out, dblp))
        return out

    def decrypt(self, ct: Ct) -> np.ndarray:
        return decode(self.decrypt_coeffs(ct), self.N, ct.scale)

    def import_ct(self, limbs: np.ndarray, scale: float) -> Ct:
        limbs = np.ascontiguousarray(limbs, dtype=np.uint64)
        level = limbs.shape[1] - 1
        return Ct(self, lib().oc_ct_import(self.h, _p(limbs, u64p), level), scale)

    # evaluator ops (scales: mul s_a s_b / q_l, rescale s / q_l) --------
    def add(self, a: Ct, b: Ct) -> Ct:
        if a.level != b.level:
            raise SchedError("add: level mismatch")
        if abs(a.scale - b.scale) > 1e-9 * a.scale:
            raise SchedError(f"add: scale mismatch {a.scale} {b.scale}")
        return Ct(self, lib().oc_add(self.h, a.h, b.h), a.scale)

    def sub(self, a: Ct, b: Ct) -> Ct:
        if a.level != b.level:
            raise SchedError("sub: level mismatch")
        if abs(a.scale - b.scale) > 1e-9 * a.scale:
            raise SchedError(f"sub: scale mismatch {a.scale} {b.scale}")
        return Ct(self, lib().oc_sub(self.h, a.h, b.h), a.scale)

    def mul_int(self, a: Ct, k: int) -> Ct:
        return Ct(self, lib().oc_mul_int(self.h, a.h, int(k)), a.scale)

    def add_const(self, a: Ct, c: float) -> Ct:
        return Ct(self, lib().oc_add_const_int(self.h, a.h, llround(c * a.scale)), a.scale)

    def drop(self, a: Ct, level: int) -> Ct:
        if level == a.level:
            return a
        return Ct(self, lib().oc_drop(self.h, a.h, level), a.scale)

    def rescale(self, a: Ct) -> Ct:
        return Ct(self, lib().oc_rescale(self.h, a.h), a.scale / self.q[a.level])

    def _const_K(self, a: Ct, kappa: float, s_want: float) -> int:
        if a.level < 1:
            raise SchedError("constant multiply needs a level")
        q = float(self.q[a.level])
        K = llround(((kappa * s_want) * q) / a.scale)
        if K == 0 or abs(K) >= 2 ** 62:
            raise SchedError(f"constant {kappa} not encodable (K={K})")
        return K

    def cm_exact(self, a: Ct, kappa: float, s_want: float) -> Ct:
        """x * kappa with one rescale; the declared scale is the exact one."""
        K = self._const_K(a, kappa, s_want)
        q = float(self.q[a.level])
        s = ((a.scale * float(K)) / q) / kappa
        return Ct(self, lib().oc_mul_int_rescale(self.h, a.h, K), s)

    def cm_target(self, a: Ct, kappa: float, s_target: float) -> Ct:
        """x * kappa with one rescale, declared at the requested scale."""
        K = self._const_K(a, kappa, s_target)
        return Ct(self, lib().oc_mul_int_rescale(self.h, a.h, K), s_target)

    def mul(self, a: Ct, b: Ct) -> Ct:
        if a.level != b.level:
            raise SchedError("mul: level mismatch")
        if a.level < 1:
            raise SchedError("mul needs a level")
        q = float(self.q[a.level])
        if self.plain:
            return self.rescale(self.mul_relin(a, b))
        return Ct(self, lib().oc_mul(self.h, a.h, b.h), (a.scale * b.scale) / q)

    def mul_relin(self, a: Ct, b: Ct) -> Ct:
        """tensor product and relinearisation (ModDown by P), no rescale"""
        if a.level != b.level:
            raise SchedError("mul: level mismatch")
        return Ct(self, lib().oc_mul_norescale(self.h, a.h, b.h), a.scale * b.scale)

    def rotate(self, a: Ct, r: int) -> Ct:
        return Ct(self, lib().oc_rotate(self.h, a.h, int(r)), a.scale)

    def keygen_galois(self, kidx: int, galois: int):
        if lib().oc_keygen_galois(self.h, int(kidx), ctypes.c_uint64(int(galois))) != 0:
            raise SchedError("bad key index")

    def rotate_gal(self, a: Ct, kidx: int, galois: int) -> Ct:
        """automorphism X -> X^galois with key kidx (5^r: rotation by r; 2N-1: conjugation)"""
        h = lib().oc_rotate_gal(self.h, a.h, int(kidx), ctypes.c_uint64(int(galois)))
        if not h:
            raise SchedError("missing Galois key")
        return Ct(self, h, a.scale)

    def mul_plain(self, a: Ct, m: np.ndarray, pscale: float) -> Ct:
        """product with the integer plaintext m encoded at pscale (no rescale)"""
        m = np.ascontiguousarray(m, dtype=np.int64)
        assert m.size == self.N
        return Ct(self, lib().oc_mul_plain(self.h, a.h, _p(m, i64p)), a.scale * pscale)

    def modraise(self, a: Ct, level: int, scale: float) -> Ct:
        """level-0 ciphertext lifted to `level`, declared at `scale`"""
        h = lib().oc_modraise(self.h, a.h, int(level))
        if not h:
            raise SchedError("modraise needs a level-0 ciphertext")
        return Ct(self, h, scale)

    # composite steps of Alg. 2 -------------------------------------------
    def rotsum(self, x: Ct) -> Ct:
        """Rotate-and-sum (Sec. 3.2): every slot ends up holding the sum of all slots.
        hoist 0: x <- x + rot(x, 2^r), r = 0..log2(slots)-1, one key switch each.
        hoist h >= 1: steps of radix R = 2^h, x <- x + sum_{r=1}^{R-1} rot(x, r k) for
        k = 1, R, R^2, ... (the last step takes the remaining bits), each step one
        hoisted ModUp, the key products of its R-1 rotations summed; with several steps
        c0 is carried as P c0 over Q u P (oc_rotsum_carried): c1 takes one ModDown a step,
        c0 one at the end."""
        if self.prm.hoist <= 0 or self.plain:
            for r in range(int(math.log2(self.slots))):
                x = self.add(x, self.rotate(x, r))
            return x
        keys = rotation_keys(self.slots, self.prm.hoist)
        steps = hoist_steps(self.slots, self.prm.hoist)
        if len(steps) == 1:
            return self.rotsum_step(x, steps[0], keys)
        return self.rotsum_carried(x, steps, keys)

    def rotsum_carried(self, x: Ct, steps, keys: dict) -> Ct:
        """every hoisted step of a rotate-and-sum in one call, c0 carried as P c0 over Q u P
        between steps (oc_rotsum_carried)"""
        flat = [a for st in steps for a in st]
        nr = (ctypes.c_int * len(steps))(*[len(st) for st in steps])
        kid = (ctypes.c_int * len(flat))(*[keys[a] for a in flat])
        gal = np.array([pow(5, a, 2 * self.N) for a in flat], dtype=np.uint64)
        h = lib().oc_rotsum_carried(self.h, x.h, len(steps), nr, kid, _p(gal, u64p))
        if not h:
            raise SchedError("rotate-and-sum: missing key")
        return Ct(self, h, x.scale)

    def rotsum_step(self, x: Ct, amounts: Sequence[int], keys: dict) -> Ct:
        """x + sum_r rot(x, a_r) with one hoisted key switch (oc_rotsum_step)."""
        kid = (ctypes.c_int * len(amounts))(*[keys[a] for a in amounts])
        gal = np.array([pow(5, a, 2 * self.N) for a in amounts], dtype=np.uint64)
        h = lib().oc_rotsum_step(self.h, x.h, len(amounts), kid, _p(gal, u64p))
        if not h:
            raise SchedError("rotsum step: missing key")
        return Ct(self, h, x.scale)

    def sum_list(self, xs: List[Ct]) -> Ct:
        acc = xs[0]
        for x in xs[1:]:
            acc = self.add(acc, x)
        return acc

    def power(self, y: Ct, p: int) -> Ct:
        """y^p by repeated squaring; depth ceil(log2(p+1)) - ... (Sec. 3.2: log p mults)."""
        if p < 1:
            raise SchedError("p must be >= 1")
        pw = [y]
        for _ in range(1, p.bit_length()):
            pw.append(self.mul(pw[-1], pw[-1]))
        acc = None
        for i in range(p.bit_length()):
            if (p >> i) & 1:
                if acc is None:
                    acc = pw[i]
                else:
                    lv = min(acc.level, pw[i].level)
                    acc = self.mul(self.drop(acc, lv), self.drop(pw[i], lv))
        return acc

    def invsqr(self, U: Ct, coef: Sequence[float], C: float, newton: int, s_final: float,
               goldschmidt: bool = False) -> Ct:
        """Initial-guess polynomial sum_k coef[k] u^k (coefficients already times C) plus
        `newton` refinements landing at scale s_final: Newton steps
        h <- 1.5 h - (0.5/C^2) u h^3, or Goldschmidt's coupled iteration for the inverse
        square root (App. B.1): with y = h/C and b = u y^2,  r = (3 - b)/2,  y <- y r,
        b <- b r^2; here b is carried halved (b' = b/2, r = 1.5 - b')."""
        d = len(coef) - 1
        q = self.q
        lu = U.level
        su = U.scale
        S = s_final if newton == 0 else self.Delta
        if goldschmidt and newton > 0:
            # the scale of h is multiplied by scale(r_k)/q at every update; pick the
            # starting scale so that the last update lands on s_final
            lh0 = lu - {1: 1, 2: 2, 3: 2, 4: 3}[d]
            lev, s_b, factor = lh0 - 2, self.Delta, 1.0
            for k in range(newton):
                if k > 0:
                    s_r2 = s_b * s_b / float(q[lev])
                    s_b = s_b * s_r2 / float(q[lev - 1])
                    lev -= 2
                factor = factor * s_b / float(q[lev])
            S = s_final / factor
        if d == 1:
            H = self.add_const(self.cm_target(U, coef[1], S), coef[0])
        elif d == 2:
            U2 = self.mul(U, U)
            T2 = self.cm_target(U2, coef[2], S)
            T1 = self.cm_target(self.drop(U, lu - 1), coef[1], S)
            H = self.add_const(self.add(T2, T1), coef[0])
        elif d == 3:
            U2 = self.mul(U, U)
            s2 = U2.scale
            sA = (S * float(q[lu - 1])) / s2
            T3 = self.mul(self.cm_target(U, coef[3], sA), U2)
            T2 = self.cm_target(U2, coef[2], S)
            T1 = self.cm_target(self.drop(U, lu - 1), coef[1], S)
            H = self.add_const(self.add(self.add(T3, T2), T1), coef[0])
        elif d == 4:
            U2 = self.mul(U, U)
            s2 = U2.scale
            sC = (S * float(q[lu - 2])) / s2
            T4 = self.mul(self.cm_target(U2, coef[4], sC), self.drop(U2, lu - 2))
            sD = (S * float(q[lu - 2])) / su
            T3 = self.mul(self.cm_target(U2, coef[3], sD), self.drop(U, lu - 2))
            T2 = self.cm_target(self.drop(U2, lu - 2), coef[2], S)
            T1 = self.cm_target(self.drop(U, lu - 2), coef[1], S)
            H = self.add_const(self.add(self.add(self.add(T4, T3), T2), T1), coef[0])
        else:
            raise SchedError("initial-guess degree must be 1..4")
        if goldschmidt and newton > 0:
            lh = H.level
            G2 = self.mul(H, H)                                    # h^2
            sA = (self.Delta * float(q[lh - 1])) / G2.scale
            A = self.drop(self.cm_target(U, 0.5 / (C * C), sA), lh - 1)
            Bh = self.mul(A, G2)                                   # b'_0 = u h^2 / (2 C^2)
            R = self.add_const(self.mul_int(Bh, -1), 1.5)          # r_0
            H = self.mul(self.drop(H, R.level), R)                 # h_1 = h_0 r_0
            for _ in range(1, newton):
                R2 = self.mul(R, R)
                Bh = self.mul(self.drop(Bh, R2.level), R2)         # b'_k = b'_{k-1} r^2
                R = self.add_const(self.mul_int(Bh, -1), 1.5)
                H = self.mul(self.drop(H, R.level), R)
            return H
        for it in range(newton):
            St = s_final if it == newton - 1 else self.Delta
            lh, sh = H.level, H.scale
            G2 = self.mul(H, H)
            sA = (((St * float(q[lh])) * float(q[lh - 1])) / sh) / G2.scale
            A = self.drop(self.cm_target(U, -0.5 / (C * C), sA), lh)
            B = self.mul(A, H)
            T = self.mul(B, G2)
            L1 = self.drop(self.cm_target(H, 1.5, St), lh - 2)
            H = self.add(T, L1)
        return H


def scaled_normalise(O: Oracle, U: Ct, E: List[Ct], coef: Sequence[float], steps, C: float,
                     gain: float = 1.0) -> List[Ct]:
    """z = E h + gain with h ~ C u^(-1/2) (C already carrying the gain, the iterate's
    prescale) from the guess g and the scaled refinements
    x <- x (a_k - b_k x^2) (x = g sqrt(u)), carried on E (the wide-domain form):
      Ey = E (C g),  W = b_0 u g^2 = b_0 x_0^2 (the guess evaluated twice from U: C g at the
      scale that puts E C g at Delta, sqrt(b_0) g at the scale that puts W at Delta);
      per step: r = a_k - W (no level), every Ey <- Ey r, and unless it is the last step
      W <- (W b_{k+1}/b_k) r^2 (the constant multiply lands at the scale that puts the new W at
      Delta, in parallel with r^2: two levels a step);
      z = Ey + gain.
    Ey carries (y - mu)/(c sigma) x_k and W carries b_k x_k^2, so no ciphertext holds
    u^(-1/2) itself, whose range spans the domain's decades."""
    d = len(coef) - 1
    q = O.q
    lg = U.level - invsqr_depth(d, 0)
    H0 = O.invsqr(U, [g * C for g in coef], C, 0, (O.Delta * float(q[lg])) / E[0].scale)
    b0 = float(steps[0][1])
    sG = math.sqrt(((O.Delta * float(q[lg])) * float(q[lg - 1])) / U.scale)
    G0 = O.invsqr(U, [g * math.sqrt(b0) for g in coef], 1.0, 0, sG)
    Ey = [O.mul(O.drop(e, lg), H0) for e in E]
    W = O.mul(O.drop(U, lg - 1), O.mul(G0, G0))
    for k, (a, b) in enumerate(steps):
        R = O.add_const(O.mul_int(W, -1), a)
        Ey = [O.mul(O.drop(e, R.level), R) for e in Ey]
        if k + 1 < len(steps):
            L = W.level
            sV = ((O.Delta * float(q[L])) * float(q[L - 1])) / (R.scale * R.scale)
            V = O.cm_target(W, float(steps[k + 1][1]) / b, sV)
            W = O.mul(V, O.mul(R, R))
    return [O.add_const(e, gain) for e in Ey]


def invsqr_depth(degree: int, newton: int, goldschmidt: bool = False) -> int:
    """Levels of the initial guess plus its refinements; Goldschmidt's first b = u h^2
    needs h^2 before the first update, one level more than Newton's steps."""
    return {1: 1, 2: 2, 3: 2, 4: 3}[degree] + 2 * newton + (1 if goldschmidt and newton > 0 else 0)


@dataclass
class HECfg:
    """Schedule constants of the encrypted CutMax for one request."""
    T: int
    p: Sequence[int]
    c: Sequence[float]
    v_lo: Sequence[float]
    v_hi: Sequence[float]
    coef: Sequence[Sequence[float]]   # per iteration, power basis of g(u) ~ u^(-1/2), u = var/v_hi
    newton: int = 0
    goldschmidt: bool = False          # refinements by Goldschmidt's iteration instead of Newton's
    sum_lo: float = 1.0                # bounds of mean(y^(T)) = sum/n
    sum_hi: float = 3.0
    gold_d: int = 3
    # per iteration, the (a_k, b_k) of scaled refinements x <- x (a_k - b_k x^2) of the guess
    # (replace newton; an empty list keeps the guess alone)
    scaled: Optional[Sequence[Sequence[Sequence[float]]]] = None

    def inv_depth(self, t: int) -> int:
        d = len(self.coef[t]) - 1
        if self.scaled is not None:
            return invsqr_depth(d, 0) + 2 * len(self.scaled[t])
        return invsqr_depth(d, self.newton, self.goldschmidt)

    def prescale(self) -> List[int]:
        """Per iteration t, the exponent e of the power of two 2^(-e) by which its output is
        scaled.  CutMax is unchanged when its iterate is multiplied by a positive constant
        (Alg. 1: the next semi-standardisation, or the final division by the sum, removes
        it), while one constant multiply cannot resolve a factor below 1/q: deep schedules
        (p = 16 after the first iteration, Table 2) reach variances near 1e12, whose
        1 / (n sqrt(n v)) is smaller.  e is the least exponent that brings the next
        iteration's variance bound under 2^8, or for the last iteration the bound of the
        mean under 2^4; it is applied as the factor 2^(-e/p) on the normalised iterate."""
        es = []
        for t in range(self.T):
            e = 0
            if t + 1 < self.T:
                while math.ldexp(float(self.v_hi[t + 1]), -2 * e) > 256.0:
                    e += 1
            else:
                while math.ldexp(float(self.sum_hi), -e) > 16.0:
                    e += 1
            es.append(e)
        return es

    def levels_needed(self) -> int:
        lv = 0
        for t in range(self.T):
            lv += 2 + self.inv_depth(t) + 1 \
                + (int(self.p[t]).bit_length() - 1) \
                + (1 if bin(int(self.p[t])).count("1") > 1 else 0)
        return lv + self.gold_d + 3


def cutmax_he(O: Oracle, Y: List[Ct], cfg: HECfg, rotsum_cache=None, n_real: int = None,
              pad: float = 0.0) -> List[Ct]:
    """Alg. 2 on one request whose packed vector spans len(Y) ciphertexts.

    With n_real (masked padding) the moments and the final sum are taken over the first
    n_real slots only, so the first n_real outputs are CutMax of those entries alone.
    The pad slots all hold one common value, which a tracker ciphertext follows through
    the same steps (it starts as the trivial encryption of the pad value); every slot
    sum subtracts (pad slot count) x tracker, and the variance sum subtracts the same
    multiple of the tracker's square, formed as the square of sqrt(pad slot count) times
    the tracker's centred value (the same quantity, without multiplying the product's
    rounding noise by the pad count)."""
    a = len(Y)
    masked = n_real is not None and n_real < a * O.slots
    n = n_real if masked else a * O.slots
    npad = a * O.slots - n
    P = None
    if masked:
        P = O.mul_int(Y[0], 0)
        if pad != 0.0:
            P = O.add_const(P, pad)
    es = cfg.prescale()
    for t in range(cfg.T):
        S = O.rotsum(O.sum_list(Y))
        if masked:
            S = O.sub(S, O.mul_int(P, npad))
        Yall = Y + ([P] if masked else [])
        D = [O.sub(O.mul_int(y, n), S) for y in Yall]
        # this iteration's input was prescaled by 2^(-e) (the variance by 4^(-e))
        v_hi = math.ldexp(float(cfg.v_hi[t]), -2 * es[t - 1]) if t > 0 else float(cfg.v_hi[t])
        gain = math.pow(2.0, -float(es[t]) / float(cfg.p[t])) if es[t] > 0 else 1.0
        kE = 1.0 / (float(n) * math.sqrt(float(n) * v_hi))
        E = [O.cm_exact(d, kE, O.Delta) for d in D]
        F = [O.mul(e, e) for e in E[:a]]
        U = O.rotsum(O.sum_list(F))
        if masked:
            # the pad slots' share npad E_R^2, evaluated as (sqrt(npad) E_R)^2 so that the
            # product's rounding noise is not multiplied by npad
            Ep = O.cm_target(D[a], kE * math.sqrt(float(npad)), E[a].scale)
            U = O.sub(U, O.mul(Ep, Ep))
        C = math.sqrt(float(n)) / cfg.c[t] * gain
        lh = U.level - cfg.inv_depth(t)
        if lh < 1:
            raise SchedError("chain too short")
        sE = E[0].scale
        if cfg.scaled is not None and len(cfg.scaled[t]) > 0:
            Yn = scaled_normalise(O, U, E, cfg.coef[t], cfg.scaled[t], C, gain)
        else:
            S_H = (O.Delta * float(O.q[lh])) / sE
            H = O.invsqr(U, [g * C for g in cfg.coef[t]], C, cfg.newton, S_H, cfg.goldschmidt)
            Yn = [O.add_const(O.mul(O.drop(e, H.level), H), gain) for e in E]
        Yall = [O.power(y, int(cfg.p[t])) for y in Yn]
        Y, P = Yall[:a], (Yall[a] if masked else None)
    S = O.rotsum(O.sum_list(Y))
    if masked:
        S = O.sub(S, O.mul_int(P, npad))
    B = math.ldexp(float(cfg.sum_hi), -es[-1]) * float(n)
    X = O.cm_exact(S, 1.0 / B, O.Delta)
    E0 = O.add_const(O.mul_int(X, -1), 1.0)
    P = O.add_const(E0, 1.0)
    Ei = E0
    for _ in range(cfg.gold_d):
        Ei = O.mul(Ei, Ei)
        P = O.mul(O.drop(P, Ei.level), O.add_const(Ei, 1.0))
    Z = []
    for y in Y:
        yb = O.cm_exact(y, 1.0 / B, O.Delta)
        Z.append(O.mul(O.drop(yb, P.level), P))
    return Z


def topp_he(O: Oracle, X: List[Ct], G: List[Ct], temperature: float, cfg: HECfg,
            prescaled: bool = False, n_real: int = None) -> List[Ct]:
    """Alg. 3 server side: CutMax(X + tau*G) (equal to CutMax(X/tau + G))."""
    return cutmax_he(O, topp_input(O, X, G, temperature, prescaled), cfg, n_real=n_real)


def topp_input(O: Oracle, X: List[Ct], G: List[Ct], temperature: float, prescaled: bool = False) -> List[Ct]:
    """The sampler's CutMax input X + tau*G: the noise times tau by one constant multiply
    declared at the logits' scale (one level, the logits dropped to match), or X + G when
    the client already scaled the noise."""
    if prescaled:
        return [O.add(x, g) for x, g in zip(X, G)]
    Gs = [O.cm_target(g, temperature, x.scale) for x, g in zip(X, G)]
    return [O.add(O.drop(x, gs.level), gs) for x, gs in zip(X, Gs)]
