"""ctypes binding of libcutmax_he.so (the C ABI in include/he.h).

Argument marshalling only: every step of the encrypted CutMax runs in the
library's HIP kernels.  There is no CPU fallback: if the library is missing or
no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcutmax_he.so")

HE_OK, HE_EINVAL, HE_ENOMEM, HE_EDEVICE, HE_EDEPTH, HE_ERANGE, HE_ESTATE, HE_EIO = 0, -1, -2, -3, -4, -5, -6, -7
HE_NOISE_PRESCALED = 1
HE_REFINE_GOLDSCHMIDT = 2
HE_MASK_PAD = 4
HE_BOOT = 8
HE_REFINE_SCALED = 16
HE_OPT_GRAPH, HE_OPT_NTT_VARIANT, HE_OPT_BOOT_HOIST, HE_OPT_WORKSPACE_LIMIT = 1, 2, 3, 4

_c_u32p = ctypes.POINTER(ctypes.c_uint32)
_c_u64p = ctypes.POINTER(ctypes.c_uint64)
_c_i64p = ctypes.POINTER(ctypes.c_int64)
_c_dp = ctypes.POINTER(ctypes.c_double)
_V = ctypes.c_void_p


class HeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"he error {code}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_q", ctypes.c_uint32), ("q0_bits", ctypes.c_uint32),
                ("q_bits", ctypes.c_uint32), ("p_bits", ctypes.c_uint32), ("dnum", ctypes.c_uint32),
                ("log2_scale", ctypes.c_double), ("seed", ctypes.c_uint64), ("device", ctypes.c_int),
                ("stream", _V), ("hoist", ctypes.c_uint32), ("n_hi", ctypes.c_uint32),
                ("hi_bits", ctypes.c_uint32), ("secret_hw", ctypes.c_uint32)]


class _BootCfg(ctypes.Structure):
    _fields_ = [("n_cts", ctypes.c_uint32), ("n_stc", ctypes.c_uint32), ("K", ctypes.c_uint32),
                ("ratio_bits", ctypes.c_uint32), ("cheb_deg", ctypes.c_uint32), ("r", ctypes.c_uint32),
                ("log2_s_eval", ctypes.c_double), ("correct_bits", ctypes.c_uint32)]


class _Cfg(ctypes.Structure):
    _fields_ = [("T", ctypes.c_uint32), ("p", _c_u32p), ("c", _c_dp), ("var_lo", _c_dp),
                ("var_hi", _c_dp), ("init_degree", ctypes.c_uint32), ("init_coef", _c_dp),
                ("newton_steps", ctypes.c_uint32), ("sum_lo", ctypes.c_double),
                ("sum_hi", ctypes.c_double), ("gold_d", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("ref_steps", _c_u32p), ("ref_coef", _c_dp), ("ref_range", _c_dp)]


_lib = None


def lib():
    """Load the library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2509_08383_amd.build first")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "he_ctx_create": [ctypes.POINTER(_Params), ctypes.POINTER(_V)],
            "he_ctx_info": [_V, _c_u32p, _c_u32p, _c_u32p, _c_u32p, _c_u64p],
            "he_encrypt": [_V, _c_dp, ctypes.c_size_t, ctypes.c_double, ctypes.POINTER(_V)],
            "he_encrypt_coeffs": [_V, _c_i64p, ctypes.c_uint32, ctypes.c_double, ctypes.c_size_t,
                                  ctypes.POINTER(_V)],
            "he_decrypt": [_V, _V, _c_dp, ctypes.c_size_t],
            "he_cutmax": [_V, ctypes.POINTER(_V), ctypes.c_size_t, ctypes.POINTER(_Cfg), ctypes.POINTER(_V)],
            "he_topp_sample": [_V, ctypes.POINTER(_V), ctypes.POINTER(_V), ctypes.c_size_t, ctypes.c_double,
                               ctypes.c_double, ctypes.POINTER(_Cfg), ctypes.POINTER(_V)],
            "he_topp_noise": [ctypes.c_double, _c_dp, ctypes.c_size_t, _c_dp],
            "he_ct_set_pad": [_V, ctypes.c_double],
            "he_gumbel_sample": [_V, ctypes.POINTER(_V), ctypes.POINTER(_V), ctypes.c_size_t, ctypes.c_double,
                                 ctypes.POINTER(_Cfg), ctypes.POINTER(_V)],
            "he_gumbel_noise": [_c_dp, ctypes.c_size_t, _c_dp],
            "he_invsqrt_guess_fit": [ctypes.c_double, ctypes.c_uint32, _c_dp],
            "he_invsqrt_scaled_plan": [ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32, _c_dp, _c_dp, _c_dp],
            "he_ct_info": [_V, _c_u32p, _c_u32p, _c_dp, ctypes.POINTER(ctypes.c_size_t)],
            "he_ct_export": [_V, _V, _c_u64p, ctypes.c_size_t],
            "he_ct_import": [_V, _c_u64p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_size_t,
                             ctypes.POINTER(_V)],
            "he_add": [_V, _V, _V, ctypes.POINTER(_V)],
            "he_sub": [_V, _V, _V, ctypes.POINTER(_V)],
            "he_mul": [_V, _V, _V, ctypes.POINTER(_V)],
            "he_mul_int": [_V, _V, ctypes.c_int64, ctypes.POINTER(_V)],
            "he_add_const": [_V, _V, ctypes.c_double, ctypes.POINTER(_V)],
            "he_rescale": [_V, _V, ctypes.POINTER(_V)],
            "he_cmul": [_V, _V, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.POINTER(_V)],
            "he_rotate": [_V, _V, ctypes.c_uint32, ctypes.POINTER(_V)],
            "he_rotsum": [_V, _V, ctypes.POINTER(_V)],
            "he_rotsum_noalloc": [_V, _V, _V],
            "he_drop": [_V, _V, ctypes.c_uint32, ctypes.POINTER(_V)],
            "he_bench_ntt": [_V, ctypes.c_uint32, ctypes.c_uint32, _c_dp, _c_dp],
            "he_bench_copy": [_V, ctypes.c_uint32, ctypes.c_uint32, _c_dp],
            "he_last_cutmax_ms": [_V, _c_dp],
            "he_sync": [_V],
            "he_set_option": [_V, ctypes.c_int, ctypes.c_int64],
            "he_ntt_tuning": [_V, ctypes.POINTER(ctypes.c_int32), ctypes.c_uint32],
            "he_ntt_tuning_report": [_V, ctypes.c_char_p, ctypes.c_size_t],
            "he_profile_begin": [_V],
            "he_profile_end": [_V, ctypes.c_char_p, ctypes.c_size_t],
            "he_boot_setup": [_V, ctypes.POINTER(_BootCfg)],
            "he_bootstrap": [_V, _V, ctypes.c_double, ctypes.POINTER(_V)],
            "he_keygen_galois": [_V, ctypes.c_uint32, ctypes.c_uint64],
            "he_rotate_gal": [_V, _V, ctypes.c_uint32, ctypes.c_uint64, ctypes.POINTER(_V)],
            "he_mul_plain": [_V, _V, _c_i64p, ctypes.c_double, ctypes.POINTER(_V)],
            "he_modraise": [_V, _V, ctypes.c_uint32, ctypes.c_double, ctypes.POINTER(_V)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.he_ctx_destroy.argtypes = [_V]
        L.he_ctx_destroy.restype = None
        L.he_ct_free.argtypes = [_V]
        L.he_ct_free.restype = None
        L.he_last_error.argtypes = []
        L.he_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != HE_OK:
        raise HeError(rc, lib().he_last_error().decode())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_c_dp)


@dataclass
class Params:
    log_n: int
    n_q: int
    q0_bits: int
    q_bits: int
    p_bits: int
    dnum: int
    log2_scale: float
    seed: int = 1
    hoist: int = 0  # rotate-and-sum: 0 one rotation at a time, h = hoisted radix-2^h steps
    n_hi: int = 0      # the top n_hi Q primes have hi_bits bits (the levels a bootstrap uses first)
    hi_bits: int = 0
    secret_hw: int = 0  # 0 dense ternary secret, h > 0 sparse ternary with h nonzeros


@dataclass
class BootCfg:
    """Bootstrap configuration (he_boot_cfg)."""
    n_cts: int = 3
    n_stc: int = 3
    K: int = 0
    ratio_bits: int = 12
    cheb_deg: int = 31
    r: int = 3
    log2_s_eval: float = 48.0
    correct_bits: int = 0   # > 0: a second pass removes the first pass's error (bound 2^-correct_bits)

    def levels(self) -> int:
        import math
        return self.n_cts + 1 + int(math.ceil(math.log2(self.cheb_deg + 1))) + 1 + self.r + self.n_stc


# parameter sets: a non-secure toy chain at N = 2^12 and the 128-bit chain at N = 2^16
TOY = Params(log_n=12, n_q=36, q0_bits=40, q_bits=30, p_bits=40, dnum=3, log2_scale=30, seed=7, hoist=3)
SECURE = Params(log_n=16, n_q=30, q0_bits=48, q_bits=40, p_bits=48, dnum=3, log2_scale=40, seed=11, hoist=3)
# bootstrappable sets: 48-bit primes on the levels the bootstrap consumes first (CoeffToSlot
# and EvalMod), 40-bit scaling primes below, a sparse ternary secret
TOY_BOOT = Params(log_n=12, n_q=20, q0_bits=48, q_bits=40, p_bits=48, dnum=3, log2_scale=40, seed=5, hoist=3,
                  n_hi=13, hi_bits=48, secret_hw=64)
BOOT = Params(log_n=16, n_q=29, q0_bits=48, q_bits=40, p_bits=48, dnum=3, log2_scale=40, seed=13, hoist=3,
              n_hi=13, hi_bits=48, secret_hw=192)


@dataclass
class CutmaxCfg:
    """Hyper-parameters of one CutMax call (he_cutmax_cfg)."""
    T: int
    p: Sequence[int]
    c: Sequence[float]
    var_lo: Sequence[float]
    var_hi: Sequence[float]
    init_degree: int = 3
    init_coef: Optional[Sequence[Sequence[float]]] = None   # [T][degree+1], g(u) ~ u^-1/2
    newton_steps: int = 0
    sum_lo: float = 1.0
    sum_hi: float = 3.0
    gold_d: int = 3
    flags: int = 0
    # HE_REFINE_SCALED: per iteration, the (a_k, b_k) pairs and the K+1 (l_k, h_k) ranges
    ref_steps: Optional[Sequence[Sequence[Sequence[float]]]] = None
    ref_range: Optional[Sequence[Sequence[Sequence[float]]]] = None
    _keep: list = field(default_factory=list, repr=False)

    def c_struct(self) -> _Cfg:
        T = self.T
        p = (ctypes.c_uint32 * T)(*[int(v) for v in self.p])
        c = (ctypes.c_double * T)(*[float(v) for v in self.c])
        lo = (ctypes.c_double * T)(*[float(v) for v in self.var_lo])
        hi = (ctypes.c_double * T)(*[float(v) for v in self.var_hi])
        coef = None
        if self.init_coef is not None:
            flat = [float(v) for row in self.init_coef for v in row]
            assert len(flat) == T * (self.init_degree + 1)
            coef = (ctypes.c_double * len(flat))(*flat)
        self._keep = [p, c, lo, hi, coef]
        rs = rc = rr = None
        if self.ref_steps is not None:
            assert self.ref_range is not None and len(self.ref_steps) == T and len(self.ref_range) == T
            rs = (ctypes.c_uint32 * T)(*[len(st) for st in self.ref_steps])
            fc = [float(v) for st in self.ref_steps for ab in st for v in ab]
            fr = [float(v) for rg in self.ref_range for lh in rg for v in lh]
            assert len(fr) == 2 * sum(len(st) + 1 for st in self.ref_steps)
            rc = (ctypes.c_double * max(1, len(fc)))(*fc)
            rr = (ctypes.c_double * len(fr))(*fr)
            self._keep += [rs, rc, rr]
        s = _Cfg()
        s.T, s.p, s.c, s.var_lo, s.var_hi = T, p, c, lo, hi
        s.init_degree = self.init_degree
        s.init_coef = ctypes.cast(coef, _c_dp) if coef is not None else None
        s.newton_steps, s.sum_lo, s.sum_hi = self.newton_steps, self.sum_lo, self.sum_hi
        s.gold_d, s.flags = self.gold_d, self.flags
        if rs is not None:
            s.ref_steps = ctypes.cast(rs, _c_u32p)
            s.ref_coef = ctypes.cast(rc, _c_dp)
            s.ref_range = ctypes.cast(rr, _c_dp)
        return s


class Ciphertext:
    def __init__(self, ctx: "Context", h):
        self.ctx, self.h = ctx, h

    def __del__(self):
        try:
            if self.h:
                lib().he_ct_free(self.h)
                self.h = None
        except Exception:
            pass

    def info(self):
        a, lv, n = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_size_t()
        sc = ctypes.c_double()
        _check(lib().he_ct_info(self.h, ctypes.byref(a), ctypes.byref(lv), ctypes.byref(sc), ctypes.byref(n)))
        return a.value, lv.value, sc.value, n.value

    @property
    def a(self):
        return self.info()[0]

    @property
    def level(self):
        return self.info()[1]

    @property
    def scale(self):
        return self.info()[2]

    @property
    def n(self):
        return self.info()[3]

    def set_pad(self, pad: float):
        """Record the value of the pad slots (handles from encrypt_coeffs or import)."""
        _check(lib().he_ct_set_pad(self.h, pad))


class Context:
    """One CKKS context on one GPU (he_ctx)."""

    def __init__(self, prm: Params, device: int = 0, stream: Optional[int] = None):
        P = _Params(prm.log_n, prm.n_q, prm.q0_bits, prm.q_bits, prm.p_bits, prm.dnum, float(prm.log2_scale),
                    prm.seed, device, stream, prm.hoist, prm.n_hi, prm.hi_bits, prm.secret_hw)
        h = _V()
        _check(lib().he_ctx_create(ctypes.byref(P), ctypes.byref(h)))
        self.h = h
        self.prm = prm
        N, s, L, A = (ctypes.c_uint32() for _ in range(4))
        _check(lib().he_ctx_info(self.h, ctypes.byref(N), ctypes.byref(s), ctypes.byref(L), ctypes.byref(A), None))
        self.N, self.slots, self.L, self.alpha = N.value, s.value, L.value, A.value
        pr = np.empty(self.L + 1 + self.alpha, dtype=np.uint64)
        _check(lib().he_ctx_info(self.h, None, None, None, None, pr.ctypes.data_as(_c_u64p)))
        self.primes = [int(v) for v in pr]
        self.Delta = 2.0 ** prm.log2_scale

    def close(self):
        if getattr(self, "h", None):
            lib().he_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _out(self):
        return _V()

    # client ------------------------------------------------------------------
    def encrypt(self, x, pad: float = 0.0) -> Ciphertext:
        """pad: value of the slots beyond len(x) when x is padded; float('nan') pads with
        the mean of x (what masked CutMax, HE_MASK_PAD, wants)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        h = _V()
        _check(lib().he_encrypt(self.h, _dp(x), x.size, pad, ctypes.byref(h)))
        return Ciphertext(self, h)

    def encrypt_coeffs(self, m, scale: float, n: int) -> Ciphertext:
        m = np.ascontiguousarray(m, dtype=np.int64)
        a = m.size // self.N
        h = _V()
        _check(lib().he_encrypt_coeffs(self.h, m.ctypes.data_as(_c_i64p), a, scale, n, ctypes.byref(h)))
        return Ciphertext(self, h)

    def decrypt(self, ct: Ciphertext, n: Optional[int] = None) -> np.ndarray:
        n = ct.n if n is None else n
        out = np.empty(n, dtype=np.float64)
        _check(lib().he_decrypt(self.h, ct.h, _dp(out), n))
        return out

    def export(self, ct: Ciphertext) -> np.ndarray:
        a, lv, _, _ = ct.info()
        out = np.empty((a, 2, lv + 1, self.N), dtype=np.uint64)
        _check(lib().he_ct_export(self.h, ct.h, out.ctypes.data_as(_c_u64p), out.size))
        return out

    def import_ct(self, limbs: np.ndarray, scale: float, n: int) -> Ciphertext:
        limbs = np.ascontiguousarray(limbs, dtype=np.uint64)
        a, _, lv1, _ = limbs.shape
        h = _V()
        _check(lib().he_ct_import(self.h, limbs.ctypes.data_as(_c_u64p), a, lv1 - 1, scale, n, ctypes.byref(h)))
        return Ciphertext(self, h)

    # server ------------------------------------------------------------------
    def cutmax(self, cts: List[Ciphertext], cfg: CutmaxCfg) -> List[Ciphertext]:
        B = len(cts)
        ins = (_V * B)(*[c.h for c in cts])
        outs = (_V * B)()
        s = cfg.c_struct()
        _check(lib().he_cutmax(self.h, ins, B, ctypes.byref(s), outs))
        return [Ciphertext(self, _V(o)) for o in outs]

    def topp_sample(self, logits: List[Ciphertext], noise: List[Ciphertext], top_p: float,
                    temperature: float, cfg: CutmaxCfg) -> List[Ciphertext]:
        B = len(logits)
        ins = (_V * B)(*[c.h for c in logits])
        nz = (_V * B)(*[c.h for c in noise])
        outs = (_V * B)()
        s = cfg.c_struct()
        _check(lib().he_topp_sample(self.h, ins, nz, B, top_p, temperature, ctypes.byref(s), outs))
        return [Ciphertext(self, _V(o)) for o in outs]

    def gumbel_sample(self, logits: List[Ciphertext], noise: List[Ciphertext], temperature: float,
                      cfg: CutmaxCfg) -> List[Ciphertext]:
        B = len(logits)
        ins = (_V * B)(*[c.h for c in logits])
        nz = (_V * B)(*[c.h for c in noise])
        outs = (_V * B)()
        s = cfg.c_struct()
        _check(lib().he_gumbel_sample(self.h, ins, nz, B, temperature, ctypes.byref(s), outs))
        return [Ciphertext(self, _V(o)) for o in outs]

    def _op(self, name, *args):
        h = _V()
        _check(getattr(lib(), name)(self.h, *args, ctypes.byref(h)))
        return Ciphertext(self, h)

    def add(self, a, b):
        return self._op("he_add", a.h, b.h)

    def sub(self, a, b):
        return self._op("he_sub", a.h, b.h)

    def mul(self, a, b):
        return self._op("he_mul", a.h, b.h)

    def mul_int(self, a, k: int):
        return self._op("he_mul_int", a.h, int(k))

    def add_const(self, a, c: float):
        return self._op("he_add_const", a.h, float(c))

    def rescale(self, a):
        return self._op("he_rescale", a.h)

    def cmul(self, a, kappa: float, s_want: float, exact: bool):
        return self._op("he_cmul", a.h, float(kappa), float(s_want), int(bool(exact)))

    def rotate(self, a, r: int):
        return self._op("he_rotate", a.h, int(r))

    def rotsum(self, a):
        return self._op("he_rotsum", a.h)

    def drop(self, a, level: int):
        return self._op("he_drop", a.h, int(level))

    def rotsum_noalloc(self, a, out):
        """rotate-and-sum of a into the existing handle out, with no device allocation"""
        _check(lib().he_rotsum_noalloc(self.h, a.h, out.h))
        return out

    # bootstrapping -------------------------------------------------------------
    def boot_setup(self, cfg: BootCfg):
        c = _BootCfg(cfg.n_cts, cfg.n_stc, cfg.K, cfg.ratio_bits, cfg.cheb_deg, cfg.r, float(cfg.log2_s_eval),
                     cfg.correct_bits)
        _check(lib().he_boot_setup(self.h, ctypes.byref(c)))

    def bootstrap(self, a, bound: float):
        return self._op("he_bootstrap", a.h, float(bound))

    def keygen_galois(self, kidx: int, galois: int):
        _check(lib().he_keygen_galois(self.h, int(kidx), ctypes.c_uint64(int(galois))))

    def rotate_gal(self, a, kidx: int, galois: int):
        return self._op("he_rotate_gal", a.h, int(kidx), ctypes.c_uint64(int(galois)))

    def mul_plain(self, a, m, pscale: float):
        m = np.ascontiguousarray(m, dtype=np.int64)
        assert m.size == self.N
        return self._op("he_mul_plain", a.h, m.ctypes.data_as(_c_i64p), float(pscale))

    def modraise(self, a, level: int, scale: float):
        return self._op("he_modraise", a.h, int(level), float(scale))

    # measurement ---------------------------------------------------------------
    def bench_ntt(self, vectors: int, iters: int):
        f, i = ctypes.c_double(), ctypes.c_double()
        _check(lib().he_bench_ntt(self.h, vectors, iters, ctypes.byref(f), ctypes.byref(i)))
        return f.value, i.value

    def bench_copy(self, vectors: int, iters: int) -> float:
        v = ctypes.c_double()
        _check(lib().he_bench_copy(self.h, vectors, iters, ctypes.byref(v)))
        return v.value

    def last_cutmax_ms(self) -> float:
        v = ctypes.c_double()
        _check(lib().he_last_cutmax_ms(self.h, ctypes.byref(v)))
        return v.value

    def sync(self):
        _check(lib().he_sync(self.h))

    def set_option(self, opt: int, value: int):
        _check(lib().he_set_option(self.h, opt, int(value)))

    def ntt_tuning(self):
        v = (ctypes.c_int32 * 8)()
        _check(lib().he_ntt_tuning(self.h, v, 8))
        return list(v)

    def ntt_tuning_report(self) -> dict:
        """every NTT schedule candidate the autotuner timed, per batch bucket"""
        import json
        buf = ctypes.create_string_buffer(1 << 14)
        _check(lib().he_ntt_tuning_report(self.h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def profile_begin(self):
        _check(lib().he_profile_begin(self.h))

    def profile_end(self) -> dict:
        import json
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().he_profile_end(self.h, buf, len(buf)))
        return {k: (v[0], v[1], v[2]) for k, v in json.loads(buf.value.decode()).items()}


_c_fp = ctypes.POINTER(ctypes.c_float)
MLP_NPARAM = 321


def _mlp_lib():
    L = lib()
    if not getattr(L, "_mlp_ready", False):
        sig = {
            "he_mlp_create": [ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_V)],
            "he_mlp_set_params": [_V, _c_fp, ctypes.c_size_t, ctypes.c_float, ctypes.c_float],
            "he_mlp_get_params": [_V, _c_fp, ctypes.c_size_t, _c_fp, _c_fp],
            "he_mlp_grad": [_V, _c_fp, ctypes.c_size_t, _c_fp, _c_fp],
            "he_mlp_forward": [_V, _c_fp, ctypes.c_size_t, _c_fp],
            "he_mlp_train": [_V, _c_fp, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_float,
                             ctypes.c_uint64, _c_fp],
            "he_mlp_to_poly": [_V, _c_dp],
            "he_mlp_save": [_V, ctypes.c_char_p],
            "he_mlp_load": [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(_V)],
            "he_mlp_file_poly": [ctypes.c_char_p, _c_dp],
            "he_variance_log": [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_int, _c_fp, _c_fp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.he_mlp_destroy.argtypes = [_V]
        L.he_mlp_destroy.restype = None
        L.he_mlp_last_error.restype = ctypes.c_char_p
        L._mlp_ready = True
    return L


def _mcheck(rc: int):
    if rc != HE_OK:
        raise HeError(rc, _mlp_lib().he_mlp_last_error().decode())


def _fp(a):
    return a.ctypes.data_as(_c_fp)


class InvSqrtMLP:
    """The learned initial guess (he_mlp): FP32 training on the GPU, collapse to a quartic."""

    def __init__(self, seed: int = 0, device: int = 0, _handle=None):
        if _handle is not None:
            self.h = _handle
            return
        h = _V()
        _mcheck(_mlp_lib().he_mlp_create(seed, device, ctypes.byref(h)))
        self.h = h

    @classmethod
    def load(cls, path: str, device: int = 0) -> "InvSqrtMLP":
        """a network from a file written by save (he_mlp_load)"""
        h = _V()
        _mcheck(_mlp_lib().he_mlp_load(os.fsencode(path), device, ctypes.byref(h)))
        return cls(_handle=h)

    def save(self, path: str):
        """weights, normalisation and collapsed quartic to `path` (he_mlp_save)"""
        _mcheck(_mlp_lib().he_mlp_save(self.h, os.fsencode(path)))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                _mlp_lib().he_mlp_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def set_params(self, theta, mean: float, sd: float):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        _mcheck(_mlp_lib().he_mlp_set_params(self.h, _fp(t), t.size, mean, sd))

    def get_params(self):
        t = np.empty(MLP_NPARAM, dtype=np.float32)
        m, s = ctypes.c_float(), ctypes.c_float()
        _mcheck(_mlp_lib().he_mlp_get_params(self.h, _fp(t), t.size, ctypes.byref(m), ctypes.byref(s)))
        return t, m.value, s.value

    def grad(self, u):
        u = np.ascontiguousarray(u, dtype=np.float32)
        g = np.empty(MLP_NPARAM, dtype=np.float32)
        loss = ctypes.c_float()
        _mcheck(_mlp_lib().he_mlp_grad(self.h, _fp(u), u.size, ctypes.byref(loss), _fp(g)))
        return loss.value, g

    def forward(self, u):
        u = np.ascontiguousarray(u, dtype=np.float32)
        y = np.empty_like(u)
        _mcheck(_mlp_lib().he_mlp_forward(self.h, _fp(u), u.size, _fp(y)))
        return y

    def train(self, u, epochs: int = 20, batch: int = 1024, lr: float = 1e-2, seed: int = 0) -> float:
        u = np.ascontiguousarray(u, dtype=np.float32)
        loss = ctypes.c_float()
        _mcheck(_mlp_lib().he_mlp_train(self.h, _fp(u), u.size, epochs, batch, lr, seed, ctypes.byref(loss)))
        return loss.value

    def to_poly(self) -> np.ndarray:
        c = np.empty(5, dtype=np.float64)
        _mcheck(_mlp_lib().he_mlp_to_poly(self.h, _dp(c)))
        return c


def mlp_file_poly(path: str) -> np.ndarray:
    """the collapsed quartic c0..c4 stored in a learned-guess file (he_mlp_file_poly; no GPU)"""
    c = np.empty(5, dtype=np.float64)
    _mcheck(_mlp_lib().he_mlp_file_poly(os.fsencode(path), _dp(c)))
    return c


def variance_log(seed: int, runs: int, vocab: int = 32000, slots: int = 32768, T: int = 3, p: int = 3,
                 c: float = 5.0, device: int = 0):
    """Variances entering each iteration of `runs` plaintext CutMax runs (GPU), and the
    mean of the last iterate."""
    v = np.empty((runs, T), dtype=np.float32)
    ym = np.empty(runs, dtype=np.float32)
    _mcheck(_mlp_lib().he_variance_log(seed, runs, vocab, slots, T, p, c, device, _fp(v), _fp(ym)))
    return v, ym


def gumbel_noise(u: np.ndarray) -> np.ndarray:
    """Client helper: G = -ln(-ln U) (Sec. 3.3, Gumbel definition)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    g = np.empty_like(u)
    _check(lib().he_gumbel_noise(_dp(u), u.size, _dp(g)))
    return g


def topp_noise(top_p: float, u: np.ndarray) -> np.ndarray:
    """Client helper: G = U^(1/alpha), alpha = ln(1-p)/ln p (Alg. 3 lines 1-4)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    g = np.empty_like(u)
    _check(lib().he_topp_noise(float(top_p), _dp(u), u.size, _dp(g)))
    return g


def invsqrt_guess_fit(u_lo: float, degree: int) -> np.ndarray:
    """Host helper: power-basis coefficients of the Chebyshev interpolant of u^(-1/2) on
    [u_lo, 1] (the fixed initial guess he_cutmax uses when no coefficients are given)."""
    c = np.empty(degree + 1, dtype=np.float64)
    _check(lib().he_invsqrt_guess_fit(float(u_lo), int(degree), _dp(c)))
    return c


def invsqrt_scaled_plan(u_lo: float, degree: int, K: int):
    """Host helper: (guess coefficients, [(a_k, b_k)], [(l_k, h_k)]) of the wide-domain
    inverse square root on [u_lo, 1] (he_invsqrt_scaled_plan)."""
    c = np.empty(degree + 1, dtype=np.float64)
    st = np.empty(max(1, 2 * K), dtype=np.float64)
    rg = np.empty(2 * (K + 1), dtype=np.float64)
    _check(lib().he_invsqrt_scaled_plan(float(u_lo), int(degree), int(K), _dp(c), _dp(st), _dp(rg)))
    return c, [tuple(st[2 * k:2 * k + 2]) for k in range(K)], [tuple(rg[2 * k:2 * k + 2]) for k in range(K + 1)]
