"""O1: plaintext CutMax in float64 -- test infrastructure, not part of the product.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg
may import this module.  It shares no code with the HIP path.

Two forms of Algorithm 1 (CutMax) are given:

* ``cutmax_exact``  -- Algorithm 1 with the true 1/sqrt(var) and the true
  division by the sum (Sec. 3.1, Alg. 1; c-semi-standardisation of App. E, Def.
  "c-semi-standardization").  It defines the arg-max the method must recover.
* ``cutmax_mirror`` -- the same iteration with the polynomial inverse square
  root and the Goldschmidt inverse that the encrypted schedule evaluates
  (Sec. 3.2, Alg. 2; App. B.1 for the Goldschmidt product).  It is the binding
  reference for decrypted results: the difference between it and a decryption
  is CKKS error only.

Readings of the paper used here:

* Alg. 1 normalises ``Y^(T)`` although the loop last writes ``Y^(T+1)``; the
  last computed iterate is normalised (otherwise the last iteration is wasted).
* mean and variance are population moments over every slot of the packed
  vector (Alg. 1 lines 3-4; App. E preliminaries), pad slots included.
* the range-scaled inverse square root is ``invsqr(x/b)/sqrt(b)`` (Sec. 3.2,
  condition (ii) writes ``/b``, which is the scaling for ``inv``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


# ----------------------------------------------------------------------------
# packing
# ----------------------------------------------------------------------------
def slot_layout(x: np.ndarray, slots: int, pad: float = 0.0):
    """Pack a length-n vector into a*slots CKKS slots.

    If n divides ``slots`` the vector is replicated slots/n times (mean and
    variance are then exactly those of x); otherwise it is padded with ``pad``
    up to a = ceil(n/slots) ciphertexts (Sec. 3.2 assumes n = a*s; App. D,
    Fig. 6a splits n > s over several ciphertexts).
    Returns (packed vector, a, replicated).
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n <= slots and slots % n == 0:
        return np.tile(x, slots // n), 1, True
    a = -(-n // slots)
    y = np.full(a * slots, pad, dtype=np.float64)
    y[:n] = x
    return y, a, False


# ----------------------------------------------------------------------------
# Algorithm 1, exact form
# ----------------------------------------------------------------------------
def _per_iter(v, T):
    if np.isscalar(v):
        return [v] * T
    v = list(v)
    assert len(v) == T
    return v


@dataclass
class Trace:
    mean: List[float] = field(default_factory=list)
    var: List[float] = field(default_factory=list)
    z_min: List[float] = field(default_factory=list)
    ys: List[np.ndarray] = field(default_factory=list)


def semi_standardize(y: np.ndarray, c: float) -> np.ndarray:
    """S_c(y)_i = (y_i - mu_y) / (c sigma_y) + 1 with population moments (App. E)."""
    mu = y.mean()
    sd = math.sqrt(((y - mu) ** 2).mean())
    return (y - mu) / (c * sd) + 1.0


def cutmax_exact(x: np.ndarray, p, c, T: int, trace: Optional[Trace] = None) -> np.ndarray:
    """Algorithm 1: T rounds of y <- S_c(y)^p, then Z = y / sum(y)."""
    ps, cs = _per_iter(p, T), _per_iter(c, T)
    y = np.asarray(x, dtype=np.float64).copy()
    for t in range(T):
        mu = y.mean()
        var = ((y - mu) ** 2).mean()
        z = (y - mu) / (cs[t] * math.sqrt(var)) + 1.0
        if trace is not None:
            trace.mean.append(float(mu))
            trace.var.append(float(var))
            trace.z_min.append(float(z.min()))
        y = z ** int(ps[t])
        if trace is not None:
            trace.ys.append(y.copy())
    return y / y.sum()


# ----------------------------------------------------------------------------
# polynomial building blocks (App. B.1)
# ----------------------------------------------------------------------------
def goldschmidt_factor(e, d: int):
    """prod_{i=0}^{d} (1 + e^(2^i)); equals 1/x for e = 1 - x in the limit (App. B.1)."""
    f = 1.0 + e
    ei = e
    for _ in range(d):
        ei = ei * ei
        f = f * (1.0 + ei)
    return f


def chebyshev_invsqrt(u_lo: float, degree: int, scale: float = 1.0) -> np.ndarray:
    """Power-basis coefficients a_0..a_d of the polynomial interpolating
    scale/sqrt(u) at the degree+1 Chebyshev nodes of the first kind on [u_lo, 1]."""
    d = int(degree)
    k = np.arange(d + 1)
    t = np.cos(np.pi * (k + 0.5) / (d + 1))
    u = 0.5 * (1.0 + u_lo) + 0.5 * (1.0 - u_lo) * t
    f = scale / np.sqrt(u)
    V = np.vander(u, d + 1, increasing=True)
    return np.linalg.solve(V, f)


def poly_eval(coef: Sequence[float], u):
    """sum_k coef[k] u^k."""
    acc = 0.0
    for k in range(len(coef) - 1, -1, -1):
        acc = acc * u + coef[k]
    return acc


def newton_invsqrt_step(h, u, C: float):
    """One Newton step for h ~ C/sqrt(u):  h <- 1.5 h - (0.5/C^2) u h^3."""
    return 1.5 * h - (0.5 / (C * C)) * u * h * h * h


def goldschmidt_invsqrt(x, y0, K: int):
    """Goldschmidt's inverse-square-root iteration (the invsqr method App. B.1 cites):
    b_0 = x y_0^2;  r_k = (3 - b_k)/2;  y_{k+1} = y_k r_k;  b_{k+1} = b_k r_k^2.
    y_K approximates 1/sqrt(x); b_k stays equal to x y_k^2."""
    y = y0
    b = x * y0 * y0
    for _ in range(K):
        r = (3.0 - b) / 2.0
        y = y * r
        b = b * r * r
    return y


def scaled_newton_step(l: float, h: float):
    """One refinement x -> x (a - b x^2) of x = y sqrt(u) (y ~ u^(-1/2)) chosen for the
    range [l, h] of x (0 < l < h): the cubic's maximum sits at m = sqrt(a / 3b) and it
    equioscillates, f(l) = f(h) = 1 - delta and f(m) = 1 + delta, so [l, h] maps onto
    [1 - delta, 1 + delta] with the smallest delta a cubic of this form reaches.  From
    f(l) = f(h): a = b (h^2 + h l + l^2); then m^2 = (h^2 + h l + l^2) / 3, f(m) = 2 b m^3 and
    f(l) = b l h (h + l); 1 - delta + 1 + delta = 2 gives b.  a = 1.5, b = 0.5 (Newton's
    step for the inverse square root) is the limit l, h -> 1.
    Returns (a, b, 1 - delta, 1 + delta)."""
    s2 = h * h + h * l + l * l
    m3 = (s2 / 3.0) ** 1.5
    b = 2.0 / (l * h * (h + l) + 2.0 * m3)
    a = b * s2
    delta = 1.0 - b * l * h * (h + l)
    return a, b, 1.0 - delta, 1.0 + delta


def guess_range(coef: Sequence[float], u_lo: float, points: int = 20001, margin: float = 1e-3):
    """[min, max] of x = g(u) sqrt(u) over [u_lo, 1] on a geometric grid, widened by a
    relative margin (the range only picks the refinement constants and the bootstrap bounds)."""
    u = np.geomspace(u_lo, 1.0, points)
    x = poly_eval(coef, u) * np.sqrt(u)
    if x.min() <= 0:
        raise DomainError("initial guess not positive on the domain")
    return float(x.min()) * (1.0 - margin), float(x.max()) * (1.0 + margin)


def scaled_invsqrt_plan(u_lo: float, degree: int, K: int):
    """Wide-domain inverse square root on [u_lo, 1]: the degree-d Chebyshev guess g, then
    K refinements x -> x (a_k - b_k x^2) each chosen for the range of x it receives.
    Returns (g, [(a_k, b_k)], [(l_k, h_k)] for k = 0..K: the range before step k and after
    the last)."""
    g = chebyshev_invsqrt(u_lo, degree)
    lo, hi = guess_range(g, u_lo)
    steps, ranges = [], [(lo, hi)]
    for _ in range(K):
        a, b, lo, hi = scaled_newton_step(lo, hi)
        steps.append((a, b))
        ranges.append((lo, hi))
    return g, steps, ranges


def scaled_invsqrt(u, g: Sequence[float], steps) -> np.ndarray:
    """g(u) refined by the coupled form of the steps: y = g(u), w = u y^2 (= x^2), then per
    step r = a - b w, y <- y r, w <- w r^2.  Approximates u^(-1/2)."""
    y = poly_eval(g, u)
    w = u * y * y
    for a, b in steps:
        r = a - b * w
        y = y * r
        w = w * r * r
    return y


# ----------------------------------------------------------------------------
# Algorithm 2 mirrored in the clear
# ----------------------------------------------------------------------------
@dataclass
class MirrorCfg:
    T: int
    p: Sequence[int]
    c: Sequence[float]
    v_hi: Sequence[float]          # invsqr domain upper bound per iteration (variance units)
    v_lo: Sequence[float]          # lower bound (checked, used for the default fit)
    coef: Sequence[Sequence[float]]  # initial guess g(u) ~ u^(-1/2) per iteration, power basis
    #                                  in u = var/v_hi; the schedule multiplies by C_t = sqrt(n)/c_t
    newton: int = 0                # refinement steps after the initial guess
    goldschmidt: bool = False      # refine with Goldschmidt's iteration instead of Newton's
    B: float = 1.0                 # final sum is mapped to x = S/B in (0, 1]
    gold_d: int = 3                # Goldschmidt degree (d+1 factors)
    sum_lo: float = 0.0
    scaled: Optional[Sequence[Sequence[Sequence[float]]]] = None  # per iteration, (a_k, b_k) of the
    #                                  scaled refinements after the guess (replaces newton)


class DomainError(ValueError):
    """A variance or sum left the declared approximation domain (Sec. 3.2, (ii))."""


def cutmax_mirror(y0: np.ndarray, cfg: MirrorCfg, check: bool = True,
                  trace: Optional[Trace] = None) -> np.ndarray:
    """The encrypted CutMax schedule evaluated in float64 on the packed vector y0.

    Per iteration (Alg. 2 lines 3-7, with the constants folded as the
    encrypted schedule folds them):
        u  = var / v_hi                     (variance mapped into (0, 1])
        h  = poly(u) [+ Newton or Goldschmidt steps]  ~ (sqrt(n)/c) / sqrt(u)
        z  = (y - mu) / sqrt(n v_hi) * h + 1   == (y - mu)/(c sigma) + 1 when h is exact
        y  = z^p
    then (Alg. 2 line 8) Z = (y / B) * prod_i (1 + e^(2^i)),  e = 1 - sum(y)/B.
    """
    y = np.asarray(y0, dtype=np.float64).copy()
    n = y.size
    for t in range(cfg.T):
        mu = y.mean()
        var = ((y - mu) ** 2).mean()
        if check and not (cfg.v_lo[t] <= var <= cfg.v_hi[t]):
            raise DomainError(f"iteration {t}: variance {var} outside [{cfg.v_lo[t]}, {cfg.v_hi[t]}]")
        u = var / cfg.v_hi[t]
        C = math.sqrt(n) / cfg.c[t]
        h = poly_eval([g * C for g in cfg.coef[t]], u)
        if cfg.scaled is not None:
            h = C * scaled_invsqrt(u, cfg.coef[t], cfg.scaled[t])
        elif cfg.goldschmidt:
            h = C * goldschmidt_invsqrt(u, h / C, cfg.newton)
        else:
            for _ in range(cfg.newton):
                h = newton_invsqrt_step(h, u, C)
        z = (y - mu) / math.sqrt(n * cfg.v_hi[t]) * h + 1.0
        if trace is not None:
            trace.mean.append(float(mu))
            trace.var.append(float(var))
            trace.z_min.append(float(z.min()))
        y = z ** int(cfg.p[t])
        if trace is not None:
            trace.ys.append(y.copy())
    S = y.sum()
    if check and not (cfg.sum_lo <= S <= cfg.B):
        raise DomainError(f"final sum {S} outside [{cfg.sum_lo}, {cfg.B}]")
    e = 1.0 - S / cfg.B
    return (y / cfg.B) * goldschmidt_factor(e, cfg.gold_d)


# ----------------------------------------------------------------------------
# theory (App. E)
# ----------------------------------------------------------------------------
def tmin(n: int, p: int, c: float, delta: float, k: float) -> int:
    """Iterations sufficient for a gap ratio >= k (Theorem "CutMax Convergence",
    bound with Gamma^(0) >= 1): ceil(ln k / (p ln(1 + delta/(c + sqrt n))))."""
    return int(math.ceil(math.log(k) / (p * math.log1p(delta / (c + math.sqrt(n))))))


def top2(y: np.ndarray):
    """(i*, i**): index of the maximum and of the runner-up (App. E, Def. "Max elements")."""
    order = np.argsort(y)
    return int(order[-1]), int(order[-2])


def delta_gap(y: np.ndarray) -> float:
    """Largest delta with y_{i*} - y_{i**} >= delta * sigma_y (App. E, Def. "delta-gap bound")."""
    i1, i2 = top2(y)
    return float((y[i1] - y[i2]) / y.std())


def gap_ratio(y: np.ndarray) -> float:
    """Gamma(y) = y_{i*} / y_{i**} (App. E, Def. "Gap Ratio")."""
    i1, i2 = top2(y)
    return float(y[i1] / y[i2])


# ----------------------------------------------------------------------------
# nucleus sampler pieces (Sec. 3.3, Lemma "Beta", Alg. 3)
# ----------------------------------------------------------------------------
def beta_alpha(top_p: float) -> float:
    """alpha = ln(1-p)/ln(p), so that G ~ Beta(alpha,1) has P(G > p) = p (Lemma "Beta")."""
    return math.log(1.0 - top_p) / math.log(top_p)


def beta_noise(u: np.ndarray, alpha: float) -> np.ndarray:
    """Inverse CDF of Beta(alpha, 1): F^{-1}(u) = u^(1/alpha) (Alg. 3, line 4)."""
    return np.power(u, 1.0 / alpha)


def nucleus_argmax(x: np.ndarray, g: np.ndarray, temperature: float) -> int:
    """The token a one-shot sampler selects: argmax(x/temperature + G) (Alg. 3 with Beta
    noise; the Gumbel-max trick of Sec. 3.3 with Gumbel noise)."""
    return int(np.argmax(np.asarray(x) / temperature + np.asarray(g)))


def gumbel_noise(u: np.ndarray) -> np.ndarray:
    """G = -ln(-ln U) turns U ~ Uniform(0,1) into Gumbel(0,1) (Sec. 3.3, Gumbel definition)."""
    return -np.log(-np.log(np.asarray(u, dtype=np.float64)))


def violation_rate(x: np.ndarray, picks: Sequence[int], top_p: float, temperature: float = 1.0) -> float:
    """Fraction of sampled tokens outside the top-p nucleus of softmax(x/temperature)
    (the measure of Sec. 4, "Nucleus Sampling", Fig. 4)."""
    inside = np.zeros(np.asarray(x).size, dtype=bool)
    inside[nucleus_set(x, top_p, temperature)] = True
    picks = np.asarray(picks, dtype=np.int64)
    return float(1.0 - inside[picks].mean()) if picks.size else 0.0


def nucleus_set(x: np.ndarray, top_p: float, temperature: float = 1.0) -> np.ndarray:
    """Indices of the smallest top-ranked set whose softmax mass reaches top_p."""
    z = np.asarray(x, dtype=np.float64) / temperature
    pr = np.exp(z - z.max())
    pr /= pr.sum()
    order = np.argsort(-pr)
    cum = np.cumsum(pr[order])
    k = int(np.searchsorted(cum, top_p) + 1)
    return order[:k]
