"""More pins of the CPU RNS-CKKS oracle (O2), for the parts the GPU path is compared against
word for word: every initial-guess degree of the encrypted inverse square root (Alg. 2
line 5, App. B.1) against the FP64 polynomial, the odd and even powers (Alg. 2 line 7)
against y^p, the nucleus sampler's server step (Alg. 3) against CutMax of x + tau G, and the
kernel-shaped schedule (hoisted rotate-and-sum, relinearisation with the rescale folded into
its ModDown) against the plain form of Sec. 3.2 (one rotation per bit, relinearise then
rescale) on the same ciphertext."""
import math

import numpy as np
import pytest

from oracle import ckks
from oracle.cutmax_fp64 import (MirrorCfg, beta_alpha, beta_noise, chebyshev_invsqrt, cutmax_mirror, poly_eval,
                                slot_layout)
from workloads import toy_logits, uniform_noise

TOY = ckks.Params(log_n=10, n_q=8, q0_bits=40, q_bits=30, p_bits=40, dnum=3, log2_scale=30, seed=3)
# the toy CutMax chain of the GPU tests (N = 2^12, 35 scaling primes of 30 bits)
CFG1 = ckks.Params(log_n=12, n_q=36, q0_bits=40, q_bits=30, p_bits=40, dnum=3, log2_scale=30, seed=7, hoist=3)


@pytest.fixture(scope="module")
def toy():
    O = ckks.Oracle(TOY)
    O.keygen(True, range(int(math.log2(O.slots))))
    return O


@pytest.fixture(scope="module")
def cfg1():
    O = ckks.Oracle(CFG1)
    O.keygen_cutmax()
    return O


DEPTH = {1: 1, 2: 2, 3: 2, 4: 3}


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
@pytest.mark.parametrize("kind", ["chebyshev", "generic"])
def test_encrypted_initial_guess_every_degree(toy, degree, kind):
    """the encrypted initial guess sum_k a_k u^k (no refinement) decrypts to the FP64
    polynomial on the same u, at level L - depth (1/2/2/3 for degree 1/2/3/4) and at the
    requested scale; every term contributes far more than the tolerance, so a dropped or
    mis-scaled term fails"""
    rng = np.random.default_rng(100 + degree)
    u = rng.uniform(0.3, 1.0, toy.slots)
    C = 2.0
    if kind == "chebyshev":
        coef = list(chebyshev_invsqrt(0.3, degree))
    else:
        coef = list(rng.uniform(0.2, 0.9, degree + 1) * np.where(np.arange(degree + 1) % 2, -1.0, 1.0))
    tol = 2e-4
    ref = C * poly_eval(coef, u)
    for k in range(degree + 1):
        assert np.abs(C * coef[k] * u ** k).min() > 50 * tol, (k, coef)
    H = toy.invsqr(toy.encrypt(u), [g * C for g in coef], C, 0, toy.Delta)
    assert H.level == toy.L - DEPTH[degree] == toy.L - ckks.invsqr_depth(degree, 0)
    assert abs(H.scale / toy.Delta - 1) < 1e-12
    np.testing.assert_allclose(toy.decrypt(H), ref, atol=tol)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7])
def test_encrypted_power(toy, p):
    """y^p by repeated squaring (Alg. 2 line 7): decrypts to y^p, in floor(log2 p) squarings
    plus one level when p is not a power of two"""
    y = np.random.default_rng(200 + p).uniform(0.5, 1.5, toy.slots)
    Y = toy.power(toy.encrypt(y), p)
    depth = (p.bit_length() - 1) + (1 if bin(p).count("1") > 1 else 0)
    assert Y.level == toy.L - depth
    np.testing.assert_allclose(toy.decrypt(Y), y ** p, atol=1e-3 * 1.5 ** p)


def _toy_cutmax_cfg(T):
    p, c = [3] * T, [5.0] * T
    vlo, vhi = [0.5, 0.25, 0.3, 0.6][:T], [2.0, 0.75, 3.0, 128.0][:T]
    coef = [list(chebyshev_invsqrt(vlo[t] / vhi[t], 3)) for t in range(T)]
    return p, c, vlo, vhi, coef


@pytest.mark.parametrize("prescaled", [False, True])
def test_topp_server_step_is_cutmax_of_noisy_logits(cfg1, prescaled):
    """Alg. 3 server side: the encrypted CutMax(X + tau G) decrypts to the FP64 mirror of
    CutMax on x + tau g (within 1e-3) and its argmax is the sampler's pick argmax(x/tau + g)
    on the same noise; the input step decrypts to x + tau g (the temperature multiply
    costs one level unless the noise is pre-scaled)"""
    O = cfg1
    T, tau, top_p = 2, 0.8, 0.9
    x = toy_logits(61)
    g = beta_noise(uniform_noise(62, x.size), beta_alpha(top_p))
    y, _, _ = slot_layout(x, O.slots)
    gy, _, _ = slot_layout(g, O.slots)
    p, c, vlo, vhi, coef = _toy_cutmax_cfg(T)
    hc = ckks.HECfg(T=T, p=p, c=c, v_lo=vlo, v_hi=vhi, coef=coef, sum_lo=1.0, sum_hi=3.0, gold_d=3)
    X = O.encrypt(y)
    Gn = O.encrypt(tau * gy if prescaled else gy)
    Z = ckks.topp_he(O, [X], [Gn], tau, hc, prescaled=prescaled)[0]
    assert Z.level == O.L - hc.levels_needed() - (0 if prescaled else 1)
    dz = O.decrypt(Z)
    n = y.size
    mc = MirrorCfg(T=T, p=p, c=c, v_hi=vhi, v_lo=vlo, coef=coef, B=3.0 * n, gold_d=3, sum_lo=1.0 * n)
    want = cutmax_mirror(y + tau * gy, mc)
    assert np.abs(dz - want).max() < 1e-3
    assert int(np.argmax(dz[:x.size])) == int(np.argmax(x / tau + g))
    # the input step on its own: x + tau g within the fresh CKKS noise at scale 2^30
    Xt = ckks.topp_input(O, [X], [Gn], tau, prescaled)[0]
    np.testing.assert_allclose(O.decrypt(Xt), y + tau * gy, atol=2e-5)


def test_kernel_shaped_schedule_matches_plain_form(cfg1):
    """the oracle's CutMax as the kernels shape it (rotate-and-sum in hoisted radix-8 steps
    with the automorphisms applied to the extended digits; every ciphertext product
    divided by P q_l in one ModDown) against the plain form on the same ciphertext (the
    log2(s) single rotations of Sec. 3.2, relinearisation by P then a rescale by q_l):
    both run the same levels and scales and decrypt to the same Z within 5e-4 (the two
    forms round differently; at scale 2^30 each is 4e-5..2e-4 from the FP64 mirror and
    they differ by 8e-5..2.6e-4 over seeds 63-65, against max Z near 0.17), and each is
    within 1e-3 of the mirror"""
    O = cfg1
    T = 4
    x = toy_logits(63)
    y, _, _ = slot_layout(x, O.slots)
    n = y.size
    p, c, vlo, vhi, coef = _toy_cutmax_cfg(T)
    hc = ckks.HECfg(T=T, p=p, c=c, v_lo=vlo, v_hi=vhi, coef=coef, sum_lo=1.0, sum_hi=3.0, gold_d=3)
    X = O.encrypt(y)
    O.plain = False
    Zk = ckks.cutmax_he(O, [X], hc)[0]
    O.plain = True
    try:
        Zp = ckks.cutmax_he(O, [X], hc)[0]
    finally:
        O.plain = False
    assert Zk.level == Zp.level == O.L - hc.levels_needed()
    assert Zk.scale == Zp.scale
    assert not np.array_equal(Zk.export(), Zp.export())
    dk, dp = O.decrypt(Zk), O.decrypt(Zp)
    assert np.abs(dk - dp).max() < 5e-4, np.abs(dk - dp).max()
    mc = MirrorCfg(T=T, p=p, c=c, v_hi=vhi, v_lo=vlo, coef=coef, B=3.0 * n, gold_d=3, sum_lo=1.0 * n)
    ref = cutmax_mirror(y, mc)
    assert np.abs(dk - ref).max() < 1e-3 and np.abs(dp - ref).max() < 1e-3
    assert int(np.argmax(dk[:x.size])) == int(np.argmax(dp[:x.size])) == int(np.argmax(x))


def test_plain_rotsum_and_mul_match_the_kernel_shaped_ones(cfg1):
    """one rotate-and-sum and one product, plain against kernel-shaped, on the same
    ciphertext at the top level and at a level with a partial digit: the decrypted
    coefficients differ by the noise of the two forms only, far below the scale"""
    O = cfg1
    s1 = int(np.abs(O.secret().astype(np.int64)).sum())
    rng = np.random.default_rng(64)
    x, z = rng.uniform(-1, 1, O.slots), rng.uniform(-1, 1, O.slots)
    cx, cz = O.encrypt(x), O.encrypt(z)
    for lv in (O.L, 4):
        a, b = O.drop(cx, lv), O.drop(cz, lv)
        O.plain = False
        rk, mk = O.rotsum(a), O.mul(a, b)
        O.plain = True
        try:
            rp, mp = O.rotsum(a), O.mul(a, b)
        finally:
            O.plain = False
        assert rk.level == rp.level == lv and mk.level == mp.level == lv - 1
        dr = O.decrypt_coeffs(rk) - O.decrypt_coeffs(rp)
        dm = O.decrypt_coeffs(mk) - O.decrypt_coeffs(mp)
        # the 15 single rotations add and double their key-switch noise one after the
        # other, the hoisted steps add it once per step: the sums differ by up to about
        # 2^17 per coefficient (measured 1.3e5 at level 4), 1e-4 of the scale 2^30; a
        # dropped key or automorphism term would differ by a multiple of the modulus
        assert np.abs(dr).max() < 2.0 ** 18, np.abs(dr).max()
        assert np.abs(O.decrypt(rk) - O.decrypt(rp)).max() < 1e-3
        # one centred rounding against two: below 1 + |s|_1 per coefficient
        assert np.abs(dm).max() < 1 + s1, (np.abs(dm).max(), s1)
        np.testing.assert_allclose(O.decrypt(rp), x.sum(), atol=1e-3)
        np.testing.assert_allclose(O.decrypt(mp), x * z, atol=1e-4)
