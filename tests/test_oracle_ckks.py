"""Pins of the CPU RNS-CKKS oracle (O2) against textbook definitions and the CKKS
properties the paper relies on (Sec. 2.1 correctness/homomorphism; Sec. 3.2 rotations)."""
import dataclasses
import math
import os

import numpy as np
import pytest

from oracle import ckks
from oracle.cutmax_fp64 import (MirrorCfg, chebyshev_invsqrt, cutmax_exact, cutmax_mirror, goldschmidt_invsqrt,
                                newton_invsqrt_step, poly_eval, slot_layout)
from workloads import random_residues, toy_logits

GOLD = os.path.join(os.path.dirname(__file__), "golden")

TOY = ckks.Params(log_n=10, n_q=8, q0_bits=40, q_bits=30, p_bits=40, dnum=3, log2_scale=30, seed=3)
CFG1 = ckks.Params(log_n=12, n_q=36, q0_bits=40, q_bits=30, p_bits=40, dnum=3, log2_scale=30, seed=7)


@pytest.fixture(scope="module")
def toy():
    O = ckks.Oracle(TOY)
    O.keygen(True, range(int(math.log2(O.slots))))
    return O


def test_philox_known_answers():
    with open(os.path.join(GOLD, "philox_kat.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            v = [int(t, 16) for t in ln.split()]
            assert ckks.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def _is_prime_trial(n):
    # independent check: Fermat with many bases plus small-factor trial division
    if any(n % p == 0 for p in range(2, 2000)):
        return False
    return all(pow(a, n - 1, n) == 1 for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41))


def test_primes_are_ntt_friendly():
    O = ckks.Oracle(CFG1)
    assert O.L == 35 and O.alpha == 12 and len(set(O.q)) == O.np
    for i, q in enumerate(O.q):
        bits = 40 if (i == 0 or i > O.L) else 30
        assert q < 2 ** bits and q > 2 ** (bits - 1)
        assert q % (2 * O.N) == 1
        assert _is_prime_trial(q)


@pytest.mark.parametrize("log_n", [3, 4, 6])
def test_ring_mul_matches_schoolbook(log_n):
    """NTT-based negacyclic product == schoolbook convolution mod (X^N + 1, q)."""
    prm = ckks.Params(log_n=log_n, n_q=2, q0_bits=40, q_bits=30, p_bits=40, dnum=1, log2_scale=20)
    O = ckks.Oracle(prm)
    N = O.N
    for pi in range(O.np):
        q = O.q[pi]
        a, b = random_residues(100 + pi, [q, q], N)
        a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
        c1 = np.empty(N, dtype=np.uint64)
        c2 = np.empty(N, dtype=np.uint64)
        ckks.lib().oc_ring_mul(O.h, pi, a.ctypes.data_as(ckks.u64p), b.ctypes.data_as(ckks.u64p),
                               c1.ctypes.data_as(ckks.u64p))
        ckks.lib().oc_schoolbook(a.ctypes.data_as(ckks.u64p), b.ctypes.data_as(ckks.u64p),
                                 c2.ctypes.data_as(ckks.u64p), N, q)
        # independent pure-Python schoolbook as well
        ai, bi = [int(v) for v in a], [int(v) for v in b]
        ref = [0] * N
        for i in range(N):
            for j in range(N):
                k = i + j
                if k < N:
                    ref[k] += ai[i] * bi[j]
                else:
                    ref[k - N] -= ai[i] * bi[j]
        ref = [v % q for v in ref]
        assert [int(v) for v in c2] == ref
        assert [int(v) for v in c1] == ref


def test_encode_decode_routes_agree():
    N, scale = 1024, 2.0 ** 30
    z = np.random.default_rng(0).uniform(-5, 5, N // 2)
    m1 = ckks.encode_direct(z, N, scale)
    m2 = ckks.encode_fft(z, N, scale)
    assert np.abs(m1 - m2).max() <= 1
    np.testing.assert_allclose(ckks.decode_direct(m1, N, scale), z, atol=1e-7)
    np.testing.assert_allclose(ckks.decode_fft(m1, N, scale), z, atol=1e-7)
    # the constant polynomial c*scale decodes to c in every slot
    m = np.zeros(N)
    m[0] = 3 * scale
    np.testing.assert_allclose(ckks.decode_direct(m, N, scale), 3.0, atol=1e-12)


def test_secret_is_ternary(toy):
    s = toy.secret()
    assert set(np.unique(s).tolist()) <= {-1, 0, 1}
    frac = np.bincount(s + 1) / s.size
    assert np.all(np.abs(frac - 1 / 3) < 0.06)


def test_decrypt_encrypt_identity(toy):
    z = np.random.default_rng(1).uniform(-10, 10, toy.slots)
    ct = toy.encrypt(z)
    assert ct.level == toy.L
    np.testing.assert_allclose(toy.decrypt(ct), z, atol=1e-5)
    # fresh encryptions of the same message differ (nonce advances)
    ct2 = toy.encrypt(z)
    assert not np.array_equal(ct.export(), ct2.export())


def test_homomorphic_add_mul_rescale_rotate(toy):
    rng = np.random.default_rng(2)
    x = rng.uniform(-2, 2, toy.slots)
    y = rng.uniform(-2, 2, toy.slots)
    cx, cy = toy.encrypt(x), toy.encrypt(y)
    np.testing.assert_allclose(toy.decrypt(toy.add(cx, cy)), x + y, atol=1e-5)
    np.testing.assert_allclose(toy.decrypt(toy.sub(cx, cy)), x - y, atol=1e-5)
    np.testing.assert_allclose(toy.decrypt(toy.mul_int(cx, -7)), -7 * x, atol=1e-4)
    np.testing.assert_allclose(toy.decrypt(toy.add_const(cx, 1.5)), x + 1.5, atol=1e-5)
    m = toy.mul(cx, cy)
    assert m.level == toy.L - 1
    np.testing.assert_allclose(toy.decrypt(m), x * y, atol=1e-4)
    r = toy.rescale(toy.mul_int(cx, 1 << 30))
    assert r.level == toy.L - 1 and r.scale == toy.Delta / toy.q[toy.L]
    np.testing.assert_allclose(toy.decrypt(r) / 2.0 ** 30, x, atol=1e-4)
    for rr in range(int(math.log2(toy.slots))):
        np.testing.assert_allclose(toy.decrypt(toy.rotate(cx, rr)), np.roll(x, -(1 << rr)), atol=1e-4)
    ce = toy.cm_exact(cx, 0.37, toy.Delta)
    np.testing.assert_allclose(toy.decrypt(ce), 0.37 * x, atol=1e-4)
    ct_ = toy.cm_target(cx, -1.25, 2.0 ** 29)
    assert ct_.scale == 2.0 ** 29
    np.testing.assert_allclose(toy.decrypt(ct_), -1.25 * x, atol=1e-4)


def test_merged_relinearise_rescale_matches_two_steps(toy):
    """mul divides by P q_l in one ModDown; relinearising (ModDown by P) and then
    rescaling (by q_l) gives the same product up to the roundings: a centred rounding of
    (c0, c1) decrypts to an error below (1 + |s|_1)/2 per coefficient, so the decrypted
    coefficients of the two differ by less than 1 + |s|_1 (a dropped term or a wrong
    constant differs by a multiple of the modulus), at the top level and with a partial
    digit"""
    s1 = int(np.abs(toy.secret().astype(np.int64)).sum())
    rng = np.random.default_rng(12)
    x, y = rng.uniform(-2, 2, toy.slots), rng.uniform(-2, 2, toy.slots)
    cx, cy = toy.encrypt(x), toy.encrypt(y)
    for lv in (toy.L, 4):
        a, b = toy.drop(cx, lv), toy.drop(cy, lv)
        merged = toy.mul(a, b)
        two = toy.rescale(ckks.Ct(toy, ckks.lib().oc_mul_norescale(toy.h, a.h, b.h), a.scale * b.scale))
        assert merged.level == two.level == lv - 1
        d = toy.decrypt_coeffs(merged) - toy.decrypt_coeffs(two)
        assert np.abs(d).max() < 1 + s1, (np.abs(d).max(), s1)
        np.testing.assert_allclose(toy.decrypt(merged), x * y, atol=1e-4)


def test_rotate_and_mul_at_low_levels(toy):
    """Partial key-switch digits below the top level still switch keys correctly."""
    x = np.random.default_rng(3).uniform(-1, 1, toy.slots)
    cx = toy.encrypt(x)
    for lv in (1, 2, 3, 5):
        d = toy.drop(cx, lv)
        np.testing.assert_allclose(toy.decrypt(toy.rotate(d, 2)), np.roll(x, -4), atol=1e-4)
        np.testing.assert_allclose(toy.decrypt(toy.mul(d, d)), x * x, atol=1e-4)


def test_rotsum(toy):
    x = np.random.default_rng(4).uniform(-1, 1, toy.slots)
    s = toy.decrypt(toy.rotsum(toy.encrypt(x)))
    np.testing.assert_allclose(s, x.sum(), atol=1e-3)


@pytest.mark.parametrize("h", [1, 2, 3])
def test_hoist_plan_covers_every_shift_once(h):
    """picking one amount (or none) per step of the hoisted plan gives every shift
    0..slots-1 exactly once, which is what makes the steps a rotate-and-sum"""
    for slots in (2, 8, 512, 2048, 32768):
        sums = [0]
        for step in ckks.hoist_steps(slots, h):
            sums = [s + a for s in sums for a in [0] + step]
        assert sorted(sums) == list(range(slots))
        keys = ckks.rotation_keys(slots, h)
        lg = int(math.log2(slots))
        assert all(keys[1 << e] == 1 + e for e in range(lg))
        assert sorted(keys.values()) == list(range(1, 1 + len(keys)))


@pytest.mark.parametrize("h", [1, 2, 3])
def test_hoisted_rotsum_gives_the_slot_sum(h):
    O = ckks.Oracle(dataclasses.replace(TOY, hoist=h))
    O.keygen_cutmax()
    x = np.random.default_rng(40 + h).uniform(-1, 1, O.slots)
    cx = O.encrypt(x)
    np.testing.assert_allclose(O.decrypt(O.rotsum(cx)), x.sum(), atol=1e-3)
    # one step on its own, at a level with a partial last digit
    keys = ckks.rotation_keys(O.slots, h)
    amounts = ckks.hoist_steps(O.slots, h)[0]
    d = O.drop(cx, 4)
    want = x + sum(np.roll(x, -a) for a in amounts)
    np.testing.assert_allclose(O.decrypt(O.rotsum_step(d, amounts, keys)), want, atol=1e-4)


@pytest.mark.parametrize("h", [2, 3])
def test_carried_rotsum_equals_the_step_by_step_form(h):
    """c0 carried as P c0 over Q u P between hoisted steps, one ModDown at the end: the same
    rotations as a ModDown per step (the sum of x over every rotation of every step), so
    both decrypt to the slot sum; they differ only by the ModDowns' rounding, on the order
    of the encryption noise (2^-30 scale on the toy chain), also at a level whose last
    digit is partial.  A carried c0 missing its factor P (or a step's rotated copies)
    would be off by the whole slot sum."""
    O = ckks.Oracle(dataclasses.replace(TOY, hoist=h))
    O.keygen_cutmax()
    x = np.random.default_rng(70 + h).uniform(-1, 1, O.slots)
    keys = ckks.rotation_keys(O.slots, h)
    steps = ckks.hoist_steps(O.slots, h)
    assert len(steps) >= 2
    for lv in (O.L, 4):
        cx = O.drop(O.encrypt(x), lv)
        stepwise = cx
        for amounts in steps:
            stepwise = O.rotsum_step(stepwise, amounts, keys)
        carried = O.rotsum_carried(cx, steps, keys)
        assert carried.level == lv
        dc, ds = O.decrypt(carried), O.decrypt(stepwise)
        np.testing.assert_allclose(dc, x.sum(), atol=1e-3)
        assert np.abs(dc - ds).max() < 1e-5


def test_tampered_limb_is_detected(toy):
    x = np.random.default_rng(5).uniform(-1, 1, toy.slots)
    ct = toy.encrypt(x)
    limbs = ct.export()
    limbs[0, 0, 10] = (int(limbs[0, 0, 10]) + 12345) % toy.q[0]
    bad = toy.import_ct(limbs, ct.scale)
    assert np.abs(toy.decrypt(bad) - x).max() > 1e-3


def _cfg1_schedule(O, y, T=4):
    n = y.size
    p, c = [3] * T, [5.0] * T
    vlo, vhi = [0.5, 0.25, 0.3, 0.6][:T], [2.0, 0.75, 3.0, 128.0][:T]
    coef = [chebyshev_invsqrt(vlo[t] / vhi[t], 3) for t in range(T)]
    he = ckks.HECfg(T=T, p=p, c=c, v_lo=vlo, v_hi=vhi, coef=coef, sum_lo=1.0, sum_hi=3.0, gold_d=3)
    mc = MirrorCfg(T=T, p=p, c=c, v_hi=vhi, v_lo=vlo, coef=coef, B=3.0 * n, gold_d=3, sum_lo=1.0 * n)
    return he, mc


@pytest.mark.slow
def test_he_cutmax_matches_mirror_config1():
    """Alg. 2 on the oracle CKKS: decrypted Z within 1e-3 of the FP64 mirror, argmax recovered."""
    O = ckks.Oracle(CFG1)
    O.keygen_cutmax()
    x = toy_logits(11)
    y, a, rep = slot_layout(x, O.slots)
    he, mc = _cfg1_schedule(O, y)
    assert he.levels_needed() <= O.L
    Z = ckks.cutmax_he(O, [O.encrypt(y)], he)
    dz = O.decrypt(Z[0])
    assert np.abs(dz - cutmax_mirror(y, mc)).max() < 1e-3
    assert int(np.argmax(dz[:x.size])) == int(np.argmax(x))
    assert abs(dz.sum() - 1) < 1e-2
    # and the exact Algorithm 1 picks the same index
    assert int(np.argmax(cutmax_exact(y, 3, 5.0, 4))) == int(np.argmax(x))


def test_schedule_rejects_short_chain(toy):
    x = toy_logits(1, 512)
    he, _ = _cfg1_schedule(toy, x)
    with pytest.raises(ckks.SchedError):
        ckks.cutmax_he(toy, [toy.encrypt(x)], he)


@pytest.mark.parametrize("gold", [False, True])
def test_encrypted_invsqr_refinements(toy, gold):
    """the encrypted inverse square root (degree-1 guess + 2 refinements, Newton or
    Goldschmidt) decrypts to the FP64 iteration on the same u and lands at the requested
    scale; Goldschmidt takes one level more"""
    u = np.random.default_rng(4).uniform(0.3, 1.0, toy.slots)
    C = 2.0
    coef = chebyshev_invsqrt(0.3, 1)
    H = toy.invsqr(toy.encrypt(u), [g * C for g in coef], C, 2, toy.Delta, goldschmidt=gold)
    assert H.level == toy.L - ckks.invsqr_depth(1, 2, gold)
    assert H.level == toy.L - (6 if gold else 5)
    assert abs(H.scale / toy.Delta - 1) < 1e-12
    h0 = poly_eval(coef, u)
    if gold:
        ref = C * goldschmidt_invsqrt(u, h0, 2)
    else:
        ref = C * newton_invsqrt_step(newton_invsqrt_step(h0, u, 1.0), u, 1.0)
    np.testing.assert_allclose(toy.decrypt(H), ref, atol=1e-3)
    assert np.abs(ref * np.sqrt(u) / C - 1).max() < 2e-3


@pytest.mark.slow
def test_masked_padding_gives_cutmax_of_the_logits_alone():
    """Masked padding: 1500 all-negative logits padded (with their mean) to 2048 slots;
    the encrypted schedule with the pad tracker decrypts, on the first 1500 slots, to the
    FP64 mirror run on the 1500 logits alone (another vector length), and recovers the
    argmax; without masking the pad slots would enter mean and variance"""
    O = ckks.Oracle(ckks.Params(log_n=12, n_q=36, q0_bits=48, q_bits=40, p_bits=48, dnum=3, log2_scale=40, seed=7))
    O.keygen_cutmax()
    x = toy_logits(41, 1500) - 6.0
    pad = float(x.mean())
    y = np.full(O.slots, pad)
    y[:x.size] = x
    T = 4
    vlo, vhi = [0.5, 0.25, 0.3, 0.6], [2.0, 0.75, 3.0, 128.0]
    coef = [list(chebyshev_invsqrt(vlo[t] / vhi[t], 3)) for t in range(T)]
    hc = ckks.HECfg(T=T, p=[3] * T, c=[5.0] * T, v_lo=vlo, v_hi=vhi, coef=coef, sum_lo=1.0, sum_hi=3.0, gold_d=3)
    Z = ckks.cutmax_he(O, [O.encrypt(y)], hc, n_real=x.size, pad=pad)[0]
    dz = O.decrypt(Z)[:x.size]
    mc = MirrorCfg(T=T, p=[3] * T, c=[5.0] * T, v_hi=vhi, v_lo=vlo, coef=coef, B=3.0 * x.size, gold_d=3,
                   sum_lo=1.0 * x.size)
    assert np.abs(dz - cutmax_mirror(x, mc)).max() < 1e-4
    assert int(np.argmax(dz)) == int(np.argmax(x))
    assert abs(dz.sum() - 1.0) < 1e-2


@pytest.mark.slow
def test_scaled_refinement_schedule_decrypts_to_the_mirror():
    """the wide-domain inverse square root in the encrypted schedule (the guess evaluated
    twice from u, then x <- x (a_k - b_k x^2) carried on E and on W = b_k x_k^2, the
    Table 2 form): three iterations with a 200x variance domain and 3 scaled steps, a plain
    guess, and 1 step, decrypt to the FP64 mirror of the same steps within 1e-6 at 2^40 and
    recover the argmax; the level count matches the schedule's"""
    from oracle.cutmax_fp64 import scaled_invsqrt_plan
    O = ckks.Oracle(ckks.Params(log_n=12, n_q=36, q0_bits=48, q_bits=40, p_bits=48, dnum=3, log2_scale=40,
                                seed=7, hoist=3))
    O.keygen_cutmax()
    x = toy_logits(5)
    y, _, _ = slot_layout(x, O.slots)
    T, K = 3, [3, 0, 1]
    vlo, vhi = [0.01, 0.25, 0.3], [2.0, 0.75, 3.0]
    coef, steps = [], []
    for t in range(T):
        g, st, _ = scaled_invsqrt_plan(vlo[t] / vhi[t], 3, K[t])
        coef.append(list(g))
        steps.append(st)
    hc = ckks.HECfg(T=T, p=[3] * T, c=[5.0] * T, v_lo=vlo, v_hi=vhi, coef=coef, sum_lo=1.0, sum_hi=3.0, gold_d=3,
                    scaled=steps)
    assert hc.levels_needed() == 35
    Z = ckks.cutmax_he(O, [O.encrypt(y)], hc)[0]
    assert Z.level == 0
    mc = MirrorCfg(T=T, p=[3] * T, c=[5.0] * T, v_hi=vhi, v_lo=vlo, coef=coef, B=3.0 * y.size, gold_d=3,
                   sum_lo=1.0 * y.size, scaled=steps)
    z = O.decrypt(Z)
    assert np.abs(z - cutmax_mirror(y, mc)).max() < 1e-6
    assert int(np.argmax(z[:x.size])) == int(np.argmax(x))


@pytest.mark.slow
def test_prescaled_schedule_decrypts_to_the_mirror():
    """a schedule whose bounds turn on the iterate's power-of-two prescale: p = 16 first,
    so the second variance bound is 1e7, and the mean bound before the final division is
    1.6e4 (the prescale is 2^-8 on the first output and 2^-10 on the last; at Table 2's
    sizes, n = 32768 and variances near 4e12, it is what keeps 1/(n sqrt(n v)) above the
    1/q a constant multiply resolves).  CutMax is invariant under it, so the decryption
    equals the FP64 mirror, which has none, within 1e-6: a gain applied to the normaliser
    but not to the added constant, or to the bounds but not to the iterate, fails this"""
    from oracle.cutmax_fp64 import scaled_invsqrt_plan
    O = ckks.Oracle(ckks.Params(log_n=12, n_q=36, q0_bits=48, q_bits=40, p_bits=48, dnum=3, log2_scale=40,
                                seed=7, hoist=3))
    O.keygen_cutmax()
    x = toy_logits(5)
    y, _, _ = slot_layout(x, O.slots)
    T, p, c = 2, [16, 8], [5.0, 5.0]
    vlo, vhi = [0.5, 1e6], [2.0, 1e7]
    coef, steps = [], []
    for t in range(T):
        g, st, _ = scaled_invsqrt_plan(vlo[t] / vhi[t], 3, 1)
        coef.append(list(g))
        steps.append(st)
    hc = ckks.HECfg(T=T, p=p, c=c, v_lo=vlo, v_hi=vhi, coef=coef, sum_lo=4e3, sum_hi=1.6e4, gold_d=5,
                    scaled=steps)
    assert hc.prescale() == [8, 10]
    assert hc.levels_needed() == 29
    Z = ckks.cutmax_he(O, [O.encrypt(y)], hc)[0]
    mc = MirrorCfg(T=T, p=p, c=c, v_hi=vhi, v_lo=vlo, coef=coef, B=1.6e4 * y.size, gold_d=5,
                   sum_lo=4e3 * y.size, scaled=steps)
    z = O.decrypt(Z)
    ref = cutmax_mirror(y, mc)
    assert np.abs(z - ref).max() < 1e-6
    assert int(np.argmax(z[:x.size])) == int(np.argmax(x))
    # the mirror is not trivial here: the top logit holds nearly all the mass
    assert ref.max() > 0.49
