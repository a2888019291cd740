"""Pins of the oracle's CKKS bootstrap (oracle/boot.py) against closed forms:
the decoding matrix written out from its definition, the butterfly factorisation,
the baby-step giant-step identity, the EvalMod polynomial against sin, ModRaise's
m + q_0 I identity, the absence of a key-switch noise bias, and the round trip of
an encrypted vector through the whole bootstrap."""
import math

import numpy as np
import pytest

from oracle import boot as B
from oracle import ckks

TOY_BOOT = ckks.Params(log_n=12, n_q=20, q0_bits=48, q_bits=40, p_bits=48, dnum=3, log2_scale=40,
                       seed=5, hoist=3, n_hi=13, hi_bits=48, secret_hw=64)


def dense(D, s):
    M = np.zeros((s, s), dtype=np.complex128)
    for d, v in D.items():
        for t in range(s):
            M[t, (t + d) % s] += v[t]
    return M


@pytest.mark.parametrize("N", [16, 64, 256])
def test_decode_matrix_is_the_slot_map(N):
    """U w with w_k = m_k + i m_{k+N/2} equals the slots of m, by direct evaluation
    of m at zeta^{t_j} (the decoding of Sec. 2.1's CKKS)."""
    rng = np.random.default_rng(N)
    m = rng.integers(-1000, 1000, N).astype(np.float64)
    s = N // 2
    w = m[:s] + 1j * m[s:]
    t = ckks.slot_exponents(N)
    direct = np.array([sum(m[k] * np.exp(1j * np.pi * (t[j] * k % (2 * N)) / N) for k in range(N))
                       for j in range(s)])
    assert np.allclose(B.decode_matrix(N) @ w, direct, rtol=0, atol=1e-8)
    assert np.allclose((B.decode_matrix(N) @ w).real, ckks.decode_direct(m, N, 1.0), atol=1e-8)


@pytest.mark.parametrize("N,n", [(64, 1), (64, 2), (256, 3), (256, 4)])
def test_butterfly_groups_factor_the_decoding_matrix(N, n):
    s = N // 2
    P = np.eye(s)[B.bitrev_perm(s)]
    U = B.decode_matrix(N)
    M = np.eye(s, dtype=np.complex128)
    for D in B.stage_groups(s, n, False):
        M = dense(D, s) @ M
    assert np.abs(M @ P - U).max() < 1e-10
    Mi = np.eye(s, dtype=np.complex128)
    for D in B.stage_groups(s, n, True):
        Mi = dense(D, s) @ Mi
    assert np.abs(P @ Mi - np.linalg.inv(U)).max() < 1e-12


@pytest.mark.parametrize("inverse", [True, False])
def test_bsgs_identity(inverse):
    s = 512
    rng = np.random.default_rng(3)
    v = rng.normal(size=s) + 1j * rng.normal(size=s)
    for D in B.stage_groups(s, 3, inverse):
        plan = B.bsgs_plan(D, s)
        out = np.zeros(s, dtype=np.complex128)
        for a, terms in plan.terms.items():
            shift = a * plan.B * plan.h0
            inner = sum(np.roll(D[d], shift) * np.roll(v, -b * plan.h0) for b, d in terms)
            out += np.roll(inner, -shift)
        assert np.abs(out - B.apply_diag(D, v)).max() < 1e-9
        assert all(0 <= b < plan.B for ts in plan.terms.values() for b, _ in ts)
        assert plan.B * plan.B >= len(D) and (plan.B == 1 or (plan.B // 2) ** 2 < len(D))


def test_encode_complex_round_trip_and_real_case():
    N = 256
    rng = np.random.default_rng(5)
    z = rng.uniform(-1, 1, N // 2) + 1j * rng.uniform(-1, 1, N // 2)
    m = B.encode_complex(z, N, 2.0 ** 30)
    assert np.abs(B.decode_complex(m, N, 2.0 ** 30) - z).max() < 1e-6
    x = rng.uniform(-1, 1, N // 2)
    assert np.array_equal(B.encode_complex(x, N, 2.0 ** 30), ckks.encode_direct(x, N, 2.0 ** 30))


@pytest.mark.parametrize("K,r,deg", [(14, 3, 31), (24, 3, 31), (14, 4, 15)])
def test_eval_mod_polynomial_is_sine(K, r, deg):
    """the interpolant in z = 2 y^2 - 1 followed by r double angles equals sin(2 pi x)
    on [-K, K] (plaintext arithmetic)"""
    cfg = B.BootCfg(K=K, r=r, cheb_deg=deg)
    Bk = K + 0.5
    c = B.eval_mod_coeffs(cfg, Bk)
    x = np.linspace(-K, K, 20001)
    y = (x - 0.25) / Bk
    v = np.polynomial.chebyshev.chebval(2 * y * y - 1, c)
    for _ in range(r):
        v = 2 * v * v - 1
    assert np.abs(v - np.sin(2 * np.pi * x)).max() < 1e-9
    # the integer part vanishes, the fraction survives: sin(2 pi (I + f)) / 2 pi ~ f
    f = 1e-5
    assert abs(np.sin(2 * np.pi * (3 + f)) / (2 * np.pi) - f) < 1e-13


def test_levels_used():
    assert B.levels_used(B.BootCfg()) == 3 + 1 + 5 + 1 + 3 + 3


@pytest.fixture(scope="module")
def toy():
    O = ckks.Oracle(TOY_BOOT)
    O.keygen_cutmax()
    cfg = B.BootCfg()
    keys = B.keygen_boot(O, cfg)
    return O, cfg, keys


def test_sparse_secret(toy):
    O, _, _ = toy
    s = O.secret()
    assert int((s != 0).sum()) == 64 and set(np.unique(s)) <= {-1, 0, 1}


def test_modraise_identity(toy):
    """the raised ciphertext decrypts to m + q_0 I: equal to m modulo q_0, with a
    small integer I"""
    O, cfg, _ = toy
    rng = np.random.default_rng(7)
    ct = O.cm_target(O.drop(O.encrypt(rng.uniform(-1, 1, O.slots)), 1), 1.0, 2.0 ** 36)
    m0 = O.decrypt_coeffs(ct)
    R = O.modraise(ct, O.L, 1.0)
    mr = O.decrypt_coeffs(R)
    I = np.round((mr - m0) / O.q[0])
    assert np.array_equal(mr, m0 + O.q[0] * I)
    assert 0 < np.abs(I).max() <= cfg.k_bound(64)


def test_keyswitch_noise_has_no_offset(toy):
    """the rotation's noise polynomial has mean ~0 (centred ModUp digits): a constant
    offset would sum coherently into the slots near slot 0"""
    O, _, keys = toy
    N = O.N
    rng = np.random.default_rng(9)
    m = rng.integers(-2 ** 40, 2 ** 40, N)
    ct = O.drop(O.encrypt_coeffs(m, 2.0 ** 48), 16)
    g = 5
    r = O.rotate_gal(ct, keys[g], g)
    mu = O.decrypt_coeffs(ct)
    rot = np.zeros(N)
    for i in range(N):
        e = (i * g) % (2 * N)
        if e < N:
            rot[e] += mu[i]
        else:
            rot[e - N] -= mu[i]
    e = O.decrypt_coeffs(r) - rot
    assert abs(e.mean()) < 5 * e.std() / math.sqrt(N)


def test_bootstrap_round_trip(toy):
    """a level-3 ciphertext of values in [-1, 1] comes back at level L - 16 with the
    same values; a wrong sign, index or constant anywhere makes the error O(1)"""
    O, cfg, keys = toy
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, O.slots)
    ct = O.drop(O.encrypt(x), 3)
    out = B.bootstrap(O, ct, 1.0, cfg, keys)
    assert out.level == O.L - B.levels_used(cfg)
    assert abs(out.scale / O.Delta - 1) < 1e-9
    err = np.abs(O.decrypt(out) - x).max()
    assert err < 1e-3, err
    # structured input: a constant vector (all its energy in one coefficient)
    c = np.full(O.slots, 0.75)
    out = B.bootstrap(O, O.drop(O.encrypt(c), 2), 1.0, cfg, keys)
    assert np.abs(O.decrypt(out) - c).max() < 1e-3


def _is_prime(n: int) -> bool:
    """deterministic Miller-Rabin for n < 3.3e24 (bases 2..41)"""
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41):
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_mixed_chain_primes():
    """q0 of q0_bits, q1..q_{L-n_hi} of q_bits, the top n_hi of hi_bits, then P: each the
    first prime 2^b - k 2N + 1 (k = 1, 2, ..) not taken before"""
    O = ckks.Oracle(TOY_BOOT)
    N, L = O.N, O.L
    bits = [TOY_BOOT.q0_bits] + [TOY_BOOT.hi_bits if i >= TOY_BOOT.n_q - TOY_BOOT.n_hi else TOY_BOOT.q_bits
                                 for i in range(1, TOY_BOOT.n_q)] + [TOY_BOOT.p_bits] * O.alpha
    taken = []
    for q, b in zip(O.q, bits):
        k = 1
        while True:
            c = 2 ** b - k * 2 * N + 1
            if c not in taken and _is_prime(c):
                break
            k += 1
        assert q == c, (q, c, b)
        taken.append(q)
    assert sum(1 for q in O.q[1:L + 1] if q.bit_length() == 48) == TOY_BOOT.n_hi
