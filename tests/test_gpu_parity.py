"""GPU parity: the HIP path against the CPU oracle, bit-exact on every ciphertext limb
from the same seed and the same encoded plaintext, and decrypted CutMax against the
FP64 mirror within 1e-3 (Alg. 2), argmax agreement with Alg. 1."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import ckks  # noqa: E402
from oracle.cutmax_fp64 import (MirrorCfg, chebyshev_invsqrt, cutmax_exact, cutmax_mirror,  # noqa: E402
                                slot_layout)
from workloads import llm_logits, random_small_poly, toy_logits  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_params(p):
    return ckks.Params(log_n=p.log_n, n_q=p.n_q, q0_bits=p.q0_bits, q_bits=p.q_bits, p_bits=p.p_bits,
                       dnum=p.dnum, log2_scale=p.log2_scale, seed=p.seed, hoist=p.hoist)


class Pair:
    """A GPU context and an oracle context with the same parameters and seed,
    kept in lockstep (both advance their encryption counter per ciphertext)."""

    def __init__(self, prm):
        from paper_2509_08383_amd import he
        self.he = he
        self.G = he.Context(prm)
        self.O = ckks.Oracle(_oracle_params(prm))
        self.O.keygen_cutmax()
        assert self.G.primes == self.O.q

    def enc(self, m, scale=None):
        scale = self.O.Delta if scale is None else scale
        g = self.G.encrypt_coeffs(m, scale, self.G.slots)
        o = self.O.encrypt_coeffs(m, scale)
        return g, o

    def enc_values(self, z):
        return self.enc(ckks.encode(z, self.O.N, self.O.Delta))

    def same(self, g, o, what):
        eg = self.G.export(g)[0]
        eo = o.export()
        assert eg.shape == eo.shape, (what, eg.shape, eo.shape)
        bad = int((eg != eo).sum())
        assert bad == 0, f"{what}: {bad} limb words differ"
        assert g.level == o.level, what
        assert g.scale == o.scale, (what, g.scale, o.scale)


@pytest.fixture(scope="module")
def toy():
    from paper_2509_08383_amd import he
    say("[gpu] building toy pair")
    return Pair(he.TOY)


def test_encrypt_bit_exact(toy):
    say("[gpu] encrypt bit-exact (toy)")
    m = random_small_poly(1, toy.O.N, 2 ** 35)
    g, o = toy.enc(m)
    toy.same(g, o, "encrypt")
    g2, o2 = toy.enc(m)
    toy.same(g2, o2, "encrypt#2")


def test_decrypt_roundtrip(toy):
    z = np.random.default_rng(2).uniform(-3, 3, toy.G.slots)
    ct = toy.G.encrypt(z)
    toy.O.nonce = toy.O.nonce + 1        # keep the counters in lockstep
    np.testing.assert_allclose(toy.G.decrypt(ct), z, atol=2e-5)


def test_encoder_matches_oracle_encoder(toy):
    z = np.random.default_rng(3).uniform(-3, 3, toy.G.slots)
    ct = toy.G.encrypt(z)
    toy.O.nonce = toy.O.nonce + 1
    # the GPU ciphertext decrypted by the oracle gives the oracle's encoding within +-1 per
    # coefficient plus fresh noise
    o = toy.O.import_ct(toy.G.export(ct)[0], ct.scale)
    got = toy.O.decrypt_coeffs(o)
    want = ckks.encode(z, toy.O.N, toy.O.Delta)
    assert np.abs(got - want).max() < 200


def _pairs_of_ops(P):
    rng = np.random.default_rng(5)
    x = rng.uniform(-2, 2, P.G.slots)
    y = rng.uniform(-2, 2, P.G.slots)
    gx, ox = P.enc_values(x)
    gy, oy = P.enc_values(y)
    return gx, ox, gy, oy


@pytest.mark.parametrize("op", ["add", "sub", "mul_int", "add_const", "rescale", "cm_exact",
                                "cm_target", "mul", "drop"])
def test_elementwise_ops_bit_exact(toy, op):
    say(f"[gpu] op {op} (toy)")
    G, O = toy.G, toy.O
    gx, ox, gy, oy = _pairs_of_ops(toy)
    if op == "add":
        toy.same(G.add(gx, gy), O.add(ox, oy), op)
    elif op == "sub":
        toy.same(G.sub(gx, gy), O.sub(ox, oy), op)
    elif op == "mul_int":
        toy.same(G.mul_int(gx, -12345), O.mul_int(ox, -12345), op)
    elif op == "add_const":
        toy.same(G.add_const(gx, -2.75), O.add_const(ox, -2.75), op)
    elif op == "rescale":
        toy.same(G.rescale(gx), O.rescale(ox), op)
    elif op == "cm_exact":
        toy.same(G.cmul(gx, 0.3721, O.Delta, True), O.cm_exact(ox, 0.3721, O.Delta), op)
    elif op == "cm_target":
        toy.same(G.cmul(gx, -1.25, 2.0 ** 29, False), O.cm_target(ox, -1.25, 2.0 ** 29), op)
    elif op == "mul":
        toy.same(G.mul(gx, gy), O.mul(ox, oy), op)
        np.testing.assert_allclose(G.decrypt(G.mul(gx, gy)), G.decrypt(gx) * G.decrypt(gy), atol=1e-3)
    elif op == "drop":
        toy.same(G.drop(gx, 3), O.drop(ox, 3), op)


@pytest.mark.parametrize("r", [0, 1, 5, 10])
def test_rotate_bit_exact(toy, r):
    say(f"[gpu] rotate {r} (toy)")
    gx, ox, _, _ = _pairs_of_ops(toy)
    toy.same(toy.G.rotate(gx, r), toy.O.rotate(ox, r), f"rotate {r}")


def test_rotate_and_mul_low_levels_bit_exact(toy):
    """partial key-switch digits below the top level"""
    gx, ox, gy, oy = _pairs_of_ops(toy)
    for lv in (1, 2, 13, 24):
        gd, od = toy.G.drop(gx, lv), toy.O.drop(ox, lv)
        toy.same(toy.G.rotate(gd, 3), toy.O.rotate(od, 3), f"rotate@{lv}")
        toy.same(toy.G.mul(gd, toy.G.drop(gy, lv)), toy.O.mul(od, toy.O.drop(oy, lv)), f"mul@{lv}")


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6])
def test_ntt_variants_bit_exact(toy, variant):
    """every NTT schedule the autotuner can pick (workgroup width x pass-2 twiddle form)
    gives the same ciphertexts"""
    from paper_2509_08383_amd import he
    say(f"[gpu] ntt variant {variant}")
    gx, ox, gy, oy = _pairs_of_ops(toy)
    toy.G.set_option(he.HE_OPT_NTT_VARIANT, variant)
    try:
        toy.same(toy.G.mul(gx, gy), toy.O.mul(ox, oy), f"mul v{variant}")
        toy.same(toy.G.rotate(gx, 4), toy.O.rotate(ox, 4), f"rotate v{variant}")
    finally:
        toy.G.set_option(he.HE_OPT_NTT_VARIANT, 0)
    assert all(1 <= v <= 6 for v in toy.G.ntt_tuning())


def test_ntt_tuning_report_lists_every_candidate(toy):
    """the autotuner timed all 6 schedules in each of its 6 buckets and kept the fastest"""
    rep = toy.G.ntt_tuning_report()
    assert rep["logN"] == 12 and len(rep["variants"]) == 6 and len(rep["buckets"]) == 6
    counts = [b["vectors"] for b in rep["buckets"]]
    assert counts == sorted(counts) and counts[-1] > 1024
    for b in rep["buckets"]:
        assert len(b["ms"]) == 6 and all(m > 0 for m in b["ms"])
        assert b["choice"] == 1 + int(np.argmin(b["ms"]))
    assert toy.G.ntt_tuning()[:6] == [b["choice"] for b in rep["buckets"]]


def test_rotsum_bit_exact(toy):
    gx, ox, _, _ = _pairs_of_ops(toy)
    toy.same(toy.G.rotsum(gx), toy.O.rotsum(ox), "rotsum")


@pytest.mark.parametrize("h", [0, 1, 2])
def test_rotsum_hoisting_variants_bit_exact(h):
    """rotate-and-sum one rotation at a time (h = 0) and in hoisted radix-2^h steps, on a
    short chain (8 Q primes, alpha = 3) at the top level and with a partial last digit"""
    from paper_2509_08383_amd import he
    say(f"[gpu] rotsum hoist={h}")
    P = Pair(he.Params(log_n=12, n_q=8, q0_bits=40, q_bits=30, p_bits=40, dnum=3, log2_scale=30, seed=9, hoist=h))
    z = np.random.default_rng(50 + h).uniform(-1, 1, P.O.slots)
    gx, ox = P.enc_values(z)
    P.same(P.G.rotsum(gx), P.O.rotsum(ox), f"rotsum h={h}")
    P.same(P.G.rotsum(P.G.drop(gx, 4)), P.O.rotsum(P.O.drop(ox, 4)), f"rotsum h={h} level 4")
    np.testing.assert_allclose(P.O.decrypt(P.O.rotsum(ox)), z.sum(), atol=1e-2)
    # two ciphertexts in one handle: the batched kernels (keys reused across ciphertexts)
    m = np.concatenate([ckks.encode(np.random.default_rng(60 + h + k).uniform(-1, 1, P.O.slots), P.O.N, P.O.Delta)
                        for k in range(2)])
    g2 = P.G.encrypt_coeffs(m, P.O.Delta, 2 * P.G.slots)
    o2 = [P.O.encrypt_coeffs(m[k * P.O.N:(k + 1) * P.O.N], P.O.Delta) for k in range(2)]
    eg = P.G.export(P.G.rotsum(g2))
    for k in range(2):
        assert int((eg[k] != P.O.rotsum(o2[k]).export()).sum()) == 0, f"rotsum h={h} batch ct {k}"


def toy_cfg(n, T=4):
    p, c = [3] * T, [5.0] * T
    vlo, vhi = [0.5, 0.25, 0.3, 0.6][:T], [2.0, 0.75, 3.0, 128.0][:T]
    coef = [list(chebyshev_invsqrt(vlo[t] / vhi[t], 3)) for t in range(T)]
    return p, c, vlo, vhi, coef


def test_cutmax_toy_bit_exact_and_mirror(toy):
    """toy: N=2^12, 1024 logits replicated to 2048 slots, T=4, p=3, c=5."""
    from paper_2509_08383_amd import he
    say("[gpu] cutmax toy bit-exact")
    x = toy_logits(21)
    y, a, rep = slot_layout(x, toy.G.slots)
    n = y.size
    p, c, vlo, vhi, coef = toy_cfg(n)
    g, o = toy.enc_values(y)
    cfg = he.CutmaxCfg(T=4, p=p, c=c, var_lo=vlo, var_hi=vhi, init_degree=3, init_coef=coef,
                       sum_lo=1.0, sum_hi=3.0, gold_d=3)
    Zg = toy.G.cutmax([g], cfg)[0]
    hc = ckks.HECfg(T=4, p=p, c=c, v_lo=vlo, v_hi=vhi, coef=coef, sum_lo=1.0, sum_hi=3.0, gold_d=3)
    Zo = ckks.cutmax_he(toy.O, [o], hc)[0]
    toy.same(Zg, Zo, "cutmax")
    dz = toy.G.decrypt(Zg, n)
    mc = MirrorCfg(T=4, p=p, c=c, v_hi=vhi, v_lo=vlo, coef=coef, B=3.0 * n, gold_d=3, sum_lo=1.0 * n)
    assert np.abs(dz - cutmax_mirror(y, mc)).max() < 1e-3
    assert int(np.argmax(dz[:x.size])) == int(np.argmax(x))
    assert int(np.argmax(cutmax_exact(y, 3, 5.0, 4)[:x.size])) == int(np.argmax(x))


@pytest.mark.parametrize("gold", [False, True])
def test_cutmax_toy_refinements_bit_exact(toy, gold):
    """T=2 with a degree-1 guess and 2 refinements per iteration, Newton or Goldschmidt
    (HE_REFINE_GOLDSCHMIDT): bit-exact against the oracle's schedule, within 1e-3 of the
    FP64 mirror, argmax recovered"""
    from paper_2509_08383_amd import he
    say(f"[gpu] cutmax toy refinements (goldschmidt={gold})")
    x = toy_logits(23)
    y, a, rep = slot_layout(x, toy.G.slots)
    n = y.size
    p, c, vlo, vhi, _ = toy_cfg(n, T=2)
    coef = [list(chebyshev_invsqrt(vlo[t] / vhi[t], 1)) for t in range(2)]
    g, o = toy.enc_values(y)
    cfg = he.CutmaxCfg(T=2, p=p, c=c, var_lo=vlo, var_hi=vhi, init_degree=1, init_coef=coef, newton_steps=2,
                       sum_lo=1.0, sum_hi=3.0, gold_d=3, flags=he.HE_REFINE_GOLDSCHMIDT if gold else 0)
    Zg = toy.G.cutmax([g], cfg)[0]
    hc = ckks.HECfg(T=2, p=p, c=c, v_lo=vlo, v_hi=vhi, coef=coef, newton=2, goldschmidt=gold, sum_lo=1.0,
                    sum_hi=3.0, gold_d=3)
    Zo = ckks.cutmax_he(toy.O, [o], hc)[0]
    toy.same(Zg, Zo, "cutmax refinements")
    assert Zg.level == toy.G.L - hc.levels_needed()
    dz = toy.G.decrypt(Zg, n)
    mc = MirrorCfg(T=2, p=p, c=c, v_hi=vhi, v_lo=vlo, coef=coef, newton=2, goldschmidt=gold, B=3.0 * n, gold_d=3,
                   sum_lo=1.0 * n)
    assert np.abs(dz - cutmax_mirror(y, mc)).max() < 1e-3
    assert int(np.argmax(dz[:x.size])) == int(np.argmax(x))


def test_cutmax_toy_masked_padding_bit_exact(toy):
    """HE_MASK_PAD on 1500 logits padded with their mean to 2048 slots, batched with a
    replicated request: bit-exact against the oracle's masked schedule (pad tracker),
    the argmax recovered; the replicated request is unchanged by the flag"""
    from paper_2509_08383_amd import he
    say("[gpu] cutmax toy masked padding")
    x = toy_logits(41, 1500) - 6.0
    pad = float(x.mean())
    y = np.full(toy.G.slots, pad)
    y[:x.size] = x
    m = ckks.encode(y, toy.O.N, toy.O.Delta)
    g = toy.G.encrypt_coeffs(m, toy.O.Delta, x.size)
    g.set_pad(pad)
    o = toy.O.encrypt_coeffs(m, toy.O.Delta)
    xr = toy_logits(42, 1024)
    yr, _, _ = slot_layout(xr, toy.G.slots)
    gr, orr = toy.enc_values(yr)
    p, c, vlo, vhi, coef = toy_cfg(2048)
    flags = he.HE_MASK_PAD
    cfg = he.CutmaxCfg(T=4, p=p, c=c, var_lo=vlo, var_hi=vhi, init_degree=3, init_coef=coef, sum_lo=1.0, sum_hi=3.0,
                       gold_d=3, flags=flags)
    Zg = toy.G.cutmax([g, gr], cfg)
    hc = ckks.HECfg(T=4, p=p, c=c, v_lo=vlo, v_hi=vhi, coef=coef, sum_lo=1.0, sum_hi=3.0, gold_d=3)
    Zo = ckks.cutmax_he(toy.O, [o], hc, n_real=x.size, pad=pad)[0]
    toy.same(Zg[0], Zo, "masked cutmax")
    Zr = ckks.cutmax_he(toy.O, [orr], hc)[0]
    toy.same(Zg[1], Zr, "replicated request beside a masked one")
    dz = toy.G.decrypt(Zg[0], x.size)
    assert int(np.argmax(dz)) == int(np.argmax(x))
    # the toy chain's 2^30 scale: the tracker subtraction multiplies its error by the
    # pad count, so the mirror of the logits alone is matched to 2e-2 here (1e-3 at 2^40)
    mc = MirrorCfg(T=4, p=p, c=c, v_hi=vhi, v_lo=vlo, coef=coef, B=3.0 * x.size, gold_d=3, sum_lo=1.0 * x.size)
    assert np.abs(dz - cutmax_mirror(x, mc)).max() < 2e-2


def test_cutmax_toy_batch_mixed_counts(toy):
    """batched form: requests with 1 and 2 ciphertexts advance together; each equals its
    single-request run bit for bit (n > s splits over several ciphertexts, App. D)."""
    from paper_2509_08383_amd import he
    say("[gpu] cutmax toy batch")
    # toy-family logits (the toy chain's 2^30 scale leaves ~1e-3 of CKKS error on LLM-like
    # logits with their wider variance range; those run at N = 2^16)
    xs = [toy_logits(31, 1024), toy_logits(32, 3000), toy_logits(33, 1024)]
    cts = [toy.G.encrypt(x) for x in xs]
    toy.O.nonce = toy.O.nonce + sum(c.a for c in cts)
    p, c, vlo, vhi, coef = toy_cfg(2048)
    # one domain for the replicated and the zero-padded requests
    vlo2 = [0.5, 0.2, 0.3, 0.6]
    vhi2 = [32.0, 0.9, 16.0, 512.0]
    coef = [list(chebyshev_invsqrt(vlo2[t] / vhi2[t], 3)) for t in range(4)]
    cfg = he.CutmaxCfg(T=4, p=p, c=c, var_lo=vlo2, var_hi=vhi2, init_coef=coef, sum_lo=1.0, sum_hi=3.0)
    Zb = toy.G.cutmax(cts, cfg)
    for i, (x, ct) in enumerate(zip(xs, cts)):
        Zs = toy.G.cutmax([ct], cfg)[0]
        eb, es = toy.G.export(Zb[i]), toy.G.export(Zs)
        assert np.array_equal(eb, es), f"request {i}: batched != single"
        y, a, rep = slot_layout(x, toy.G.slots)
        assert Zb[i].a == a
        dz = toy.G.decrypt(Zb[i], y.size)
        mc = MirrorCfg(T=4, p=p, c=c, v_hi=vhi2, v_lo=vlo2, coef=coef, B=3.0 * y.size, gold_d=3,
                       sum_lo=1.0 * y.size)
        assert np.abs(dz - cutmax_mirror(y, mc)).max() < 1e-3
        assert int(np.argmax(dz[:x.size])) == int(np.argmax(x))


def test_cutmax_graph_replays_match_eager(toy):
    """HIP-graph mode: the first call captures, later calls replay; every replay (with eager
    work in between) equals the eager result bit for bit."""
    from paper_2509_08383_amd import he
    say("[gpu] graph capture/replay")
    x = toy_logits(51)
    ct = toy.G.encrypt(x)
    toy.O.nonce = toy.O.nonce + 1
    p, c, vlo, vhi, coef = toy_cfg(2048)
    cfg = he.CutmaxCfg(T=4, p=p, c=c, var_lo=vlo, var_hi=vhi, init_coef=coef, sum_lo=1.0, sum_hi=3.0)
    ref = toy.G.export(toy.G.cutmax([ct], cfg)[0])
    toy.G.set_option(he.HE_OPT_GRAPH, 1)
    try:
        for i in range(4):
            z = toy.G.export(toy.G.cutmax([ct], cfg)[0])
            assert np.array_equal(z, ref), f"graph call {i} differs"
            other = toy.G.encrypt(toy_logits(60 + i))       # eager work between replays
            toy.O.nonce = toy.O.nonce + 1
            toy.G.mul(other, other)
    finally:
        toy.G.set_option(he.HE_OPT_GRAPH, 0)


def test_graphs_recaptured_after_the_workspace_grows():
    """a captured graph holds workspace addresses: a larger call that grows the workspace
    drops the cached graphs, and the next call of the first shape captures again and still
    equals the eager result bit for bit"""
    from paper_2509_08383_amd import he
    say("[gpu] graph cache across workspace growth")
    G = he.Context(he.TOY)
    p, c, vlo, vhi, coef = toy_cfg(2048)
    vlo2, vhi2 = [0.5, 0.2, 0.3, 0.6], [32.0, 0.9, 16.0, 512.0]
    coef2 = [list(chebyshev_invsqrt(vlo2[t] / vhi2[t], 3)) for t in range(4)]
    cfg = he.CutmaxCfg(T=4, p=p, c=c, var_lo=vlo2, var_hi=vhi2, init_coef=coef2, sum_lo=1.0, sum_hi=3.0)
    small = G.encrypt(toy_logits(71))
    big = [G.encrypt(toy_logits(72 + r, 3000)) for r in range(6)]
    ref = G.export(G.cutmax([small], cfg)[0])
    G.set_option(he.HE_OPT_GRAPH, 1)
    for k in range(2):
        assert np.array_equal(G.export(G.cutmax([small], cfg)[0]), ref), k
    Zb = G.cutmax(big, cfg)                             # grows the workspace
    for k in range(2):
        assert np.array_equal(G.export(G.cutmax([small], cfg)[0]), ref), k
    G.set_option(he.HE_OPT_GRAPH, 0)
    Ze = G.cutmax(big, cfg)
    for r in range(6):
        assert np.array_equal(G.export(Zb[r]), G.export(Ze[r])), r


def test_cutmax_errors_are_reported(toy):
    from paper_2509_08383_amd import he
    x = toy_logits(41)
    ct = toy.G.encrypt(x)
    toy.O.nonce = toy.O.nonce + 1
    p, c, vlo, vhi, coef = toy_cfg(2048)
    deep = he.CutmaxCfg(T=6, p=[3] * 6, c=[5.0] * 6, var_lo=[0.5] * 6, var_hi=[2.0] * 6, sum_lo=1.0, sum_hi=3.0)
    with pytest.raises(he.HeError) as e:
        toy.G.cutmax([ct], deep)
    assert e.value.code == he.HE_EDEPTH
    bad = he.CutmaxCfg(T=1, p=[3], c=[5.0], var_lo=[2.0], var_hi=[1.0])
    with pytest.raises(he.HeError) as e:
        toy.G.cutmax([ct], bad)
    assert e.value.code == he.HE_EINVAL


def test_edge_inputs_are_rejected_or_handled(toy):
    """empty input and mismatched levels are errors; a tied maximum is split evenly, as
    in the FP64 mirror, and the recovered index is one of the tied entries"""
    from paper_2509_08383_amd import he
    with pytest.raises(he.HeError) as e:
        toy.G.encrypt(np.zeros(0))
    assert e.value.code == he.HE_EINVAL
    x = toy_logits(43)
    a = toy.G.encrypt(x)
    toy.O.nonce = toy.O.nonce + 1        # keep the counters in lockstep
    with pytest.raises(he.HeError) as e:
        toy.G.add(a, toy.G.drop(a, 3))
    assert e.value.code in (he.HE_ESTATE, he.HE_EINVAL)
    with pytest.raises(he.HeError) as e:
        toy.G.decrypt(a, toy.G.slots + 1)
    assert e.value.code == he.HE_EINVAL
    for bad in (np.nan, np.inf, 2.0 ** 40):
        with pytest.raises(he.HeError) as e:
            toy.G.encrypt(np.array([1.0, bad, 0.5]))
        assert e.value.code == he.HE_EINVAL
    with pytest.raises(he.HeError) as e:
        a.set_pad(float("inf"))
    assert e.value.code == he.HE_EINVAL
    # tie: the two largest logits made equal
    i, j = int(np.argmax(x)), int(np.argsort(x)[-2])
    x[j] = x[i]
    y, _, _ = slot_layout(x, toy.G.slots)
    p, c, vlo, vhi, coef = toy_cfg(y.size)
    cfg = he.CutmaxCfg(T=4, p=p, c=c, var_lo=vlo, var_hi=vhi, init_degree=3, init_coef=coef, sum_lo=1.0,
                       sum_hi=3.0, gold_d=3)
    ct = toy.G.encrypt(x)
    toy.O.nonce = toy.O.nonce + 1
    z = toy.G.decrypt(toy.G.cutmax([ct], cfg)[0], y.size)
    mc = MirrorCfg(T=4, p=p, c=c, v_hi=vhi, v_lo=vlo, coef=coef, B=3.0 * y.size, gold_d=3, sum_lo=1.0 * y.size)
    assert np.abs(z - cutmax_mirror(y, mc)).max() < 1e-3
    assert int(np.argmax(z[:x.size])) in (i, j)


@pytest.mark.parametrize("degree", [2, 4])
def test_cutmax_toy_guess_degrees_bit_exact(toy, degree):
    """the degree-2 and degree-4 initial guesses (degree 4 is the form the learned network
    collapses to, evaluated in depth 3) inside the whole toy CutMax: bit-exact against the
    oracle's schedule, within 1e-3 of the FP64 mirror, argmax recovered"""
    from paper_2509_08383_amd import he
    say(f"[gpu] cutmax toy degree-{degree} guess bit-exact")
    T = 4 if degree == 2 else 3
    x = toy_logits(25 + degree)
    y, a, rep = slot_layout(x, toy.G.slots)
    n = y.size
    p, c, vlo, vhi, _ = toy_cfg(n, T=T)
    coef = [list(chebyshev_invsqrt(vlo[t] / vhi[t], degree)) for t in range(T)]
    g, o = toy.enc_values(y)
    cfg = he.CutmaxCfg(T=T, p=p, c=c, var_lo=vlo, var_hi=vhi, init_degree=degree, init_coef=coef,
                       sum_lo=1.0, sum_hi=3.0, gold_d=3)
    Zg = toy.G.cutmax([g], cfg)[0]
    hc = ckks.HECfg(T=T, p=p, c=c, v_lo=vlo, v_hi=vhi, coef=coef, sum_lo=1.0, sum_hi=3.0, gold_d=3)
    Zo = ckks.cutmax_he(toy.O, [o], hc)[0]
    toy.same(Zg, Zo, f"cutmax degree {degree}")
    assert Zg.level == toy.G.L - hc.levels_needed()
    dz = toy.G.decrypt(Zg, n)
    mc = MirrorCfg(T=T, p=p, c=c, v_hi=vhi, v_lo=vlo, coef=coef, B=3.0 * n, gold_d=3, sum_lo=1.0 * n)
    assert np.abs(dz - cutmax_mirror(y, mc)).max() < 1e-3
    assert int(np.argmax(dz[:x.size])) == int(np.argmax(x))


@pytest.mark.parametrize("sampler", ["topp", "gumbel"])
@pytest.mark.parametrize("prescaled", [False, True])
def test_samplers_toy_bit_exact(toy, sampler, prescaled):
    """the samplers' server step CutMax(X + tau G) (Alg. 3; the Gumbel-max form of Sec. 3.3
    runs the same step): with the temperature multiply on the noise ciphertext, or with
    noise the client already scaled, bit-exact against the oracle's topp_he, and the
    decrypted one-hot picks argmax(x/tau + g)"""
    from paper_2509_08383_amd import he
    from oracle.cutmax_fp64 import beta_alpha, beta_noise, gumbel_noise
    from workloads import uniform_noise
    say(f"[gpu] {sampler} sampler toy bit-exact (prescaled={prescaled})")
    tau, top_p, T = 0.8, 0.9, 3
    x = toy_logits(27)
    u = uniform_noise(28, x.size)
    gn = beta_noise(u, beta_alpha(top_p)) if sampler == "topp" else gumbel_noise(u)
    y, _, _ = slot_layout(x, toy.G.slots)
    gy, _, _ = slot_layout(gn, toy.G.slots)
    n = y.size
    p, c = [3] * T, [5.0] * T
    # Gumbel noise (variance pi^2/6 times tau^2) widens the first variance
    vlo, vhi = [0.5, 0.25, 0.3], [4.0, 0.75, 3.0]
    coef = [list(chebyshev_invsqrt(vlo[t] / vhi[t], 3)) for t in range(T)]
    gx, ox = toy.enc_values(y)
    gg, og = toy.enc_values(tau * gy if prescaled else gy)
    cfg = he.CutmaxCfg(T=T, p=p, c=c, var_lo=vlo, var_hi=vhi, init_degree=3, init_coef=coef, sum_lo=1.0,
                       sum_hi=3.0, gold_d=3, flags=he.HE_NOISE_PRESCALED if prescaled else 0)
    if sampler == "topp":
        Zg = toy.G.topp_sample([gx], [gg], top_p, tau, cfg)[0]
    else:
        Zg = toy.G.gumbel_sample([gx], [gg], tau, cfg)[0]
    hc = ckks.HECfg(T=T, p=p, c=c, v_lo=vlo, v_hi=vhi, coef=coef, sum_lo=1.0, sum_hi=3.0, gold_d=3)
    Zo = ckks.topp_he(toy.O, [ox], [og], tau, hc, prescaled=prescaled)[0]
    toy.same(Zg, Zo, f"{sampler} sample")
    dz = toy.G.decrypt(Zg, n)
    mc = MirrorCfg(T=T, p=p, c=c, v_hi=vhi, v_lo=vlo, coef=coef, B=3.0 * n, gold_d=3, sum_lo=1.0 * n)
    assert np.abs(dz - cutmax_mirror(y + tau * gy, mc)).max() < 1e-3
    assert int(np.argmax(dz[:x.size])) == int(np.argmax(x / tau + gn))


def test_foreign_operands_and_bad_options_are_rejected(toy):
    """a second operand from another context (another chain and limb stride) is
    refused with HE_EINVAL before any kernel runs, for add, sub and mul; an NTT variant out
    of range is refused, and a valid one drops the captured graphs (a later replay still
    equals the eager result)"""
    from paper_2509_08383_amd import he
    say("[gpu] foreign operands, option checks")
    # the same ring degree with another chain: another limb stride and prime set
    other = he.Context(he.Params(log_n=12, n_q=6, q0_bits=40, q_bits=30, p_bits=40, dnum=3, log2_scale=30, seed=5))
    a = toy.G.encrypt(np.ones(8))
    b = other.encrypt(np.ones(8))
    toy.O.nonce = toy.O.nonce + 1
    a = toy.G.drop(a, b.level)       # same level: only the context differs
    assert a.level == b.level == 5
    for op in (toy.G.add, toy.G.sub, toy.G.mul):
        with pytest.raises(he.HeError) as e:
            op(a, b)
        assert e.value.code == he.HE_EINVAL and "context" in str(e.value)
    for bad in (-1, 99):
        with pytest.raises(he.HeError) as e:
            toy.G.set_option(he.HE_OPT_NTT_VARIANT, bad)
        assert e.value.code == he.HE_EINVAL
    x = toy_logits(52)
    ct = toy.G.encrypt(x)
    toy.O.nonce = toy.O.nonce + 1
    p, c, vlo, vhi, coef = toy_cfg(2048)
    cfg = he.CutmaxCfg(T=4, p=p, c=c, var_lo=vlo, var_hi=vhi, init_coef=coef, sum_lo=1.0, sum_hi=3.0)
    ref = toy.G.export(toy.G.cutmax([ct], cfg)[0])
    toy.G.set_option(he.HE_OPT_GRAPH, 1)
    try:
        for v in (1, 2, 0):
            toy.G.set_option(he.HE_OPT_NTT_VARIANT, v)
            for _ in range(2):
                assert np.array_equal(toy.G.export(toy.G.cutmax([ct], cfg)[0]), ref), v
    finally:
        toy.G.set_option(he.HE_OPT_GRAPH, 0)
        toy.G.set_option(he.HE_OPT_NTT_VARIANT, 0)
    other.close()


def _scaled_cfg(he, K, vlo, vhi):
    from oracle.cutmax_fp64 import scaled_invsqrt_plan
    coef, steps, ranges = [], [], []
    for t in range(len(K)):
        g, st, rg = scaled_invsqrt_plan(vlo[t] / vhi[t], 3, K[t])
        coef.append(list(g))
        steps.append(st)
        ranges.append(rg)
    return coef, steps, ranges


def test_cutmax_scaled_refinement_bit_exact():
    """the wide-domain inverse square root (HE_REFINE_SCALED: guess, then x <- x (a_k - b_k
    x^2) carried on E h and on W = b_k x_k^2, the form of the Table 2 schedule) on a 2^40
    toy chain: three iterations with 3, 0 and 1 refinements; one request word for word
    against the oracle's schedule, and a batch of two requests (1 and 2 ciphertexts) whose
    outputs equal the oracle's run of each; decrypted within 1e-3 of the FP64 mirror"""
    from paper_2509_08383_amd import he
    say("[gpu] scaled refinement schedule bit-exact (2^40 toy chain)")
    P = Pair(he.Params(log_n=12, n_q=36, q0_bits=48, q_bits=40, p_bits=48, dnum=3, log2_scale=40, seed=7, hoist=3))
    T, K = 3, [3, 0, 1]
    vlo, vhi = [0.01, 0.25, 0.3], [2.0, 0.75, 3.0]
    coef, steps, ranges = _scaled_cfg(he, K, vlo, vhi)
    cfg = he.CutmaxCfg(T=T, p=[3] * T, c=[5.0] * T, var_lo=vlo, var_hi=vhi, init_degree=3, init_coef=coef,
                       sum_lo=1.0, sum_hi=3.0, gold_d=3, flags=he.HE_REFINE_SCALED, ref_steps=steps,
                       ref_range=ranges)
    hc = ckks.HECfg(T=T, p=[3] * T, c=[5.0] * T, v_lo=vlo, v_hi=vhi, coef=coef, sum_lo=1.0, sum_hi=3.0, gold_d=3,
                    scaled=steps)
    x = toy_logits(5)
    y, _, _ = slot_layout(x, P.G.slots)
    g, o = P.enc_values(y)
    Zg = P.G.cutmax([g], cfg)[0]
    P.same(Zg, ckks.cutmax_he(P.O, [o], hc)[0], "scaled cutmax")
    mc = MirrorCfg(T=T, p=[3] * T, c=[5.0] * T, v_hi=vhi, v_lo=vlo, coef=coef, B=3.0 * y.size, gold_d=3,
                   sum_lo=1.0 * y.size, scaled=steps)
    z = P.G.decrypt(Zg, y.size)
    assert np.abs(z - cutmax_mirror(y, mc)).max() < 1e-3
    assert int(np.argmax(z[:x.size])) == int(np.argmax(x))
    # two requests in one call: 1024 logits (1 ciphertext) and 3000 (2 ciphertexts)
    x2 = toy_logits(6, 3000)
    y2, a2, _ = slot_layout(x2, P.G.slots)
    m1 = ckks.encode(y, P.O.N, P.O.Delta)
    m2 = [ckks.encode(y2[k * P.G.slots:(k + 1) * P.G.slots], P.O.N, P.O.Delta) for k in range(a2)]
    g1 = P.G.encrypt_coeffs(m1, P.O.Delta, y.size)
    o1 = P.O.encrypt_coeffs(m1, P.O.Delta)
    g2 = P.G.encrypt_coeffs(np.concatenate(m2), P.O.Delta, y2.size)
    o2 = [P.O.encrypt_coeffs(m, P.O.Delta) for m in m2]
    Z = P.G.cutmax([g1, g2], cfg)
    P.same(Z[0], ckks.cutmax_he(P.O, [o1], hc)[0], "batched request 0")
    Zo2 = ckks.cutmax_he(P.O, o2, hc)
    eg = P.G.export(Z[1])
    for k in range(a2):
        assert int((eg[k] != Zo2[k].export()).sum()) == 0, f"batched request 1, ciphertext {k}"
    bad = he.CutmaxCfg(T=T, p=[3] * T, c=[5.0] * T, var_lo=vlo, var_hi=vhi, init_degree=3, init_coef=coef,
                       flags=he.HE_REFINE_SCALED, ref_steps=steps, ref_range=[[(1.0, 0.5)] * (k + 1) for k in K])
    with pytest.raises(he.HeError) as e:
        P.G.cutmax([g1], bad)
    assert e.value.code == he.HE_EINVAL



def test_cutmax_prescaled_bit_exact():
    """bounds that turn on the iterate's power-of-two prescale (p = 16 first: variance bound
    1e7 for the second iteration, 2^-8 on the first output; mean bound 1.6e4, 2^-10 on the
    last) on the 2^40 toy chain: a replicated request word for word against the oracle's
    schedule, and a masked 1500-logit request (its pad tracker takes the same gain) beside
    it equal to the oracle's masked run; both decrypt within 1e-3 of the FP64 mirror, which
    has no prescale (CutMax is invariant under it)"""
    from paper_2509_08383_amd import he
    say("[gpu] prescaled schedule bit-exact (2^40 toy chain)")
    P = Pair(he.Params(log_n=12, n_q=36, q0_bits=48, q_bits=40, p_bits=48, dnum=3, log2_scale=40, seed=7, hoist=3))
    T, p, c = 2, [16, 8], [5.0, 5.0]
    vlo, vhi = [0.5, 1e4], [2.0, 1e7]
    coef, steps, ranges = _scaled_cfg(he, [1, 3], vlo, vhi)
    cfg = he.CutmaxCfg(T=T, p=p, c=c, var_lo=vlo, var_hi=vhi, init_degree=3, init_coef=coef, sum_lo=4e3,
                       sum_hi=1.6e4, gold_d=5, flags=he.HE_REFINE_SCALED | he.HE_MASK_PAD, ref_steps=steps,
                       ref_range=ranges)
    hc = ckks.HECfg(T=T, p=p, c=c, v_lo=vlo, v_hi=vhi, coef=coef, sum_lo=4e3, sum_hi=1.6e4, gold_d=5, scaled=steps)
    assert hc.prescale() == [8, 10]
    x = toy_logits(5)
    y, _, _ = slot_layout(x, P.G.slots)
    m1 = ckks.encode(y, P.O.N, P.O.Delta)
    g1 = P.G.encrypt_coeffs(m1, P.O.Delta, y.size)
    o1 = P.O.encrypt_coeffs(m1, P.O.Delta)
    xm = toy_logits(41, 1500)
    pad = float(xm.mean())
    ym = np.full(P.G.slots, pad)
    ym[:xm.size] = xm
    m2 = ckks.encode(ym, P.O.N, P.O.Delta)
    g2 = P.G.encrypt_coeffs(m2, P.O.Delta, xm.size)
    g2.set_pad(pad)
    o2 = P.O.encrypt_coeffs(m2, P.O.Delta)
    Z = P.G.cutmax([g1, g2], cfg)
    P.same(Z[0], ckks.cutmax_he(P.O, [o1], hc)[0], "prescaled cutmax")
    P.same(Z[1], ckks.cutmax_he(P.O, [o2], hc, n_real=xm.size, pad=pad)[0], "prescaled masked cutmax")
    # (the replicated request holds x twice: its argmax is taken over the first copy)
    for v, xs, k in ((y, x, 0), (xm, xm, 1)):
        mc = MirrorCfg(T=T, p=p, c=c, v_hi=vhi, v_lo=vlo, coef=coef, B=1.6e4 * v.size, gold_d=5,
                       sum_lo=4e3 * v.size, scaled=steps)
        z = P.G.decrypt(Z[k], v.size)
        assert np.abs(z - cutmax_mirror(v, mc)).max() < 1e-3
        assert int(np.argmax(z[:xs.size])) == int(np.argmax(xs))


def test_workspace_limit_returns_enomem_and_recovers(toy):
    """HE_OPT_WORKSPACE_LIMIT: under a 1 MiB limit a CutMax and a rotate-and-sum return
    HE_ENOMEM (the failure a full device gives, forced from the host after the call's
    planning and before any allocation or kernel), create no output, and leave the context
    usable; the entry point that allocates nothing still runs; with a limit the call fits in
    and with none, the outputs equal the first call's word for word"""
    from paper_2509_08383_amd import he
    say("[gpu] workspace limit -> HE_ENOMEM, then recovery")
    G = toy.G
    x = toy_logits(9)
    y, _, _ = slot_layout(x, G.slots)
    g, _ = toy.enc_values(y)
    p, c, vlo, vhi, coef = toy_cfg(y.size)
    cfg = he.CutmaxCfg(T=4, p=p, c=c, var_lo=vlo, var_hi=vhi, init_degree=3, init_coef=coef, sum_lo=1.0,
                       sum_hi=3.0, gold_d=3)
    ref = G.export(G.cutmax([g], cfg)[0])
    ref_rs = G.export(G.rotsum(g))
    try:
        G.set_option(he.HE_OPT_WORKSPACE_LIMIT, 1 << 20)
        for f in (lambda: G.cutmax([g], cfg), lambda: G.rotsum(g)):
            with pytest.raises(he.HeError) as e:
                f()
            assert e.value.code == he.HE_ENOMEM and "workspace limit" in str(e.value)
        with pytest.raises(he.HeError) as e:
            G.set_option(he.HE_OPT_WORKSPACE_LIMIT, -1)
        assert e.value.code == he.HE_EINVAL
        G.set_option(he.HE_OPT_WORKSPACE_LIMIT, 256 << 20)
        assert (G.export(G.cutmax([g], cfg)[0]) == ref).all()
        dst, _ = toy.enc_values(y)  # (encryption uses the workspace too)
        G.set_option(he.HE_OPT_WORKSPACE_LIMIT, 1 << 20)
        with pytest.raises(he.HeError) as e:
            toy.G.encrypt(y)
        assert e.value.code == he.HE_ENOMEM
        G.rotsum_noalloc(g, dst)
        assert (G.export(dst) == ref_rs).all()
    finally:
        G.set_option(he.HE_OPT_WORKSPACE_LIMIT, 0)
    assert (G.export(G.cutmax([g], cfg)[0]) == ref).all()
    assert (G.export(G.rotsum(g)) == ref_rs).all()
