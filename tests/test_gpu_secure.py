"""GPU parity at the 128-bit parameter set (N = 2^16, 30 Q primes, dnum = 3): primitives
and a two-ciphertext rotate-and-sum bit-exact against the CPU oracle at full size; the measured T=3 CutMax on 32000 LLM-like logits
bit-exact against the oracle and within 1e-3 of the FP64 mirror with the argmax recovered; the
batched form (16 mixed requests with 1- and 4-ciphertext requests) with a request of each kind
bit-exact against the oracle."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import ckks  # noqa: E402
from oracle.cutmax_fp64 import (MirrorCfg, chebyshev_invsqrt, cutmax_exact, cutmax_mirror,  # noqa: E402
                                slot_layout)
from workloads import llm_logits  # noqa: E402
from test_gpu_parity import Pair, say  # noqa: E402

VLO, VHI = [12.0, 0.4, 0.8], [24.0, 0.9, 16.0]


@pytest.fixture(scope="module")
def sec():
    from paper_2509_08383_amd import he
    say("[gpu] building secure pair (N=2^16)")
    return Pair(he.SECURE)


def cfg2(he, T=3, coef=None, degree=3):
    if coef is None:
        coef = [list(chebyshev_invsqrt(VLO[t] / VHI[t], degree)) for t in range(T)]
    return he.CutmaxCfg(T=T, p=[3] * T, c=[5.0] * T, var_lo=VLO[:T], var_hi=VHI[:T], init_degree=degree,
                        init_coef=coef, sum_lo=1.0, sum_hi=3.0, gold_d=3), coef


def mirror2(y, coef, T=3):
    return MirrorCfg(T=T, p=[3] * T, c=[5.0] * T, v_hi=VHI[:T], v_lo=VLO[:T], coef=coef, B=3.0 * y.size,
                     gold_d=3, sum_lo=1.0 * y.size)


def test_secure_chain(sec):
    G = sec.G
    assert G.N == 65536 and G.L == 29 and G.alpha == 10
    bits = sum(math.log2(q) for q in G.primes)
    assert bits <= 1772, bits           # 128-bit bound at N = 2^16, ternary secret


def test_encrypt_and_primitives_full_size(sec):
    say("[gpu] secure: encrypt/mul/rotate/cmul bit-exact")
    rng = np.random.default_rng(9)
    x = rng.uniform(-4, 4, sec.G.slots)
    y = rng.uniform(-4, 4, sec.G.slots)
    gx, ox = sec.enc_values(x)
    gy, oy = sec.enc_values(y)
    sec.same(gx, ox, "encrypt")
    sec.same(sec.G.mul(gx, gy), sec.O.mul(ox, oy), "mul")
    sec.same(sec.G.rotate(gx, 14), sec.O.rotate(ox, 14), "rotate 2^14")
    sec.same(sec.G.rotate(gx, 0), sec.O.rotate(ox, 0), "rotate 1")
    sec.same(sec.G.cmul(gx, 1e-3, sec.O.Delta, True), sec.O.cm_exact(ox, 1e-3, sec.O.Delta), "cm_exact")
    lv = 9
    sec.same(sec.G.mul(sec.G.drop(gx, lv), sec.G.drop(gy, lv)), sec.O.mul(sec.O.drop(ox, lv), sec.O.drop(oy, lv)),
             "mul@9")
    np.testing.assert_allclose(sec.G.decrypt(sec.G.mul(gx, gy)), x * y, atol=1e-6)


def test_rotsum_two_ciphertexts_full_size(sec):
    """rotate-and-sum of a two-ciphertext handle at the top level and at level 12: the
    batched key products (keys held in registers for the first two hoisted steps, sources
    staged in LDS for the last three, two ciphertexts each), the fused basis conversions
    with two ciphertexts and the chained first inverse passes, word for word against the
    oracle on each ciphertext"""
    say("[gpu] secure: rotsum of a 2-ciphertext handle")
    rng = np.random.default_rng(21)
    m = np.concatenate([ckks.encode(rng.uniform(-1, 1, sec.O.slots), sec.O.N, sec.O.Delta) for _ in range(2)])
    g2 = sec.G.encrypt_coeffs(m, sec.O.Delta, 2 * sec.G.slots)
    o2 = [sec.O.encrypt_coeffs(m[k * sec.O.N:(k + 1) * sec.O.N], sec.O.Delta) for k in range(2)]
    for lv in (None, 12):
        gi = g2 if lv is None else sec.G.drop(g2, lv)
        oi = o2 if lv is None else [sec.O.drop(o, lv) for o in o2]
        eg = sec.G.export(sec.G.rotsum(gi))
        assert eg.shape[0] == 2
        for k in range(2):
            bad = int((eg[k] != sec.O.rotsum(oi[k]).export()).sum())
            assert bad == 0, f"level {lv}, ciphertext {k}: {bad} words differ"


def test_ntt_variants_full_size(sec):
    """at N = 2^16 every NTT schedule (4, 8 or 16 sub-transforms per workgroup, table or
    factored pass-2 twiddles) gives the oracle's product and rotation word for word, on a
    single ciphertext and inside a two-ciphertext rotate-and-sum"""
    from paper_2509_08383_amd import he
    say("[gpu] secure: NTT schedules bit-exact")
    rng = np.random.default_rng(19)
    gx, ox = sec.enc_values(rng.uniform(-2, 2, sec.G.slots))
    gy, oy = sec.enc_values(rng.uniform(-2, 2, sec.G.slots))
    want_mul = sec.O.mul(ox, oy).export()
    want_rot = sec.O.rotate(ox, 3).export()
    two = sec.G.encrypt(rng.uniform(-1, 1, 2 * sec.G.slots))
    sec.O.nonce = sec.O.nonce + 2
    ref_rs = None
    try:
        for v in range(1, 7):
            sec.G.set_option(he.HE_OPT_NTT_VARIANT, v)
            assert np.array_equal(sec.G.export(sec.G.mul(gx, gy))[0], want_mul), v
            assert np.array_equal(sec.G.export(sec.G.rotate(gx, 3))[0], want_rot), v
            rs = sec.G.export(sec.G.rotsum(two))
            if ref_rs is None:
                ref_rs = rs
            assert np.array_equal(rs, ref_rs), v
    finally:
        sec.G.set_option(he.HE_OPT_NTT_VARIANT, 0)
    rep = sec.G.ntt_tuning_report()
    say(f"  tuning: {[(b['vectors'], b['choice'], [round(m, 4) for m in b['ms']]) for b in rep['buckets']]}")
    assert rep["logN"] == 16 and all(b["choice"] == 1 + int(np.argmin(b["ms"])) for b in rep["buckets"])


def test_cutmax_secure_T1_bit_exact(sec):
    """one CutMax iteration plus the final inverse at full size, bit for bit"""
    from paper_2509_08383_amd import he
    say("[gpu] secure: CutMax T=1 bit-exact")
    x = llm_logits(101)
    y, a, _ = slot_layout(x, sec.G.slots)
    cfg, coef = cfg2(he, T=1)
    g, o = sec.enc_values(y)
    Zg = sec.G.cutmax([g], cfg)[0]
    Zo = ckks.cutmax_he(sec.O, [o], ckks.HECfg(T=1, p=[3], c=[5.0], v_lo=VLO[:1], v_hi=VHI[:1], coef=coef,
                                               sum_lo=1.0, sum_hi=3.0))[0]
    sec.same(Zg, Zo, "cutmax T=1")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cutmax_config2_vs_mirror(sec, seed):
    """32000 logits (3 Gumbel - 1.1 ln rank) zero-padded to 32768 slots, T=3, p=3, c=5"""
    from paper_2509_08383_amd import he
    say(f"[gpu] secure: CutMax 32000 logits seed {seed}")
    x = llm_logits(seed)
    y, a, _ = slot_layout(x, sec.G.slots)
    cfg, coef = cfg2(he)
    ct = sec.G.encrypt(x)
    sec.O.nonce = sec.O.nonce + 1
    Z = sec.G.cutmax([ct], cfg)[0]
    assert Z.level == sec.G.L - 27
    dz = sec.G.decrypt(Z, y.size)
    err = np.abs(dz - cutmax_mirror(y, mirror2(y, coef))).max()
    say(f"  |Z - mirror| = {err:.3e}, {sec.G.last_cutmax_ms():.1f} ms")
    assert err < 1e-3
    assert int(np.argmax(dz[:x.size])) == int(np.argmax(x))
    assert int(np.argmax(cutmax_exact(y, 3, 5.0, 3)[:x.size])) == int(np.argmax(x))


def test_cutmax_config2_bit_exact(sec):
    """the measured workload itself (the bench's 32000-logit input, T=3, p=3, c=5, degree-3
    guess, d=3) at N = 2^16: every limb of Z equals the oracle's from the same seed and the
    same encoded plaintext, and Z decrypts to the FP64 mirror within 1e-3"""
    from paper_2509_08383_amd import he
    say("[gpu] secure: CutMax T=3 on the bench input, bit-exact against the oracle")
    x = llm_logits(0)
    y, a, _ = slot_layout(x, sec.G.slots)
    cfg, coef = cfg2(he)
    g, o = sec.enc_values(y)
    Zg = sec.G.cutmax([g], cfg)[0]
    say(f"  GPU {sec.G.last_cutmax_ms():.1f} ms; running the oracle")
    Zo = ckks.cutmax_he(sec.O, [o], ckks.HECfg(T=3, p=[3] * 3, c=[5.0] * 3, v_lo=VLO, v_hi=VHI, coef=coef,
                                               sum_lo=1.0, sum_hi=3.0, gold_d=3))[0]
    sec.same(Zg, Zo, "cutmax T=3")
    assert Zg.level == sec.G.L - 27
    dz = sec.G.decrypt(Zg, y.size)
    assert np.abs(dz - cutmax_mirror(y, mirror2(y, coef))).max() < 1e-3
    assert int(np.argmax(dz[:x.size])) == int(np.argmax(x))


def test_cutmax_config3_batched(sec):
    """16 requests, even ids 32000 logits (1 ciphertext), odd ids 128256 (4 ciphertexts):
    requests 0 (1 ciphertext) and 1 (4 ciphertexts) are encrypted from the same plaintexts
    as the oracle's and their batched outputs equal the oracle's CutMax word for word; every
    request decrypts to its FP64 mirror within 1e-3 and recovers its argmax"""
    from paper_2509_08383_amd import he
    say("[gpu] secure: batched 16 requests")
    xs = [llm_logits(200 + r, 32000 if r % 2 == 0 else 128256) for r in range(16)]
    cfg, coef = cfg2(he)
    ys = [slot_layout(x, sec.G.slots)[0] for x in xs]
    # requests 0 and 1 through the pair (same plaintexts, counters in lockstep)
    m0 = ckks.encode(ys[0], sec.O.N, sec.O.Delta)
    g0 = sec.G.encrypt_coeffs(m0, sec.O.Delta, ys[0].size)
    o0 = sec.O.encrypt_coeffs(m0, sec.O.Delta)
    m1 = [ckks.encode(ys[1][k * sec.G.slots:(k + 1) * sec.G.slots], sec.O.N, sec.O.Delta) for k in range(4)]
    g1 = sec.G.encrypt_coeffs(np.concatenate(m1), sec.O.Delta, ys[1].size)
    o1 = [sec.O.encrypt_coeffs(m, sec.O.Delta) for m in m1]
    rest = [sec.G.encrypt(x) for x in xs[2:]]
    sec.O.nonce = sec.O.nonce + sum(c.a for c in rest)
    cts = [g0, g1] + rest
    assert [c.a for c in cts] == [1, 4] * 8
    Z = sec.G.cutmax(cts, cfg)
    say(f"  batch of 16: {sec.G.last_cutmax_ms():.1f} ms")
    for r in range(16):
        dz = sec.G.decrypt(Z[r], ys[r].size)
        err = np.abs(dz - cutmax_mirror(ys[r], mirror2(ys[r], coef))).max()
        assert err < 1e-3, (r, err)
        assert int(np.argmax(dz[:xs[r].size])) == int(np.argmax(xs[r])), r
    hc = ckks.HECfg(T=3, p=[3] * 3, c=[5.0] * 3, v_lo=VLO, v_hi=VHI, coef=coef, sum_lo=1.0, sum_hi=3.0, gold_d=3)
    say("  oracle: request 0 (1 ciphertext)")
    sec.same(Z[0], ckks.cutmax_he(sec.O, [o0], hc)[0], "batched request 0")
    say("  oracle: request 1 (4 ciphertexts)")
    Zo1 = ckks.cutmax_he(sec.O, o1, hc)
    eg = sec.G.export(Z[1])
    assert eg.shape[0] == 4
    for k in range(4):
        bad = int((eg[k] != Zo1[k].export()).sum())
        assert bad == 0, f"batched request 1, ciphertext {k}: {bad} words differ"
    assert Z[1].level == Zo1[0].level and Z[1].scale == Zo1[0].scale


def test_goldschmidt_and_newton_refinements_at_full_size(sec):
    """T=2, degree-1 guess + 2 refinements on 32000 logits: Newton and Goldschmidt both
    match the FP64 mirror within 1e-3 and recover the argmax; Goldschmidt ends one level
    lower per iteration"""
    from paper_2509_08383_amd import he
    say("[gpu] refinements at N=2^16")
    G = sec.G
    x = llm_logits(5)
    y, _, _ = slot_layout(x, G.slots)
    ct = G.encrypt(x)
    coef = [list(chebyshev_invsqrt(VLO[t] / VHI[t], 1)) for t in range(2)]
    lv = {}
    for gold in (False, True):
        cfg = he.CutmaxCfg(T=2, p=[3] * 2, c=[5.0] * 2, var_lo=VLO[:2], var_hi=VHI[:2], init_degree=1, init_coef=coef,
                           newton_steps=2, sum_lo=1.0, sum_hi=3.0, gold_d=3,
                           flags=he.HE_REFINE_GOLDSCHMIDT if gold else 0)
        Z = G.cutmax([ct], cfg)[0]
        Z = G.cutmax([ct], cfg)[0]
        say(f"  goldschmidt={gold}: {G.last_cutmax_ms():.2f} ms, output level {Z.level}")
        lv[gold] = Z.level
        mc = MirrorCfg(T=2, p=[3] * 2, c=[5.0] * 2, v_hi=VHI[:2], v_lo=VLO[:2], coef=coef, newton=2, goldschmidt=gold,
                       B=3.0 * y.size, gold_d=3, sum_lo=1.0 * y.size)
        z = G.decrypt(Z, y.size)
        assert np.abs(z - cutmax_mirror(y, mc)).max() < 1e-3
        assert int(np.argmax(z[:x.size])) == int(np.argmax(x))
    assert lv[False] - lv[True] == 2


@pytest.mark.parametrize("shift", [0.0, 20.0])
def test_masked_padding_full_size(sec, shift):
    """HE_MASK_PAD at N = 2^16 on 32000 logits padded with their mean (he_encrypt pad=NaN):
    the first 32000 outputs match the FP64 mirror run on the 32000 logits alone within
    1e-3 and recover the argmax, also when every logit is negative (shift 20)"""
    from paper_2509_08383_amd import he
    say(f"[gpu] masked padding at N=2^16 (shift {shift})")
    G = sec.G
    x = llm_logits(9) - shift
    ct = G.encrypt(x, pad=float("nan"))
    vlo, vhi = [12.0, 0.4, 0.8], [24.0, 0.9, 16.0]
    coef = [list(chebyshev_invsqrt(vlo[t] / vhi[t], 3)) for t in range(3)]
    cfg = he.CutmaxCfg(T=3, p=[3] * 3, c=[5.0] * 3, var_lo=vlo, var_hi=vhi, init_degree=3, init_coef=coef,
                       sum_lo=1.0, sum_hi=3.0, gold_d=3, flags=he.HE_MASK_PAD)
    Z = G.cutmax([ct], cfg)[0]
    Z = G.cutmax([ct], cfg)[0]
    say(f"  {G.last_cutmax_ms():.2f} ms")
    z = G.decrypt(Z, x.size)
    mc = MirrorCfg(T=3, p=[3] * 3, c=[5.0] * 3, v_hi=vhi, v_lo=vlo, coef=coef, B=3.0 * x.size, gold_d=3,
                   sum_lo=1.0 * x.size)
    err = np.abs(z - cutmax_mirror(x, mc)).max()
    say(f"  max |z - mirror(x)| = {err:.2e}")
    assert err < 1e-3
    assert int(np.argmax(z)) == int(np.argmax(x))


def test_bench_configuration_graph_replay():
    """the configuration bench.py times: a fresh 128-bit context with HIP-graph replay, the
    library's own degree-3 Chebyshev fit, the bench's 32000-logit input; the capture and two
    replays equal the eager run bit for bit and decrypt to the FP64 mirror within 1e-3; the
    16-request batch likewise replays bit-exactly"""
    from paper_2509_08383_amd import he
    say("[gpu] bench configuration: graph capture and replays")
    G = he.Context(he.SECURE)
    cfg = he.CutmaxCfg(T=3, p=[3] * 3, c=[5.0] * 3, var_lo=VLO, var_hi=VHI, init_degree=3, init_coef=None,
                       newton_steps=0, sum_lo=1.0, sum_hi=3.0, gold_d=3)
    x = llm_logits(0)
    y, _, _ = slot_layout(x, G.slots)
    ct = G.encrypt(x)
    xs = [llm_logits(200 + r, 32000 if r % 2 == 0 else 128256) for r in range(16)]
    cts = [G.encrypt(v) for v in xs]
    eager = G.export(G.cutmax([ct], cfg)[0])
    eager_b = [G.export(z) for z in G.cutmax(cts, cfg)]
    G.set_option(he.HE_OPT_GRAPH, 1)
    runs = [G.cutmax([ct], cfg)[0] for _ in range(3)]
    say(f"  replay {G.last_cutmax_ms():.2f} ms")
    for k, z in enumerate(runs):
        assert np.array_equal(G.export(z), eager), k
    for _ in range(2):
        Zb = G.cutmax(cts, cfg)
        for r in (0, 1, 14, 15):
            assert np.array_equal(G.export(Zb[r]), eager_b[r]), r
    coef = [list(chebyshev_invsqrt(VLO[t] / VHI[t], 3)) for t in range(3)]
    dz = G.decrypt(runs[-1], y.size)
    assert np.abs(dz - cutmax_mirror(y, mirror2(y, coef))).max() < 1e-3
    assert int(np.argmax(dz[:x.size])) == int(np.argmax(x))


@pytest.mark.parametrize("masked", [False, True])
def test_qwen_vocabulary_five_ciphertexts(sec, masked):
    """the largest vocabulary of the paper's experiments (Qwen2.5, 151936 logits, Table 2) in
    5 ciphertexts of 32768 slots, zero-padded or masked with mean padding: the decrypted
    outputs match the FP64 mirror of the packed vector (or of the logits alone) within 1e-3 and
    recover the argmax"""
    from paper_2509_08383_amd import he
    say(f"[gpu] 151936 logits in 5 ciphertexts (masked={masked})")
    G = sec.G
    x = llm_logits(300, 151936)
    ct = G.encrypt(x, pad=float("nan") if masked else 0.0)
    assert ct.a == 5
    cfg, coef = cfg2(he)
    if masked:
        cfg.flags = he.HE_MASK_PAD
    Z = G.cutmax([ct], cfg)[0]
    say(f"  {G.last_cutmax_ms():.1f} ms")
    if masked:
        z = G.decrypt(Z, x.size)
        mc = MirrorCfg(T=3, p=[3] * 3, c=[5.0] * 3, v_hi=VHI, v_lo=VLO, coef=coef, B=3.0 * x.size, gold_d=3,
                       sum_lo=1.0 * x.size)
        ref = cutmax_mirror(x, mc)
    else:
        y, _, _ = slot_layout(x, G.slots)
        z = G.decrypt(Z, y.size)
        ref = cutmax_mirror(y, mirror2(y, coef))
    assert np.abs(z - ref).max() < 1e-3
    assert int(np.argmax(z[:x.size])) == int(np.argmax(x))
