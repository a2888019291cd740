"""GPU checks of the encrypted Gumbel-max sampler (Sec. 3.3, Gumbel-max trick) and an
encrypted violation-rate count (Sec. 4, "Nucleus Sampling", Fig. 4) on 32000-token
LLM-like logits: the client turns uniform draws into Gumbel(0,1) or Beta(alpha, 1)
noise and encrypts it; the server runs CutMax on X + tau*G; the decrypted one-hot
picks the token argmax(x/tau + G) picks on the same noise."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle.cutmax_fp64 import (MirrorCfg, beta_alpha, beta_noise, chebyshev_invsqrt, cutmax_mirror,  # noqa: E402
                                gumbel_noise, nucleus_argmax, slot_layout, violation_rate)
from workloads import llm_logits, llm_logits_var, uniform_noise  # noqa: E402
from test_gpu_parity import say  # noqa: E402
from test_gpu_topp import VHI, VLO, _cfg  # noqa: E402

TAU = 0.8


@pytest.mark.parametrize("prescaled", [False, True])
def test_gumbel_sample_batch8(prescaled):
    from paper_2509_08383_amd import he
    say(f"[gpu] Gumbel-max sampling batch 8 (prescaled={prescaled})")
    G = he.Context(he.SECURE)
    xs = [llm_logits(700 + r) for r in range(8)]
    gs = [he.gumbel_noise(uniform_noise(1900 + r, xs[r].size)) for r in range(8)]
    cts = [G.encrypt(x) for x in xs]
    nz = [G.encrypt(TAU * g if prescaled else g) for g in gs]
    cfg, coef, gold = _cfg(he, prescaled)
    Z = G.gumbel_sample(cts, nz, TAU, cfg)
    say(f"  {G.last_cutmax_ms():.1f} ms for 8 requests")
    for r in range(8):
        np.testing.assert_allclose(gs[r], gumbel_noise(uniform_noise(1900 + r, xs[r].size)), rtol=1e-13, atol=1e-14)
        z = G.decrypt(Z[r], 32768)
        assert int(np.argmax(z[:32000])) == nucleus_argmax(xs[r], gs[r], TAU), r
        if r < 2:
            y, _, _ = slot_layout(xs[r] + TAU * gs[r], G.slots)
            mc = MirrorCfg(T=3, p=[3] * 3, c=[5.0] * 3, v_hi=VHI, v_lo=VLO, coef=coef, B=3.0 * y.size, gold_d=gold,
                           sum_lo=1.0 * y.size)
            assert np.abs(z - cutmax_mirror(y, mc)).max() < 1e-3


def test_gumbel_sample_rejects_bad_arguments():
    from paper_2509_08383_amd import he
    G = he.Context(he.TOY)
    x = G.encrypt(np.zeros(8))
    cfg, _, _ = _cfg(he, False)
    with pytest.raises(he.HeError):
        G.gumbel_sample([x], [x], 0.0, cfg)


def test_encrypted_violation_counts():
    """A small encrypted run of the Fig. 4 measurement: 4 prompts x 4 draws per sampler at
    p = 0.9, tau = 1; every encrypted pick equals the plaintext pick on the same noise, the
    Beta-cut picks never leave the nucleus, and the Gumbel-max violations equal those of the
    plaintext picks."""
    from paper_2509_08383_amd import he
    say("[gpu] encrypted violation counts, 4 prompts x 4 draws x 2 samplers")
    P, S, D = 0.9, 4, 4
    G = he.Context(he.SECURE)
    # with the per-prompt Gumbel scale and Zipf exponent of these logits, the variances of
    # the three iterations span about [6, 37], [0.33, 0.77] and [1, 116]
    vlo, vhi = [5.0, 0.3, 0.6], [48.0, 1.0, 128.0]
    cfg = he.CutmaxCfg(T=3, p=[3] * 3, c=[5.0] * 3, var_lo=vlo, var_hi=vhi,
                       init_coef=[list(chebyshev_invsqrt(vlo[t] / vhi[t], 3)) for t in range(3)], sum_lo=1.0,
                       sum_hi=4.0, gold_d=3, flags=he.HE_NOISE_PRESCALED)
    al = beta_alpha(P)
    xs = [llm_logits_var(5000 + s) for s in range(S)]
    cts = [G.encrypt(x) for x in xs]
    picks = {"gumbel": [[] for _ in range(S)], "beta": [[] for _ in range(S)]}
    for d in range(D):
        us = [uniform_noise(9000 + 16 * s + d, xs[s].size) for s in range(S)]
        for kind in ("gumbel", "beta"):
            gs = [he.gumbel_noise(u) if kind == "gumbel" else he.topp_noise(P, u) for u in us]
            nz = [G.encrypt(g) for g in gs]
            Z = (G.gumbel_sample(cts, nz, 1.0, cfg) if kind == "gumbel" else G.topp_sample(cts, nz, P, 1.0, cfg))
            for s in range(S):
                pick = int(np.argmax(G.decrypt(Z[s], 32768)[:32000]))
                ref = beta_noise(us[s], al) if kind == "beta" else gumbel_noise(us[s])
                assert pick == nucleus_argmax(xs[s], ref, 1.0), (kind, s, d)
                picks[kind][s].append(pick)
    vg = [violation_rate(xs[s], picks["gumbel"][s], P) for s in range(S)]
    vb = [violation_rate(xs[s], picks["beta"][s], P) for s in range(S)]
    say(f"  Gumbel-max violation rate {np.mean(vg):.3f}, Beta-cut {np.mean(vb):.3f}")
    assert max(vb) == 0.0


def test_gumbel_sample_with_masked_padding():
    """Gumbel-max sampling with HE_MASK_PAD: logits padded with their mean, noise with 0, so
    the pad slots of X + tau G hold the logits' pad value the tracker starts from; the
    decrypted outputs on the 32000 real slots match the FP64 mirror of x + tau g alone and
    pick argmax(x/tau + G)"""
    from paper_2509_08383_amd import he
    say("[gpu] Gumbel-max sampling with masked padding")
    G = he.Context(he.SECURE)
    xs = [llm_logits(710 + r) for r in range(4)]
    gs = [he.gumbel_noise(uniform_noise(1910 + r, xs[r].size)) for r in range(4)]
    cts = [G.encrypt(x, pad=float("nan")) for x in xs]
    nz = [G.encrypt(g) for g in gs]
    cfg, coef, gold = _cfg(he, False)
    cfg.flags = he.HE_MASK_PAD
    Z = G.gumbel_sample(cts, nz, TAU, cfg)
    for r in range(4):
        z = G.decrypt(Z[r], xs[r].size)
        assert int(np.argmax(z)) == nucleus_argmax(xs[r], gs[r], TAU), r
        w = xs[r] + TAU * gs[r]
        mc = MirrorCfg(T=3, p=[3] * 3, c=[5.0] * 3, v_hi=VHI, v_lo=VLO, coef=coef, B=3.0 * w.size, gold_d=gold,
                       sum_lo=1.0 * w.size)
        assert np.abs(z - cutmax_mirror(w, mc)).max() < 1e-3, r
