"""GPU checks of the encrypted one-shot nucleus sampler (Alg. 3): 32000-token
logits at temperature 0.8, client-drawn uniform noise turned into Beta(alpha, 1) noise
(alpha = ln(0.1)/ln(0.9)) and encrypted, batch 8; the decrypted one-hot approximation
picks the token the FP64 sampler argmax(x/tau + G) picks on the same noise."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle.cutmax_fp64 import (MirrorCfg, beta_alpha, beta_noise, chebyshev_invsqrt, cutmax_mirror,  # noqa: E402
                                nucleus_argmax, nucleus_set, slot_layout)
from workloads import llm_logits, uniform_noise  # noqa: E402
from test_gpu_parity import say  # noqa: E402

VLO, VHI = [12.0, 0.4, 0.8], [24.0, 0.9, 16.0]
TOP_P, TAU = 0.9, 0.8


def _cfg(he, prescaled):
    coef = [list(chebyshev_invsqrt(VLO[t] / VHI[t], 3)) for t in range(3)]
    gold = 3       # 27 levels; the temperature multiply (not prescaled) uses the 28th
    return he.CutmaxCfg(T=3, p=[3] * 3, c=[5.0] * 3, var_lo=VLO, var_hi=VHI, init_coef=coef, sum_lo=1.0,
                        sum_hi=3.0, gold_d=gold, flags=he.HE_NOISE_PRESCALED if prescaled else 0), coef, gold


@pytest.mark.parametrize("prescaled", [False, True])
def test_topp_sample_batch8(prescaled):
    from paper_2509_08383_amd import he
    say(f"[gpu] nucleus sampling batch 8 (prescaled={prescaled})")
    G = he.Context(he.SECURE)
    alpha = beta_alpha(TOP_P)
    xs = [llm_logits(700 + r) for r in range(8)]
    gs = [beta_noise(uniform_noise(900 + r, xs[r].size), alpha) for r in range(8)]
    cts = [G.encrypt(x) for x in xs]
    nz = [G.encrypt(TAU * g if prescaled else g) for g in gs]
    cfg, coef, gold = _cfg(he, prescaled)
    Z = G.topp_sample(cts, nz, TOP_P, TAU, cfg)
    say(f"  {G.last_cutmax_ms():.1f} ms for 8 requests")
    inside = 0
    for r in range(8):
        pick = nucleus_argmax(xs[r], gs[r], TAU)
        z = G.decrypt(Z[r], 32768)
        assert int(np.argmax(z[:32000])) == pick, r
        inside += int(pick in set(nucleus_set(xs[r], TOP_P, TAU).tolist()))
        if r < 2:
            y, _, _ = slot_layout(xs[r] + TAU * gs[r], G.slots)
            mc = MirrorCfg(T=3, p=[3] * 3, c=[5.0] * 3, v_hi=VHI, v_lo=VLO, coef=coef, B=3.0 * y.size, gold_d=gold,
                           sum_lo=1.0 * y.size)
            assert np.abs(z - cutmax_mirror(y, mc)).max() < 1e-3
    assert inside == 8


def test_topp_noise_helper_matches_lemma():
    from paper_2509_08383_amd import he
    u = uniform_noise(3, 10000)
    np.testing.assert_allclose(he.topp_noise(TOP_P, u), beta_noise(u, beta_alpha(TOP_P)), rtol=1e-14)
