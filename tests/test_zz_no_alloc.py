"""GPU: the rotate-and-sum entry point that allocates nothing (he_rotsum_noalloc) against
he_rotsum, word for word, on two calls in a row (the second with a smaller input), at the
toy size and at N = 2^16; a call whose workspace exceeds the static scratch is refused
before any kernel runs."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check_pair(G, ct, out, what):
    ref = G.rotsum(ct)
    G.rotsum_noalloc(ct, out)
    ea, eb = G.export(ref), G.export(out)
    assert ea.shape == eb.shape, (what, ea.shape, eb.shape)
    bad = int((ea != eb).sum())
    assert bad == 0, f"{what}: {bad} words differ"
    assert ref.info()[1] == out.info()[1] and ref.info()[2] == out.info()[2], what
    return ref


def test_rotsum_noalloc_matches_rotsum_toy():
    from paper_2509_08383_amd import he
    say("[gpu] no-alloc rotate-and-sum, toy")
    G = he.Context(he.TOY)
    rng = np.random.default_rng(31)
    # first call: a 3-ciphertext handle at the top level
    x = rng.uniform(-1, 1, 3 * G.slots)
    ct = G.encrypt(x)
    out = G.encrypt(np.zeros(3 * G.slots))
    ref = _check_pair(G, ct, out, "3 ciphertexts, top level")
    np.testing.assert_allclose(G.decrypt(out)[:G.slots], np.full(G.slots, x[:G.slots].sum()), atol=1e-3)
    # second call, smaller: one ciphertext at a low level (partial key-switch digit)
    y = rng.uniform(-1, 1, G.slots)
    ct2 = G.drop(G.encrypt(y), 4)
    out2 = G.encrypt(np.zeros(G.slots))
    _check_pair(G, ct2, out2, "1 ciphertext, level 4")
    # in place (out is the input) equals the out-of-place result
    G.rotsum_noalloc(ct, ct)
    assert np.array_equal(G.export(ct), G.export(ref))
    # refused: too large for the scratch, or mismatched handles
    big = G.encrypt(np.zeros(40 * G.slots))
    with pytest.raises(he.HeError) as e:
        G.rotsum_noalloc(big, big)
    assert e.value.code == he.HE_ENOMEM
    with pytest.raises(he.HeError) as e:
        G.rotsum_noalloc(ct2, out)
    assert e.value.code == he.HE_EINVAL
    G.close()


def test_rotsum_noalloc_matches_rotsum_full_size():
    from paper_2509_08383_amd import he
    say("[gpu] no-alloc rotate-and-sum, N=2^16")
    G = he.Context(he.SECURE)
    rng = np.random.default_rng(32)
    x = rng.uniform(-1, 1, G.slots)
    ct = G.encrypt(x)
    out = G.encrypt(np.zeros(G.slots))
    _check_pair(G, ct, out, "N=2^16 top level")
    np.testing.assert_allclose(G.decrypt(out)[:8], np.full(8, x.sum()), atol=1e-4)
    ct2 = G.drop(G.encrypt(rng.uniform(-1, 1, G.slots)), 11)
    _check_pair(G, ct2, out, "N=2^16 level 11")
    two = G.encrypt(rng.uniform(-1, 1, 2 * G.slots))
    with pytest.raises(he.HeError) as e:
        G.rotsum_noalloc(two, G.encrypt(np.zeros(2 * G.slots)))
    assert e.value.code == he.HE_ENOMEM
    G.close()
