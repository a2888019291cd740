"""The block structure of NTT-domain automorphisms that the staged rotation key products
rely on (host-side check of the mathematics, no GPU).

With the NTT output at position j holding the evaluation at psi^(2 brev(j) + 1), the
automorphism X -> X^g reads position src(j) with 2 brev(src) + 1 = g (2 brev(j) + 1) mod 2N.
Two facts are used: every aligned block of 256 positions is sent onto one aligned block
(and every aligned 64-position wave onto one aligned 64-word range), and which block
depends only on g mod N/128.  For a radix-8 rotate-and-sum over N/2 slots the Galois
elements 5^(r 8^s) then take at most one residue besides 1 in the last steps, so those
steps read their sources from at most two blocks."""
import numpy as np
import pytest


def brev(x, bits):
    return int(format(x, f"0{bits}b")[::-1], 2)


def src_map(g, logn):
    n = 1 << logn
    e = np.array([brev(j, logn) for j in range(n)], dtype=np.int64)
    t = (g * (2 * e + 1)) % (2 * n)
    e2 = (t - 1) // 2
    return np.array([brev(int(v), logn) for v in e2], dtype=np.int64)


@pytest.mark.parametrize("logn", [12, 14])
def test_blocks_map_onto_blocks_by_residue(logn):
    n, m = 1 << logn, 2 << logn
    rm = n // 128
    seen = {}
    for k in list(range(1, 24)) + [n // 2 - 1, n // 4]:
        for g in (pow(5, k, m), (m - pow(5, k, m)) % m):
            s = src_map(g, logn)
            blocks = s.reshape(-1, 256) >> 8
            assert (blocks == blocks[:, :1]).all()               # one source block per block
            waves = s.reshape(-1, 64) >> 6
            assert (waves == waves[:, :1]).all()                 # one 64-word range per wave
            bmap = tuple(blocks[:, 0])
            assert seen.setdefault(g % rm, bmap) == bmap         # depends on g mod N/128 only
            if g % rm == 1:
                assert bmap == tuple(range(n // 256))            # residue 1: every block itself


def test_radix8_steps_have_few_source_blocks_at_n65536():
    n, m = 1 << 16, 2 << 16
    rm = n // 128
    step, res = 1, []
    while step < n // 2:
        res.append(sorted({pow(5, r * step, m) % rm for r in range(1, 8)}))
        step *= 8
    assert [len(r) for r in res] == [7, 7, 2, 1, 1]
    assert res[2] == [1, 257] and res[3] == [1] and res[4] == [1]
