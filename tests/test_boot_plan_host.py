"""CPU check of the library's host-side bootstrap plan (csrc/boot_plan.cpp, compiled here
with g++ into a small driver) against the oracle's independent plan (oracle/boot.py):
butterfly groups of the slot decoding map as diagonals, the baby-step giant-step split and
its rotation amounts, the complex-slot encoder and the Chebyshev interpolant."""
import math
import os
import subprocess

import numpy as np
import pytest

from oracle import boot as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "boot_plan_driver.cpp")
PLAN = os.path.join(ROOT, "paper_2509_08383_amd", "csrc", "boot_plan.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("plan") / "boot_plan_driver")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, SRC, PLAN], check=True)
    return exe


@pytest.mark.parametrize("s,n,inv", [(64, 2, 1), (64, 3, 0), (256, 3, 1), (256, 3, 0), (2048, 3, 1),
                                     (2048, 3, 0), (1024, 4, 1)])
def test_host_plan_matches_oracle_plan(driver, s, n, inv):
    out = subprocess.run([driver, str(s), str(n), str(inv)], capture_output=True, text=True,
                         check=True).stdout.splitlines()
    groups = B.stage_groups(s, n, bool(inv))
    gi, D, seen = -1, None, 0
    for line in out:
        f = line.split()
        if f[0] == "G":
            gi += 1
            D = groups[gi]
            P = B.bsgs_plan(D, s)
            assert (int(f[2]), int(f[3]), int(f[4])) == (len(D), P.h0, P.B)
        elif f[0] == "D":
            v = np.array(f[2:], dtype=float)
            v = v[0::2] + 1j * v[1::2]
            assert np.abs(v - D[int(f[1])]).max() < 1e-12
            seen += 1
        elif f[0] == "R":
            assert [int(x) for x in f[1:]] == B.bsgs_plan(D, s).rotations(s)
        elif f[0] == "M":
            m = np.array(f[1:], dtype=np.int64)
            z = np.array([complex(math.sin(i * 0.37), math.cos(i * 1.3)) for i in range(s)])
            mo = B.encode_complex(z, 2 * s, 2.0 ** 40)
            # two FFTs round differently in the last place: coefficients within one unit
            assert np.abs(m - mo).max() <= 1
            assert np.abs(B.decode_complex(m, 2 * s, 2.0 ** 40) - z).max() < 1e-9
        elif f[0] == "C":
            c = np.array(f[1:], dtype=float)
            co = np.polynomial.chebyshev.chebinterpolate(
                lambda x: np.cos(3 * np.sqrt(np.maximum(0, (1 + x) / 2))), 31)
            assert np.abs(c - co).max() < 1e-13
    assert gi == n - 1 and seen == sum(len(g) for g in groups)
