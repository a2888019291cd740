"""CPU checks of the boundary: the library loads and exports every entry point include/he.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "he.h")
LIB = os.path.join(ROOT, "paper_2509_08383_amd", "libcutmax_he.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(he_[a-z0-9_]+)\s*\(", text)))


def _ensure_built():
    if not os.path.exists(LIB):
        from paper_2509_08383_amd import build
        build.build(verbose=False)


def test_header_declares_the_five_calls():
    names = declared_functions()
    for n in ("he_ctx_create", "he_encrypt", "he_cutmax", "he_topp_sample", "he_decrypt"):
        assert n in names


def test_library_exports_every_declared_symbol():
    _ensure_built()
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_topp_noise_is_host_only():
    """he_topp_noise needs no GPU: G = U^(1/alpha), alpha = ln(1-p)/ln p (Alg. 3)."""
    _ensure_built()
    import numpy as np
    from paper_2509_08383_amd import he
    from oracle.cutmax_fp64 import beta_alpha, beta_noise
    from workloads import uniform_noise
    u = uniform_noise(3, 1000)
    g = he.topp_noise(0.9, u)
    np.testing.assert_allclose(g, beta_noise(u, beta_alpha(0.9)), rtol=1e-14)
    with pytest.raises(he.HeError):
        he.topp_noise(1.5, u)


def test_gumbel_noise_is_host_only():
    """he_gumbel_noise needs no GPU: G = -ln(-ln U) (Sec. 3.3); U outside (0, 1) is an error."""
    _ensure_built()
    import numpy as np
    from paper_2509_08383_amd import he
    from oracle.cutmax_fp64 import gumbel_noise
    from workloads import uniform_noise
    u = uniform_noise(5, 1000)
    np.testing.assert_allclose(he.gumbel_noise(u), gumbel_noise(u), rtol=1e-13, atol=1e-14)
    for bad in (0.0, 1.0):
        with pytest.raises(he.HeError):
            he.gumbel_noise(np.array([0.5, bad]))


def test_errors_without_gpu_are_loud():
    """Creating a context without a GPU fails with an error, never a silent fallback."""
    _ensure_built()
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2509_08383_amd import he
    with pytest.raises(he.HeError):
        he.Context(he.TOY)


@pytest.mark.gpu
def test_plain_c_client_recovers_the_argmax():
    """a C program that sees only include/he.h (host pointers in, host pointers out) runs
    encrypt, CutMax and decrypt on the GPU and recovers the plaintext arg-max"""
    import subprocess
    exe = os.path.join(ROOT, "tests", "c_client", "cutmax_client")
    if not os.path.exists(exe):
        pytest.skip("the C client is built by __graft_entry__.build()")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    got, want = r.stdout.split()[1:3]
    assert got == want


@pytest.mark.gpu
def test_plain_c_client_bootstraps():
    """the same C program drives he_boot_setup and he_bootstrap through the ABI: 2048 values
    in [-1, 1] come back from level 3 to level 3 (19 - 16) within 1e-3"""
    import subprocess
    exe = os.path.join(ROOT, "tests", "c_client", "cutmax_client")
    if not os.path.exists(exe):
        pytest.skip("the C client is built by __graft_entry__.build()")
    r = subprocess.run([exe, "boot"], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    f = r.stdout.split()
    assert f[0] == "boot" and float(f[2]) < 1e-3 and f[4] == "3"


def test_invsqrt_guess_fit_is_host_only_and_matches_the_oracle():
    """he_invsqrt_guess_fit needs no GPU: the Chebyshev interpolant of u^(-1/2) on
    [u_lo, 1] (Sec. 3.2 (ii), a known domain) equals the oracle's own fit, and its
    interpolation nodes are exact"""
    _ensure_built()
    import numpy as np
    from paper_2509_08383_amd import he
    from oracle.cutmax_fp64 import chebyshev_invsqrt, poly_eval
    for u_lo in (0.05, 0.5):
        for d in (1, 2, 3, 4):
            c = he.invsqrt_guess_fit(u_lo, d)
            np.testing.assert_allclose(c, chebyshev_invsqrt(u_lo, d), rtol=1e-9, atol=1e-9)
            k = np.arange(d + 1)
            nodes = 0.5 * (1 + u_lo) + 0.5 * (1 - u_lo) * np.cos((2 * k + 1) * np.pi / (2 * (d + 1)))
            np.testing.assert_allclose(poly_eval(c, nodes), nodes ** -0.5, rtol=1e-9)
    with pytest.raises(he.HeError):
        he.invsqrt_guess_fit(1.5, 3)


def test_invsqrt_scaled_plan_is_host_only_and_matches_the_oracle():
    """he_invsqrt_scaled_plan needs no GPU: its guess, refinement constants and ranges equal
    the oracle's own plan for the same domain (wide-domain inverse square root of the Table 2
    schedule), and it refuses a bad domain"""
    _ensure_built()
    import numpy as np
    from paper_2509_08383_amd import he
    from oracle.cutmax_fp64 import scaled_invsqrt_plan
    for u_lo, K in ((2.5e-6, 7), (2.5e-4, 5), (0.5, 0)):
        g, st, rg = he.invsqrt_scaled_plan(u_lo, 3, K)
        go, sto, rgo = scaled_invsqrt_plan(u_lo, 3, K)
        np.testing.assert_allclose(g, go, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(np.array(st).reshape(-1, 2) if K else np.zeros((0, 2)),
                                   np.array(sto).reshape(-1, 2) if K else np.zeros((0, 2)), rtol=1e-9)
        np.testing.assert_allclose(np.array(rg), np.array(rgo), rtol=1e-9)
    with pytest.raises(he.HeError):
        he.invsqrt_scaled_plan(0.0, 3, 2)


def _mlp_file_bytes(theta, mean, sd, poly):
    """a learned-guess file written from the layout include/he.h documents (he_mlp_save)"""
    import struct
    import numpy as np
    body = b"HEMLPv1\n" + struct.pack("<IIff", 321, 16, mean, sd) + np.asarray(theta, "<f4").tobytes() \
        + np.asarray(poly, "<f8").tobytes()
    h = 0xcbf29ce484222325
    for byte in body:
        h = ((h ^ byte) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return body + struct.pack("<Q", h)


def test_learned_guess_file_is_read_without_gpu(tmp_path):
    """he_mlp_file_poly reads the collapsed quartic of a learned-guess file with no GPU: a
    file built here from the documented layout, with the quartic from the independent
    collapse (oracle/mlp_ref.to_poly), is accepted and its coefficients returned as stored;
    a flipped weight byte (checksum), a stored quartic that is not the weights' collapse
    (checksum recomputed), a truncated file, another magic and a missing file are refused"""
    _ensure_built()
    import numpy as np
    from paper_2509_08383_amd import he
    from oracle.mlp_ref import to_poly
    rng = np.random.default_rng(3)
    theta = (0.3 * rng.standard_normal(321)).astype(np.float32)
    mean, sd = np.float32(0.42), np.float32(0.29)
    poly = to_poly(theta.astype(np.float64), float(mean), float(sd))
    good = _mlp_file_bytes(theta, mean, sd, poly)
    assert len(good) == 1356
    f = tmp_path / "guess.bin"
    f.write_bytes(good)
    assert (he.mlp_file_poly(str(f)) == poly).all()
    cases = {}
    flipped = bytearray(good)
    flipped[24 + 4 * 100] ^= 0x01
    cases["checksum"] = bytes(flipped)
    off = poly.copy()
    off[2] *= 1.0 + 1e-6
    cases["collapse"] = _mlp_file_bytes(theta, mean, sd, off)
    cases["bytes"] = good[:-9]
    cases["not a learned-guess file"] = b"HEMLPv2\n" + good[8:]
    for what, data in cases.items():
        f.write_bytes(data)
        with pytest.raises(he.HeError) as e:
            he.mlp_file_poly(str(f))
        assert e.value.code == he.HE_EINVAL and what in str(e.value), (what, str(e.value))
    with pytest.raises(he.HeError) as e:
        he.mlp_file_poly(str(tmp_path / "missing.bin"))
    assert e.value.code == he.HE_EIO
