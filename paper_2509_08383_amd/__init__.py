"""Encrypted CutMax (arXiv 2509.08383) on MI355X: RNS-CKKS with hand-written gfx950 HIP kernels.

The compute path is ``libcutmax_he.so`` (C ABI in ``include/he.h``); ``he`` is its ctypes binding.
"""
from . import he  # noqa: F401
