"""Seeded synthetic inputs shared by the tests, the oracle checks and bench.py.

This module draws random numbers only.  It holds none of the method's
arithmetic (no CutMax step, no CKKS step): every generator returns plain
float64 arrays built from ``numpy.random.default_rng(seed)``.

The paper evaluates on next-token logits of Mistral-7B (|V| = 32,768),
Qwen2.5-0.5B (|V| ~ 150K) and GPT-2 over arXiv abstracts (Sec. 4, Table 2);
neither the data nor the weights are available, so these generators stand in
for them with LLM-like shapes:

* ``toy_logits``     N(0,1) values with the maximum lifted by a gap ~ U[0.5, 2]
* ``llm_logits``     3 * Gumbel(0,1) minus 1.1 * ln(rank) over a random
                     permutation of ranks 1..V (a Zipf(1.1) rank bias in log space)
* ``llm_logits_var`` the same family with the Gumbel scale ~ U[1.5, 4.5] and the
                     Zipf exponent ~ U[0.9, 1.3] drawn per vector
* ``uniform_noise``  U(0,1) draws a client uses for the nucleus sampler's noise
"""
from __future__ import annotations

import numpy as np

VOCAB_MISTRAL_LIKE = 32000
VOCAB_LLAMA3_LIKE = 128256


def toy_logits(seed: int, n: int = 1024) -> np.ndarray:
    """n values ~ N(0,1); the arg-max entry is raised to runner-up + g, g ~ U[0.5, 2]."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n)
    i = int(np.argmax(x))
    g = rng.uniform(0.5, 2.0)
    rest = np.delete(x, i)
    x[i] = rest.max() + g
    return x


def llm_logits(seed: int, vocab: int = VOCAB_MISTRAL_LIKE, scale: float = 3.0,
               zipf: float = 1.1) -> np.ndarray:
    """x_i = scale * G_i - zipf * ln(r_i), G ~ Gumbel(0,1), r a random permutation of 1..vocab."""
    rng = np.random.default_rng(seed)
    g = rng.gumbel(0.0, 1.0, vocab)
    r = rng.permutation(vocab) + 1
    return scale * g - zipf * np.log(r.astype(np.float64))


def llm_logits_var(seed: int, vocab: int = VOCAB_MISTRAL_LIKE) -> np.ndarray:
    """LLM-like logits with a per-vector Gumbel scale ~ U[1.5,4.5] and Zipf exponent ~ U[0.9,1.3]."""
    rng = np.random.default_rng(seed)
    scale = rng.uniform(1.5, 4.5)
    zipf = rng.uniform(0.9, 1.3)
    sub = int(rng.integers(0, 2**31 - 1))
    return llm_logits(sub, vocab, scale, zipf)


def uniform_noise(seed: int, n: int) -> np.ndarray:
    """n draws of U(0,1), open at 0 (values below 1e-300 are bumped up)."""
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    return np.maximum(u, 1e-300)


def random_residues(seed: int, primes, n: int) -> np.ndarray:
    """Uniform residues mod each prime: array [len(primes), n] of uint64."""
    rng = np.random.default_rng(seed)
    out = np.empty((len(primes), n), dtype=np.uint64)
    for i, q in enumerate(primes):
        out[i] = rng.integers(0, int(q), size=n, dtype=np.uint64)
    return out


def random_small_poly(seed: int, n: int, bound: int) -> np.ndarray:
    """n integers uniform in [-bound, bound] (int64), e.g. a plaintext polynomial."""
    rng = np.random.default_rng(seed)
    return rng.integers(-bound, bound + 1, size=n, dtype=np.int64)
