"""Seeded synthetic workloads (random draws only, no method arithmetic)."""
from .logits import (toy_logits, llm_logits, llm_logits_var, uniform_noise,  # noqa: F401
                     random_residues, random_small_poly,
                     VOCAB_MISTRAL_LIKE, VOCAB_LLAMA3_LIKE)
