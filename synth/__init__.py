"""Seeded synthetic inputs shared by the tests, the oracle and the benchmark.

This package only builds input matrices (planted spectra, noise, offsets and
ragged batches).  It contains none of the randomized-SVD arithmetic, so the
oracle and the HIP path can both consume its output without sharing any part
of the method.
"""
from .matrices import (  # noqa: F401
    haar, planted, planted_torch, spectrum, CONFIGS, harmonic_2000x1000, tall_exp_matrix,
    tall_exp_offsets, poly_bf16_torch, ragged_batch, paper_lowrank_product,
)
