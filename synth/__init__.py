"""Seeded synthetic inputs for the stable-screening Lasso solver.

This package is the only code shared by the FP64 oracle's tests and the GPU
path's tests and benchmark.  It builds dictionaries, their structured or
low-precision approximations (with exact per-atom error bounds), and signals.
It holds none of the solver's arithmetic: no FISTA step, no dual point, no
screening test, no switching rule.
"""
from .workloads import (  # noqa: F401
    SEED_BASE, Stage, Problem, rng_for,
    kron_dictionary, nkp_factors, kron_stage, quantized_stage, exact_stage,
    signals, config1, config2, config3, config4, config5, config6, kron_near_exact,
    faust_chain, faust_dictionary, faust_stage, with_lq_bounds,
    bf16_round, fp8_e4m3_round, fp8_e4m3_decode, bf16_decode,
)
