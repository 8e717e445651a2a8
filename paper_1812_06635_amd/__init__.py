"""stablel1 -- Lasso with stable safe screening over fast approximate
dictionaries (Dantas & Gribonval, arXiv 1812.06635), native to MI355X (gfx950).

The solver runs in the HIP library built from ``csrc/`` (C ABI in
``include/stablel1.h``); this package only marshals torch tensors to it.
"""
from .api import (Dict, LassoFunction, adjoint, grad, lambda_max, lasso, last_solve_clock, last_solve_phases,  # noqa: F401
                  tune_kron,
                  solve_path,
                  last_solve_profile,
                  measure_rc, solve, upload_stage)
from ._lib import load as load_library  # noqa: F401
