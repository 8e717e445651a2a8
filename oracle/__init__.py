"""FP64 CPU oracle for the stable-screening Lasso solver -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from this package.  The GPU solver never
calls, links or loads it, and it shares no code with the GPU path: the two meet
only through the seeded inputs of the ``synth`` package.

Modules
-------
lasso      the plain definition: the Lasso solution by FISTA in FP64 with the
           exact dictionary and no screening, a support polish and a KKT
           certificate, plus a brute-force enumeration for tiny problems.
screening  the paper's method step by step (Algorithm 1 with Algorithm 2,
           FISTA updates, the stable GAP Safe test of Table I) in FP64, used
           as the per-iteration reference for the GPU trace.
"""
from . import lasso, screening  # noqa: F401
