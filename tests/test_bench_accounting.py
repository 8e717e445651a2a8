"""The benchmark's per-kernel work model (host code): the split of each signal's
iterations between the whole-solve phase on the Kronecker approximations, the grid
kernels and the tail kernel, and the bytes and flops it attributes to each."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import synth  # noqa: E402


def _trace(p):
    # signal 0: 3 iterations on the first approximation, then 5 on A; signal 1: 2 on the
    # second approximation, then 6 on A; 100 preserved atoms and 5 nonzeros throughout
    I = len(p.stages) - 1
    tr = np.zeros((2, 10, 13))
    tr[0, :3, 1], tr[0, 3:8, 1] = 0, I
    tr[1, :2, 1], tr[1, 2:8, 1] = 1, I
    tr[:, :, 2] = 100
    tr[:, :, 12] = 5
    return tr, np.array([8, 8])


def test_rows_split_between_the_three_engine_parts():
    p = synth.config4(batch=2, n=(16, 32))
    tr, its = _trace(p)
    s0, s1 = bench.row_split(p, tr, its, "hybrid", 4, True)
    assert list(s0) == [3, 2] and list(s1) == [7, 6]
    s0, s1 = bench.row_split(p, tr, its, "hybrid", 4, False)     # approximations on the grid kernels
    assert list(s0) == [0, 0] and list(s1) == [4, 4]
    s0, s1 = bench.row_split(p, tr, its, "grid", 10 ** 9, False)
    assert list(s0) == [0, 0] and list(s1) == [8, 8]


def test_work_attributed_to_each_part():
    p = synth.config4(batch=2, n=(16, 32))
    tr, its = _trace(p)
    s0, s1 = bench.row_split(p, tr, its, "hybrid", 4, True)
    w = bench.kernel_work(p, tr, its, s0, s1, True, gram_cap=0, gemm_min=0, kron_first=True)
    st = p.stages
    n1, k1, n2, k2 = st[0].dims
    f0 = 2.0 * st[0].R * k2 * n1 * (n2 + k1)
    n1, k1, n2, k2 = st[1].dims
    f1 = 2.0 * st[1].R * k2 * n1 * (n2 + k1)
    assert w["kwg_it"] == 5 and w["kwg_flops"] == 3 * f0 + 2 * f1
    # 8 grid rows on A (FP32 columns): correlations, forward gathers, residuals, updates
    N = p.N
    assert w["adj_bytes"][0] == 8 * 100 * N * 4
    assert w["fwd_bytes"][0] == 8 * (N * (4 + 8) + 12 * 5 + 5 * N * 4)
    assert w["upd_bytes"][0] == 8 * 100 * bench.UPD_BYTES_PER_ATOM
    assert w["step_bytes"] == w["fwd_bytes"][0] + w["upd_bytes"][0]
    # 1 + 2 tail rows, in column mode (no Gram capacity given)
    assert w["dense_it"][1] == 3 and w["adj_bytes"][1] == 3 * 100 * N * 4
