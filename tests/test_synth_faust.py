"""FAuST inputs (products of sparse factors, the structured family used for the
MEG operator in Section V-G): the stored factors, their dense value, the per-atom
error bounds and the relative-complexity model, each checked against an
independent computation."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from synth import workloads as sw


def _small():
    return synth.config6(N=64, K=515, depth=3, col_nnz=(8, 8, 24), keeps=(8, 12, 16), lam_frac=0.2)


def test_factor_chain_applied_with_sparse_products_matches_the_dense_value():
    p = _small()
    rng = np.random.default_rng(0)
    for st in p.stages[:-1]:
        mats = [sp.csr_matrix((np.asarray(v, dtype=np.float64), ci, rp), shape=(st.dims[l], st.dims[l + 1]))
                for l, (rp, ci, v) in enumerate(st.factors)]
        V = st.values()
        assert V.shape == (p.N, p.K)
        for _ in range(3):
            x = rng.standard_normal(p.K)
            u = x
            for M in reversed(mats):          # S_1 (S_2 (... (S_J x)))
                u = M @ u
            np.testing.assert_allclose(u, V @ x, rtol=1e-12, atol=1e-12 * np.abs(V).sum())
            z = rng.standard_normal(p.N)
            g = z
            for M in mats:                    # S_J^T (... (S_1^T z))
                g = M.T @ g
            np.testing.assert_allclose(g, V.T @ z, rtol=1e-12, atol=1e-12 * np.abs(V).sum())


def test_csr_layout_rows_sorted_and_in_range():
    for st in _small().stages[:-1]:
        assert st.kind == "faust" and st.dims[0] == st.N and st.dims[-1] == st.K
        for l, (rp, ci, v) in enumerate(st.factors):
            assert rp.dtype == np.int32 and ci.dtype == np.int32 and rp[0] == 0 and rp[-1] == len(ci) == len(v)
            assert np.all(np.diff(rp) >= 0) and np.all((ci >= 0) & (ci < st.dims[l + 1]))
            for r in range(st.dims[l]):
                row = ci[rp[r]:rp[r + 1]]
                assert np.all(np.diff(row) > 0)   # strictly increasing columns in a row


def test_error_bounds_cover_every_atom_and_shrink_with_the_kept_entries():
    p = _small()
    means = []
    for st in p.stages[:-1]:
        d = np.linalg.norm(p.A - st.values(), axis=0)
        assert np.all(d <= st.eps) and np.all(st.eps <= d + 1e-9)
        means.append(float(st.eps.mean()))
    assert means == sorted(means, reverse=True) and means[0] > means[-1]


def test_relative_complexity_is_the_nonzero_count_over_nk():
    p = _small()
    for st in p.stages[:-1]:
        nnz = sum(int(np.count_nonzero(M)) for M in st.factor_matrices())
        assert st.rc_theory == pytest.approx(nnz / (p.N * p.K), rel=1e-15)


def test_pruning_keeps_the_largest_entries_of_each_last_factor_column():
    A, S = sw.faust_dictionary(sw.rng_for(6, 7, 0), (32, 32, 100), (8, 12), 0.01, "f64")
    st = sw.faust_stage(A, S, 5, "f64")
    last = st.factor_matrices()[-1]
    assert np.all(np.count_nonzero(last, axis=0) == 5)
    full = np.abs(S[-1])
    for j in range(full.shape[1]):
        kept = np.abs(last[:, j])[last[:, j] != 0]
        dropped = full[:, j][(last[:, j] == 0) & (full[:, j] != 0)]
        assert dropped.size == 7 and kept.min() >= dropped.max()
