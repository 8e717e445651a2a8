"""GPU parity of the HIP solver against the FP64 oracle (run with -m gpu).

Every call goes through the C ABI (via the ctypes binding).  Inputs come from
the seeded generators in ``synth``; expected values come from ``oracle`` only.
"""
import numpy as np
import pytest

import oracle.lasso as ol
import oracle.screening as osc
import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sl1():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1812_06635_amd as m
    m.load_library()
    return m


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _run(sl1, p, tol, stages=None, **kw):
    import torch
    ups = [sl1.upload_stage(s) for s in (stages or p.stages)]
    st = stages or p.stages
    wt = torch.float64 if p.work == "f64" else torch.float32
    out = sl1.solve(ups, [s.L for s in st], [s.rc_theory for s in st], _t(p.atom_norm), _t(p.Y, wt), _t(p.lam),
                    tol=tol, **kw)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
    return res


# ---------------------------------------------------------------------------
# kernel-level parity: every adjoint variant, atom by atom
# ---------------------------------------------------------------------------
ADJ_CASES = [
    ("C1 kron f64 + dense f64", lambda: synth.config1(), 1e-12),
    ("C2-small kron f32", lambda: synth.config2(n=(16, 32)), 2e-5),
    ("C3-small dense fp8/bf16/f32", lambda: synth.config3(N=256, K=1024), 1e-12),
    ("C3 ragged N=2500", lambda: synth.config3(N=2500, K=600, s=20), 1e-12),
    ("C4-small kron bf16", lambda: synth.config4(batch=3, n=(16, 32)), 3e-5),
    ("C4-small kron fp8", lambda: synth.config4(batch=3, n=(16, 32), factor_dtype="fp8"), 3e-5),
    ("C4 kron fp8 n=(32,64)", lambda: synth.config4(batch=2, factor_dtype="fp8"), 3e-5),
    ("kron f32 n=(32,64) R=4", lambda: synth.config2(n=(32, 64), R_A=4, Rs=(1, 4)), 2e-5),
    ("C6-small faust f32 ragged K", lambda: synth.config6(N=64, K=1537, depth=3, col_nnz=(8, 8, 24),
                                                          keeps=(8, 16), batch=3), 1e-12),
    ("faust f64 one factor", lambda: synth.config6(N=48, K=333, depth=1, col_nnz=(12,), keeps=(6,),
                                                   dtype="f64", work="f64", batch=2), 1e-12),
]


@pytest.mark.parametrize("name,maker,rtol", ADJ_CASES, ids=[c[0] for c in ADJ_CASES])
def test_adjoint_kernels_match_oracle_products(sl1, name, maker, rtol):
    import torch
    p = maker()
    wt = torch.float64 if p.work == "f64" else torch.float32
    for k, st in enumerate(p.stages):
        _say(f"adjoint {name} stage {k} {st.label}")
        d = sl1.upload_stage(st)
        g, z = sl1.adjoint(d, _t(p.Y, wt))
        g, z = g.cpu().numpy(), z.cpu().numpy().astype(np.float64)
        At = st.values()
        ref = z @ At                                   # a~_j^T z in FP64
        if st.kind == "kron":                          # accumulation scale: sum_r |b_r| kron |c_r|
            Bv, Cv = st.factor_values()
            Aabs = synth.workloads._kron_sum(np.abs(Bv), np.abs(Cv))
        elif st.kind == "faust":                       # |S_1| ... |S_J|
            Aabs = None
            for M in st.factor_matrices():
                Aabs = np.abs(M) if Aabs is None else Aabs @ np.abs(M)
        else:
            Aabs = np.abs(At)
        scale = np.abs(z) @ Aabs + 1e-300
        err = np.abs(g - ref) / scale
        assert np.max(err) <= rtol, (name, k, float(np.max(err)))
        # z is y itself except for BF16 and FP8 Kronecker stages (rounded to BF16)
        if st.kind == "kron" and st.dtype in ("bf16", "fp8"):
            assert np.all(np.abs(z - p.Y) <= 2.0 ** -8 * np.abs(p.Y))
        else:
            assert np.array_equal(z, p.Y)
        # lambda'_max is an upper bound of the exact quantity and tight
        lm = sl1.lambda_max(d, _t(p.Y, wt)).cpu().numpy()
        for b in range(p.batch):
            exact = osc.stable_lambda_max(At, st.eps, p.Y[b])
            assert lm[b] >= exact * (1 - 1e-12)
            assert lm[b] <= exact * (1 + max(rtol * 10, 2 ** -5 if st.dtype in ("bf16", "fp8") and st.kind == "kron"
                                             else 0))
        d.free()


TILE_CASES = [
    ("C1 kron f64", lambda: synth.config1(), 1e-12),
    ("kron f32 n=(32,64) R=4", lambda: synth.config2(n=(32, 64), R_A=4, Rs=(1, 4)), 2e-5),
    ("C4 kron bf16", lambda: synth.config4(batch=2), 3e-5),
    ("C4 kron fp8", lambda: synth.config4(batch=2, factor_dtype="fp8"), 3e-5),
]
SHAPES = [(a, b) for a in (16, 32, 64, 128) for b in (16, 32, 64, 128)]


@pytest.mark.parametrize("name,maker,rtol", TILE_CASES, ids=[c[0] for c in TILE_CASES])
def test_every_kronecker_tile_shape_matches_oracle_products(sl1, name, maker, rtol):
    # the structured correlation kernel with each usable item shape (kt2 x kt1 atoms)
    # atom by atom against FP64 products of the stored factors
    import torch
    from paper_1812_06635_amd._lib import Stablel1Error
    p = maker()
    wt = torch.float64 if p.work == "f64" else torch.float32
    for k, st in enumerate(p.stages[:-1]):
        d = sl1.upload_stage(st)
        At = st.values()
        Bv, Cv = st.factor_values()
        Aabs = synth.workloads._kron_sum(np.abs(Bv), np.abs(Cv))
        tried = 0
        for kt2, kt1 in SHAPES:
            try:
                d.set_tile(kt2, kt1)
            except Stablel1Error:
                continue                            # not a usable shape for this stage
            _say(f"tile {kt2}x{kt1} {name} stage {k}")
            g, z = sl1.adjoint(d, _t(p.Y, wt))
            g, z = g.cpu().numpy(), z.cpu().numpy().astype(np.float64)
            err = np.abs(g - z @ At) / (np.abs(z) @ Aabs + 1e-300)
            assert np.max(err) <= rtol, (name, k, kt2, kt1, float(np.max(err)))
            tried += 1
        assert tried >= 3
        d.free()


def test_kronecker_tile_autotuner(sl1):
    # the tuner times every usable shape on the batched workload's stages, records the
    # fastest, and the solve with the tuned shapes reaches the Lasso solution
    _say("tile autotuner on the batched dictionary (64 signals)")
    import torch
    p = synth.config4(batch=64)
    ups = [sl1.upload_stage(s) for s in p.stages]
    shapes, ms = sl1.tune_kron(ups, batch=p.batch)
    assert shapes[-1] is None and ms[-1] == 0.0
    for (kt2, kt1), t, st in zip(shapes[:-1], ms[:-1], p.stages[:-1]):
        n1, k1, n2, k2 = st.dims
        assert k2 % kt2 == 0 and k1 % kt1 == 0 and kt2 * kt1 >= 512 and t > 0
    out = sl1.solve(ups, [s.L for s in p.stages], [s.rc_theory for s in p.stages], _t(p.atom_norm),
                    _t(p.Y, torch.float32), _t(p.lam), tol=1e-9)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
    assert res["status"] == 0
    for b in range(0, p.batch, 8):
        _check_solution(p, res, b)


# ---------------------------------------------------------------------------
# the method: per-iteration trace against the FP64 method reference (C1)
# ---------------------------------------------------------------------------
ENGINES = ["grid", "wg"]


# the hybrid engine runs the Kronecker approximations in the whole-solve kernel and hands
# the signal to its tail kernel on reaching A (or, approximations on the grid kernels, after
# 2 iterations: chunk = 2), so the tail's Gram mode (or its column mode) runs most of the
# traced iterations
TRACE_ENGINES = {"grid": dict(engine="grid"), "wg": dict(engine="wg"),
                 "hybrid-gram": dict(engine="hybrid", chunk=2, tail_gram=True),
                 "hybrid-columns": dict(engine="hybrid", chunk=2, tail_gram=False),
                 "hybrid-grid-first": dict(engine="hybrid", chunk=2, tail_gram=True, kron_first=False)}


@pytest.mark.parametrize("engine", list(TRACE_ENGINES))
@pytest.mark.parametrize("real,frac", [(0, 0.5), (1, 0.2), (2, 0.8)])
def test_fp64_trace_matches_method_reference(sl1, real, frac, engine):
    _say(f"trace C1 real={real} frac={frac} engine={engine}")
    p = synth.config1(realization=real, lam_frac=frac)
    out = _run(sl1, p, tol=1e-10, trace_cap=5000, **TRACE_ENGINES[engine])
    if engine.startswith("hybrid"):
        assert sl1.last_solve_phases(1, p.N, p.K)[0] == "hybrid"
        assert (sl1.last_solve_phases(1, p.N, p.K)[1]["gram_cap"] > 0) == TRACE_ENGINES[engine]["tail_gram"]
    ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in p.stages], p.atom_norm, p.Y[0], float(p.lam[0]),
                      [s.rc_theory for s in p.stages], Gamma=0.5, tol=1e-10)
    n = int(out["iters"][0])
    assert ref.converged and out["status"] == 0
    assert n == ref.iters
    tr = out["trace"][0][:n]
    assert [int(r) for r in tr[:, 1]] == [r.stage for r in ref.trace]              # stage sequence
    assert [int(r) for r in tr[:, 2]] == [r.n_active for r in ref.trace]           # |A_t|
    assert [int(r) for r in tr[:, 3]] == [r.n_keep for r in ref.trace]             # |A_t+1|
    assert [int(r) for r in tr[:, 4]] == [r.K_t for r in ref.trace]                # K_t
    Gc = np.array([r.G_conv for r in ref.trace])
    # in Gram mode ||rho||^2 and y^T rho come from y^T y - c^T x and x^T G x: their FP64
    # rounding, ~n u (||y|| + sum |x_k| ||a_k||)^2, bounds the absolute gap difference
    gram = engine in ("hybrid-gram", "hybrid-grid-first")
    np.testing.assert_allclose(tr[:, 6], Gc, rtol=1e-7, atol=1e-10 if gram else 1e-12)
    approx = tr[:, 1] < len(p.stages) - 1
    np.testing.assert_allclose(tr[approx, 9], np.array([r.gamma for r in ref.trace])[approx], rtol=1e-6, atol=1e-9)
    # on A the rounding allowance (~1e-13 per atom) keeps gamma within a hair of 1; in Gram mode the
    # stable scaling also carries the Gram forms' error bound eta ||a_j|| (~1e-12 here)
    tol_g = 1e-9 if gram else 1e-12
    assert np.all(np.abs(tr[~approx, 9] - 1) <= tol_g * tr[~approx, 11] / np.maximum(tr[~approx, 5], 1e-300) + 1e-9)
    np.testing.assert_allclose(out["x"][0], ref.x, rtol=0, atol=1e-9 * max(1, np.abs(ref.x).max()))
    # and the Lasso solution itself
    sol = ol.solve(p.A, p.Y[0], float(p.lam[0]), L=p.stages[-1].L)
    x = out["x"][0]
    assert not np.any((out["screened"][0] == 1) & (sol["x"] != 0))
    assert (ol.primal(p.A, p.Y[0], float(p.lam[0]), x) - sol["P"]) / sol["P"] <= 1e-7
    assert np.linalg.norm(x - sol["x"]) <= 1e-4 * np.linalg.norm(sol["x"])
    assert out["gap"][0] < 1e-10


# ---------------------------------------------------------------------------
# the method in FP32 (with FP64 gap and test) at oracle-friendly sizes
# ---------------------------------------------------------------------------
def _check_solution(p, out, b, obj_tol=1e-5, x_tol=1e-4):
    y, lam = p.Y[b], float(p.lam[b])
    sol = ol.solve(p.A, y, lam, L=p.stages[-1].L)
    x = out["x"][b].astype(np.float64)
    unsafe = int(np.sum((out["screened"][b] == 1) & (sol["x"] != 0)))
    rel_obj = (ol.primal(p.A, y, lam, x) - sol["P"]) / sol["P"]
    rel_x = np.linalg.norm(x - sol["x"]) / max(np.linalg.norm(sol["x"]), 1e-300)
    assert unsafe == 0, f"signal {b}: {unsafe} unsafe rejections"
    assert rel_obj <= obj_tol, f"signal {b}: objective error {rel_obj:.3e}"
    if np.linalg.norm(sol["x"]) > 0:
        assert rel_x <= x_tol, f"signal {b}: x error {rel_x:.3e}"
    else:
        assert np.all(x == 0)
    return rel_obj, rel_x


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("frac", [0.3, 0.5, 0.8])
def test_fp32_kronecker_method(sl1, frac, engine):
    _say(f"C2-small f32 kron frac={frac} engine={engine}")
    p = synth.config2(n=(16, 32), lam_frac=frac)
    out = _run(sl1, p, tol=1e-10, engine=engine)
    assert out["status"] == 0 and out["stage"][0] == len(p.stages) - 1
    _check_solution(p, out, 0)


@pytest.mark.parametrize("engine", ENGINES)
def test_low_precision_dense_method(sl1, engine):
    _say(f"C3-small fp8/bf16/f32 dense engine={engine}")
    p = synth.config3(N=256, K=1024, s=20, batch=4)
    out = _run(sl1, p, tol=1e-10, engine=engine)
    assert out["status"] == 0
    for b in range(p.batch):
        _check_solution(p, out, b)


@pytest.mark.parametrize("engine", ENGINES)
def test_low_precision_dense_ragged(sl1, engine):
    _say(f"C3 ragged N=2500 K=600 engine={engine}")
    p = synth.config3(N=2500, K=600, s=20, batch=2)
    out = _run(sl1, p, tol=1e-10, engine=engine)
    for b in range(p.batch):
        _check_solution(p, out, b)


@pytest.mark.parametrize("engine", ENGINES)
def test_batched_bf16_kronecker_method(sl1, engine):
    _say(f"C4-small batch 24 bf16 kron engine={engine}")
    p = synth.config4(batch=24, n=(16, 32))
    out = _run(sl1, p, tol=1e-10, engine=engine)
    assert out["status"] == 0
    assert len(set(out["iters"].tolist())) > 1           # uneven convergence inside one launch
    for b in range(p.batch):
        _check_solution(p, out, b)


@pytest.mark.parametrize("engine", ["grid", "hybrid"])
@pytest.mark.parametrize("n", [(16, 32), (32, 64)], ids=["small", "C4-size"])
def test_batched_fp8_kronecker_method(sl1, engine, n):
    # Kronecker factors stored in FP8 E4M3 (decoded exactly to BF16 for the matrix
    # cores): every signal safe and at the Lasso solution
    _say(f"batch 24 fp8 kron n={n} engine={engine}")
    p = synth.config4(batch=24, n=n, factor_dtype="fp8")
    out = _run(sl1, p, tol=1e-10, engine=engine)
    assert out["status"] == 0
    assert len(set(out["iters"].tolist())) > 1           # uneven convergence inside one launch
    for b in range(p.batch):
        _check_solution(p, out, b)


def test_fp8_kronecker_refused_by_the_whole_solve_engine(sl1):
    _say("fp8 kron stages, forced whole-solve engine")
    from paper_1812_06635_amd._lib import ELIMIT, Stablel1Error
    p = synth.config4(batch=2, n=(16, 32), factor_dtype="fp8")
    with pytest.raises(Stablel1Error) as e:
        _run(sl1, p, tol=1e-8, engine="wg")
    assert e.value.code == ELIMIT
    out = _run(sl1, p, tol=1e-8)                                  # the automatic choice avoids it
    assert out["status"] == 0


# ---------------------------------------------------------------------------
# FAuST approximations (products of sparse factors)
# ---------------------------------------------------------------------------
def test_faust_fp64_trace_matches_method_reference(sl1):
    _say("trace C6-small faust f64 grid")
    p = synth.config6(N=64, K=515, depth=3, col_nnz=(8, 8, 24), keeps=(8, 12, 16), lam_frac=0.2,
                      dtype="f64", work="f64")
    out = _run(sl1, p, tol=1e-10, trace_cap=20000, engine="grid")
    ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in p.stages], p.atom_norm, p.Y[0], float(p.lam[0]),
                      [s.rc_theory for s in p.stages], Gamma=0.5, tol=1e-10)
    n = int(out["iters"][0])
    assert ref.converged and out["status"] == 0 and n == ref.iters and n <= 20000
    tr = out["trace"][0][:n]
    assert [int(r) for r in tr[:, 1]] == [r.stage for r in ref.trace]
    assert [int(r) for r in tr[:, 2]] == [r.n_active for r in ref.trace]
    assert [int(r) for r in tr[:, 3]] == [r.n_keep for r in ref.trace]
    assert [int(r) for r in tr[:, 4]] == [r.K_t for r in ref.trace]
    assert max(int(r) for r in tr[:, 1]) >= 1              # the FAuST stages were used
    np.testing.assert_allclose(out["x"][0], ref.x, rtol=0, atol=1e-9 * max(1, np.abs(ref.x).max()))
    _check_solution(p, out, 0, obj_tol=1e-7)


@pytest.mark.parametrize("engine", ["grid", "hybrid"])
def test_faust_method_batch(sl1, engine):
    _say(f"C6-small faust f32 batch 6 engine={engine}")
    p = synth.config6(N=64, K=1537, depth=3, col_nnz=(8, 8, 24), keeps=(8, 12, 16), lam_frac=0.15, batch=6)
    out = _run(sl1, p, tol=1e-10, engine=engine)
    assert out["status"] == 0 and np.all(out["stage"] == len(p.stages) - 1)
    for b in range(p.batch):
        _check_solution(p, out, b)


def test_faust_meg_shape_method(sl1):
    _say("C6 faust MEG shape 204 x 8193, batch 2")
    p = synth.config6(batch=2)
    out = _run(sl1, p, tol=1e-8)
    assert out["status"] == 0
    for b in range(p.batch):
        _check_solution(p, out, b)


def test_faust_refused_by_the_whole_solve_engine(sl1):
    from paper_1812_06635_amd._lib import ELIMIT, Stablel1Error
    p = synth.config6(N=64, K=515, depth=2, col_nnz=(8, 16), keeps=(8,), lam_frac=0.3)
    with pytest.raises(Stablel1Error) as e:
        _run(sl1, p, tol=1e-8, engine="wg")
    assert e.value.code == ELIMIT


# ---------------------------------------------------------------------------
# warm starts (initial iterate x0) and lambda paths
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("engine", ENGINES)
def test_warm_start_trace_matches_method_reference(sl1, engine):
    _say(f"warm start trace C1 engine={engine}")
    p = synth.config1(realization=1, lam_frac=0.5)
    x0 = ol.solve(p.A, p.Y[0], 0.7 * float(p.lam_max[0]), L=p.stages[-1].L)["x"]
    out = _run(sl1, p, tol=1e-10, trace_cap=5000, engine=engine, x0=_t(x0[None, :]))
    ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in p.stages], p.atom_norm, p.Y[0], float(p.lam[0]),
                      [s.rc_theory for s in p.stages], Gamma=0.5, tol=1e-10, x0=x0)
    n = int(out["iters"][0])
    assert ref.converged and out["status"] == 0 and n == ref.iters
    tr = out["trace"][0][:n]
    assert [int(r) for r in tr[:, 1]] == [r.stage for r in ref.trace]
    assert [int(r) for r in tr[:, 2]] == [r.n_active for r in ref.trace]
    assert [int(r) for r in tr[:, 3]] == [r.n_keep for r in ref.trace]
    assert [int(r) for r in tr[:, 4]] == [r.K_t for r in ref.trace]
    assert int(tr[0, 12]) == int(np.count_nonzero(x0))        # ||x_0||_0 of the warm start
    np.testing.assert_allclose(tr[0, 10], np.abs(x0).sum(), rtol=1e-13)
    np.testing.assert_allclose(out["x"][0], ref.x, rtol=0, atol=1e-9 * max(1, np.abs(ref.x).max()))
    _check_solution(p, out, 0, obj_tol=1e-7)


@pytest.mark.parametrize("engine,gram", [("grid", True), ("wg", True), ("hybrid", True), ("hybrid", False)],
                         ids=["grid", "wg", "hybrid-gram", "hybrid-columns"])
def test_rejected_nonzero_restarts_momentum_like_the_method_reference(sl1, engine, gram):
    # a warm start with spurious coefficients on atoms near the dual constraint: the test
    # rejects one of them at t = 5 while x_t[j] != 0 (preserved set of 6 atoms), after
    # which the momentum restarts; the hybrid engine hands over after 2 iterations, so
    # its tail (Gram or column mode) meets the rejection
    _say(f"restart after a rejected nonzero, C1 exact stage, engine={engine} gram={gram}")
    p = synth.config1(realization=0, lam_frac=0.5)
    y, lam = p.Y[0], float(p.lam[0])
    sol = ol.solve(p.A, y, lam, L=p.stages[-1].L)
    corr = p.A.T @ sol["theta"]
    cand = np.flatnonzero((sol["x"] == 0) & (np.abs(corr) > 0.8) & (np.abs(corr) < 0.95))
    x0 = sol["x"].copy()
    x0[cand] = 0.1 * np.sign(corr[cand])
    ex = p.stages[-1:]
    out = _run(sl1, p, tol=1e-10, stages=ex, trace_cap=5000, engine=engine, tail_gram=gram, chunk=2,
               x0=_t(x0[None, :]))
    ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in ex], p.atom_norm, y, lam, [1.0], tol=1e-10, x0=x0)
    n = int(out["iters"][0])
    assert ref.converged and out["status"] == 0 and n == ref.iters
    tr = out["trace"][0][:n]
    assert [int(r) for r in tr[:, 2]] == [r.n_active for r in ref.trace]
    assert [int(r) for r in tr[:, 3]] == [r.n_keep for r in ref.trace]
    assert [int(r) for r in tr[:, 4]] == [r.K_t for r in ref.trace]
    np.testing.assert_allclose(tr[:, 6], np.array([r.G_conv for r in ref.trace]), rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(tr[:, 10], np.array([r.x_l1 for r in ref.trace]), rtol=1e-9)
    np.testing.assert_allclose(out["x"][0], ref.x, rtol=0, atol=1e-9 * max(1, np.abs(ref.x).max()))
    _check_solution(p, out, 0, obj_tol=1e-7)
    if engine == "hybrid":
        assert sl1.last_solve_phases(1, p.N, p.K)[0] == "hybrid"


@pytest.mark.parametrize("engine", ["grid", "hybrid"])
def test_warm_started_path_matches_cold_solves(sl1, engine):
    _say(f"lambda path C4-small batch 8 engine={engine}")
    import torch
    p = synth.config4(batch=8, n=(16, 32))
    ups = [sl1.upload_stage(s) for s in p.stages]
    Ls, rc = [s.L for s in p.stages], [s.rc_theory for s in p.stages]
    Y = _t(p.Y, torch.float32)
    lams = [_t(f * p.lam_max) for f in (0.8, 0.5, 0.3)]
    for stages, Lx, rcx in ((ups, Ls, rc), (ups[-1:], Ls[-1:], [1.0])):
        warm = sl1.solve_path(stages, Lx, rcx, _t(p.atom_norm), Y, lams, tol=1e-9, engine=engine)
        cold = sl1.solve_path(stages, Lx, rcx, _t(p.atom_norm), Y, lams, warm=False, tol=1e-9, engine=engine)
        it_w = it_c = 0
        for k, (w, c) in enumerate(zip(warm, cold)):
            w = {kk: (v.cpu().numpy() if hasattr(v, "cpu") else v) for kk, v in w.items()}
            c = {kk: (v.cpu().numpy() if hasattr(v, "cpu") else v) for kk, v in c.items()}
            assert w["status"] == 0 and c["status"] == 0
            q = synth.config4(batch=8, n=(16, 32))
            q.lam = lams[k].cpu().numpy()
            for b in range(p.batch):
                _check_solution(q, w, b)
                rel = np.linalg.norm(w["x"][b] - c["x"][b]) / max(np.linalg.norm(c["x"][b]), 1e-300)
                assert rel <= 1e-5, (k, b, rel)
            it_w += int(w["iters"].sum())
            it_c += int(c["iters"].sum())
        if len(stages) == 1:
            assert it_w < it_c


def test_warm_start_rejects_non_finite_entries(sl1):
    _say("x0 with a NaN")
    from paper_1812_06635_amd._lib import Stablel1Error
    p = synth.config1()
    x0 = np.zeros((1, p.K))
    x0[0, 5] = np.nan
    with pytest.raises(Stablel1Error):
        _run(sl1, p, tol=1e-8, engine="grid", x0=_t(x0))


# ---------------------------------------------------------------------------
# edge cases and error paths
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("engine", ENGINES)
def test_lambda_above_lambda_max_returns_zero(sl1, engine):
    _say(f"lambda >= lambda_max engine={engine}")
    p = synth.config1()
    p.lam = p.lam_max * 1.01
    out = _run(sl1, p, tol=1e-12, engine=engine)
    assert out["status"] == 0
    assert np.all(out["x"] == 0) and out["gap"][0] <= 1e-12
    # x = 0 is optimal at once on A: the solve stops there (Section I-A), without
    # needing any further screening
    assert out["stage"][0] == len(p.stages) - 1


@pytest.mark.parametrize("engine", ENGINES)
def test_max_iter_zero_and_cap(sl1, engine):
    _say(f"max_iter 0 and 5 engine={engine}")
    p = synth.config1()
    out = _run(sl1, p, tol=1e-12, max_iter=0, check=False, engine=engine)
    assert out["status"] == 1 and out["iters"][0] == 0 and np.all(out["x"] == 0)
    out = _run(sl1, p, tol=1e-14, max_iter=5, check=False, engine=engine)
    assert out["status"] == 1 and out["iters"][0] == 5


@pytest.mark.parametrize("engine", ENGINES)
def test_invalid_lambda_is_reported(sl1, engine):
    _say(f"invalid lambda engine={engine}")
    from paper_1812_06635_amd._lib import Stablel1Error
    p = synth.config1()
    p.lam = np.array([-1.0])
    with pytest.raises(Stablel1Error):
        _run(sl1, p, tol=1e-8, engine=engine)
    p.lam = np.array([np.nan])
    with pytest.raises(Stablel1Error):
        _run(sl1, p, tol=1e-8, engine=engine)


def test_graph_replay_equals_direct_launches(sl1):
    _say("graph vs direct")
    p = synth.config4(batch=6, n=(16, 32))
    a = _run(sl1, p, tol=1e-7, use_graph=True)
    b = _run(sl1, p, tol=1e-7, use_graph=False, chunk=5)
    np.testing.assert_array_equal(a["x"], b["x"])
    np.testing.assert_array_equal(a["iters"], b["iters"])
    np.testing.assert_array_equal(a["screened"], b["screened"])


def test_engines_agree_and_relaunch_is_exact(sl1):
    # both engines take the same decisions; the whole-solve engine split over
    # many bounded launches (256 iterations each) gives bit-identical results
    _say("engines agree; whole-solve relaunch")
    import paper_1812_06635_amd as m
    p = synth.config4(batch=12, n=(16, 32))
    g = _run(sl1, p, tol=1e-9, engine="grid")
    w = _run(sl1, p, tol=1e-9, engine="wg")
    w1 = _run(sl1, p, tol=1e-9, engine="wg", chunk=1)
    assert m.last_solve_phases(p.batch, p.N, p.K)[0] == "wg"
    np.testing.assert_array_equal(w["x"], w1["x"])
    np.testing.assert_array_equal(w["iters"], w1["iters"])
    np.testing.assert_array_equal(w["screened"], w1["screened"])
    assert int(w["iters"].max()) > 256                 # the relaunch path was taken
    np.testing.assert_array_equal(g["stage"], w["stage"])
    assert np.all(np.abs(g["iters"] - w["iters"]) <= 2)
    for b in range(p.batch):
        rel = np.linalg.norm(g["x"][b] - w["x"][b]) / max(np.linalg.norm(g["x"][b]), 1e-300)
        assert rel <= 1e-4, f"signal {b}: engines differ by {rel:.2e}"


def test_auto_engine_choice(sl1):
    _say("auto engine choice")
    import paper_1812_06635_amd as m
    p = synth.config4(batch=40, n=(16, 32))                 # N*K = 2^18: whole-solve engine
    _run(sl1, p, tol=1e-6)
    assert m.last_solve_phases(p.batch, p.N, p.K)[0] == "wg"
    q = synth.config2(n=(32, 64), R_A=4, Rs=(1, 4))        # one signal, N*K = 2^22: grid, then the tail
    _run(sl1, q, tol=1e-6)
    assert m.last_solve_phases(1, q.N, q.K)[0] in ("grid", "hybrid")
    _run(sl1, q, tol=1e-6, engine="grid")
    assert m.last_solve_phases(1, q.N, q.K)[0] == "grid"


@pytest.mark.parametrize("gram", [True, False], ids=["gram", "columns"])
def test_hybrid_hand_over_matches_grid(sl1, gram):
    # the full batched dictionary (N=1024, K=4096) on 12 signals: the grid kernels
    # hand the tail to the tail kernel (Gram or column mode); decisions and
    # solutions agree
    _say(f"hybrid hand-over, batched dictionary, 12 signals, gram={gram}")
    import paper_1812_06635_amd as m
    p = synth.config4(batch=12)
    g = _run(sl1, p, tol=1e-9, engine="grid")
    h = _run(sl1, p, tol=1e-9, engine="hybrid", trace_cap=4000, tail_gram=gram)
    assert m.last_solve_phases(p.batch, p.N, p.K)[0] == "hybrid"
    assert g["status"] == 0 and h["status"] == 0
    np.testing.assert_array_equal(g["stage"], h["stage"])
    assert np.all(np.abs(g["iters"] - h["iters"]) <= 2)
    for b in range(p.batch):
        rel = np.linalg.norm(g["x"][b] - h["x"][b]) / max(np.linalg.norm(g["x"][b]), 1e-300)
        assert rel <= 1e-4, f"signal {b}: engines differ by {rel:.2e}"
        n = int(h["iters"][b])
        tr = h["trace"][b][:n]
        assert np.array_equal(tr[:, 0], np.arange(n))                  # one trace row per iteration
        assert np.all(tr[1:, 2] == tr[:-1, 3])                          # |A_t+1| carried over
    for b in range(p.batch):
        _check_solution(p, h, b)


@pytest.mark.parametrize("step", [True, False], ids=["step", "split"])
def test_hybrid_kron_first_matches_grid_first(sl1, step):
    # the full batched dictionary on 12 signals: the Kronecker approximations run in the
    # whole-solve kernel; signals that reach A with large preserved sets go on in the grid
    # kernels (their lists converted), which later hand the rest to the tail kernel.  The
    # decisions and solutions agree with the hybrid solve that runs the approximations on
    # the grid kernels.
    _say(f"hybrid, approximations in the whole-solve kernel vs on the grid, batched dictionary, 12 signals, "
         f"step={step}")
    import paper_1812_06635_amd as m
    p = synth.config4(batch=12)
    g = _run(sl1, p, tol=1e-9, engine="hybrid", kron_first=False)
    h = _run(sl1, p, tol=1e-9, engine="hybrid", trace_cap=4000, profile=True, step=step)
    ph = m.last_solve_phases(p.batch, p.N, p.K)
    prof = m.last_solve_profile(p.batch, p.N, p.K)
    assert ph[0] == "hybrid"
    assert ph[1]["wg_launches"] >= 2 and ph[1]["kron_wg_ms"] > 0   # the approximations' phase, then the tail
    assert prof["adj_kron"][1] == 0                                 # grid kernels on A only
    assert (prof["step"][1] > 0) == step and (prof["fwd"][1] > 0) == (not step)
    assert g["status"] == 0 and h["status"] == 0
    np.testing.assert_array_equal(g["stage"], h["stage"])
    assert np.all(np.abs(g["iters"] - h["iters"]) <= 2), (g["iters"], h["iters"])
    for b in range(p.batch):
        rel = np.linalg.norm(g["x"][b] - h["x"][b]) / max(np.linalg.norm(g["x"][b]), 1e-300)
        assert rel <= 1e-4, f"signal {b}: paths differ by {rel:.2e}"
        n = int(h["iters"][b])
        tr = h["trace"][b][:n]
        assert np.array_equal(tr[:, 0], np.arange(n))                  # one trace row per iteration
        assert np.all(tr[1:, 2] == tr[:-1, 3])                          # |A_t+1| carried over
        assert np.all(np.diff(tr[:, 1]) >= 0)                           # stages only advance
    for b in range(p.batch):
        _check_solution(p, h, b)


def test_late_kronecker_signals_run_beside_the_grid(sl1):
    # 256 signals of the batched dictionary: the grid kernels start once at most 256 / 128
    # live signals are still on the approximations; those go on in a whole-solve launch on
    # a second stream and join at the next chunk boundary.  Decisions and solutions agree
    # with the solve whose grid kernels wait for every signal.
    _say("hybrid, late Kronecker-phase signals beside the grid vs waiting for all, batched dictionary, "
         "256 signals")
    import paper_1812_06635_amd as m
    p = synth.config4(batch=256)
    a = _run(sl1, p, tol=1e-9, engine="hybrid", park_all=True, profile=True)
    ph_a = m.last_solve_phases(p.batch, p.N, p.K)[1]
    h = _run(sl1, p, tol=1e-9, engine="hybrid", profile=True)
    ph_h = m.last_solve_phases(p.batch, p.N, p.K)[1]
    prof_h = m.last_solve_profile(p.batch, p.N, p.K)
    _say(f"whole-solve launches (approximations' phase / all): {ph_a['kron_wg_launches']} / {ph_a['wg_launches']} "
         f"waiting for all, {ph_h['kron_wg_launches']} / {ph_h['wg_launches']} with one beside")
    # the launch beside the grid is one more launch of the approximations' phase (the
    # tail's launches, 476 iterations each here, may differ, as the late signals join the
    # grid a chunk later).  Whether a signal is still short of A when at most 2 remain
    # depends on the workgroups' timing: when none is, no launch goes beside and the
    # solve is the waiting one; either way the results below must agree.
    beside = ph_h["kron_wg_launches"] - ph_a["kron_wg_launches"]
    assert beside in (0, 1), (ph_a, ph_h)
    assert prof_h["adj_kron"][1] == 0 and prof_h["step"][1] > 0      # step launches on A only
    assert a["status"] == 0 and h["status"] == 0
    np.testing.assert_array_equal(a["stage"], h["stage"])
    assert np.all(np.abs(a["iters"] - h["iters"]) <= 2), np.flatnonzero(np.abs(a["iters"] - h["iters"]) > 2)
    for b in range(p.batch):
        rel = np.linalg.norm(a["x"][b] - h["x"][b]) / max(np.linalg.norm(a["x"][b]), 1e-300)
        assert rel <= 1e-4, f"signal {b}: paths differ by {rel:.2e}"
    for b in np.argsort(-h["iters"])[:6]:
        _check_solution(p, h, int(b))


def _exact_only(p):
    import dataclasses
    return dataclasses.replace(p, stages=[p.stages[-1]])


STEP_CASES = [
    ("C1 exact stage alone, f64", lambda: _exact_only(synth.config1(realization=1, lam_frac=0.3))),
    ("C3-small dense fp8 -> bf16 -> f32", lambda: synth.config3(N=256, K=1024, s=20, batch=3)),
    ("C3 ragged N=2500 (three forward items)", lambda: synth.config3(N=2500, K=600, s=20, batch=2)),
]


@pytest.mark.parametrize("step", [True, False], ids=["step", "split"])
@pytest.mark.parametrize("name,maker", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_dense_trace_matches_method_reference(sl1, name, maker, step):
    # dense stages only: the grid engine's per-signal step launch (update of t and
    # forward of t + 1 in one block) and the separate chip-wide launches give the
    # method reference's trace, iteration by iteration
    _say(f"dense trace vs method reference: {name}, step={step}")
    import paper_1812_06635_amd as m
    p = maker()
    out = _run(sl1, p, tol=1e-10, engine="grid", trace_cap=6000, step=step, profile=True)
    prof = m.last_solve_profile(p.batch, p.N, p.K)
    assert (prof["step"][1] > 0) == step and (prof["fwd"][1] > 0) == (not step)
    assert out["status"] == 0
    for b in range(p.batch):
        ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in p.stages], p.atom_norm, p.Y[b], float(p.lam[b]),
                          [s.rc_theory for s in p.stages], Gamma=0.5, tol=1e-10)
        n = int(out["iters"][b])
        assert ref.converged and n == ref.iters, (b, n, ref.iters)
        tr = out["trace"][b][:n]
        assert [int(r) for r in tr[:, 1]] == [r.stage for r in ref.trace]
        assert [int(r) for r in tr[:, 2]] == [r.n_active for r in ref.trace]
        assert [int(r) for r in tr[:, 3]] == [r.n_keep for r in ref.trace]
        assert [int(r) for r in tr[:, 4]] == [r.K_t for r in ref.trace]
        np.testing.assert_allclose(tr[:, 6], [r.G_conv for r in ref.trace], rtol=1e-7, atol=1e-12)
        np.testing.assert_allclose(out["x"][b], ref.x, rtol=0, atol=1e-9 * max(1, np.abs(ref.x).max()))


def _bf16_exact(p):
    # the column-scaled BF16 copy taken as the exact dictionary of its own problem
    import dataclasses
    st = dataclasses.replace(p.stages[1], eps=np.zeros(p.K), label="bf16 (exact)")
    A = st.values()
    return dataclasses.replace(p, A=A, stages=[st], atom_norm=np.linalg.norm(A, axis=0))


TAIL_CASES = [
    ("C3-small dense fp8/bf16/f32", lambda: synth.config3(N=256, K=1024, s=20, batch=4)),
    ("C3 ragged N=2500 (N % 16 = 4)", lambda: synth.config3(N=2500, K=600, s=20, batch=2)),
    ("column-scaled BF16 as the exact stage", lambda: _bf16_exact(synth.config3(N=256, K=1024, s=20, batch=3))),
]


@pytest.mark.parametrize("name,maker", TAIL_CASES, ids=[c[0] for c in TAIL_CASES])
def test_tail_modes_match_grid(sl1, name, maker):
    # dense last stages: the hybrid solve hands over at once and its tail kernel
    # switches to the Gram form when |A_t| fits; the column mode and the grid
    # engine solve the same problem with the same decisions
    _say(f"tail modes vs grid: {name}")
    import paper_1812_06635_amd as m
    p = maker()
    stages = None
    g = _run(sl1, p, tol=1e-10, stages=stages, engine="grid")
    runs = {}
    for gram in (True, False):
        runs[gram] = _run(sl1, p, tol=1e-10, stages=stages, engine="hybrid", trace_cap=20000, tail_gram=gram)
        assert m.last_solve_phases(p.batch, p.N, p.K)[0] == "hybrid"
    for gram, h in runs.items():
        assert g["status"] == 0 and h["status"] == 0
        np.testing.assert_array_equal(g["stage"], h["stage"])
        assert np.all(np.abs(g["iters"] - h["iters"]) <= 3), (gram, g["iters"], h["iters"])
        for b in range(p.batch):
            rel = np.linalg.norm(g["x"][b] - h["x"][b]) / max(np.linalg.norm(g["x"][b]), 1e-300)
            assert rel <= 1e-6, f"gram={gram} signal {b}: differs from grid by {rel:.2e}"
            n = int(h["iters"][b])
            tr = h["trace"][b][:n]
            assert np.array_equal(tr[:, 0], np.arange(n))
            assert np.all(tr[1:, 2] == tr[:-1, 3])
            assert np.all(tr[:, 7] >= 0.0) and np.all(tr[:, 5] >= -1e-9 * tr[:, 11])
            # the screened sets agree up to atoms decided within rounding of the threshold
            assert np.sum(g["screened"][b] != h["screened"][b]) <= 2
    for b in range(p.batch):
        _check_solution(p, runs[True], b)


def test_identical_signals_finishing_together(sl1):
    # 256 copies of one signal on the batched dictionary: the forward launch then
    # gives each block two of a signal's four row items, and every copy stops in
    # the same launch (control state of a finishing signal vs. its other blocks)
    _say("256 identical signals, grid engine")
    import torch
    p = synth.config4(batch=512)
    sig = 203
    ups = [sl1.upload_stage(s) for s in p.stages]
    Ls, rc = [s.L for s in p.stages], [0.037, 0.037, 0.040, 1.0]
    an = _t(p.atom_norm)
    one = sl1.solve(ups, Ls, rc, an, _t(p.Y[sig:sig + 1], torch.float32), _t(p.lam[sig:sig + 1]), tol=1e-7,
                    engine="grid")
    many = sl1.solve(ups, Ls, rc, an, _t(np.tile(p.Y[sig], (256, 1)), torch.float32),
                     _t(np.tile(p.lam[sig], 256)), tol=1e-7, engine="grid")
    torch.cuda.synchronize()
    x1 = one["x"].cpu().numpy()[0]
    X = many["x"].cpu().numpy()
    assert one["status"] == 0 and many["status"] == 0
    assert np.all(many["iters"].cpu().numpy() == int(one["iters"][0]))
    for b in range(256):
        rel = np.linalg.norm(X[b] - x1) / np.linalg.norm(x1)
        assert rel <= 1e-9, f"copy {b} differs from the single solve by {rel:.2e}"
    sol = ol.solve(p.A, p.Y[sig], float(p.lam[sig]), L=p.stages[-1].L)
    assert np.linalg.norm(x1 - sol["x"]) <= 1e-4 * np.linalg.norm(sol["x"])


@pytest.mark.parametrize("engine", ENGINES)
def test_exact_only_sequence_is_gap_safe(sl1, engine):
    # one stage (the exact A): the stable test is GAP Safe, gamma = 1
    _say(f"exact-only sequence engine={engine}")
    p = synth.config1()
    st = [p.stages[-1]]
    out = _run(sl1, p, tol=1e-10, stages=st, trace_cap=3000, engine=engine)
    ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in st], p.atom_norm, p.Y[0], float(p.lam[0]), [1.0],
                      tol=1e-10)
    n = int(out["iters"][0])
    assert n == ref.iters
    assert [int(v) for v in out["trace"][0][:n, 2]] == [r.n_active for r in ref.trace]
    tr = out["trace"][0][:n]
    assert np.all(np.abs(tr[:, 9] - 1) <= 1e-12 * tr[:, 11] / np.maximum(tr[:, 5], 1e-300) + 1e-9)


# ---------------------------------------------------------------------------
# implicit adjoint
# ---------------------------------------------------------------------------
def test_implicit_adjoint_matches_finite_differences(sl1):
    import torch
    _say("grad vs FD")
    p = synth.config5(batch=3, n=(16, 32), R_A=8, Rs=(4, 8))
    out = _run(sl1, p, tol=1e-10)
    x = out["x"].astype(np.float64)
    A = p.A
    exact = sl1.upload_stage(p.stages[-1])
    dx = 2.0 * (x - p.X0)
    dy, dlam = sl1.grad(exact, _t(out["x"]), _t(p.Y, torch.float32), _t(p.lam), _t(dx))
    dy, dlam = dy.cpu().numpy().astype(np.float64), dlam.cpu().numpy()
    rng = np.random.default_rng(5)
    for b in range(p.batch):
        y, lam = p.Y[b], float(p.lam[b])

        def loss(yy, ll):
            s = ol.solve(A, yy, ll, L=p.stages[-1].L, tol=1e-15)
            return float(np.sum((s["x"] - p.X0[b]) ** 2)), s

        _, s0 = loss(y, lam)
        assert s0["margin"] > 1e-4
        # closed form on the oracle support (FP64)
        S = s0["support"]
        G = A[:, S].T @ A[:, S]
        v = 2 * (s0["x"] - p.X0[b])[S]
        w = np.linalg.solve(G, v)
        g_ref = A[:, S] @ w
        l_ref = -np.sign(s0["x"][S]) @ w
        assert np.linalg.norm(dy[b] - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
        assert abs(dlam[b] - l_ref) <= 1e-4 * abs(l_ref) + 1e-8
        # central differences, h = 1e-6
        u = rng.standard_normal(len(y))
        u /= np.linalg.norm(u)
        h = 1e-6
        fd = (loss(y + h * u, lam)[0] - loss(y - h * u, lam)[0]) / (2 * h)
        assert abs(fd - dy[b] @ u) <= 1e-4 * max(1.0, abs(fd))
        fdl = (loss(y, lam + h)[0] - loss(y, lam - h)[0]) / (2 * h)
        assert abs(fdl - dlam[b]) <= 1e-4 * max(1.0, abs(fdl))


def test_autograd_function_backward(sl1):
    import torch
    _say("autograd")
    p = synth.config5(batch=2, n=(16, 32), R_A=8, Rs=(8,))
    ups = [sl1.upload_stage(s) for s in p.stages]
    y = _t(p.Y, torch.float32).requires_grad_(True)
    lam = _t(p.lam).requires_grad_(True)
    x = sl1.lasso(y, lam, ups, [s.L for s in p.stages], [s.rc_theory for s in p.stages], _t(p.atom_norm),
                  tol=1e-8)
    loss = ((x.double() - _t(p.X0)) ** 2).sum()
    loss.backward()
    assert y.grad is not None and lam.grad is not None
    assert torch.isfinite(y.grad).all() and torch.isfinite(lam.grad).all()


# ---------------------------------------------------------------------------
# ISTA and the stable Dynamic Safe test (Table I, fourth row; Table III)
# ---------------------------------------------------------------------------
RULE_VARIANTS = [("fista", "dst"), ("ista", "gap"), ("ista", "dst")]


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("update,rule", RULE_VARIANTS, ids=[f"{u}-{r}" for u, r in RULE_VARIANTS])
@pytest.mark.parametrize("real,frac", [(0, 0.5), (1, 0.2)])
def test_variant_trace_matches_method_reference(sl1, real, frac, update, rule, engine):
    _say(f"trace C1 {update}/{rule} real={real} frac={frac} engine={engine}")
    p = synth.config1(realization=real, lam_frac=frac)
    out = _run(sl1, p, tol=1e-10, trace_cap=20000, engine=engine, update=update, rule=rule)
    ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in p.stages], p.atom_norm, p.Y[0], float(p.lam[0]),
                      [s.rc_theory for s in p.stages], Gamma=0.5, tol=1e-10, update=update, rule=rule)
    n = int(out["iters"][0])
    assert ref.converged and out["status"] == 0
    assert n == ref.iters
    tr = out["trace"][0][:n]
    assert [int(r) for r in tr[:, 1]] == [r.stage for r in ref.trace]
    assert [int(r) for r in tr[:, 2]] == [r.n_active for r in ref.trace]
    assert [int(r) for r in tr[:, 3]] == [r.n_keep for r in ref.trace]
    assert [int(r) for r in tr[:, 4]] == [r.K_t for r in ref.trace]
    np.testing.assert_allclose(tr[:, 6], np.array([r.G_conv for r in ref.trace]), rtol=1e-7, atol=1e-12)
    # the sphere radius of the rule, squared (the GAP radius is sqrt(2 (G' + delta)) / lambda,
    # so compare R^2 with the absolute gap accuracy; the GPU's Dynamic Safe radius also
    # carries its rounding widening)
    lam = float(p.lam[0])
    np.testing.assert_allclose(tr[:, 8] ** 2, np.array([r.R_stable for r in ref.trace]) ** 2, rtol=1e-6,
                               atol=2e-10 / lam ** 2)
    sol = ol.solve(p.A, p.Y[0], float(p.lam[0]), L=p.stages[-1].L)
    x = out["x"][0]
    assert not np.any((out["screened"][0] == 1) & (sol["x"] != 0))
    assert (ol.primal(p.A, p.Y[0], float(p.lam[0]), x) - sol["P"]) / sol["P"] <= 1e-7
    assert np.linalg.norm(x - sol["x"]) <= 1e-4 * np.linalg.norm(sol["x"])


@pytest.mark.parametrize("update,rule", RULE_VARIANTS, ids=[f"{u}-{r}" for u, r in RULE_VARIANTS])
def test_variants_hybrid_tail_match_grid(sl1, update, rule):
    # the batched dictionary (12 signals) and a dense low-precision sequence: the
    # hybrid solve's tail (Gram and column modes) agrees with the grid engine
    _say(f"variants {update}/{rule}: hybrid tail vs grid")
    for p in (synth.config4(batch=12), synth.config3(N=256, K=1024, s=20, batch=3)):
        g = _run(sl1, p, tol=1e-9, engine="grid", update=update, rule=rule)
        assert g["status"] == 0
        for gram in (True, False):
            h = _run(sl1, p, tol=1e-9, engine="hybrid", tail_gram=gram, update=update, rule=rule)
            assert h["status"] == 0
            np.testing.assert_array_equal(g["stage"], h["stage"])
            assert np.all(np.abs(g["iters"] - h["iters"]) <= 3), (gram, g["iters"], h["iters"])
            for b in range(p.batch):
                rel = np.linalg.norm(g["x"][b] - h["x"][b]) / max(np.linalg.norm(g["x"][b]), 1e-300)
                assert rel <= 1e-6, f"{p.name} gram={gram} signal {b}: {rel:.2e}"
        for b in (0, p.batch - 1):
            _check_solution(p, g, b)


def test_dst_requires_a_dense_exact_stage(sl1):
    # a^T y is formed with the dense correlation kernel; a Kronecker exact stage is refused
    import torch
    p = synth.config2(n=(16, 32))
    kr = [s for s in p.stages if s.kind == "kron"][-1]
    import dataclasses
    ex = dataclasses.replace(kr, eps=np.zeros(p.K))
    with pytest.raises(Exception):
        _run(sl1, p, tol=1e-6, stages=[ex], rule="dst")
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# batched correlations (one FP64 matrix-core product for large preserved sets)
# ---------------------------------------------------------------------------
def _product_iterations(on, p, gmin, gemm_signals, chunk=16):
    """Per iteration t, the number of signals whose correlations went through the
    batched product: signals qualifying at t (exact dense stage, |A_t| >= gmin),
    counted when the product ran in t's chunk (the first chunk: batch >=
    gemm_signals; a later one: at least gemm_signals signals qualified at the
    previous chunk's last iteration)."""
    I = len(p.stages) - 1
    n = int(np.max(on["iters"]))
    q = np.zeros((p.batch, n + 1), dtype=bool)
    for b in range(p.batch):
        k = int(on["iters"][b])
        tr = on["trace"][b][:k]
        q[b, :k] = (tr[:, 1] == I) & (tr[:, 2] >= gmin)
    cnt = q.sum(axis=0)
    used = np.zeros(n + 1, dtype=np.int64)
    for t in range(n + 1):
        c = t // chunk
        gate = p.batch >= gemm_signals if c == 0 else cnt[c * chunk - 1] >= gemm_signals
        used[t] = cnt[t] if gate else 0
    return used


@pytest.mark.parametrize("rule", ["gap", "dst"])
def test_batched_correlations_match_streaming(sl1, rule):
    # grid engine with the batched product forced on for any qualifying signal
    # (gemm_signals=1) and without it: same decisions, same x.  With a handful of
    # signals the product tiles are few, so their rows are split over blocks.
    import paper_1812_06635_amd as m
    used_by = {}
    for p in (synth.config4(batch=12), synth.config3(N=256, K=1024, s=20, batch=3),
              synth.config3(N=2500, K=600, s=20, batch=2)):
        _say(f"batched correlations vs streaming: {p.name} N={p.N} K={p.K} rule={rule}")
        on = _run(sl1, p, tol=1e-9, engine="grid", rule=rule, trace_cap=20000, gemm_signals=1)
        gmin = m.last_solve_phases(p.batch, p.N, p.K)[1]["gemm_min"]
        off = _run(sl1, p, tol=1e-9, engine="grid", rule=rule, batched_gemm=False)
        assert on["status"] == 0 and off["status"] == 0 and gmin > 0
        used_by[(p.name, p.N)] = int(_product_iterations(on, p, gmin, 1).sum())
        np.testing.assert_array_equal(on["stage"], off["stage"])
        assert np.all(np.abs(on["iters"] - off["iters"]) <= 2), (on["iters"], off["iters"])
        for b in range(p.batch):
            rel = np.linalg.norm(on["x"][b] - off["x"][b]) / max(np.linalg.norm(off["x"][b]), 1e-300)
            assert rel <= 1e-7, f"{p.name} signal {b}: {rel:.2e}"
        for b in (0, p.batch - 1):
            _check_solution(p, on, b)
    # the batched dictionary and the small dense sequence do go through the product
    assert used_by[("C4", 1024)] > 0 and used_by[("C3", 256)] > 0, used_by


def test_batched_product_many_and_few_signals_match_streaming(sl1):
    # 320 signals: 300 copies of one signal, which qualify together (five signal
    # tiles, one of them partial), and 20 distinct ones, which qualify a few at a
    # time (one partial signal tile)
    import dataclasses
    import paper_1812_06635_amd as m
    q = synth.config4(batch=21)
    # the copied signal: the one qualifying at the most iterations
    pre = _run(sl1, q, tol=1e-9, engine="grid", trace_cap=20000, gemm_signals=1)
    gmin = m.last_solve_phases(q.batch, q.N, q.K)[1]["gemm_min"]
    nq = [int(np.sum((pre["trace"][b][:int(pre["iters"][b]), 1] == len(q.stages) - 1) &
                     (pre["trace"][b][:int(pre["iters"][b]), 2] >= gmin))) for b in range(q.batch)]
    c = int(np.argmax(nq))
    assert nq[c] > 0, nq
    sel = np.array([c] * 300 + [b for b in range(q.batch) if b != c])
    p = dataclasses.replace(q, Y=q.Y[sel].copy(), lam=q.lam[sel].copy(), X0=q.X0[sel].copy(),
                            lam_max=q.lam_max[sel].copy())
    _say(f"batched product, many and few signals: {p.name} batch={p.batch}")
    on = _run(sl1, p, tol=1e-9, engine="grid", trace_cap=20000, gemm_signals=1)
    gmin = m.last_solve_phases(p.batch, p.N, p.K)[1]["gemm_min"]
    off = _run(sl1, p, tol=1e-9, engine="grid", batched_gemm=False)
    assert on["status"] == 0 and off["status"] == 0 and gmin > 0
    used = _product_iterations(on, p, gmin, 1)
    assert used.max() > 256, used.max()                   # many signals at once
    assert np.any((used > 0) & (used <= 64)), used        # one partial signal tile
    np.testing.assert_array_equal(on["stage"], off["stage"])
    assert np.all(np.abs(on["iters"] - off["iters"]) <= 2)
    for b in range(p.batch):
        rel = np.linalg.norm(on["x"][b] - off["x"][b]) / max(np.linalg.norm(off["x"][b]), 1e-300)
        assert rel <= 1e-7, f"signal {b}: {rel:.2e}"
    for b in (0, p.batch - 1):
        _check_solution(p, on, b)
    # the copies of one signal end identical
    assert np.all(on["iters"][:300] == on["iters"][0])
    np.testing.assert_array_equal(on["x"][:300], np.broadcast_to(on["x"][0], (300, p.K)))


# ---------------------------------------------------------------------------
# screening at regular intervals (Algorithm 1's variation)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("engine", ENGINES)
def test_interval_screening_trace_matches_method_reference(sl1, engine):
    _say(f"trace C1 screen_every=3 engine={engine}")
    p = synth.config1(realization=1, lam_frac=0.3)
    out = _run(sl1, p, tol=1e-10, trace_cap=5000, engine=engine, screen_every=3)
    ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in p.stages], p.atom_norm, p.Y[0], float(p.lam[0]),
                      [s.rc_theory for s in p.stages], Gamma=0.5, tol=1e-10, screen_every=3)
    n = int(out["iters"][0])
    assert ref.converged and out["status"] == 0 and n == ref.iters
    tr = out["trace"][0][:n]
    assert [int(r) for r in tr[:, 1]] == [r.stage for r in ref.trace]
    assert [int(r) for r in tr[:, 2]] == [r.n_active for r in ref.trace]
    assert [int(r) for r in tr[:, 3]] == [r.n_keep for r in ref.trace]
    assert [int(r) for r in tr[:, 4]] == [r.K_t for r in ref.trace]
    assert all(int(r[3]) == int(r[2]) for r in tr if int(r[0]) % 3 != 0)
    _check_solution(p, out, 0, obj_tol=1e-7)


def test_interval_screening_hybrid_tail_matches_grid(sl1):
    _say("screen_every=4: hybrid tail vs grid")
    p = synth.config4(batch=12)
    g = _run(sl1, p, tol=1e-9, engine="grid", screen_every=4)
    for gram in (True, False):
        h = _run(sl1, p, tol=1e-9, engine="hybrid", tail_gram=gram, screen_every=4)
        assert g["status"] == 0 and h["status"] == 0
        assert np.all(np.abs(g["iters"] - h["iters"]) <= 3)
        for b in range(p.batch):
            rel = np.linalg.norm(g["x"][b] - h["x"][b]) / max(np.linalg.norm(g["x"][b]), 1e-300)
            assert rel <= 1e-6
    for b in (0, 11):
        _check_solution(p, g, b)


# ---------------------------------------------------------------------------
# error bounds in other l_q norms (Lemma 1, Lemma 2, Theorem 1 with an l_q zone)
# ---------------------------------------------------------------------------
# (name, q, lambda fraction of C1 realization 2): cases where the approximations reject atoms
LQ_CASES = [("q=1", 1.0, 0.8), ("q=1.5", 1.5, 0.7), ("q=3", 3.0, 0.7), ("q=inf", np.inf, 0.8),
            ("inf then 1", "mixed", 0.8)]


def _lq_problem(q, frac):
    p = synth.config1(realization=2, lam_frac=frac)
    if q == "mixed":
        return synth.with_lq_bounds(synth.with_lq_bounds(p, np.inf, stages=[0]), 1.0, stages=[1, 2])
    return synth.with_lq_bounds(p, q)


@pytest.mark.parametrize("engine", ["grid", "hybrid"])
@pytest.mark.parametrize("name,q,frac", LQ_CASES, ids=[c[0] for c in LQ_CASES])
def test_lq_bounds_trace_matches_method_reference(sl1, name, q, frac, engine):
    _say(f"trace C1 l_q bounds {name} engine={engine}")
    p = _lq_problem(q, frac)
    out = _run(sl1, p, tol=1e-10, trace_cap=5000, engine=engine)
    ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in p.stages], p.atom_norm, p.Y[0], float(p.lam[0]),
                      [s.rc_theory for s in p.stages], Gamma=0.5, tol=1e-10, q=[s.q for s in p.stages])
    n = int(out["iters"][0])
    assert ref.converged and out["status"] == 0 and n == ref.iters
    tr = out["trace"][0][:n]
    assert [int(r) for r in tr[:, 1]] == [r.stage for r in ref.trace]
    assert [int(r) for r in tr[:, 2]] == [r.n_active for r in ref.trace]
    assert [int(r) for r in tr[:, 3]] == [r.n_keep for r in ref.trace]
    assert [int(r) for r in tr[:, 4]] == [r.K_t for r in ref.trace]
    np.testing.assert_allclose(tr[:, 6], [r.G_conv for r in ref.trace], rtol=1e-7, atol=1e-12)
    approx = tr[:, 1] < len(p.stages) - 1
    assert approx.any()
    np.testing.assert_allclose(tr[approx, 5], np.array([r.G_stable for r in ref.trace])[approx], rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(tr[approx, 7], np.array([r.delta for r in ref.trace])[approx], rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(tr[approx, 9], np.array([r.gamma for r in ref.trace])[approx], rtol=1e-6, atol=1e-9)
    # the approximations reject atoms, none of the solution's support
    assert sum(int(r[2]) - int(r[3]) for r in tr if r[1] < len(p.stages) - 1) > 0
    _check_solution(p, out, 0, obj_tol=1e-7)


@pytest.mark.parametrize("q", [1.0, 1.5, 3.0, np.inf])
def test_lq_lambda_max_matches_oracle(sl1, q):
    import torch
    for name, p in (("C1 kron f64", synth.config1()), ("C3-small dense", synth.config3(N=256, K=1024, batch=3))):
        p = synth.with_lq_bounds(p, q)
        wt = torch.float64 if p.work == "f64" else torch.float32
        for k, st in enumerate(p.stages[:-1]):
            _say(f"lambda'_max {name} stage {k} q={q}")
            d = sl1.upload_stage(st)
            lm = sl1.lambda_max(d, _t(p.Y, wt)).cpu().numpy()
            At = st.values()
            for b in range(p.batch):
                exact = osc.stable_lambda_max(At, st.eps, p.Y[b], q=q)
                assert exact * (1 - 1e-12) <= lm[b] <= exact * (1 + 1e-9), (name, k, b)
            d.free()


def test_lq_engine_routing(sl1):
    from paper_1812_06635_amd._lib import ELIMIT, Stablel1Error
    _say("l_q bounds: whole-solve engine refused, hybrid with an l_q last stage = grid")
    p = synth.with_lq_bounds(synth.config1(realization=1, lam_frac=0.5), np.inf)
    with pytest.raises(Stablel1Error) as e:
        _run(sl1, p, tol=1e-10, engine="wg")
    assert e.value.code == ELIMIT
    # every stage, the exact one included, with l_inf bounds (eps = 0 for A)
    pe = synth.with_lq_bounds(p, np.inf, stages=range(len(p.stages)))
    assert pe.stages[-1].q == np.inf and not np.any(pe.stages[-1].eps)
    g = _run(sl1, pe, tol=1e-10, engine="grid")
    h = _run(sl1, pe, tol=1e-10, engine="hybrid")
    a = _run(sl1, pe, tol=1e-10)
    for o in (h, a):
        assert np.array_equal(o["iters"], g["iters"]) and np.array_equal(o["x"], g["x"])
    _check_solution(pe, g, 0, obj_tol=1e-7)


def test_lq_low_precision_dense_batch(sl1):
    _say("C3-small fp8/bf16/f32 dense, l_inf bounds, batch 4")
    p = synth.with_lq_bounds(synth.config3(N=256, K=1024, s=20, batch=4), np.inf)
    out = _run(sl1, p, tol=1e-10, engine="grid")
    assert out["status"] == 0
    for b in range(p.batch):
        _check_solution(p, out, b)
    h = _run(sl1, p, tol=1e-10, engine="hybrid")
    for b in range(p.batch):
        _check_solution(p, h, b)


# ---------------------------------------------------------------------------
# the GAP dome (a dome region, Section I-E's extension), intersected with the sphere
# ---------------------------------------------------------------------------
DOME_CASES = [(0, 0.5, "fista"), (1, 0.5, "fista"), (2, 0.8, "fista"), (1, 0.3, "ista")]


@pytest.mark.parametrize("real,frac,update", DOME_CASES)
def test_dome_trace_matches_method_reference(sl1, real, frac, update):
    _say(f"trace C1 dome real={real} frac={frac} {update}")
    p = synth.config1(realization=real, lam_frac=frac)
    out = _run(sl1, p, tol=1e-10, trace_cap=5000, engine="grid", rule="dome", update=update)
    ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in p.stages], p.atom_norm, p.Y[0], float(p.lam[0]),
                      [s.rc_theory for s in p.stages], Gamma=0.5, tol=1e-10, rule="dome", update=update)
    n = int(out["iters"][0])
    assert ref.converged and out["status"] == 0 and n == ref.iters
    tr = out["trace"][0][:n]
    assert [int(r) for r in tr[:, 1]] == [r.stage for r in ref.trace]
    assert [int(r) for r in tr[:, 2]] == [r.n_active for r in ref.trace]
    assert [int(r) for r in tr[:, 3]] == [r.n_keep for r in ref.trace]
    assert [int(r) for r in tr[:, 4]] == [r.K_t for r in ref.trace]
    np.testing.assert_allclose(tr[:, 6], [r.G_conv for r in ref.trace], rtol=1e-7, atol=1e-12)
    _check_solution(p, out, 0, obj_tol=1e-7)


def test_dome_screens_at_least_as_early_as_the_sphere(sl1):
    # the dome test never exceeds the sphere test at the same point; on this case it
    # shrinks the preserved sets sooner (oracle: 15631 vs 4458 atom-iterations)
    _say("dome vs GAP sphere, C1 real=1 frac=0.5")
    p = synth.config1(realization=1, lam_frac=0.5)
    g = _run(sl1, p, tol=1e-10, trace_cap=5000, engine="grid")
    d = _run(sl1, p, tol=1e-10, trace_cap=5000, engine="grid", rule="dome")
    work = lambda o: int(o["trace"][0][:int(o["iters"][0]), 2].sum())
    assert work(d) < 0.5 * work(g)
    _check_solution(p, d, 0, obj_tol=1e-7)


def test_dome_engines_lq_bounds_and_batch(sl1):
    from paper_1812_06635_amd._lib import ELIMIT, Stablel1Error
    _say("dome: whole-solve engine refused, hybrid = grid, l_inf bounds trace, bf16 Kronecker batch")
    p = synth.config1(realization=2, lam_frac=0.8)
    with pytest.raises(Stablel1Error) as e:
        _run(sl1, p, tol=1e-10, engine="wg", rule="dome")
    assert e.value.code == ELIMIT
    g = _run(sl1, p, tol=1e-10, engine="grid", rule="dome")
    for eng in ("hybrid", "auto"):
        h = _run(sl1, p, tol=1e-10, engine=eng, rule="dome")
        assert np.array_equal(h["iters"], g["iters"]) and np.array_equal(h["x"], g["x"])
    pq = synth.with_lq_bounds(p, np.inf)
    out = _run(sl1, pq, tol=1e-10, trace_cap=5000, rule="dome")
    ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in pq.stages], p.atom_norm, p.Y[0], float(p.lam[0]),
                      [s.rc_theory for s in pq.stages], tol=1e-10, rule="dome", q=[s.q for s in pq.stages])
    n = int(out["iters"][0])
    assert n == ref.iters
    assert [int(r) for r in out["trace"][0][:n, 3]] == [r.n_keep for r in ref.trace]
    pb = synth.config4(batch=24, n=(16, 32))
    ob = _run(sl1, pb, tol=1e-10, rule="dome")
    assert ob["status"] == 0
    for b in range(pb.batch):
        _check_solution(pb, ob, b)


# ---------------------------------------------------------------------------
# the newer options together with the older ones, against the method reference
# ---------------------------------------------------------------------------
def _combo(name):
    if name == "dst l_inf":
        return synth.with_lq_bounds(synth.config1(realization=2, lam_frac=0.8), np.inf), dict(rule="dst"), None
    if name == "dome every 3":
        return synth.config1(realization=1, lam_frac=0.5), dict(rule="dome", screen_every=3), None
    if name == "faust q=3":            # the FAuST trace case above, bounds in l3
        p = synth.config6(N=64, K=515, depth=3, col_nnz=(8, 8, 24), keeps=(8, 12, 16), lam_frac=0.2,
                          dtype="f64", work="f64")
        return synth.with_lq_bounds(p, 3.0), dict(), None
    if name == "warm l1":
        p = synth.with_lq_bounds(synth.config1(realization=0, lam_frac=0.5), 1.0)
        sol = ol.solve(p.A, p.Y[0], 0.6 * float(p.lam_max[0]), L=p.stages[-1].L)
        return p, dict(), sol["x"]
    raise ValueError(name)


COMBOS = ["dst l_inf", "dome every 3", "faust q=3", "warm l1"]


@pytest.mark.parametrize("name", COMBOS)
def test_option_combinations_trace_matches_method_reference(sl1, name):
    import torch
    _say(f"trace combination {name}")
    p, kw, x0 = _combo(name)
    gkw = dict(kw)
    if x0 is not None:
        gkw["x0"] = torch.from_numpy(np.ascontiguousarray(x0[None, :])).cuda()
    out = _run(sl1, p, tol=1e-10, trace_cap=20000, engine="grid", **gkw)
    ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in p.stages], p.atom_norm, p.Y[0], float(p.lam[0]),
                      [s.rc_theory for s in p.stages], Gamma=0.5, tol=1e-10, q=[s.q for s in p.stages],
                      x0=x0, **kw)
    n = int(out["iters"][0])
    assert ref.converged and out["status"] == 0 and n == ref.iters
    tr = out["trace"][0][:n]
    assert [int(r) for r in tr[:, 1]] == [r.stage for r in ref.trace]
    assert [int(r) for r in tr[:, 2]] == [r.n_active for r in ref.trace]
    assert [int(r) for r in tr[:, 3]] == [r.n_keep for r in ref.trace]
    assert [int(r) for r in tr[:, 4]] == [r.K_t for r in ref.trace]
    np.testing.assert_allclose(tr[:, 6], [r.G_conv for r in ref.trace], rtol=1e-7, atol=1e-12)
    _check_solution(p, out, 0, obj_tol=1e-7)


@pytest.mark.parametrize("engine", ["grid", "hybrid"])
def test_lq_bounds_on_bf16_kronecker_batch(sl1, engine):
    # z is the BF16-rounded residual on these stages; its l1 norm comes from that same z
    _say(f"C4-small bf16 kron, l_inf bounds, batch 24, engine={engine}")
    p = synth.with_lq_bounds(synth.config4(batch=24, n=(16, 32)), np.inf)
    out = _run(sl1, p, tol=1e-10, engine=engine)
    assert out["status"] == 0
    for b in range(p.batch):
        _check_solution(p, out, b)


def test_lq_bounds_through_the_batched_product(sl1):
    # every stage (the exact one too) with l_inf bounds: the batched product's epilogue
    # reads the stored dual norms; against the streaming correlations
    _say("C4-small, all stages l_inf, batched product vs streaming")
    p = synth.config4(batch=24, n=(16, 32))
    p = synth.with_lq_bounds(p, np.inf, stages=range(len(p.stages)))
    prod = _run(sl1, p, tol=1e-10, engine="grid", gemm_signals=1, profile=True)
    assert sl1.last_solve_profile(p.batch, p.N, p.K)["adj_gemm"][1] > 0      # the product ran
    strm = _run(sl1, p, tol=1e-10, engine="grid", batched_gemm=False)
    assert prod["status"] == 0 and strm["status"] == 0
    assert np.all(np.abs(prod["iters"] - strm["iters"]) <= 3)
    for b in range(p.batch):
        _check_solution(p, prod, b)
        rel = np.linalg.norm(prod["x"][b] - strm["x"][b]) / max(np.linalg.norm(strm["x"][b]), 1e-300)
        assert rel <= 1e-6


def test_dome_on_fp32_kronecker(sl1):
    _say("C2-small f32 kron, dome rule")
    for frac in (0.3, 0.8):
        p = synth.config2(n=(16, 32), lam_frac=frac)
        out = _run(sl1, p, tol=1e-10, rule="dome")
        assert out["status"] == 0
        _check_solution(p, out, 0)
