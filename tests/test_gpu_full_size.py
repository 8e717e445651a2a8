"""GPU parity at the full sizes of the workloads (run with -m gpu): the batched
low-precision Kronecker workload on all 512 signals, the single-signal Kronecker
dictionary (N=4096, K=16384) at three lambdas, the dense precision workload
(N=2500, K=10000), the implicit adjoint on four signals of the large Kronecker
dictionary, the structured adjoint with two column tiles, and Kronecker tile
skipping.  Expected values come from ``oracle`` only (``oracle.pool`` runs its
per-signal solves in worker processes)."""
import numpy as np
import pytest

import oracle.lasso as ol
import oracle.pool as opool
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
    st = stages or p.stages
    ups = [sl1.upload_stage(s) for s in st]
    wt = torch.float64 if p.work == "f64" else torch.float32
    out = sl1.solve(ups, [s.L for s in st], [s.rc_theory for s in st], _t(p.atom_norm), _t(p.Y, wt), _t(p.lam),
                    tol=tol, **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


def _errors(p, out, b, xs, Ps):
    """unsafe rejections, relative objective error and ||x - x*|| / ||x*|| of signal b."""
    y, lam = p.Y[b], float(p.lam[b])
    x = out["x"][b].astype(np.float64)
    unsafe = int(np.sum((out["screened"][b] == 1) & (xs != 0)))
    rel_obj = (ol.primal(p.A, y, lam, x) - Ps) / Ps
    nx = np.linalg.norm(xs)
    rel_x = np.linalg.norm(x - xs) / nx if nx > 0 else float(np.abs(x).max())
    return unsafe, rel_obj, rel_x


@pytest.mark.timeout(900)
def test_batched_workload_all_512_signals(sl1):
    # the headline workload at its full size and batch, solved to gap 1e-10 (at gap 1e-9 the
    # distance to x* of an ill-conditioned support, ~sqrt(2 G) / sigma_min(A_S), can exceed the
    # 1e-4 bar): every signal against the Lasso solution
    _say("C4 full: 512 signals, N=1024, K=4096, BF16 Kronecker stages then FP32 A, tol 1e-10")
    p = synth.config4()
    out = _run(sl1, p, tol=1e-10)
    assert out["status"] == 0, f"signals above the gap: {np.flatnonzero(out['gap'] >= 1e-10)}"
    assert np.all(out["stage"] == len(p.stages) - 1) and np.all(out["gap"] < 1e-10)

    def progress(done, total):
        if done % 64 == 0 or done == total:
            _say(f"C4 full: oracle solved {done} of {total} signals")

    ref = opool.solve_batch(p.A, p.Y, p.lam, p.stages[-1].L, progress=progress)
    err = np.zeros((p.batch, 3))
    for b in range(p.batch):
        xs, Ps, kkt, _ = ref[b]
        assert kkt <= 1e-9, f"oracle not certified on signal {b}"
        err[b] = _errors(p, out, b, xs, Ps)
    w = np.argmax(err, axis=0)
    _say(f"C4 full: unsafe {int(err[:, 0].sum())}, max rel objective {err[w[1], 1]:.2e} (signal {w[1]}), "
         f"max rel x {err[w[2], 2]:.2e} (signal {w[2]})")
    assert err[:, 0].sum() == 0, f"unsafe rejections on signals {np.flatnonzero(err[:, 0])}"
    assert err[:, 1].max() <= 1e-5 and err[:, 2].max() <= 1e-4


@pytest.mark.parametrize("frac", [0.3, 0.5, 0.8])
def test_single_signal_kronecker_full_size(sl1, frac):
    # N=4096 (64x64), K=16384 (128x128), R_A=8, FP32 factors R = 1, 2, 4, 8 then the FP32 A:
    # its Kronecker stages take k1 = 128 atoms per row of tiles (two 64-atom column tiles)
    _say(f"C2 full: N=4096, K=16384, lambda = {frac} lambda_max")
    p = synth.config2(lam_frac=frac)
    out = _run(sl1, p, tol=1e-9)
    assert out["status"] == 0 and out["stage"][0] == len(p.stages) - 1
    sol = ol.solve(p.A, p.Y[0], float(p.lam[0]), L=p.stages[-1].L)
    assert sol["kkt"] <= 1e-9
    unsafe, rel_obj, rel_x = _errors(p, out, 0, sol["x"], sol["P"])
    _say(f"C2 full frac={frac}: iters {int(out['iters'][0])}, |S| {sol['support'].size}, "
         f"rel objective {rel_obj:.2e}, rel x {rel_x:.2e}")
    assert unsafe == 0 and rel_obj <= 1e-5 and rel_x <= 1e-4


def test_kronecker_adjoint_with_two_column_tiles(sl1):
    # the correlation kernel of the N=4096, K=16384 Kronecker stages (k1 = 128: atoms
    # j1 >= 64 in the second column tile) atom by atom against FP64 products
    import torch
    p = synth.config2()
    for k, st in enumerate(p.stages[:-1]):
        _say(f"adjoint C2 full stage {k} {st.label}")
        d = sl1.upload_stage(st)
        g, z = sl1.adjoint(d, _t(p.Y, torch.float32))
        g, z = g.cpu().numpy(), z.cpu().numpy().astype(np.float64)
        At = st.values()
        ref = z @ At
        Bv, Cv = st.factor_values()
        scale = np.abs(z) @ synth.workloads._kron_sum(np.abs(Bv), np.abs(Cv)) + 1e-300
        err = np.abs(g - ref) / scale
        assert np.max(err) <= 2e-5, (k, float(np.max(err)))
        half = p.K // 2                   # j1 >= 64: the second column tile
        assert np.max(err[:, half:]) <= 2e-5
        d.free()


def test_dense_precision_workload_full_size(sl1):
    # N=2500, K=10000 dense i.i.d. A (FP32 = exact), stages FP8-E4M3 and BF16 column-scaled
    # copies then A; y = A x0 normalised, lambda = 0.5 lambda_max
    _say("C3 full: N=2500, K=10000, FP8 -> BF16 -> FP32")
    p = synth.config3()
    out = _run(sl1, p, tol=1e-9)
    assert out["status"] == 0 and out["stage"][0] == len(p.stages) - 1
    sol = ol.solve(p.A, p.Y[0], float(p.lam[0]), L=p.stages[-1].L)
    assert sol["kkt"] <= 1e-9
    unsafe, rel_obj, rel_x = _errors(p, out, 0, sol["x"], sol["P"])
    _say(f"C3 full: iters {int(out['iters'][0])}, |S| {sol['support'].size}, rel objective {rel_obj:.2e}, "
         f"rel x {rel_x:.2e}")
    assert unsafe == 0 and rel_obj <= 1e-5 and rel_x <= 1e-4


def test_implicit_adjoint_full_size(sl1):
    # four signals on the N=4096, K=16384 dictionary (FP32 forward with the method,
    # backward by the implicit adjoint) against the closed form on the oracle's support and
    # central differences of the oracle's solution map (h = 1e-6; each perturbed solution is
    # the oracle's support solve, certified by the optimality conditions)
    import torch
    _say("C5 full: implicit adjoint, 4 signals, N=4096, K=16384")
    p = synth.config5(batch=4)
    out = _run(sl1, p, tol=1e-10)
    assert out["status"] == 0
    A = p.A
    exact = sl1.upload_stage(p.stages[-1])
    x = out["x"].astype(np.float64)
    dx = 2.0 * (x - p.X0)
    dy, dlam = sl1.grad(exact, _t(out["x"]), _t(p.Y, torch.float32), _t(p.lam), _t(dx))
    dy, dlam = dy.cpu().numpy().astype(np.float64), dlam.cpu().numpy()
    rng = np.random.default_rng(7)
    for b in range(p.batch):
        y, lam = p.Y[b], float(p.lam[b])
        sol = ol.solve(A, y, lam, L=p.stages[-1].L, tol=1e-15)
        xs = sol["x"]
        assert sol["kkt"] <= 1e-10 and sol["margin"] > 1e-4     # certified, strict complementarity
        S = np.flatnonzero(xs)
        AS = A[:, S]
        G = AS.T @ AS
        v = 2 * (xs - p.X0[b])[S]
        w = np.linalg.solve(G, v)
        g_ref = AS @ w
        l_ref = -np.sign(xs[S]) @ w
        assert np.linalg.norm(dy[b] - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
        assert abs(dlam[b] - l_ref) <= 1e-4 * abs(l_ref) + 1e-8

        def loss(yy, ll):
            xp = ol.polish(A, yy, ll, xs)
            assert xp is not None and ol.kkt_residual(A, yy, ll, xp) <= 1e-9
            return float(np.sum((xp - p.X0[b]) ** 2))

        u = rng.standard_normal(len(y))
        u /= np.linalg.norm(u)
        h = 1e-6
        fd = (loss(y + h * u, lam) - loss(y - h * u, lam)) / (2 * h)
        assert abs(fd - dy[b] @ u) <= 1e-4 * max(1.0, abs(fd))
        fdl = (loss(y, lam + h) - loss(y, lam - h)) / (2 * h)
        assert abs(fdl - dlam[b]) <= 1e-4 * max(1.0, abs(fdl))


def test_kronecker_tile_skipping_runs_and_matches_the_method_reference(sl1):
    # A dictionary that is one Kronecker product up to noise 1e-3 (eps ~ 1e-3 on its
    # structured stage), held on that stage (relative complexity 0 and Gamma = 0 switch
    # off Algorithm 2): the preserved set falls below K/16 atoms, from where the
    # correlation launch skips the tiles whose atoms are all screened; the per-iteration
    # trace still equals the method reference's (FP64, N=256, K=1024)
    _say("tile skipping: near-exact Kronecker dictionary held on its structured stage for 300 iterations")
    import torch
    p = synth.kron_near_exact(noise=1e-3, lam_frac=0.5)
    st = p.stages
    ups = [sl1.upload_stage(s) for s in st]
    n_it = 300
    res = sl1.solve(ups, [s.L for s in st], [0.0, 1.0], _t(p.atom_norm), _t(p.Y, torch.float64), _t(p.lam),
                    Gamma=0.0, tol=1e-10, max_iter=n_it, trace_cap=n_it + 1, engine="grid", check=False)
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}
    ref = osc.fast_l1([(s.values(), s.eps, s.L) for s in st], p.atom_norm, p.Y[0], float(p.lam[0]), [0.0, 1.0],
                      Gamma=0.0, tol=1e-10, max_iter=n_it)
    assert not ref.converged and int(out["iters"][0]) == ref.iters == n_it
    tr = out["trace"][0][:n_it]
    assert np.all(tr[:, 1] == 0)                                     # never left the structured stage
    skipping = tr[:, 2] * 16 <= p.K
    assert skipping.sum() >= 200, "the preserved set must fall below K/16 on the Kronecker stage"
    assert [int(r) for r in tr[:, 2]] == [r.n_active for r in ref.trace]
    assert [int(r) for r in tr[:, 3]] == [r.n_keep for r in ref.trace]
    assert [int(r) for r in tr[:, 4]] == [r.K_t for r in ref.trace]
    np.testing.assert_allclose(tr[:, 6], np.array([r.G_conv for r in ref.trace]), rtol=1e-7, atol=1e-12)
    np.testing.assert_allclose(out["x"][0], ref.x, rtol=0, atol=1e-9 * max(1, np.abs(ref.x).max()))
    # and the default method on this dictionary reaches the Lasso solution safely
    full = _run(sl1, p, tol=1e-10, engine="grid")
    sol = ol.solve(p.A, p.Y[0], float(p.lam[0]), L=st[-1].L)
    unsafe, rel_obj, rel_x = _errors(p, full, 0, sol["x"], sol["P"])
    assert unsafe == 0 and rel_obj <= 1e-7 and rel_x <= 1e-4
