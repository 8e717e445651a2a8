"""Pins of the FP64 method reference (Algorithms 1-2, stable GAP Safe) against
the paper's lemmas and theorem, its printed table values, and the exact Lasso
solution (no GPU)."""
import itertools

import numpy as np
import pytest

import oracle.lasso as ol
import oracle.screening as osc
import synth
from synth import workloads as sw


def _stages(p):
    return [(s.values(), s.eps, s.L) for s in p.stages]


def _approx(rng, A, level):
    """An approximation A~ = A - E with known per-atom bounds eps_j >= ||e_j||."""
    E = level * rng.standard_normal(A.shape) / np.sqrt(A.shape[0])
    At = A - E
    eps = np.linalg.norm(E, axis=0) * (1 + 1e-12)
    return At, eps


def test_sphere_test_closed_form_is_the_supremum():
    # Appendix A: sup_{theta in B(c,R)} |a^T theta| = |a^T c| + R ||a||_2, attained
    # at c +- R a/||a|| and never exceeded by sampled points.
    rng = np.random.default_rng(0)
    for _ in range(50):
        a, c = rng.standard_normal(12), rng.standard_normal(12)
        R = rng.random() * 2
        mu = osc.sphere_test(a @ c, R, np.linalg.norm(a))
        u = rng.standard_normal((2000, 12))
        u *= (rng.random((2000, 1)) ** (1 / 12)) / np.linalg.norm(u, axis=1, keepdims=True)
        assert np.max(np.abs((c + R * u) @ a)) <= mu + 1e-12
        best = c + np.sign(a @ c) * R * a / np.linalg.norm(a)
        assert abs(abs(a @ best) - mu) < 1e-12


def test_stable_zone_test_bounds_every_atom_of_the_zone():
    # Lemma 1: for every a in B(a~, eps) with ||a|| = alpha and theta in B(c, R),
    # |a^T theta| <= |a~^T c| + eps ||c|| + R alpha.
    rng = np.random.default_rng(1)
    for _ in range(50):
        at, c = rng.standard_normal(10), rng.standard_normal(10)
        eps, R = rng.random() * 0.5, rng.random()
        e = rng.standard_normal(10)
        e *= eps * rng.random() / np.linalg.norm(e)
        a = at + e
        alpha = np.linalg.norm(a)
        bound = osc.stable_sphere_test(at @ c, eps, np.linalg.norm(c), R, alpha)
        u = rng.standard_normal((1000, 10))
        u *= (rng.random((1000, 1)) ** 0.1) / np.linalg.norm(u, axis=1, keepdims=True)
        assert np.max(np.abs((c + R * u) @ a)) <= bound + 1e-12


@pytest.mark.parametrize("level", [0.01, 0.3, 1.0])
def test_lemma2_stable_dual_scaling_is_feasible_for_both_dictionaries(level):
    rng = np.random.default_rng(2)
    A = rng.standard_normal((30, 80))
    A /= np.linalg.norm(A, axis=0)
    At, eps = _approx(rng, A, level)
    for _ in range(100):
        z = rng.standard_normal(30)
        theta = z / osc.stable_dual_scaling(At.T @ z, eps, np.linalg.norm(z))
        assert np.max(np.abs(A.T @ theta)) <= 1 + 1e-12
        assert np.max(np.abs(At.T @ theta)) <= 1 + 1e-12
    # eps = 0 recovers the conventional scaling Theta(z|A)
    z = rng.standard_normal(30)
    np.testing.assert_allclose(z / osc.stable_dual_scaling(A.T @ z, 0 * eps, np.linalg.norm(z)),
                               z / max(1, np.max(np.abs(A.T @ z))), rtol=1e-15)


@pytest.mark.parametrize("level", [0.02, 0.2])
def test_theorem1_stable_gap_sphere_contains_the_dual_solution(level):
    rng = np.random.default_rng(3)
    N, K = 25, 60
    A = rng.standard_normal((N, K))
    A /= np.linalg.norm(A, axis=0)
    At, eps = _approx(rng, A, level)
    y = A @ (rng.standard_normal(K) * (rng.random(K) < 0.1)) + 0.1 * rng.standard_normal(N)
    for frac in (0.1, 0.5, 0.9):
        lam = frac * ol.lambda_max(A, y)
        theta_star = ol.solve(A, y, lam)["theta"]
        for _ in range(60):
            x = rng.standard_normal(K) * (rng.random(K) < 0.2)
            rho = y - At @ x
            r2 = rho @ rho
            s0 = (y @ rho) / (lam * r2)
            s = osc.clip_scale(s0, np.max(np.abs(At.T @ rho) + eps * np.sqrt(r2)))
            P = 0.5 * r2 + lam * np.abs(x).sum()
            G = P - osc.dual_value_along(s, lam, y @ rho, r2, y @ y)
            R, _ = osc.stable_gap_radius(G, np.sqrt(r2), eps.max(), np.abs(x).sum(), lam)
            assert np.linalg.norm(theta_star - s * rho) <= R * (1 + 1e-12) + 1e-12


def test_stable_lambda_max_upper_bounds_lambda_max():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((20, 50))
    A /= np.linalg.norm(A, axis=0)
    for level in (0.0, 0.05, 0.5):
        At, eps = _approx(rng, A, level) if level else (A, np.zeros(50))
        y = rng.standard_normal(20)
        lm = osc.stable_lambda_max(At, eps, y)
        assert lm >= ol.lambda_max(A, y) - 1e-12
        if level == 0.0:
            assert lm == pytest.approx(ol.lambda_max(A, y), rel=1e-15)


def test_switch_dictionary_truth_table():
    # Algorithm 2: speed first (to I), then convergence (to i+1), else stay; I absorbs.
    I, K = 4, 1000
    assert osc.switch_dictionary(0, I, 0.9, 0.5, 100, 0.15, K) == I       # 100 <= 150
    assert osc.switch_dictionary(0, I, 0.1, 0.5, 100, 0.15, K) == I       # speed beats convergence
    assert osc.switch_dictionary(1, I, 0.4, 0.5, 900, 0.30, K) == 2
    assert osc.switch_dictionary(1, I, 0.5, 0.5, 900, 0.30, K) == 2       # gamma <= Gamma
    assert osc.switch_dictionary(1, I, 0.6, 0.5, 900, 0.30, K) == 1
    assert osc.switch_dictionary(I, I, 0.0, 0.5, 0, 1.0, K) == I


def test_theoretical_relative_complexity_matches_table_iv():
    # Table IV, theoretical row: RC = n_kron (1/sqrt(N) + 1/sqrt(K)) at N=2500, K=10000.
    rows = [l.split() for l in open(__file__.replace("test_oracle_screening.py", "golden/rc_table.txt"))
            if l.strip() and not l.startswith("#")]
    for n_kron, rc in rows:
        assert sw.kron_rc(int(n_kron), 50, 100) == pytest.approx(float(rc), abs=1e-12)


def _check_method(p, b=0, Gamma=0.5, tol=1e-10, **kw):
    y, lam = p.Y[b], float(p.lam[b])
    sol = ol.solve(p.A, y, lam, L=p.stages[-1].L)
    res = osc.fast_l1(_stages(p), p.atom_norm, y, lam, [s.rc_theory for s in p.stages],
                      Gamma=Gamma, tol=tol, **kw)
    return sol, res


@pytest.mark.parametrize("maker", [
    lambda: synth.config1(),
    lambda: synth.config1(realization=1, lam_frac=0.2),
    lambda: synth.config1(realization=2, lam_frac=0.8),
    lambda: synth.config2(n=(16, 32), lam_frac=0.3),
    lambda: synth.config3(N=256, K=1024),
    lambda: synth.config4(batch=1, n=(16, 32)),
    lambda: synth.config6(N=64, K=512, depth=3, col_nnz=(16, 16, 32), keeps=(16, 20, 24), lam_frac=0.2),
])
def test_method_is_safe_and_reaches_the_lasso_solution(maker):
    p = maker()
    sol, res = _check_method(p)
    assert res.converged
    xs = sol["x"]
    # zero unsafe rejections: no screened atom in the support of x*
    assert not np.any(res.screened & (xs != 0))
    # relative objective error and distance to x*
    P = ol.primal(p.A, p.Y[0], float(p.lam[0]), res.x)
    assert (P - sol["P"]) / sol["P"] <= 1e-7
    assert np.linalg.norm(res.x - xs) <= 1e-4 * np.linalg.norm(xs)
    # nested preserved sets, 0 <= gamma <= 1, K_t <= |A_t|
    na = [r.n_active for r in res.trace]
    assert all(a >= b for a, b in zip(na, na[1:]))
    for r in res.trace:
        assert -1e-12 <= r.gamma <= 1 + 1e-9
        assert r.K_t <= r.n_active
        assert r.n_keep <= r.n_active
    # stages only move forward and end on A
    st = [r.stage for r in res.trace]
    assert all(a <= b for a, b in zip(st, st[1:])) and res.stage == len(p.stages) - 1


def test_eps_zero_reduces_to_gap_safe():
    # With the single exact stage the stable test is GAP Safe (Table I): gamma = 1,
    # delta = 0 and R' = sqrt(2 G)/lam with the conventional gap.
    p = synth.config1()
    sol, res = _check_method(p)
    ex = [p.stages[-1]]
    y, lam = p.Y[0], float(p.lam[0])
    r2 = osc.fast_l1([(s.values(), s.eps, s.L) for s in ex], p.atom_norm, y, lam, [1.0], tol=1e-10)
    for r in r2.trace:
        assert r.gamma == 1.0 and r.delta == 0.0
        assert r.R_stable == pytest.approx(np.sqrt(2 * max(r.G_conv, 0)) / lam, rel=1e-14)
        # Section IV-C: with eps = 0 on A the look-ahead test (same sphere, atoms of A,
        # no eps term) is the screening test itself, so K_t counts exactly the atoms the
        # test keeps (the 1e-12 margin band holds none of them here)
        assert r.K_t == r.n_keep
    assert np.linalg.norm(r2.x - sol["x"]) <= 1e-6 * np.linalg.norm(sol["x"])
    assert not np.any(r2.screened & (sol["x"] != 0))


def test_planted_unsafe_bounds_are_caught():
    # Shrinking every eps (a mistake planted in the oracle, on the CPU) makes the
    # stable test unsafe; the safety check must notice on at least one case.
    caught = 0
    for real, frac in itertools.product(range(3), (0.2, 0.5)):
        p = synth.config1(realization=real, lam_frac=frac)
        sol, res = _check_method(p, eps_scale=0.0, Gamma=0.01)
        unsafe = np.any(res.screened & (sol["x"] != 0))
        wrong = np.linalg.norm(res.x - sol["x"]) > 1e-4 * np.linalg.norm(sol["x"])
        caught += bool(unsafe or wrong)
    assert caught > 0


def test_nkp_svd_recovers_exact_kronecker_sums():
    # Eckart-Young on the rearranged matrix: an exact R-term Kronecker sum is
    # recovered, and the truncation error equals the tail singular values.
    rng = np.random.default_rng(9)
    n1, k1, n2, k2, R = 4, 6, 5, 3, 3
    B = rng.standard_normal((R, n1, k1))
    C = rng.standard_normal((R, n2, k2))
    A = sum(np.kron(B[r], C[r]) for r in range(R))
    Bh, Ch, s = sw.nkp_factors(A, n1, k1, n2, k2, R)
    np.testing.assert_allclose(sum(np.kron(Bh[r], Ch[r]) for r in range(R)), A, atol=1e-12)
    A2 = A + 0.1 * rng.standard_normal(A.shape)
    for Rt in (1, 2, 3):
        Bh, Ch, _ = sw.nkp_factors(A2, n1, k1, n2, k2, Rt)
        At = sum(np.kron(Bh[r], Ch[r]) for r in range(Rt))
        sv = np.linalg.svd(sw._rearrange(A2, n1, k1, n2, k2), compute_uv=False)
        assert np.sum((A2 - At) ** 2) == pytest.approx(np.sum(sv[Rt:] ** 2), rel=1e-10)


def test_quantizers_match_library_rounding():
    torch = pytest.importorskip("torch")
    v = np.random.default_rng(0).standard_normal(200000).astype(np.float32) * 60
    v = np.concatenate([v, np.float32([0, -0.0, 448, -448, 2 ** -9, 2 ** -10, 3 * 2 ** -11])])
    q = synth.fp8_e4m3_decode(synth.fp8_e4m3_round(v))
    qt = torch.from_numpy(np.clip(v, -448, 448)).to(torch.float8_e4m3fn).double().numpy()
    assert np.array_equal(q, qt)
    b = synth.bf16_decode(synth.bf16_round(v))
    assert np.array_equal(b, torch.from_numpy(v).to(torch.bfloat16).double().numpy())


def test_stage_error_bounds_are_exact_column_errors():
    p = synth.config3(N=256, K=1024)
    for st in p.stages[:-1]:
        err = np.linalg.norm(p.A - st.values(), axis=0)
        assert np.all(st.eps >= err) and np.all(st.eps <= err * (1 + 1e-9) + 1e-12)
    q = synth.config4(batch=1, n=(16, 32))
    for st in q.stages[:-1]:
        err = np.linalg.norm(q.A - st.values(), axis=0)
        assert np.all(st.eps >= err)


# ---------------------------------------------------------------------------
# ISTA and the stable Dynamic Safe sphere (Table I, fourth row; Table III)
# ---------------------------------------------------------------------------
def test_dual_solution_is_the_feasible_point_nearest_y_over_lambda():
    # theta* = (y - A x*)/lambda is the projection of y/lambda onto the dual
    # feasible set (Section II), so every feasible theta is at least as far from
    # y/lambda: this is what makes B(y/lambda, ||theta - y/lambda||) safe.
    rng = np.random.default_rng(5)
    for real, frac in ((0, 0.5), (1, 0.2), (2, 0.8)):
        p = synth.config1(realization=real, lam_frac=frac)
        A, y, lam = p.A, p.Y[0], float(p.lam[0])
        sol = ol.solve(A, y, lam, L=p.stages[-1].L)
        th = (y - A @ sol["x"]) / lam
        assert np.max(np.abs(A.T @ th)) <= 1 + 1e-9
        d_star = np.linalg.norm(th - y / lam)
        for _ in range(200):
            z = rng.standard_normal(y.shape) + rng.uniform(0, 3) * y
            t = z / max(1.0, np.max(np.abs(A.T @ z)))      # feasible: ||A^T t||_inf <= 1
            assert d_star <= np.linalg.norm(t - y / lam) * (1 + 1e-12)


VARIANTS = [("fista", "dst"), ("ista", "gap"), ("ista", "dst")]


@pytest.mark.parametrize("update,rule", VARIANTS, ids=[f"{u}-{r}" for u, r in VARIANTS])
@pytest.mark.parametrize("maker", [
    lambda: synth.config1(),
    lambda: synth.config1(realization=1, lam_frac=0.2),
    lambda: synth.config1(realization=2, lam_frac=0.8),
    lambda: synth.config3(N=256, K=1024),
])
def test_method_variants_are_safe_and_reach_the_lasso_solution(maker, update, rule):
    p = maker()
    sol, res = _check_method(p, update=update, rule=rule)
    assert res.converged
    assert not np.any(res.screened & (sol["x"] != 0))
    P = ol.primal(p.A, p.Y[0], float(p.lam[0]), res.x)
    assert (P - sol["P"]) / sol["P"] <= 1e-7
    assert np.linalg.norm(res.x - sol["x"]) <= 1e-4 * np.linalg.norm(sol["x"])
    na = [r.n_active for r in res.trace]
    assert all(a >= b for a, b in zip(na, na[1:]))
    for r in res.trace:
        assert r.K_t <= r.n_active and -1e-12 <= r.gamma <= 1 + 1e-9
    if rule == "dst":
        # every traced radius covers the dual solution (centre y/lambda)
        y, lam = p.Y[0], float(p.lam[0])
        d_star = np.linalg.norm((y - p.A @ sol["x"]) / lam - y / lam)
        assert all(r.R_stable >= d_star * (1 - 1e-9) for r in res.trace)


def test_ista_objective_decreases_on_a_fixed_preserved_set():
    # ISTA is a descent method for the problem restricted to the preserved set: on
    # the exact stage, between iterations that screen nothing, P(x_t) never rises.
    p = synth.config1()
    _, r = _check_method(p, update="ista", rule="gap")
    I = len(p.stages) - 1
    rows = r.trace
    for a, b in zip(rows, rows[1:]):
        if a.stage == I and b.stage == I and a.n_keep == a.n_active:
            assert b.P <= a.P * (1 + 1e-13)


def test_dynamic_safe_screens_less_than_gap_safe_at_the_end():
    # Table I: the GAP sphere shrinks to theta* while the Dynamic Safe radius stays
    # at least ||theta* - y/lambda||, so at convergence GAP preserves fewer atoms.
    p = synth.config1(lam_frac=0.5)
    _, rg = _check_method(p)
    _, rd = _check_method(p, rule="dst")
    assert rg.trace[-1].n_keep <= rd.trace[-1].n_keep


def test_planted_unsafe_dynamic_radius_is_caught():
    # A radius scaled to zero (a mistake planted in the oracle) must break safety
    # or exactness on at least one case.
    caught = 0
    for real, frac in itertools.product(range(3), (0.2, 0.5)):
        p = synth.config1(realization=real, lam_frac=frac)
        sol, res = _check_method(p, rule="dst", radius_scale=0.0)
        unsafe = np.any(res.screened & (sol["x"] != 0))
        wrong = np.linalg.norm(res.x - sol["x"]) > 1e-4 * np.linalg.norm(sol["x"])
        caught += bool(unsafe or wrong)
    assert caught > 0


@pytest.mark.parametrize("k", [3, 7])
def test_screening_every_k_iterations_is_safe_and_exact(k):
    # Algorithm 1's variation: rejections only every k iterations.  The preserved
    # sets only shrink at those iterations and the Lasso solution is unchanged.
    p = synth.config1(realization=1, lam_frac=0.3)
    sol, res = _check_method(p, screen_every=k)
    assert res.converged and not np.any(res.screened & (sol["x"] != 0))
    assert np.linalg.norm(res.x - sol["x"]) <= 1e-4 * np.linalg.norm(sol["x"])
    for r in res.trace:
        if r.t % k != 0:
            assert r.n_keep == r.n_active
    assert any(r.n_keep < r.n_active for r in res.trace)


# ---------------------------------------------------------------------------
# warm starts along a lambda path (the sequential setting of Section I-D)
# ---------------------------------------------------------------------------
def test_warm_start_at_the_solution_needs_few_iterations_on_a():
    # on the exact dictionary alone (plain FISTA + stable GAP Safe) a start at x*
    # stops almost at once; with approximate stages first the iterate moves toward
    # the approximate problems' solutions, so Algorithm 1 keeps its cost
    p = synth.config1(realization=1, lam_frac=0.4)
    y, lam = p.Y[0], float(p.lam[0])
    sol = ol.solve(p.A, y, lam, L=p.stages[-1].L, tol=1e-14)
    exact = _stages(p)[-1:]
    cold = osc.fast_l1(exact, p.atom_norm, y, lam, [1.0], tol=1e-10)
    warm = osc.fast_l1(exact, p.atom_norm, y, lam, [1.0], tol=1e-10, x0=sol["x"])
    assert cold.converged and warm.converged
    assert warm.iters * 10 <= cold.iters
    assert not np.any(warm.screened & (sol["x"] != 0))
    assert np.linalg.norm(warm.x - sol["x"]) <= 1e-5 * np.linalg.norm(sol["x"])
    staged = osc.fast_l1(_stages(p), p.atom_norm, y, lam, [s.rc_theory for s in p.stages], tol=1e-10,
                         x0=sol["x"])
    assert staged.converged and not np.any(staged.screened & (sol["x"] != 0))


@pytest.mark.parametrize("maker", [lambda: synth.config1(realization=2),
                                   lambda: synth.config4(batch=1, n=(16, 32))])
def test_warm_started_path_is_safe_and_matches_cold_solves(maker):
    p = maker()
    y = p.Y[0]
    rc = [s.rc_theory for s in p.stages]
    for stages, rcs in ((_stages(p), rc), (_stages(p)[-1:], [1.0])):
        x0 = None
        it_warm = it_cold = 0
        for frac in (0.8, 0.5, 0.3):
            lam = frac * float(p.lam_max[0])
            sol = ol.solve(p.A, y, lam, L=p.stages[-1].L)
            warm = osc.fast_l1(stages, p.atom_norm, y, lam, rcs, tol=1e-10, x0=x0)
            cold = osc.fast_l1(stages, p.atom_norm, y, lam, rcs, tol=1e-10)
            assert warm.converged and cold.converged
            assert not np.any(warm.screened & (sol["x"] != 0))          # safe from any start
            assert (ol.primal(p.A, y, lam, warm.x) - sol["P"]) / sol["P"] <= 1e-7
            assert np.linalg.norm(warm.x - cold.x) <= 1e-4 * max(np.linalg.norm(cold.x), 1e-300)
            it_warm += warm.iters
            it_cold += cold.iters
            x0 = warm.x
        if len(stages) == 1:
            assert it_warm < it_cold                 # the path pays on the exact dictionary


def test_warm_start_from_any_point_keeps_the_first_step_plain():
    # from an arbitrary x0 the first step has no momentum: it equals a proximal
    # gradient step from x0 on the first stage (Section I-B)
    p = synth.config1()
    y, lam = p.Y[0], float(p.lam[0])
    rng = np.random.default_rng(3)
    x0 = np.where(rng.random(p.K) < 0.05, rng.standard_normal(p.K), 0.0)
    At, eps, L = _stages(p)[0]
    res = osc.fast_l1(_stages(p), p.atom_norm, y, lam, [s.rc_theory for s in p.stages], tol=1e-10,
                      x0=x0, max_iter=1)
    v = x0 + At.T @ (y - At @ x0) / L
    x1 = np.sign(v) * np.maximum(np.abs(v) - lam / L, 0.0)
    keep = ~res.screened
    np.testing.assert_allclose(res.x[keep], x1[keep], rtol=1e-12, atol=1e-14)


def test_look_ahead_count_on_a_hand_built_case():
    # K_t of Section IV-C worked out by hand at t = 0 (x_0 = 0, so rho~_0 = y).
    # y = (1, 0), lambda = 1/2; approximate atoms a~_A = (0.1, 0.3), a~_B = (0.2, 0.3),
    # a~_C = (0.6, 0), a~_D = (0.05, 1); exact atoms a_j = a~_j / ||a~_j|| except
    # a_C = (1, 0); bounds eps = (0.7, 0.64, 0.4, 0.00125) >= ||a_j - a~_j||.
    #   g = A~^T y = (0.1, 0.2, 0.6, 0.05); stable scaling max_j (|g_j| + eps_j ||y||) = 1
    #   (atom C), so s' = min(1/lambda, 1) = 1 and theta' = y;
    #   G' = 1/2 - (lambda - lambda^2/2) = 1/8, delta = 0 (x = 0), R' = sqrt(2 G')/lambda = 1;
    #   conventional: s~ = 1/0.6 = 5/3, G~ = 1/2 - (5/6 - 25/72) = 1/72, gamma = 1/9.
    #   K_0 counts |s' g_j| + R' ||a~_j|| >= 1:  A 0.1 + 0.316 = 0.42, B 0.2 + 0.361 = 0.56,
    #   C 0.6 + 0.6 = 1.2, D 0.05 + 1.001 = 1.05  ->  K_0 = 2 (C and D).
    #   Readings that would differ: adding eps_j |s'| ||y|| (A 1.12, B 1.20: K_0 = 4); ||a_j||
    #   for ||a~_j|| (A 1.1, B 1.2: K_0 = 4); the conventional sphere (theta~, sqrt(2G~)/lambda
    #   = 1/3: only C, K_0 = 1).  The screening test itself keeps all four at t = 0
    #   (|g_j| + eps_j + 1 >= 1).
    At = np.array([[0.1, 0.2, 0.6, 0.05], [0.3, 0.3, 0.0, 1.0]])
    A = At / np.linalg.norm(At, axis=0)
    A[:, 2] = (1.0, 0.0)
    eps = np.array([0.7, 0.64, 0.4, 0.00125])
    assert np.all(np.linalg.norm(A - At, axis=0) <= eps)
    y, lam = np.array([1.0, 0.0]), 0.5
    L0, L1 = np.linalg.norm(At, 2) ** 2, np.linalg.norm(A, 2) ** 2
    res = osc.fast_l1([(At, eps, L0), (A, np.zeros(4), L1)], np.ones(4), y, lam, [0.0, 1.0],
                      Gamma=0.0, tol=1e-12, max_iter=1)
    r = res.trace[0]
    assert r.t == 0 and r.stage == 0 and r.n_active == 4 and r.n_keep == 4
    assert r.K_t == 2
    assert r.G_stable == pytest.approx(1 / 8, rel=1e-14)
    assert r.R_stable == pytest.approx(1.0, rel=1e-14)
    assert r.G_conv == pytest.approx(1 / 72, rel=1e-12)
    assert r.gamma == pytest.approx(1 / 9, rel=1e-12)
    assert r.delta == 0.0


def _iterate(stages, atom_norm, y, lam, x0, t):
    """x_t and the preserved set A_t of the method (the result returned at max_iter = t)."""
    res = osc.fast_l1(stages, atom_norm, y, lam, [1.0] * len(stages), tol=0.0, max_iter=t, x0=x0,
                      keep_trace=False)
    return res.x, ~res.screened


def test_rejecting_a_nonzero_coefficient_restarts_the_momentum():
    # A warm start with spurious coefficients on atoms near the dual constraint makes the
    # test reject an atom at some t >= 1 while x_t[j] != 0.  FISTA's gradient at the
    # extrapolated point, taken by linearity from g_{t+1} and g_t, would then mix x_t
    # before and after the zeroing; the method restarts the momentum instead, so the
    # step from x_{t+1} is the plain proximal step on the preserved set (Section I-B).
    p = synth.config1(realization=0, lam_frac=0.5)
    y, lam = p.Y[0], float(p.lam[0])
    sol = ol.solve(p.A, y, lam)
    corr = p.A.T @ sol["theta"]
    cand = np.flatnonzero((sol["x"] == 0) & (np.abs(corr) > 0.8) & (np.abs(corr) < 0.95))
    x0 = sol["x"].copy()
    x0[cand] = 0.1 * np.sign(corr[cand])
    ex = p.stages[-1]
    stages = [(ex.values(), ex.eps, ex.L)]
    A, L = stages[0][0], stages[0][2]
    hit = None
    x_prev, act_prev = _iterate(stages, p.atom_norm, y, lam, x0, 1)
    for t in range(1, 40):
        x_next, act_next = _iterate(stages, p.atom_norm, y, lam, x0, t + 1)
        if np.any(x_prev[act_prev & ~act_next] != 0.0):
            hit = t
            break
        x_prev, act_prev = x_next, act_next
    assert hit is not None, "the case must reject a nonzero coefficient at some t >= 1"
    x1, _ = _iterate(stages, p.atom_norm, y, lam, x0, hit + 1)
    x2, act2 = _iterate(stages, p.atom_norm, y, lam, x0, hit + 2)
    v = x1 + A.T @ (y - A @ x1) / L
    plain = np.sign(v) * np.maximum(np.abs(v) - lam / L, 0.0)
    np.testing.assert_allclose(x2[act2], plain[act2], rtol=1e-12, atol=1e-14)
    assert not np.any(x2[~act2])
    # and the solve stays safe and exact
    res = osc.fast_l1(stages, p.atom_norm, y, lam, [1.0], tol=1e-10, x0=x0)
    assert not np.any(res.screened & (sol["x"] != 0))
    assert np.linalg.norm(res.x - sol["x"]) <= 1e-6 * np.linalg.norm(sol["x"])
