"""Pins of the oracle's GAP dome rule (a dome region, the extension named in
Section I-E and the conclusion; the zone bounds of Lemma 1; the gap bound of
Theorem 1) against a constrained optimiser, sampled regions, the projection
property of the dual solution and the exact Lasso solution (no GPU)."""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle.lasso as ol
import oracle.screening as osc
import synth


def _unit(rng, n):
    v = rng.standard_normal(n)
    return v / np.linalg.norm(v)


def _in_ball(rng, n, size):
    u = rng.standard_normal((size, n))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return u * rng.random((size, 1)) ** (1.0 / n)


def _dome(y, lam, theta, rin2):
    """Centre, radius, unit normal and cut offset of the GAP dome of theta."""
    d = y / lam - theta
    Rd = float(np.linalg.norm(d))
    m = 0.5 * (y / lam + theta)
    n = d / Rd
    dc = osc.gap_dome_cut(Rd, rin2)
    return m, 0.5 * Rd, n, dc * 0.5 * Rd, Rd


@pytest.mark.parametrize("delta", [-0.9, -0.4, 0.0, 0.3, 0.8, 1.0])
def test_dome_cap_is_the_supremum(delta):
    # sup {u^T v : ||v|| <= 1, n^T v <= delta}: the closed form against SLSQP, an explicit
    # maximiser and samples of the cut ball; monotone in both arguments
    rng = np.random.default_rng(int(10 * (delta + 1)))
    n_dim = 6
    for _ in range(25):
        u, n = _unit(rng, n_dim), _unit(rng, n_dim)
        t = float(n @ u)
        cap = float(osc.dome_cap(delta, t))
        res = minimize(lambda v: -(u @ v), np.zeros(n_dim), method="SLSQP",
                       constraints=[{"type": "ineq", "fun": lambda v: 1.0 - v @ v},
                                    {"type": "ineq", "fun": lambda v: delta - n @ v}],
                       options={"ftol": 1e-14, "maxiter": 500})
        assert abs(-res.fun - cap) < 1e-6
        if t <= delta:
            best = u
        else:                                        # on the cut circle, towards u
            w = u - t * n
            best = delta * n + np.sqrt(1 - delta ** 2) * w / np.linalg.norm(w)
        assert np.linalg.norm(best) <= 1 + 1e-12 and n @ best <= delta + 1e-12
        assert abs(u @ best - cap) < 1e-12
        v = _in_ball(rng, n_dim, 3000)
        v = v[v @ n <= delta]
        if len(v):
            assert np.max(v @ u) <= cap + 1e-12
    ts = np.linspace(-1, 1, 41)
    assert np.all(np.diff(osc.dome_cap(delta, ts)) <= 1e-15)
    ds = np.linspace(-1, 1, 41)
    for t in (-0.5, 0.2, 0.9):
        assert np.all(np.diff(osc.dome_cap(ds, t)) >= -1e-15)


def test_dome_test_with_exact_atoms_is_the_supremum_over_the_dome():
    # eps = 0: the test is sup over the dome of |a^T theta|, attained on its boundary
    rng = np.random.default_rng(21)
    N, lam = 7, 0.7
    for _ in range(40):
        y, theta, a = rng.standard_normal(N), rng.standard_normal(N), rng.standard_normal(N)
        Rd = np.linalg.norm(y / lam - theta)
        rin2 = rng.random() * Rd ** 2
        m, r, n, off, _ = _dome(y, lam, theta, rin2)
        mu = float(osc.stable_dome_test(a @ y / lam, a @ theta, 0.0, Rd, rin2, np.linalg.norm(a)))
        best = 0.0
        for sign in (1.0, -1.0):
            res = minimize(lambda v: -sign * (a @ (m + r * v)), np.zeros(N), method="SLSQP",
                           constraints=[{"type": "ineq", "fun": lambda v: 1.0 - v @ v},
                                        {"type": "ineq", "fun": lambda v: off / r - n @ v}],
                           options={"ftol": 1e-14, "maxiter": 500})
            best = max(best, -res.fun)
        assert abs(best - mu) <= 1e-6 * max(1.0, mu)
        th = m + r * _in_ball(rng, N, 2000)
        th = th[(th - m) @ n <= off]
        if len(th):
            assert np.max(np.abs(th @ a)) <= mu + 1e-12


def _feasible_scaling(A, rho):
    return rho / max(1.0, float(np.max(np.abs(A.T @ rho))))


@pytest.mark.parametrize("seed", range(5))
def test_gap_dome_contains_the_dual_solution(seed):
    # theta* = (y - A x*)/lambda lies in the ball with diameter [theta, y/lambda] for any
    # feasible theta and beyond the cut given by the primal value, for exact and for
    # approximate dictionaries (stable point theta', P(x|A~) + delta(x) of Theorem 1)
    rng = np.random.default_rng(100 + seed)
    N, K = 14, 36
    A = rng.standard_normal((N, K))
    A /= np.linalg.norm(A, axis=0)
    y = rng.standard_normal(N)
    lam = 0.3 * float(np.max(np.abs(A.T @ y)))
    sol = ol.solve(A, y, lam)
    ts = (y - A @ sol["x"]) / lam
    for level in (0.0, 0.05, 0.3):
        E = level * rng.standard_normal((N, K)) / np.sqrt(N)
        At = A - E
        eps = np.linalg.norm(E, axis=0) * (1 + 1e-12)
        for _ in range(10):
            x = sol["x"] + rng.standard_normal(K) * (rng.random(K) < 0.3) * rng.random()
            rho = y - At @ x
            g = At.T @ rho
            m_st = osc.stable_dual_scaling(g, eps, np.linalg.norm(rho))
            r2 = float(rho @ rho)
            s = osc.clip_scale(float(y @ rho) / (lam * r2), m_st)
            theta = s * rho
            assert np.max(np.abs(A.T @ theta)) <= 1 + 1e-12                  # Lemma 2
            P = 0.5 * r2 + lam * np.abs(x).sum()
            _, delta = osc.stable_gap_radius(0.0, np.sqrt(r2), eps.max(), np.abs(x).sum(), lam)
            rin2 = max(float(y @ y) - 2 * (P + delta), 0.0) / lam ** 2
            m, r, n, off, _ = _dome(y, lam, theta, rin2)
            assert np.linalg.norm(ts - m) <= r * (1 + 1e-9) + 1e-12
            assert n @ (ts - m) <= off + 1e-9 * r + 1e-12


def test_gap_dome_collapses_to_the_dual_solution_at_the_optimum():
    # at x = x* and theta = theta* the cut sits at the far end of the ball (delta_c = -1)
    # and the dome test is |a_j^T theta*| itself
    rng = np.random.default_rng(7)
    N, K = 12, 30
    A = rng.standard_normal((N, K))
    A /= np.linalg.norm(A, axis=0)
    y = rng.standard_normal(N)
    lam = 0.4 * float(np.max(np.abs(A.T @ y)))
    sol = ol.solve(A, y, lam)
    ts = (y - A @ sol["x"]) / lam
    P = ol.primal(A, y, lam, sol["x"])
    rin2 = max(float(y @ y) - 2 * P, 0.0) / lam ** 2
    Rd = float(np.linalg.norm(y / lam - ts))
    assert osc.gap_dome_cut(Rd, rin2) <= -1 + 1e-8
    mu = osc.stable_dome_test(A.T @ y / lam, A.T @ ts, 0.0, Rd, rin2, np.linalg.norm(A, axis=0))
    assert np.max(np.abs(mu - np.abs(A.T @ ts))) <= 1e-4
    gap_sphere = osc.sphere_test(A.T @ ts, np.sqrt(2 * max(P - ol.dual(y, lam, ts), 0)) / lam, 1.0)
    assert np.all(mu <= np.maximum(gap_sphere, np.abs(A.T @ ts)) + 1e-4)


@pytest.mark.parametrize("q", [2.0, np.inf])
def test_stable_dome_test_bounds_every_atom_of_the_zone(q):
    # Lemma 1's zone (||a - a~||_q <= eps, ||a||_2 = alpha) against the dome of theta':
    # |a^T theta| <= the stable test for sampled zone atoms and dome points
    rng = np.random.default_rng(31)
    N, lam = 8, 0.6
    qs = osc.dual_exponent(q)
    for _ in range(30):
        y, theta, at = rng.standard_normal(N), rng.standard_normal(N), rng.standard_normal(N)
        eps = 0.3 * rng.random()
        Rd = np.linalg.norm(y / lam - theta)
        rin2 = rng.random() * Rd ** 2
        m, r, n, off, _ = _dome(y, lam, theta, rin2)
        th = m + r * _in_ball(rng, N, 1500)
        th = th[(th - m) @ n <= off]
        for _ in range(20):
            e = rng.standard_normal(N)
            e *= eps * rng.random() / osc.lq_norm(e, q)
            a = at + e
            mu = float(osc.stable_dome_test(a @ y / lam, at @ theta, eps * osc.lq_norm(theta, qs), Rd, rin2,
                                            np.linalg.norm(a)))
            if len(th):
                assert np.max(np.abs(th @ a)) <= mu + 1e-12


@pytest.mark.parametrize("real,frac", [(0, 0.5), (1, 0.3), (2, 0.8)])
def test_method_with_the_dome_is_safe_and_solves(real, frac):
    p = synth.config1(realization=real, lam_frac=frac)
    stages = [(s.values(), s.eps, s.L) for s in p.stages]
    y, lam = p.Y[0], float(p.lam[0])
    rc = [s.rc_theory for s in p.stages]
    sol = ol.solve(p.A, y, lam, L=p.stages[-1].L)
    for update in ("fista", "ista"):
        res = osc.fast_l1(stages, p.atom_norm, y, lam, rc, tol=1e-10, rule="dome", update=update)
        assert res.converged
        assert not np.any(res.screened & (sol["x"] != 0))
        assert np.linalg.norm(res.x - sol["x"]) <= 1e-4 * np.linalg.norm(sol["x"])
    # with l_inf bounds too
    pq = synth.with_lq_bounds(p, np.inf)
    res = osc.fast_l1([(s.values(), s.eps, s.L) for s in pq.stages], p.atom_norm, y, lam, rc, tol=1e-10,
                      rule="dome", q=[s.q for s in pq.stages])
    assert res.converged and not np.any(res.screened & (sol["x"] != 0))


def test_dome_without_a_cut_is_the_ball_with_diameter_theta_to_y_over_lambda():
    # rin2 = 0 leaves the cut at the far side of the ball (delta_c = 1): the dome test is
    # then the closed-form sphere test of B((y/lambda + theta)/2, ||y/lambda - theta||/2)
    rng = np.random.default_rng(41)
    N, K, lam = 9, 25, 0.8
    for _ in range(20):
        y, theta, A = rng.standard_normal(N), rng.standard_normal(N), rng.standard_normal((N, K))
        Rd = float(np.linalg.norm(y / lam - theta))
        assert osc.gap_dome_cut(Rd, 0.0) == 1.0
        mu = osc.stable_dome_test(A.T @ y / lam, A.T @ theta, 0.0, Rd, 0.0, np.linalg.norm(A, axis=0))
        ref = osc.sphere_test(A.T @ (0.5 * (y / lam + theta)), 0.5 * Rd, np.linalg.norm(A, axis=0))
        np.testing.assert_allclose(mu, ref, rtol=1e-13, atol=1e-13)
