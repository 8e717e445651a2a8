"""Pins of the oracle's l_q error bounds (Lemma 1 and Lemma 2 with an l_q zone,
the Appendix's dual-norm and Hoelder constants, Theorem 1 with the l2 bound the
constant gives) against linear programs, vertex enumeration, closed forms and
the exact Lasso solution (no GPU)."""
import itertools

import numpy as np
import pytest
from scipy.optimize import linprog, minimize

import oracle.lasso as ol
import oracle.screening as osc
import synth

QS = [1.0, 1.5, 3.0, np.inf]


def _unit_lq(rng, n, q, size):
    """Random points of the unit l_q sphere (directions scaled to norm 1)."""
    u = rng.standard_normal((size, n)) * rng.random((size, 1)) ** 3
    nrm = np.array([osc.lq_norm(v, q) for v in u])
    return u / nrm[:, None]


def _holder_maximizer(c, q):
    """A unit-l_q vector u with u^T c = ||c||_{q*} (the equality case of Hoelder)."""
    qs = osc.dual_exponent(q)
    if np.isinf(qs):                      # q = 1: all mass on one largest entry
        u = np.zeros_like(c)
        i = int(np.argmax(np.abs(c)))
        u[i] = np.sign(c[i])
        return u
    if qs == 1.0:                         # q = inf: the sign vector
        return np.sign(c)
    w = np.sign(c) * np.abs(c) ** (qs - 1.0)
    return w / osc.lq_norm(w, q)


def _l2_maximizer(n, q):
    """A unit-l_q vector of largest l2 norm: a coordinate vector for q <= 2, the
    flat vector n^(-1/q) (1, ..., 1) for q >= 2."""
    if q <= 2.0:
        w = np.zeros(n)
        w[0] = 1.0
        return w
    return np.full(n, float(n) ** (-1.0 / q))


def test_dual_exponent_is_the_conjugate():
    for q in [1.25, 1.5, 2.0, 3.0, 7.0]:
        qs = osc.dual_exponent(q)
        assert abs(1.0 / q + 1.0 / qs - 1.0) < 1e-15
    assert osc.dual_exponent(1.0) == np.inf
    assert osc.dual_exponent(np.inf) == 1.0
    assert osc.dual_exponent(2.0) == 2.0
    for bad in [0.5, 0.0, -1.0, np.nan]:
        with pytest.raises(ValueError):
            osc.dual_exponent(bad)


def test_lq_norm_definition_and_no_underflow():
    rng = np.random.default_rng(0)
    for p in [1.0, 1.5, 2.0, 3.0, np.inf]:
        v = rng.standard_normal(37)
        assert abs(osc.lq_norm(v, p) - np.linalg.norm(v, ord=p)) <= 1e-14 * np.linalg.norm(v, ord=p)
        assert abs(osc.lq_norm(-2.5 * np.ones(9), p) - 2.5 * 9.0 ** (0.0 if np.isinf(p) else 1.0 / p)) < 1e-13
    # homogeneity keeps large exponents finite where the plain sum underflows
    v = 1e-3 * np.ones(50)
    assert np.sum(v ** 400) == 0.0
    assert abs(osc.lq_norm(v, 400.0) - 1e-3 * 50.0 ** (1 / 400)) < 1e-17
    assert osc.lq_norm(np.zeros(4), 3.0) == 0.0


@pytest.mark.parametrize("seed", range(4))
def test_dual_norm_is_the_supremum_over_the_lq_ball(seed):
    # Appendix, first part: sup_{||u||_q <= 1} u^T c = ||c||_{q*}.  For q = inf and
    # q = 1 the supremum is a linear program; for other q a constrained optimiser
    # reaches it, the Hoelder equality case attains it and no sampled point exceeds it.
    rng = np.random.default_rng(seed)
    n = 7
    c = rng.standard_normal(n)
    box = linprog(-c, bounds=[(-1, 1)] * n, method="highs")                 # q = inf
    assert abs(-box.fun - osc.lq_norm(c, osc.dual_exponent(np.inf))) < 1e-9
    l1 = linprog(-np.concatenate([c, -c]), A_ub=np.ones((1, 2 * n)), b_ub=[1.0],
                 bounds=[(0, None)] * (2 * n), method="highs")             # q = 1
    assert abs(-l1.fun - osc.lq_norm(c, osc.dual_exponent(1.0))) < 1e-9
    for q in QS:
        qs = osc.dual_exponent(q)
        u = _holder_maximizer(c, q)
        assert abs(osc.lq_norm(u, q) - 1.0) < 1e-12
        assert abs(u @ c - osc.lq_norm(c, qs)) < 1e-12 * osc.lq_norm(c, qs)
        samples = _unit_lq(rng, n, q, 4000)
        assert np.max(samples @ c) <= osc.lq_norm(c, qs) * (1 + 1e-12)
    q = 3.0
    res = minimize(lambda u: -(u @ c), np.zeros(n), method="SLSQP",
                   constraints=[{"type": "ineq", "fun": lambda u: 1.0 - np.sum(np.abs(u) ** q)}],
                   options={"ftol": 1e-12, "maxiter": 500})
    assert abs(-res.fun - osc.lq_norm(c, 1.5)) < 1e-5


@pytest.mark.parametrize("q", [1.0, 1.5, 2.0, 3.0, np.inf])
def test_l2_constant_is_the_largest_l2_norm_of_the_lq_ball(q):
    # Appendix, second part with p* = 2: sup_{||u||_q <= 1} ||u||_2 = N^((1/2 - 1/q)_+).
    rng = np.random.default_rng(3)
    n = 8
    C = osc.l2_constant(q, n)
    w = _l2_maximizer(n, q)
    assert abs(osc.lq_norm(w, q) - 1.0) < 1e-12 and abs(np.linalg.norm(w) - C) < 1e-12
    assert np.max(np.linalg.norm(_unit_lq(rng, n, q, 5000), axis=1)) <= C * (1 + 1e-12)
    # a convex function peaks at a vertex: the cube's 2^n and the cross-polytope's 2n
    if np.isinf(q):
        best = max(np.linalg.norm(np.array(s)) for s in itertools.product([-1.0, 1.0], repeat=n))
        assert abs(best - C) < 1e-12 and abs(C - np.sqrt(n)) < 1e-12
    if q == 1.0:
        best = max(np.linalg.norm(s * np.eye(n)[i]) for i in range(n) for s in (-1.0, 1.0))
        assert best == C == 1.0


@pytest.mark.parametrize("q", QS)
def test_lemma1_lq_zone_test_bounds_and_is_attained(q):
    # Lemma 1 with S' = B_q(a~, eps) restricted to ||a||_2 = alpha: every a of the zone
    # and theta of B(c, R) give |a^T theta| <= |a~^T c| + eps ||c||_{q*} + R alpha, with
    # equality for the error aligned with c and theta = c + R a / ||a||.
    rng = np.random.default_rng(5)
    n = 9
    qs = osc.dual_exponent(q)
    for _ in range(30):
        at, c = rng.standard_normal(n), rng.standard_normal(n)
        if at @ c < 0:
            at = -at
        eps, R = 0.5 * rng.random(), rng.random()
        a = at + eps * _holder_maximizer(c, q)
        alpha = np.linalg.norm(a)
        bound = osc.stable_sphere_test(at @ c, eps, osc.lq_norm(c, qs), R, alpha)
        theta = c + R * a / alpha
        assert abs(a @ theta - bound) <= 1e-12 * bound
        for e in eps * _unit_lq(rng, n, q, 300) * rng.random((300, 1)):
            ae = at + e
            v = abs(ae @ c) + R * np.linalg.norm(ae)          # sup over the ball (Appendix A)
            assert v <= osc.stable_sphere_test(at @ c, eps, osc.lq_norm(c, qs), R, np.linalg.norm(ae)) + 1e-12


@pytest.mark.parametrize("q", QS)
def test_lemma2_lq_bounds_give_a_feasible_and_tight_dual_point(q):
    # Lemma 2 with ||a_j - a~_j||_q <= eps_j: Theta'(z) is feasible for A whatever the
    # errors, and an error aligned with z on the maximising atom makes it touch the
    # boundary, |a_j^T theta| = 1: the dual norm can be neither smaller nor larger.
    rng = np.random.default_rng(7)
    N, K = 16, 40
    qs = osc.dual_exponent(q)
    for _ in range(20):
        At = rng.standard_normal((N, K))
        z = 3.0 * rng.standard_normal(N)
        eps = 0.5 * rng.random(K)
        zq = osc.lq_norm(z, qs)
        corr = At.T @ z
        m = osc.stable_dual_scaling(corr, eps, zq)
        assert m > 1.0
        theta = z / m
        for _ in range(5):
            E = eps[None, :] * _unit_lq(rng, N, q, K).T * rng.random((1, K))
            assert np.max(np.abs((At + E).T @ theta)) <= 1.0 + 1e-12
        j = int(np.argmax(np.abs(corr) + eps * zq))
        E = np.zeros((N, K))
        E[:, j] = eps[j] * np.sign(corr[j]) * _holder_maximizer(z, q)
        assert abs(osc.lq_norm(E[:, j], q) - eps[j]) < 1e-12
        A = At + E
        assert abs(np.max(np.abs(A.T @ theta)) - 1.0) < 1e-12
        assert np.max(np.abs(At.T @ theta)) <= 1.0 + 1e-12           # feasible for A~ too


@pytest.mark.parametrize("q", QS)
def test_theorem1_delta_with_lq_bounds_covers_the_primal_change(q):
    # Theorem 1 with r = 1 needs E >= ||A - A~||_{1->2} = max_j ||e_j||_2; from l_q
    # bounds that is C max_j eps_j, C = N^((1/2 - 1/q)_+).  P(x|A) - P(x|A~) <= delta(x)
    # for every admissible error, with equality for x = t e_1, an error of largest l2
    # norm in the l_q ball and a residual along it -- so C cannot be dropped for q > 2.
    rng = np.random.default_rng(11)
    N, K, lam = 12, 30, 0.3
    C = osc.l2_constant(q, N)

    def change(A, At, x, y):
        return ol.primal(A, y, lam, x) - ol.primal(At, y, lam, x)

    for _ in range(20):
        At = rng.standard_normal((N, K))
        eps = 0.4 * rng.random(K)
        x = rng.standard_normal(K) * (rng.random(K) < 0.3)
        y = rng.standard_normal(N)
        E = eps[None, :] * _unit_lq(rng, N, q, K).T
        rho = y - At @ x
        _, delta = osc.stable_gap_radius(0.0, np.linalg.norm(rho), C * eps.max(), np.abs(x).sum(), lam)
        assert change(At + E, At, x, y) <= delta * (1 + 1e-12) + 1e-12
    # the equality case
    At = rng.standard_normal((N, K))
    t, e1, c = 1.7, 0.25, 0.9
    w = _l2_maximizer(N, q)
    x = np.zeros(K)
    x[0] = t
    y = At @ x + c * w / np.linalg.norm(w)
    E = np.zeros((N, K))
    E[:, 0] = -e1 * w
    eps = np.full(K, e1)
    got = change(At + E, At, x, y)
    _, delta = osc.stable_gap_radius(0.0, c, C * e1, t, lam)
    assert abs(got - delta) <= 1e-12 * delta
    if q > 2.0:
        _, too_small = osc.stable_gap_radius(0.0, c, e1, t, lam)
        assert got > too_small * (1 + 1e-3)


@pytest.mark.parametrize("q", QS)
def test_stable_lambda_max_with_lq_bounds(q):
    # lambda'_max = max_j (|a~_j^T y| + eps_j ||y||_{q*}) bounds ||A^T y||_inf for any
    # admissible error and equals it for the aligned error on the maximising atom.
    rng = np.random.default_rng(13)
    N, K = 10, 25
    qs = osc.dual_exponent(q)
    At, y = rng.standard_normal((N, K)), rng.standard_normal(N)
    eps = 0.3 * rng.random(K)
    lm = osc.stable_lambda_max(At, eps, y, q=q)
    for _ in range(20):
        E = eps[None, :] * _unit_lq(rng, N, q, K).T
        assert np.max(np.abs((At + E).T @ y)) <= lm * (1 + 1e-12)
    j = int(np.argmax(np.abs(At.T @ y) + eps * osc.lq_norm(y, qs)))
    E = np.zeros((N, K))
    E[:, j] = eps[j] * np.sign(At[:, j] @ y) * _holder_maximizer(y, q)
    assert abs(np.max(np.abs((At + E).T @ y)) - lm) <= 1e-12 * lm
    assert osc.stable_lambda_max(At, eps, y, q=2.0) == osc.stable_lambda_max(At, eps, y)


@pytest.mark.parametrize("q", [1.0, 3.0, np.inf])
def test_method_with_lq_bounds_is_safe_and_solves(q):
    # Algorithm 1 run on Kronecker approximations whose bounds are l_q norms of the
    # column errors: no atom of the solution's support is rejected, the preserved set
    # shrinks, the approximations are used, and the returned point solves the Lasso.
    p = synth.with_lq_bounds(synth.config1(realization=2, lam_frac=0.8), q)
    stages = [(s.values(), s.eps, s.L) for s in p.stages]
    y, lam = p.Y[0], float(p.lam[0])
    res = osc.fast_l1(stages, p.atom_norm, y, lam, [s.rc_theory for s in p.stages], tol=1e-10,
                      q=[s.q for s in p.stages])
    sol = ol.solve(p.A, y, lam, L=p.stages[-1].L)
    assert res.converged
    assert not np.any(res.screened & (sol["x"] != 0))
    assert res.screened.sum() > 0
    assert min(r.stage for r in res.trace) == 0
    on_approx = sum(r.n_active - r.n_keep for r in res.trace if r.stage < len(p.stages) - 1)
    if q in (1.0, np.inf):          # these runs stay on the approximations while they reject atoms
        assert on_approx > 0
    assert np.linalg.norm(res.x - sol["x"]) <= 1e-4 * np.linalg.norm(sol["x"])


def test_l2_bounds_through_the_lq_path_reproduce_the_default_trace():
    p = synth.config1(realization=0, lam_frac=0.5)
    p2 = synth.with_lq_bounds(p, 2.0)
    for a, b in zip(p.stages[:-1], p2.stages[:-1]):
        assert np.array_equal(a.eps, b.eps)
    args = ([(s.values(), s.eps, s.L) for s in p.stages], p.atom_norm, p.Y[0], float(p.lam[0]),
            [s.rc_theory for s in p.stages])
    r1 = osc.fast_l1(*args, tol=1e-10)
    r2 = osc.fast_l1(*args, tol=1e-10, q=2.0)
    assert r1.iters == r2.iters and np.array_equal(r1.x, r2.x)
    assert [(a.n_keep, a.K_t, a.G_stable) for a in r1.trace] == [(b.n_keep, b.K_t, b.G_stable) for b in r2.trace]


def test_lq_bounds_per_stage_and_rejection_of_q_below_one():
    p = synth.config1(realization=2, lam_frac=0.5)
    p = synth.with_lq_bounds(synth.with_lq_bounds(p, np.inf, stages=[0]), 1.0, stages=[1])
    assert [s.q for s in p.stages] == [np.inf, 1.0, 2.0, 2.0]
    stages = [(s.values(), s.eps, s.L) for s in p.stages]
    y, lam = p.Y[0], float(p.lam[0])
    res = osc.fast_l1(stages, p.atom_norm, y, lam, [s.rc_theory for s in p.stages], tol=1e-10,
                      q=[s.q for s in p.stages])
    sol = ol.solve(p.A, y, lam, L=p.stages[-1].L)
    assert res.converged and not np.any(res.screened & (sol["x"] != 0))
    with pytest.raises(ValueError):
        osc.fast_l1(stages, p.atom_norm, y, lam, [s.rc_theory for s in p.stages], q=0.5, max_iter=2)
