"""Pins of the FP64 Lasso oracle against facts fixed by the paper and the
mathematics (no GPU).  Each test would fail under a plausible mistake in the
oracle: a dropped term, a wrong sign, a transposed operand."""
import numpy as np
import pytest

import oracle.lasso as ol
import synth


def _rand_problem(seed, N=20, K=40):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, K))
    A /= np.linalg.norm(A, axis=0)
    x0 = np.zeros(K)
    x0[rng.choice(K, 4, replace=False)] = rng.standard_normal(4)
    y = A @ x0 + 0.05 * rng.standard_normal(N)
    return A, y


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lambda_at_or_above_lambda_max_gives_zero(seed):
    # Section I-A: x* = 0 is the unique solution iff lam >= ||A^T y||_inf.
    A, y = _rand_problem(seed)
    lmax = ol.lambda_max(A, y)
    assert np.isclose(lmax, np.max(np.abs(A.T @ y)))
    L = np.linalg.norm(A, 2) ** 2
    x, gap, _ = ol.fista(A, y, lmax * (1 + 1e-9), L, tol=1e-14, max_iter=200)
    assert np.all(x == 0) and gap < 1e-10
    # just below lambda_max the solution is not zero: exactly one atom enters first
    x, gap, _ = ol.fista(A, y, lmax * 0.98, L, tol=1e-14, max_iter=20000)
    assert np.count_nonzero(x) == 1
    assert np.argmax(np.abs(A.T @ y)) == np.flatnonzero(x)[0]


@pytest.mark.parametrize("seed", [0, 3])
def test_orthonormal_dictionary_closed_form(seed):
    # With A^T A = I the problem separates: x* = ST_lam(A^T y).
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((48, 48)))
    y = rng.standard_normal(48)
    lam = 0.4 * ol.lambda_max(Q, y)
    x, gap, _ = ol.fista(Q, y, lam, 1.0, tol=1e-15, max_iter=5000)
    expect = np.sign(Q.T @ y) * np.maximum(np.abs(Q.T @ y) - lam, 0)
    np.testing.assert_allclose(x, expect, atol=1e-12)
    sol = ol.solve(Q, y, lam)
    np.testing.assert_allclose(sol["x"], expect, atol=1e-12)


def test_kronecker_of_orthogonal_factors_closed_form():
    # B kron C with orthogonal square B, C is orthonormal (the Kronecker layout of
    # the structured dictionaries); the oracle must reproduce ST_lam(A^T y).
    rng = np.random.default_rng(7)
    B, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    C, _ = np.linalg.qr(rng.standard_normal((5, 5)))
    A = np.kron(B, C)
    y = rng.standard_normal(30)
    lam = 0.3 * ol.lambda_max(A, y)
    sol = ol.solve(A, y, lam, L=1.0)
    expect = np.sign(A.T @ y) * np.maximum(np.abs(A.T @ y) - lam, 0)
    np.testing.assert_allclose(sol["x"], expect, atol=1e-12)


@pytest.mark.parametrize("seed,frac", [(10, 0.2), (11, 0.5), (12, 0.8), (13, 0.05)])
def test_brute_force_enumeration_agrees(seed, frac):
    # Exact solution by enumerating supports and signs (K = 8) versus FISTA+polish.
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((6, 8))
    A /= np.linalg.norm(A, axis=0)
    y = rng.standard_normal(6)
    lam = frac * ol.lambda_max(A, y)
    xb = ol.brute_force(A, y, lam)
    sol = ol.solve(A, y, lam, tol=1e-15)
    np.testing.assert_allclose(sol["x"], xb, atol=1e-9)
    assert abs(ol.primal(A, y, lam, xb) - sol["P"]) < 1e-11


@pytest.mark.parametrize("seed", [0, 1])
def test_weak_and_strong_duality(seed):
    # D(theta) <= P(x) for every x and every theta in Delta_A (Section II); equality
    # at (x*, theta* = (y - A x*)/lam).
    A, y = _rand_problem(seed)
    lam = 0.3 * ol.lambda_max(A, y)
    rng = np.random.default_rng(100 + seed)
    for _ in range(200):
        x = rng.standard_normal(A.shape[1]) * (rng.random(A.shape[1]) < 0.2)
        th = rng.standard_normal(A.shape[0])
        th /= max(1.0, np.max(np.abs(A.T @ th)))          # into Delta_A
        assert ol.dual(y, lam, th) <= ol.primal(A, y, lam, x) + 1e-12
    sol = ol.solve(A, y, lam)
    th = sol["theta"]
    assert np.max(np.abs(A.T @ th)) <= 1 + 1e-9
    assert abs(ol.primal(A, y, lam, sol["x"]) - ol.dual(y, lam, th)) < 1e-9
    # primal-dual link y = A x* + lam theta*
    np.testing.assert_allclose(A @ sol["x"] + lam * th, y, atol=1e-12)


def test_dynamic_dual_point_is_feasible_and_gap_nonnegative():
    A, y = _rand_problem(5)
    lam = 0.2 * ol.lambda_max(A, y)
    rng = np.random.default_rng(5)
    for _ in range(100):
        x = rng.standard_normal(A.shape[1]) * (rng.random(A.shape[1]) < 0.3)
        gap, th = ol.duality_gap(A, y, lam, x)
        assert np.max(np.abs(A.T @ th)) <= 1 + 1e-12
        assert gap >= -1e-12
        # the scaled point is the best multiple of the residual direction that is
        # feasible (Section II-C, proposition on dual scaling): no other feasible
        # multiple has a larger dual value.
        rho = y - A @ x
        m = np.max(np.abs(A.T @ rho))
        for s in np.linspace(-1 / m, 1 / m, 41):
            assert ol.dual(y, lam, s * rho) <= ol.dual(y, lam, th) + 1e-12


def test_soft_threshold_is_prox_of_l1():
    # ST_u(z) minimises 1/2 (v - z)^2 + u |v| (checked on a fine grid)
    grid = np.linspace(-5, 5, 200001)
    for z in [-3.2, -0.4, 0.0, 0.7, 2.5]:
        for u in [0.0, 0.5, 1.0]:
            v = grid[np.argmin(0.5 * (grid - z) ** 2 + u * np.abs(grid))]
            assert abs(ol.soft_threshold(np.array([z]), u)[0] - v) < 1e-4


def test_oracle_certifies_config1():
    p = synth.config1()
    sol = ol.solve(p.A, p.Y[0], float(p.lam[0]), L=p.stages[-1].L)
    assert sol["kkt"] < 1e-10
    assert sol["gap"] < 1e-12
    assert sol["margin"] > 0
    assert 0 < len(sol["support"]) < p.K
