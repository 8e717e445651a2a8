"""The Lasso solution by its plain definition, in FP64 -- TEST INFRASTRUCTURE.

Parity status: pinned.  Each function below is checked in ``tests/`` against
facts the paper and the mathematics fix independently of this code: the
lambda >= lambda_max closed form (Section I-A), the soft-thresholding closed
form for orthonormal dictionaries, brute-force enumeration of supports and
signs on tiny problems, weak duality, and the KKT conditions (Section II).

Notation follows the paper: y in R^N, A = [a_1 .. a_K] in R^{N x K},
P(x|A) = 1/2 ||Ax - y||^2 + lam ||x||_1 (Section I-A, the Lasso problem),
D(theta) = 1/2 ||y||^2 - lam^2/2 ||theta - y/lam||^2 over the dual feasible set
Delta_A = {theta : ||A^T theta||_inf <= 1} (Section II, the dual problem).
"""
from __future__ import annotations

import itertools

import numpy as np


def primal(A, y, lam, x):
    """P(x|A) of the Lasso problem (Section I-A)."""
    r = A @ x - y
    return 0.5 * float(r @ r) + lam * float(np.sum(np.abs(x)))


def dual(y, lam, theta):
    """D(theta) of the dual problem (Section II)."""
    d = theta - y / lam
    return 0.5 * float(y @ y) - 0.5 * lam * lam * float(d @ d)


def lambda_max(A, y):
    """lambda_max = ||A^T y||_inf; x* = 0 iff lam >= lambda_max (Section I-A)."""
    return float(np.max(np.abs(A.T @ y)))


def soft_threshold(z, u):
    """ST_u(z) = sign(z) (|z| - u)_+ (Section I-B)."""
    return np.sign(z) * np.maximum(np.abs(z) - u, 0.0)


def dynamic_dual_point(A, y, lam, rho):
    """theta = [y^T rho / (lam ||rho||^2)] clipped to +-1/||A^T rho||_inf, times rho
    (the dynamic dual point of Section II-C: dual scaling of the projection of
    y/lam onto the residual direction)."""
    rr = float(rho @ rho)
    if rr == 0.0:
        return np.zeros_like(rho)
    s0 = float(y @ rho) / (lam * rr)
    m = float(np.max(np.abs(A.T @ rho))) if A.shape[1] else 0.0
    if m > 0.0:
        s0 = min(max(s0, -1.0 / m), 1.0 / m)
    return s0 * rho


def duality_gap(A, y, lam, x):
    """G(x, theta|A) = P(x|A) - D(theta) with theta the dynamic dual point built
    from the residual y - Ax (Section II-C, GAP Safe sphere)."""
    rho = y - A @ x
    theta = dynamic_dual_point(A, y, lam, rho)
    return primal(A, y, lam, x) - dual(y, lam, theta), theta


def fista(A, y, lam, L, tol=1e-13, max_iter=200000, check_every=10, x_init=None):
    """Plain FISTA (Beck & Teboulle, the accelerated proximal gradient method the
    paper cites for FISTA) with constant step 1/L, L >= ||A||_2^2, exact A, no
    screening.  Stops when the duality gap falls below tol * max(1, P(x))."""
    N, K = A.shape
    x = np.zeros(K) if x_init is None else np.array(x_init, dtype=np.float64)
    x_old = x.copy()
    point = x.copy()                # the extrapolated point (y_k in Beck & Teboulle)
    t = 1.0
    gap = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        grad = A.T @ (A @ point - y)
        x_new = soft_threshold(point - grad / L, lam / L)
        t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        point = x_new + ((t - 1.0) / t_new) * (x_new - x_old)
        x_old = x_new
        x = x_new
        t = t_new
        if it % check_every == 0:
            gap, _ = duality_gap(A, y, lam, x)
            if gap < tol * max(1.0, primal(A, y, lam, x)):
                break
    gap, _ = duality_gap(A, y, lam, x)
    return x, gap, it


def kkt_residual(A, y, lam, x):
    """Largest violation of the optimality conditions of Section II:
    |a_j^T (y - Ax)| <= lam for all j, and = lam sign(x_j) on the support.
    Returned relative to lam."""
    c = A.T @ (y - A @ x)
    supp = x != 0
    off = np.max(np.abs(c[~supp]) - lam, initial=0.0)
    on = np.max(np.abs(c[supp] - lam * np.sign(x[supp])), initial=0.0)
    return max(off, on, 0.0) / lam


def polish(A, y, lam, x):
    """Solve the optimality conditions on the support S and signs s of x:
    A_S^T A_S x_S = A_S^T y - lam s (Section II, optimality conditions).
    Returns the polished vector, or None when it is not sign-consistent."""
    S = np.flatnonzero(x)
    if S.size == 0:
        return np.zeros_like(x)
    s = np.sign(x[S])
    AS = A[:, S]
    G = AS.T @ AS
    rhs = AS.T @ y - lam * s
    try:
        xs = np.linalg.solve(G, rhs)
    except np.linalg.LinAlgError:
        xs = np.linalg.lstsq(G, rhs, rcond=None)[0]
    if np.any(np.sign(xs) != s):
        return None
    out = np.zeros_like(x)
    out[S] = xs
    return out


def solve(A, y, lam, L=None, tol=1e-13, max_iter=200000):
    """x* of the Lasso by FISTA in FP64, polished on its support and certified by
    the KKT conditions.  Returns a dict with x, P, gap, theta = (y - Ax)/lam
    (the primal-dual link of Section II), the support, the KKT residual and the
    strict complementarity margin min_{j not in S} (1 - |a_j^T theta|)."""
    if L is None:
        L = float(np.linalg.norm(A, 2)) ** 2 * (1 + 1e-12)
    lmax = lambda_max(A, y)
    if lam >= lmax:
        x = np.zeros(A.shape[1])
        it = 0
    else:
        x, _, it = fista(A, y, lam, L, tol=tol, max_iter=max_iter)
        xp = polish(A, y, lam, x)
        if xp is not None and kkt_residual(A, y, lam, xp) <= kkt_residual(A, y, lam, x):
            x = xp
    gap, _ = duality_gap(A, y, lam, x)
    theta = (y - A @ x) / lam
    supp = np.flatnonzero(x)
    corr = np.abs(A.T @ theta)
    mask = np.ones(A.shape[1], dtype=bool)
    mask[supp] = False
    margin = float(np.min(1.0 - corr[mask])) if mask.any() else np.inf
    return dict(x=x, P=primal(A, y, lam, x), gap=gap, theta=theta, support=supp,
                kkt=kkt_residual(A, y, lam, x), margin=margin, iters=it, L=L)


def brute_force(A, y, lam):
    """Exact Lasso solution of a tiny problem by enumerating every support S and
    sign pattern s, solving A_S^T A_S x_S = A_S^T y - lam s and keeping the
    candidates that satisfy all optimality conditions; the smallest objective
    wins.  Independent of any iterative method; use with K <= 10."""
    N, K = A.shape
    best = (primal(A, y, lam, np.zeros(K)), np.zeros(K))
    for size in range(1, min(N, K) + 1):
        for S in itertools.combinations(range(K), size):
            AS = A[:, S]
            G = AS.T @ AS
            if np.linalg.cond(G) > 1e12:
                continue
            for s in itertools.product((-1.0, 1.0), repeat=size):
                s = np.asarray(s)
                xs = np.linalg.solve(G, AS.T @ y - lam * s)
                if np.any(np.sign(xs) != s):
                    continue
                x = np.zeros(K)
                x[list(S)] = xs
                if kkt_residual(A, y, lam, x) > 1e-9:
                    continue
                p = primal(A, y, lam, x)
                if p < best[0] - 1e-12:
                    best = (p, x)
    return best[1]
