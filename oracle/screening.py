"""The paper's method step by step in FP64 -- TEST INFRASTRUCTURE.

Algorithm 1 (FastL1) with Algorithm 2 (SwitchDictionary), a FISTA update, and
the stable GAP Safe sphere test (Table I, last row), written from Sections
III and IV in the paper's order and notation.  It is the per-iteration
reference the GPU trace is compared with.  Parity status: pinned (Lemma 2,
Theorem 1, the eps = 0 reduction to GAP Safe, nested preserved sets, zero
unsafe rejections against ``oracle.lasso.solve``); the switching quantities
gamma_t and K_t have no printed values in the paper and are pinned only by
their invariants (0 <= gamma_t <= 1, K_t <= |A_t|).

Readings of points the paper leaves open (each stated where it is used):
  * FISTA is only cited; the update is Beck & Teboulle's with constant step
    1/L_i, L_i = ||A~^i||_2^2, and its momentum restarts on a dictionary switch.
  * Screening uses the prox output x_t and rho~_t = y - A~ x_t (Section III-C).
    The gradient at the extrapolated point is obtained by linearity from the
    two correlation vectors A~^T rho~_t and A~^T rho~_{t-1}.  That identity
    needs x_{t-1} as it was when A~^T rho~_{t-1} was formed; when a rejection
    zeroes a nonzero coefficient it would not hold, so the momentum restarts
    after such a rejection, as after a switch (the step is then exact).
  * The maxima defining alpha'_t, and the error scale of Theorem 1 with
    r = 1 (E = max_j eps_j, the largest column error), run over the preserved
    set A_t, as Algorithm 1 restricts the dictionary to A_t before each update.
  * An atom is rejected when its test value is below 1 - margin.
  * K_t uses the conventional sphere test on the approximate atoms with the
    same sphere (theta'_t, R'_t).
  * The stop test is the conventional duality gap once A~ = A (Section IV).
  * Screening at regular intervals (Algorithm 1's stated variation): atoms are
    rejected only every screen_every iterations; K_t and the switch are
    evaluated at every iteration.
  * Error bounds in any l_q norm (Lemma 1, Lemma 2, the Appendix): eps_j bounds
    ||a_j - a~_j||_q, q in [1, inf]; the dual scaling and the test then use the
    dual norm ||z||_{q*} (1/q + 1/q* = 1), and Theorem 1 (an l2 statement) takes
    E = N^((1/2 - 1/q)_+) max_j eps_j, the Hoelder constant of the Appendix with
    p* = 2 bounding ||a_j - a~_j||_2 by the l_q bound.  q = 2 is the default.
  * A dome region (the extension Section I-E and the conclusion point to; no formula
    is printed): the GAP dome of theta'_t (gap_dome_cut), tested with the same zone
    bounds as Lemma 1 and intersected with the stable GAP sphere, a^T y formed once on
    the exact dictionary as for stable Dynamic Safe.
  * Options beside FISTA + stable GAP Safe (Table III's other combinations):
    ISTA (the update of Section I-B, no momentum), and the stable Dynamic Safe
    sphere B(y/lambda, ||theta'_t - y/lambda||) (Table I, fourth row) tested
    with a_j^T y given: the product with the exact A is formed once, as the
    footnote to Table I allows, so the test needs no eps term.  Its look-ahead
    count K_t uses the same sphere with ||a~_j|| in place of ||a_j||.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .lasso import soft_threshold


def dual_exponent(q):
    """q* with 1/q + 1/q* = 1 (q = 1 gives inf, q = inf gives 1): the exponent of the
    dual norm that the l_q zone of Lemma 1 brings into the tests (Appendix)."""
    q = float(q)
    if q < 1.0 or np.isnan(q):
        raise ValueError("q must lie in [1, inf]")
    if q == 1.0:
        return np.inf
    if np.isinf(q):
        return 1.0
    return q / (q - 1.0)


def lq_norm(v, p):
    """||v||_p for p in [1, inf], written as m (sum (|v_i|/m)^p)^(1/p) with m = max |v_i|
    (the definition, by homogeneity) so that large p cannot underflow."""
    a = np.abs(np.asarray(v, dtype=np.float64)).ravel()
    m = float(np.max(a, initial=0.0))
    if m == 0.0 or np.isinf(p):
        return m
    return m * float(np.sum((a / m) ** p)) ** (1.0 / p)


def l2_constant(q, N):
    """sup of ||u||_2 over the unit l_q ball of R^N, N^((1/2 - 1/q)_+): the constant C
    of the Appendix with p* = 2 (Hoelder), so ||e||_2 <= C ||e||_q."""
    return float(N) ** max(0.5 - 1.0 / float(q), 0.0)


def sphere_test(at_c, radius, a_norm):
    """mu(a|B(c,R)) = |a^T c| + R ||a||_2 (closed form of Section II-B, p = 2)."""
    return np.abs(at_c) + radius * a_norm


def stable_sphere_test(at_c, eps, c_norm, radius, a_norm):
    """mu(S'|B(c,R)) = |a~^T c| + eps ||c||_{q*} + R a for the norm-restricted zone
    (Section III-B, Lemma 1, p = 2); c_norm is ||c||_{q*} of the bounds' norm q."""
    return np.abs(at_c) + eps * c_norm + radius * a_norm


def stable_dual_scaling(corr, eps, z_norm):
    """max(1, max_j (|a~_j^T z| + eps_j ||z||_{q*})): the divisor of the stable dual
    scaling Theta'(z|A~, eps) (Section III-C, Lemma 2); z_norm is ||z||_{q*}."""
    m = float(np.max(np.abs(corr) + eps * z_norm, initial=0.0))
    return max(1.0, m)


def clip_scale(s0, m):
    """[s0]_{-1/m}^{1/m} (no clipping when m = 0)."""
    if m <= 0.0:
        return s0
    return min(max(s0, -1.0 / m), 1.0 / m)


def dual_value_along(s, lam, y_dot_z, z_sq, y_sq):
    """D(s z) = 1/2||y||^2 - lam^2/2 ||s z - y/lam||^2 written with the scalars
    y^T z and ||z||^2 (Section II, dual problem)."""
    return lam * s * y_dot_z - 0.5 * lam * lam * s * s * z_sq


def stable_gap_radius(gap_tilde_A, res_norm, E, x_l1, lam):
    """R' = sqrt(2 G(x, theta|A~) + 2 delta(x)) / lam with
    delta(x) = ||y - A~x|| E ||x||_1 + E^2 ||x||_1^2 / 2 (Theorem 1, r = 1)."""
    delta = res_norm * E * x_l1 + 0.5 * E * E * x_l1 * x_l1
    return np.sqrt(2.0 * max(gap_tilde_A, 0.0) + 2.0 * delta) / lam, delta


def dynamic_radius(theta, y, lam):
    """R = ||theta - y/lambda||_2: radius of the (stable) Dynamic Safe sphere
    centred at y/lambda (Table I, third and fourth rows)."""
    return float(np.linalg.norm(theta - y / lam))


def stable_lambda_max(At, eps, y, q=2.0):
    """lambda'_max = max_j (|a~_j^T y| + eps_j ||y||_{q*}) >= lambda_max (Section III-C,
    stable static sphere), eps_j bounding ||a_j - a~_j||_q."""
    qs = dual_exponent(q)
    y_norm = np.linalg.norm(y) if qs == 2.0 else lq_norm(y, qs)
    return float(np.max(np.abs(At.T @ y) + eps * y_norm))


def dome_cap(delta, t):
    """sup {u^T v : ||v||_2 <= 1, n^T v <= delta} for unit vectors u, n with n^T u = t
    (-1 <= delta, t <= 1): 1 when the ball's own maximiser u meets the cut (t <= delta),
    otherwise the maximum over the cut circle, delta t + sqrt(1 - delta^2) sqrt(1 - t^2).
    Non-increasing in t and non-decreasing in delta."""
    delta = np.clip(np.asarray(delta, dtype=np.float64), -1.0, 1.0)
    t = np.clip(np.asarray(t, dtype=np.float64), -1.0, 1.0)
    cut = delta * t + np.sqrt(1.0 - delta * delta) * np.sqrt(1.0 - t * t)
    return np.where(t <= delta, 1.0, cut)


def gap_dome_cut(Rd, rin2):
    """Normalised cut level of the GAP dome.  theta* is the projection of y/lambda on
    the dual feasible set (Section II-C), so for a feasible theta it lies in the ball
    B(m, Rd/2) with diameter [theta, y/lambda] (m the midpoint, Rd = ||y/lambda - theta||);
    weak duality with P(x|A) <= P(x|A~) + delta(x) (Theorem 1) keeps it at distance
    >= sqrt(rin2) from y/lambda, rin2 = (||y||^2 - 2(P(x|A~) + delta(x)))_+ / lambda^2.
    As y/lambda lies on that ball's sphere, the two give the half-space
    n^T (theta - m) <= delta_c Rd/2 with n = (y/lambda - theta)/Rd and
    delta_c = 1 - 2 rin2 / Rd^2 (clipped to [-1, 1]; Rd = 0 leaves the single point y/lambda)."""
    if Rd <= 0.0:
        return -1.0
    return float(min(1.0, max(-1.0, 1.0 - 2.0 * rin2 / (Rd * Rd))))


def stable_dome_test(cy, sg, e, Rd, rin2, a_norm):
    """Upper bound of sup |a^T theta| over the atoms a of the zone (Lemma 1's restricted
    zone, ||a||_2 = a_norm) and theta in the GAP dome of theta' = s z (gap_dome_cut):
    with m = (y/lambda + theta')/2, a^T m lies within (cy + sg)/2 +- e/2 and
    Rd a^T n within (cy - sg) +- e, where cy = a^T y / lambda (the exact product, given),
    sg = s a~^T z and e = eps |s| ||z||_{q*} (the zone term); the supremum over the dome
    is a^T m + (Rd/2) a_norm dome_cap(delta_c, a^T n / a_norm), and dome_cap falls with its
    second argument, so its smallest value in the range bounds it.  Both signs of a."""
    cy, sg, e, a_norm = (np.asarray(v, dtype=np.float64) for v in (cy, sg, e, a_norm))
    dc = gap_dome_cut(Rd, rin2)
    out = None
    for sign in (1.0, -1.0):
        am = sign * (cy + sg) / 2.0 + e / 2.0
        if Rd > 0.0:
            with np.errstate(divide="ignore", invalid="ignore"):
                t = np.where(a_norm > 0, (sign * (cy - sg) - e) / (Rd * a_norm), -1.0)
            val = am + 0.5 * Rd * a_norm * dome_cap(dc, t)
        else:
            val = am
        out = val if out is None else np.maximum(out, val)
    return out


def switch_dictionary(i, I, gamma, Gamma, K_t, rc_i, K):
    """Algorithm 2: speed criterion (K_t <= RC(A~^i) K) jumps to A; otherwise the
    convergence criterion (gamma_t <= Gamma) moves to the next approximation."""
    if i >= I:
        return I
    if K_t <= rc_i * K:
        return I
    if gamma <= Gamma:
        return i + 1
    return i


@dataclass
class TraceRow:
    t: int
    stage: int
    n_active: int          # |A_t| before the test
    n_keep: int            # |A_{t+1}|
    K_t: int
    G_stable: float        # G(x_t, theta'_t | A~)
    G_conv: float          # G(x_t, theta~_t | A~)
    delta: float
    R_stable: float        # radius of the rule's sphere (R' of GAP, or ||theta' - y/lambda||)
    gamma: float
    x_l1: float
    P: float


@dataclass
class Result:
    x: np.ndarray
    gap: float             # conventional gap with A at the returned x
    gap_cert: float        # G' + delta at the returned x
    screened: np.ndarray   # bool (K,), True = rejected
    iters: int
    stage: int
    converged: bool
    trace: list = field(default_factory=list)


def fast_l1(stages, atom_norm, y, lam, rc, Gamma=0.5, tol=1e-6, max_iter=100000, margin=1e-12,
            eps_scale=1.0, keep_trace=True, update="fista", rule="gap", radius_scale=1.0, screen_every=1,
            x0=None, q=2.0):
    """Algorithm 1 (FastL1) with FISTA (or ISTA) and the stable GAP Safe (or
    stable Dynamic Safe) test.

    stages     list of (At, eps, L): At is the (N, K) FP64 matrix of the i-th
               approximation (the last one is A, with eps = 0), eps its per-atom
               error bounds (l2 unless q says otherwise) and L its Lipschitz constant.
    atom_norm  ||a_j||_2 of the exact atoms (the restricted zone of Lemma 1).
    rc         relative complexity RC(A~^i) of each stage (Section IV-B).
    eps_scale  multiplies every eps (a value below 1 plants an unsafe bound; the
               tests use it to show that the safety check can fail).
    update     "fista" or "ista" (Section I-B: x_{t+1} = ST(x_t + A~^T rho~_t / L)).
    rule       "gap" (stable GAP Safe), "dst" (stable Dynamic Safe) or "dome" (the stable
               GAP Safe sphere intersected with the GAP dome of the same dual point).
    radius_scale  multiplies the sphere radius (below 1 plants an unsafe test).
    screen_every  atoms are rejected only at iterations t with t % screen_every == 0
               (the variation of Algorithm 1 that screens at regular intervals); the
               dual points, gaps and K_t are formed at every iteration.
    x0         initial iterate (warm start, e.g. the solution at the previous lambda
               of a path, the sequential setting Section I-D mentions); default 0.
               The preserved set still starts with every atom, and the first step
               has no momentum, so screening stays safe whatever x0 is.
    q          norm of the error bounds, one value or one per stage: eps_j of stage i
               bounds ||a_j - a~^i_j||_{q_i}, 1 <= q_i <= inf (Lemma 1 with an l_q zone).
    """
    if update not in ("fista", "ista") or rule not in ("gap", "dst", "dome"):
        raise ValueError("update must be fista|ista and rule gap|dst|dome")
    I = len(stages) - 1
    N, K = stages[0][0].shape
    qs_list = [float(v) for v in (np.broadcast_to(np.asarray(q, dtype=np.float64), (I + 1,)))]
    for v in qs_list:
        dual_exponent(v)                                   # rejects q < 1
    y = np.asarray(y, dtype=np.float64)
    y_sq = float(y @ y)
    x = np.zeros(K) if x0 is None else np.array(x0, dtype=np.float64)
    x_prev = x.copy()
    g_prev = np.zeros(K)
    active = np.ones(K, dtype=bool)
    i = 0
    tau = 1.0
    k_since = 0
    trace = []
    At, eps, L = stages[0]
    at_norms = [np.linalg.norm(s[0], axis=0) for s in stages]
    # stable Dynamic Safe and the GAP dome: a_j^T y with the exact dictionary, formed once
    aty = stages[I][0].T @ y if rule in ("dst", "dome") else None
    res = None
    for t in range(max_iter + 1):
        At, eps, L = stages[i]
        eps = eps * eps_scale
        act = np.flatnonzero(active)
        # ---- products on the preserved set (restriction step of Algorithm 1)
        rho = y - At[:, act] @ x[act]
        g = np.zeros(K)
        g[act] = At[:, act].T @ rho
        # ---- stable dual point theta'_t and conventional theta~_t (Section III-C, IV-A)
        r_sq = float(rho @ rho)
        r_norm = np.sqrt(r_sq)
        y_rho = float(y @ rho)
        s0 = y_rho / (lam * r_sq) if r_sq > 0 else 0.0
        # ||rho~_t||_{q*}: the norm that the l_q error bounds of this stage pair with
        q_dual = dual_exponent(qs_list[i])
        z_norm = r_norm if q_dual == 2.0 else lq_norm(rho, q_dual)
        m_stable = float(np.max(np.abs(g[act]) + eps[act] * z_norm, initial=0.0))
        m_conv = float(np.max(np.abs(g[act]), initial=0.0))
        s_stable = clip_scale(s0, m_stable)
        s_conv = clip_scale(s0, m_conv)
        x_l1 = float(np.sum(np.abs(x)))
        P = 0.5 * r_sq + lam * x_l1
        G_stable = P - dual_value_along(s_stable, lam, y_rho, r_sq, y_sq)
        G_conv = P - dual_value_along(s_conv, lam, y_rho, r_sq, y_sq)
        E = float(np.max(eps[act], initial=0.0))
        if qs_list[i] != 2.0:                              # ||a_j - a~_j||_2 <= C ||a_j - a~_j||_q
            E *= l2_constant(qs_list[i], N)
        R_stable, delta = stable_gap_radius(G_stable, r_norm, E, x_l1, lam)
        if rule == "dst":
            R_test = dynamic_radius(s_stable * rho, y, lam)       # ||theta'_t - y/lambda||
        else:
            R_test = float(R_stable)
        R_test *= radius_scale
        gamma = G_conv / G_stable if G_stable > 0 else 1.0
        # ---- stopping criterion: conventional gap once A~ = A (Section IV)
        if i == I and G_conv < tol:
            res = Result(x=x.copy(), gap=G_conv, gap_cert=G_stable + delta, screened=~active,
                         iters=t, stage=i, converged=True, trace=trace)
            break
        if t == max_iter:
            res = Result(x=x.copy(), gap=G_conv, gap_cert=G_stable + delta, screened=~active,
                         iters=t, stage=i, converged=False, trace=trace)
            break
        # ---- update of the preserved coefficients (FISTA or ISTA step)
        if k_since == 0 or update == "ista":
            beta = 0.0
        else:
            tau_next = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * tau * tau))
            beta = (tau - 1.0) / tau_next
            tau = tau_next
        k_since += 1
        z = x + beta * (x - x_prev)
        h = (1.0 + beta) * g - beta * g_prev
        x_new = np.zeros(K)
        x_new[act] = soft_threshold(z[act] + h[act] / L, lam / L)
        # ---- dynamic screening with the stable sphere of the rule (Table I)
        if rule == "dst":
            mu = sphere_test(aty / lam, R_test, atom_norm)     # centre y/lambda, a^T y given
        else:
            c_norm = abs(s_stable) * z_norm                   # ||theta'_t||_{q*}
            mu = stable_sphere_test(s_stable * g, eps, c_norm, R_test, atom_norm)
        if rule == "dome":
            # the GAP dome of theta'_t, intersected with the GAP sphere: the smaller test
            Rd = dynamic_radius(s_stable * rho, y, lam)
            rin2 = max(y_sq - 2.0 * (P + delta), 0.0) / (lam * lam)
            mu = np.minimum(mu, stable_dome_test(aty / lam, s_stable * g, eps * c_norm, Rd, rin2, atom_norm))
        keep = active & (mu >= 1.0 - margin)
        if t % max(1, screen_every) != 0:
            keep = active.copy()
        # ---- look-ahead estimate K_t (Section IV-C)
        if rule == "dst":
            mu_conv = sphere_test(aty / lam, R_test, at_norms[i])
        else:
            mu_conv = sphere_test(s_stable * g, R_test, at_norms[i])
        if rule == "dome":
            mu_conv = np.minimum(mu_conv, stable_dome_test(aty / lam, s_stable * g, 0.0, Rd, rin2, at_norms[i]))
        K_t = int(np.count_nonzero(active & (mu_conv >= 1.0)))
        # a rejection that zeroes a nonzero coefficient of x_t: the next step's gradient
        # by linearity, (1+beta) g_{t+1} - beta g_t, would take g_t at x_t before the
        # zeroing, so the momentum restarts there (beta = 0: the step is exact)
        rejected_nonzero = bool(np.any(x[active & ~keep] != 0.0))
        x_new[~keep] = 0.0
        x[~keep] = 0.0
        if keep_trace:
            trace.append(TraceRow(t=t, stage=i, n_active=int(act.size), n_keep=int(keep.sum()), K_t=K_t,
                                  G_stable=G_stable, G_conv=G_conv, delta=delta, R_stable=float(R_test),
                                  gamma=gamma, x_l1=x_l1, P=P))
        # ---- switching criterion (Algorithm 2)
        i_next = switch_dictionary(i, I, gamma, Gamma, K_t, rc[i], K)
        if i_next != i or rejected_nonzero:
            k_since = 0
            tau = 1.0
        x_prev = x
        x = x_new
        g_prev = g
        active = keep
        i = i_next
    return res
