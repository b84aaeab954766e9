"""Pins of the oracle's HPR on the primal reformulations (Appendix A of
arXiv 2507.02470: Algorithm 6 on "QP-primal-s", Algorithm 7 on
"QP-primal-sv"), the baselines the paper compares HPR-QP with in Table 1.

What fixes them, independently of the oracle's closed forms:
  - every step is the minimiser of the subproblem the algorithm states; the
    tests build that subproblem densely from the augmented Lagrangian and the
    proximal terms S_x, S_v as printed, and check an optimality certificate
    (a box-constrained strictly convex QP, with an l1 term where phi has one);
  - the step is a preconditioned proximal-point step, so in the metric of the
    oracle it must be firmly nonexpansive (a wrong metric or step breaks it);
  - the Halpern iteration's O(1/k) bound on the fixed-point residual;
  - the optimum of tiny QPs by brute-force active sets, and agreement with
    HPR-QP's solution.
"""
import numpy as np
import pytest
import scipy.optimize as so

import oracle
import qpgen
from oracle.oracle import split_trace
from tests import pins


def _dense(qp):
    return qp.Q_dense(), qp.A_scipy().toarray()


def _lams(qp):
    Q, A = _dense(qp)
    lamA = 1.01 * np.linalg.eigvalsh(A @ A.T).max() if qp.m else 0.0
    lamQ = 1.01 * np.linalg.eigvalsh(Q).max() if qp.qkind != "zero" else 0.0
    return lamA, lamQ


def _box_l1_certificate(H, f, L, U, lam, x, tol):
    """x minimises 1/2 x'Hx + f'x + lam ||x||_1 over [L, U] (H PD) iff, per
    coordinate, -g lies in lam d|x_j| + N_[L_j, U_j](x_j), g = (Hx + f)_j."""
    g = H @ x + f
    assert np.all(x >= L - tol) and np.all(x <= U + tol)
    for j in range(len(x)):
        lo, hi = (-lam, lam) if abs(x[j]) <= tol else (lam * np.sign(x[j]),) * 2
        at_L, at_U = abs(x[j] - L[j]) <= tol, abs(x[j] - U[j]) <= tol
        if at_L:
            lo = -np.inf
        if at_U:
            hi = np.inf
        assert lo - tol <= -g[j] <= hi + tol, (j, x[j], g[j], lo, hi)
    return g


def _tiny(seed, l1=0.0):
    qp = qpgen.make_tiny(seed, n=3 + seed % 3, m=1 + seed % 3, n_eq=seed % 2,
                         psd_rank=(2 if seed % 4 == 3 else None))
    if l1:
        qp.L = np.minimum(qp.L, -1.0)
        qp.U = np.maximum(qp.U, 1.0)
        qp.l1_weight = l1
    return qp


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("seed,l1", [(0, 0.0), (1, 0.0), (2, 0.0), (3, 0.0), (5, 0.0), (6, 0.3), (7, 1.5)])
def test_primal_steps_solve_their_subproblems(variant, seed, l1):
    """Steps 1-3 of Algorithms 6/7: each block is the minimiser of L_sigma plus
    the stated proximal term, with the other blocks at their latest values."""
    qp = _tiny(seed, l1)
    Q, A = _dense(qp)
    n, m = qp.n, qp.m
    lamA, lamQ = _lams(qp)
    rng = np.random.default_rng(100 + seed)
    for sigma in (0.3, 2.0):
        x, v, t = rng.normal(size=n), rng.normal(size=n), rng.normal(size=n)
        y = rng.normal(size=m)
        b = oracle.primal_step(qp, variant, sigma, lamA, lamQ, x, y, v, t)
        tol = 1e-9 * (1 + np.abs(x).max() + np.abs(y).max() + np.abs(t).max())
        # s-block: min over s in [l, u] of <s, y> + sigma/2 ||Ax - s||^2
        Ax = A @ x
        gs = _box_l1_certificate(sigma * np.eye(m), y - sigma * Ax, qp.l, qp.u, 0.0, b["s"], tol)
        # Step 2 (2.1): ybar = y + sigma (sbar - Ax)
        np.testing.assert_allclose(b["y"], y + sigma * (b["s"] - Ax), atol=tol * 10)
        if variant == 1:
            # Step 3: min over x in C of L_sigma(x, sbar; ybar) + 1/2 ||x - x^k||^2_{S_x},
            # S_x = lamQ I - Q + sigma (lamA I - A^T A)
            Sx = lamQ * np.eye(n) - Q + sigma * (lamA * np.eye(n) - A.T @ A)
            H = Q + sigma * A.T @ A + Sx
            f = qp.c - A.T @ b["y"] - sigma * A.T @ b["s"] - Sx @ x
        else:
            # Step 1, v-block: min over v of 1/2 v'Qv + <v, t> + sigma/2 ||x - v||^2
            # + 1/2 ||v - v^k||^2_{S_v}, S_v = lamQ I - Q (unconstrained)
            Sv = lamQ * np.eye(n) - Q
            vb = np.linalg.solve(Q + sigma * np.eye(n) + Sv, -(t - sigma * x - Sv @ v))
            np.testing.assert_allclose(b["v"], vb, atol=tol * 10)
            # Step 2.2: tbar = t + sigma (vbar - x)
            np.testing.assert_allclose(b["t"], t + sigma * (vb - x), atol=tol * 10)
            # Step 3 with S_x = sigma (lamA I - A^T A)
            Sx = sigma * (lamA * np.eye(n) - A.T @ A)
            H = sigma * A.T @ A + sigma * np.eye(n) + Sx
            f = qp.c - A.T @ b["y"] - b["t"] - sigma * A.T @ b["s"] - sigma * b["v"] - Sx @ x
        g = _box_l1_certificate(H, f, qp.L, qp.U, l1, b["x"], tol * 100)
        # zbar is the x-step multiplier: the gradient of the smooth part at xbar
        np.testing.assert_allclose(b["z"], g, atol=tol * 100)


def _rand_state(rng, n, m, scale=1.0):
    return dict(x=scale * rng.normal(size=n), v=scale * rng.normal(size=n),
                y=scale * rng.normal(size=m), t=scale * rng.normal(size=n))


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("seed", [0, 1, 3, 4, 6])
def test_primal_step_firmly_nonexpansive_in_its_metric(variant, seed):
    """ubar = (M + T)^{-1} M u for the maximal monotone KKT operator T of the
    reformulation, hence ||ubar - ubar'||_M^2 <= <ubar - ubar', u - u'>_M and
    M is positive semidefinite."""
    qp = _tiny(seed, 0.4 if seed == 6 else 0.0)
    n, m = qp.n, qp.m
    lamA, lamQ = _lams(qp)
    rng = np.random.default_rng(7 + seed)

    def mn2(sigma, d):
        return oracle.primal_mnorm2(qp, variant, sigma, lamA, lamQ, d["x"], d["y"], d["v"], d["t"])

    def bar(sigma, u):
        b = oracle.primal_step(qp, variant, sigma, lamA, lamQ, u["x"], u["y"], u["v"], u["t"])
        out = dict(x=b["x"], y=b["y"], v=b["v"] if variant == 2 else np.zeros(n),
                   t=b["t"] if variant == 2 else np.zeros(n))
        return out

    for sigma in (0.1, 1.0, 7.0):
        for _ in range(40):
            d = _rand_state(rng, n, m)
            if variant == 1:
                d["v"][:] = 0.0; d["t"][:] = 0.0
            assert mn2(sigma, d) >= -1e-12 * (1 + sum(np.dot(a, a) for a in d.values()))
            u1, u2 = _rand_state(rng, n, m, 3.0), _rand_state(rng, n, m, 3.0)
            b1, b2 = bar(sigma, u1), bar(sigma, u2)
            db = {k: b1[k] - b2[k] for k in b1}
            du = {k: (u1[k] - u2[k]) if (variant == 2 or k in ("x", "y")) else np.zeros_like(u1[k]) for k in u1}
            lhs = mn2(sigma, db)
            inner = 0.25 * (mn2(sigma, {k: db[k] + du[k] for k in db}) - mn2(sigma, {k: db[k] - du[k] for k in db}))
            scale = 1e-10 * (1 + mn2(sigma, du))
            assert lhs <= inner + scale, (sigma, lhs, inner)


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("seed", range(8))
def test_primal_methods_reach_bruteforce_optimum(variant, seed):
    qp = _tiny(seed)
    Q, A = _dense(qp)
    best = pins.kkt_enumerate(Q, qp.c, qp.L, qp.U, A, qp.l, qp.u)
    lamA, lamQ = _lams(qp)
    r = oracle.solve(qp, tol=1e-10, max_iter=400_000, check_every=10, lambda_A=lamA, lambda_Q=lamQ,
                     method=variant)
    assert r.term == "solved" and r.kkt <= 1e-10
    assert r.pobj == pytest.approx(best[0], rel=1e-7, abs=1e-8)
    if seed % 4 != 3:
        np.testing.assert_allclose(r.x, best[1], atol=1e-6)


@pytest.mark.parametrize("variant", [1, 2])
def test_primal_halpern_rate_without_restart(variant):
    """Halpern's bound for a nonexpansive map in the metric M (fixed sigma, no
    restart): ||u^k - ubar^{k+1}||_M <= ||u^0 - u*||_M / (k + 1), u* a fixed point."""
    qp = qpgen.make_tiny(33, n=5, m=3, n_eq=1)
    Q, A = _dense(qp)
    obj, xs, ys, zs = pins.kkt_enumerate(Q, qp.c, qp.L, qp.U, A, qp.l, qp.u)
    lamA, lamQ = _lams(qp)
    for sigma in (0.2, 1.0, 5.0):
        # the fixed point of the PR map: (x*, y*) (variant 2 also v* = x*, t* = -Q x*)
        d = dict(x=-xs, y=-ys, v=-xs if variant == 2 else None, t=(Q @ xs) if variant == 2 else None)
        R0 = np.sqrt(oracle.primal_mnorm2(qp, variant, sigma, lamA, lamQ, d["x"], d["y"], d["v"], d["t"]))
        K = 300
        r = oracle.solve(qp, tol=0.0, max_iter=K, check_every=1, lambda_A=lamA, lambda_Q=lamQ, sigma0=sigma,
                         enable_restart=False, enable_sigma_update=False, log_cap=K, method=variant)
        k = r.check_log[:, 0]; R = r.check_log[:, 2]
        assert np.all(R <= R0 / k * (1 + 1e-6) + 1e-12)


@pytest.mark.parametrize("variant", [1, 2])
def test_primal_trace_follows_steps_four_and_five(variant):
    """Steps 4-5: every carried block (x, y and, for Algorithm 7, v) moves to
    1/(k+2) u^0 + (k+1)/(k+2) (2 ubar - u) within an epoch; for Algorithm 6
    the traced bars are the step's output from the traced state."""
    qp = _tiny(4)
    lamA, lamQ = _lams(qp)
    K, sigma = 40, 0.7
    r = oracle.solve(qp, tol=0.0, max_iter=K, check_every=K, lambda_A=lamA, lambda_Q=lamQ, sigma0=sigma,
                     trace_iters=K, method=variant)
    tr = split_trace(r.trace, qp.n, qp.m)
    prev = dict(y=np.zeros(qp.m), w=np.zeros(qp.n), x=np.zeros(qp.n))
    for k in range(K):
        rho = 1.0 / (k + 2)
        for a, b in (("y", "ybar"), ("w", "wbar"), ("x", "xbar")):
            want = rho * 0.0 + (1 - rho) * (2 * tr[b][k] - prev[a])
            np.testing.assert_allclose(tr[a][k], want, atol=1e-12 * (1 + np.abs(want).max()))
        if variant == 1:
            b = oracle.primal_step(qp, 1, sigma, lamA, lamQ, prev["x"], prev["y"])
            np.testing.assert_allclose(tr["xbar"][k], b["x"], atol=1e-12 * (1 + np.abs(b["x"]).max()))
            np.testing.assert_allclose(tr["ybar"][k], b["y"], atol=1e-12 * (1 + np.abs(b["y"]).max()))
        prev = dict(y=tr["y"][k], w=tr["w"][k], x=tr["x"][k])


def test_primal_first_sigma_update_minimises_the_metric_distance():
    """At a restart the new sigma is the minimiser over sigma of
    ||ubar - u^{r,0}||_M^2 (the M of Algorithm 6), smoothed with
    beta = exp(-1) at the first restart (ratio 1)."""
    qp = qpgen.make_small_ccqp()
    lamA, lamQ = _lams(qp)
    K = 400
    r = oracle.solve(qp, tol=0.0, max_iter=K, check_every=10, lambda_A=lamA, lambda_Q=lamQ,
                     trace_iters=K, log_cap=100, method=1)
    log = r.check_log
    first = int(np.flatnonzero(log[:, 7] == 1)[0])
    k, s_used, s_next = int(log[first, 0]), log[first, 6], log[first, 8]
    tr = split_trace(r.trace, qp.n, qp.m)
    dx, dy = tr["xbar"][k - 1], tr["ybar"][k - 1]          # anchor of epoch 0: the origin
    f = lambda ls: oracle.primal_mnorm2(qp, 1, np.exp(ls), lamA, lamQ, dx, dy)
    res = so.minimize_scalar(f, bracket=(np.log(s_used) - 3, np.log(s_used) + 3), tol=1e-12)
    beta = np.exp(-1.0)
    expect = np.exp(beta * res.x + (1 - beta) * np.log(s_used))
    assert s_next == pytest.approx(expect, rel=1e-6)


def test_primal_trace_layout_and_output():
    """Variant 1 has no v: the trace holds x in the w slots and w = xbar."""
    qp = _tiny(2)
    r = oracle.solve(qp, tol=0.0, max_iter=20, check_every=10, trace_iters=20, method=1)
    tr = split_trace(r.trace, qp.n, qp.m)
    np.testing.assert_array_equal(tr["w"], tr["x"])
    np.testing.assert_array_equal(tr["wbar"], tr["xbar"])
    np.testing.assert_array_equal(r.w, r.x)


def test_dual_and_primal_agree_and_dual_needs_fewer_iterations():
    """Table 1's observation on a small CCQP: all three reach the same optimum;
    HPR-QP needs far fewer iterations than HPR on either primal form."""
    qp = qpgen.make_small_ccqp()
    rs = [oracle.solve(qp, tol=1e-8, max_iter=300_000, method=k) for k in (0, 1, 2)]
    assert all(r.term == "solved" for r in rs)
    for r in rs[1:]:
        assert r.pobj == pytest.approx(rs[0].pobj, rel=1e-7)
        assert r.iters > 5 * rs[0].iters
