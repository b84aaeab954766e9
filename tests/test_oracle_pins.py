"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names the passage of arXiv 2507.02470 it relies on.  None of them
needs a GPU.
"""
import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

import oracle
import qpgen
from oracle.oracle import split_trace
from tests import pins


def _dense(qp):
    return qp.Q_dense(), qp.A_scipy().toarray()


# ---------------------------------------------------------------------------
# Linear operators (Section 1: Q may be explicit, Kronecker or structured)
# ---------------------------------------------------------------------------
def test_operators_match_scipy_and_kron():
    rng = np.random.default_rng(7)
    qp = qpgen.make_small_ccqp(seed=3, n=40, m=20, nb=15, density=0.2)
    x = rng.standard_normal(qp.n); y = rng.standard_normal(qp.m)
    Q, A = _dense(qp)
    np.testing.assert_allclose(oracle.apply_Q(qp, x), Q @ x, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(oracle.apply_A(qp, x), A @ x, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(oracle.apply_AT(qp, y), A.T @ y, rtol=1e-13, atol=1e-12)
    # Kronecker: (B kron C) vec(X) = vec(C X B^T) holds for any factors; use
    # unsymmetric ones of different sizes so that a transposed factor shows
    B = rng.standard_normal((5, 5))
    Cm = rng.standard_normal((3, 3))
    kq = qpgen.QP(n=15, m=0, qkind="kron", c=np.zeros(15), L=np.zeros(15), U=np.ones(15),
                  a_rowptr=np.zeros(1, np.int32), a_col=np.zeros(0, np.int32), a_val=np.zeros(0),
                  l=np.zeros(0), u=np.zeros(0), kron_B=B, kron_C=Cm)
    xk = rng.standard_normal(15)
    np.testing.assert_allclose(oracle.apply_Q(kq, xk), np.kron(B, Cm) @ xk, rtol=1e-12, atol=1e-12)
    # diag + low rank
    pq = qpgen.make_portfolio(11, n=60)
    xp = rng.standard_normal(60)
    np.testing.assert_allclose(oracle.apply_Q(pq, xp), pq.Q_dense() @ xp, rtol=1e-12, atol=1e-14)


def test_factored_kronecker_operator_matches_np_kron_and_the_c_oracle():
    """oracle.apply_Q_kron_factored (numpy products, for the d = 2048 QAP
    relaxation): against np.kron of the dense Q = B (x) C - I (x) S - T (x) I
    (Section 4.5) with unsymmetric factors of different sizes, so that a
    transposed factor or a wrong vec order shows, and against the C oracle's
    orc_apply_Q on the QAP relaxation itself."""
    rng = np.random.default_rng(17)
    p, s = 5, 3
    B, Cm = rng.standard_normal((p, p)), rng.standard_normal((s, s))
    S, T = rng.standard_normal((s, s)), rng.standard_normal((p, p))
    for withS, withT in ((False, False), (True, False), (False, True), (True, True)):
        kq = qpgen.QP(n=p * s, m=0, qkind="kron", c=np.zeros(p * s), L=np.zeros(p * s), U=np.ones(p * s),
                      a_rowptr=np.zeros(1, np.int32), a_col=np.zeros(0, np.int32), a_val=np.zeros(0),
                      l=np.zeros(0), u=np.zeros(0), kron_B=B, kron_C=Cm,
                      kron_S=S if withS else None, kron_T=T if withT else None)
        Qd = np.kron(B, Cm) - (np.kron(np.eye(p), S) if withS else 0) - (np.kron(T, np.eye(s)) if withT else 0)
        x = rng.standard_normal(p * s)
        np.testing.assert_allclose(oracle.apply_Q_kron_factored(kq, x), Qd @ x, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(oracle.apply_Q_kron_factored(kq, x), oracle.apply_Q(kq, x), rtol=1e-12,
                                   atol=1e-12)
    for d in (7, 40):
        qp = qpgen.make_qap(seed=50 + d, d=d)
        x = rng.standard_normal(qp.n)
        ref = oracle.apply_Q(qp, x)
        assert np.max(np.abs(oracle.apply_Q_kron_factored(qp, x) - ref)) <= 1e-13 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# Power method (Section 4.1, parameter setting)
# ---------------------------------------------------------------------------
def test_power_method_vs_eigvalsh_and_closed_forms():
    qp = qpgen.make_small_ccqp()
    Q, A = _dense(qp)
    lamA, _ = oracle.power(qp, "A", qpgen.power_start(qp.m))
    lamQ, _ = oracle.power(qp, "Q", qpgen.power_start(qp.n))
    assert lamA == pytest.approx(np.linalg.eigvalsh(A @ A.T).max(), rel=1e-5)
    assert lamQ == pytest.approx(np.linalg.eigvalsh(Q).max(), rel=1e-5)
    # assignment constraints of a d x d matrix: lambda_1(A A^T) = 2d exactly
    kq = qpgen.make_kron(d=12)
    lamAk, _ = oracle.power(kq, "A", qpgen.power_start(kq.m))
    assert lamAk == pytest.approx(24.0, rel=1e-6)
    # lambda_1(B kron C) = lambda_1(B) lambda_1(C)
    lamQk, _ = oracle.power(kq, "Q", qpgen.power_start(kq.n), maxit=20000, tol=1e-10)
    ref = np.linalg.eigvalsh(kq.kron_B).max() * np.linalg.eigvalsh(kq.kron_C).max()
    assert lamQk == pytest.approx(ref, rel=1e-6)


def test_sigma0_rule_hand_example():
    # b = max(|l|,|u|) with infinities read as 0: l=[1,-inf], u=[1,3] -> b=[1,3];
    # c=[3,4,0] -> sigma0 = sqrt(10)/5
    qp = qpgen.from_dense(np.eye(3), [3.0, 4.0, 0.0], -np.ones(3), np.ones(3),
                          [[1, 0, 0], [0, 1, 1]], [1.0, -np.inf], [1.0, 3.0])
    assert oracle.sigma0(qp) == pytest.approx(np.sqrt(10.0) / 5.0, rel=1e-15)
    qp.c[:] = 0.0
    assert oracle.sigma0(qp) == 1.0          # ||c|| outside [1e-16, 1e16] -> 1


# ---------------------------------------------------------------------------
# Metric M ("eq:metric-M") assembled densely vs the theta decomposition
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("psd_rank", [None, 2])
def test_mnorm_matches_dense_metric(psd_rank):
    qp = qpgen.make_tiny(21, n=5, m=3, psd_rank=psd_rank)
    Q, A = _dense(qp)
    lamA = 1.05 * np.linalg.eigvalsh(A @ A.T).max()
    lamQ = 1.02 * np.linalg.eigvalsh(Q).max()
    rng = np.random.default_rng(1)
    for sigma in (0.3, 1.0, 4.0):
        M, V = pins.dense_metric_M(Q, A, sigma, lamA, lamQ)
        ev = np.linalg.eigvalsh(0.5 * (M + M.T))
        assert ev.min() > -1e-9 * ev.max()          # M is PSD
        for _ in range(3):
            dy, dw, dx = rng.standard_normal(3), rng.standard_normal(5), rng.standard_normal(5)
            om = V.T @ dw                              # coordinates of Pi_W(dw)
            vec = np.concatenate([dy, om, dx])
            dense = vec @ M @ vec
            got = oracle.mnorm2(qp, sigma, lamA, lamQ, dy, dw, dx)   # unprojected shadow dw
            assert got == pytest.approx(dense, rel=1e-10, abs=1e-10)


# ---------------------------------------------------------------------------
# Sigma update ("eq:update-sigma-approx", Algorithm 5)
# ---------------------------------------------------------------------------
def test_sigma_argmin():
    # theta_3 = 0: HPR-LP rule sqrt(theta_2/theta_1)
    assert oracle.sigma_argmin(4.0, 9.0, 0.0, 2.0) == pytest.approx(1.5, rel=1e-14)
    rng = np.random.default_rng(5)
    for _ in range(20):
        th1, th2, th3 = 10 ** rng.uniform(-3, 3, 3)
        lamQ = 10 ** rng.uniform(-2, 2)
        # derivative of f by the quotient rule, root by Brent's method
        fp = lambda s: th1 - th2 / s ** 2 + th3 * s * (2 + lamQ * s) / (1 + lamQ * s) ** 2
        ref = so.brentq(fp, 1e-12, 1e12, xtol=1e-300, rtol=1e-15, maxiter=1000)
        got = oracle.sigma_argmin(th1, th2, th3, lamQ)
        assert got == pytest.approx(ref, rel=1e-12)


# ---------------------------------------------------------------------------
# Final optimum: brute-force active sets (tiny), closed forms, LP, KKT solve
# ---------------------------------------------------------------------------
def _solve(qp, **kw):
    Q, A = _dense(qp)
    lamA = 1.01 * np.linalg.eigvalsh(A @ A.T).max() if qp.m else 0.0
    lamQ = 1.01 * np.linalg.eigvalsh(Q).max() if qp.qkind != "zero" else 0.0
    kw.setdefault("lambda_A", lamA)
    kw.setdefault("lambda_Q", lamQ)
    kw.setdefault("max_iter", 200_000)
    kw.setdefault("check_every", 10)
    return oracle.solve(qp, **kw)


@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_active_sets(seed):
    n = 3 + seed % 3
    m = 1 + seed % 3
    qp = qpgen.make_tiny(seed, n=n, m=m, n_eq=seed % 2, psd_rank=(2 if seed % 4 == 3 else None))
    Q, A = _dense(qp)
    best = pins.kkt_enumerate(Q, qp.c, qp.L, qp.U, A, qp.l, qp.u)
    assert best is not None
    r = _solve(qp, tol=1e-10)
    assert r.term == "solved" and r.kkt <= 1e-10
    assert r.pobj == pytest.approx(best[0], rel=1e-7, abs=1e-8)
    if seed % 4 != 3:           # Q positive definite: x* unique
        np.testing.assert_allclose(r.x, best[1], atol=1e-6)


def test_no_constraints_diag_closed_form():
    # Remark 2.1: without Ax in K the method cycles z -> x -> w
    rng = np.random.default_rng(2)
    n = 30
    d = rng.uniform(0.1, 2.0, n); c = rng.standard_normal(n) * 3
    L = -np.ones(n); U = np.ones(n); L[:3] = -np.inf; U[3:6] = np.inf
    qp = qpgen.from_dense(np.diag(d), c, L, U, np.zeros((0, n)), [], [])
    r = _solve(qp, tol=1e-11)
    assert r.term == "solved"
    np.testing.assert_allclose(r.x, pins.diag_box_closed_form(d, c, L, U), atol=1e-9)


def test_diag_budget_bisection():
    rng = np.random.default_rng(4)
    n = 50
    d = rng.uniform(0.01, 0.1, n); c = -rng.normal(0.05, 0.02, n)
    L = np.zeros(n); U = np.full(n, 0.3)
    qp = qpgen.from_dense(np.diag(d), c, L, U, np.ones((1, n)), [1.0], [1.0])
    r = _solve(qp, tol=1e-11)
    xs, nu = pins.diag_budget_bisect(d, c, L, U)
    assert r.term == "solved"
    np.testing.assert_allclose(r.x, xs, atol=1e-8)
    assert r.y[0] == pytest.approx(nu, rel=1e-6)


def test_equality_only_direct_kkt():
    rng = np.random.default_rng(8)
    n, m = 12, 4
    G = rng.standard_normal((n, n)); Q = G @ G.T / n + 0.5 * np.eye(n)
    A = rng.standard_normal((m, n)); b = rng.standard_normal(m); c = rng.standard_normal(n)
    qp = qpgen.from_dense(Q, c, np.full(n, -np.inf), np.full(n, np.inf), A, b, b)
    r = _solve(qp, tol=1e-12)
    xs, ys = pins.equality_kkt(Q, c, A, b)
    np.testing.assert_allclose(r.x, xs, atol=1e-8)
    np.testing.assert_allclose(r.y, ys, atol=1e-7)


def test_lp_reduction_matches_highs():
    # Remark 2.1: Q = 0 and phi = delta_C gives HPR-LP
    rng = np.random.default_rng(9)
    n, m = 20, 8
    A = rng.standard_normal((m, n)); x0 = rng.uniform(0, 1, n)
    b = A @ x0
    l = b.copy(); u = b.copy(); l[4:] = -np.inf; u[4:] = b[4:] + 0.5
    c = rng.uniform(-1, 1, n)
    L = np.zeros(n); U = np.full(n, 2.0)
    qp = qpgen.from_dense(np.zeros((n, n)), c, L, U, A, l, u, qkind="zero")
    r = _solve(qp, tol=1e-10)
    ref = so.linprog(c, A_ub=A[4:], b_ub=u[4:], A_eq=A[:4], b_eq=b[:4], bounds=list(zip(L, U)), method="highs")
    assert ref.status == 0
    assert r.term == "solved"
    assert r.pobj == pytest.approx(ref.fun, rel=1e-7, abs=1e-8)


# ---------------------------------------------------------------------------
# Iteration-level pins
# ---------------------------------------------------------------------------
def test_fixed_point_at_kkt_solution():
    # A KKT point u* = (y*, w* = x*, x*) is a fixed point of Algorithm 3.
    qp = qpgen.make_tiny(30, n=5, m=3, n_eq=1)
    Q, A = _dense(qp)
    obj, xs, ys, zs = pins.kkt_enumerate(Q, qp.c, qp.L, qp.U, A, qp.l, qp.u)
    r = _solve(qp, tol=0.0, max_iter=3, check_every=1000, y0=ys, w0=xs, x0=xs, trace_iters=3)
    tr = split_trace(r.trace, qp.n, qp.m)
    for k in range(3):
        np.testing.assert_allclose(tr["xbar"][k], xs, atol=1e-11)
        np.testing.assert_allclose(tr["ybar"][k], ys, atol=1e-11)
        np.testing.assert_allclose(Q @ tr["wbar"][k], Q @ xs, atol=1e-11)
        np.testing.assert_allclose(tr["x"][k], xs, atol=1e-11)


def test_subproblem_optimality_along_trace():
    """Each step of Algorithm 3 checked from first principles on the trace:
    Step 1/2: xbar = x + sigma(-Qw + A^T y + zbar - c) lies in argmax_{x in C} <-zbar, x>;
    Step 3-1/3-3: Q wbar = Q(sigma lamQ w + xbar + sigma(-Qw + A^T ybar + zbar - c))/(1+sigma lamQ);
    Step 3-2: 0 in d delta*_K(-.)(ybar) + A xbar + sigma A(-Q w_half + A^T ybar + zbar - c) + sigma S_y (ybar - y);
    Step 5: u^{k+1} = u^0/(k+2) + (k+1)/(k+2) (2 ubar - u^k)."""
    qp = qpgen.make_small_ccqp(seed=5, n=30, m=12, nb=10, density=0.25)
    Q, A = _dense(qp)
    lamA = 1.01 * np.linalg.eigvalsh(A @ A.T).max(); lamQ = 1.01 * np.linalg.eigvalsh(Q).max()
    sigma = 0.7
    K = 25
    r = oracle.solve(qp, tol=0.0, max_iter=K, check_every=10 ** 6, lambda_A=lamA, lambda_Q=lamQ,
                     sigma0=sigma, trace_iters=K)
    tr = split_trace(r.trace, qp.n, qp.m)
    y, w, x = np.zeros(qp.m), np.zeros(qp.n), np.zeros(qp.n)
    sQ = sigma * lamQ
    for k in range(K):
        yb, wb, xb = tr["ybar"][k], tr["wbar"][k], tr["xbar"][k]
        zb = (xb - x) / sigma + Q @ w - A.T @ y + qp.c                  # Step 2 solved for zbar
        tol = 1e-9 * (1 + np.abs(xb).max())
        assert np.all(xb >= qp.L - tol) and np.all(xb <= qp.U + tol)
        assert np.all(np.abs(xb[zb > 1e-9] - qp.L[zb > 1e-9]) < 1e-8)
        assert np.all(np.abs(xb[zb < -1e-9] - qp.U[zb < -1e-9]) < 1e-8)
        wh = (sQ * w + xb + sigma * (-Q @ w + A.T @ y + zb - qp.c)) / (1 + sQ)      # Step 3-1
        wt = (sQ * w + xb + sigma * (-Q @ w + A.T @ yb + zb - qp.c)) / (1 + sQ)     # Step 3-3
        np.testing.assert_allclose(Q @ wb, Q @ wt, atol=1e-9 * (1 + np.abs(Q @ wt).max()))
        Sy = lamA * np.eye(qp.m) - A @ A.T
        v = A @ xb + sigma * A @ (-Q @ wh + A.T @ yb + zb - qp.c) + sigma * Sy @ (yb - y)
        # v must be a maximiser of <-ybar, s> over s in K
        tv = 1e-8 * (1 + np.abs(v).max())
        assert np.all(v >= qp.l - tv) and np.all(v <= qp.u + tv)
        pos, neg = yb > 1e-10, yb < -1e-10
        np.testing.assert_allclose(v[pos], qp.l[pos], atol=tv)
        np.testing.assert_allclose(v[neg], qp.u[neg], atol=tv)
        rho = 1.0 / (k + 2)
        yn = rho * 0 + (1 - rho) * (2 * yb - y)
        wn = (1 - rho) * (2 * wb - w)
        xn = (1 - rho) * (2 * xb - x)
        np.testing.assert_allclose(tr["y"][k], yn, atol=1e-10 * (1 + np.abs(yn).max()))
        np.testing.assert_allclose(tr["w"][k], wn, atol=1e-10 * (1 + np.abs(wn).max()))
        np.testing.assert_allclose(tr["x"][k], xn, atol=1e-10 * (1 + np.abs(xn).max()))
        y, w, x = tr["y"][k], tr["w"][k], tr["x"][k]


def test_o_one_over_k_bound_without_restart():
    """Theorem 2.2: ||u^k - ubar^{k+1}||_M <= ||u^0 - u*||_M / (k+1) with a
    fixed sigma and no restart."""
    qp = qpgen.make_tiny(33, n=5, m=3, n_eq=1)
    Q, A = _dense(qp)
    obj, xs, ys, zs = pins.kkt_enumerate(Q, qp.c, qp.L, qp.U, A, qp.l, qp.u)
    lamA = 1.01 * np.linalg.eigvalsh(A @ A.T).max(); lamQ = 1.01 * np.linalg.eigvalsh(Q).max()
    for sigma in (0.2, 1.0, 5.0):
        R0 = np.sqrt(oracle.mnorm2(qp, sigma, lamA, lamQ, -ys, -xs, -xs))
        K = 300
        r = oracle.solve(qp, tol=0.0, max_iter=K, check_every=1, lambda_A=lamA, lambda_Q=lamQ,
                         sigma0=sigma, enable_restart=False, enable_sigma_update=False, log_cap=K)
        k = r.check_log[:, 0]; R = r.check_log[:, 2]
        assert np.all(R <= R0 / k * (1 + 1e-9) + 1e-13)


def test_restart_schedule_with_criterion_three():
    # eq:restart_3 at the first check of epoch 0 always holds (t = k), and the
    # sigma update keeps sigma positive and finite.
    qp = qpgen.make_small_ccqp()
    r = oracle.solve(qp, tol=1e-8, max_iter=2000, check_every=100, log_cap=100,
                     power_start_A=qpgen.power_start(qp.m), power_start_Q=qpgen.power_start(qp.n))
    log = r.check_log
    assert log[0, 0] == 100 and log[0, 7] == 1.0
    assert np.all(np.isfinite(log[:, 8])) and np.all(log[:, 8] > 0)


# ---------------------------------------------------------------------------
# Restart rule (Section 3.2, "eq:restart_1".."eq:restart_3") and the alpha_3
# tightening (Section 4.1, parameter setting): hand-worked cases with the
# paper's alpha = (0.2, 0.8, 0.5)
# ---------------------------------------------------------------------------
A1, A2, A3 = 0.2, 0.8, 0.5
DECAY, STALL, LONG = oracle.oracle.RESTART_DECAY, oracle.oracle.RESTART_STALL, oracle.oracle.RESTART_LONG


def _rt(R, Rr0, Rprev, t, k, a3=A3):
    return oracle.restart_test(R, Rr0, Rprev, t, k, A1, A2, a3)


def test_restart_sufficient_decay_alone_and_at_equality():
    # "eq:restart_1": R~_{r,t+1} <= alpha1 R~_{r,0}.  R = 0.19 < 0.2; the epoch's
    # first check (Rprev < 0), t = 10 < 0.5 * 100
    assert _rt(0.19, 1.0, -1.0, 10, 100) == DECAY
    # equality: 0.2 * 1.25 rounds to exactly 0.25, so R = 0.25 satisfies "<="
    assert 0.2 * 1.25 == 0.25
    assert _rt(0.25, 1.25, 0.3, 10, 100) == DECAY
    # just missing: one ulp above; R < Rprev keeps criterion 2 out
    assert _rt(np.nextafter(0.25, 1.0), 1.25, 0.3, 10, 100) == 0


def test_restart_insufficient_local_progress():
    # "eq:restart_2": R~_{r,t+1} <= alpha2 R~_{r,0} and R~_{r,t+1} > R~_{r,t}
    assert _rt(0.5, 1.0, 0.4, 10, 100) == STALL               # decayed to 0.5 but went up
    assert _rt(0.5, 1.0, 0.6, 10, 100) == 0                   # still going down
    assert _rt(0.5, 1.0, 0.5, 10, 100) == 0                   # equal is not an increase
    assert _rt(np.nextafter(0.5, 1.0), 1.0, 0.5, 10, 100) == STALL
    # first part at equality: 0.8 * 1.25 rounds to exactly 1.0
    assert 0.8 * 1.25 == 1.0
    assert _rt(1.0, 1.25, 0.9, 10, 100) == STALL
    assert _rt(np.nextafter(1.0, 2.0), 1.25, 0.9, 10, 100) == 0
    # an increase above alpha2 R~_{r,0} is not enough
    assert _rt(0.9, 1.0, 0.85, 10, 100) == 0
    # the epoch's first check has no R~_{r,t} to compare with: never criterion 2
    assert _rt(0.5, 1.0, -1.0, 10, 100) == 0
    # at or below alpha1 both hold
    assert _rt(0.1, 1.0, 0.05, 10, 100) == DECAY | STALL


def test_restart_long_inner_loop():
    # "eq:restart_3": t >= alpha3 k (t and k counted after the iteration)
    assert _rt(0.9, 1.0, 0.95, 50, 100) == LONG               # equality
    assert _rt(0.9, 1.0, 0.95, 49, 100) == 0
    assert _rt(0.9, 1.0, 0.95, 100, 100) == LONG              # epoch 0: t = k always holds
    # after the tightening: 0.2 * 100 rounds to exactly 20
    assert 0.2 * 100 == 20.0
    assert _rt(0.9, 1.0, 0.95, 20, 100, a3=0.2) == LONG
    assert _rt(0.9, 1.0, 0.95, 19, 100, a3=0.2) == 0
    assert _rt(0.9, 1.0, 0.95, 49, 100, a3=0.2) == LONG
    # all three at once
    assert _rt(0.1, 1.0, 0.05, 60, 100) == DECAY | STALL | LONG


def test_alpha3_tightening():
    # Section 4.1: alpha3 becomes 0.2 when R~_{r,tau_r-1}/R~_{0,tau_0-1} <= 0.1
    assert oracle.alpha3_next(0.5, 0.1) == 0.2
    assert oracle.alpha3_next(0.5, 0.05) == 0.2
    assert oracle.alpha3_next(0.5, np.nextafter(0.1, 1.0)) == 0.5
    assert oracle.alpha3_next(0.5, 0.5) == 0.5
    # once tightened it stays (reading: the tightening is permanent)
    assert oracle.alpha3_next(0.2, 0.9) == 0.2


def _replay_restarts(qp, check_every, K):
    """Run the oracle with a trace and a check log, recompute R~ of every
    iteration from the traced iterates with the metric M (pinned against the
    dense metric above), and replay every check's decision with the pinned
    restart test: R~_{r,0} from the epoch's first iteration, the previous check
    of the same epoch, t counted from the last restart, R~_{0,tau_0-1} from the
    first restart and alpha3 through its tightening rule."""
    r = oracle.solve(qp, tol=1e-8, max_iter=K, check_every=check_every, log_cap=K, trace_iters=K,
                     power_start_A=qpgen.power_start(qp.m), power_start_Q=qpgen.power_start(qp.n))
    log = r.check_log
    tr = split_trace(r.trace, qp.n, qp.m)
    nit = int(log[-1, 0])
    assert nit <= K
    sig = np.zeros(nit + 1)
    prev = 0
    for row in log:                      # sigma is constant between checks
        sig[prev + 1:int(row[0]) + 1] = row[6]
        prev = int(row[0])
    Rk = np.zeros(nit + 1)
    for k in range(1, nit + 1):
        if k == 1:
            y0, w0, x0 = np.zeros(qp.m), np.zeros(qp.n), np.zeros(qp.n)
        else:
            y0, w0, x0 = tr["y"][k - 2], tr["w"][k - 2], tr["x"][k - 2]
        m2 = oracle.mnorm2(qp, sig[k], r.lambda_A, r.lambda_Q, y0 - tr["ybar"][k - 1],
                           w0 - tr["wbar"][k - 1], x0 - tr["xbar"][k - 1])
        Rk[k] = np.sqrt(max(m2, 0.0))
    kstart, Rprev, a3, R0ref, fired, tightened = 0, -1.0, A3, None, 0, False
    for i, row in enumerate(log):
        k, t, R, restarted = int(row[0]), int(row[1]), row[2], int(row[7])
        assert k % check_every == 0 and t == k - kstart and R == Rk[k]
        mask = _rt(R, Rk[kstart + 1], Rprev, t, k, a3)
        last = i == len(log) - 1
        if not (last and r.term == "solved"):
            assert bool(mask) == bool(restarted), (k, mask, restarted)
        Rprev = R
        if restarted:
            fired |= mask
            if R0ref is None:
                R0ref = R
            a3n = oracle.alpha3_next(a3, R / R0ref)
            tightened |= a3n != a3
            a3, Rprev, kstart = a3n, -1.0, k
            assert int(row[9]) == int(log[i - 1, 9] if i else 0) + 1
    return r, fired, tightened


def test_restart_decisions_replayed_from_trace():
    # every check of a full solve of the small CCQP, with every criterion and
    # the alpha3 tightening exercised along the way
    qp = qpgen.make_small_ccqp()
    r, fired, tightened = _replay_restarts(qp, 3, 2000)
    assert r.term == "solved" and r.restarts >= 10
    assert fired == DECAY | STALL | LONG and tightened


def test_small_ccqp_solution_certificate():
    qp = qpgen.make_small_ccqp()
    r = oracle.solve(qp, tol=1e-8, max_iter=200_000, power_start_A=qpgen.power_start(qp.m),
                     power_start_Q=qpgen.power_start(qp.n))
    assert r.term == "solved"
    Q, A = _dense(qp)
    kkt, P, D = pins.kkt_residual_numpy(Q, qp.c, qp.L, qp.U, A, qp.l, qp.u, r.x, r.y, r.z)
    assert kkt <= 1e-8
    assert r.pobj == pytest.approx(P, rel=1e-12)


def test_residuals_reference_values():
    qp = qpgen.make_tiny(40, n=4, m=2)
    Q, A = _dense(qp)
    rng = np.random.default_rng(0)
    y, z, x = rng.standard_normal(2), rng.standard_normal(4), rng.standard_normal(4)
    # z with a finite bound on each side where nonzero keeps the dual finite
    z[np.isinf(qp.L) & (z > 0)] *= -1
    got = oracle.residuals(qp, y, z, x)
    kkt, P, D = pins.kkt_residual_numpy(Q, qp.c, qp.L, qp.U, A, qp.l, qp.u, x, y, z)
    if np.isfinite(D):
        assert got["kkt"] == pytest.approx(kkt, rel=1e-12)
        assert got["pobj"] == pytest.approx(P, rel=1e-13)


def test_first_sigma_update_from_dense_thetas():
    """Algorithm 5 at the first restart: the smoothing ratio is exactly 1, so
    sigma_1 = exp(e^-1 log sigma_new + (1 - e^-1) log sigma_0), with
    sigma_new the minimiser of f built from the theta's of "eq:theta"
    (anchor u^{0,0} = 0).  The theta's are formed densely here and the
    minimiser found by Brent's method on f'."""
    qp = qpgen.make_small_ccqp(seed=6, n=40, m=16, nb=12, density=0.2)
    Q, A = _dense(qp)
    lamA = 1.01 * np.linalg.eigvalsh(A @ A.T).max(); lamQ = 1.01 * np.linalg.eigvalsh(Q).max()
    T = 20
    r = oracle.solve(qp, tol=0.0, max_iter=2 * T, check_every=T, lambda_A=lamA, lambda_Q=lamQ,
                     trace_iters=T, log_cap=4)
    tr = split_trace(r.trace, qp.n, qp.m)
    assert r.check_log[0, 7] == 1.0              # eq:restart_3 fires (t = k)
    yb, wb, xb = tr["ybar"][T - 1], tr["wbar"][T - 1], tr["xbar"][T - 1]
    th1 = lamA * yb @ yb + lamQ * wb @ Q @ wb - 2 * (Q @ wb) @ (A.T @ yb)
    th2 = xb @ xb
    th3 = (A.T @ yb) @ Q @ (A.T @ yb)
    fp = lambda s: th1 - th2 / s ** 2 + th3 * s * (2 + lamQ * s) / (1 + lamQ * s) ** 2
    snew = so.brentq(fp, 1e-9, 1e9, xtol=1e-300, rtol=1e-15)
    s0 = r.check_log[0, 6]
    beta = np.exp(-1.0)
    assert r.check_log[0, 8] == pytest.approx(np.exp(beta * np.log(snew) + (1 - beta) * np.log(s0)), rel=1e-10)
    # the restarted state is the bar point of the restart iteration
    np.testing.assert_allclose(tr["x"][T - 1], xb, rtol=0, atol=0)


# ---------------------------------------------------------------------------
# Diagonal preconditioning (Section 4.1, "Preconditioning": Ruiz x10, then
# Pock-Chambolle with alpha = 1, Q explicit; termination on the given problem)
# ---------------------------------------------------------------------------
def _scaled_K(qp, D, E):
    """Dense D-E scaled K = [[Q, A^T], [A, 0]] (the matrix the scaling equilibrates)."""
    Q, A = _dense(qp)
    n, m = qp.n, qp.m
    K = np.zeros((n + m, n + m))
    K[:n, :n] = Q
    K[n:, :n] = A
    K[:n, n:] = A.T
    s = np.concatenate([D, E])
    return s[:, None] * K * s[None, :]


def _badly_scaled(qp, seed):
    """The same kind of QP with variables and rows rescaled by 10^U(-2, 2)."""
    rng = np.random.default_rng(seed)
    Q, A = _dense(qp)
    s = 10.0 ** rng.uniform(-2, 2, qp.n)
    r = 10.0 ** rng.uniform(-2, 2, qp.m)
    return qpgen.from_dense(s[:, None] * Q * s[None, :], s * qp.c, qp.L / s, qp.U / s,
                            r[:, None] * A * s[None, :], r * qp.l, r * qp.u)


def test_scaling_closed_forms():
    rng = np.random.default_rng(21)
    n = 20
    # diagonal Q and no rows: one Ruiz pass gives D = q^(-1/2) and the unit
    # diagonal, which later passes and Pock-Chambolle leave unchanged
    q = 10.0 ** rng.uniform(-2, 2, n)
    qp = qpgen.from_dense(np.diag(q), rng.standard_normal(n), -np.ones(n), np.ones(n), np.zeros((0, n)), [], [])
    D, E = oracle.scaling(qp, ruiz_iters=10)
    np.testing.assert_allclose(D, q ** -0.5, rtol=1e-14)
    # Q = 0 and one row alpha 1^T: Ruiz gives D = E = alpha^(-1/2) (all entries 1);
    # Pock-Chambolle then divides E by the square root of the row's 1-norm n
    alpha = 37.0
    qp = qpgen.from_dense(np.zeros((n, n)), rng.standard_normal(n), -np.ones(n), np.ones(n),
                          alpha * np.ones((1, n)), [-1.0], [1.0])
    D, E = oracle.scaling(qp, ruiz_iters=10)
    np.testing.assert_allclose(D, alpha ** -0.5, rtol=1e-14)
    np.testing.assert_allclose(E, alpha ** -0.5 / np.sqrt(n), rtol=1e-14)


def test_ruiz_equilibrates_and_pock_chambolle_bound():
    qp = _badly_scaled(qpgen.make_small_ccqp(), 5)
    # Ruiz's iteration converges to rows of unit inf-norm (Ruiz 2001)
    D, E = oracle.scaling(qp, ruiz_iters=60, pock_chambolle=False)
    K = _scaled_K(qp, D, E)
    rmax = np.abs(K).max(axis=1)
    nz = rmax > 0
    np.testing.assert_allclose(rmax[nz], 1.0, atol=1e-6)
    # Pock-Chambolle with alpha = 1 bounds the scaled operator: ||D K D||_2 <= 1
    # (Pock & Chambolle 2011, Lemma 2), alone and after the Ruiz passes
    for ruiz in (0, 10):
        D, E = oracle.scaling(qp, ruiz_iters=ruiz, pock_chambolle=True)
        assert np.linalg.norm(_scaled_K(qp, D, E), 2) <= 1.0 + 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_preconditioned_solve_bruteforce(seed):
    n = 3 + seed % 3
    m = 1 + seed % 3
    qp = _badly_scaled(qpgen.make_tiny(100 + seed, n=n, m=m, n_eq=seed % 2), seed)
    Q, A = _dense(qp)
    best = pins.kkt_enumerate(Q, qp.c, qp.L, qp.U, A, qp.l, qp.u)
    assert best is not None
    r = oracle.solve(qp, tol=1e-10, max_iter=400_000, check_every=10, precondition=True)
    assert r.term == "solved"
    assert r.pobj == pytest.approx(best[0], rel=1e-7, abs=1e-8)
    xs = np.maximum(np.abs(best[1]), 1.0)
    np.testing.assert_allclose(r.x / xs, best[1] / xs, atol=1e-6)
    # the stopping test was taken on the given problem at the returned point
    res = oracle.residuals(qp, r.y, r.z, r.x)
    assert res["kkt"] <= 1e-10
    for k in ("eta_p", "eta_d", "eta_gap"):
        assert getattr(r, k) == pytest.approx(res[k], rel=1e-9, abs=1e-15)


# ---------------------------------------------------------------------------
# phi(x) = lambda ||x||_1 (+ box) and the matrix-free Gram Q = Ahat^T Ahat:
# the Lasso of Section 4.4 (m = 0: the z -> x -> w cycle of Remark 2.1)
# ---------------------------------------------------------------------------
def test_lasso_subgradient_optimality():
    qp = qpgen.make_lasso()
    r = oracle.solve(qp, tol=1e-10, max_iter=200_000)
    assert r.term == "solved"
    Ah, bh, lam = qp.Ahat_scipy(), qp.meta["bhat"], qp.l1_weight
    g = Ah.T @ (Ah @ r.x - bh)                 # gradient of 1/2||Ahat x - bhat||^2
    on = np.abs(r.x) > 1e-12
    assert on.any() and (~on).any()
    np.testing.assert_allclose(g[on], -lam * np.sign(r.x[on]), atol=1e-8 * lam)
    assert np.abs(g[~on]).max() <= lam * (1 + 1e-8)
    # primal objective of the Lasso itself (constant 1/2||bhat||^2 dropped in the QP)
    f = 0.5 * np.sum((Ah @ r.x - bh) ** 2) + lam * np.abs(r.x).sum()
    assert r.pobj + 0.5 * bh @ bh == pytest.approx(f, rel=1e-12)


def test_lasso_orthonormal_design_closed_form():
    # Ahat with orthonormal columns: Q = I and x* = soft(Ahat^T bhat, lambda)
    rng = np.random.default_rng(8)
    p, q = 60, 25
    Ah = np.linalg.qr(rng.standard_normal((p, q)))[0]
    bh = rng.standard_normal(p) * 3
    g = Ah.T @ bh
    lam = 0.5 * np.abs(g).max()
    qp = qpgen.make_lasso(seed=1, p=4, q=q)    # then replace the data
    rp, ci, vv = (np.asarray(a) for a in (sp.csr_matrix(Ah).indptr, sp.csr_matrix(Ah).indices,
                                          sp.csr_matrix(Ah).data))
    qp.gram_rowptr, qp.gram_col, qp.gram_val, qp.gram_p = rp.astype(np.int32), ci.astype(np.int32), vv, p
    qp.c, qp.l1_weight = -g, lam
    r = oracle.solve(qp, tol=1e-11, max_iter=100_000)
    assert r.term == "solved"
    np.testing.assert_allclose(r.x, np.sign(g) * np.maximum(np.abs(g) - lam, 0.0), atol=1e-9)
    # lambda >= ||Ahat^T bhat||_inf: the solution is 0
    qp.l1_weight = 1.01 * np.abs(g).max()
    r0 = oracle.solve(qp, tol=1e-11, max_iter=100_000)
    assert r0.term == "solved" and np.abs(r0.x).max() <= 1e-9


@pytest.mark.parametrize("seed", range(4))
def test_l1_with_box_and_rows_bruteforce(seed):
    # lambda ||x||_1 + box with rows, against the split QP in (x+, x-) >= 0:
    # min 1/2 (x+ - x-)'Q(x+ - x-) + c'(x+ - x-) + lambda 1'(x+ + x-),
    # L <= x+ - x- <= U and l <= A(x+ - x-) <= u as rows, by active sets
    n, m = 3, 1 + seed % 2
    qp = qpgen.make_tiny(200 + seed, n=n, m=m, n_eq=seed % 2)
    Q, A = _dense(qp)
    lam = 0.7
    qp.l1_weight = lam
    I = np.eye(n)
    Q2 = np.block([[Q, -Q], [-Q, Q]])
    c2 = np.concatenate([qp.c + lam, -qp.c + lam])
    fin = np.isfinite(qp.L) | np.isfinite(qp.U)
    A2 = np.vstack([np.hstack([A, -A]), np.hstack([I, -I])[fin]])
    l2 = np.concatenate([qp.l, qp.L[fin]]); u2 = np.concatenate([qp.u, qp.U[fin]])
    best = pins.kkt_enumerate(Q2, c2, np.zeros(2 * n), np.full(2 * n, np.inf), A2, l2, u2)
    assert best is not None
    r = oracle.solve(qp, tol=1e-10, max_iter=400_000, check_every=10)
    assert r.term == "solved"
    assert r.pobj == pytest.approx(best[0], rel=1e-7, abs=1e-8)
    xb = best[1][:n] - best[1][n:]
    np.testing.assert_allclose(r.x, xb, atol=1e-6)
