"""The QAP relaxation of Section 4.5 (arXiv 2507.02470): the generator's S, T
and the oracle's operator Q = 2(Bhat (x) Ahat - I (x) S - T (x) I).

Pins that do not come from the code under test:
  - (s, t) solves the LP of Section 4.5: checked against scipy's LP solver and
    against the assignment problem it is dual to (scipy's Hungarian method);
  - Qhat is PSD, and on permutation matrices X it equals the QAP objective
    tr(Ahat X Bhat X^T) minus sum(s) + sum(t) (why the CQP is a relaxation);
  - the oracle's matrix-free operator equals the explicit Kronecker matrix;
  - the relaxation's optimum plus sum(s + t) is a lower bound of the QAP
    (brute force over all permutations) reached by the oracle at 1e-9.
"""
import itertools

import numpy as np
import pytest
import scipy.optimize as so

import oracle
import qpgen


def _sym(rng, d, zero_diag=False):
    U = rng.standard_normal((d, d))
    M = U + U.T
    if zero_diag:
        np.fill_diagonal(M, 0.0)
    return M


@pytest.mark.parametrize("seed", range(5))
def test_qap_st_solves_the_lp(seed):
    rng = np.random.default_rng(seed)
    d = 6
    Ah, Bh = _sym(rng, d), _sym(rng, d, True)
    S, T, s, t, al, be = qpgen.qap_st(Ah, Bh)
    assert np.all(np.diff(al) <= 1e-12) and np.all(np.diff(be) >= -1e-12)
    Cst = np.outer(al, be)
    assert np.min(Cst - s[:, None] - t[None, :]) >= -1e-10 * np.abs(Cst).max()
    # max e'(s+t) s.t. s_i + t_j <= alpha_i beta_j  ==  min -e'(s+t)
    G = np.zeros((d * d, 2 * d))
    for i in range(d):
        for j in range(d):
            G[i * d + j, i] = 1.0
            G[i * d + j, d + j] = 1.0
    lp = so.linprog(-np.ones(2 * d), A_ub=G, b_ub=Cst.ravel(), bounds=[(None, None)] * (2 * d), method="highs")
    assert lp.status == 0
    assert s.sum() + t.sum() == pytest.approx(-lp.fun, rel=1e-9, abs=1e-9)
    # S, T share the eigenvectors of Ahat, Bhat
    np.testing.assert_allclose(S @ Ah, Ah @ S, atol=1e-9 * (1 + np.abs(Ah).max() * np.abs(S).max()))
    np.testing.assert_allclose(T @ Bh, Bh @ T, atol=1e-9 * (1 + np.abs(Bh).max() * np.abs(T).max()))


def test_qap_st_value_is_the_assignment_optimum():
    from scipy.optimize import linear_sum_assignment
    rng = np.random.default_rng(11)
    d = 40
    S, T, s, t, al, be = qpgen.qap_st(_sym(rng, d), _sym(rng, d, True))
    cost = np.outer(al, be)
    r, c = linear_sum_assignment(cost)
    assert s.sum() + t.sum() == pytest.approx(cost[r, c].sum(), rel=1e-10)


def test_qhat_psd_and_exact_on_permutations():
    qp = qpgen.make_qap(seed=3, d=6)
    Ah, Bh = qp.meta["Ahat"], qp.meta["Bhat"]
    Qh = 0.5 * qp.Q_dense()
    ev = np.linalg.eigvalsh(0.5 * (Qh + Qh.T))
    assert ev.min() >= -1e-10 * np.abs(ev).max()
    const = qp.meta["s"].sum() + qp.meta["t"].sum()
    rng = np.random.default_rng(0)
    for _ in range(20):
        X = np.eye(6)[rng.permutation(6)]
        x = X.ravel(order="F")
        assert x @ Qh @ x + const == pytest.approx(np.trace(Ah @ X @ Bh @ X.T), rel=1e-10, abs=1e-10)


def test_oracle_applies_the_qap_operator():
    qp = qpgen.make_qap(seed=5, d=7)
    Ah, Bh = qp.meta["Ahat"], qp.meta["Bhat"]
    S, T = 0.5 * qp.kron_S, 0.5 * qp.kron_T
    rng = np.random.default_rng(1)
    for _ in range(3):
        X = rng.standard_normal((7, 7))
        x = X.ravel(order="F")
        want = (2.0 * (Ah @ X @ Bh - S @ X - X @ T)).ravel(order="F")
        got = oracle.apply_Q(qp, x)
        np.testing.assert_allclose(got, want, atol=1e-12 * (1 + np.abs(want).max()))
        np.testing.assert_allclose(got, qp.Q_dense() @ x, atol=1e-12 * (1 + np.abs(want).max()))


def test_qap_relaxation_is_a_lower_bound_reached_by_the_oracle():
    d = 5
    qp = qpgen.make_qap(seed=9, d=d)
    Ah, Bh = qp.meta["Ahat"], qp.meta["Bhat"]
    r = oracle.solve(qp, tol=1e-9, max_iter=400_000)
    assert r.term == "solved"
    X = r.x.reshape(d, d, order="F")
    assert X.min() >= -1e-9
    np.testing.assert_allclose(X.sum(0), 1.0, atol=1e-7)
    np.testing.assert_allclose(X.sum(1), 1.0, atol=1e-7)
    bound = r.pobj + qp.meta["s"].sum() + qp.meta["t"].sum()
    best = min(np.trace(Ah @ P @ Bh @ P.T) for P in (np.eye(d)[list(pm)] for pm in itertools.permutations(range(d))))
    assert bound <= best + 1e-7 * abs(best)
    # KKT certificate written out here (numpy): Q x - A^T y - z = 0, z >= 0 on
    # x >= 0, x_j z_j = 0, so x is optimal; a generic NLP solver started
    # anywhere does not get below it
    Q = qp.Q_dense()
    A = qp.A_scipy().toarray()
    x, y, z = r.x, r.y, r.z
    scale = 1 + np.abs(Q @ x).max()
    assert np.abs(Q @ x - A.T @ y - z).max() <= 1e-7 * scale
    assert z.min() >= -1e-7 * scale and np.abs(x * z).max() <= 1e-7 * scale
    Qh = 0.5 * Q
    res = so.minimize(lambda v: v @ Qh @ v, np.full(d * d, 1.0 / d), jac=lambda v: 2 * Qh @ v,
                      bounds=[(0, None)] * (d * d), constraints=[dict(type="eq", fun=lambda v: A @ v - 1.0,
                                                                      jac=lambda v: A)],
                      method="SLSQP", options=dict(ftol=1e-14, maxiter=1000))
    assert res.fun >= r.pobj - 1e-7 * abs(r.pobj)
