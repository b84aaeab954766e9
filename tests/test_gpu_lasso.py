"""GPU parity of phi = lambda ||x||_1 (+ box) and of the matrix-free Gram
operator Q = Ahat^T Ahat (the Lasso of Section 4.4, m = 0: the z -> x -> w
cycle of Remark 2.1) against the CPU oracle, through the C ABI.

Tolerances as for the CQP tests: operator 1e-13 relative; iterates over the
first 50 iterations 1e-10 of the largest entry; power method 1e-9; final
solutions both at relative KKT <= 1e-8 with objectives within 1e-6.
"""
import numpy as np
import pytest

import oracle
import qpgen
from oracle.oracle import split_trace

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_02470_amd import load
    load()


def _S():
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    return DeviceProblem, Solver


def _max_rel(a, b):
    return np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b)))


def _l1_box_csr():
    qp = qpgen.make_small_ccqp(seed=21, n=250, m=90, nb=40, density=0.05)
    qp.l1_weight = 0.8
    return qp


def _cases():
    return [qpgen.make_lasso(),
            qpgen.make_lasso(seed=77, p=777, q=3001, density=0.02),   # ragged sizes, p < q
            _l1_box_csr()]


def test_gram_operator_and_power_method():
    DP, Solver = _S()
    rng = np.random.default_rng(3)
    for qp in _cases()[:2]:
        s = Solver(DP(qp), power_start_Q=qpgen.power_start(qp.n), max_iter=1)
        x = rng.standard_normal(qp.n)
        Ah = qp.Ahat_scipy()
        assert _max_rel(s.apply("Q", x).cpu().numpy(), Ah.T @ (Ah @ x)) < 1e-13
        lq, _ = oracle.power(qp, "Q", qpgen.power_start(qp.n))
        assert s.power_info()["est_Q"] == pytest.approx(lq, rel=1e-9)
        s.close()


def test_iterates_match_oracle():
    DP, Solver = _S()
    K = 50
    for qp in _cases():
        lamQ = 1.01 * np.linalg.eigvalsh(qp.Q_dense()).max()
        lamA = 1.01 * np.linalg.eigvalsh(qp.A_scipy().toarray() @ qp.A_scipy().toarray().T).max() if qp.m else 0.0
        ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=10, lambda_A=lamA, lambda_Q=lamQ,
                          trace_iters=K, log_cap=K)
        s = Solver(DP(qp), lambda_A=lamA, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=10,
                   trace_iters=K, log_cap=K)
        rg = s.solve()
        s.close()
        np.testing.assert_array_equal(rg.check_log[:, 7], ro.check_log[:, 7])
        for col in (2, 3, 4, 5):
            np.testing.assert_allclose(rg.check_log[:, col], ro.check_log[:, col], rtol=1e-9, atol=1e-15)
        to = split_trace(ro.trace, qp.n, qp.m)
        tg = split_trace(rg.trace, qp.n, qp.m)
        for k in range(K):
            for name in ("y", "w", "x", "ybar", "wbar", "xbar"):
                if to[name].shape[1] == 0:
                    continue
                e = _max_rel(tg[name][k], to[name][k])
                assert e <= 1e-10, (k, name, e)


def test_full_solves_and_lasso_optimality():
    DP, Solver = _S()
    for qp in _cases():
        ro = oracle.solve(qp, tol=1e-8, max_iter=400_000)
        s = Solver(DP(qp), tol=1e-8, max_iter=400_000)
        rg = s.solve()
        s.close()
        assert rg.term == ro.term == "solved"
        assert rg.kkt <= 1e-8
        assert abs(rg.pobj - ro.pobj) <= 1e-6 * max(1.0, abs(ro.pobj))
        if qp.qkind == "gram":
            # subgradient optimality of the Lasso at the GPU's x
            x = rg.x.cpu().numpy()
            Ah, bh, lam = qp.Ahat_scipy(), qp.meta["bhat"], qp.l1_weight
            g = Ah.T @ (Ah @ x - bh)
            on = np.abs(x) > 1e-9 * max(1.0, np.abs(x).max())
            assert np.abs(g[on] + lam * np.sign(x[on])).max() <= 1e-5 * lam
            assert np.abs(g[~on]).max() <= lam * (1 + 1e-6)


def test_benchmark_size_kernels_match_oracle():
    """The benchmark's Lasso (p = 1e4, q = 5e5, 5e7 nonzeros) runs its Ahat x
    product on the column-split layout and Ahat^T t on the row-split kernel
    gathering from LDS by default: the Q operator against the oracle's, then
    three iterations with a check after each against the oracle.  lambda_Q is
    the host bound ||Ahat||_1 ||Ahat||_inf >= lambda_max(Ahat^T Ahat) on both
    sides (the power method would cost the oracle minutes here)."""
    import time
    DP, Solver = _S()
    t0 = time.time()
    qp = qpgen.make_lasso(seed=1006, p=10_000, q=500_000, density=0.01)
    Ah = qp.Ahat_scipy()
    lamQ = float(abs(Ah).sum(axis=0).max() * abs(Ah).sum(axis=1).max())
    print(f"lasso built ({time.time() - t0:.1f} s)", flush=True)
    dp = DP(qp)
    K = 3
    s = Solver(dp, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=1, log_cap=K)
    x = np.random.default_rng(4).standard_normal(qp.n)
    got = s.apply("Q", x).cpu().numpy()
    ref = oracle.apply_Q(qp, x)
    assert _max_rel(got, ref) < 1e-13
    rg = s.solve()
    s.close()
    print(f"gpu done ({time.time() - t0:.1f} s)", flush=True)
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=1, lambda_Q=lamQ, log_cap=K)
    print(f"oracle done ({time.time() - t0:.1f} s)", flush=True)
    np.testing.assert_allclose(rg.check_log[:, 2:6], ro.check_log[:, 2:6], rtol=1e-9, atol=1e-15)
    for name in ("w", "x", "z"):
        assert _max_rel(getattr(rg, name).cpu().numpy(), getattr(ro, name)) <= 1e-10, name


def test_batch_rejects_l1():
    from paper_2507_02470_amd.batch import BatchSolver
    from paper_2507_02470_amd._native import HPRQPError
    qp = qpgen.make_portfolio(3, n=60)
    qp.l1_weight = 0.1
    with pytest.raises(HPRQPError):
        BatchSolver([qp], tol=1e-8, max_iter=1000)
