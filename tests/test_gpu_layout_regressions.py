"""Regression tests for two faults of the panel-ordered products, run on the
fixed code through the C ABI:

* rows whose columns are not sorted: the layout's scatter once assumed each
  row's entries of a panel to be contiguous, leaving slots unwritten;
* more than 4,194,304 rows: the panel kernel's grid once exceeded the 4096
  block partials a reduction slot holds, so the reductions (merit, residuals,
  power method) read across slot boundaries.

Tolerances as in the other parity tests: products 1e-13 relative, iterates
1e-10 relative per vector, power estimates and check-log quantities 1e-9.
"""
import time

import numpy as np
import pytest

import oracle
import qpgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PANEL = -3      # lanes-per-row code of the panel-ordered product


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_02470_amd import load
    load()


def _max_rel(a, b):
    return np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b)))


def _compare_runs(rg, ro, tag):
    assert rg.iters == ro.iters, (tag, rg.iters, ro.iters)
    for name in ("y", "z", "w", "x"):
        e = _max_rel(getattr(rg, name).cpu().numpy(), getattr(ro, name))
        print(f"  {tag} {name}: max rel diff {e:.3e}", flush=True)
        assert e <= 1e-10, (tag, name, e)
    assert rg.check_log.shape == ro.check_log.shape
    np.testing.assert_array_equal(rg.check_log[:, [0, 1, 7]], ro.check_log[:, [0, 1, 7]])
    for col in (2, 3, 4, 5, 6, 8):
        np.testing.assert_allclose(rg.check_log[:, col], ro.check_log[:, col], rtol=1e-9, atol=0.0)


def test_unsorted_columns_default_path_above_half_million_columns():
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    t0 = time.time()
    # 600,000 columns: A and Q gather from 4.8 MB vectors, so the default
    # kernel for both is the panel-ordered product
    base = qpgen.make_random_large(seed=1101, n=600_000, m=300_000)
    qp = qpgen.shuffle_row_entries(base, seed=7)
    for rp, ci in ((qp.a_rowptr, qp.a_col), (qp.q_rowptr, qp.q_col)):
        rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
        down = (np.diff(ci) < 0) & (rows[1:] == rows[:-1])
        assert np.unique(rows[1:][down]).size > len(rp) // 2      # most rows are out of order
    print(f"shuffled random QP n={qp.n} m={qp.m} ({time.time() - t0:.1f} s)", flush=True)
    la, _ = oracle.power(qp, "A", qpgen.power_start(qp.m))
    lq, _ = oracle.power(qp, "Q", qpgen.power_start(qp.n))
    lamA, lamQ = 1.01 * la, 1.01 * lq
    dp = DeviceProblem(qp)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(qp.n)
    y = rng.standard_normal(qp.m)
    A = base.A_scipy()
    import scipy.sparse as sp
    Qs = sp.csr_matrix((base.q_val, base.q_col, base.q_rowptr), shape=(base.n, base.n))
    K = 50
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=10, lambda_A=lamA, lambda_Q=lamQ, log_cap=8)
    print(f"oracle {K} iterations ({time.time() - t0:.1f} s)", flush=True)
    for lanes in (-1, PANEL):          # the default choice, and the panel layout for every matrix
        s = Solver(dp, lambda_A=lamA, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=10, log_cap=8,
                   spmv_lanes=lanes, profile_kernels=1)
        assert _max_rel(s.apply("Q", x).cpu().numpy(), Qs @ x) < 1e-13, lanes
        assert _max_rel(s.apply("A", x).cpu().numpy(), A @ x) < 1e-13, lanes
        assert _max_rel(s.apply("AT", y).cpu().numpy(), A.T @ y) < 1e-13, lanes
        rg = s.solve()
        g = s.kernel_stats()["lanes_per_row"]
        s.close()
        print(f"lanes {lanes}: kernels {g} ({time.time() - t0:.1f} s)", flush=True)
        assert g["A"] == PANEL and g["Q"] == PANEL, g
        _compare_runs(rg, ro, f"lanes {lanes}")


def test_panel_products_above_4096_workgroups_of_rows():
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    t0 = time.time()
    # n = 4.5e6 rows of Q (17,579 row blocks of 256): more than 4096
    # workgroups' worth of row blocks at any row blocks per workgroup <= 4
    qp = qpgen.make_random_large(seed=1102, n=4_500_000, m=40_000)
    print(f"random QP n={qp.n} m={qp.m} nnzQ={qp.q_nnz} ({time.time() - t0:.1f} s)", flush=True)
    sa, sq = qpgen.power_start(qp.m), qpgen.power_start(qp.n)
    dp = DeviceProblem(qp)
    s = Solver(dp, power_start_A=sa, power_start_Q=sq, tol=0.0, max_iter=1, check_every=1, spmv_lanes=PANEL)
    pi = s.power_info()
    s.close()
    la, ita = oracle.power(qp, "A", sa)
    lq, itq = oracle.power(qp, "Q", sq)
    print(f"power: gpu {pi} oracle {la} ({ita} it) {lq} ({itq} it) ({time.time() - t0:.1f} s)", flush=True)
    assert pi["est_A"] == pytest.approx(la, rel=1e-9)
    assert pi["est_Q"] == pytest.approx(lq, rel=1e-9)
    K = 2
    lamA, lamQ = 1.01 * la, 1.01 * lq
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=1, lambda_A=lamA, lambda_Q=lamQ, log_cap=4)
    for lanes in (-1, PANEL):
        s = Solver(dp, lambda_A=lamA, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=1, log_cap=4,
                   spmv_lanes=lanes, profile_kernels=1)
        rg = s.solve()
        g = s.kernel_stats()["lanes_per_row"]
        s.close()
        print(f"lanes {lanes}: kernels {g} ({time.time() - t0:.1f} s)", flush=True)
        assert g["Q"] == PANEL, g
        _compare_runs(rg, ro, f"lanes {lanes}")
