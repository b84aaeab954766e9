"""GPU parity of the single-instance HIP solver against the CPU oracle.

All calls go through the C ABI (libhprqp.so).  Tolerances:
  * operators: 1e-13 relative (FP64 products, different summation order);
  * iterates over the first 50 iterations: ||gpu - oracle||_inf <= 1e-10 max(1, ||oracle||_inf)
    per vector (same lambda's, sigma0 and start on both sides);
  * final solutions: both at max(eta_p, eta_d, eta_gap) <= 1e-8 and objectives
    within 1e-6 relative.
"""
import numpy as np
import pytest
import scipy.sparse as sp

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


def _lams(qp):
    A = qp.A_scipy().toarray()
    lamA = 1.01 * np.linalg.eigvalsh(A @ A.T).max() if qp.m else 0.0
    lamQ = 1.01 * np.linalg.eigvalsh(qp.Q_dense()).max() if qp.qkind != "zero" else 0.0
    return lamA, lamQ


def _max_rel(a, b):
    return np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b)))


# ---------------------------------------------------------------------------
def test_operators_csr_kron_lowrank():
    DP, Solver = _S()
    rng = np.random.default_rng(0)
    cases = [qpgen.make_small_ccqp(seed=11, n=3000, m=1700, nb=400, density=0.003),
             qpgen.make_kron(seed=4, d=37),                    # ragged 16x16 tiles
             qpgen.make_portfolio(12, n=777)]
    for qp in cases:
        print("operators:", qp.meta.get("workload"), qp.n, qp.m, flush=True)
        x = rng.standard_normal(qp.n); y = rng.standard_normal(qp.m)
        dp = DP(qp)
        # default, CSR-stream, gathering from LDS, panel-ordered, row-split from LDS (1, 4, 64 lanes)
        for lanes in (-1, 0, -2, -3, -101, -104, -164):
            s = Solver(dp, lambda_A=1.0, lambda_Q=1.0, spmv_lanes=lanes)
            Qd = qp.Q_dense() if qp.n <= 4000 else None
            ref_q = Qd @ x
            got = s.apply("Q", x).cpu().numpy()
            assert _max_rel(got, ref_q) < 1e-13, lanes
            A = qp.A_scipy()
            assert _max_rel(s.apply("A", x).cpu().numpy(), A @ x) < 1e-13, lanes
            assert _max_rel(s.apply("AT", y).cpu().numpy(), A.T @ y) < 1e-13, lanes
            s.close()


def test_operators_large_csr_all_lane_groups():
    """Rows from 0 to 300 nonzeros, several tiles and a ragged tail, every lanes-per-row choice."""
    DP, Solver = _S()
    rng = np.random.default_rng(1)
    n = 70_001
    lens = rng.choice([0, 1, 3, 7, 30, 300], size=n, p=[0.05, 0.2, 0.3, 0.3, 0.14, 0.01])
    rows = np.repeat(np.arange(n), lens)
    cols = rng.integers(0, n, size=rows.size)
    Q = sp.csr_matrix((rng.standard_normal(rows.size), (rows, cols)), shape=(n, n))
    Q = (Q + Q.T).tocsr()
    qp = qpgen.QP(n=n, m=0, qkind="csr", c=np.zeros(n), L=-np.ones(n), U=np.ones(n),
                  a_rowptr=np.zeros(1, np.int32), a_col=np.zeros(0, np.int32), a_val=np.zeros(0),
                  l=np.zeros(0), u=np.zeros(0), q_rowptr=Q.indptr.astype(np.int32),
                  q_col=Q.indices.astype(np.int32), q_val=Q.data.astype(np.float64))
    x = rng.standard_normal(n)
    ref = Q @ x
    s = Solver(DP(qp), lambda_Q=1.0, spmv_autotune=1)
    assert _max_rel(s.apply("Q", x).cpu().numpy(), ref) < 1e-13
    s.close()
    dp = DP(qp)
    # (-116: a vector over the LDS limit, so 16 lanes gathering from memory)
    for g in (-3, 0, 1, 2, 4, 8, 16, 32, 64, 128, 256, -116):
        s = Solver(dp, lambda_Q=1.0, spmv_lanes=g)
        assert _max_rel(s.apply("Q", x).cpu().numpy(), ref) < 1e-13, g
        s.close()


def test_long_rows_and_every_kernel_in_the_iteration():
    """A Gram Q with rows of thousands of nonzeros (the Lasso shape) through the
    whole iteration with every SpMV kernel: iterates agree with the oracle."""
    DP, Solver = _S()
    qp = qpgen.make_lasso(seed=5, p=40, q=9000, density=0.3)     # 2700 nonzeros per row of Ahat
    lamQ = 1.01 * oracle.power(qp, "Q", qpgen.power_start(qp.n), maxit=5000, tol=1e-10)[0]
    K = 30
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=10, lambda_Q=lamQ, trace_iters=K)
    to = split_trace(ro.trace, qp.n, qp.m)
    dp = DP(qp)
    for g in (-3, -2, 0, 1, 8, 64, 128, 256, -108, -164):
        s = Solver(dp, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=10, trace_iters=K, spmv_lanes=g)
        rg = s.solve()
        s.close()
        tg = split_trace(rg.trace, qp.n, qp.m)
        for name in ("w", "x", "wbar", "xbar"):
            assert _max_rel(tg[name][K - 1], to[name][K - 1]) <= 1e-10, (g, name)


def test_column_split_product():
    """The column-split product (spmv_lanes = -4): a wide matrix with long rows
    whose columns come in random order, with repeats and an empty row, against
    scipy; then a Lasso whose Ahat is wider than the LDS limit through 30
    iterations against the oracle."""
    DP, Solver = _S()
    rng = np.random.default_rng(7)
    m, n = 300, 60_001
    lens = rng.integers(1500, 2500, size=m)
    lens[5] = 0
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    cols = rng.integers(0, n, size=int(rp[-1])).astype(np.int32)     # unsorted, repeats possible
    vals = rng.standard_normal(cols.size)
    qp = qpgen.QP(n=n, m=m, qkind="zero", c=np.zeros(n), L=-np.ones(n), U=np.ones(n),
                  a_rowptr=rp, a_col=cols, a_val=vals, l=-np.ones(m), u=np.ones(m))
    A = sp.csr_matrix((vals, cols, rp), shape=(m, n))
    x = rng.standard_normal(n)
    s = Solver(DP(qp), lambda_A=1.0, spmv_lanes=-4, small_path=0)
    assert s.kernel_stats()["lanes_per_row"]["A"] == -4
    assert _max_rel(s.apply("A", x).cpu().numpy(), A @ x) < 1e-13
    s.close()
    # sparser rows over a vector beyond the L2: the wide panels (16,384
    # columns, 1024-thread workgroups, two passes of 1,024 rows in each
    # workgroup), chosen by default
    m, n = 2000, 600_003
    lens = rng.integers(100, 200, size=m)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    cols = rng.integers(0, n, size=int(rp[-1])).astype(np.int32)
    vals = rng.standard_normal(cols.size)
    qp = qpgen.QP(n=n, m=m, qkind="zero", c=np.zeros(n), L=-np.ones(n), U=np.ones(n),
                  a_rowptr=rp, a_col=cols, a_val=vals, l=-np.ones(m), u=np.ones(m))
    A = sp.csr_matrix((vals, cols, rp), shape=(m, n))
    x = rng.standard_normal(n)
    s = Solver(DP(qp), lambda_A=1.0, small_path=0)
    assert s.kernel_stats()["lanes_per_row"]["A"] == -4
    assert _max_rel(s.apply("A", x).cpu().numpy(), A @ x) < 1e-13
    s.close()
    # three passes of 1,024 rows per workgroup, the middle one without entries in
    # every panel but the first (its rows' columns all lie in the first 16,384)
    m = 3000
    lens = rng.integers(100, 200, size=m)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    cols = rng.integers(0, n, size=int(rp[-1])).astype(np.int32)
    mid = slice(int(rp[1024]), int(rp[2048]))
    cols[mid] = rng.integers(0, 16_384, size=mid.stop - mid.start)
    vals = rng.standard_normal(cols.size)
    qp = qpgen.QP(n=n, m=m, qkind="zero", c=np.zeros(n), L=-np.ones(n), U=np.ones(n),
                  a_rowptr=rp, a_col=cols, a_val=vals, l=-np.ones(m), u=np.ones(m))
    A = sp.csr_matrix((vals, cols, rp), shape=(m, n))
    s = Solver(DP(qp), lambda_A=1.0, small_path=0)
    assert s.kernel_stats()["lanes_per_row"]["A"] == -4
    assert _max_rel(s.apply("A", x).cpu().numpy(), A @ x) < 1e-13
    s.close()

    # Lasso, narrow panels (6000 nonzeros per row of Ahat) and wide ones (150)
    for qp in (qpgen.make_lasso(seed=9, p=40, q=20_000, density=0.3),
               qpgen.make_lasso_rows(seed=10, p=2_000, q=200_000, per_row=150)):
        lamQ = 1.01 * oracle.power(qp, "Q", qpgen.power_start(qp.n), maxit=5000, tol=1e-10)[0]
        K = 30
        ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=10, lambda_Q=lamQ, trace_iters=K)
        to = split_trace(ro.trace, qp.n, qp.m)
        s = Solver(DP(qp), lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=10, trace_iters=K, spmv_lanes=-4)
        rg = s.solve()
        s.close()
        tg = split_trace(rg.trace, qp.n, qp.m)
        for name in ("w", "x", "wbar", "xbar"):
            assert _max_rel(tg[name][K - 1], to[name][K - 1]) <= 1e-10, (qp.gram_p, name)


def test_column_split_with_more_row_groups_than_partial_slots():
    """A (300,000 x 20,000, 10 per row) and A^T on the column-split layout
    (wide panels): the row sums of A take 4,688 groups of 64 rows, more than a
    reduction slot's 4,096 partials, so the summing kernel walks them in
    grid-stride order.  Ten iterations of an LP with checks every 5 against the
    oracle (the checks reduce through that kernel)."""
    DP, Solver = _S()
    rng = np.random.default_rng(11)
    m, n = 300_000, 20_000
    rows = np.repeat(np.arange(m), 10)
    cols = rng.integers(0, n, size=rows.size)
    A = sp.csr_matrix((rng.standard_normal(rows.size), (rows, cols)), shape=(m, n))
    x0 = rng.uniform(0, 1, n)
    ax = A @ x0
    l = np.where(np.arange(m) % 2 == 0, ax, -np.inf)
    u = ax + rng.uniform(0, 1, m)
    qp = qpgen.QP(n=n, m=m, qkind="zero", c=rng.standard_normal(n), L=np.zeros(n), U=np.full(n, 2.0),
                  a_rowptr=A.indptr.astype(np.int32), a_col=A.indices.astype(np.int32), a_val=A.data.copy(),
                  l=l, u=u)
    lamA = 1.01 * oracle.power(qp, "A", qpgen.power_start(m), maxit=5000, tol=1e-10)[0]
    K = 10
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=5, lambda_A=lamA, lambda_Q=0.0, log_cap=4)
    s = Solver(DP(qp), lambda_A=lamA, lambda_Q=0.0, tol=0.0, max_iter=K, check_every=5, log_cap=4,
               spmv_lanes=-4, small_path=0)
    g = s.kernel_stats()["lanes_per_row"]
    assert g["A"] == -4 and g["AT"] == -4, g
    x = rng.standard_normal(n)
    assert _max_rel(s.apply("A", x).cpu().numpy(), A @ x) < 1e-13
    rg = s.solve()
    s.close()
    np.testing.assert_array_equal(rg.check_log[:, 7], ro.check_log[:, 7])
    np.testing.assert_allclose(rg.check_log[:, 2:6], ro.check_log[:, 2:6], rtol=1e-9, atol=1e-15)
    for name in ("y", "z", "w", "x"):
        assert _max_rel(getattr(rg, name).cpu().numpy(), getattr(ro, name)) <= 1e-10, name


def test_lds_row_split_codes():
    """spmv_lanes = -100 - g selects the row-split kernel gathering from LDS
    (reported back by kernel_stats); other codes below -100 are rejected."""
    from paper_2507_02470_amd._native import HPRQPError
    DP, Solver = _S()
    qp = qpgen.make_small_ccqp(seed=21, n=2500, m=900, nb=300, density=0.004)
    dp = DP(qp)
    for bad in (-103, -228, -100):
        with pytest.raises(HPRQPError):
            Solver(dp, lambda_A=1.0, lambda_Q=1.0, spmv_lanes=bad)
    s = Solver(dp, lambda_A=1.0, lambda_Q=1.0, spmv_lanes=-132, max_iter=10, small_path=0)
    s.solve()
    assert s.kernel_stats()["lanes_per_row"] == dict(A=-132, AT=-132, Q=-132)
    x = np.random.default_rng(2).standard_normal(qp.n)
    assert _max_rel(s.apply("Q", x).cpu().numpy(), qp.Q_dense() @ x) < 1e-13
    s.close()


def test_panel_layout_falls_back_when_a_chunk_is_too_large():
    """A dense 2048 x 2048 Q puts 131,072 nonzeros in each (row block, panel)
    chunk, beyond the layout's 16-bit offsets: spmv_lanes = -3 must keep the
    default kernel for it and still give the right products."""
    DP, Solver = _S()
    rng = np.random.default_rng(3)
    n = 2048
    G = rng.standard_normal((n, 64))
    Qd = G @ G.T / 64
    qp = qpgen.from_dense(Qd, rng.standard_normal(n), -np.ones(n), np.ones(n), np.zeros((0, n)), [], [])
    x = rng.standard_normal(n)
    s = Solver(DP(qp), lambda_Q=1.0, spmv_lanes=-3)
    assert _max_rel(s.apply("Q", x).cpu().numpy(), Qd @ x) < 1e-13
    s.close()


@pytest.mark.parametrize("density", [0.003, 0.01])
def test_panel_ordered_products_in_the_iteration(density):
    """All three CSR matrices (A, A^T, Q) in the panel-ordered layout: the
    traced iterates of 50 iterations with restarts against the oracle.  At
    density 0.01 the rows of Q hold ~120 nonzeros, so each (row block, panel)
    chunk takes several LDS passes (the prefetching Q d product's tail loop)."""
    DP, Solver = _S()
    qp = qpgen.make_small_ccqp(seed=13, n=3000, m=1700, nb=400, density=density)
    print(f"panel iteration: density={density} nnz_Q={len(qp.q_col)}", flush=True)
    lamA = 1.01 * oracle.power(qp, "A", qpgen.power_start(qp.m), maxit=5000, tol=1e-12)[0]
    lamQ = 1.01 * oracle.power(qp, "Q", qpgen.power_start(qp.n), maxit=5000, tol=1e-12)[0]
    K = 50
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=10, lambda_A=lamA, lambda_Q=lamQ, trace_iters=K,
                      log_cap=K)
    s = Solver(DP(qp), lambda_A=lamA, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=10, trace_iters=K,
               log_cap=K, spmv_lanes=-3)
    rg = s.solve()
    s.close()
    np.testing.assert_array_equal(rg.check_log[:, 7], ro.check_log[:, 7])
    to, tg = split_trace(ro.trace, qp.n, qp.m), split_trace(rg.trace, qp.n, qp.m)
    for k in range(K):
        for name in ("y", "w", "x", "ybar", "wbar", "xbar"):
            assert _max_rel(tg[name][k], to[name][k]) <= 1e-10, (k, name)


def test_power_method_matches_oracle():
    DP, Solver = _S()
    for qp in (qpgen.make_small_ccqp(), qpgen.make_kron(seed=5, d=20), qpgen.make_portfolio(3, n=400)):
        sa, sq = qpgen.power_start(qp.m), qpgen.power_start(qp.n)
        s = Solver(DP(qp), power_start_A=sa, power_start_Q=sq)
        pi = s.power_info()
        la, ita = oracle.power(qp, "A", sa)
        lq, itq = oracle.power(qp, "Q", sq)
        print("power:", qp.meta.get("workload"), pi, la, ita, lq, itq, flush=True)
        assert pi["est_A"] == pytest.approx(la, rel=1e-9)
        assert pi["est_Q"] == pytest.approx(lq, rel=1e-9)
        s.close()


# ---------------------------------------------------------------------------
def _iterate_parity(qp, check_every, K=50, sigma0=0.0):
    DP, Solver = _S()
    lamA, lamQ = _lams(qp)
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=check_every, lambda_A=lamA, lambda_Q=lamQ,
                      sigma0=sigma0, trace_iters=K, log_cap=K)
    s = Solver(DP(qp), lambda_A=lamA, lambda_Q=lamQ, sigma0=sigma0, tol=0.0, max_iter=K,
               check_every=check_every, trace_iters=K, log_cap=K)
    rg = s.solve()
    s.close()
    to = split_trace(ro.trace, qp.n, qp.m)
    tg = split_trace(rg.trace, qp.n, qp.m)
    # same restart decisions
    np.testing.assert_array_equal(rg.check_log[:, 7], ro.check_log[:, 7])
    worst = 0.0
    for k in range(K):
        for name in ("y", "w", "x", "ybar", "wbar", "xbar"):
            if to[name].shape[1] == 0:
                continue
            e = _max_rel(tg[name][k], to[name][k])
            worst = max(worst, e)
            assert e <= 1e-10, (k, name, e)
    return worst, rg, ro


@pytest.mark.parametrize("check_every", [100, 10, 1])
def test_iterates_match_oracle_small_ccqp(check_every):
    qp = qpgen.make_small_ccqp()
    worst, rg, ro = _iterate_parity(qp, check_every)
    print(f"small_ccqp T={check_every}: worst rel diff {worst:.2e}, restarts {rg.restarts}", flush=True)


@pytest.mark.parametrize("make", [
    lambda: qpgen.make_kron(seed=6, d=21),
    lambda: qpgen.make_portfolio(7, n=333),
    lambda: qpgen.make_tiny(3, n=5, m=3, n_eq=1),
    lambda: qpgen.make_tiny(4, n=6, m=0),
    lambda: qpgen.make_tiny(5, n=8, m=4, qkind="zero"),
])
def test_iterates_match_oracle_other_kinds(make):
    qp = make()
    worst, rg, ro = _iterate_parity(qp, 7)
    print(f"{qp.qkind} n={qp.n} m={qp.m}: worst {worst:.2e}", flush=True)


# ---------------------------------------------------------------------------
def _full_solve(qp, **kw):
    DP, Solver = _S()
    sa, sq = qpgen.power_start(qp.m), qpgen.power_start(qp.n)
    s = Solver(DP(qp), power_start_A=sa, power_start_Q=sq, tol=1e-8, max_iter=kw.pop("max_iter", 400_000), **kw)
    rg = s.solve()
    s.close()
    ro = oracle.solve(qp, tol=1e-8, max_iter=400_000, power_start_A=sa, power_start_Q=sq,
                      check_every=kw.get("check_every", 100))
    return rg, ro


def test_full_solve_small_ccqp():
    qp = qpgen.make_small_ccqp()
    rg, ro = _full_solve(qp)
    print("small_ccqp gpu:", rg.term, rg.iters, rg.kkt, rg.pobj, "oracle:", ro.term, ro.iters, ro.kkt, ro.pobj,
          flush=True)
    assert rg.term == "solved" and ro.term == "solved"
    assert rg.kkt <= 1e-8
    assert abs(rg.pobj - ro.pobj) <= 1e-6 * max(1.0, abs(ro.pobj))
    # independent certificate: the oracle's stopping quantities at the GPU's point
    res = oracle.residuals(qp, rg.y.cpu().numpy(), rg.z.cpu().numpy(), rg.x.cpu().numpy())
    assert res["kkt"] <= 1.5e-8


def test_full_solve_kron_and_portfolio():
    for qp in (qpgen.make_kron(seed=8, d=24), qpgen.make_portfolio(9, n=500)):
        rg, ro = _full_solve(qp)
        print(qp.qkind, "gpu:", rg.term, rg.iters, rg.kkt, "oracle:", ro.term, ro.iters, ro.kkt, flush=True)
        assert rg.term == "solved" and ro.term == "solved"
        assert abs(rg.pobj - ro.pobj) <= 1e-6 * max(1.0, abs(ro.pobj))
        res = oracle.residuals(qp, rg.y.cpu().numpy(), rg.z.cpu().numpy(), rg.x.cpu().numpy())
        assert res["kkt"] <= 1.5e-8


def test_residuals_entry_point_matches_oracle():
    DP, Solver = _S()
    qp = qpgen.make_small_ccqp()
    rng = np.random.default_rng(3)
    y, z, x = rng.standard_normal(qp.m), rng.standard_normal(qp.n), rng.uniform(-10, 10, qp.n)
    s = Solver(DP(qp), lambda_A=10.0, lambda_Q=10.0)
    g = s.residuals(y, z, x)
    o = oracle.residuals(qp, y, z, x)
    s.close()
    for k in ("eta_p", "eta_d", "eta_gap", "pobj", "dobj"):
        if np.isfinite(o[k]):
            assert g[k] == pytest.approx(o[k], rel=1e-12, abs=1e-14), k
        else:
            assert g[k] == o[k]


def test_graph_replay_is_bitwise_identical_and_deterministic():
    DP, Solver = _S()
    qp = qpgen.make_small_ccqp()
    lamA, lamQ = _lams(qp)
    outs = []
    for use_graph in (1, 1, 0):
        s = Solver(DP(qp), lambda_A=lamA, lambda_Q=lamQ, max_iter=700, tol=0.0, use_graph=use_graph)
        r = s.solve()
        outs.append(torch.cat([r.y, r.z, r.w, r.x]).cpu().numpy())
        s.close()
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


def test_invalid_inputs_are_rejected():
    DP, Solver = _S()
    from paper_2507_02470_amd import HPRQPError
    qp = qpgen.make_small_ccqp()
    bad = qp.copy(); bad.l[60] = bad.u[60] + 1.0
    with pytest.raises(HPRQPError, match="ERR_BOUNDS"):
        Solver(DP(bad), lambda_A=1.0, lambda_Q=1.0)
    bad = qp.copy(); bad.c[3] = np.nan
    with pytest.raises(HPRQPError, match="ERR_BOUNDS"):
        Solver(DP(bad), lambda_A=1.0, lambda_Q=1.0)
    bad = qp.copy(); bad.a_col = bad.a_col.copy(); bad.a_col[5] = qp.n + 7
    with pytest.raises(HPRQPError, match="ERR_SHAPE"):
        Solver(DP(bad), lambda_A=1.0, lambda_Q=1.0)


def test_max_iter_and_warm_start():
    DP, Solver = _S()
    qp = qpgen.make_small_ccqp()
    lamA, lamQ = _lams(qp)
    s = Solver(DP(qp), lambda_A=lamA, lambda_Q=lamQ, max_iter=130)
    r = s.solve()
    assert r.term == "max_iter" and r.iters == 130
    # a warm start at a solved point (accurate to ~1e-8, restarting from sigma0)
    # needs far fewer iterations than the cold start
    s2 = Solver(DP(qp), lambda_A=lamA, lambda_Q=lamQ)
    r2 = s2.solve()
    assert r2.term == "solved"
    r3 = s2.solve(y0=r2.y, w0=r2.w, x0=r2.x)
    assert r3.term == "solved" and r3.iters <= r2.iters // 2
    s.close(); s2.close()
