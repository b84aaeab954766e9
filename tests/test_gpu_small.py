"""The one-workgroup segment path for small explicit-Q problems
(small_path = 1): each check segment of Algorithm 4 runs as a single
1024-thread workgroup whose phases are the four products with the fused
epilogues.  Compared with the CPU oracle after whole segments (the traced
path would bypass it): outputs (y, z, w, x) within 1e-10 relative, the check
log's restart decisions identical and its scalars within 1e-7 relative (1e-13
absolute for the normalised residuals near convergence); full
solves at 1e-8 KKT with the oracle's objective.
"""
import numpy as np
import pytest

import oracle
import qpgen

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


def _l1(qp, lam):
    qp.L = np.minimum(qp.L, -1.0)
    qp.U = np.maximum(qp.U, 1.0)
    qp.l1_weight = lam
    return qp


@pytest.mark.parametrize("name,make,T,K", [
    ("small_ccqp", lambda: qpgen.make_small_ccqp(), 100, 600),
    ("small_ccqp_T7", lambda: qpgen.make_small_ccqp(), 7, 140),
    ("tiny_m0", lambda: qpgen.make_tiny(4, n=6, m=0), 10, 200),
    ("tiny_zeroQ", lambda: qpgen.make_tiny(5, n=8, m=4, qkind="zero"), 10, 200),
    ("tiny_l1", lambda: _l1(qpgen.make_tiny(6, n=7, m=3, n_eq=1), 0.3), 10, 200),
    ("wide_rows", lambda: qpgen.make_tiny(9, n=1500, m=900, n_eq=300), 50, 300),
])
def test_small_path_segments_match_oracle(name, make, T, K):
    DP, Solver = _S()
    qp = make()
    lamA, lamQ = _lams(qp) if qp.n <= 400 else (0.0, 0.0)
    if qp.n > 400:
        lamA = 1.01 * oracle.power(qp, "A", qpgen.power_start(qp.m))[0]
        lamQ = 1.01 * oracle.power(qp, "Q", qpgen.power_start(qp.n))[0]
    print(f"small path {name}: n={qp.n} m={qp.m} T={T} K={K}", flush=True)
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=T, lambda_A=lamA, lambda_Q=lamQ, log_cap=K)
    s = Solver(DP(qp), lambda_A=lamA, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=T, log_cap=K,
               small_path=1)
    rg = s.solve()
    s.close()
    assert rg.iters == ro.iters == K
    np.testing.assert_array_equal(rg.check_log[:, [0, 1, 7]], ro.check_log[:, [0, 1, 7]])
    # the eta's are normalised by 1 + norms >= 1, so near convergence they carry an
    # absolute rounding of ~1e-15; R~ and sigma at later restarts come from differences
    # u - ubar and ubar - u_a of nearly equal vectors, whose relative rounding grows as
    # they shrink (observed up to 1.1e-8 on the LP after 15 restarts)
    np.testing.assert_allclose(rg.check_log[:, 2:7], ro.check_log[:, 2:7], rtol=1e-7, atol=1e-13)
    for nm in ("y", "z", "w", "x"):
        a = getattr(rg, nm).cpu().numpy()
        if a.size:
            e = _max_rel(a, getattr(ro, nm))
            print(f"  {nm}: {e:.2e}", flush=True)
            assert e <= 1e-10, (nm, e)


@pytest.mark.parametrize("method", [1, 2])
@pytest.mark.parametrize("name,make,T,K", [
    ("small_ccqp", lambda: qpgen.make_small_ccqp(), 100, 400),
    ("tiny_m0", lambda: qpgen.make_tiny(4, n=6, m=0), 10, 120),
    ("tiny_l1", lambda: _l1(qpgen.make_tiny(6, n=7, m=3, n_eq=1), 0.3), 10, 120),
])
def test_small_path_primal_methods_match_oracle(method, name, make, T, K):
    """HPR on the primal reformulations (Algorithms 6 and 7) in one workgroup per
    segment: outputs after whole segments and the check log against the oracle."""
    DP, Solver = _S()
    qp = make()
    lamA, lamQ = _lams(qp)
    print(f"small path primal {name}: method={method} T={T} K={K}", flush=True)
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=T, lambda_A=lamA, lambda_Q=lamQ, log_cap=K,
                      method=method)
    s = Solver(DP(qp), lambda_A=lamA, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=T, log_cap=K,
               small_path=1, method=method)
    rg = s.solve()
    s.close()
    assert rg.iters == ro.iters == K
    np.testing.assert_array_equal(rg.check_log[:, [0, 1, 7]], ro.check_log[:, [0, 1, 7]])
    np.testing.assert_allclose(rg.check_log[:, 2:7], ro.check_log[:, 2:7], rtol=1e-7, atol=1e-13)
    for nm in ("y", "z", "w", "x"):
        a = getattr(rg, nm).cpu().numpy()
        if a.size:
            e = _max_rel(a, getattr(ro, nm))
            print(f"  {nm}: {e:.2e}", flush=True)
            assert e <= 1e-10, (nm, e)


@pytest.mark.parametrize("precondition", [False, True])
def test_small_path_full_solve(precondition):
    DP, Solver = _S()
    qp = qpgen.make_small_ccqp()
    if precondition:
        qp = qpgen.rescale(qp, seed=4, decades=1.5)
    sa, sq = qpgen.power_start(qp.m), qpgen.power_start(qp.n)
    s = Solver(DP(qp), power_start_A=sa, power_start_Q=sq, tol=1e-8, max_iter=400_000, small_path=1,
               precondition=int(precondition))
    rg = s.solve()
    s.close()
    ro = oracle.solve(qp, tol=1e-8, max_iter=400_000, power_start_A=sa, power_start_Q=sq,
                      precondition=precondition)
    print(f"precondition={precondition}: gpu {rg.term} {rg.iters} {rg.pobj}; oracle {ro.term} {ro.iters} {ro.pobj}",
          flush=True)
    assert rg.term == "solved" and ro.term == "solved" and rg.kkt <= 1e-8
    assert abs(rg.pobj - ro.pobj) <= 1e-6 * max(1.0, abs(ro.pobj))
    res = oracle.residuals(qp, rg.y.cpu().numpy(), rg.z.cpu().numpy(), rg.x.cpu().numpy())
    assert res["kkt"] <= 1.5e-8


def test_small_path_options():
    from paper_2507_02470_amd._native import HPRQPError
    DP, Solver = _S()
    with pytest.raises(HPRQPError):
        Solver(DP(qpgen.make_kron(seed=1, d=5)), lambda_A=1.0, lambda_Q=1.0, small_path=1)
    with pytest.raises(HPRQPError):
        Solver(DP(qpgen.make_small_ccqp()), lambda_A=1.0, lambda_Q=1.0, small_path=2)
    # both paths on one problem: same decisions, iterates within rounding
    qp = qpgen.make_small_ccqp()
    lamA, lamQ = _lams(qp)
    out = []
    for sp in (0, 1):
        s = Solver(DP(qp), lambda_A=lamA, lambda_Q=lamQ, tol=0.0, max_iter=500, check_every=100, log_cap=10,
                   small_path=sp)
        out.append(s.solve())
        s.close()
    np.testing.assert_array_equal(out[0].check_log[:, 7], out[1].check_log[:, 7])
    assert _max_rel(out[1].x.cpu().numpy(), out[0].x.cpu().numpy()) <= 1e-12
