"""GPU parity of the QAP-relaxation operator (Section 4.5 of arXiv
2507.02470): Q = 2(Bhat (x) Ahat - I (x) S - T (x) I) applied as one FP64-MFMA
GEMM (C X) and one three-term GEMM (C X B^T - X T^T - S X), against the CPU
oracle, through the C ABI.

Tolerances: operator 1e-13 relative to max|Q x| (FP64, different summation
order); iterates 1e-10 relative per vector over the traced iterations (same
lambda's, sigma0 and start); full solves at 1e-8 KKT with objectives within
1e-6 relative.  lambda_A = 2d and lambda_Q = 2 max_ij(alpha_i beta_j - s_i - t_j)
are the closed-form spectral radii of A A^T and Q (times 1.01).
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


def _lams(qp):
    d = qp.meta["d"]
    al, be, s, t = qp.meta["alpha"], qp.meta["beta"], qp.meta["s"], qp.meta["t"]
    lamQ = 2.0 * (np.outer(al, be) - s[:, None] - t[None, :]).max()
    return 1.01 * 2.0 * d, 1.01 * lamQ


def _max_rel(a, b):
    return np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("kernel", [0, 1, 2, 4, 8])
@pytest.mark.parametrize("d", [5, 16, 21, 40, 70, 129])
@pytest.mark.parametrize("terms", ["ST", "S", "T", ""])
def test_qap_operator_matches_oracle(d, terms, kernel):
    """Both product kernels (K-split; LDS-tiled with 1, 2, 4 or 8 split-K groups),
    sizes below, at and across the 16- and 64-wide tiles."""
    DP, Solver = _S()
    qp = qpgen.make_qap(seed=100 + d, d=d)
    if "S" not in terms:
        qp.kron_S = None
    if "T" not in terms:
        qp.kron_T = None
    print(f"qap operator d={d} terms={terms} kernel={kernel}", flush=True)
    s = Solver(DP(qp), lambda_A=1.0, lambda_Q=1.0, tol=0.0, max_iter=1, kron_kernel=kernel)
    rng = np.random.default_rng(d)
    for _ in range(3):
        x = rng.standard_normal(qp.n)
        got = s.apply("Q", x).cpu().numpy()
        want = oracle.apply_Q(qp, x)
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)), (d, terms)
    s.close()


@pytest.mark.parametrize("d,check_every,kernel", [(9, 7, -1), (16, 10, -1), (16, 10, 1), (67, 10, 4)])
def test_qap_iterates_match_oracle(d, check_every, kernel):
    DP, Solver = _S()
    qp = qpgen.make_qap(seed=200 + d, d=d)
    lamA, lamQ = _lams(qp)
    K = 50
    print(f"qap iterates d={d} T={check_every} kernel={kernel}", flush=True)
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=check_every, lambda_A=lamA, lambda_Q=lamQ,
                      trace_iters=K, log_cap=K)
    s = Solver(DP(qp), lambda_A=lamA, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=check_every,
               trace_iters=K, log_cap=K, kron_kernel=kernel)
    rg = s.solve()
    s.close()
    np.testing.assert_array_equal(rg.check_log[:, 7], ro.check_log[:, 7])
    to, tg = split_trace(ro.trace, qp.n, qp.m), split_trace(rg.trace, qp.n, qp.m)
    for k in range(K):
        for name in ("y", "w", "x", "ybar", "wbar", "xbar"):
            e = _max_rel(tg[name][k], to[name][k])
            assert e <= 1e-10, (k, name, e)


def test_qap_full_solve_matches_oracle():
    DP, Solver = _S()
    qp = qpgen.make_qap(seed=301, d=12)
    lamA, lamQ = _lams(qp)
    s = Solver(DP(qp), lambda_A=lamA, lambda_Q=lamQ, tol=1e-8, max_iter=400_000)
    rg = s.solve()
    s.close()
    ro = oracle.solve(qp, tol=1e-8, max_iter=400_000, lambda_A=lamA, lambda_Q=lamQ)
    print(f"qap d=12: gpu {rg.term} {rg.iters} {rg.pobj}; oracle {ro.term} {ro.iters} {ro.pobj}", flush=True)
    assert rg.term == "solved" and ro.term == "solved" and rg.kkt <= 1e-8
    assert abs(rg.pobj - ro.pobj) <= 1e-6 * max(1.0, abs(ro.pobj))
    res = oracle.residuals(qp, rg.y.cpu().numpy(), rg.z.cpu().numpy(), rg.x.cpu().numpy())
    assert res["kkt"] <= 1.5e-8


def test_qap_d256_power_method_and_first_segment():
    """The synthetic QAP relaxation at d = 256 (n = 65,536), as the benchmark
    runs it: the device power method against the closed-form spectral radii,
    then one check segment of 20 iterations (graph replay) against the oracle."""
    DP, Solver = _S()
    qp = qpgen.make_qap(d=256)
    lamA, lamQ = _lams(qp)
    dp = DP(qp)
    s = Solver(dp, power_start_A=qpgen.power_start(qp.m), power_start_Q=qpgen.power_start(qp.n), tol=0.0,
               max_iter=1)
    pi = s.power_info()
    s.close()
    print(f"qap d=256 power: {pi}, closed forms {lamA / 1.01} {lamQ / 1.01}", flush=True)
    assert pi["est_A"] == pytest.approx(lamA / 1.01, rel=1e-5)
    assert pi["est_Q"] <= lamQ / 1.01 * (1 + 1e-9) and pi["est_Q"] >= 0.9 * lamQ / 1.01
    K = 20
    s = Solver(dp, lambda_A=lamA, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=K, log_cap=2)
    rg = s.solve()
    s.close()
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=K, lambda_A=lamA, lambda_Q=lamQ, log_cap=2)
    for name in ("y", "z", "w", "x"):
        e = _max_rel(getattr(rg, name).cpu().numpy(), getattr(ro, name))
        print(f"  {name}: {e:.2e}", flush=True)
        assert e <= 1e-10, (name, e)
    np.testing.assert_allclose(rg.check_log[:, 2:7], ro.check_log[:, 2:7], rtol=1e-9)


@pytest.mark.parametrize("kernel", [1, 4])
def test_plain_kronecker_through_the_tiled_kernel(kernel):
    """Q = B (x) C without S, T (the d = 300 workload's operator) on the tiled
    kernel: operator and the first 30 iterates against the oracle."""
    DP, Solver = _S()
    qp = qpgen.make_kron(seed=6, d=33)
    A = qp.A_scipy().toarray()
    lamA = 1.01 * np.linalg.eigvalsh(A @ A.T).max()
    lamQ = 1.01 * np.linalg.eigvalsh(qp.kron_B).max() * np.linalg.eigvalsh(qp.kron_C).max()
    K = 30
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=10, lambda_A=lamA, lambda_Q=lamQ, trace_iters=K)
    s = Solver(DP(qp), lambda_A=lamA, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=10, trace_iters=K,
               kron_kernel=kernel)
    x = np.random.default_rng(2).standard_normal(qp.n)
    q = s.apply("Q", x).cpu().numpy()
    want = oracle.apply_Q(qp, x)
    assert np.max(np.abs(q - want)) <= 1e-13 * np.max(np.abs(want))
    rg = s.solve()
    s.close()
    to, tg = split_trace(ro.trace, qp.n, qp.m), split_trace(rg.trace, qp.n, qp.m)
    for k in range(K):
        for name in ("y", "w", "x", "ybar", "wbar", "xbar"):
            assert _max_rel(tg[name][k], to[name][k]) <= 1e-10, (k, name)


def test_invalid_kron_kernel_is_rejected():
    from paper_2507_02470_amd._native import HPRQPError
    DP, Solver = _S()
    qp = qpgen.make_qap(seed=1, d=6)
    with pytest.raises(HPRQPError):
        Solver(DP(qp), lambda_A=1.0, lambda_Q=1.0, kron_kernel=3)
