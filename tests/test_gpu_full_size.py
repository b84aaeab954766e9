"""Parity at the full size of the random sparse QP (n = 1,000,000, m = 500,000,
10 nonzeros per row of A, Q = D + S) in the launch configuration the
benchmark times: check segments of 100 iterations replayed from a captured
graph, SpMV kernels picked by the autotuner, all through the C ABI.

The oracle runs the same power methods and the first 100 iterations at this
size (tens of seconds on one core).  Tolerances as in the small-instance
tests: power-method estimates 1e-9 relative (same start, same stopping rule);
the iterate after 100 iterations ||gpu - oracle||_inf <= 1e-10 max(1, ||oracle||_inf)
per vector; the merit, the residuals and sigma of the check 1e-9 relative.
"""
import time

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


def _max_rel(a, b):
    return np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b)))


@pytest.fixture(scope="module")
def large():
    from paper_2507_02470_amd.solver import DeviceProblem
    t0 = time.time()
    qp = qpgen.make_random_large()
    print(f"random_large n={qp.n} m={qp.m} nnzA={qp.a_nnz} nnzQ={qp.q_nnz} ({time.time() - t0:.1f} s)", flush=True)
    return qp, DeviceProblem(qp), {}


def test_random_large_power_method_and_first_segment_match_oracle(large):
    from paper_2507_02470_amd.solver import Solver
    t0 = time.time()
    qp, dp, cache = large
    sa, sq = qpgen.power_start(qp.m), qpgen.power_start(qp.n)

    # power method on the device (as the benchmark runs it) against the oracle's
    s = Solver(dp, power_start_A=sa, power_start_Q=sq, tol=0.0, max_iter=1, check_every=100, spmv_autotune=1)
    pi = s.power_info()
    s.close()
    la, ita = oracle.power(qp, "A", sa)
    lq, itq = oracle.power(qp, "Q", sq)
    print(f"power: gpu {pi} oracle {la} ({ita} it) {lq} ({itq} it) ({time.time() - t0:.1f} s)", flush=True)
    assert pi["est_A"] == pytest.approx(la, rel=1e-9)
    assert pi["est_Q"] == pytest.approx(lq, rel=1e-9)
    cache["lam"] = (la, lq)

    # the first check segment (100 iterations, graph replay) with the same lambda's
    K = 100
    lamA, lamQ = 1.01 * la, 1.01 * lq
    s = Solver(dp, lambda_A=lamA, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=K, spmv_autotune=1,
               log_cap=4)
    rg = s.solve()
    s.close()
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=K, lambda_A=lamA, lambda_Q=lamQ, log_cap=4)
    print(f"iterations: gpu {rg.iters} oracle {ro.iters} ({time.time() - t0:.1f} s)", flush=True)
    assert rg.iters == ro.iters == K
    for name in ("y", "z", "w", "x"):
        e = _max_rel(getattr(rg, name).cpu().numpy(), getattr(ro, name))
        print(f"  {name}: max rel diff {e:.3e}", flush=True)
        assert e <= 1e-10, (name, e)
    # check log: k, t, R, eta_p, eta_d, eta_gap, sigma used, restarted, sigma next
    assert rg.check_log.shape == ro.check_log.shape
    np.testing.assert_array_equal(rg.check_log[:, [0, 1, 7]], ro.check_log[:, [0, 1, 7]])
    for col in (2, 3, 4, 5, 6, 8):
        np.testing.assert_allclose(rg.check_log[:, col], ro.check_log[:, col], rtol=1e-9, atol=0.0)


def test_random_large_first_segment_of_primal_method_matches_oracle(large):
    """HPR on the primal reformulation with A x = s (Algorithm 6) at full size:
    the first check segment of 100 iterations, graph replay, same tolerances."""
    from paper_2507_02470_amd.solver import Solver
    qp, dp, cache = large
    la, lq = cache.get("lam") or (oracle.power(qp, "A", qpgen.power_start(qp.m))[0],
                                  oracle.power(qp, "Q", qpgen.power_start(qp.n))[0])
    K = 100
    lamA, lamQ = 1.01 * la, 1.01 * lq
    t0 = time.time()
    s = Solver(dp, lambda_A=lamA, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=K, spmv_autotune=1,
               log_cap=4, method=1)
    rg = s.solve()
    s.close()
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=K, lambda_A=lamA, lambda_Q=lamQ, log_cap=4, method=1)
    print(f"method 1 iterations: gpu {rg.iters} oracle {ro.iters} ({time.time() - t0:.1f} s)", flush=True)
    assert rg.iters == ro.iters == K
    for name in ("y", "z", "w", "x"):
        e = _max_rel(getattr(rg, name).cpu().numpy(), getattr(ro, name))
        print(f"  {name}: max rel diff {e:.3e}", flush=True)
        assert e <= 1e-10, (name, e)
    np.testing.assert_array_equal(rg.check_log[:, [0, 1, 7]], ro.check_log[:, [0, 1, 7]])
    for col in (2, 3, 4, 5, 6, 8):
        np.testing.assert_allclose(rg.check_log[:, col], ro.check_log[:, col], rtol=1e-9, atol=0.0)
