"""The two largest workloads of the paper at their published sizes.

* Random Lasso at the first large size of the paper's random Lasso table
  (p = 2e5, q = 5e6; 2e8 nonzeros, 1000 per row of Ahat: the paper does not
  print the density): Q = Ahat^T Ahat matrix-free, so both products gather
  over more than 4,096 workgroups' worth of rows.  The device power method
  lies between the Rayleigh quotient of its start and ||Ahat||_1 ||Ahat||_inf
  (>= lambda_max(Ahat^T Ahat)); two iterations with a check after each, with
  that bound as lambda_Q on both sides, against the oracle (about a minute of
  CPU): iterates 1e-10 relative, check log 1e-9, decisions equal.
* QAP relaxation at d = 2048 (n = 4.2e6) of the paper's large QAP table: the
  device power method against the closed-form spectral radii, and one product
  Q x against the oracle's factored form of the same operator (its plain C
  loops take minutes per product at this size; the factored form is pinned to
  them at small d), within 2 d 2^-53 (|C||X||B|^T + |S||X| + |X||T|^T), the
  summation bound of the GEMMs.
"""
import time

import numpy as np
import pytest
import scipy.sparse as sp

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


def test_lasso_table_size_power_method_and_two_checks_match_oracle():
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    t0 = time.time()
    qp = qpgen.make_lasso_rows(seed=1008, p=200_000, q=5_000_000, per_row=1000)
    p, q = qp.gram_p, qp.n
    Ah = sp.csr_matrix((qp.gram_val, qp.gram_col, qp.gram_rowptr), shape=(p, q))
    absA = abs(Ah)
    lamQ = float(np.asarray(absA.sum(axis=0)).max() * np.asarray(absA.sum(axis=1)).max())
    v = qpgen.power_start(q)
    rq = float(np.linalg.norm(Ah @ v) ** 2 / np.linalg.norm(v) ** 2)
    print(f"lasso p={p} q={q} nnz={Ah.nnz} ({time.time() - t0:.1f} s): bound {lamQ:.4g}, start quotient {rq:.4g}",
          flush=True)
    dp = DeviceProblem(qp)
    s = Solver(dp, power_start_Q=v, tol=0.0, max_iter=1, check_every=1)
    pi = s.power_info()
    s.close()
    print(f"power {pi} ({time.time() - t0:.1f} s)", flush=True)
    assert rq * (1 - 1e-12) <= pi["est_Q"] <= lamQ
    K = 2
    s = Solver(dp, lambda_A=0.0, lambda_Q=lamQ, tol=0.0, max_iter=K, check_every=1, log_cap=4, profile_kernels=1)
    rg = s.solve()
    g = s.kernel_stats()["lanes_per_row"]
    s.close()
    print(f"gpu kernels {g} ({time.time() - t0:.1f} s)", flush=True)
    ro = oracle.solve(qp, tol=0.0, max_iter=K, check_every=1, lambda_A=0.0, lambda_Q=lamQ, log_cap=4)
    print(f"oracle done ({time.time() - t0:.1f} s)", flush=True)
    assert rg.iters == ro.iters == K
    for name in ("y", "z", "w", "x"):
        if name == "y" and qp.m == 0:
            continue
        e = _max_rel(getattr(rg, name).cpu().numpy(), getattr(ro, name))
        print(f"  {name}: max rel diff {e:.3e}", flush=True)
        assert e <= 1e-10, (name, e)
    assert rg.check_log.shape == ro.check_log.shape
    np.testing.assert_array_equal(rg.check_log[:, [0, 1, 7]], ro.check_log[:, [0, 1, 7]])
    for col in (2, 3, 4, 5, 6, 8):
        np.testing.assert_allclose(rg.check_log[:, col], ro.check_log[:, col], rtol=1e-9, atol=0.0)


def test_qap_d2048_power_method_and_operator():
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    t0 = time.time()
    d = 2048
    qp = qpgen.make_qap(d=d)
    al, be, sv, tv = qp.meta["alpha"], qp.meta["beta"], qp.meta["s"], qp.meta["t"]
    lamA = 2.0 * d                                          # A A^T of the assignment constraints
    lamQ = 2.0 * (np.outer(al, be) - sv[:, None] - tv[None, :]).max()
    print(f"qap d={d} ({time.time() - t0:.1f} s)", flush=True)
    dp = DeviceProblem(qp)
    s = Solver(dp, power_start_A=qpgen.power_start(qp.m), power_start_Q=qpgen.power_start(qp.n), tol=0.0,
               max_iter=1)
    pi = s.power_info()
    print(f"power {pi}, closed forms {lamA} {lamQ} ({time.time() - t0:.1f} s)", flush=True)
    assert pi["est_A"] == pytest.approx(lamA, rel=1e-5)
    assert 0.9 * lamQ <= pi["est_Q"] <= lamQ * (1 + 1e-9)
    x = np.random.default_rng(5).standard_normal(qp.n)
    got = s.apply("Q", x).cpu().numpy()
    s.close()
    ref = oracle.apply_Q_kron_factored(qp, x)
    X = np.abs(x.reshape(d, d).T)
    B, Cm, S, T = (np.abs(np.asarray(a)) for a in (qp.kron_B, qp.kron_C, qp.kron_S, qp.kron_T))
    bound = 2 * d * 2.0 ** -53 * (Cm @ X @ B.T + S @ X + X @ T.T)
    err = np.abs(got - ref).reshape(d, d).T
    print(f"operator: max err / bound {float((err / bound).max()):.3g}, max rel {_max_rel(got, ref):.3g} "
          f"({time.time() - t0:.1f} s)", flush=True)
    assert np.all(err <= bound)
