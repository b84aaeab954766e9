"""CPU tests of host-side helpers: the row-built random Lasso generator and
the lambda bounds the benchmark's CPU-baseline legs give the oracle."""
import numpy as np
import pytest
import scipy.sparse as sp

import qpgen


def test_lasso_rows_generator_structure():
    qp = qpgen.make_lasso_rows(seed=3, p=60, q=2000, per_row=40)
    rp, ci, v = qp.gram_rowptr, qp.gram_col, qp.gram_val
    assert rp.dtype == np.int32 and ci.dtype == np.int32 and rp[0] == 0 and rp[-1] == ci.size == v.size
    lens = np.diff(rp)
    assert lens.max() <= 40 and lens.min() >= 30                    # repeats dropped, few of them
    for r in range(qp.gram_p):
        row = ci[rp[r]:rp[r + 1]]
        assert np.all(np.diff(row) > 0) and row.min() >= 0 and row.max() < qp.n   # sorted, distinct, in range
    Ah = sp.csr_matrix((v, ci, rp), shape=(qp.gram_p, qp.n))
    g = -qp.c
    np.testing.assert_allclose(g, Ah.T @ qp.meta["bhat"], rtol=1e-12, atol=1e-12)
    assert qp.l1_weight == pytest.approx(0.2 * np.abs(g).max())
    assert qp.m == 0 and np.all(np.isinf(qp.L)) and np.all(np.isinf(qp.U))


@pytest.mark.parametrize("make", [
    lambda: qpgen.make_small_ccqp(),
    lambda: qpgen.make_kron(seed=4, d=9),
    lambda: qpgen.make_qap(seed=5, d=7),
    lambda: qpgen.make_portfolio(6, n=80),
    lambda: qpgen.make_lasso(seed=7, p=30, q=50, density=0.3),
])
def test_host_lambda_bounds_are_upper_bounds(make):
    import bench
    qp = make()
    lam_A, lam_Q = bench.host_lambdas(qp)
    if qp.m:
        A = qp.A_scipy().toarray()
        assert lam_A >= np.linalg.eigvalsh(A @ A.T).max() * (1 - 1e-12)
    else:
        assert lam_A == 0.0
    assert lam_Q >= np.abs(np.linalg.eigvalsh(qp.Q_dense())).max() * (1 - 1e-12)
