"""hprqp_residuals_noalloc (the entry point for callers that cannot allocate)
against hprqp_residuals of a handle, through the C ABI, on consecutive calls
whose inputs shrink from one call to the next (the library's static
workspace keeps the previous call's contents), for every kind of Q, then its
error paths.  Tolerance: the stopping quantities and objectives 1e-12
relative (A^T y is summed by atomics in the allocation-free path, in a fixed
order in the handle's), ||Q(w - x)||_inf likewise.
"""
import numpy as np
import pytest

import qpgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_02470_amd import load
    load()


def _cases():
    A = np.random.default_rng(9).standard_normal((8, 20))
    lp = qpgen.from_dense(np.zeros((20, 20)), np.random.default_rng(3).uniform(-1, 1, 20), np.zeros(20),
                          np.full(20, 2.0), A, np.full(8, -1.0), np.full(8, 1.0), qkind="zero")
    big = qpgen.make_random_large(seed=77, n=400_000, m=150_000)      # several hundred blocks, ragged tail
    return [("csr_large", big),
            ("csr_ccqp_3000", qpgen.make_small_ccqp(seed=11, n=3000, m=1700, nb=400, density=0.003)),
            ("kron_37", qpgen.make_kron(seed=4, d=37)),
            ("lowrank_777", qpgen.make_portfolio(12, n=777)),
            ("qap_24", qpgen.make_qap(seed=5, d=24)),
            ("gram_lasso", qpgen.make_lasso(seed=6, p=150, q=500)),
            ("csr_ccqp_200", qpgen.make_small_ccqp()),
            ("zero_lp_20", lp)]


def _close(a, b, tol=1e-12):
    if np.isnan(b):
        return np.isnan(a)
    return abs(a - b) <= tol * max(1.0, abs(b))


def test_noalloc_residuals_match_handle_on_shrinking_calls():
    from paper_2507_02470_amd.solver import DeviceProblem, Solver, residuals_noalloc
    prev_n = None
    for name, qp in _cases():
        assert prev_n is None or qp.n < prev_n
        prev_n = qp.n
        dp = DeviceProblem(qp)
        s = Solver(dp, tol=0.0, max_iter=150, check_every=50)
        r = s.solve()                           # an iterate that is not a solution yet
        rng = np.random.default_rng(len(name))
        w = r.w + torch.as_tensor(rng.standard_normal(qp.n) * 1e-3, device=r.w.device)
        for ww in (w, None):
            ref = s.residuals(r.y, r.z, r.x, w=ww)
            got = residuals_noalloc(dp, r.y, r.z, r.x, w=ww)
            print(name, {k: f"{got[k]:.6e}/{ref[k]:.6e}" for k in ("eta_p", "eta_d", "eta_gap", "pobj", "qwx_gap")},
                  flush=True)
            for k in ("eta_p", "eta_d", "eta_gap", "pobj", "dobj", "qwx_gap"):
                assert _close(got[k], ref[k]), (name, k, got[k], ref[k])
        s.close()


def test_noalloc_rejects_bad_input_and_oversized_problems():
    from paper_2507_02470_amd import _native as N
    from paper_2507_02470_amd.solver import DeviceProblem, residuals_noalloc
    qp = qpgen.make_small_ccqp()
    bad = qp.copy()
    bad.a_col = bad.a_col.copy()
    bad.a_col[3] = qp.n + 5                     # a column outside [0, n): found by validation, never read
    z, x, y = np.zeros(qp.n), np.zeros(qp.n), np.zeros(qp.m)
    with pytest.raises(RuntimeError, match="ERR_SHAPE"):
        residuals_noalloc(DeviceProblem(bad), y, z, x)
    bad = qp.copy()
    bad.L = bad.L.copy()
    bad.L[0] = 20.0                             # L > U
    with pytest.raises(RuntimeError, match="ERR_BOUNDS"):
        residuals_noalloc(DeviceProblem(bad), y, z, x)
    # 4.2e6 variables with w: 8 n bytes of vectors beyond the workspace
    n = 4_200_000
    big = qpgen.QP(n=n, m=0, qkind="zero", c=np.zeros(n), L=np.zeros(n), U=np.ones(n),
                   a_rowptr=np.zeros(1, np.int32), a_col=np.zeros(0, np.int32), a_val=np.zeros(0),
                   l=np.zeros(0), u=np.zeros(0))
    dp = DeviceProblem(big)
    v = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="ERR_UNSUPPORTED"):
        residuals_noalloc(dp, None, v, v, w=v)
    got = residuals_noalloc(dp, None, v, v)     # without w it fits
    assert got["eta_p"] == 0.0 and got["eta_d"] == 0.0 and np.isnan(got["qwx_gap"])
