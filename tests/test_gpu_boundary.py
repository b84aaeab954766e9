"""Boundary items of the C ABI on the GPU: the diagnostic ||Q(w - x)||_inf of
the shadow iterate w_Q (Proposition 2.4) reported by hprqp_solve,
hprqp_residuals and hprqp_solve_batch, and the time limit of Section 4.1
forced from the host (a limit of 1e-9 s ends every solve at its first check;
no kernel is made to wait or fail).

||Q(w - x)||_inf is compared with numpy's dense Q @ (w - x) at the returned
point (1e-12 relative to max(1, ||Q x||_inf)); at a point with relative KKT
residual 1e-8 it is small (observed ~1e-6 max(1, ||Q x||_inf) on the small
CCQP; asserted <= 1e-4 of it), since the shadow satisfies Q w* = Q x* at a
solution.
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


def _qwx_ref(Q, w, x):
    return float(np.max(np.abs(Q @ (w - x)), initial=0.0))


@pytest.mark.parametrize("case", ["small_ccqp", "psd_rank2", "precond"])
def test_solve_and_residuals_report_qwx_gap(case):
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    if case == "psd_rank2":
        qp = qpgen.make_tiny(31, n=6, m=2, psd_rank=2)    # w drifts in ker Q, Q w -> Q x
    else:
        qp = qpgen.make_small_ccqp()
    Q = qp.Q_dense()
    s = Solver(DeviceProblem(qp), tol=1e-8, max_iter=200_000, precondition=int(case == "precond"))
    r = s.solve()
    assert r.term == "solved"
    w, x = r.w.cpu().numpy(), r.x.cpu().numpy()
    scale = max(1.0, float(np.max(np.abs(Q @ x))))
    ref = _qwx_ref(Q, w, x)
    print(f"{case}: qwx_gap {r.qwx_gap:.3e} (numpy {ref:.3e}), ||w - x|| {np.max(np.abs(w - x)):.3e}", flush=True)
    assert abs(r.qwx_gap - ref) <= 1e-12 * scale
    assert r.qwx_gap <= 1e-4 * scale
    g = s.residuals(r.y, r.z, r.x, w=r.w)
    assert abs(g["qwx_gap"] - ref) <= 1e-12 * scale
    assert g["kkt"] <= 1e-8
    # a point where w and x differ: the number is the product, not a flag
    rng = np.random.default_rng(5)
    w2 = x + rng.standard_normal(qp.n)
    g2 = s.residuals(r.y, r.z, r.x, w=w2)
    ref2 = _qwx_ref(Q, w2, x)
    assert abs(g2["qwx_gap"] - ref2) <= 1e-12 * max(1.0, ref2)
    assert np.isnan(s.residuals(r.y, r.z, r.x)["qwx_gap"])
    s.close()


def test_single_solve_time_limit_at_first_check():
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    qp = qpgen.make_small_ccqp()
    for small_path in (1, 0):            # one-workgroup segments and four launches per iteration
        s = Solver(DeviceProblem(qp), tol=1e-8, max_iter=100_000, check_every=100, time_limit_s=1e-9,
                   small_path=small_path)
        r = s.solve()
        s.close()
        assert r.term == "time_limit" and r.iters == 100, (small_path, r.term, r.iters)
    o = oracle.solve(qp, tol=1e-8, max_iter=100_000, check_every=100, time_limit_s=1e-9)
    assert o.term == "time_limit" and o.iters == 100


def test_batch_qwx_gap_and_time_limit():
    from paper_2507_02470_amd.batch import BatchSolver
    qps = [qpgen.make_portfolio(21_000 + i, n=n) for i, n in enumerate((60, 500, 1000, 1500, 2048))]
    b = BatchSolver(qps, tol=1e-8, max_iter=100_000)
    r = b.solve()
    b.close()
    for i, q in enumerate(qps):
        f = r.infos[i]
        Q = q.Q_dense()
        x = r.x[i]
        scale = max(1.0, float(np.max(np.abs(Q @ x))))
        ref = _qwx_ref(Q, r.w[i], x)
        print(f"n={q.n}: {f['term']} {f['iters']} it, qwx_gap {f['qwx_gap']:.3e} (numpy {ref:.3e})", flush=True)
        assert f["term"] == "solved"
        assert abs(f["qwx_gap"] - ref) <= 1e-12 * scale
        assert f["qwx_gap"] <= 1e-4 * scale
    # the time limit counts from the start of the batched solve: every
    # instance stops at its first check
    b = BatchSolver(qps, tol=1e-8, max_iter=100_000, check_every=100, time_limit_s=1e-9)
    r = b.solve()
    b.close()
    assert [f["term"] for f in r.infos] == ["time_limit"] * len(qps)
    assert [f["iters"] for f in r.infos] == [100] * len(qps)


@pytest.mark.parametrize("n,offset", [(0, 0), (1, 0), (3, 1), (1001, 0), (1001, 1), (1 << 20, 0), ((1 << 20) + 7, 1)])
def test_stream_copy_exact(n, offset):
    """hprqp_stream_copy (the benchmark's counter calibration): an exact copy for
    any length, 16-byte aligned (vector path) or not (offset 1: scalar path);
    nothing written past n; n < 0 rejected."""
    import ctypes as C
    from paper_2507_02470_amd import _native as N
    lib = N.load()
    src = torch.rand(n + offset + 8, dtype=torch.float64, device="cuda")
    dst = torch.full((n + offset + 8,), -1.0, dtype=torch.float64, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ms = C.c_double(-1.0)
    N.check(lib.hprqp_stream_copy(C.c_void_p(src[offset:].data_ptr()), C.c_void_p(dst[offset:].data_ptr()), n, st,
                                  C.byref(ms)))
    torch.cuda.synchronize()
    assert torch.equal(dst[offset:offset + n], src[offset:offset + n])
    assert torch.all(dst[:offset] == -1.0) and torch.all(dst[offset + n:] == -1.0)
    assert ms.value >= 0.0
    assert lib.hprqp_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), -1, st, None) == 1
