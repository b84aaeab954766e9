"""GPU parity of the batched persistent solver against the CPU oracle.

Every instance of a batch runs the whole of Algorithm 4 + 5 on the device;
each is compared with an oracle solve of the same instance (same power-method
start: all ones).  Tolerances as for the single-instance path: iterates at
1e-10 relative after 50 iterations (with restarts), objective within 1e-6
relative and max(eta_p, eta_d, eta_gap) <= 1e-8 for full solves.
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


def _B():
    from paper_2507_02470_amd.batch import BatchSolver
    return BatchSolver


def _rel(a, b):
    return np.max(np.abs(a - b), initial=0.0) / max(1.0, np.max(np.abs(b), initial=0.0))


# (n <= 1024 runs on the 256-thread kernel, larger n on the 512-thread one)
SIZES = [50, 63, 64, 65, 511, 512, 513, 1000, 1024, 1025, 1537, 2000, 2048]


def _insts(seed0=20_000):
    return [qpgen.make_portfolio(seed0 + i, n=n) for i, n in enumerate(SIZES)]


@pytest.mark.parametrize("threads", [0, 64, 128, 256, 512])
def test_batch_iterates_match_oracle_after_50(threads):
    """Every size class (n <= 256, 512, 1024, 2048, each with sizes at its
    edges) on every block size that can hold it: batch_threads forces one
    block size on the classes it fits, the others keep the default."""
    BS = _B()
    qps = _insts()
    print("batch sizes:", [q.n for q in qps], "threads", threads, flush=True)
    b = BS(qps, tol=0.0, max_iter=50, check_every=10, batch_threads=threads)
    sh = b.shapes()
    print("shapes:", sh, flush=True)
    want = [threads if threads and 4 * threads >= cmax else (512 if cmax == 2048 else 256)
            for cmax in sh["class_max_n"]]
    assert sh["threads"] == want
    r = b.solve()
    b.close()
    for i, q in enumerate(qps):
        o = oracle.solve(q, tol=0.0, max_iter=50, check_every=10)
        f = r.infos[i]
        assert f["iters"] == o.iters == 50
        assert f["restarts"] == o.restarts, (i, f["restarts"], o.restarts)
        assert f["lambda_A"] == pytest.approx(o.lambda_A, rel=1e-12)
        assert f["lambda_Q"] == pytest.approx(o.lambda_Q, rel=1e-12)
        for name, g, ref in (("y", r.y[i], o.y), ("z", r.z[i], o.z), ("w", r.w[i], o.w), ("x", r.x[i], o.x)):
            e = _rel(g, ref)
            assert e <= 1e-10, (i, q.n, name, e)


def _no_rows(q):
    """The same QP without the constraints l <= Ax <= u (m = 0)."""
    q.m = 0
    q.a_rowptr = np.zeros(1, dtype=np.int32)
    q.a_col = np.zeros(0, dtype=np.int32)
    q.a_val = np.zeros(0)
    q.l = np.zeros(0)
    q.u = np.zeros(0)
    return q


@pytest.mark.parametrize("ranks", [(10, 3, 10), (16, 3, 10, 16)])
def test_batch_ranks_and_instances_without_rows(ranks):
    """Instances of rank below the kernel's (F padded with zero columns), the
    rank-16 kernel (F read from memory at every product) and instances with
    m = 0 in the same batch: iterates after 60 iterations against the oracle."""
    BS = _B()
    ns = [700, 64, 1537, 2000]
    qps = [qpgen.make_portfolio(40_000 + i, n=ns[i], rank=r) for i, r in enumerate(ranks)]
    qps.append(_no_rows(qpgen.make_portfolio(40_100, n=513, rank=ranks[0])))
    qps.append(_no_rows(qpgen.make_portfolio(40_101, n=2048, rank=ranks[-1])))
    print("batch ranks:", [q.lr_F.shape[1] for q in qps], "m:", [q.m for q in qps], flush=True)
    b = BS(qps, tol=0.0, max_iter=60, check_every=20)
    r = b.solve()
    b.close()
    for i, q in enumerate(qps):
        o = oracle.solve(q, tol=0.0, max_iter=60, check_every=20)
        f = r.infos[i]
        assert f["iters"] == o.iters == 60
        assert f["restarts"] == o.restarts, (i, f["restarts"], o.restarts)
        assert f["lambda_Q"] == pytest.approx(o.lambda_Q, rel=1e-12)
        pairs = [("z", r.z[i], o.z), ("w", r.w[i], o.w), ("x", r.x[i], o.x)]
        if q.m:
            pairs.append(("y", r.y[i], o.y))
        for name, g, ref in pairs:
            e = _rel(g, ref)
            assert e <= 1e-10, (i, q.n, q.m, name, e)


def test_batch_autotuned_shapes():
    """The shape autotuner: every class with 8 or more instances has every
    fitting block size timed, the chosen one is among them (or the default),
    and the solve with the tuned shapes matches the oracle."""
    BS = _B()
    sizes = [60 + 7 * i for i in range(12)] + [300 + 15 * i for i in range(10)] + \
            [600 + 37 * i for i in range(10)] + [1100 + 80 * i for i in range(9)]
    qps = [qpgen.make_portfolio(45_000 + i, n=n) for i, n in enumerate(sizes)]
    b = BS(qps, tol=1e-8, max_iter=100_000, spmv_autotune=1)
    sh = b.shapes()
    print("tuned shapes:", sh, flush=True)
    assert sh["instances"] == [12, 10, 10, 9]
    for c, cmax in enumerate(sh["class_max_n"]):
        fit = [t for t in (64, 128, 256, 512) if 4 * t >= cmax]
        assert sorted(t for (cm, t) in sh["timed_us"] if cm == cmax) == fit
        assert sh["threads"][c] in fit
    r = b.solve()
    b.close()
    for i, q in enumerate(qps[::5]):
        f = r.infos[5 * i]
        o = oracle.solve(q, tol=1e-8, max_iter=100_000)
        assert f["term"] == "solved" and o.term == "solved"
        assert abs(f["pobj"] - o.pobj) <= 1e-6 * max(1.0, abs(o.pobj))


def test_batch_full_solves_match_oracle():
    BS = _B()
    qps = [qpgen.make_portfolio(30_000 + i) for i in range(12)]
    b = BS(qps, tol=1e-8, max_iter=500_000)
    r = b.solve()
    b.close()
    print("iters:", r.iters.tolist(), "kernel s:", r.kernel_s, flush=True)
    for i, q in enumerate(qps):
        f = r.infos[i]
        assert f["term"] == "solved" and f["kkt"] <= 1e-8, (i, f)
        o = oracle.solve(q, tol=1e-8, max_iter=500_000)
        assert o.term == "solved"
        assert abs(f["pobj"] - o.pobj) <= 1e-6 * max(1.0, abs(o.pobj))
        res = oracle.residuals(q, r.y[i], r.z[i], r.x[i])
        assert res["kkt"] <= 1.5e-8, (i, res)


def test_batch_permutation_invariance_bitwise():
    BS = _B()
    qps = _insts(40_000)
    perm = np.random.default_rng(0).permutation(len(qps))
    b1 = BS(qps, tol=1e-8, max_iter=3000)
    r1 = b1.solve()
    b2 = BS([qps[p] for p in perm], tol=1e-8, max_iter=3000)
    r2 = b2.solve()
    b1.close(); b2.close()
    for j, p in enumerate(perm):
        for a, c in ((r1.x[p], r2.x[j]), (r1.y[p], r2.y[j]), (r1.w[p], r2.w[j]), (r1.z[p], r2.z[j])):
            assert np.array_equal(a, c)
        assert r1.infos[p]["iters"] == r2.infos[j]["iters"]


def test_batch_priority_order_changes_nothing_but_time():
    """hprqp_batch_set_priority reorders each kernel's queue; every instance's
    result and iteration count stay bit-identical (including non-finite
    priorities, and after restoring the default order)."""
    BS = _B()
    qps = _insts(45_000)
    b = BS(qps, tol=1e-8, max_iter=3000)
    r1 = b.solve()
    rng = np.random.default_rng(1)
    pr = rng.standard_normal(len(qps)).astype(np.float32)
    pr[::5] = np.nan; pr[1] = np.inf; pr[2] = -np.inf
    outs = []
    for p in (torch.as_tensor(pr, device="cuda"), None):
        b.set_priority(p)
        outs.append(b.solve())
    with pytest.raises(ValueError):
        b.set_priority(torch.zeros(len(qps) + 1, device="cuda"))
    b.close()
    for r2 in outs:
        for j in range(len(qps)):
            for a, c in ((r1.x[j], r2.x[j]), (r1.y[j], r2.y[j]), (r1.w[j], r2.w[j]), (r1.z[j], r2.z[j])):
                assert np.array_equal(a, c)
            assert r1.infos[j]["iters"] == r2.infos[j]["iters"]


def test_batch_shared_structure_and_warm_start():
    BS = _B()
    base = qpgen.make_portfolio_family_base()
    samples = [qpgen.portfolio_family_sample(base, 300_000 + j) for j in range(8)]
    b = BS(samples, shared=base, tol=1e-8, max_iter=200_000)
    r = b.solve()
    for j in range(8):
        q = qpgen.family_member(base, 300_000 + j)
        o = oracle.solve(q, tol=1e-8, max_iter=200_000)
        f = r.infos[j]
        assert f["term"] == "solved"
        assert abs(f["pobj"] - o.pobj) <= 1e-6 * max(1.0, abs(o.pobj))
    # warm start from the solution: far fewer iterations
    y0 = np.concatenate(r.y); w0 = np.concatenate(r.w); x0 = np.concatenate(r.x)
    r2 = b.solve(y0=y0, w0=w0, x0=x0)
    b.close()
    assert all(f["term"] == "solved" for f in r2.infos)
    assert r2.iters.mean() < 0.5 * r.iters.mean()


def test_batch_matches_single_instance_solver():
    BS = _B()
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    q = qpgen.make_portfolio(50_001, n=900)
    b = BS([q], tol=1e-8, max_iter=200_000)
    rb = b.solve()
    b.close()
    s = Solver(DeviceProblem(q), power_start_A=np.ones(q.m), power_start_Q=np.ones(q.n), tol=1e-8)
    rs = s.solve()
    s.close()
    assert rs.term == "solved" and rb.infos[0]["term"] == "solved"
    assert rb.infos[0]["lambda_Q"] == pytest.approx(rs.lambda_Q, rel=1e-9)
    assert abs(rb.infos[0]["pobj"] - rs.pobj) <= 1e-6 * max(1.0, abs(rs.pobj))


def test_batch_rejects_bad_input():
    BS = _B()
    from paper_2507_02470_amd import HPRQPError
    qps = _insts(60_000)[:3]
    bad = qps[1].copy(); bad.L[3] = bad.U[3] + 1
    with pytest.raises(HPRQPError, match="ERR_BOUNDS"):
        BS([qps[0], bad, qps[2]])
    big = qpgen.make_portfolio(1, n=2049)
    with pytest.raises(HPRQPError, match="ERR_UNSUPPORTED"):
        BS([big])
