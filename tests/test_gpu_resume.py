"""Checkpoint and resume of HPR-QP (hprqp_solve_resume) through the C ABI.

A solve cut short by max_iter saves the start of its last epoch (Algorithm 5:
r, u^{r,0}, sigma_r, plus k and the restart-test state of Section 4.1).  Every
quantity of an epoch is a deterministic function of that state, so a solve
resumed from it must repeat the uninterrupted solve bit for bit: the same
iteration count, restarts, check log and output iterates.  The saved scalars
are also checked against the interrupted solve's own check log.
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


def _S():
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    return DeviceProblem, Solver


CASES = {
    # the one-workgroup small path, no preconditioning
    "small_ccqp": (lambda: qpgen.make_small_ccqp(), {}),
    # the multi-kernel path on a preconditioned handle (state in scaled variables)
    "random_precond": (lambda: qpgen.make_random_large(seed=1011, n=20_000, m=10_000), dict(precondition=1)),
    # m = 0 (no y in the state) with the matrix-free Gram Q and phi = lambda ||x||_1
    "lasso_m0": (lambda: qpgen.make_lasso(seed=1012, p=300, q=900), {}),
}


def _same(a, b):
    return torch.equal(a, b)


@pytest.mark.parametrize("case", sorted(CASES))
def test_resume_repeats_the_uninterrupted_solve(case):
    make, kw = CASES[case]
    DP, Solver = _S()
    qp = make()
    dp = DP(qp)
    big = 400_000
    s = Solver(dp, tol=1e-8, max_iter=big, log_cap=20_000, **kw)
    full = s.solve()
    assert full.term == "solved", full.term
    log = full.check_log
    kr = log[log[:, 7] == 1, 0].astype(np.int64)
    assert len(kr) >= 2, f"{case}: needs a few restarts, got {len(kr)}"
    # cut in the middle of an epoch and off the check grid
    K1 = int(kr[len(kr) // 2]) + 37
    assert K1 < full.iters
    s.set_options(max_iter=K1)
    part = s.solve(checkpoint=True)
    assert part.term == "max_iter" and part.iters == K1
    st = part.state
    plog = part.check_log
    prow = plog[plog[:, 7] == 1]
    assert st.k == int(prow[-1, 0]) and st.restarts == int(prow[-1, 9]) == part.restarts
    assert st.sigma == prow[-1, 8] == part.sigma
    assert st.R0ref > 0 and st.alpha3 in (s.opts.alpha3, 0.2)
    assert st.k < K1
    # the cut solve saw exactly the uninterrupted solve's checks before K1,
    # then one check of its own at K1 (off the check grid)
    assert plog[-1, 0] == K1
    np.testing.assert_array_equal(plog[:-1], log[log[:, 0] < K1])

    s.set_options(max_iter=big)
    res = s.solve(resume=st)
    assert res.term == full.term and res.iters == full.iters and res.restarts == full.restarts
    assert res.sigma == full.sigma and res.R_last == full.R_last
    assert (res.eta_p, res.eta_d, res.eta_gap) == (full.eta_p, full.eta_d, full.eta_gap)
    for a, b in ((res.y, full.y), (res.z, full.z), (res.w, full.w), (res.x, full.x)):
        assert _same(a, b)
    # the resumed solve's checks are the uninterrupted solve's checks after the epoch start
    np.testing.assert_array_equal(res.check_log, log[log[:, 0] > st.k])

    # a chain of two interruptions ends in the same place
    K2 = (K1 + full.iters) // 2 + 11
    s.set_options(max_iter=K2)
    mid = s.solve(resume=st, checkpoint=True)
    assert mid.iters == min(K2, full.iters) and mid.state.k >= st.k
    s.set_options(max_iter=big)
    last = s.solve(resume=mid.state, checkpoint=True)
    assert last.iters == full.iters and _same(last.x, full.x) and _same(last.y, full.y)
    # the final save is the start of the last epoch of the whole solve
    assert last.state.k == int(kr[-1]) and last.state.restarts == full.restarts
    s.close()


def test_resume_rejects_bad_states():
    from paper_2507_02470_amd._native import HPRQPError
    DP, Solver = _S()
    qp = qpgen.make_small_ccqp()
    dp = DP(qp)
    s = Solver(dp, tol=0.0, max_iter=300)
    part = s.solve(checkpoint=True)
    st = part.state
    assert part.term == "max_iter" and 0 <= st.k < 300
    done = type(st)(**{**st.__dict__, "k": 300})      # nothing left to run
    with pytest.raises(HPRQPError, match="max_iter"):
        s.solve(resume=done)
    bad = type(st)(**{**st.__dict__, "sigma": -1.0})
    with pytest.raises(HPRQPError, match="sigma"):
        s.solve(resume=bad)
    with pytest.raises(ValueError):
        s.solve(y0=np.zeros(qp.m), resume=st)
    s.close()
    p = Solver(dp, tol=1e-8, max_iter=300, method=1)
    with pytest.raises(HPRQPError, match="method 0"):
        p.solve(checkpoint=True)
    p.close()


def test_resume_after_a_time_limit():
    """A solve stopped by the time limit at its first check, resumed without
    one, ends where the uninterrupted solve ends."""
    DP, Solver = _S()
    qp = qpgen.make_small_ccqp()
    dp = DP(qp)
    s = Solver(dp, tol=1e-8, max_iter=400_000)
    full = s.solve()
    assert full.term == "solved" and full.restarts >= 1
    s.set_options(time_limit_s=1e-9)
    part = s.solve(checkpoint=True)
    assert part.term == "time_limit" and part.iters == 100
    assert part.state.k == 0 and part.state.restarts == 0      # still in the first epoch
    s.set_options(time_limit_s=0.0)
    res = s.solve(resume=part.state)
    assert res.term == full.term and res.iters == full.iters and res.restarts == full.restarts
    for a, b in ((res.y, full.y), (res.z, full.z), (res.w, full.w), (res.x, full.x)):
        assert _same(a, b)
    s.close()
