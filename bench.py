#!/usr/bin/env python3
"""HPR-QP throughput on one MI355X.

Workload (default): the random sparse QP with n = 1,000,000 variables and
m = 500,000 rows (A: 10 nonzeros per row at uniformly random columns,
Q = D + S with ~5 nonzeros per row, half the rows equalities, box [0, 10]),
FP64, seeded synthetic data.

A "step" is one check segment: `check_every` = 100 iterations of
Algorithm 4 (every product, projection, Halpern update and the merit /
stopping reductions of the check) plus the host's restart / sigma decision.
The timed region is one hprqp_solve call of K segments started from the
origin, inputs already resident in HBM.

Printed: ONE JSON line with iterations/s (value), the roofline of the
dominant kernel (HIP-event durations measured during the timed region),
the time to 1e-8 relative KKT, and the CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
T_CHECK = 100


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(qp) -> dict:
    """Algorithmic bytes per launch of the four per-iteration products.

    CSR data: 12 B per nonzero (8 B value + 4 B column) + 4 B per row pointer;
    the gathered input vector counts once (8 B per entry); every streamed
    vector read or written by the fused epilogue counts 8 B per entry."""
    n, m = qp.n, qp.m
    nzA, nzQ = qp.a_nnz, qp.q_nnz
    return {
        # Q xhat: Q, xhat (gathered), Qw; writes v, q1
        "q_xhat": 12 * nzQ + 4 * (n + 1) + 8 * n + 8 * n + 16 * n,
        # A v: A, v (gathered); reads y, y_a, l, u; writes ybar, y
        "a_v": 12 * nzA + 4 * (m + 1) + 8 * n + 32 * m + 16 * m,
        # A^T ybar: A^T, ybar (gathered); reads ATy, ATy_a; writes d, ATy
        "at_ybar": 12 * nzA + 4 * (n + 1) + 8 * m + 16 * n + 16 * n,
        # Q d + Halpern + next z/x step: Q, d (gathered); reads xhat, w, Qw, q1,
        # w_a, Qw_a, x_a, ATy, c, L, U; writes w, Qw, xhat
        "q_d_halpern": 12 * nzQ + 4 * (n + 1) + 8 * n + 88 * n + 24 * n,
    }


# sources of the single-instance solver's kernels and launches (the batched
# solver and the MLP do not enter the dominant kernel)
SOLVER_SOURCES = ("common.hpp", "spmv.hpp", "epilogues.hpp", "epilogues_primal.hpp", "qops.hpp", "small.hpp",
                  "panel.hpp", "split.hpp", "solver.hip")


def src_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2507_02470_amd", "csrc")
    for f in SOLVER_SOURCES:
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload: str):
    """HBM traffic per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel sources (else None)."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("src_hash") != src_hash():
        return None
    return d.get("traffic_bytes_per_launch")


def host_lambdas(qp):
    """Upper bounds of lambda_1(A A^T) and lambda_1(Q) from the host copy of
    the data alone (no GPU result): ||A||_1 ||A||_inf, and for Q its largest
    absolute row sum (CSR, symmetric), ||B||_inf ||C||_inf (+ ||S||_inf +
    ||T||_inf) for a Kronecker Q, max d + ||F||_F^2 for diag(d) + F F^T, or
    ||Ahat||_1 ||Ahat||_inf for Ahat^T Ahat.  The oracle's timed iterations
    take them as its lambda's: the cost of an iteration does not depend on
    them."""
    import numpy as np
    import scipy.sparse as sp

    def n1ninf(rp, ci, v, rows, cols):
        M = abs(sp.csr_matrix((v, ci, rp), shape=(rows, cols)))
        return float(np.asarray(M.sum(axis=0)).max(initial=0.0) * np.asarray(M.sum(axis=1)).max(initial=0.0))

    lam_A = n1ninf(qp.a_rowptr, qp.a_col, qp.a_val, qp.m, qp.n) if qp.m else 0.0
    if qp.qkind == "csr":
        Qm = abs(sp.csr_matrix((qp.q_val, qp.q_col, qp.q_rowptr), shape=(qp.n, qp.n)))
        lam_Q = float(np.asarray(Qm.sum(axis=1)).max(initial=0.0))
    elif qp.qkind == "kron":
        inf = lambda M: float(np.abs(np.asarray(M)).sum(axis=1).max())
        lam_Q = inf(qp.kron_B) * inf(qp.kron_C)
        for M in (qp.kron_S, qp.kron_T):
            if M is not None:
                lam_Q += inf(M)
    elif qp.qkind == "lowrank":
        lam_Q = float(np.max(qp.lr_d) + np.sum(np.asarray(qp.lr_F) ** 2))
    elif qp.qkind == "gram":
        lam_Q = n1ninf(qp.gram_rowptr, qp.gram_col, qp.gram_val, qp.gram_p, qp.n)
    else:
        lam_Q = 0.0
    return max(lam_A, 0.0), max(lam_Q, 0.0)


def host_cpu():
    """The host the oracle runs on: CPU model, logical CPUs, and the CPUs this
    process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return dict(model=model, logical_cpus=os.cpu_count(), usable_cpus=usable)


def oracle_rate(qp, iters=200, budget_s=20.0):
    """The oracle as it stands, single thread, on the first `iters` iterations
    (fewer when two iterations show that `iters` would exceed `budget_s`), with
    the lambda's of host_lambdas and its own sigma0 rule: (iterations, seconds)."""
    import oracle
    lam_A, lam_Q = host_lambdas(qp)
    t0 = time.perf_counter()
    oracle.solve(qp, tol=0.0, max_iter=2, check_every=T_CHECK, lambda_A=lam_A, lambda_Q=lam_Q)
    per_it = (time.perf_counter() - t0) / 2
    iters = int(max(2, min(iters, budget_s / max(per_it, 1e-9))))
    t0 = time.perf_counter()
    r = oracle.solve(qp, tol=0.0, max_iter=iters, check_every=T_CHECK, lambda_A=lam_A, lambda_Q=lam_Q)
    return r.iters, time.perf_counter() - t0


def cpu_baseline(qp, iters, budget_s=20.0):
    """oracle_rate as the bench line's cpu_baseline, with the host it ran on."""
    n, dt = oracle_rate(qp, iters, budget_s)
    return dict(value=n / dt, unit="iterations/s", cores=1, kind="oracle", host=host_cpu(),
                sample=f"first {n} iterations of the same instance (single-threaded FP64 C, "
                       f"lambda's from host-side bounds of the data), {dt:.1f} s")


FP64_PEAK_TFLOPS = 78.6    # MI355X dense FP64 MFMA, published
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X FP64 vector, published
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 MFMA, published


def extra_kron(steps, cpu):
    """Matrix-free Q = B (x) C (d = 300, n = 90,000) with assignment rows."""
    import torch
    import qpgen
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    qp = qpgen.make_kron()
    s = Solver(DeviceProblem(qp), power_start_A=qpgen.power_start(qp.m), power_start_Q=qpgen.power_start(qp.n),
               check_every=T_CHECK, tol=0.0, max_iter=T_CHECK, spmv_autotune=1)
    s.solve()
    s.set_options(tol=0.0, max_iter=steps * T_CHECK, profile_kernels=1, time_limit_s=0.0)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    r = s.solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - ta
    ks = s.kernel_stats()
    d = qp.kron_B.shape[0]
    q_flop = 2 * 2.0 * d * d * d            # two d x d x d GEMMs per Q product
    q_ms = 0.5 * (ks["avg_ms"]["q_xhat"] + ks["avg_ms"]["q_d_halpern"])
    out = dict(workload="kron_assignment", n=qp.n, m=qp.m, d=d, iterations_per_s=round(r.iters / dt, 1),
               us_per_iteration=round(dt / r.iters * 1e6, 2), kernel_avg_us={k: round(v * 1e3, 2) for k, v in
                                                                              ks["avg_ms"].items()},
               q_product=dict(flop=q_flop, avg_us=round(q_ms * 1e3, 2),
                              tflops=round(q_flop / (q_ms * 1e-3) / 1e12, 2),
                              fp64_mfma_util=round(q_flop / (q_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)))
    s.set_options(tol=1e-8, max_iter=2_000_000, profile_kernels=0, time_limit_s=60.0)
    rt = s.solve()
    out["time_to_1e-8"] = dict(term=rt.term, iterations=rt.iters, kkt=rt.kkt,
                               time_s=round(rt.t_setup_s + rt.t_solve_s, 4))
    if cpu:
        n_it, dt_o = oracle_rate(qp)
        out["cpu_oracle_iterations_per_s"] = round(n_it / dt_o, 3)
        out["cpu_oracle_sample"] = dict(iterations=n_it, seconds=round(dt_o, 2), cores=1, host=host_cpu())
    s.close()
    return out


def extra_qap(dims, steps, cpu, time_cap):
    """The synthetic QAP relaxation of Section 4.5 (d points in the unit square,
    Ahat their distance matrix, Bhat symmetric U[0,1) with zero diagonal),
    Q = 2(Bhat (x) Ahat - I (x) S - T (x) I) applied matrix-free: per d the
    iteration rate, the FP64-MFMA rate of the Q product (C X, then the
    three-term C X B^T - X T^T - S X: 8 d^3 flop) and the solve to 1e-8
    (power method included, capped at `time_cap` seconds)."""
    import torch
    import qpgen
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    out = {}
    for d in dims:
        qp = qpgen.make_qap(d=d)
        s = Solver(DeviceProblem(qp), power_start_A=qpgen.power_start(qp.m),
                   power_start_Q=qpgen.power_start(qp.n), check_every=T_CHECK, tol=0.0, max_iter=T_CHECK,
                   spmv_autotune=1)
        s.solve()
        s.set_options(tol=0.0, max_iter=steps * T_CHECK, profile_kernels=1, time_limit_s=0.0)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r = s.solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - ta
        ks = s.kernel_stats()["avg_ms"]
        q_flop = 8.0 * d ** 3
        q_ms = 0.5 * (ks["q_xhat"] + ks["q_d_halpern"])
        s.set_options(tol=1e-8, max_iter=50_000_000, profile_kernels=0, time_limit_s=time_cap)
        rt = s.solve()
        o = dict(n=qp.n, m=qp.m, iterations_per_s=round(r.iters / dt, 1),
                 us_per_iteration=round(dt / r.iters * 1e6, 2),
                 q_product=dict(flop=q_flop, avg_us=round(q_ms * 1e3, 2),
                                tflops=round(q_flop / (q_ms * 1e-3) / 1e12, 2),
                                fp64_mfma_util=round(q_flop / (q_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)),
                 time_to_1e8=dict(term=rt.term, iterations=rt.iters, kkt=rt.kkt, restarts=rt.restarts,
                                  time_s=round(rt.t_setup_s + rt.t_solve_s, 3), time_cap_s=time_cap,
                                  relaxation_bound=rt.pobj + float(qp.meta["s"].sum() + qp.meta["t"].sum())))
        if cpu and d <= 256:
            n_it, dt_o = oracle_rate(qp)
            o["cpu_oracle_iterations_per_s"] = round(n_it / dt_o, 3)
            o["cpu_oracle_sample"] = dict(iterations=n_it, seconds=round(dt_o, 2), cores=1)
        s.close()
        out[f"d{d}"] = o
        log(f"qap d={d}: {o}")
    return out


def extra_precond(qp_large, dp_large, cpu):
    """Diagonal preconditioning (Ruiz x10 + Pock-Chambolle): the random QP to
    1e-8 with it, and a badly scaled small QP (variables and rows rescaled by
    10^U(-2,2)) with and without it.  Solve times follow the paper's protocol:
    power method counted, preconditioning reported apart."""
    import qpgen
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    out = {}
    s = Solver(dp_large, power_start_A=qpgen.power_start(qp_large.m), power_start_Q=qpgen.power_start(qp_large.n),
               check_every=T_CHECK, tol=1e-8, max_iter=2_000_000, time_limit_s=60.0, precondition=1,
               spmv_autotune=1)
    r = s.solve()
    s.close()
    out["random_large"] = dict(term=r.term, iterations=r.iters, restarts=r.restarts, kkt=r.kkt,
                               t_precond_s=round(r.t_precond_s, 4),
                               time_to_tol_s=round(r.t_setup_s - r.t_precond_s + r.t_solve_s, 4), pobj=r.pobj)
    qp = qpgen.rescale(qpgen.make_small_ccqp(), 3)
    dp = DeviceProblem(qp)
    res = {}
    for pc in (1, 0):
        s = Solver(dp, check_every=T_CHECK, tol=1e-8, max_iter=200_000, precondition=pc)
        r = s.solve()
        s.close()
        res["with" if pc else "without"] = dict(term=r.term, iterations=r.iters, kkt=r.kkt,
                                                time_s=round(r.t_setup_s - r.t_precond_s + r.t_solve_s, 4))
    out["badly_scaled_small_ccqp"] = dict(n=qp.n, m=qp.m, **res)
    if cpu:
        import oracle
        t0 = time.perf_counter()
        ro = oracle.solve(qp, tol=1e-8, max_iter=200_000, precondition=True)
        out["badly_scaled_small_ccqp"]["cpu_oracle_with"] = dict(term=ro.term, iterations=ro.iters,
                                                                 time_s=round(time.perf_counter() - t0, 3))
    return out


def extra_lasso(steps, cpu, p=10_000, q=500_000, per_row=0, time_cap=60.0):
    """Lasso 1/2||Ahat x - bhat||^2 + lambda ||x||_1 (Section 4.4) of the paper's
    random Lasso table, lambda = ||Ahat^T bhat||_inf / 5; Q = Ahat^T Ahat
    matrix-free.  Default: its first size (p = 1e4 rows, q = 5e5 variables)
    with 1% N(0,1) entries; per_row > 0: Ahat built row by row with that many
    entries per row (the larger sizes, e.g. p = 2e5, q = 5e6, 1000 per row)."""
    import torch
    import qpgen
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    if per_row > 0:
        qp = qpgen.make_lasso_rows(seed=1008, p=p, q=q, per_row=per_row)
    else:
        qp = qpgen.make_lasso(seed=1006, p=p, q=q, density=0.01)
    nnz = int(qp.gram_rowptr[-1])
    dp = DeviceProblem(qp)
    s = Solver(dp, power_start_Q=qpgen.power_start(qp.n), check_every=T_CHECK, tol=0.0, max_iter=T_CHECK,
               spmv_autotune=1)
    s.solve()
    s.set_options(tol=0.0, max_iter=steps * T_CHECK, profile_kernels=1, time_limit_s=0.0)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    r = s.solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - ta
    ks = s.kernel_stats()
    q_us = ks["avg_ms"]["q_xhat"] * 1e3
    # Q xhat = Ahat^T (Ahat xhat) with its epilogue: both matrices once (12 B per
    # nonzero + row pointers); Ahat xhat written and gathered once (16 p); xhat
    # gathered once, xhat and Qw read, v and q1 written (40 n)
    q_bytes = 2 * 12 * nnz + 4 * (qp.gram_p + 1) + 4 * (qp.n + 1) + 16 * qp.gram_p + 40 * qp.n
    out = dict(workload="lasso", p=qp.gram_p, q=qp.n, nnz=nnz, l1_weight=qp.l1_weight,
               iterations_per_s=round(r.iters / dt, 1), us_per_iteration=round(dt / r.iters * 1e6, 2),
               q_product=dict(avg_us=round(q_us, 2), algorithmic_bytes=q_bytes,
                              GBps=round(q_bytes / (q_us * 1e-6) / 1e9, 1)))
    s.set_options(tol=1e-8, max_iter=2_000_000, profile_kernels=0, time_limit_s=time_cap)
    rt = s.solve()
    out["time_to_1e-8"] = dict(term=rt.term, iterations=rt.iters, restarts=rt.restarts, kkt=rt.kkt,
                               time_s=round(rt.t_setup_s + rt.t_solve_s, 4), pobj=rt.pobj, time_cap_s=time_cap)
    s.close()
    if cpu:
        n_it, dt_o = oracle_rate(qp)
        out["cpu_oracle_iterations_per_s"] = round(n_it / dt_o, 3)
        out["cpu_oracle_sample"] = dict(iterations=n_it, seconds=round(dt_o, 2), cores=1)
    return out


def extra_batch(count, cpu):
    """`count` independent portfolio QPs (n ~ U{50..2000}) in one persistent launch."""
    import numpy as np
    import torch
    import qpgen
    from paper_2507_02470_amd.batch import BatchSolver
    qps = qpgen.make_portfolio_batch(count)

    def timed(**opts):
        tc = time.perf_counter()
        b = BatchSolver(qps, tol=1e-8, max_iter=200_000, **opts)
        torch.cuda.synchronize()
        tc = time.perf_counter() - tc
        b.solve(split=False)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r = b.solve(split=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - ta
        sh = b.shapes()
        b.close()
        return r, dt, tc, sh

    # default shapes, then the shapes the autotuner picks at create (reported)
    r0, dt0, tc0, sh0 = timed()
    r, dt, tc, sh = timed(spmv_autotune=1)
    log(f"batch: default shapes {sh0['threads']} kernel {r0.kernel_s:.4f} s; tuned {sh['threads']} "
        f"kernel {r.kernel_s:.4f} s (create {tc:.3f} s incl. tuning)")
    it = r.iters
    terms = [f["term"] for f in r.infos]
    # FP64 vector work per iteration of an instance (n variables, rank r, nnz(A)):
    # two Q products of 4nr + 2n, A v and A^T ybar 2 nnz(A) each, about 40n of
    # elementwise updates; the persistent kernel is latency-bound, so this is
    # reported against the FP64 vector peak as an ALU roofline
    flops = sum(float(it[i]) * (2 * (4 * q.n * q.lr_F.shape[1] + 2 * q.n) + 4 * q.a_nnz + 40 * q.n)
                for i, q in enumerate(qps))
    achieved = flops / r.kernel_s / 1e12
    out = dict(workload="portfolio_batch", instances=count, sum_n=int(sum(q.n for q in qps)),
               solved=terms.count("solved"), wall_s=round(dt, 4), kernel_s=round(r.kernel_s, 4),
               instances_per_s=round(count / dt, 1), instance_iterations_per_s=round(float(it.sum()) / dt, 1),
               iterations_mean=round(float(it.mean()), 1), iterations_max=int(it.max()),
               max_kkt=float(max(f["kkt"] for f in r.infos)),
               roofline=dict(bound="alu", achieved=round(achieved, 3), peak=FP64_VECTOR_PEAK_TFLOPS,
                             unit="TFLOP/s", frac=round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4),
                             flop_per_batch=flops),
               shapes=dict(class_max_n=sh["class_max_n"], instances=sh["instances"], threads=sh["threads"],
                           tuned_us_per_instance_iteration={f"n<={c},{t}thr": round(v, 4)
                                                            for (c, t), v in sh["timed_us"].items()},
                           create_s_with_tuning=round(tc, 3)),
               default_shapes=dict(threads=sh0["threads"], kernel_s=round(r0.kernel_s, 4), wall_s=round(dt0, 4),
                                   iterations_mean=round(float(r0.iters.mean()), 1)))
    if cpu:
        import oracle
        sample = sorted(range(count), key=lambda i: qps[i].n)[::max(1, count // 64)][:64]
        t0 = time.perf_counter()
        its = 0
        for i in sample:
            its += oracle.solve(qps[i], tol=1e-8, max_iter=200_000).iters
        tc = time.perf_counter() - t0
        cores = os.cpu_count() or 1
        out["cpu_oracle"] = dict(instances_per_s=round(len(sample) / tc, 2),
                                 instance_iterations_per_s=round(its / tc, 1), cores=1, host=host_cpu(),
                                 sample=f"{len(sample)} instances stratified by n, solved one after another",
                                 projected_all_cores=dict(instances_per_s=round(cores * len(sample) / tc, 1),
                                                          cores=cores, kind="projected (independent instances)"))
    return out


def extra_small(cpu):
    """The small CCQP (n = 200, m = 100): launch-latency bound, graph replay."""
    import torch
    import qpgen
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    qp = qpgen.make_small_ccqp()
    s = Solver(DeviceProblem(qp), check_every=T_CHECK, tol=0.0, max_iter=T_CHECK)
    s.solve()
    s.set_options(tol=0.0, max_iter=20 * T_CHECK)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    r = s.solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - ta
    s.set_options(tol=1e-8, max_iter=1_000_000)
    rt = s.solve()
    s.close()
    out = {"workload": "small_ccqp", "n": qp.n, "m": qp.m, "us_per_iteration": round(dt / r.iters * 1e6, 2),
           "time_to_1e-8": dict(term=rt.term, iterations=rt.iters, time_s=round(rt.t_setup_s + rt.t_solve_s, 4))}
    if cpu:
        import oracle
        t0 = time.perf_counter()
        ro = oracle.solve(qp, tol=1e-8, max_iter=1_000_000)
        out["cpu_oracle_full_solve"] = dict(term=ro.term, iterations=ro.iters, time_s=round(time.perf_counter() - t0, 4),
                                            cores=1)
    return out


def extra_ablation(qp, dp, lamA, lamQ, steps, cpu, time_cap):
    """HPR-QP against HPR on the primal reformulations (Appendix A: method 1,
    Algorithm 6; method 2, Algorithm 7), the comparison of Table 1: full solves
    of the small CCQP, and on the random QP the iteration rate and the solve to
    1e-8 (capped at `time_cap` seconds per method)."""
    import torch
    import qpgen
    from paper_2507_02470_amd.solver import DeviceProblem, Solver
    small = qpgen.make_small_ccqp()
    sdp = DeviceProblem(small)
    out = {"small_ccqp": {}, "random_large": {}}
    for meth in (0, 1, 2):
        s = Solver(sdp, power_start_A=qpgen.power_start(small.m), power_start_Q=qpgen.power_start(small.n),
                   tol=1e-8, max_iter=2_000_000, method=meth)
        s.solve()
        r = s.solve()
        s.close()
        out["small_ccqp"][f"method{meth}"] = dict(term=r.term, iterations=r.iters, restarts=r.restarts,
                                                  time_s=round(r.t_setup_s + r.t_solve_s, 4), pobj=r.pobj)
    for meth in (1, 2):
        s = Solver(dp, lambda_A=lamA, lambda_Q=lamQ, check_every=T_CHECK, tol=0.0, max_iter=T_CHECK,
                   spmv_autotune=1, method=meth)
        s.solve()
        s.set_options(tol=0.0, max_iter=steps * T_CHECK, profile_kernels=1, time_limit_s=0.0)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r = s.solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - ta
        ks = s.kernel_stats()["avg_ms"]
        s.set_options(tol=1e-8, max_iter=50_000_000, profile_kernels=0, time_limit_s=time_cap)
        rt = s.solve()
        s.close()
        out["random_large"][f"method{meth}"] = dict(
            iterations_per_s=round(r.iters / dt, 1), us_per_iteration=round(dt / r.iters * 1e6, 2),
            product_avg_us={"Q": round(ks["q_xhat"] * 1e3, 2), "A": round(ks["a_v"] * 1e3, 2),
                            "AT": round(ks["at_ybar"] * 1e3, 2)},
            to_1e8=dict(term=rt.term, iterations=rt.iters, kkt=rt.kkt, time_s=round(rt.t_solve_s, 3),
                        time_cap_s=time_cap))
    if cpu:
        import oracle
        for meth in (1, 2):
            t0 = time.perf_counter()
            ro = oracle.solve(small, tol=1e-8, max_iter=2_000_000, method=meth,
                              power_start_A=qpgen.power_start(small.m), power_start_Q=qpgen.power_start(small.n))
            out["small_ccqp"][f"method{meth}"]["cpu_oracle"] = dict(term=ro.term, iterations=ro.iters,
                                                                    time_s=round(time.perf_counter() - t0, 3),
                                                                    cores=1)
    return out


def extra_mlp(steps=20):
    """The warm-start network (1021 -> 512 -> 512 -> 2022, the n = 1000
    portfolio family's) on random inputs: the forward pass at batch 512 (the
    warm-start evaluation) and a training step (forward, backward, Adam) at
    batch 128; GEMM time and useful FLOPs from the library's HIP events."""
    import numpy as np
    import torch
    from paper_2507_02470_amd.surrogate import MLP, init_params
    dims = (1021, 512, 512, 2022)
    net = MLP(dims, 512, init_params(dims, 0))
    rng = np.random.default_rng(0)
    X = torch.as_tensor(rng.standard_normal((512, dims[0])), dtype=torch.float32, device="cuda")
    T = torch.as_tensor(rng.standard_normal((512, dims[3])), dtype=torch.float32, device="cuda")
    fw = []
    for _ in range(steps + 2):
        net.forward(X)
        fw.append(net.gemm_stats())
    tr = []
    for i in range(steps + 2):
        b0 = (i % 4) * 128
        net.loss_grad(X[b0:b0 + 128], T[b0:b0 + 128], want_grad=False)
        tr.append(net.gemm_stats())
        net.adam(1e-4)
    torch.cuda.synchronize()
    net.close()
    med = lambda v: sorted(v)[len(v) // 2]
    f_ms, f_fl = med([x[0] for x in fw[2:]]), fw[-1][1]
    t_ms, t_fl = med([x[0] for x in tr[2:]]), tr[-1][1]
    f_tf, t_tf = f_fl / (f_ms * 1e-3) / 1e12, t_fl / (t_ms * 1e-3) / 1e12
    return dict(dims=list(dims), forward=dict(batch=512, gemm_ms=round(f_ms, 4), tflops=round(f_tf, 2)),
                train_step=dict(batch=128, gemm_ms=round(t_ms, 4), tflops=round(t_tf, 2)),
                roofline=dict(bound="mfma", kernel="k_gemm_bf16 (+ k_splitk_reduce)", achieved=round(f_tf, 2),
                              peak=BF16_PEAK_TFLOPS, unit="TFLOP/s", frac=round(f_tf / BF16_PEAK_TFLOPS, 5),
                              traffic=None, flop_per_forward=f_fl))


def calibrate_copy(reps=5, mib=4096):
    """The library's plain streaming copy of `mib` MiB (k_stream_copy2), after
    a 256 MiB fill that evicts the caches before each run: the counter scale
    (each run reads and writes mib MiB) and the HBM rate plain streaming
    reaches (read + write bytes over the HIP-event time; 4 GiB, so that the
    launch and the ramp are a small part of it)."""
    import ctypes as C
    import torch
    from paper_2507_02470_amd import _native as N
    lib = N.load()
    a = torch.rand(mib << 17, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    flush = torch.empty(32 << 20, dtype=torch.float64, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ms = []
    for _ in range(reps):
        flush.fill_(1.0)
        t = C.c_double()
        N.check(lib.hprqp_stream_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), a.numel(), st, C.byref(t)))
        ms.append(t.value)
    assert torch.equal(a, b)
    nbytes = 2 * a.numel() * 8
    del a, b, flush
    return dict(kernel="k_stream_copy2", bytes_read=nbytes // 2, bytes_written=nbytes // 2, runs=reps,
                best_ms=round(min(ms), 4), median_ms=round(sorted(ms)[reps // 2], 4),
                best_GBps=round(nbytes / (min(ms) * 1e-3) / 1e9, 1),
                median_GBps=round(nbytes / (sorted(ms)[reps // 2] * 1e-3) / 1e9, 1))


def _rounded(st):
    """{median, min, max} of repeated timings, in seconds to 0.1 ms."""
    return {k: round(v, 4) for k, v in st.items()}


def extra_warm_cold(n_train, n_eval, epochs):
    """Learned warm start on the parametric portfolio family (n = 1000, m = 21)."""
    import numpy as np
    import torch
    import qpgen
    from paper_2507_02470_amd.surrogate import (WarmStartSurrogate, family_features, solve_family, targets_from,
                                                warm_vs_cold)
    base = qpgen.make_portfolio_family_base()
    t0 = time.perf_counter()
    train = [qpgen.portfolio_family_sample(base, 100_000 + j) for j in range(n_train)]
    held = [qpgen.portfolio_family_sample(base, 200_000 + j) for j in range(n_eval)]
    tg = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = solve_family(base, train)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    X = np.stack([family_features(c, u) for (c, l, u) in train])
    T = targets_from(r, n_train, base.n, base.m)
    sur = WarmStartSurrogate(base, hidden=512, max_batch=512, seed=0)
    t0 = time.perf_counter()
    hist = sur.fit(X, T, epochs=epochs, batch=128, lr=1e-3, lr_final=1e-5, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    # BF16 MFMA throughput of the forward GEMMs on one evaluation batch
    Xe = np.stack([family_features(c, u) for (c, l, u) in held[:512]])
    sur.net.forward(Xe)
    ms, fl = sur.net.gemm_stats()
    mlp = extra_mlp()
    # first use of the warm-start path (network, unpack, the check of its flags)
    # outside the timed comparison
    bool(sur.starts(Xe)[3].bool().any())
    res = warm_vs_cold(sur, held)
    ic, iw = res["iters_cold"], res["iters_warm"]
    return dict(workload="portfolio_family", n=base.n, m=base.m, train_samples=n_train, eval_samples=n_eval,
                epochs=epochs, t_generate_s=round(tg, 2), t_solve_training_set_s=round(t_data, 2),
                t_train_s=round(t_train, 2), loss_first=hist[0], loss_last=hist[-1],
                repeats=res["repeats"],
                cold=dict(iterations_mean=round(float(ic.mean()), 1), iterations_median=float(np.median(ic)),
                          iterations_max=int(ic.max()),
                          wall_s=_rounded(res["wall_cold"]), kernel_s=_rounded(res["kernel_cold"])),
                warm=dict(iterations_mean=round(float(iw.mean()), 1), iterations_median=float(np.median(iw)),
                          iterations_max=int(iw.max()),
                          wall_s=_rounded(res["wall_warm"]), kernel_s=_rounded(res["kernel_warm"]),
                          fallback=res["fallback"]),
                cold_in_predicted_order=dict(kernel_s=_rounded(res["kernel_cold_ordered"])),
                wall_saving_frac=round(1.0 - res["t_warm_s"] / res["t_cold_s"], 4),
                fewer_iterations_frac=round(float(np.mean(iw < ic)), 4),
                max_kkt_warm=float(res["kkt_warm"].max()),
                max_obj_rel_diff=float(np.max(np.abs(res["obj_warm"] - res["obj_cold"]) /
                                              np.maximum(1.0, np.abs(res["obj_cold"])))),
                prediction_rel_err_w=round(res["pred_rel_err_w"], 4),
                prediction_rel_err_y=round(res["pred_rel_err_y"], 4),
                mlp_gemms=dict(forward=mlp["forward"], train_step=mlp["train_step"]),
                mlp_forward_gemm=dict(batch=512, ms=round(ms, 4), tflops=round(fl / (ms * 1e-3) / 1e12, 2),
                                      bf16_mfma_util=round(fl / (ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, 5)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="random_large",
                    choices=["random_large", "small_ccqp", "kron", "qap", "batch", "mlp", "lasso"])
    ap.add_argument("--qap-d", type=int, default=512, help="d of --workload qap (n = d^2)")
    ap.add_argument("--lasso-p", type=int, default=10_000, help="rows of Ahat, --workload lasso")
    ap.add_argument("--lasso-q", type=int, default=500_000, help="variables, --workload lasso")
    ap.add_argument("--lasso-per-row", type=int, default=0,
                    help="entries per row of Ahat (0: 1%% density), --workload lasso")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tol-solve", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=200)
    ap.add_argument("--tol-time-limit", type=float, default=120.0)
    ap.add_argument("--no-extras", action="store_true", help="skip the Kronecker, batch and warm-start workloads")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default SpMV kernel choice")
    ap.add_argument("--calibrate-copy", action="store_true", default=None,
                    help="run the library's streaming copy after the timed region (the default for the random QP): "
                         "the counter scale and the HBM rate plain streaming reaches")
    ap.add_argument("--no-calibrate-copy", dest="calibrate_copy", action="store_false")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--train-samples", type=int, default=50_000)
    ap.add_argument("--eval-samples", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--qap-dims", type=int, nargs="*", default=[256, 512],
                    help="sizes d of the synthetic QAP relaxations (n = d^2)")
    ap.add_argument("--qap-time-cap", type=float, default=30.0, help="seconds per QAP solve to 1e-8")
    ap.add_argument("--ablation-time-cap", type=float, default=15.0,
                    help="seconds per primal method for its solve of the random QP to 1e-8")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the HPR-QP path here is "
              f"single-GPU, see the multi-GPU design notes", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import qpgen
    from paper_2507_02470_amd.solver import DeviceProblem, Solver

    t0 = time.perf_counter()
    if args.workload == "random_large":
        qp = qpgen.make_random_large()
        wl = dict(workload="random_large", n=qp.n, m=qp.m, nnz_A=qp.a_nnz, nnz_Q=qp.q_nnz, seed=1001)
    elif args.workload == "kron":
        qp = qpgen.make_kron()
        wl = dict(workload="kron_assignment", n=qp.n, m=qp.m, d=300, seed=1002)
    elif args.workload == "qap":
        qp = qpgen.make_qap(d=args.qap_d)
        wl = dict(workload="qap_relaxation", n=qp.n, m=qp.m, d=args.qap_d, seed=1007)
    elif args.workload == "lasso":
        la = extra_lasso(args.steps, not args.no_cpu_baseline, args.lasso_p, args.lasso_q, args.lasso_per_row,
                         args.tol_time_limit)
        print(json.dumps(dict(metric="HPR-QP iterations/s (FP64, Lasso, Q = Ahat^T Ahat matrix-free)",
                              value=la["iterations_per_s"], unit="iterations/s", n_gpus=1, higher_is_better=True,
                              dtype="f64", data="synthetic (seeded random Lasso)",
                              config=dict(workload="lasso", p=la["p"], q=la["q"], nnz=la["nnz"]),
                              roofline=None, cpu_baseline=None, detail=la)))
        return
    elif args.workload == "mlp":
        # the warm-start network's GEMMs alone (what the rocprofv3 trace of them covers)
        m = extra_mlp(args.steps)
        print(json.dumps(dict(metric="BF16 MFMA TFLOP/s (warm-start network GEMMs)", value=m["forward"]["tflops"],
                              unit="TFLOP/s", n_gpus=1, higher_is_better=True, dtype="bf16 (FP32 accumulate)",
                              data="synthetic (random inputs, random-init weights)",
                              config=dict(workload="mlp_1021_512_512_2022"), roofline=m["roofline"], detail=m)))
        return
    elif args.workload == "batch":
        # the batched solver alone (what the batch leg of the extras reports)
        b = extra_batch(args.batch_count, not args.no_cpu_baseline)
        print(json.dumps(dict(metric="instances/s (batched HPR-QP to 1e-8)", value=b["instances_per_s"],
                              unit="instances/s", n_gpus=1, higher_is_better=True, dtype="f64",
                              data="synthetic (seeded portfolio generator)", config=dict(workload="portfolio_batch",
                              instances=args.batch_count), roofline=b["roofline"], cpu_baseline=b.get("cpu_oracle"),
                              detail=b)))
        return
    else:
        qp = qpgen.make_small_ccqp()
        wl = dict(workload="small_ccqp", n=qp.n, m=qp.m, seed=1000)
    log(f"generated {wl} in {time.perf_counter() - t0:.1f}s")
    dp = DeviceProblem(qp)
    torch.cuda.synchronize()
    s = Solver(dp, power_start_A=qpgen.power_start(qp.m), power_start_Q=qpgen.power_start(qp.n),
               check_every=T_CHECK, tol=0.0, max_iter=max(1, args.warmup) * T_CHECK, spmv_autotune=0 if args.no_autotune else 1,
               profile_kernels=0)
    pi = s.power_info()
    log(f"create: power A {pi['it_A']} its, Q {pi['it_Q']} its")
    # warmup (also captures the segment graph)
    s.solve()
    torch.cuda.synchronize()
    # timed region
    K = args.steps
    s.set_options(tol=0.0, max_iter=K * T_CHECK, profile_kernels=1, time_limit_s=0.0)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    r = s.solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - ta
    its = r.iters
    value = its / dt
    log(f"timed: {its} iterations in {dt:.3f}s -> {value:.1f} it/s (restarts {r.restarts})")
    ks = s.kernel_stats()
    log(f"kernel stats: {ks}")

    # roofline of the dominant kernel (largest share of timed kernel time)
    by = kernel_bytes(qp) if qp.qkind == "csr" else None
    roofline = None
    if qp.qkind == "kron":
        # Kronecker / QAP-relaxation Q product on FP64 MFMA: 2 d^3 flop per GEMM term
        # (C X, then C X B^T and, for the QAP relaxation, X T^T and S X)
        d = qp.kron_C.shape[0]
        flop = (8.0 if qp.kron_S is not None else 4.0) * d ** 3
        dom = max(("q_xhat", "q_d_halpern"), key=lambda k: ks["avg_ms"][k])
        avg_s = ks["avg_ms"][dom] * 1e-3
        roofline = dict(bound="mfma", kernel=dom, achieved=round(flop / avg_s / 1e12, 3), peak=FP64_PEAK_TFLOPS,
                        unit="TFLOP/s", frac=round(flop / avg_s / 1e12 / FP64_PEAK_TFLOPS, 4), traffic=None,
                        flop_per_launch=flop, avg_launch_us=round(avg_s * 1e6, 2),
                        launches_timed=ks["launches"][dom])
    if by is not None:
        dom = max(ks["avg_ms"], key=lambda k: ks["avg_ms"][k])
        avg_s = ks["avg_ms"][dom] * 1e-3
        achieved = by[dom] / avg_s / 1e9
        traffic = read_traffic(dom, wl["workload"])
        roofline = dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                        algorithmic_bytes_per_launch=by[dom], avg_launch_us=round(avg_s * 1e6, 2),
                        launches_timed=ks["launches"][dom])
        iter_bytes = sum(by.values())
        kern_s = sum(ks["avg_ms"].values()) * 1e-3
        roofline["iteration"] = dict(algorithmic_bytes=iter_bytes,
                                     kernel_GBps=round(iter_bytes / kern_s / 1e9, 1),
                                     wall_GBps=round(iter_bytes * value / 1e9, 1))
    # time to 1e-8 relative KKT (power method + setup included)
    tol_run = None
    if not args.no_tol_solve:
        s.set_options(tol=1e-8, max_iter=2_000_000, profile_kernels=0, time_limit_s=args.tol_time_limit)
        rt = s.solve()
        tol_run = dict(term=rt.term, iterations=rt.iters, kkt=rt.kkt, restarts=rt.restarts,
                       t_setup_s=round(rt.t_setup_s, 4), t_solve_s=round(rt.t_solve_s, 4),
                       time_to_tol_s=round(rt.t_setup_s + rt.t_solve_s, 4), pobj=rt.pobj)
        log(f"to 1e-8: {tol_run}")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(qp, args.cpu_iters)
        log(f"cpu baseline: {cpu}")
    s.close()
    copy_cal = None
    if args.calibrate_copy is None:
        args.calibrate_copy = args.workload == "random_large"
    if args.calibrate_copy:
        copy_cal = calibrate_copy()
        log(f"calibration copy (hprqp_stream_copy): {copy_cal}")
    extras = None
    if not args.no_extras and args.workload == "random_large":
        extras = {}
        extras["small_ccqp"] = extra_small(not args.no_cpu_baseline)
        log(f"small: {extras['small_ccqp']}")
        extras["primal_ablation"] = extra_ablation(qp, dp, r.lambda_A, r.lambda_Q, max(5, args.steps // 2),
                                                   not args.no_cpu_baseline, args.ablation_time_cap)
        log(f"ablation: {extras['primal_ablation']}")
        extras["precond"] = extra_precond(qp, dp, not args.no_cpu_baseline)
        log(f"precond: {extras['precond']}")
        extras["lasso"] = extra_lasso(max(5, args.steps // 2), not args.no_cpu_baseline)
        log(f"lasso: {extras['lasso']}")
        extras["kron"] = extra_kron(max(5, args.steps // 2), not args.no_cpu_baseline)
        log(f"kron: {extras['kron']}")
        extras["qap_relaxation"] = extra_qap(args.qap_dims, max(3, args.steps // 4), not args.no_cpu_baseline,
                                             args.qap_time_cap)
        extras["batch"] = extra_batch(args.batch_count, not args.no_cpu_baseline)
        log(f"batch: {extras['batch']}")
        extras["warm_vs_cold"] = extra_warm_cold(args.train_samples, args.eval_samples, args.epochs)
        log(f"warm vs cold: {extras['warm_vs_cold']}")
    out = {
        "metric": "HPR-QP iterations/s (FP64, relative-KKT stopping test every 100 iterations)",
        "value": round(value, 2),
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(dt / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator, shapes of the random QP class)",
        "config": dict(wl, step=f"{T_CHECK} iterations + check", lanes_per_row=ks["lanes_per_row"]),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_1e-8": tol_run,
        "hbm_copy_calibration": copy_cal,
        "extras": extras,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
