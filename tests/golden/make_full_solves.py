"""Writes tests/golden/full_solves.json: the oracle's full solves (to 1e-8
relative KKT, Section 4.1) of the two large synthetic workloads, which take
minutes on one core, so the GPU tests compare against stored values.

    python tests/golden/make_full_solves.py

Calls only the oracle (and the seeded generators): Algorithm 4 + 5 with the
parameters of Section 4.1 (alpha = 0.2/0.8/0.5, power method, sigma0 rule,
checks every 100 iterations), from the origin.
"""
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import qpgen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_solves.json")


def solve(name, qp):
    t0 = time.time()
    r = oracle.solve(qp, tol=1e-8, max_iter=200_000, check_every=100,
                     power_start_A=qpgen.power_start(qp.m), power_start_Q=qpgen.power_start(qp.n))
    rec = dict(workload=name, n=qp.n, m=qp.m, term=r.term, iters=r.iters, restarts=r.restarts,
               pobj=r.pobj, dobj=r.dobj, eta_p=r.eta_p, eta_d=r.eta_d, eta_gap=r.eta_gap,
               lambda_A=r.lambda_A, lambda_Q=r.lambda_Q, sigma0=r.sigma0, sigma=r.sigma,
               oracle_seconds=round(time.time() - t0, 1))
    print(json.dumps(rec), flush=True)
    return rec


def main():
    recs = {}
    recs["kron_d300"] = solve("kron_d300", qpgen.make_kron())
    recs["random_large"] = solve("random_large", qpgen.make_random_large())
    recs["_generated_by"] = dict(script="tests/golden/make_full_solves.py", host=platform.node(),
                                 cpu=platform.processor() or platform.machine())
    with open(OUT, "w") as f:
        json.dump(recs, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
