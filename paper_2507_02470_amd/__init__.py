"""MI355X-native HPR-QP (arXiv 2507.02470): dual Halpern Peaceman-Rachford
for convex QPs, FP64 on gfx950 behind the C ABI of include/hprqp.h.

* ``solver.Solver`` / ``solver.DeviceProblem`` -- single-instance solves.
* ``batch.BatchSolver``                        -- many independent QPs in one
  persistent kernel.
* ``surrogate``                                -- BF16-MFMA MLP warm start.
"""
from ._native import load, LIB_PATH, HPRQPError  # noqa: F401
