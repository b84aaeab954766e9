"""CPU oracle for HPR-QP (arXiv 2507.02470) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports it and
shares no code with it.

* ``hprqp_oracle.c`` -- plain single-threaded FP64 C: Algorithm 4 + 5, the
  metric M, the stopping quantities, the power method, the diagonal
  preconditioning of Section 4.1, and HPR on the primal reformulations of
  Appendix A (Algorithms 6 and 7).  Loaded via ctypes.
* ``mlp.py``         -- numpy FP64 forward/backward of the warm-start MLP.
"""
from .oracle import (  # noqa: F401
    build_oracle, solve, residuals, apply_Q, apply_Q_kron_factored, apply_A, apply_AT, power, sigma0,
    thetas, mnorm2, sigma_argmin, restart_test, alpha3_next, scaling, primal_step, primal_mnorm2, OracleResult, TERM_NAMES,
)
