"""ctypes front-end of the C oracle (TEST INFRASTRUCTURE ONLY).

Marshals :class:`qpgen.QP` numpy arrays into ``orc_problem`` and calls the
plain C implementation in ``hprqp_oracle.c``.  No solver arithmetic lives in
this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hprqp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_hprqp.so")
TERM_NAMES = {0: "solved", 1: "max_iter", 2: "time_limit", 3: "numerical"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int), ("m", C.c_int), ("qkind", C.c_int),
                ("q_rowptr", _ip), ("q_col", _ip), ("q_val", _dp),
                ("kron_p", C.c_int), ("kron_s", C.c_int), ("kron_B", _dp), ("kron_C", _dp),
                ("lr_rank", C.c_int), ("lr_d", _dp), ("lr_F", _dp),
                ("c", _dp), ("L", _dp), ("U", _dp),
                ("a_rowptr", _ip), ("a_col", _ip), ("a_val", _dp),
                ("l", _dp), ("u", _dp),
                ("l1_weight", C.c_double),
                ("gram_p", C.c_int), ("gram_rowptr", _ip), ("gram_col", _ip), ("gram_val", _dp),
                ("kron_S", _dp), ("kron_T", _dp)]


class _Options(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int64), ("check_every", C.c_int),
                ("time_limit_s", C.c_double), ("sigma0", C.c_double),
                ("lambda_A", C.c_double), ("lambda_Q", C.c_double),
                ("power_start_A", _dp), ("power_start_Q", _dp),
                ("alpha1", C.c_double), ("alpha2", C.c_double), ("alpha3", C.c_double),
                ("enable_restart", C.c_int), ("enable_sigma_update", C.c_int),
                ("trace_iters", C.c_int), ("trace", _dp),
                ("log_cap", C.c_int), ("check_log", _dp),
                ("precondition", C.c_int), ("ruiz_iters", C.c_int), ("method", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("term", C.c_int), ("iters", C.c_int64), ("restarts", C.c_int), ("n_log", C.c_int),
                ("sigma", C.c_double), ("sigma0", C.c_double), ("lambda_A", C.c_double),
                ("lambda_Q", C.c_double), ("eta_p", C.c_double), ("eta_d", C.c_double),
                ("eta_gap", C.c_double), ("pobj", C.c_double), ("dobj", C.c_double),
                ("R_last", C.c_double), ("t_solve_s", C.c_double)]


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math) into a shared library."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        # HPRQP_ORACLE_LIB lets the mutation test load a deliberately broken copy
        _lib = C.CDLL(os.environ.get("HPRQP_ORACLE_LIB") or build_oracle())
        _lib.orc_solve.argtypes = [C.POINTER(_Problem), C.POINTER(_Options), _dp, _dp, _dp,
                                   _dp, _dp, _dp, _dp, C.POINTER(_Info)]
        _lib.orc_residuals.argtypes = [C.POINTER(_Problem), _dp, _dp, _dp, _dp]
        for f in ("orc_apply_Q", "orc_apply_A", "orc_apply_AT"):
            getattr(_lib, f).argtypes = [C.POINTER(_Problem), _dp, _dp]
        _lib.orc_power.argtypes = [C.POINTER(_Problem), C.c_int, _dp, C.c_int, C.c_double, _ip]
        _lib.orc_power.restype = C.c_double
        _lib.orc_sigma0.argtypes = [C.POINTER(_Problem)]
        _lib.orc_sigma0.restype = C.c_double
        _lib.orc_thetas.argtypes = [C.POINTER(_Problem), C.c_double, C.c_double, _dp, _dp, _dp, _dp]
        _lib.orc_mnorm2.argtypes = [C.POINTER(_Problem), C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
        _lib.orc_mnorm2.restype = C.c_double
        _lib.orc_sigma_argmin.argtypes = [C.c_double] * 4
        _lib.orc_sigma_argmin.restype = C.c_double
        _lib.orc_restart_test.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int64, C.c_int64,
                                          C.c_double, C.c_double, C.c_double]
        _lib.orc_restart_test.restype = C.c_int
        _lib.orc_alpha3_next.argtypes = [C.c_double, C.c_double]
        _lib.orc_alpha3_next.restype = C.c_double
        _lib.orc_scaling.argtypes = [C.POINTER(_Problem), C.c_int, C.c_int, _dp, _dp]
        _lib.orc_primal_step.argtypes = [C.POINTER(_Problem), C.c_int, C.c_double, C.c_double, C.c_double,
                                         _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        _lib.orc_primal_mnorm2.argtypes = [C.POINTER(_Problem), C.c_int, C.c_double, C.c_double, C.c_double,
                                           _dp, _dp, _dp, _dp]
        _lib.orc_primal_mnorm2.restype = C.c_double
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_ip) if a is not None else None


class _Marshal:
    """Keeps contiguous copies alive while the C struct points at them."""

    QK = {"zero": 0, "csr": 1, "kron": 2, "lowrank": 3, "gram": 4}

    def __init__(self, qp):
        f64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        i32 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.int32)
        self.keep = []
        k = lambda a: (self.keep.append(a), a)[1]
        P = _Problem()
        P.n, P.m, P.qkind = qp.n, qp.m, self.QK[qp.qkind]
        if qp.qkind == "csr":
            P.q_rowptr = _i(k(i32(qp.q_rowptr))); P.q_col = _i(k(i32(qp.q_col)))
            P.q_val = _d(k(f64(qp.q_val)))
        if qp.qkind == "kron":
            P.kron_p = qp.kron_B.shape[0]; P.kron_s = qp.kron_C.shape[0]
            P.kron_B = _d(k(np.asfortranarray(qp.kron_B, dtype=np.float64).ravel(order="F")))
            P.kron_C = _d(k(np.asfortranarray(qp.kron_C, dtype=np.float64).ravel(order="F")))
            if getattr(qp, "kron_S", None) is not None:
                P.kron_S = _d(k(np.asfortranarray(qp.kron_S, dtype=np.float64).ravel(order="F")))
            if getattr(qp, "kron_T", None) is not None:
                P.kron_T = _d(k(np.asfortranarray(qp.kron_T, dtype=np.float64).ravel(order="F")))
        if qp.qkind == "lowrank":
            P.lr_rank = qp.lr_F.shape[1]
            P.lr_d = _d(k(f64(qp.lr_d))); P.lr_F = _d(k(f64(qp.lr_F)))
        if qp.qkind == "gram":
            P.gram_p = qp.gram_p
            P.gram_rowptr = _i(k(i32(qp.gram_rowptr))); P.gram_col = _i(k(i32(qp.gram_col)))
            P.gram_val = _d(k(f64(qp.gram_val) if qp.gram_val.size else np.zeros(1)))
        P.l1_weight = float(getattr(qp, "l1_weight", 0.0))
        P.c = _d(k(f64(qp.c))); P.L = _d(k(f64(qp.L))); P.U = _d(k(f64(qp.U)))
        P.a_rowptr = _i(k(i32(qp.a_rowptr))); P.a_col = _i(k(i32(qp.a_col)))
        P.a_val = _d(k(f64(qp.a_val) if qp.a_val.size else np.zeros(1)))
        P.l = _d(k(f64(qp.l) if qp.m else np.zeros(1))); P.u = _d(k(f64(qp.u) if qp.m else np.zeros(1)))
        self.P = P


@dataclass
class OracleResult:
    y: np.ndarray
    z: np.ndarray
    w: np.ndarray
    x: np.ndarray
    term: str
    iters: int
    restarts: int
    sigma: float
    sigma0: float
    lambda_A: float
    lambda_Q: float
    eta_p: float
    eta_d: float
    eta_gap: float
    pobj: float
    dobj: float
    R_last: float
    t_solve_s: float
    trace: np.ndarray | None = None
    check_log: np.ndarray | None = None

    @property
    def kkt(self) -> float:
        return max(self.eta_p, self.eta_d, self.eta_gap)


def solve(qp, tol=1e-8, max_iter=100_000, check_every=100, time_limit_s=0.0, sigma0=0.0,
          lambda_A=0.0, lambda_Q=0.0, alpha=(0.2, 0.8, 0.5), enable_restart=True,
          enable_sigma_update=True, trace_iters=0, log_cap=0, y0=None, w0=None, x0=None,
          power_start_A=None, power_start_Q=None, precondition=False, ruiz_iters=10,
          method=0) -> OracleResult:
    """Algorithm 4 (method 0) or HPR on the primal reformulation of Algorithm 6
    (method 1) / Algorithm 7 (method 2); for methods 1/2, w0 starts v (method 2)
    and the returned w is xbar (method 1) or vbar (method 2)."""
    L = _L()
    M = _Marshal(qp)
    O = _Options()
    O.tol, O.max_iter, O.check_every, O.time_limit_s = tol, int(max_iter), int(check_every), time_limit_s
    O.sigma0, O.lambda_A, O.lambda_Q = sigma0, lambda_A, lambda_Q
    psA = np.ascontiguousarray(power_start_A if power_start_A is not None else np.ones(max(qp.m, 1)), dtype=np.float64)
    psQ = np.ascontiguousarray(power_start_Q if power_start_Q is not None else np.ones(qp.n), dtype=np.float64)
    O.power_start_A, O.power_start_Q = _d(psA), _d(psQ)
    O.alpha1, O.alpha2, O.alpha3 = alpha
    O.enable_restart, O.enable_sigma_update = int(enable_restart), int(enable_sigma_update)
    O.precondition, O.ruiz_iters, O.method = int(precondition), int(ruiz_iters), int(method)
    trace = None
    if trace_iters > 0:
        trace = np.zeros((trace_iters, 2 * qp.m + 4 * qp.n))
        O.trace_iters, O.trace = trace_iters, _d(trace)
    log = None
    if log_cap > 0:
        log = np.zeros((log_cap, 10))
        O.log_cap, O.check_log = log_cap, _d(log)
    n, m = qp.n, qp.m
    y, z, w, x = np.zeros(max(m, 1)), np.zeros(n), np.zeros(n), np.zeros(n)
    keep = []

    def opt_vec(a, k):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(k)
        keep.append(a)
        return _d(a)

    info = _Info()
    L.orc_solve(C.byref(M.P), C.byref(O), opt_vec(y0, m) if m else None, opt_vec(w0, n), opt_vec(x0, n),
                _d(y), _d(z), _d(w), _d(x), C.byref(info))
    return OracleResult(y=y[:m].copy(), z=z, w=w, x=x, term=TERM_NAMES[info.term], iters=int(info.iters),
                        restarts=int(info.restarts), sigma=info.sigma, sigma0=info.sigma0,
                        lambda_A=info.lambda_A, lambda_Q=info.lambda_Q, eta_p=info.eta_p,
                        eta_d=info.eta_d, eta_gap=info.eta_gap, pobj=info.pobj, dobj=info.dobj,
                        R_last=info.R_last, t_solve_s=info.t_solve_s, trace=trace,
                        check_log=None if log is None else log[:info.n_log].copy())


def split_trace(trace: np.ndarray, n: int, m: int) -> dict:
    """Row layout [y, w, x, ybar, wbar, xbar] -> dict of (K, len) arrays."""
    o = 0
    out = {}
    for name, k in (("y", m), ("w", n), ("x", n), ("ybar", m), ("wbar", n), ("xbar", n)):
        out[name] = trace[:, o:o + k]
        o += k
    return out


def residuals(qp, y, z, x) -> dict:
    M = _Marshal(qp)
    out = np.zeros(5)
    yy = np.ascontiguousarray(y if qp.m else np.zeros(1), dtype=np.float64)
    zz = np.ascontiguousarray(z, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    _L().orc_residuals(C.byref(M.P), _d(yy), _d(zz), _d(xx), _d(out))
    return dict(eta_p=out[0], eta_d=out[1], eta_gap=out[2], pobj=out[3], dobj=out[4],
                kkt=max(out[0], out[1], out[2]))


def _apply(name, qp, v, k_out):
    M = _Marshal(qp)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(max(k_out, 1))
    getattr(_L(), name)(C.byref(M.P), _d(vv), _d(out))
    return out[:k_out]


def apply_Q(qp, x):
    return _apply("orc_apply_Q", qp, x, qp.n)


def apply_A(qp, x):
    return _apply("orc_apply_A", qp, x, qp.m)


def apply_AT(qp, y):
    return _apply("orc_apply_AT", qp, y if qp.m else np.zeros(1), qp.n)


def apply_Q_kron_factored(qp, x):
    """The Kronecker operator of Section 4.5 through numpy matrix products:
    Q vec(X) = vec(C X B^T) - vec(S X) - vec(X T^T), X the s x p matrix whose
    columns are the consecutive blocks of x (vec stacks columns).  The same
    definition as orc_apply_Q (pinned to it at small sizes); for sizes at
    which the C oracle's plain loops take minutes per product (d = 2048)."""
    B, Cm = np.asarray(qp.kron_B, dtype=np.float64), np.asarray(qp.kron_C, dtype=np.float64)
    p, s = B.shape[0], Cm.shape[0]
    X = np.asarray(x, dtype=np.float64).reshape(p, s).T
    out = Cm @ X @ B.T
    if getattr(qp, "kron_S", None) is not None:
        out -= np.asarray(qp.kron_S, dtype=np.float64) @ X
    if getattr(qp, "kron_T", None) is not None:
        out -= X @ np.asarray(qp.kron_T, dtype=np.float64).T
    return np.ascontiguousarray(out.T).ravel()


def power(qp, which: str, start, maxit=5000, tol=1e-6):
    M = _Marshal(qp)
    s = np.ascontiguousarray(start, dtype=np.float64)
    it = C.c_int(0)
    lam = _L().orc_power(C.byref(M.P), 0 if which == "A" else 1, _d(s), maxit, tol, C.byref(it))
    return lam, it.value


def scaling(qp, ruiz_iters=10, pock_chambolle=True):
    """Scale factors (D, E) of the diagonal preconditioning (Section 4.1)."""
    M = _Marshal(qp)
    D, E = np.zeros(qp.n), np.zeros(max(qp.m, 1))
    _L().orc_scaling(C.byref(M.P), int(ruiz_iters), int(pock_chambolle), _d(D), _d(E))
    return D, E[:qp.m].copy()


def sigma0(qp) -> float:
    M = _Marshal(qp)
    return _L().orc_sigma0(C.byref(M.P))


def thetas(qp, lamA, lamQ, dy, dw, dx):
    M = _Marshal(qp)
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (dy if qp.m else np.zeros(1), dw, dx)]
    out = np.zeros(4)
    _L().orc_thetas(C.byref(M.P), lamA, lamQ, _d(a[0]), _d(a[1]), _d(a[2]), _d(out))
    return out


def mnorm2(qp, sigma, lamA, lamQ, dy, dw, dx) -> float:
    M = _Marshal(qp)
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (dy if qp.m else np.zeros(1), dw, dx)]
    return _L().orc_mnorm2(C.byref(M.P), sigma, lamA, lamQ, _d(a[0]), _d(a[1]), _d(a[2]))


def sigma_argmin(th1, th2, th3, lamQ) -> float:
    return _L().orc_sigma_argmin(th1, th2, th3, lamQ)


RESTART_DECAY, RESTART_STALL, RESTART_LONG = 1, 2, 4


def restart_test(R, Rr0, Rprev, t, k, alpha1=0.2, alpha2=0.8, alpha3=0.5) -> int:
    """Bit mask of the restart criteria of Section 3.2 that hold at a check
    (1: "eq:restart_1", 2: "eq:restart_2", 4: "eq:restart_3"); Rprev < 0 means
    the epoch has no earlier check."""
    return int(_L().orc_restart_test(float(R), float(Rr0), float(Rprev), int(t), int(k),
                                     float(alpha1), float(alpha2), float(alpha3)))


def alpha3_next(alpha3, ratio) -> float:
    """alpha_3 after a restart whose ratio R~_{r,tau_r-1}/R~_{0,tau_0-1} is `ratio` (Section 4.1)."""
    return float(_L().orc_alpha3_next(float(alpha3), float(ratio)))


def primal_step(qp, variant, sigma, lamA, lamQ, x, y, v=None, t=None) -> dict:
    """Steps 1-3 of Algorithm 6 (variant 1) or 7 (variant 2) from (x, v, y, t)."""
    M = _Marshal(qp)
    n, m = qp.n, qp.m
    f = lambda a, k: np.ascontiguousarray(np.zeros(max(k, 1)) if a is None else
                                          (a if k else np.zeros(1)), dtype=np.float64)
    xx, vv, yy, tt = f(x, n), f(v, n), f(y, m), f(t, n)
    sb, yb = np.zeros(max(m, 1)), np.zeros(max(m, 1))
    vb, tb, xb, zb = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    _L().orc_primal_step(C.byref(M.P), int(variant), sigma, lamA, lamQ, _d(xx), _d(vv), _d(yy), _d(tt),
                         _d(sb), _d(yb), _d(vb), _d(tb), _d(xb), _d(zb))
    return dict(s=sb[:m].copy(), y=yb[:m].copy(), v=vb, t=tb, x=xb, z=zb)


def primal_mnorm2(qp, variant, sigma, lamA, lamQ, dx, dy, dv=None, dt=None) -> float:
    M = _Marshal(qp)
    n, m = qp.n, qp.m
    f = lambda a, k: np.ascontiguousarray(np.zeros(max(k, 1)) if a is None else
                                          (a if k else np.zeros(1)), dtype=np.float64)
    a = [f(dx, n), f(dv, n), f(dy, m), f(dt, n)]
    return _L().orc_primal_mnorm2(C.byref(M.P), int(variant), sigma, lamA, lamQ, *[_d(v) for v in a])
