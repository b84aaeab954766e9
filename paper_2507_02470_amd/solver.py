"""Python front-end of the HPR-QP library: upload a QP into torch device
tensors and call the C ABI (hprqp_create / hprqp_solve / hprqp_residuals /
hprqp_apply).  Marshalling only; no solver arithmetic here.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N

QKIND = {"zero": 0, "csr": 1, "kron": 2, "lowrank": 3, "gram": 4}


def _dev(a, dtype, device):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(device)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class DeviceProblem:
    """Device copies of a QP (qpgen.QP-like object) and the C struct that
    points at them.  Keep this object alive while a handle uses it."""

    def __init__(self, qp, device="cuda"):
        f64, i32 = torch.float64, torch.int32
        self.n, self.m, self.qkind = int(qp.n), int(qp.m), qp.qkind
        self.t = {}
        t = self.t
        t["c"] = _dev(qp.c, f64, device)
        t["L"] = _dev(qp.L, f64, device)
        t["U"] = _dev(qp.U, f64, device)
        t["a_rowptr"] = _dev(qp.a_rowptr, i32, device)
        t["a_col"] = _dev(qp.a_col if len(qp.a_col) else np.zeros(1), i32, device)
        t["a_val"] = _dev(qp.a_val if len(qp.a_val) else np.zeros(1), f64, device)
        t["l"] = _dev(qp.l if self.m else np.zeros(1), f64, device)
        t["u"] = _dev(qp.u if self.m else np.zeros(1), f64, device)
        P = N.hprqp_problem()
        P.n, P.m, P.qkind = self.n, self.m, QKIND[qp.qkind]
        if qp.qkind == "csr":
            t["q_rowptr"] = _dev(qp.q_rowptr, i32, device)
            t["q_col"] = _dev(qp.q_col, i32, device)
            t["q_val"] = _dev(qp.q_val, f64, device)
            P.q_rowptr, P.q_col, P.q_val = (t["q_rowptr"].data_ptr(), t["q_col"].data_ptr(),
                                            t["q_val"].data_ptr())
            P.q_nnz = int(qp.q_rowptr[-1])
        elif qp.qkind == "kron":
            t["kron_B"] = _dev(np.asarray(qp.kron_B).ravel(order="F"), f64, device)
            t["kron_C"] = _dev(np.asarray(qp.kron_C).ravel(order="F"), f64, device)
            P.kron_p, P.kron_s = qp.kron_B.shape[0], qp.kron_C.shape[0]
            P.kron_B, P.kron_C = t["kron_B"].data_ptr(), t["kron_C"].data_ptr()
            for nm in ("kron_S", "kron_T"):
                if getattr(qp, nm, None) is not None:
                    t[nm] = _dev(np.asarray(getattr(qp, nm)).ravel(order="F"), f64, device)
                    setattr(P, nm, t[nm].data_ptr())
        elif qp.qkind == "lowrank":
            t["lr_d"] = _dev(qp.lr_d, f64, device)
            t["lr_F"] = _dev(qp.lr_F, f64, device)
            P.lr_rank = qp.lr_F.shape[1]
            P.lr_d, P.lr_F = t["lr_d"].data_ptr(), t["lr_F"].data_ptr()
        elif qp.qkind == "gram":
            t["gram_rowptr"] = _dev(qp.gram_rowptr, i32, device)
            t["gram_col"] = _dev(qp.gram_col if len(qp.gram_col) else np.zeros(1), i32, device)
            t["gram_val"] = _dev(qp.gram_val if len(qp.gram_val) else np.zeros(1), f64, device)
            P.gram_p = int(qp.gram_p)
            P.gram_rowptr, P.gram_col, P.gram_val = (t["gram_rowptr"].data_ptr(), t["gram_col"].data_ptr(),
                                                     t["gram_val"].data_ptr())
            P.gram_nnz = int(qp.gram_rowptr[-1])
        P.l1_weight = float(getattr(qp, "l1_weight", 0.0))
        P.c, P.L, P.U = t["c"].data_ptr(), t["L"].data_ptr(), t["U"].data_ptr()
        P.a_rowptr, P.a_col, P.a_val = t["a_rowptr"].data_ptr(), t["a_col"].data_ptr(), t["a_val"].data_ptr()
        P.a_nnz = int(qp.a_rowptr[-1])
        P.l, P.u = t["l"].data_ptr(), t["u"].data_ptr()
        self.P = P


def residuals_noalloc(dprob: DeviceProblem, y, z, x, w=None) -> dict:
    """hprqp_residuals_noalloc: the stopping quantities of Section 4.1 (and
    ||Q(w - x)||_inf) of the problem at (y, z, x) with no handle, computed in
    the library's static workspace; the work runs on torch's current stream."""
    lib = N.load()
    dev = torch.device("cuda", torch.cuda.current_device())
    f64 = dict(dtype=torch.float64, device=dev)
    yy = torch.as_tensor(y if dprob.m else np.zeros(1), **f64).contiguous()
    zz = torch.as_tensor(z, **f64).contiguous(); xx = torch.as_tensor(x, **f64).contiguous()
    ww = None if w is None else torch.as_tensor(w, **f64).contiguous()
    info = N.hprqp_info()
    st = torch.cuda.current_stream(dev)
    N.check(lib.hprqp_residuals_noalloc(C.byref(dprob.P), _ptr(yy), _ptr(zz), _ptr(ww), _ptr(xx), C.byref(info),
                                        C.c_void_p(st.cuda_stream)))
    return dict(eta_p=info.eta_p, eta_d=info.eta_d, eta_gap=info.eta_gap, pobj=info.pobj, dobj=info.dobj,
                kkt=max(info.eta_p, info.eta_d, info.eta_gap), qwx_gap=info.qwx_gap)


def default_options(**kw) -> N.hprqp_options:
    o = N.hprqp_options()
    N.load().hprqp_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


@dataclass
class Result:
    y: torch.Tensor
    z: torch.Tensor
    w: torch.Tensor
    x: torch.Tensor
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
    t_setup_s: float
    t_solve_s: float
    t_precond_s: float = 0.0
    qwx_gap: float = float("nan")
    trace: np.ndarray | None = None
    check_log: np.ndarray | None = None
    state: "State | None" = None

    @property
    def kkt(self) -> float:
        return max(self.eta_p, self.eta_d, self.eta_gap)


@dataclass
class State:
    """Start of the last epoch of a solve (restart index, first inner iterate
    in the handle's internal variables, sigma, total iteration count and the
    restart-test state): Solver.solve(resume=state) continues from it exactly."""
    k: int
    restarts: int
    sigma: float
    R0ref: float
    alpha3: float
    y: torch.Tensor
    w: torch.Tensor
    x: torch.Tensor


class Solver:
    """One HPR-QP handle (hprqp_create) bound to a DeviceProblem."""

    def __init__(self, dprob: DeviceProblem, power_start_A=None, power_start_Q=None, **opts):
        self.lib = N.load()
        self.dp = dprob
        self.device = dprob.t["c"].device
        self._keep = []
        if power_start_A is not None:
            a = _dev(power_start_A, torch.float64, self.device); self._keep.append(a)
            opts["power_start_A"] = a.data_ptr()
        if power_start_Q is not None:
            q = _dev(power_start_Q, torch.float64, self.device); self._keep.append(q)
            opts["power_start_Q"] = q.data_ptr()
        self.trace_iters = int(opts.get("trace_iters", 0))
        self.log_cap = int(opts.pop("log_cap", 0))
        self.opts = default_options(**{k: v for k, v in opts.items() if k not in ("trace_iters",)})
        self.trace = None
        if self.trace_iters > 0:
            self.trace = np.zeros((self.trace_iters, 2 * dprob.m + 4 * dprob.n))
            self.opts.trace_iters = self.trace_iters
            self.opts.trace_host = self.trace.ctypes.data_as(C.POINTER(C.c_double))
        self.log = None
        if self.log_cap > 0:
            self.log = np.zeros((self.log_cap, 10))
            self.opts.log_cap = self.log_cap
            self.opts.check_log_host = self.log.ctypes.data_as(C.POINTER(C.c_double))
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        N.check(self.lib.hprqp_create(C.byref(dprob.P), C.byref(self.opts),
                                      C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def set_options(self, **kw):
        """Change per-solve options (hprqp_set_options); setup choices stay."""
        for k, v in kw.items():
            if not hasattr(self.opts, k):
                raise KeyError(k)
            setattr(self.opts, k, v)
        N.check(self.lib.hprqp_set_options(self.h, C.byref(self.opts)))

    def close(self):
        if getattr(self, "h", None):
            self.lib.hprqp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, y0=None, w0=None, x0=None, resume: State | None = None, checkpoint: bool = False) -> Result:
        """Algorithm 4 from the warm start (y0, w0, x0), or from a saved
        epoch start (resume); checkpoint=True also returns the start of the
        last epoch as Result.state (HPR-QP, method 0)."""
        n, m = self.dp.n, self.dp.m
        f64 = dict(dtype=torch.float64, device=self.device)
        y = torch.empty(max(m, 1), **f64)
        z = torch.empty(n, **f64); w = torch.empty(n, **f64); x = torch.empty(n, **f64)
        info = N.hprqp_info()
        state = None
        if resume is None and not checkpoint:
            ins = [None if a is None else torch.as_tensor(a, **f64).contiguous() for a in (y0, w0, x0)]
            N.check(self.lib.hprqp_solve(self.h, _ptr(ins[0]), _ptr(ins[1]), _ptr(ins[2]), _ptr(y), _ptr(z),
                                         _ptr(w), _ptr(x), C.byref(info)))
        else:
            if any(a is not None for a in (y0, w0, x0)):
                raise ValueError("a solve with resume or checkpoint starts from the origin or the resumed state")
            rs = None
            if resume is not None:
                held = [torch.as_tensor(a, **f64).contiguous() for a in (resume.y, resume.w, resume.x)]
                rs = N.hprqp_state(k=resume.k, restarts=resume.restarts, sigma=resume.sigma, R0ref=resume.R0ref,
                                   alpha3=resume.alpha3, y=_ptr(held[0]) if m else None, w=_ptr(held[1]),
                                   x=_ptr(held[2]))
            sv = None
            if checkpoint:
                sy = torch.empty(max(m, 1), **f64); sw = torch.empty(n, **f64); sx = torch.empty(n, **f64)
                sv = N.hprqp_state(y=_ptr(sy), w=_ptr(sw), x=_ptr(sx))
            N.check(self.lib.hprqp_solve_resume(self.h, None if rs is None else C.byref(rs),
                                                None if sv is None else C.byref(sv), _ptr(y), _ptr(z), _ptr(w),
                                                _ptr(x), C.byref(info)))
            if checkpoint:
                state = State(k=int(sv.k), restarts=int(sv.restarts), sigma=sv.sigma, R0ref=sv.R0ref,
                              alpha3=sv.alpha3, y=sy[:m], w=sw, x=sx)
        return Result(y=y[:m], z=z, w=w, x=x, term=N.TERM[info.term], iters=int(info.iters),
                      restarts=int(info.restarts), sigma=info.sigma, sigma0=info.sigma0,
                      lambda_A=info.lambda_A, lambda_Q=info.lambda_Q, eta_p=info.eta_p, eta_d=info.eta_d,
                      eta_gap=info.eta_gap, pobj=info.pobj, dobj=info.dobj, R_last=info.R_last,
                      t_setup_s=info.t_setup_s, t_solve_s=info.t_solve_s, t_precond_s=info.t_precond_s,
                      qwx_gap=info.qwx_gap,
                      trace=None if self.trace is None else self.trace.copy(),
                      check_log=None if self.log is None else self.log[:info.n_log].copy(), state=state)

    def residuals(self, y, z, x, w=None) -> dict:
        f64 = dict(dtype=torch.float64, device=self.device)
        yy = torch.as_tensor(y if self.dp.m else np.zeros(1), **f64).contiguous()
        zz = torch.as_tensor(z, **f64).contiguous(); xx = torch.as_tensor(x, **f64).contiguous()
        ww = None if w is None else torch.as_tensor(w, **f64).contiguous()
        info = N.hprqp_info()
        N.check(self.lib.hprqp_residuals(self.h, _ptr(yy), _ptr(zz), _ptr(ww), _ptr(xx), C.byref(info)))
        return dict(eta_p=info.eta_p, eta_d=info.eta_d, eta_gap=info.eta_gap, pobj=info.pobj, dobj=info.dobj,
                    kkt=max(info.eta_p, info.eta_d, info.eta_gap), qwx_gap=info.qwx_gap)

    def apply(self, op: str, v) -> torch.Tensor:
        code = {"Q": 0, "A": 1, "AT": 2}[op]
        f64 = dict(dtype=torch.float64, device=self.device)
        vin = torch.as_tensor(v, **f64).contiguous()
        k = self.dp.m if op == "A" else self.dp.n
        out = torch.empty(max(k, 1), **f64)
        N.check(self.lib.hprqp_apply(self.h, code, _ptr(vin), _ptr(out)))
        return out[:k]

    def kernel_stats(self) -> dict:
        """Mean HIP-event duration (ms) and launch count of the four products
        of an iteration, from the last solve with profile_kernels=1."""
        avg = (C.c_double * 4)(); cnt = (C.c_int64 * 4)(); g = (C.c_int32 * 3)()
        N.check(self.lib.hprqp_kernel_stats(self.h, avg, cnt, g))
        names = ("q_xhat", "a_v", "at_ybar", "q_d_halpern")
        return dict(avg_ms={k: avg[i] for i, k in enumerate(names)},
                    launches={k: cnt[i] for i, k in enumerate(names)},
                    lanes_per_row=dict(A=g[0], AT=g[1], Q=g[2]))

    def scaling(self):
        """Scale factors (D, E) of the diagonal preconditioning (ones without it)."""
        f64 = dict(dtype=torch.float64, device=self.device)
        D = torch.empty(self.dp.n, **f64); E = torch.empty(max(self.dp.m, 1), **f64)
        N.check(self.lib.hprqp_scaling(self.h, _ptr(D), _ptr(E)))
        return D, E[:self.dp.m]

    def power_info(self):
        ea, eq = C.c_double(), C.c_double()
        ia, iq = C.c_int32(), C.c_int32()
        N.check(self.lib.hprqp_power_info(self.h, C.byref(ea), C.byref(ia), C.byref(eq), C.byref(iq)))
        return dict(est_A=ea.value, it_A=ia.value, est_Q=eq.value, it_Q=iq.value)
