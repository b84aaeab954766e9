"""Batched HPR-QP front-end: upload many low-rank QPs into concatenated
device tensors and call hprqp_batch_create / hprqp_solve_batch.  Marshalling
only; every step of the method runs in the persistent HIP kernel."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N
from .solver import default_options


def _cat(arrs, dtype):
    if not arrs:
        return np.zeros(1, dtype=dtype), np.zeros(1, dtype=np.int64)
    sizes = np.array([len(a) for a in arrs], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    flat = np.concatenate([np.asarray(a, dtype=dtype).ravel() for a in arrs]) if sizes.sum() else np.zeros(1, dtype)
    return flat, offs


@dataclass
class BatchResult:
    y: list
    z: list
    w: list
    x: list
    infos: list
    kernel_s: float

    @property
    def iters(self):
        return np.array([f["iters"] for f in self.infos])


def _problem_dtype():
    """numpy view of hprqp_problem (pointers as uint64)."""
    S = N.hprqp_problem
    kinds = {C.c_int32: np.int32, C.c_int64: np.int64, C.c_double: np.float64}
    return np.dtype(dict(names=[f for f, _ in S._fields_],
                         formats=[kinds.get(ct, np.uint64) for _, ct in S._fields_],
                         offsets=[getattr(S, f).offset for f, _ in S._fields_], itemsize=C.sizeof(S)))


class BatchSolver:
    """Solve many QPs with Q = diag(d) + F F^T in one persistent kernel.

    `shared`: if given, a base QP whose Q (d, F), A and box (L, U) every
    instance shares; then `instances` may be tuples (c, l, u) only."""

    def __init__(self, instances, device="cuda", shared=None, **opts):
        self.lib = N.load()
        f64, i32 = torch.float64, torch.int32
        self.count = len(instances)
        self.shared = shared
        dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(device)
        if shared is not None:
            base = shared
            ns = [base.n] * self.count
            ms = [base.m] * self.count
            cs = [inst[0] for inst in instances]
            ls = [inst[1] for inst in instances]
            us = [inst[2] for inst in instances]
            self.t = dict(c=dev(np.concatenate(cs), f64), l=dev(np.concatenate(ls) if base.m else np.zeros(1), f64),
                          u=dev(np.concatenate(us) if base.m else np.zeros(1), f64),
                          L=dev(base.L, f64), U=dev(base.U, f64), d=dev(base.lr_d, f64),
                          F=dev(base.lr_F.ravel(), f64), arp=dev(base.a_rowptr, i32),
                          aci=dev(base.a_col if len(base.a_col) else np.zeros(1), i32),
                          aval=dev(base.a_val if len(base.a_val) else np.zeros(1), f64))
            P = (N.hprqp_problem * self.count)()
            t = self.t
            # every instance's descriptor at once, through a structured view of the array
            a = np.frombuffer((C.c_char * C.sizeof(P)).from_buffer(P), dtype=_problem_dtype())
            i = np.arange(self.count, dtype=np.uint64)
            a["n"], a["m"], a["qkind"] = base.n, base.m, 3
            a["lr_rank"] = base.lr_F.shape[1]
            a["lr_d"], a["lr_F"] = t["d"].data_ptr(), t["F"].data_ptr()
            a["c"] = np.uint64(t["c"].data_ptr()) + np.uint64(8 * base.n) * i
            a["L"], a["U"] = t["L"].data_ptr(), t["U"].data_ptr()
            a["a_rowptr"], a["a_col"], a["a_val"] = t["arp"].data_ptr(), t["aci"].data_ptr(), t["aval"].data_ptr()
            a["a_nnz"] = int(base.a_rowptr[-1])
            a["l"] = np.uint64(t["l"].data_ptr()) + np.uint64(8 * base.m) * i
            a["u"] = np.uint64(t["u"].data_ptr()) + np.uint64(8 * base.m) * i
        else:
            qps = instances
            ns = [q.n for q in qps]
            ms = [q.m for q in qps]
            flat = {}
            offs = {}
            for key, get, dt in (("c", lambda q: q.c, np.float64), ("L", lambda q: q.L, np.float64),
                                 ("U", lambda q: q.U, np.float64), ("l", lambda q: q.l, np.float64),
                                 ("u", lambda q: q.u, np.float64), ("d", lambda q: q.lr_d, np.float64),
                                 ("F", lambda q: q.lr_F.ravel(), np.float64),
                                 ("arp", lambda q: q.a_rowptr, np.int32), ("aci", lambda q: q.a_col, np.int32),
                                 ("aval", lambda q: q.a_val, np.float64)):
                flat[key], offs[key] = _cat([get(q) for q in qps], dt)
            self.t = {k: dev(v, torch.float64 if v.dtype == np.float64 else i32) for k, v in flat.items()}
            t = self.t
            P = (N.hprqp_problem * self.count)()
            for i, q in enumerate(qps):
                if q.qkind != "lowrank":
                    raise ValueError("batched solve needs Q = diag(d) + F F^T instances")
                p = P[i]
                p.n, p.m, p.qkind = q.n, q.m, 3
                p.lr_rank = q.lr_F.shape[1]
                ptr = lambda key, isz: t[key].data_ptr() + isz * int(offs[key][i])
                p.c, p.L, p.U = ptr("c", 8), ptr("L", 8), ptr("U", 8)
                p.l, p.u = ptr("l", 8), ptr("u", 8)
                p.lr_d, p.lr_F = ptr("d", 8), ptr("F", 8)
                p.a_rowptr, p.a_col, p.a_val = ptr("arp", 4), ptr("aci", 4), ptr("aval", 8)
                p.a_nnz = int(q.a_rowptr[-1])
                p.l1_weight = float(getattr(q, "l1_weight", 0.0))
        self.P = P
        self.ns = np.array(ns, dtype=np.int64)
        self.ms = np.array(ms, dtype=np.int64)
        self.off_n = np.concatenate([[0], np.cumsum(self.ns)[:-1]])
        self.off_m = np.concatenate([[0], np.cumsum(self.ms)[:-1]])
        self.total_n, self.total_m = int(self.ns.sum()), int(self.ms.sum())
        self.opts = default_options(**opts)
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        N.check(self.lib.hprqp_batch_create(self.count, P, C.byref(self.opts), C.c_void_p(self.stream.cuda_stream),
                                            C.byref(h)))
        self.h = h

    def shared_features(self) -> torch.Tensor:
        """[c; u] of every instance of a shared-structure batch as a (count,
        n + m) float32 device tensor, from the copies already on the device."""
        if self.shared is None:
            raise ValueError("shared_features needs a batch built with `shared`")
        from .surrogate import _load
        n, m = self.shared.n, self.shared.m
        X = torch.empty((self.count, n + m), dtype=torch.float32, device=self.device)
        lib = _load()
        N.check(lib.hprqp_family_features(self.count, n, m, C.c_void_p(self.t["c"].data_ptr()),
                                          C.c_void_p(self.t["u"].data_ptr()) if m else None,
                                          C.c_void_p(X.data_ptr()), C.c_void_p(self.stream.cuda_stream)))
        return X

    def shapes(self) -> dict:
        """Size classes (n <= 256, 512, 1024, 2048) of the batch: instances,
        threads per workgroup of each, and the autotuner's measured kernel
        time per instance-iteration (us) of every block size it timed."""
        cnt = (C.c_int32 * 4)(); thr = (C.c_int32 * 4)(); us = (C.c_double * 16)()
        N.check(self.lib.hprqp_batch_shapes(self.h, cnt, thr, us))
        return dict(class_max_n=[256, 512, 1024, 2048], instances=list(cnt), threads=list(thr),
                    timed_us={(256 << c, 64 << j): us[4 * c + j] for c in range(4) for j in range(4) if us[4 * c + j] > 0})

    def set_priority(self, priority=None):
        """Queue order of the next solves: highest priority first (a device
        float32 tensor of `count` predicted solve lengths); None restores the
        default order.  Changes the time of a solve, not its results."""
        if priority is None:
            N.check(self.lib.hprqp_batch_set_priority(self.h, None))
            return
        p = torch.as_tensor(priority, dtype=torch.float32, device=self.device).contiguous()
        if p.numel() != self.count:
            raise ValueError(f"priority needs {self.count} entries, got {p.numel()}")
        N.check(self.lib.hprqp_batch_set_priority(self.h, C.c_void_p(p.data_ptr())))

    def close(self):
        if getattr(self, "h", None):
            self.lib.hprqp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, y0=None, w0=None, x0=None, split=True) -> BatchResult:
        f64 = dict(dtype=torch.float64, device=self.device)
        y = torch.empty(max(self.total_m, 1), **f64)
        z = torch.empty(self.total_n, **f64); w = torch.empty(self.total_n, **f64); x = torch.empty(self.total_n, **f64)
        ins = [None if a is None else torch.as_tensor(a, **f64).contiguous() for a in (y0, w0, x0)]
        ptr = lambda a: None if a is None else C.c_void_p(a.data_ptr())
        infos = (N.hprqp_info * self.count)()
        N.check(self.lib.hprqp_solve_batch(self.h, ptr(ins[0]), ptr(ins[1]), ptr(ins[2]), ptr(y), ptr(z), ptr(w),
                                           ptr(x), infos))
        ks = self.lib.hprqp_batch_last_kernel_s(self.h)
        inf = [dict(term=N.TERM[f.term], iters=int(f.iters), restarts=int(f.restarts), sigma=f.sigma,
                    sigma0=f.sigma0, lambda_A=f.lambda_A, lambda_Q=f.lambda_Q, eta_p=f.eta_p, eta_d=f.eta_d,
                    eta_gap=f.eta_gap, pobj=f.pobj, dobj=f.dobj, R_last=f.R_last, qwx_gap=f.qwx_gap,
                    kkt=max(f.eta_p, f.eta_d, f.eta_gap)) for f in infos]
        if not split:
            return BatchResult(y=y[:self.total_m], z=z, w=w, x=x, infos=inf, kernel_s=ks)
        yc, zc, wc, xc = (a.cpu().numpy() for a in (y, z, w, x))
        sl_n = [slice(int(o), int(o + k)) for o, k in zip(self.off_n, self.ns)]
        sl_m = [slice(int(o), int(o + k)) for o, k in zip(self.off_m, self.ms)]
        return BatchResult(y=[yc[s] for s in sl_m], z=[zc[s] for s in sl_n], w=[wc[s] for s in sl_n],
                           x=[xc[s] for s in sl_n], infos=inf, kernel_s=ks)
