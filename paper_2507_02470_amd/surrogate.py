"""Learned warm start for a parametric QP family (BF16-MFMA MLP in libhprqp.so).

A family member differs from a base portfolio QP in its objective c and its
constraint bounds (l, u); the network maps x = [c; u] to a starting point
(y, z, w) of HPR-QP.  Training targets are the FP64 solutions returned by the
batched solver; inference, training (forward, backward, Adam) and the
warm-start unpacking run in the library's kernels -- Python only moves data.
The cold start of Algorithm 4 (the origin) stays the fallback: a sample whose
prediction is not finite, or whose warm-started solve does not reach the
tolerance, is solved again from the origin.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np
import torch

from . import _native as N
from .batch import BatchSolver

_vp = C.c_void_p


def _load():
    lib = N.load()
    if not getattr(lib, "_mlp_ready", False):
        lib.hprqp_mlp_create.argtypes = [C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_float), _vp, C.POINTER(_vp)]
        lib.hprqp_mlp_num_params.argtypes = [_vp]
        lib.hprqp_mlp_num_params.restype = C.c_int64
        lib.hprqp_mlp_forward.argtypes = [_vp, C.c_int32, _vp, _vp]
        lib.hprqp_mlp_loss_grad.argtypes = [_vp, C.c_int32, _vp, _vp, _vp, C.POINTER(C.c_float), _vp]
        lib.hprqp_mlp_adam.argtypes = [_vp, C.c_float, C.c_float, C.c_float, C.c_float]
        lib.hprqp_mlp_get_params.argtypes = [_vp, C.POINTER(C.c_float)]
        lib.hprqp_mlp_set_params.argtypes = [_vp, C.POINTER(C.c_float)]
        lib.hprqp_mlp_set_scaling.argtypes = [_vp] + [C.POINTER(C.c_float)] * 4
        lib.hprqp_mlp_warm_start.argtypes = [_vp, C.c_int32, _vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]
        lib.hprqp_mlp_gemm_stats.argtypes = [_vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        lib.hprqp_mlp_destroy.argtypes = [_vp]
        lib.hprqp_mlp_destroy.restype = None
        lib.hprqp_gemm_bf16.argtypes = [C.c_int32, C.c_int32, C.c_int32, _vp, C.c_int64, C.c_int64, _vp, C.c_int64,
                                        C.c_int64, _vp, C.c_int64, C.c_int32, _vp]
        for f in ("hprqp_mlp_create", "hprqp_mlp_forward", "hprqp_mlp_loss_grad", "hprqp_mlp_adam",
                  "hprqp_mlp_get_params", "hprqp_mlp_set_params", "hprqp_mlp_set_scaling", "hprqp_mlp_warm_start",
                  "hprqp_mlp_gemm_stats", "hprqp_gemm_bf16"):
            getattr(lib, f).restype = C.c_int
        lib._mlp_ready = True
    return lib


def _p(t):
    return None if t is None else _vp(t.data_ptr())


def _fp(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


def init_params(dims, seed=0) -> np.ndarray:
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases."""
    rng = np.random.default_rng(seed)
    n_in, h1, h2, n_out = dims
    parts = []
    for rows, cols in ((h1, n_in), (h2, h1), (n_out, h2)):
        bnd = 1.0 / np.sqrt(cols)
        parts.append(rng.uniform(-bnd, bnd, rows * cols))
        parts.append(rng.uniform(-bnd, bnd, rows))
    return np.concatenate(parts).astype(np.float32)


class MLP:
    """Handle of hprqp_mlp (dims = (n_in, h1, h2, n_out))."""

    def __init__(self, dims, max_batch, params=None, device="cuda"):
        self.lib = _load()
        self.dims = tuple(int(d) for d in dims)
        self.max_batch = int(max_batch)
        self.device = torch.device(device)
        d = (C.c_int32 * 4)(*self.dims)
        buf = None
        if params is not None:
            buf, ptr = _fp(params)
        h = _vp()
        N.check(self.lib.hprqp_mlp_create(d, self.max_batch, ptr if params is not None else None,
                                          _vp(torch.cuda.current_stream(self.device).cuda_stream), C.byref(h)))
        self.h = h
        self.n_params = int(self.lib.hprqp_mlp_num_params(h))

    def close(self):
        if getattr(self, "h", None):
            self.lib.hprqp_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f32(self, a):
        return torch.as_tensor(a, dtype=torch.float32, device=self.device).contiguous()

    def set_scaling(self, in_mean, in_std, out_mean, out_std):
        arrs = [_fp(a) for a in (in_mean, in_std, out_mean, out_std)]
        N.check(self.lib.hprqp_mlp_set_scaling(self.h, *[p for _, p in arrs]))

    def forward(self, X):
        X = self._f32(X)
        Y = torch.empty((X.shape[0], self.dims[3]), dtype=torch.float32, device=self.device)
        N.check(self.lib.hprqp_mlp_forward(self.h, X.shape[0], _p(X), _p(Y)))
        return Y

    def loss_grad(self, X, T, w=None, want_grad=True):
        X, T = self._f32(X), self._f32(T)
        wt = None if w is None else self._f32(w)
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.device) if want_grad else None
        L = C.c_float(0)
        N.check(self.lib.hprqp_mlp_loss_grad(self.h, X.shape[0], _p(X), _p(T), _p(wt), C.byref(L), _p(g)))
        return float(L.value), g

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        N.check(self.lib.hprqp_mlp_adam(self.h, lr, beta1, beta2, eps))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        N.check(self.lib.hprqp_mlp_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def set_params(self, p):
        buf, ptr = _fp(p)
        N.check(self.lib.hprqp_mlp_set_params(self.h, ptr))

    def warm_start(self, X, n, m, L, U):
        X = self._f32(X)
        B = X.shape[0]
        f64 = dict(dtype=torch.float64, device=self.device)
        y0 = torch.empty((B, max(m, 1)), **f64); w0 = torch.empty((B, n), **f64); x0 = torch.empty((B, n), **f64)
        bad = torch.empty(B, dtype=torch.int32, device=self.device)
        Lt = torch.as_tensor(L, **f64).contiguous(); Ut = torch.as_tensor(U, **f64).contiguous()
        N.check(self.lib.hprqp_mlp_warm_start(self.h, B, _p(X), n, m, _p(Lt), _p(Ut), _p(y0), _p(w0), _p(x0), _p(bad)))
        return y0[:, :m], w0, x0, bad

    def gemm_stats(self):
        ms, fl = C.c_double(), C.c_double()
        N.check(self.lib.hprqp_mlp_gemm_stats(self.h, C.byref(ms), C.byref(fl)))
        return ms.value, fl.value


def gemm_bf16(A_bits: torch.Tensor, a_rs, a_cs, B_bits: torch.Tensor, b_rs, b_cs, M, N_, K, C_out: torch.Tensor,
              ldc, accumulate=False):
    """Raw BF16 GEMM of the library (inputs: int16 tensors holding BF16 bits)."""
    lib = _load()
    N.check(lib.hprqp_gemm_bf16(M, N_, K, _p(A_bits), a_rs, a_cs, _p(B_bits), b_rs, b_cs, _p(C_out), ldc,
                                int(accumulate), _vp(torch.cuda.current_stream().cuda_stream)))


# ---------------------------------------------------------------------------
# family data and training
# ---------------------------------------------------------------------------
def family_features(c, u):
    """Network input of one family member: [c; u]."""
    return np.concatenate([c, u]).astype(np.float32)


def solve_family(base, samples, tol=1e-8, max_iter=200_000, starts=None):
    """Solve family members (list of (c, l, u)) with the batched solver."""
    bs = BatchSolver(samples, shared=base, tol=tol, max_iter=max_iter)
    if starts is None:
        r = bs.solve(split=False)
    else:
        y0, w0, x0 = starts
        r = bs.solve(y0=y0.reshape(-1), w0=w0.reshape(-1), x0=x0.reshape(-1), split=False)
    bs.close()
    return r


def targets_from(r, count, n, m):
    y = r.y.reshape(count, m) if m else torch.zeros((count, 0), dtype=torch.float64, device=r.z.device)
    z = r.z.reshape(count, n)
    w = r.w.reshape(count, n)
    return torch.cat([y, z, w], dim=1).to(torch.float32)


class WarmStartSurrogate:
    def __init__(self, base, hidden=512, max_batch=512, seed=0, device="cuda"):
        self.base = base
        self.n, self.m = base.n, base.m
        self.dims = (base.n + base.m, hidden, hidden, base.m + 2 * base.n)
        self.net = MLP(self.dims, max_batch, init_params(self.dims, seed), device=device)
        self.device = torch.device(device)
        self.seed = seed

    def output_weights(self, z_weight=0.1):
        """Loss weights of [y; z; w]: z is never read by Algorithm 4 (zbar is
        recomputed from (y, w, x)), so it gets a small weight."""
        return np.concatenate([np.ones(self.m), np.full(self.n, z_weight), np.ones(self.n)]).astype(np.float32)

    def fit(self, X, T, epochs=20, batch=256, lr=1e-3, lr_final=1e-5, log=None, z_weight=0.1):
        """X: (S, n_in) float32, T: (S, n_out) float32 (device or host)."""
        wts = torch.as_tensor(self.output_weights(z_weight), device=self.device)
        X = torch.as_tensor(X, dtype=torch.float32, device=self.device)
        T = torch.as_tensor(T, dtype=torch.float32, device=self.device)
        xm, xs = X.mean(0).cpu().numpy(), X.std(0).cpu().numpy()
        tm, ts = T.mean(0).cpu().numpy(), T.std(0).cpu().numpy()
        self.net.set_scaling(xm, xs, tm, ts)
        S = X.shape[0]
        rng = np.random.default_rng(self.seed)
        steps = epochs * ((S + batch - 1) // batch)
        hist = []
        step = 0
        t0 = time.perf_counter()
        for ep in range(epochs):
            perm = torch.as_tensor(rng.permutation(S), device=self.device)
            tot = 0.0
            for b0 in range(0, S, batch):
                idx = perm[b0:b0 + batch]
                xb, tb = X.index_select(0, idx), T.index_select(0, idx)
                L, _ = self.net.loss_grad(xb, tb, wts, want_grad=False)
                lr_t = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * step / max(1, steps)))
                self.net.adam(lr_t)
                tot += L * len(idx)
                step += 1
            hist.append(tot / S)
            if log:
                log(f"epoch {ep}: loss {hist[-1]:.3e} ({time.perf_counter() - t0:.1f}s)")
        return hist

    def starts(self, X):
        """Warm starts (y0, w0, x0, bad) for the rows of X, in chunks of the network's max batch."""
        X = torch.as_tensor(X, dtype=torch.float32, device=self.device)
        parts = [self.net.warm_start(X[b0:b0 + self.net.max_batch], self.n, self.m, self.base.L, self.base.U)
                 for b0 in range(0, X.shape[0], self.net.max_batch)]
        return tuple(torch.cat([p[k] for p in parts], dim=0) for k in range(4))


def warm_vs_cold(sur: WarmStartSurrogate, samples, tol=1e-8, max_iter=200_000):
    """Solve `samples` cold and warm-started (with fallback); returns a dict of
    per-sample iterations, wall times and the fallback count.  Both timings
    include staging the samples on the device; the warm one also the network
    (its input [c; u] taken from the staged copies)."""
    base = sur.base
    n, m = base.n, base.m
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc = solve_family(base, samples, tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - t0
    t0 = time.perf_counter()
    bs = BatchSolver(samples, shared=base, tol=tol, max_iter=max_iter)
    y0, w0, x0, bad = sur.starts(bs.shared_features())
    badm = bad.bool()
    if badm.any():
        y0[badm] = 0; w0[badm] = 0; x0[badm] = 0
    rw = bs.solve(y0=y0.reshape(-1), w0=w0.reshape(-1), x0=x0.reshape(-1), split=False)
    bs.close()
    it_w = np.array([f["iters"] for f in rw.infos])
    failed = [i for i, f in enumerate(rw.infos) if f["term"] != "solved"]
    fallback = sorted(set(failed) | set(np.nonzero(badm.cpu().numpy())[0].tolist()))
    if failed:
        rf = solve_family(base, [samples[i] for i in failed], tol=tol, max_iter=max_iter)
        for j, i in enumerate(failed):
            it_w[i] += rf.infos[j]["iters"]
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    it_c = np.array([f["iters"] for f in rc.infos])
    obj_c = np.array([f["pobj"] for f in rc.infos])
    obj_w = np.array([f["pobj"] for f in rw.infos])
    # prediction error judged by the cold solution
    pred_err_w = float(torch.linalg.vector_norm(w0 - rc.w.reshape(-1, n)) / torch.linalg.vector_norm(rc.w))
    return dict(iters_cold=it_c, iters_warm=it_w, t_cold_s=t_cold, t_warm_s=t_warm, kernel_cold_s=rc.kernel_s,
                kernel_warm_s=rw.kernel_s, fallback=len(fallback), obj_cold=obj_c, obj_warm=obj_w,
                kkt_warm=np.array([f["kkt"] for f in rw.infos]), kkt_cold=np.array([f["kkt"] for f in rc.infos]),
                pred_rel_err_w=pred_err_w)
