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
        lib.hprqp_mlp_warm_start.argtypes = [_vp, C.c_int32, _vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp,
                                             _vp]
        lib.hprqp_mlp_gemm_stats.argtypes = [_vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        lib.hprqp_mlp_fit_scaling.argtypes = [_vp, C.c_int64, _vp, _vp, C.POINTER(C.c_float)]
        lib.hprqp_mlp_intermediate.argtypes = [_vp, C.c_int32, _vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        lib.hprqp_family_features.argtypes = [C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp]
        lib.hprqp_family_targets.argtypes = [C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]
        lib.hprqp_mlp_destroy.argtypes = [_vp]
        lib.hprqp_mlp_destroy.restype = None
        lib.hprqp_gemm_bf16.argtypes = [C.c_int32, C.c_int32, C.c_int32, _vp, C.c_int64, C.c_int64, _vp, C.c_int64,
                                        C.c_int64, _vp, C.c_int64, C.c_int32, C.c_int32, _vp, _vp]
        for f in ("hprqp_mlp_create", "hprqp_mlp_forward", "hprqp_mlp_loss_grad", "hprqp_mlp_adam",
                  "hprqp_mlp_get_params", "hprqp_mlp_set_params", "hprqp_mlp_set_scaling", "hprqp_mlp_warm_start",
                  "hprqp_mlp_gemm_stats", "hprqp_gemm_bf16", "hprqp_mlp_fit_scaling", "hprqp_mlp_intermediate", "hprqp_family_features",
                  "hprqp_family_targets"):
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

    def fit_scaling(self, X, T):
        """Standardization from training data (column means and standard
        deviations, computed by the library); returns them as numpy arrays."""
        X, T = self._f32(X), self._f32(T)
        n_in, n_out = self.dims[0], self.dims[3]
        st = np.zeros(2 * n_in + 2 * n_out, dtype=np.float32)
        N.check(self.lib.hprqp_mlp_fit_scaling(self.h, X.shape[0], _p(X), _p(T),
                                               st.ctypes.data_as(C.POINTER(C.c_float))))
        return st[:n_in], st[n_in:2 * n_in], st[2 * n_in:2 * n_in + n_out], st[2 * n_in + n_out:]

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

    STAGES = ("Xs", "Z1", "A1", "Z2", "A2", "Y", "dY", "dYr", "dA2", "dZ2", "dZ2r", "dA1", "dZ1", "dZ1r", "Ts")

    def intermediate(self, name) -> np.ndarray:
        """A stage tensor of the last forward / loss_grad call (test hook)."""
        k = self.STAGES.index(name)
        rows, cols = C.c_int32(), C.c_int32()
        N.check(self.lib.hprqp_mlp_intermediate(self.h, k, None, C.byref(rows), C.byref(cols)))
        out = torch.empty((rows.value, cols.value), dtype=torch.float32, device=self.device)
        N.check(self.lib.hprqp_mlp_intermediate(self.h, k, _p(out), None, None))
        return out.cpu().numpy()

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        N.check(self.lib.hprqp_mlp_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def set_params(self, p):
        buf, ptr = _fp(p)
        N.check(self.lib.hprqp_mlp_set_params(self.h, ptr))

    def warm_start(self, X, n, m, L, U):
        """(y0, w0, x0, bad, score): the FP64 start, the flags of samples
        started from the origin, and the predicted log iteration count of each
        solve (None unless the network has that output column)."""
        X = self._f32(X)
        B = X.shape[0]
        f64 = dict(dtype=torch.float64, device=self.device)
        y0 = torch.empty((B, max(m, 1)), **f64); w0 = torch.empty((B, n), **f64); x0 = torch.empty((B, n), **f64)
        bad = torch.empty(B, dtype=torch.int32, device=self.device)
        score = torch.empty(B, dtype=torch.float32, device=self.device) if self.dims[3] == m + 2 * n + 1 else None
        Lt = torch.as_tensor(L, **f64).contiguous(); Ut = torch.as_tensor(U, **f64).contiguous()
        N.check(self.lib.hprqp_mlp_warm_start(self.h, B, _p(X), n, m, _p(Lt), _p(Ut), _p(y0), _p(w0), _p(x0), _p(bad),
                                              _p(score)))
        return y0[:, :m], w0, x0, bad, score

    def gemm_stats(self):
        ms, fl = C.c_double(), C.c_double()
        N.check(self.lib.hprqp_mlp_gemm_stats(self.h, C.byref(ms), C.byref(fl)))
        return ms.value, fl.value


def gemm_bf16(A_bits: torch.Tensor, a_rs, a_cs, B_bits: torch.Tensor, b_rs, b_cs, M, N_, K, C_out: torch.Tensor,
              ldc, accumulate=False, split_k=1):
    """Raw BF16 GEMM of the library (inputs: int16 tensors holding BF16 bits);
    split_k > 1 cuts K into that many slices through a workspace."""
    lib = _load()
    ws = torch.empty(max(1, split_k * M * N_), dtype=torch.float32, device=C_out.device) if split_k > 1 else None
    N.check(lib.hprqp_gemm_bf16(M, N_, K, _p(A_bits), a_rs, a_cs, _p(B_bits), b_rs, b_cs, _p(C_out), ldc,
                                int(accumulate), int(split_k), _p(ws), _vp(torch.cuda.current_stream().cuda_stream)))


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


def targets_from(r, count, n, m, with_length=True):
    """Training targets [y; z; w] (FP32, count x (m + 2n)) of solved members,
    and with_length a last column log(iterations) of each member's solve,
    assembled by the library from the batched solver's concatenated outputs."""
    lib = _load()
    T = torch.empty((count, m + 2 * n + int(with_length)), dtype=torch.float32, device=r.z.device)
    y = r.y.contiguous() if m else None
    its = torch.as_tensor(np.array([f["iters"] for f in r.infos], dtype=np.int64), device=r.z.device) \
        if with_length else None
    z, w = r.z.contiguous(), r.w.contiguous()        # held for the call
    N.check(lib.hprqp_family_targets(count, n, m, _p(y), _p(z), _p(w), _p(its), _p(T),
                                     _vp(torch.cuda.current_stream(r.z.device).cuda_stream)))
    return T


class WarmStartSurrogate:
    def __init__(self, base, hidden=512, max_batch=512, seed=0, device="cuda", predict_length=True):
        """The network maps a member's parameters [c; u] to [y; z; w] (the
        start of Algorithm 4) and, with predict_length, one more output: the
        log iteration count of the member's solve, the priority with which
        the batched solver's queue starts the longest solves first."""
        self.base = base
        self.n, self.m = base.n, base.m
        self.dims = (base.n + base.m, hidden, hidden, base.m + 2 * base.n + int(predict_length))
        self.predict_length = bool(predict_length)
        self.net = MLP(self.dims, max_batch, init_params(self.dims, seed), device=device)
        self.device = torch.device(device)
        self.seed = seed

    def output_weights(self, out_std, z_weight=0.1, length_weight=None):
        """Loss weights of [y; z; w] that make the standardized loss a squared
        error in the solver's own units: the network is trained on
        standardized targets (each column divided by its standard deviation),
        so column j gets weight std_j^2, normalized to mean 1 inside each
        block.  Without this, the many w entries that are almost always zero
        (a member's optimal portfolio holds a few of the assets) would weigh
        as much as the few that carry the solution.  z is never read by
        Algorithm 4 (zbar is recomputed from (y, w, x)), so its block gets a
        small weight.  The length column (if any) is one output against n of
        w; it gets weight length_weight, by default n, the w block's total
        (on the n = 1000 portfolio family this ranks the held-out solves best
        of the weights tried: Spearman 0.64, against 0.59 at 100 and 0.55 at
        10)."""
        v = np.asarray(out_std, dtype=np.float64) ** 2
        out = np.full_like(v, float(self.n if length_weight is None else length_weight))
        for a, b, wt in ((0, self.m, 1.0), (self.m, self.m + self.n, z_weight),
                         (self.m + self.n, self.m + 2 * self.n, 1.0)):
            blk = v[a:b]
            mean = blk.mean() if b > a else 0.0
            out[a:b] = wt * blk / mean if mean > 0 else wt
        return out.astype(np.float32)

    def fit(self, X, T, epochs=20, batch=256, lr=1e-3, lr_final=1e-5, log=None, z_weight=0.1, length_weight=None):
        """X: (S, n_in) float32, T: (S, n_out) float32 (device or host)."""
        X = torch.as_tensor(X, dtype=torch.float32, device=self.device)
        T = torch.as_tensor(T, dtype=torch.float32, device=self.device)
        out_std = self.net.fit_scaling(X, T)[3]
        wts = torch.as_tensor(self.output_weights(out_std, z_weight, length_weight), device=self.device)
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
        """Warm starts (y0, w0, x0, bad, score) for the rows of X, in chunks of
        the network's max batch (score: None without the length output)."""
        X = torch.as_tensor(X, dtype=torch.float32, device=self.device)
        parts = [self.net.warm_start(X[b0:b0 + self.net.max_batch], self.n, self.m, self.base.L, self.base.U)
                 for b0 in range(0, X.shape[0], self.net.max_batch)]
        out = [torch.cat([p[k] for p in parts], dim=0) for k in range(4)]
        return (*out, torch.cat([p[4] for p in parts]) if self.predict_length else None)


def warm_vs_cold(sur: WarmStartSurrogate, samples, tol=1e-8, max_iter=200_000, repeats=3, order=True):
    """Solve `samples` cold and warm-started (with fallback) `repeats` times
    each, alternating; returns per-sample iterations (identical on every
    repeat: the solves are deterministic), the median, minimum and maximum
    wall and kernel times, and the fallback count.  Both wall times include
    staging the samples on the device; the warm one also the network (its
    input [c; u] taken from the staged copies), the queue order from its
    predicted solve lengths (order=True) and the fallback solves.  With the
    order, the kernel time of cold starts taken in the same order is
    reported as well, to tell the two parts of the gain apart."""
    base = sur.base
    t_cold, t_warm, k_cold, k_warm, k_cold_ord = [], [], [], [], []
    for _ in range(max(1, repeats)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = solve_family(base, samples, tol=tol, max_iter=max_iter)
        torch.cuda.synchronize()
        t_cold.append(time.perf_counter() - t0)
        k_cold.append(rc.kernel_s)
        t0 = time.perf_counter()
        bs = BatchSolver(samples, shared=base, tol=tol, max_iter=max_iter)
        y0, w0, x0, bad, score = sur.starts(bs.shared_features())   # a bad sample's start is the origin
        if order and score is not None:
            bs.set_priority(score)                   # predicted longest solves first
        rw = bs.solve(y0=y0.reshape(-1), w0=w0.reshape(-1), x0=x0.reshape(-1), split=False)
        bs.close()
        it_w = np.array([f["iters"] for f in rw.infos])
        failed = [i for i, f in enumerate(rw.infos) if f["term"] != "solved"]
        fallback = sorted(set(failed) | set(np.nonzero(bad.cpu().numpy())[0].tolist()))
        kw = rw.kernel_s
        if failed:
            rf = solve_family(base, [samples[i] for i in failed], tol=tol, max_iter=max_iter)
            kw += rf.kernel_s
            for j, i in enumerate(failed):
                it_w[i] += rf.infos[j]["iters"]
        torch.cuda.synchronize()
        t_warm.append(time.perf_counter() - t0)
        k_warm.append(kw)
        if order and score is not None:
            # the two parts apart: cold starts taken in the network's order
            bs = BatchSolver(samples, shared=base, tol=tol, max_iter=max_iter)
            bs.set_priority(score)
            k_cold_ord.append(bs.solve(split=False).kernel_s)
            bs.close()
    it_c = np.array([f["iters"] for f in rc.infos])
    obj_c = np.array([f["pobj"] for f in rc.infos])
    obj_w = np.array([f["pobj"] for f in rw.infos])
    # prediction error judged by the cold solution
    w_pred, w_cold = w0.cpu().numpy().reshape(-1), rc.w.cpu().numpy()
    y_pred, y_cold = y0.cpu().numpy().reshape(-1), rc.y.cpu().numpy().reshape(-1)
    pred_err_w = float(np.linalg.norm(w_pred - w_cold) / np.linalg.norm(w_cold))
    pred_err_y = float(np.linalg.norm(y_pred - y_cold) / max(np.linalg.norm(y_cold), 1e-300)) if base.m else 0.0
    stat = lambda v: dict(median=float(np.median(v)), min=float(np.min(v)), max=float(np.max(v)))
    return dict(iters_cold=it_c, iters_warm=it_w, t_cold_s=float(np.median(t_cold)), t_warm_s=float(np.median(t_warm)),
                kernel_cold_s=float(np.median(k_cold)), kernel_warm_s=float(np.median(k_warm)),
                wall_cold=stat(t_cold), wall_warm=stat(t_warm), kernel_cold=stat(k_cold), kernel_warm=stat(k_warm),
                kernel_cold_ordered=stat(k_cold_ord) if k_cold_ord else None,
                repeats=len(t_cold), fallback=len(fallback), obj_cold=obj_c, obj_warm=obj_w,
                kkt_warm=np.array([f["kkt"] for f in rw.infos]), kkt_cold=np.array([f["kkt"] for f in rc.infos]),
                pred_rel_err_w=pred_err_w, pred_rel_err_y=pred_err_y)
