"""Stage-by-stage element-wise checks of the library's BF16 / FP32 network
(test helper, no GPU of its own).

Every stage of the forward and backward pass is recomputed from the stage
tensors the library itself produced (exported through
hprqp_mlp_intermediate), with the formula of the FP64 reference network
(oracle/mlp.py), and compared entry by entry:

* a GEMM of BF16 operands (products exact in FP32) accumulated in FP32, K
  terms: |gpu - exact| <= K u (|A||B|)_ij + u |bias| (u = 2^-24; the
  recursive-summation bound, any order);
* an FP32 elementwise step: a few u of the magnitudes involved (the FP32
  GELU and GELU' through erff / expf: 8 u, generous);
* a rounding to BF16 of an FP32 value the library exported: exact;
* a rounding to BF16 of a value the check recomputes within e: between
  bf16(g - e) and bf16(g + e) (rounding is monotone), which is one value
  wherever [g - e, g + e] holds no BF16 rounding boundary.
Because each stage starts from the library's own inputs, no rounding
difference is carried from one stage into the next, and the bounds stay at
the size of the stage's own arithmetic.
"""
import numpy as np

from oracle import mlp as OM

U = 2.0 ** -24


def _f32inv(std):
    std = np.asarray(std, dtype=np.float32)
    return np.where(std > np.float32(1e-12), np.float32(1.0) / np.maximum(std, np.float32(1e-30)),
                    np.float32(0.0)).astype(np.float64)


def _gemm_check(name, got, A, B, bias=None):
    ref = A @ B
    bound = A.shape[1] * U * (np.abs(A) @ np.abs(B))
    if bias is not None:
        ref = ref + bias
        bound = bound + U * (np.abs(ref) + np.abs(bias))
    bad = np.abs(got - ref) > bound
    assert not bad.any(), f"{name}: {int(bad.sum())} entries outside the bound, worst {float((np.abs(got - ref) / np.maximum(bound, 1e-300)).max()):.3g}"
    return float(np.median(bound[ref != 0] / np.abs(ref[ref != 0]))) if np.any(ref != 0) else 0.0


def _close(name, got, ref, bound):
    bad = np.abs(got - ref) > bound
    assert not bad.any(), f"{name}: {int(bad.sum())} entries outside the bound"


def _round_check(name, got, g, e):
    lo, hi = OM.bf16(g - e), OM.bf16(g + e)
    ok = (got >= lo) & (got <= hi)
    assert ok.all(), f"{name}: {int((~ok).sum())} roundings outside [bf16(g - e), bf16(g + e)]"
    return float(np.mean(lo != hi))


def check_forward(net, p, X, dims, in_mean, in_std, out_mean, out_std, out_user):
    """After net.forward(X) (out_user its output): every forward stage."""
    W1, b1, W2, b2, W3, b3 = OM.unpack(p, dims)
    W1r, W2r, W3r = OM.bf16(W1), OM.bf16(W2), OM.bf16(W3)
    S = {k: net.intermediate(k).astype(np.float64) for k in ("Xs", "Z1", "A1", "Z2", "A2", "Y")}
    X = np.asarray(X, dtype=np.float32).astype(np.float64)
    xs = (X - np.asarray(in_mean, np.float32)) * _f32inv(in_std)
    amb = {"Xs": _round_check("Xs", S["Xs"], xs, 3 * U * (np.abs(xs) + np.abs(X) * _f32inv(in_std)))}
    rel = {"Z1": _gemm_check("Z1", S["Z1"], S["Xs"], W1r.T, b1)}
    amb["A1"] = _round_check("A1", S["A1"], OM.gelu(S["Z1"]), 8 * U * (np.abs(S["Z1"]) + 1e-30))
    rel["Z2"] = _gemm_check("Z2", S["Z2"], S["A1"], W2r.T, b2)
    amb["A2"] = _round_check("A2", S["A2"], OM.gelu(S["Z2"]), 8 * U * (np.abs(S["Z2"]) + 1e-30))
    rel["Y"] = _gemm_check("Y", S["Y"], S["A2"], W3r.T, b3)
    om, osd = np.asarray(out_mean, np.float32).astype(np.float64), np.asarray(out_std, np.float32).astype(np.float64)
    ref = om + osd * S["Y"]
    _close("output", np.asarray(out_user, dtype=np.float64), ref, 2 * U * (np.abs(ref) + np.abs(om)) + 1e-30)
    return S, rel, amb


def check_backward(net, p, grad, X, T, w, dims, in_mean, in_std, out_mean, out_std):
    """After net.loss_grad(X, T, w) (grad its gradient): every backward stage."""
    W1, b1, W2, b2, W3, b3 = OM.unpack(p, dims)
    W2r, W3r = OM.bf16(W2), OM.bf16(W3)
    S = {k: net.intermediate(k).astype(np.float64)
         for k in ("Xs", "Z1", "A1", "Z2", "A2", "Y", "Ts", "dY", "dYr", "dA2", "dZ2", "dZ2r", "dA1", "dZ1", "dZ1r")}
    B, N = S["Y"].shape
    T = np.asarray(T, dtype=np.float32).astype(np.float64)
    ts = (T - np.asarray(out_mean, np.float32)) * _f32inv(out_std)
    _close("Ts", S["Ts"], ts, 3 * U * (np.abs(ts) + np.abs(T) * _f32inv(out_std)) + 1e-30)
    wv = np.ones(N) if w is None else np.asarray(w, dtype=np.float32).astype(np.float64)
    sc = np.float64(np.float32(2.0 / (B * N)))
    dy = sc * wv * (S["Y"] - S["Ts"])
    _close("dY", S["dY"], dy, 4 * U * np.abs(dy) + 1e-300)
    assert np.array_equal(S["dYr"], OM.bf16(S["dY"])), "dYr"
    g = OM.unpack(np.asarray(grad, dtype=np.float64), dims)
    rel = {"W3": _gemm_check("dW3", g[4], S["dYr"].T, S["A2"])}
    db3 = S["dY"].sum(axis=0)
    _close("db3", g[5], db3, U * np.abs(db3) + B * 2.0 ** -52 * np.abs(S["dY"]).sum(axis=0) + 1e-300)
    rel["dA2"] = _gemm_check("dA2", S["dA2"], S["dYr"], W3r)
    dz2 = S["dA2"] * OM.gelu_d(S["Z2"])
    _close("dZ2", S["dZ2"], dz2, np.abs(S["dA2"]) * 8 * U * (1 + np.abs(S["Z2"])) + 2 * U * np.abs(dz2) + 1e-300)
    assert np.array_equal(S["dZ2r"], OM.bf16(S["dZ2"])), "dZ2r"
    rel["W2"] = _gemm_check("dW2", g[2], S["dZ2r"].T, S["A1"])
    db2 = S["dZ2"].sum(axis=0)
    _close("db2", g[3], db2, U * np.abs(db2) + B * 2.0 ** -52 * np.abs(S["dZ2"]).sum(axis=0) + 1e-300)
    rel["dA1"] = _gemm_check("dA1", S["dA1"], S["dZ2r"], W2r)
    dz1 = S["dA1"] * OM.gelu_d(S["Z1"])
    _close("dZ1", S["dZ1"], dz1, np.abs(S["dA1"]) * 8 * U * (1 + np.abs(S["Z1"])) + 2 * U * np.abs(dz1) + 1e-300)
    assert np.array_equal(S["dZ1r"], OM.bf16(S["dZ1"])), "dZ1r"
    rel["W1"] = _gemm_check("dW1", g[0], S["dZ1r"].T, S["Xs"])
    db1 = S["dZ1"].sum(axis=0)
    _close("db1", g[1], db1, U * np.abs(db1) + B * 2.0 ** -52 * np.abs(S["dZ1"]).sum(axis=0) + 1e-300)
    return S, rel
