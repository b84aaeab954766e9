"""GPU tests of the BF16-MFMA warm-start network.

Tolerances: a GEMM with BF16-exact inputs within the recursive-summation
bound K 2^-24 (|A||B|)_ij of FP32 accumulation; every stage of the forward
and backward pass entry by entry against its formula applied to the
library's own stage inputs (tests/mlp_bounds.py: the same GEMM bound, a few
FP32 roundings for the elementwise steps, a BF16 rounding exact or, where the
stage's own error interval holds a rounding boundary, either neighbour), so
that no rounding difference is carried from stage to stage and one wrong
weight, index or gradient entry shows; the output and the gradient as a whole
against the FP64 reference network (oracle/mlp.py) in the Frobenius norm;
Adam against its definition (Kingma and Ba) in FP64, a few FP32 roundings per
entry; the warm-start unpack and the standardization exactly or to FP32
rounding.
"""
import numpy as np
import pytest

import oracle.mlp as OM
import qpgen
from tests import mlp_bounds as MB

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_02470_amd import load
    load()


def _bits(a):
    t = torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).cuda(), t.to(torch.float64).numpy()


@pytest.mark.parametrize("M,N,K,transA,transB,split", [(64, 64, 16, 0, 0, 1), (100, 37, 51, 0, 0, 1),
                                                       (1, 2021, 512, 0, 1, 1), (256, 512, 1024, 0, 0, 1),
                                                       (513, 129, 24, 1, 1, 1), (33, 65, 1000, 1, 0, 1),
                                                       (512, 512, 1021, 0, 1, 4), (100, 37, 51, 0, 0, 3),
                                                       (128, 512, 2024, 1, 0, 8), (33, 65, 1000, 1, 1, 64),
                                                       (70, 90, 17, 0, 0, 2)])
def test_gemm_bf16_against_numpy(M, N, K, transA, transB, split):
    """The GEMM, with K split into `split` slices or not, within the
    recursive-summation bound; accumulate adds to C; split results are the
    same on every call (fixed-order reduction)."""
    from paper_2507_02470_amd.surrogate import gemm_bf16
    rng = np.random.default_rng(M * 7 + N + split)
    A = rng.standard_normal((M, K)); B = rng.standard_normal((K, N))
    if transA:   # A stored as K x M (A(i,k) = At[k, i])
        Ab, Ar = _bits(A.T.copy()); a_rs, a_cs = 1, M
    else:
        Ab, Ar = _bits(A); a_rs, a_cs = K, 1
    if transB:   # B stored as N x K
        Bb, Br = _bits(B.T.copy()); b_rs, b_cs = 1, K
    else:
        Bb, Br = _bits(B); b_rs, b_cs = N, 1
    Ae = Ar.T if transA else Ar
    Be = Br.T if transB else Br
    Cout = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    gemm_bf16(Ab, a_rs, a_cs, Bb, b_rs, b_cs, M, N, K, Cout, N, split_k=split)
    ref = Ae @ Be
    bound = K * 2.0 ** -24 * (np.abs(Ae) @ np.abs(Be)) + 1e-30
    C1 = Cout.cpu().numpy().astype(np.float64)
    err = np.abs(C1 - ref)
    assert np.all(err <= bound), float((err / bound).max())
    C0 = rng.standard_normal((M, N)).astype(np.float32)
    Cacc = torch.as_tensor(C0, device="cuda")
    gemm_bf16(Ab, a_rs, a_cs, Bb, b_rs, b_cs, M, N, K, Cacc, N, accumulate=True, split_k=split)
    ref2 = C0.astype(np.float64) + ref
    bound2 = (K + 1) * 2.0 ** -24 * (np.abs(Ae) @ np.abs(Be) + np.abs(C0)) + 1e-30
    assert np.all(np.abs(Cacc.cpu().numpy().astype(np.float64) - ref2) <= bound2)
    Cagain = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    gemm_bf16(Ab, a_rs, a_cs, Bb, b_rs, b_cs, M, N, K, Cagain, N, split_k=split)
    assert torch.equal(Cagain, Cout)


DIMS = (1021, 512, 512, 2021)


def _net(params, batch, scaling):
    from paper_2507_02470_amd.surrogate import MLP
    net = MLP(DIMS, batch, params)
    net.set_scaling(*scaling)
    return net


def _scaling(rng):
    return (rng.standard_normal(DIMS[0]).astype(np.float32), rng.uniform(0.5, 2, DIMS[0]).astype(np.float32),
            rng.standard_normal(DIMS[3]).astype(np.float32), rng.uniform(0.5, 2, DIMS[3]).astype(np.float32))


def test_forward_stages_entrywise_and_fp64_reference():
    """Every forward stage entry by entry from the library's own stage inputs
    (tests/mlp_bounds.py), and the output against the FP64 reference network
    (oracle/mlp.py, BF16 at the same operands) as a whole."""
    from paper_2507_02470_amd.surrogate import init_params
    rng = np.random.default_rng(3)
    p = init_params(DIMS, seed=1)
    sc = _scaling(rng)
    X = rng.standard_normal((48, DIMS[0])).astype(np.float32)
    net = _net(p, 64, sc)
    Y = net.forward(X).cpu().numpy().astype(np.float64)
    S, rel, amb = MB.check_forward(net, p, X, DIMS, *sc, Y)
    net.close()
    print("forward stage bounds (median relative):", rel, "BF16 roundings at a boundary:", amb, flush=True)
    assert max(rel.values()) < 1e-2          # the bounds are tight: a wrong weight or index shows
    Ys, _ = OM.forward(p, X, DIMS, emulate=True, in_mean=sc[0], in_std=sc[1])
    Yref = sc[2] + sc[3] * Ys
    rel_f = np.linalg.norm(Y - Yref) / np.linalg.norm(Yref)
    print("forward vs reference (Frobenius):", rel_f, flush=True)
    assert rel_f <= 2e-3


def test_backward_stages_entrywise_and_fp64_reference():
    from paper_2507_02470_amd.surrogate import init_params
    rng = np.random.default_rng(4)
    p = init_params(DIMS, seed=2)
    sc = _scaling(rng)
    X = rng.standard_normal((32, DIMS[0])).astype(np.float32)
    T = rng.standard_normal((32, DIMS[3])).astype(np.float32)
    w = rng.uniform(0.5, 1.5, DIMS[3]).astype(np.float32)
    net = _net(p, 64, sc)
    L, g = net.loss_grad(X, T, w)
    g = g.cpu().numpy().astype(np.float64)
    Yb = net.intermediate("Y").astype(np.float64)
    S, rel = MB.check_backward(net, p, g, X, T, w, DIMS, *sc)
    net.close()
    print("backward stage bounds (median relative):", rel, flush=True)
    assert max(rel.values()) < 1e-2
    Lr, gr = OM.loss_grad(p, X, T, DIMS, w=w, emulate=True, in_mean=sc[0], in_std=sc[1], out_mean=sc[2],
                          out_std=sc[3])
    assert L == pytest.approx(Lr, rel=1e-4)
    for name, a, b in zip(("W1", "b1", "W2", "b2", "W3", "b3"), OM.unpack(g, DIMS), OM.unpack(gr, DIMS)):
        rel_f = np.linalg.norm(a - b) / np.linalg.norm(b)
        print("grad vs reference (Frobenius)", name, rel_f, flush=True)
        assert rel_f <= 5e-3, (name, rel_f)


def test_adam_step_matches_its_definition():
    """Two Adam steps (Kingma and Ba; bias-corrected moments) on the library's
    own gradients, against the update written out in FP64 with the library's
    FP32 hyperparameters.  Tolerance per entry, from the terms of the update:
    a few FP32 roundings of each moment (carried over the steps), the bias
    corrections 1 - beta^t from an FP32 power (2 ulp of beta^t, amplified by
    beta^t / (1 - beta^t), about 500 u for beta2 = 0.999 at t = 2), and a few
    roundings of the step itself."""
    from paper_2507_02470_amd.surrogate import MLP, init_params
    U = MB.U
    rng = np.random.default_rng(8)
    dims = (40, 64, 64, 30)
    p0 = init_params(dims, 4)
    net = MLP(dims, 64, p0)
    lr, b1, b2, eps = (float(np.float32(v)) for v in (3e-3, 0.9, 0.999, 1e-8))
    m = np.zeros(p0.size); v = np.zeros(p0.size); em = np.zeros(p0.size); ev = np.zeros(p0.size)
    p = p0.astype(np.float64)
    for t in (1, 2):
        X = rng.standard_normal((64, 40)).astype(np.float32)
        T = rng.standard_normal((64, 30)).astype(np.float32)
        _, g = net.loss_grad(X, T)
        g = g.cpu().numpy().astype(np.float64)
        net.adam(lr, b1, b2, eps)
        got = net.get_params().astype(np.float64)
        em = b1 * em + 3 * U * (b1 * np.abs(m) + (1 - b1) * np.abs(g))
        ev = b2 * ev + 4 * U * (b2 * v + (1 - b2) * g * g)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        c1, c2 = 1 - b1 ** t, 1 - b2 ** t
        rc1, rc2 = 3 * U * b1 ** t / c1 + U, 3 * U * b2 ** t / c2 + U
        den = np.sqrt(v / c2) + eps
        step = lr * (m / c1) / den
        ref = p - step
        e_step = (lr / den) * (em / c1) + np.abs(step) * (rc1 + 0.5 * rc2 + 0.5 * ev / np.maximum(v, 1e-300) + 8 * U)
        tol = 2 * U * np.abs(ref) + e_step + 1e-30
        print(f"adam step {t}: max err/tol {float((np.abs(got - ref) / tol).max()):.3f}, "
              f"median tol/|step| {float(np.median(tol / np.maximum(np.abs(step), 1e-300))):.2e}", flush=True)
        assert np.all(np.abs(got - ref) <= tol)
        p = got                                    # continue from the library's FP32 parameters
    net.close()


def test_warm_start_unpack_and_standardization():
    """Pi_C of the predicted w, the predicted y, the predicted solve length,
    the origin for a sample whose prediction is not finite; the
    standardization statistics the library computes; the family features and
    targets (with and without the log iteration column) it assembles."""
    from paper_2507_02470_amd.surrogate import MLP, init_params, _load, _p, _vp
    from paper_2507_02470_amd import _native as N
    rng = np.random.default_rng(9)
    n, m = 30, 4
    dims = (n + m, 48, 48, m + 2 * n + 1)
    net = MLP(dims, 16, init_params(dims, 5))
    X = rng.standard_normal((16, n + m)).astype(np.float32)
    T = rng.standard_normal((16, dims[3])).astype(np.float32) * rng.uniform(0.1, 3, dims[3]).astype(np.float32)
    xm, xs, tm, ts = net.fit_scaling(X, T)
    np.testing.assert_allclose(xm, X.astype(np.float64).mean(0), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(xs, X.astype(np.float64).std(0, ddof=1), rtol=1e-6)
    np.testing.assert_allclose(ts, T.astype(np.float64).std(0, ddof=1), rtol=1e-6)
    L = np.full(n, -0.1); U = np.full(n, 0.1)
    X[5, 3] = np.nan                                  # sample 5: a prediction that is not finite
    P = net.forward(X).cpu().numpy().astype(np.float64)
    y0, w0, x0, bad, score = net.warm_start(X, n, m, L, U)
    y0, w0, x0, bad = y0.cpu().numpy(), w0.cpu().numpy(), x0.cpu().numpy(), bad.cpu().numpy()
    np.testing.assert_array_equal(score.cpu().numpy(), P[:, m + 2 * n].astype(np.float32))
    ok = np.arange(16) != 5
    assert bad.tolist() == [int(i == 5) for i in range(16)]
    np.testing.assert_array_equal(y0[ok], P[ok, :m])
    np.testing.assert_array_equal(w0[ok], P[ok, m + n:m + 2 * n])
    np.testing.assert_array_equal(x0[ok], np.clip(P[ok, m + n:m + 2 * n], L, U))
    assert not np.any(y0[5]) and not np.any(w0[5]) and not np.any(x0[5])
    net.close()
    # family features [c; u] and targets [y; z; w] in FP32
    lib = _load()
    B = 7
    c = torch.as_tensor(rng.standard_normal(B * n), dtype=torch.float64, device="cuda")
    u = torch.as_tensor(rng.standard_normal(B * m), dtype=torch.float64, device="cuda")
    Xf = torch.empty((B, n + m), dtype=torch.float32, device="cuda")
    st = _vp(torch.cuda.current_stream().cuda_stream)
    N.check(lib.hprqp_family_features(B, n, m, _p(c), _p(u), _p(Xf), st))
    ref = np.concatenate([c.cpu().numpy().reshape(B, n), u.cpu().numpy().reshape(B, m)], axis=1).astype(np.float32)
    np.testing.assert_array_equal(Xf.cpu().numpy(), ref)
    y = torch.as_tensor(rng.standard_normal(B * m), dtype=torch.float64, device="cuda")
    Tf = torch.empty((B, m + 2 * n), dtype=torch.float32, device="cuda")
    c2 = c * 2                        # held: a temporary's memory would be reused by the next allocation
    N.check(lib.hprqp_family_targets(B, n, m, _p(y), _p(c), _p(c2), None, _p(Tf), st))
    cc = c.cpu().numpy().reshape(B, n)
    ref = np.concatenate([y.cpu().numpy().reshape(B, m), cc, 2 * cc], axis=1).astype(np.float32)
    np.testing.assert_array_equal(Tf.cpu().numpy(), ref)
    its = np.array([0, 1, 2, 100, 800, 3600, 123457], dtype=np.int64)
    Tl = torch.empty((B, m + 2 * n + 1), dtype=torch.float32, device="cuda")
    its_d = torch.as_tensor(its, device="cuda")
    N.check(lib.hprqp_family_targets(B, n, m, _p(y), _p(c), _p(c2), _p(its_d), _p(Tl), st))
    Tl = Tl.cpu().numpy()
    np.testing.assert_array_equal(Tl[:, :-1], ref)
    np.testing.assert_array_max_ulp(Tl[:, -1], np.log(np.maximum(its, 1)).astype(np.float32), maxulp=1)


def test_adam_training_reduces_loss():
    from paper_2507_02470_amd.surrogate import MLP, init_params
    rng = np.random.default_rng(5)
    dims = (40, 64, 64, 30)
    Wt = rng.standard_normal((30, 40)) / 6
    X = rng.standard_normal((512, 40)).astype(np.float32)
    T = np.tanh(X @ Wt.T).astype(np.float32)
    net = MLP(dims, 128, init_params(dims, 3))
    first = None
    for ep in range(60):
        for b0 in range(0, 512, 128):
            L, _ = net.loss_grad(X[b0:b0 + 128], T[b0:b0 + 128], want_grad=False)
            first = L if first is None else first
            net.adam(3e-3)
    L, _ = net.loss_grad(X[:128], T[:128], want_grad=False)
    assert L < 0.1 * first, (first, L)
    net.close()


def test_warm_start_beats_cold_start_on_held_out_family_members():
    """Train on solver-generated solutions (and solve lengths) of a small
    family, then compare warm-started batched solves, queued by the
    predicted length, with cold-started ones in the default order on held-out
    members (both to 1e-8): fewer iterations, and a kernel and wall time
    whose medians over three runs each are lower, the kernel time by more
    than the runs' spread."""
    from paper_2507_02470_amd.surrogate import WarmStartSurrogate, family_features, solve_family, targets_from, \
        warm_vs_cold
    base = qpgen.make_portfolio_family_base(seed=1005, n=200)
    train = [qpgen.portfolio_family_sample(base, 100_000 + j) for j in range(5000)]
    held = [qpgen.portfolio_family_sample(base, 200_000 + j) for j in range(2048)]
    r = solve_family(base, train)
    assert all(f["term"] == "solved" for f in r.infos)
    X = np.stack([family_features(c, u) for (c, l, u) in train])
    T = targets_from(r, len(train), base.n, base.m)
    sur = WarmStartSurrogate(base, hidden=256, max_batch=256, seed=0)
    hist = sur.fit(X, T, epochs=40, batch=128, lr=1e-3, lr_final=1e-5)
    assert hist[-1] < 0.5 * hist[0]
    bool(sur.starts(X[:8])[3].bool().any())     # first use outside the timed runs
    res = warm_vs_cold(sur, held, repeats=3)
    ic, iw = res["iters_cold"], res["iters_warm"]
    print(f"cold mean {ic.mean():.1f} warm mean {iw.mean():.1f} fallback {res['fallback']} pred err w "
          f"{res['pred_rel_err_w']:.2e} y {res['pred_rel_err_y']:.2e}", flush=True)
    print("wall cold", res["wall_cold"], "warm", res["wall_warm"], flush=True)
    print("kernel cold", res["kernel_cold"], "warm", res["kernel_warm"], "cold in the predicted order",
          res["kernel_cold_ordered"], flush=True)
    assert np.all(res["kkt_warm"] <= 1e-8)
    np.testing.assert_allclose(res["obj_warm"], res["obj_cold"], rtol=1e-6, atol=1e-9)
    assert iw.mean() < 0.9 * ic.mean()
    assert res["kernel_warm"]["max"] < res["kernel_cold"]["min"]
    assert res["wall_warm"]["median"] < res["wall_cold"]["median"]
    # fallback: a network that predicts NaN starts every sample from the origin
    p = sur.net.get_params(); p[:] = np.nan
    sur.net.set_params(p)
    res2 = warm_vs_cold(sur, held[:16], repeats=1)
    assert res2["fallback"] == 16
    np.testing.assert_array_equal(res2["iters_warm"], res2["iters_cold"])
