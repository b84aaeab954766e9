"""GPU tests of the BF16-MFMA warm-start network.

Tolerances (derived in the design notes): GEMM with BF16-exact inputs within
the recursive-summation bound K 2^-24 (|A||B|)_ij of FP32 accumulation;
network output and gradients within 2e-3 / 5e-3 relative (Frobenius) of the
FP64 reference that rounds the same operands to BF16 (the remaining gap is
FP32-vs-FP64 accumulation and the rare BF16 rounding it flips)."""
import numpy as np
import pytest

import oracle.mlp as OM
import qpgen

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


@pytest.mark.parametrize("M,N,K,transA,transB", [(64, 64, 16, 0, 0), (100, 37, 51, 0, 0), (1, 2021, 512, 0, 1),
                                                 (256, 512, 1024, 0, 0), (513, 129, 24, 1, 1), (33, 65, 1000, 1, 0)])
def test_gemm_bf16_against_numpy(M, N, K, transA, transB):
    from paper_2507_02470_amd.surrogate import gemm_bf16
    rng = np.random.default_rng(M * 7 + N)
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
    gemm_bf16(Ab, a_rs, a_cs, Bb, b_rs, b_cs, M, N, K, Cout, N)
    ref = Ae @ Be
    bound = K * 2.0 ** -24 * (np.abs(Ae) @ np.abs(Be)) + 1e-30
    err = np.abs(Cout.cpu().numpy().astype(np.float64) - ref)
    assert np.all(err <= bound), float((err / bound).max())


DIMS = (1021, 512, 512, 2021)


def _net(params, batch, scaling):
    from paper_2507_02470_amd.surrogate import MLP
    net = MLP(DIMS, batch, params)
    net.set_scaling(*scaling)
    return net


def _scaling(rng):
    return (rng.standard_normal(DIMS[0]).astype(np.float32), rng.uniform(0.5, 2, DIMS[0]).astype(np.float32),
            rng.standard_normal(DIMS[3]).astype(np.float32), rng.uniform(0.5, 2, DIMS[3]).astype(np.float32))


def test_forward_matches_fp64_reference():
    from paper_2507_02470_amd.surrogate import init_params
    rng = np.random.default_rng(3)
    p = init_params(DIMS, seed=1)
    sc = _scaling(rng)
    X = rng.standard_normal((48, DIMS[0])).astype(np.float32)
    net = _net(p, 64, sc)
    Y = net.forward(X).cpu().numpy().astype(np.float64)
    Ys, _ = OM.forward(p, X, DIMS, emulate=True, in_mean=sc[0], in_std=sc[1])
    Yref = sc[2] + sc[3] * Ys
    rel = np.linalg.norm(Y - Yref) / np.linalg.norm(Yref)
    print("forward rel err", rel, flush=True)
    assert rel <= 2e-3
    net.close()


def test_gradient_matches_fp64_reference():
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
    Lr, gr = OM.loss_grad(p, X, T, DIMS, w=w, emulate=True, in_mean=sc[0], in_std=sc[1], out_mean=sc[2],
                          out_std=sc[3])
    assert L == pytest.approx(Lr, rel=1e-4)
    parts, parts_r = OM.unpack(g, DIMS), OM.unpack(gr, DIMS)
    for name, a, b in zip(("W1", "b1", "W2", "b2", "W3", "b3"), parts, parts_r):
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        print("grad", name, rel, flush=True)
        assert rel <= 5e-3, (name, rel)
    net.close()


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
    """Train on solver-generated solutions of a small family, then compare
    warm- and cold-started batched solves on held-out members (both to 1e-8)."""
    from paper_2507_02470_amd.surrogate import WarmStartSurrogate, family_features, solve_family, targets_from, \
        warm_vs_cold
    base = qpgen.make_portfolio_family_base(seed=1005, n=200)
    train = [qpgen.portfolio_family_sample(base, 100_000 + j) for j in range(3000)]
    held = [qpgen.portfolio_family_sample(base, 200_000 + j) for j in range(256)]
    r = solve_family(base, train)
    assert all(f["term"] == "solved" for f in r.infos)
    X = np.stack([family_features(c, u) for (c, l, u) in train])
    T = targets_from(r, len(train), base.n, base.m)
    sur = WarmStartSurrogate(base, hidden=256, max_batch=256, seed=0)
    hist = sur.fit(X, T, epochs=40, batch=128, lr=2e-3, lr_final=2e-5)
    assert hist[-1] < 0.5 * hist[0]
    res = warm_vs_cold(sur, held)
    ic, iw = res["iters_cold"], res["iters_warm"]
    print(f"cold mean {ic.mean():.1f} warm mean {iw.mean():.1f} fallback {res['fallback']} pred err "
          f"{res['pred_rel_err_w']:.2e} t_cold {res['t_cold_s']:.3f} t_warm {res['t_warm_s']:.3f}", flush=True)
    assert np.all(res["kkt_warm"] <= 1e-8)
    np.testing.assert_allclose(res["obj_warm"], res["obj_cold"], rtol=1e-6, atol=1e-9)
    assert iw.mean() < 0.9 * ic.mean()
    # fallback: a network that predicts NaN starts every sample from the origin
    p = sur.net.get_params(); p[:] = np.nan
    sur.net.set_params(p)
    res2 = warm_vs_cold(sur, held[:16])
    assert res2["fallback"] == 16
    np.testing.assert_array_equal(res2["iters_warm"], res2["iters_cold"])
