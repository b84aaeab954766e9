"""Pins of the FP64 MLP reference (oracle/mlp.py) against facts outside it:
central finite differences of the loss, closed forms of GELU, and an
independent BF16 conversion (torch)."""
import numpy as np
import pytest
import torch

from oracle import mlp as M


def test_bf16_rounding_matches_torch_and_hand_values():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-6, 6, 5000),
                        [0.0, -0.0, 1.0, 3.0, 0.1, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x), ref)
    assert M.bf16(0.1) == 0.10009765625           # 1.1001101b x 2^-4
    assert M.bf16(1 + 2 ** -8) == 1.0             # tie -> even
    assert M.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6  # tie -> even (upwards)


def test_gelu_closed_forms():
    assert M.gelu(0.0) == 0.0
    assert M.gelu_d(0.0) == 0.5
    assert M.gelu(8.0) == pytest.approx(8.0, rel=1e-14)
    assert M.gelu(-8.0) == pytest.approx(0.0, abs=1e-13)
    z = np.linspace(-5, 5, 41)
    h = 1e-6
    np.testing.assert_allclose(M.gelu_d(z), (M.gelu(z + h) - M.gelu(z - h)) / (2 * h), rtol=1e-8, atol=1e-9)
    # Phi(1) = 0.8413447460685429...
    assert M.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-14)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    dims = (7, 5, 6, 4)
    p = rng.standard_normal(M.num_params(dims)) * 0.5
    X = rng.standard_normal((3, 7)); T = rng.standard_normal((3, 4)); w = rng.uniform(0.5, 2, 4)
    mi, si = rng.standard_normal(7), rng.uniform(0.5, 2, 7)
    mo, so = rng.standard_normal(4), rng.uniform(0.5, 2, 4)
    kw = dict(w=w, emulate=False, in_mean=mi, in_std=si, out_mean=mo, out_std=so)
    L, g = M.loss_grad(p, X, T, dims, **kw)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p); e[i] = h
        fd[i] = (M.loss_grad(p + e, X, T, dims, **kw)[0] - M.loss_grad(p - e, X, T, dims, **kw)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_emulated_forward_is_close_to_fp64():
    rng = np.random.default_rng(2)
    dims = (30, 16, 16, 10)
    p = rng.standard_normal(M.num_params(dims)) * 0.3
    X = rng.standard_normal((8, 30))
    Ye, _ = M.forward(p, X, dims, emulate=True)
    Yf, _ = M.forward(p, X, dims, emulate=False)
    rel = np.linalg.norm(Ye - Yf) / np.linalg.norm(Yf)
    assert 0 < rel < 2e-2          # BF16 operands: ~2^-9 relative per rounding
