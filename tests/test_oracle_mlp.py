"""Pins of the learned-initial-weights reference (oracle/mlp_ref.py):
bfloat16 rounding against torch's conversion, the FP64 gradient against
central finite differences, and the Adam step against its closed form for
the first step."""
import numpy as np
import pytest

import workloads as W
from oracle import mlp_ref as R

torch = pytest.importorskip("torch")


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 100000), rng.normal(0, 1e-30, 1000),
                        rng.normal(0, 1e30, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -3.0e38, 1e-40,
                         np.inf, -np.inf]]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = R.bf16_round(x)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_fp64_gradient_matches_finite_differences():
    p = W.mlp_init_params(3).astype(np.float64)
    X, T = W.mlp_synthetic_rows(24, 4)
    _, g = R.loss_and_grad(p, X, T)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(p.size, 300, replace=False), np.arange(p.size - 129, p.size)])
    h = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += h
        lp, _ = R.loss_and_grad(q, X, T)
        q[i] -= 2 * h
        lm, _ = R.loss_and_grad(q, X, T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(6)
    p = rng.normal(size=1000)
    g = rng.normal(size=1000)
    lr = 1e-3
    p1, m, v = R.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_mode_is_close_to_fp64():
    p = W.mlp_init_params(7).astype(np.float64)
    X, T = W.mlp_synthetic_rows(64, 8)
    l64, g64 = R.loss_and_grad(p, X, T, "fp64")
    l16, g16 = R.loss_and_grad(p, X, T, "bf16")
    assert abs(l16 - l64) < 0.02 * l64
    assert np.dot(g16, g64) / np.linalg.norm(g16) / np.linalg.norm(g64) > 0.99
