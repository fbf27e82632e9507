"""Pins of the element-wise tolerances used by the GPU tests of the network
(tests/mlp_envelope.py): an independent FP32 evaluation of the network stays
inside them, and planted mistakes in that evaluation's gradient (a sign, a
transposed block, a dropped activation derivative) fall outside them."""
import numpy as np
import pytest

import workloads as W
from oracle import mlp_ref as R

import mlp_envelope as E


def _case(rows, seed):
    p = W.mlp_init_params(seed)
    X, T = W.mlp_synthetic_rows(rows, seed + 1)
    y_ref, _ = R.forward(p.astype(np.float64), X, "bf16")
    _, g_ref = R.loss_and_grad(p.astype(np.float64), X, T, "bf16")
    return p, X, T, y_ref, g_ref


@pytest.mark.parametrize("rows,seed", [(1, 13), (17, 13), (700, 13), (2000, 21), (300, 5)])
def test_fp32_evaluation_is_inside_the_tolerances(rows, seed):
    p, X, T, y_ref, g_ref = _case(rows, seed)
    y32, g32 = E.fp32_forward_backward(p, X, T)
    tol = E.grad_tolerance(p, X, T, g_ref)
    ytol = E.output_tolerance(p, X, T, y_ref)
    assert np.all(np.abs(g32 - g_ref) <= tol), np.max(np.abs(g32 - g_ref) / tol)
    assert np.all(np.abs(y32 - y_ref) <= ytol), np.max(np.abs(y32 - y_ref) / ytol)
    # margin: the observed deviations use well under half of the allowance
    assert np.max(np.abs(g32 - g_ref) / tol) < 0.5


@pytest.mark.parametrize("rows,seed", [(17, 13), (700, 13)])
def test_planted_mistakes_fall_outside(rows, seed):
    p, X, T, y_ref, g_ref = _case(rows, seed)
    _, g32 = E.fp32_forward_backward(p, X, T)
    tol = E.grad_tolerance(p, X, T, g_ref)
    # a sign error in any single entry is caught for nearly every entry
    caught = np.abs(-g32 - g_ref) > tol
    assert caught.mean() > 0.99, caught.mean()
    for blk, c in enumerate(R.unpack(caught)):
        assert c.mean() > 0.95, (blk, c.mean())
    # a transposed hidden weight gradient (W2 block)
    parts = R.unpack(g32.copy())
    parts[2] = parts[2].T.copy()
    off = ~np.eye(128, dtype=bool)
    bad = np.abs(parts[2] - R.unpack(g_ref)[2]) > R.unpack(tol)[2]
    assert bad[off].mean() > 0.9, bad[off].mean()
    # swapping two entries of a bias gradient
    parts = R.unpack(g32.copy())
    i, j = np.argmax(parts[3]), np.argmin(parts[3])
    parts[3][[i, j]] = parts[3][[j, i]]
    assert np.any(np.abs(R.pack(parts) - g_ref) > tol)
    # a dropped activation derivative in the first hidden layer
    y, (zs, acts, (W1, W2, W3, W4)) = R.forward(p.astype(np.float64), X, "bf16")
    n = len(T)
    dY = 2.0 * (y - np.asarray(T, np.float64)) / n
    sg = E._silu_grad
    dz3 = dY[:, None] * W4 * sg(zs[2])
    dz2 = (dz3 @ W3) * sg(zs[1])
    dz1_wrong = dz2 @ W2  # silu'(z1) left out
    gW1_wrong = dz1_wrong.T @ acts[0]
    gW1_tol = R.unpack(tol)[0]
    assert np.mean(np.abs(gW1_wrong - R.unpack(g_ref)[0]) > gW1_tol) > 0.9
