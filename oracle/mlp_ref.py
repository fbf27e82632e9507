"""Reference of the learned-initial-weights network (test infrastructure).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Plain numpy, written from the
network's definition: 4 -> 128 -> 128 -> 128 -> 1 with SiLU, mean squared
error, Adam.  Two modes:
  * fp64: every quantity in binary64 (for finite-difference checks);
  * bf16: the mixed precision of the GPU kernels emulated: hidden-layer
    weights and hidden activations rounded to bfloat16 (round to nearest,
    ties to even), first-layer inputs and output-layer weights in FP32,
    accumulation in float64 (the GPU accumulates in FP32, so agreement is to
    a tolerance).  Gradients pass straight through the bfloat16 rounding.
Parameter layout: W1[128][4] b1[128] W2[128][128] b2[128] W3[128][128] b3[128]
W4[128] b4.
"""
import numpy as np

SIZES = (4, 128, 128, 128, 1)


def bf16_round(x):
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7F800000) == 0x7F800000
    nan &= (u & 0x007FFFFF) != 0
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(nan, ((u >> 16) | 0x40) << 16, r)
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


def unpack(p):
    p = np.asarray(p)
    out, o = [], 0
    for fi, fo in zip(SIZES[:-1], SIZES[1:]):
        out.append(p[o:o + fi * fo].reshape(fo, fi))
        o += fi * fo
        out.append(p[o:o + fo])
        o += fo
    assert o == p.size
    return out


def pack(parts):
    return np.concatenate([np.ravel(a) for a in parts])


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(p, X, mode="fp64"):
    """Returns (y, cache)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = [np.asarray(a, dtype=np.float64) for a in unpack(p)]
    X = np.asarray(X, dtype=np.float64)
    if mode == "bf16":
        W1, W2, W3 = [bf16_round(a.astype(np.float32)).astype(np.float64) for a in (W1, W2, W3)]
        W4 = W4.astype(np.float32).astype(np.float64)
        X = X.astype(np.float32).astype(np.float64)
    zs, acts = [], [X]
    a = X
    for W, b in ((W1, b1), (W2, b2), (W3, b3)):
        z = a @ W.T + b
        h = z * _sig(z)
        if mode == "bf16":
            h = bf16_round(h.astype(np.float32)).astype(np.float64)
        zs.append(z)
        acts.append(h)
        a = h
    y = (a @ W4.T + b4)[:, 0]
    return y, (zs, acts, (W1, W2, W3, W4))


def loss_and_grad(p, X, T, mode="fp64"):
    """Mean squared error and its gradient w.r.t. the flat parameters."""
    y, (zs, acts, (W1, W2, W3, W4)) = forward(p, X, mode)
    T = np.asarray(T, dtype=np.float64)
    n = len(T)
    e = y - T
    loss = float(np.mean(e * e))
    dy = 2.0 * e / n
    gW4 = (dy[:, None] * acts[3]).sum(axis=0)[None, :]
    gb4 = np.array([dy.sum()])
    dz = (dy[:, None] * W4) * _silu_grad(zs[2])
    grads = []
    for layer, W in ((2, W3), (1, W2), (0, W1)):
        gW = dz.T @ acts[layer]
        gb = dz.sum(axis=0)
        grads.append((gW, gb))
        if layer > 0:
            dz = (dz @ W) * _silu_grad(zs[layer - 1])
    (gW3, gb3), (gW2, gb2), (gW1, gb1) = grads
    return loss, pack([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4])


def _silu_grad(z):
    s = _sig(z)
    return s * (1.0 + z * (1.0 - s))


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
