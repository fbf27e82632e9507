"""Element-wise tolerances for the network's outputs and gradients.

TEST INFRASTRUCTURE.  The GPU kernels evaluate the network with BF16 weights
and activations and FP32 arithmetic; the reference (oracle/mlp_ref.py, mode
"bf16") rounds the same quantities to BF16 but computes everything else in
binary64.  They differ in two ways:

  * FP32 rounding.  Every product, sum, exp and division of the GPU rounds
    with unit roundoff u = 2^-24; a sum of n terms is within n u (worst
    case; about sqrt(n) u in practice) of its exact value, relative to the
    sum of the terms' magnitudes.
  * BF16 flips.  Round-to-nearest-even errs by at most 2^-8 of the value, so
    when an activation's FP32 value lies within its FP32 error of the
    midpoint between two BF16 numbers, the GPU may pick the other neighbour:
    a difference of one BF16 ulp, at most 2^-7 of the activation.  Such
    flips are rare (about 1e-4 to 1e-3 of the activations at these sizes)
    and change one row's term of the sums they enter; downstream in the same
    row they shift pre-activations by |W| ulp, a relative change far below
    2^-7.

Every parameter-gradient entry g_e is a sum over rows of terms
t_r = dz_r a_r (dz: the loss derivative at a unit's pre-activation, or
dL/dy for the output layer; a: the activation or input it multiplies, or 1
for a bias).  From the reference's own values, let M_e = max_r |t_r| and
S_e = sum_r |t_r|.  The tolerance

    |g_gpu - g_ref| <= 2^-10 |g_ref| + 2^-6 M_e + 2^-14 S_e

allows two flipped activations in the entry's sum, each moving one term by
one BF16 ulp (2 x 2^-7 M_e); a relative perturbation of 2^-14 (~8 worst-case
128-term FP32 sums) of every term, which covers FP32 summation in any order
and the downstream shifts of flips elsewhere in a row; and a few FP32 ulps
of the entry itself (2^-10 |g_ref|).  Outputs y = W4 a3 + b4 get
2^-10 |y_ref| + 2^-8 S_y with S_y = sum_k |W4_k a3_k| + |b4| (a quarter of a
row's terms flipped).

A sign error, a swapped index or a dropped factor moves an entry by about
its own size; tests/test_mlp_envelope.py checks that such planted mistakes
fall outside these tolerances for nearly every entry, and that an
independent FP32 evaluation of the network stays inside them.
"""
import numpy as np

from oracle import mlp_ref as R

RTOL = 2.0 ** -10
FLIPS = 2.0 ** -6
PERTURB = 2.0 ** -14
Y_TERMS = 2.0 ** -8


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def _silu_grad(z):
    s = _sig(z)
    return s * (1.0 + z * (1.0 - s))


def terms(p, X, T):
    """Per gradient entry (flat parameter layout): (M, S) = (largest, sum of)
    |row term|, and per output row S_y; from the bf16-mode reference."""
    y, (zs, acts, (W1, W2, W3, W4)) = R.forward(np.asarray(p, dtype=np.float64), X, "bf16")
    T = np.asarray(T, dtype=np.float64)
    n = len(T)
    dY = 2.0 * (y - T) / n
    dz3 = dY[:, None] * W4 * _silu_grad(zs[2])
    dz2 = (dz3 @ W3) * _silu_grad(zs[1])
    dz1 = (dz2 @ W2) * _silu_grad(zs[0])
    Ms, Ss = [], []
    for dz, a in ((dz1, acts[0]), (dz2, acts[1]), (dz3, acts[2]), (dY[:, None], acts[3])):
        ad, aa = np.abs(dz), np.abs(a)
        Ms.append(np.max(ad[:, :, None] * aa[:, None, :], axis=0))
        Ms.append(ad.max(axis=0))
        Ss.append(ad.T @ aa)
        Ss.append(ad.sum(axis=0))
    b4 = R.unpack(np.asarray(p, dtype=np.float64))[7]
    Sy = np.abs(acts[3]) @ np.abs(W4[0]) + abs(b4[0])
    return R.pack(Ms), R.pack(Ss), Sy


def grad_tolerance(p, X, T, g_ref):
    M, S, _ = terms(p, X, T)
    return RTOL * np.abs(g_ref) + FLIPS * M + PERTURB * S


def output_tolerance(p, X, T, y_ref):
    _, _, Sy = terms(p, X, T)
    return RTOL * np.abs(y_ref) + Y_TERMS * Sy


def fp32_forward_backward(p, X, T):
    """An FP32 evaluation of the network written independently of the GPU
    kernels (numpy float32 arithmetic, BF16 weights and activations, exp in
    float32, numpy's own summation order): used only to check that the
    tolerances cover a plausible FP32 implementation.  Returns (y, grad) in
    float64."""
    f = np.float32
    W1, b1, W2, b2, W3, b3, W4, b4 = [np.asarray(a, dtype=np.float32) for a in R.unpack(p)]
    Wb = [R.bf16_round(W) for W in (W1, W2, W3)]
    x = np.asarray(X, dtype=np.float32)
    T = np.asarray(T, dtype=np.float32)
    n = len(T)

    def sig(z):
        return f(1.0) / (f(1.0) + np.exp(-z))

    zs, acts = [], [x]
    a = x
    for W, b in zip(Wb, (b1, b2, b3)):
        z = (a @ W.T + b).astype(np.float32)
        a = R.bf16_round(z * sig(z))
        zs.append(z)
        acts.append(a)
    y = (a @ W4[0] + b4[0]).astype(np.float32)
    dY = (f(2.0) * (y - T) / f(n)).astype(np.float32)

    def sg(z):
        s = sig(z)
        return s * (f(1.0) + z * (f(1.0) - s))

    dz = (dY[:, None] * W4[0][None, :]) * sg(zs[2])
    dZ = {2: dz}
    for l, W in ((2, Wb[2]), (1, Wb[1])):
        dz = ((dz @ W) * sg(zs[l - 1])).astype(np.float32)
        dZ[l - 1] = dz
    parts = []
    for l in range(3):
        parts.append(dZ[l].T @ acts[l])
        parts.append(dZ[l].sum(axis=0))
    parts.append(dY[:, None].T @ acts[3])
    parts.append(np.array([dY.sum()], dtype=np.float32))
    return y.astype(np.float64), R.pack([np.asarray(q, dtype=np.float32) for q in parts]).astype(
        np.float64)
