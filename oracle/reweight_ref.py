"""Reference of the canonical reweighting after the weight iteration.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Plain numpy in binary64, written
from the definitions.  Why (Sec. 3): a multicanonical run samples both the
gas-like and the droplet states in one simulation, and canonical averages at
any temperature follow from its data afterwards.

A run with weights W(E) visits energy E with probability proportional to
Omega(E) W(E), so its histogram H(E) estimates the density of states up to
a constant: ln Omega(E) = ln H(E) - ln W(E) on the visited bins (bins with
H(E) = 0 carry no estimate and are left out).  The canonical distribution at
inverse temperature beta (J = 1, k_B = 1) is P_beta(E) proportional to
Omega(E) exp(-beta E); from it
    ln Z(beta)  = ln sum_E exp(ln Omega(E) - beta E)   (same constant as ln Omega),
    <E>         = sum_E E P_beta(E),
    <E^2>       = sum_E E^2 P_beta(E),
    C(beta)     = beta^2 sum_E (E - <E>)^2 P_beta(E)   (specific heat, total).
The sums are shifted by the largest exponent before exp; the variance is
taken about the mean (two passes), not as <E^2> - <E>^2.
"""
import numpy as np


def reweight(lnW, H, e_lo, betas):
    """One group: lnW[b], H[b] for E = e_lo + b.  Returns an array of shape
    (len(betas), 4): ln Z, <E>, <E^2>, C per beta (NaN when no bin is
    visited)."""
    lnW = np.asarray(lnW, dtype=np.float64)
    H = np.asarray(H, dtype=np.int64)
    E = e_lo + np.arange(len(H), dtype=np.float64)
    seen = H > 0
    out = np.full((len(betas), 4), np.nan)
    if not seen.any():
        return out
    ln_omega = np.log(H[seen].astype(np.float64)) - lnW[seen]
    Es = E[seen]
    for k, beta in enumerate(betas):
        a = ln_omega - beta * Es
        m = a.max()
        w = np.exp(a - m)
        z = w.sum()
        mean = (w * Es).sum() / z
        out[k, 0] = m + np.log(z)
        out[k, 1] = mean
        out[k, 2] = (w * Es * Es).sum() / z
        out[k, 3] = beta * beta * (w * (Es - mean) ** 2).sum() / z
    return out


def reweight_observable(lnW, H, Osum, e_lo, betas):
    """Canonical average of an observable O measured during a run with weights
    W: Osum[b] is the sum of O over the H[b] measurements taken at
    E = e_lo + b, so the microcanonical mean is Osum/H on visited bins and
    <O>_beta = sum_E (Osum/H)(E) Omega(E) exp(-beta E) / Z, with the same
    ln Omega and shift as reweight().  Returns an array of len(betas) (NaN
    when no bin is visited)."""
    lnW = np.asarray(lnW, dtype=np.float64)
    H = np.asarray(H, dtype=np.int64)
    Osum = np.asarray(Osum, dtype=np.float64)
    E = e_lo + np.arange(len(H), dtype=np.float64)
    seen = H > 0
    out = np.full(len(betas), np.nan)
    if not seen.any():
        return out
    ln_omega = np.log(H[seen].astype(np.float64)) - lnW[seen]
    mean_o = Osum[seen] / H[seen]
    for k, beta in enumerate(betas):
        a = ln_omega - beta * E[seen]
        w = np.exp(a - a.max())
        out[k] = (w * mean_o).sum() / w.sum()
    return out
