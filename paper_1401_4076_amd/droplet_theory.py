"""Analytic droplet fraction (Biskup et al. in the lattice-gas form of Sec. 3).

This is the prediction the droplet measurement (mucaLargestCluster) is
compared with, not a step of the simulation.  A lattice gas of N particles on
V = L^d sites at fixed temperature, with background density rho0, reduced
compressibility kappa (kappa-hat) and surface free energy tau_w of a unit
Wulff droplet, has the particle excess dN = N - rho0 V and the excess
volume V_L = dN / (1 - 2 rho0).  With lambda the fraction of the excess held
by the largest droplet, the free energy is (Sec. 3, eq. (freeEnergy))

    F(lambda) = tau_w (lambda V_L)^((d-1)/d) + (1 - 2 rho0)^2 V_L^2 (1 - lambda)^2 / (2 kappa V)
              = tau_w V_L^((d-1)/d) (lambda^((d-1)/d) + Delta (1 - lambda)^2),

    Delta = (1 - 2 rho0)^2 / (2 kappa tau_w) * V_L^((d+1)/d) / V        (eq. (Delta)).

The equilibrium fraction minimises the bracket over [0, 1]: 0 below the
critical Delta_c, a droplet holding lambda >= lambda_c of the excess above.
With a = (d-1)/d the bracket at its non-zero stationary point equals its
value at 0 exactly when Delta_c = (1/d) ((d+1)/2)^((d+1)/d) and
lambda_c = 2/(d+1) (the values the paper quotes: 0.9186 and 2/3 in 2D, 0.8399
and 1/2 in 3D).  Above Delta_c the bracket is convex on [lambda_c, 1], so the
minimiser is the root of its derivative there (found by bisection).
"""
# Table 1: converted lattice-gas parameters at the temperatures of Sec. 4
# (2D: T = 0.375; 3D: T = 0.5, tau_w ~ 6 sigma / 4 from a low-temperature series)
PARAMS = {
    2: {"T": 0.375, "rho0": 0.00675, "kappa": 0.02708, "tau_w": 1.06125},
    3: {"T": 0.500, "rho0": 0.002739, "kappa": 0.00608, "tau_w": 2.861},
}


def critical(d):
    """(Delta_c, lambda_c) in d dimensions."""
    return (1.0 / d) * ((d + 1) / 2.0) ** ((d + 1) / d), 2.0 / (d + 1)


def bracket(d, lam, Delta):
    """lambda^((d-1)/d) + Delta (1 - lambda)^2: F / (tau_w V_L^((d-1)/d))."""
    return lam ** ((d - 1) / d) + Delta * (1.0 - lam) ** 2


def excess_volume(d, N, L, rho0):
    """V_L = (N - rho0 L^d) / (1 - 2 rho0)."""
    return (N - rho0 * L ** d) / (1.0 - 2.0 * rho0)


def delta(d, N, L, rho0, kappa, tau_w):
    """The dimensionless parameter Delta of N particles on L^d sites."""
    V = float(L) ** d
    VL = excess_volume(d, N, L, rho0)
    return (1.0 - 2.0 * rho0) ** 2 / (2.0 * kappa * tau_w) * VL ** ((d + 1) / d) / V


def fraction(d, Delta, tol=1e-14):
    """Equilibrium droplet fraction lambda(Delta): 0 below Delta_c, else the
    minimiser of the bracket on [lambda_c, 1]."""
    Dc, lc = critical(d)
    if Delta < Dc:
        return 0.0
    a = (d - 1) / d

    def slope(x):
        return a * x ** (a - 1.0) - 2.0 * Delta * (1.0 - x)

    lo, hi = lc, 1.0  # slope(lo) <= 0 < slope(hi) = a
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if slope(mid) <= 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def free_energy(d, lam, N, L, rho0, kappa, tau_w):
    """F(lambda) in its first form (sum of the droplet and fluctuation terms)."""
    V = float(L) ** d
    VL = excess_volume(d, N, L, rho0)
    return (tau_w * (lam * VL) ** ((d - 1) / d)
            + (1.0 - 2.0 * rho0) ** 2 * VL ** 2 * (1.0 - lam) ** 2 / (2.0 * kappa * V))


def transition_size(d, N, rho0, kappa, tau_w):
    """The lattice size L at which N particles reach Delta_c (Delta falls as
    L grows at fixed N), by bisection on L as a real number; None if Delta
    stays below Delta_c for every L with a positive excess."""
    Dc, _ = critical(d)
    hi = (N / rho0) ** (1.0 / d) * (1.0 - 1e-12)  # excess -> 0
    lo = 1.0
    if delta(d, N, lo, rho0, kappa, tau_w) < Dc:
        return None
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if delta(d, N, mid, rho0, kappa, tau_w) >= Dc:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def measured_fraction(d, largest, N, L, rho0):
    """lambda estimated from the particle count of the largest droplet: the
    droplet is read as liquid at density 1 - rho0, so its volume is
    largest / (1 - rho0) and its excess (1 - 2 rho0) times that; divided by
    the total excess N - rho0 L^d."""
    excess = N - rho0 * float(L) ** d
    return (1.0 - 2.0 * rho0) * largest / (1.0 - rho0) / excess
