"""Pins of the analytic droplet fraction (Sec. 3).

* The critical point against the values the paper prints
  (tests/golden/droplet_critical.txt).
* At Delta_c the two minima of the bracket are equal and the droplet one is a
  stationary point (the defining property of the closed form).
* The minimiser agrees with a brute-force search over a fine grid of lambda.
* The two forms of the free energy in the paper (the sum of droplet and
  fluctuation terms, and tau_w V_L^((d-1)/d) times the bracket with Delta)
  agree for random particle numbers, lattice sizes and fractions with the
  Table 1 parameters: a wrong exponent or factor in Delta fails this.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_1401_4076_amd import droplet_theory as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "droplet_critical.txt")


def _golden():
    rows = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            d, Dc, lc = line.split()
            rows[int(d)] = (float(Dc), float(Fraction(lc)))
    return rows


@pytest.mark.parametrize("d", [2, 3])
def test_critical_point_matches_paper(d):
    Dc, lc = T.critical(d)
    gD, gl = _golden()[d]
    assert abs(Dc - gD) < 5e-5 and lc == pytest.approx(gl, abs=1e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_critical_point_is_a_double_minimum(d):
    Dc, lc = T.critical(d)
    a = (d - 1) / d
    assert T.bracket(d, lc, Dc) == pytest.approx(T.bracket(d, 0.0, Dc), rel=1e-14)
    assert a * lc ** (a - 1) - 2 * Dc * (1 - lc) == pytest.approx(0.0, abs=1e-14)
    assert T.fraction(d, Dc * (1 - 1e-9)) == 0.0
    assert T.fraction(d, Dc) == pytest.approx(lc, abs=1e-6)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("Delta", [0.5, 0.95, 1.0, 1.3, 2.0, 5.0, 40.0])
def test_minimiser_matches_grid_search(d, Delta):
    lam = np.linspace(0.0, 1.0, 2_000_001)
    f = lam ** ((d - 1) / d) + Delta * (1 - lam) ** 2
    best = lam[np.argmin(f)]
    assert T.fraction(d, Delta) == pytest.approx(best, abs=2e-6)


@pytest.mark.parametrize("d", [2, 3])
def test_fraction_grows_to_one(d):
    Dc, lc = T.critical(d)
    xs = [T.fraction(d, Dc * (1 + k / 10)) for k in range(1, 30)]
    assert all(b > a for a, b in zip(xs, xs[1:])) and xs[0] > lc
    assert T.fraction(d, 1e8) == pytest.approx(1.0, abs=1e-5)


@pytest.mark.parametrize("d", [2, 3])
def test_two_forms_of_the_free_energy_agree(d):
    p = T.PARAMS[d]
    rng = np.random.default_rng(d)
    for _ in range(50):
        L = int(rng.integers(20, 200))
        N = int(p["rho0"] * L ** d + rng.integers(10, 2000))
        lam = float(rng.random())
        D = T.delta(d, N, L, p["rho0"], p["kappa"], p["tau_w"])
        VL = T.excess_volume(d, N, L, p["rho0"])
        second = p["tau_w"] * VL ** ((d - 1) / d) * T.bracket(d, lam, D)
        first = T.free_energy(d, lam, N, L, p["rho0"], p["kappa"], p["tau_w"])
        assert first == pytest.approx(second, rel=1e-12)


@pytest.mark.parametrize("d,N", [(2, 1000), (3, 1000)])
def test_transition_size(d, N):
    p = T.PARAMS[d]
    Lc = T.transition_size(d, N, p["rho0"], p["kappa"], p["tau_w"])
    assert Lc is not None
    Dc, _ = T.critical(d)
    assert T.delta(d, N, Lc, p["rho0"], p["kappa"], p["tau_w"]) == pytest.approx(Dc, rel=1e-9)
    assert T.delta(d, N, Lc * 0.99, p["rho0"], p["kappa"], p["tau_w"]) > Dc


@pytest.mark.parametrize("d", [2, 3])
def test_measured_fraction_reads_the_droplet_as_liquid(d):
    p = T.PARAMS[d]
    N, L = 1000, 40 if d == 3 else 200
    VL = T.excess_volume(d, N, L, p["rho0"])
    # a droplet of volume V_L at the liquid density holds the whole excess
    assert T.measured_fraction(d, VL * (1 - p["rho0"]), N, L, p["rho0"]) == pytest.approx(1.0)
    assert T.measured_fraction(d, 0, N, L, p["rho0"]) == 0.0


def test_table1_constants_follow_their_stated_origins():
    """Table 1 re-derived from how Sec. 4 says its values were obtained, so a
    mistyped constant fails: the lattice-gas temperature is the Ising one over
    4 (T^I = 1.5 in 2D, 2 in 3D); in 2D the background density is
    rho0 = (1 - m0) / 2 with the Ising spontaneous magnetisation, here Yang's
    exact m0 = (1 - sinh(2 / T^I)^-4)^(1/8) (0.0067502 against the printed
    0.00675); in 3D tau_W = 6 sigma / 4 with the interface tension
    sigma = 1.9072 of the low-temperature series (2.8608, printed ~2.861)."""
    P = T.PARAMS
    assert P[2]["T"] == 1.5 / 4 and P[3]["T"] == 2.0 / 4
    m0 = (1.0 - np.sinh(2.0 / 1.5) ** -4) ** 0.125
    assert abs((1.0 - m0) / 2.0 - P[2]["rho0"]) < 5e-7
    assert abs(6.0 * 1.9072 / 4.0 - P[3]["tau_w"]) < 5e-4


def test_table1_2d_surface_free_energy_from_the_exact_crystal_shape():
    """The 2D tau_W of Table 1 (1.06125), rescaled like the temperature
    (Sec. 4: tau_W = tau_W^I / 4), from the exact equilibrium crystal shape of
    the square-lattice Ising model at T^I = 1.5 (J = 1): the Wulff shape
    W = {cosh(x / T) + cosh(y / T) <= cosh(2 / T) coth(2 / T)} (Rottman and
    Wortis; Avron, van Beijeren, Schulman and Zia), whose half-width on an
    axis is Onsager's interface tension 2 + T ln tanh(1 / T); by Wulff's
    theorem the least boundary free energy of a droplet of area V is
    2 sqrt(|W| V), so tau_W^I = 2 sqrt(|W|)."""
    from scipy import integrate
    TI = 1.5
    C = np.cosh(2.0 / TI) / np.tanh(2.0 / TI)
    half = np.arccosh(C - 1.0) * TI
    assert abs(half - (2.0 + TI * np.log(np.tanh(1.0 / TI)))) < 1e-12
    area, _ = integrate.quad(
        lambda x: 2.0 * TI * np.arccosh(max(1.0, C - np.cosh(x / TI))), -half, half, limit=200)
    tau_w = 2.0 * np.sqrt(area) / 4.0
    assert abs(tau_w - T.PARAMS[2]["tau_w"]) < 2e-4  # 1.061353 against 1.06125
