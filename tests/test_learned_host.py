"""Host helpers of the learned-weights comparison (paper_1401_4076_amd/learned.py)."""
import math

import numpy as np

from paper_1401_4076_amd import learned as LR


def test_ln_omega_difference_ignores_offsets_and_unvisited_bins():
    a = np.array([0.0, -1.0, np.nan, -3.0, -7.0])
    b = a + 12.5  # ln Omega is known up to a constant
    assert LR.ln_omega_difference(a, b) == (0.0, 4)
    b = b.copy()
    b[4] += 2.0  # one bin off by 2: the mean offset absorbs 2/4 of it
    d, n = LR.ln_omega_difference(a, b)
    assert n == 4 and abs(d - 1.5) < 1e-12
    b[1] = np.nan  # visited by one arm only
    d, n = LR.ln_omega_difference(a, b)
    assert n == 3 and abs(d - 4.0 / 3.0) < 1e-12


def test_ln_omega_difference_without_common_bins():
    d, n = LR.ln_omega_difference([np.nan, 1.0], [2.0, np.nan])
    assert math.isnan(d) and n == 0
