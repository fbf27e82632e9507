"""Host logic of the scaling driver (no GPU): the sweeps must split evenly
over the walkers, and the speed-ups relative to the smallest p run:
S = p x iters(p0) / iters(p) (iteration model) and S = p0 x t(p0) / t(p)
(measured run times), both equal to p for a linear speed-up."""
import pytest

from paper_1401_4076_amd import scaling as S


def test_uneven_split_is_refused_before_any_device_work():
    with pytest.raises(ValueError):
        S.runs_for(2, 8, 16, 3, 2, 1, 25600, 30, 10, 0)


def test_speedups():
    res = [{"p": 1, "iters_mean": 6.0, "seconds_mean": 12.0},
           {"p": 4, "iters_mean": 3.0, "seconds_mean": 2.0},
           {"p": 8, "iters_mean": 6.0, "seconds_mean": 1.5}]
    assert S.speedups(res) == [(1.0, 1.0), (8.0, 6.0), (8.0, 8.0)]
    # relative to the smallest p run: p0 = 4 keeps S_p0 = 4
    assert S.speedups(res[1:]) == [(4.0, 4.0), (4.0, 4 * 2.0 / 1.5)]
