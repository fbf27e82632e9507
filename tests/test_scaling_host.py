"""Host logic of the scaling driver (no GPU): the sweeps must split evenly
over the walkers, and S_p = p x (mean iterations at p = 1) / (mean at p)."""
import pytest

from paper_1401_4076_amd import scaling as S


def test_uneven_split_is_refused_before_any_device_work():
    with pytest.raises(ValueError):
        S.runs_for(2, 8, 16, 3, 2, 1, 25600, 30, 10, 5, 0)


def test_speedups():
    res = [{"p": 1, "iters_mean": 6.0}, {"p": 4, "iters_mean": 3.0}, {"p": 8, "iters_mean": 6.0}]
    assert S.speedups(res) == [1.0, 8.0, 8.0]
    assert S.speedups(res[1:]) == [None, None]
