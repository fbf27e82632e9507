"""The scaling driver on the GPU against the oracle: the same runs (groups of
one context, seed, first walker id, sweeps, tunnelling target) stop after the
same number of iterations with the same tunnelling counts, although the
driver steps the run one resumed iteration at a time; every converged run
has a measured wall time."""
import numpy as np
import pytest

import oracle as O

pytest.importorskip("torch")
S = pytest.importorskip("paper_1401_4076_amd.scaling")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,L,N,p,first", [(2, 4, 3, 4, 0), (3, 3, 3, 2, 96)])
def test_runs_match_oracle(d, L, N, p, first):
    runs, total, target = 3, 40, 60  # 5-6 iterations, one resumed call each
    print("scaling", d, L, N, p, flush=True)
    res = S.runs_for(d, L, N, p, runs, 1, total, target, 60, 0, first_id=first)
    ref = O.RefContext([(d, L, N, p)] * runs, 1, first_id=first)
    lnW, P = ref.zeros_lnW(), ref.zeros_lnW()
    rc, H, it, fl = ref.run(lnW, P, total // p, 60, 0, tunnel_target=target)
    assert rc == 0 and res["converged"] == runs
    assert res["iters"] == [int(x) for x in it]
    trips = ref.tunnel()[1]
    assert res["trips"] == [int(trips[r * p:(r + 1) * p].sum()) for r in range(runs)]
    assert np.isfinite(res["iters_mean"])
    assert len(res["run_seconds"]) == runs and all(t > 0 for t in res["run_seconds"])
    assert res["first_id"] == first
