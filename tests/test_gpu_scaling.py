"""The scaling driver on the GPU against the oracle: the same runs (groups of
one context, seed, sweeps, tunnelling target) stop after the same number of
iterations with the same tunnelling counts, although the driver splits the
run into resumed chunks."""
import numpy as np
import pytest

import oracle as O

pytest.importorskip("torch")
S = pytest.importorskip("paper_1401_4076_amd.scaling")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,L,N,p", [(2, 4, 3, 4), (3, 3, 3, 2)])
def test_runs_match_oracle(d, L, N, p):
    runs, total, target = 3, 40, 60  # 5-6 iterations, over two resumed chunks
    print("scaling", d, L, N, p, flush=True)
    res = S.runs_for(d, L, N, p, runs, 1, total, target, 60, 3, 0)
    ref = O.RefContext([(d, L, N, p)] * runs, 1)
    lnW, P = ref.zeros_lnW(), ref.zeros_lnW()
    rc, H, it, fl = ref.run(lnW, P, total // p, 60, 0, tunnel_target=target)
    assert rc == 0 and res["converged"] == runs
    assert res["iters"] == [int(x) for x in it]
    trips = ref.tunnel()[1]
    assert res["trips"] == [int(trips[r * p:(r + 1) * p].sum()) for r in range(runs)]
    assert np.isfinite(res["iters_mean"])
