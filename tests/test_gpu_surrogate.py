"""The sweep surrogate end to end on the GPU, at a small scale: replicas
simulated by the library, the network trained by its own kernels, new
points chosen near the percolation line and judged by plain runs.

What the network gains over the method without it (a uniform sweep run the
plain way): the share of plain runs that land near the percolation line,
where the sweep's answer is decided."""

import numpy as np
import pytest

from paper_2609_21204_amd import surrogate as S

pytestmark = pytest.mark.gpu


def test_plain_and_batched_replica_runs_agree():
    pts = S.draw_points(np.random.default_rng(2), 6, "chains", n_range=(256, 600), seed_base=40)
    a = S.simulate(pts, steps=2000, samples=2, plain=False)
    b = S.simulate(pts, steps=2000, samples=2, plain=True)
    assert np.array_equal(a, b)
    assert np.all((a >= 0) & (a <= 1)) and np.all(a[:, 0] > 0)


def test_surrogate_concentrates_plain_runs_on_the_percolation_line():
    rep = S.run_workflow(train_replicas=1024, steps=8000, samples=4, points=64, kinds=("chains",),
                         n_range=(256, 1024), epochs=400, batch=128, pool=16384, uniform_plain=False, seed=3,
                         log=lambda m: None)
    tr, ch, arr = rep["chains"], rep["chosen"], rep["_arrays"]
    # the network learned the bonded fraction of uniform points it never saw
    assert tr["heldout_mae"][0] < 0.03
    # near the line (largest-cluster fraction 0.5 +- 0.1) the chosen points
    # land many times more often than uniform ones
    assert ch["hit_rate_chosen"] >= 0.25
    assert ch["hit_rate_chosen"] >= 5 * ch["hit_rate_uniform"]
    assert ch["plain_runs_saved"] >= 0.8
    assert ch["mae"][0] < 0.05
    # the fallback keeps the plain value wherever an output misses by > 0.02
    miss = np.any(np.abs(arr["pred"] - arr["plain"]) > S.TOLERANCE, axis=1)
    assert np.array_equal(miss, arr["fallback"]) and ch["fallbacks"] == int(miss.sum())
    assert np.array_equal(arr["kept"][miss], arr["plain"][miss])
    assert np.array_equal(arr["kept"][~miss], arr["pred"][~miss])
