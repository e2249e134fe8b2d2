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


def test_replicas_of_a_point_average_into_its_label():
    pts = S.draw_points(np.random.default_rng(4), 3, "mono", n_range=(256, 400), seed_base=70)
    rep = S.replicas_of(pts, 2)
    assert len(rep) == 6 and np.array_equal(rep.eps[3:], pts.eps) and np.array_equal(rep.seed[3:], pts.seed + S.SEED_STRIDE)
    one = S.simulate(rep, steps=800, samples=2)
    both = S.simulate(pts, steps=800, samples=2, seeds=2)
    assert np.allclose(both, 0.5 * (one[:3] + one[3:]), rtol=0, atol=1e-15)


def test_surrogate_concentrates_plain_runs_on_the_percolation_line():
    """Labels are 4-replica averages; the bonded fraction predicted at the
    chosen points meets the 0.02 bar on average against the simulation."""
    rep = S.run_workflow(train_replicas=2048, steps=8000, samples=4, points=64, kinds=("chains",),
                         n_range=(256, 1024), epochs=400, batch=128, pool=16384, uniform_plain=False, seed=3,
                         log=lambda m: None, seeds=4)
    tr, ch, arr = rep["chains"], rep["chosen"], rep["_arrays"]
    print({k: v for k, v in ch.items()}, flush=True)
    # the network learned the bonded fraction of uniform points it never saw
    assert tr["heldout_mae"][0] < 0.03
    # near the line (largest-cluster fraction 0.5 +- 0.1) the chosen points
    # land many times more often than uniform ones
    assert ch["hit_rate_chosen"] >= 0.25
    assert ch["hit_rate_chosen"] >= 5 * ch["hit_rate_uniform"]
    assert ch["plain_runs_saved"] >= 0.8
    # bonded fraction at the chosen points: mean error within the 0.02 bar
    assert ch["mae"][0] <= S.TOLERANCE
    # the fallback keeps the plain value wherever an output misses by > 0.02
    miss = np.any(np.abs(arr["pred"] - arr["plain"]) > S.TOLERANCE, axis=1)
    assert np.array_equal(miss, arr["fallback"]) and ch["fallbacks"] == int(miss.sum())
    assert np.array_equal(arr["kept"][miss], arr["plain"][miss])
    assert np.array_equal(arr["kept"][~miss], arr["pred"][~miss])
