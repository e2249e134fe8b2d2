"""Host-side logic of the sweep surrogate (no GPU): input scaling, point
draws, the initial weights, point choice, judging with fallback."""

import numpy as np

from paper_2609_21204_amd import surrogate as S


def test_features_map_the_ranges_onto_unit_interval():
    lo = S.Points(np.array([2.0]), np.array([0.05]), np.array([1]), np.array([0.8]), np.array([256]),
                  np.array([0]), "chains")
    hi = S.Points(np.array([10.0]), np.array([0.4]), np.array([4]), np.array([1.2]), np.array([8192]),
                  np.array([0]), "chains")
    assert np.allclose(lo.features(), -1.0) and np.allclose(hi.features(), 1.0)
    mid = S.Points(np.array([6.0]), np.array([0.225]), np.array([2]), np.array([1.0]), np.array([1000]),
                   np.array([0]), "chains")
    assert np.allclose(mid.features(), 0.0, atol=1e-7)


def test_draw_points_stay_in_range_and_repeat():
    a = S.draw_points(np.random.default_rng(4), 5000, "mono", seed_base=100)
    b = S.draw_points(np.random.default_rng(4), 5000, "mono", seed_base=100)
    assert np.array_equal(a.eps, b.eps) and np.array_equal(a.n, b.n)
    assert a.eps.min() >= 2.0 and a.eps.max() <= 10.0
    assert a.rho.min() >= 0.05 and a.rho.max() <= 0.4
    assert a.kT.min() >= 0.8 and a.kT.max() <= 1.2
    assert set(np.unique(a.cap_b)) == {1, 2, 4}
    assert a.n.min() >= 256 and a.n.max() <= 8192
    # log-uniform N: the median sits near the geometric mean of the range
    assert abs(np.log(np.median(a.n)) - 0.5 * np.log(256 * 8192)) < 0.1
    assert np.array_equal(a.seed, 100 + np.arange(5000))
    f = a.features()
    assert f.dtype == np.float32 and f.shape == (5000, 4) and np.all(np.abs(f) <= 1.0 + 1e-6)


def test_initial_weights():
    p = S.init_params(3)
    assert p.shape == (17410,) and p.dtype == np.float32
    w1, b1, w2, b2, w3, b3 = np.split(p, [512, 640, 17024, 17152, 17408])
    assert not b1.any() and not b2.any() and not b3.any()
    assert np.abs(w1).max() <= np.sqrt(6 / 4) and np.abs(w2).max() <= np.sqrt(6 / 128)
    assert np.abs(w3).max() <= np.sqrt(6 / 128)
    # uniform on [-b, b]: variance b^2 / 3 = 2 / fan_in
    assert abs(w2.var() - 2 / 128) < 0.05 * 2 / 128
    assert np.array_equal(p, S.init_params(3)) and not np.array_equal(p, S.init_params(4))


class _Fake:
    """A stand-in model whose largest-cluster output is eps / 10."""

    def predict(self, pts):
        return np.stack([np.zeros(len(pts)), pts.eps / 10.0], axis=1)


def test_choose_takes_the_points_predicted_nearest_the_target():
    pts = S.choose(_Fake(), np.random.default_rng(1), 50, "chains", target=0.5, pool=4000, seed_base=7)
    assert len(pts) == 50 and pts.kind == "chains"
    assert np.all(np.abs(pts.eps - 5.0) < 0.1)
    assert np.array_equal(pts.seed, 7 + np.arange(50))


def test_judge_keeps_predictions_within_tolerance_and_falls_back_otherwise():
    pred = np.array([[0.50, 0.30], [0.50, 0.30], [0.10, 0.90]])
    plain = np.array([[0.51, 0.29], [0.55, 0.30], [0.10, 0.80]])
    kept, fallback, err = S.judge(pred, plain, tol=0.02)
    assert fallback.tolist() == [False, True, True]
    assert np.array_equal(kept[0], pred[0]) and np.array_equal(kept[1:], plain[1:])
    assert np.allclose(err, np.abs(pred - plain))


def test_hit_rate():
    assert S.hit_rate([0.5, 0.39, 0.41, 0.6, 0.61, 1.0]) == 3 / 6
