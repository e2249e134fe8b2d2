"""The surrogate network's HIP kernels (through the C ABI) against the FP64
reference of oracle/mlp.py: outputs, loss, gradients (the matrix-core GEMMs
of the 128 x 128 layer included), an Adam step, training and determinism."""

import numpy as np
import pytest

from oracle import mlp
from paper_2609_21204_amd import dybond as db

pytestmark = pytest.mark.gpu


def _data(seed, n):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.5, 1.5, (n, 4)).astype(np.float32)
    t = np.stack([1 / (1 + np.exp(-2.5 * x[:, 0] + x[:, 3])),
                  0.5 + 0.45 * np.tanh(x[:, 1] * x[:, 2] - 0.5 * x[:, 0])], axis=1).astype(np.float32)
    return x, t


@pytest.fixture
def net():
    h = db.db_mlp_create(512)
    yield h
    db.db_mlp_destroy(h)


def test_forward_and_gradient_match_reference(net):
    for seed, n in ((1, 200), (2, 512), (3, 17)):
        params = mlp.init_params(seed)
        db.db_mlp_set_params(net, params)
        assert np.array_equal(db.db_mlp_get_params(net), params)
        x, t = _data(seed + 10, n)
        y_ref, _ = mlp.forward(params, x)
        y = db.db_mlp_predict(net, x)
        # FP32 on the device vs FP64 here: an activation that sits next to a
        # bf16 rounding boundary can round the other way (one bf16 ulp, 2^-8
        # relative), which moves a few outputs by up to ~1e-4; the rest agree
        # to FP32 accuracy
        err = np.abs(y.astype(np.float64) - y_ref)
        assert float(np.quantile(err, 0.98)) < 1e-6 and float(err.max()) < 1e-3, \
            f"outputs, seed {seed}: q98 {np.quantile(err, 0.98):.2e} max {err.max():.2e}"
        loss, g = db.db_mlp_loss_grad(net, x, t)
        l_ref, g_ref = mlp.loss_and_grad(params, x, t)
        assert abs(loss - l_ref) <= 1e-4 * l_ref + 1e-9, f"loss {loss} vs {l_ref}"
        k = 0
        for name, shape in mlp.SHAPES:
            size = int(np.prod(shape))
            a, b = g[k:k + size], g_ref[k:k + size]
            scale = np.max(np.abs(b))
            err = np.max(np.abs(a - b))
            assert err <= 3e-4 * scale + 1e-8, f"seed {seed} n {n} {name}: {err:.3e} vs scale {scale:.3e}"
            k += size


def test_one_adam_step_matches_reference(net):
    params = mlp.init_params(4)
    x, t = _data(5, 256)
    db.db_mlp_set_params(net, params)
    _, g_dev = db.db_mlp_loss_grad(net, x, t)
    lr = 1e-3
    db.db_mlp_train(net, x, t, batch=256, epochs=1, lr=lr, seed=1)
    p1 = db.db_mlp_get_params(net).astype(np.float64)
    z = np.zeros(mlp.N_PARAMS)
    # the update itself, from the device's gradient (one minibatch of all rows;
    # its row order differs, so entries whose gradient is near zero are left out)
    big = np.abs(g_dev) > 1e-4 * np.max(np.abs(g_dev))
    ref, _, _ = mlp.adam_step(params.astype(np.float64), g_dev.astype(np.float64), z, z, 1, lr)
    assert np.max(np.abs(p1 - ref)[big]) < 2e-7 + 1e-3 * lr
    # and the step the reference gradient prescribes: first step = -lr * sign(g)
    _, g = mlp.loss_and_grad(params, x, t)
    clear = np.abs(g) > 0.01 * np.max(np.abs(g))
    assert np.array_equal(np.sign(p1 - params)[clear], -np.sign(g)[clear])
    assert np.max(np.abs(p1 - params)) <= lr * 1.0001


def test_training_reduces_loss_deterministically():
    x, t = _data(6, 3000)
    finals, params = [], []
    for _ in range(2):
        h = db.db_mlp_create(256)
        try:
            db.db_mlp_set_params(h, mlp.init_params(7))
            l0, _ = db.db_mlp_loss_grad(h, x[:256], t[:256])
            lf = db.db_mlp_train(h, x, t, batch=128, epochs=30, lr=3e-3, seed=11)
            finals.append(lf)
            params.append(db.db_mlp_get_params(h))
        finally:
            db.db_mlp_destroy(h)
    assert finals[0] < 0.01 * l0 and finals[0] < 5e-4
    assert np.array_equal(params[0], params[1]) and finals[0] == finals[1]
    # the device's final loss agrees with the reference at the trained weights
    assert abs(finals[0] - mlp.loss(params[0], x, t)) < 1e-5


def test_bad_arguments_are_rejected(net):
    with pytest.raises(db.DybondError) as e:
        db.db_mlp_set_params(net, np.zeros(10, np.float32))
    assert e.value.name == "DB_EINVAL"
    x, t = _data(1, 600)
    with pytest.raises(db.DybondError) as e:
        db.db_mlp_loss_grad(net, x, t)                      # more rows than batch_max
    assert e.value.name == "DB_EINVAL"
    x[3, 1] = np.nan
    with pytest.raises(db.DybondError):
        db.db_mlp_predict(net, x)
