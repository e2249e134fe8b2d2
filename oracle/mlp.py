"""FP64 reference of the surrogate network (test infrastructure only).

Only tests/ and bench.py's baseline leg use this module; the library never
imports it.  Written from the textbook definitions, in FP64:

  network   x (4) -> z1 = W1 x + b1 -> a1 = SiLU(z1) (128)
                  -> z2 = W2 a1 + b2 -> a2 = SiLU(z2) (128)
                  -> z3 = W3 a2 + b3 -> y = sigmoid(z3) (2)
            SiLU(z) = z / (1 + e^-z), sigmoid(z) = 1 / (1 + e^-z)
  loss      L = mean over the batch and both outputs of (y - t)^2
  gradient  reverse-mode chain rule, one layer at a time
  Adam      Kingma & Ba (2015), with bias correction

Mixed precision is emulated exactly where the device rounds: the weights
used by every layer are the BF16 roundings of the FP32 master weights, the
input of the 128 x 128 layer (a1) is rounded to BF16, and so is the
back-propagated dz2 that enters both GEMMs of that layer's backward pass
(dW2 = dz2^T a1 and da1 = dz2 W2).  Biases, the other activations and all
accumulations stay in full precision here (FP32 on the device).

Parameters are one flat FP32 vector in the order W1 (128 x 4, row-major),
b1 (128), W2 (128 x 128), b2 (128), W3 (2 x 128), b3 (2): 17 410 numbers.
"""

import numpy as np

N_IN, N_HID, N_OUT = 4, 128, 2
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    """Split the flat parameter vector into named arrays (views, float64)."""
    flat = np.asarray(flat, dtype=np.float64)
    out, k = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = flat[k:k + size].reshape(shape)
        k += size
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    The value is first rounded to FP32 (the device keeps FP32 values), then
    its low 16 bits are rounded away: add 0x7FFF plus the lowest kept bit and
    truncate."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(f), f, out).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(flat, x, mixed=True):
    """Network output y (n, 2) and the intermediates the backward pass uses."""
    p = unpack(flat)
    W1, W2, W3 = (bf16(p["W1"]), bf16(p["W2"]), bf16(p["W3"])) if mixed else (p["W1"], p["W2"], p["W3"])
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + p["b1"]
    a1 = silu(z1)
    a1q = bf16(a1) if mixed else a1
    z2 = a1q @ W2.T + p["b2"]
    a2 = silu(z2)
    z3 = a2 @ W3.T + p["b3"]
    y = sigmoid(z3)
    return y, dict(x=x, z1=z1, a1q=a1q, z2=z2, a2=a2, y=y, W1=W1, W2=W2, W3=W3)


def loss(flat, x, t, mixed=True):
    y, _ = forward(flat, x, mixed)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def loss_and_grad(flat, x, t, mixed=True):
    """MSE loss and its gradient with respect to the flat FP32 parameters."""
    y, c = forward(flat, x, mixed)
    t = np.asarray(t, dtype=np.float64)
    n = y.shape[0]
    L = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / (n * N_OUT)
    dz3 = dy * y * (1.0 - y)
    g = {"W3": dz3.T @ c["a2"], "b3": dz3.sum(axis=0)}
    da2 = dz3 @ c["W3"]
    dz2 = da2 * dsilu(c["z2"])
    dz2q = bf16(dz2) if mixed else dz2
    g["W2"] = dz2q.T @ c["a1q"]
    g["b2"] = dz2.sum(axis=0)
    da1 = dz2q @ c["W2"]
    dz1 = da1 * dsilu(c["z1"])
    g["W1"] = dz1.T @ c["x"]
    g["b1"] = dz1.sum(axis=0)
    return L, pack(g)


def adam_step(flat, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shape[1])
            d[name] = rng.uniform(-bound, bound, shape)
        else:
            d[name] = np.zeros(shape)
    return pack(d).astype(np.float32)
