"""Per-object time-step network, plain numpy FP64 -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may use this module; the product library never imports it.

The paper keeps a time interval per object so that objects far from all others
can take long intervals and be processed rarely (Sec. "Collision Detection
with 4D AABB Trees"; Procedure advanceTime, which doubles an object's interval
while its box meets nobody).  It leaves open how long each object's step
should be.  The library adds a small regression network that predicts the
step from an object's orbital elements; any step >= 1 tick keeps the boxes
conservative, so the network changes cost, never correctness.

The network (the library's own definition, written out here as the
reference):

    x  = (a / 42164, e, i / pi, r_p / 42164, v_max / 8)     r_p = a (1 - e),
                                                            v_max = perigee speed
    h1 = relu(W1 x + b1)          W1: 64 x 5
    h2 = relu(W2 h1 + b2)         W2: 64 x 64
    y  = w3 . h2 + b3             y = log2(step in seconds)
    dt = clamp(floor(2**y / tick_s), 1, max(T, 1))   ticks

Parameters are one flat vector in the order W1 (row-major), b1, W2
(row-major), b2, w3, b3: 4609 values.  Training minimises the mean squared
error between y and a target log2 step; the optimiser is Adam (Kingma & Ba,
2015) with bias-corrected moments.

Every function here is plain FP64 numpy with no blocking or fusion.  The pins
are in tests/test_oracle_mlp.py: central finite differences of the loss
against the analytic gradient, hidden-unit permutation invariance (catches a
transposed weight), dead-ReLU and affine special cases, Adam's closed-form
first steps, vis-viva for the speed feature, and exact decode cases.
"""
import numpy as np

N_IN = 5
N_HID = 64
A_SCALE_KM = 42164.0     # geostationary radius: features of order 1
V_SCALE_KMS = 8.0

_SIZES = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)),
          ("b2", (N_HID,)), ("w3", (N_HID,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in _SIZES)   # 4609


def unpack(theta):
    """Views W1, b1, W2, b2, w3, b3 of the flat parameter vector."""
    theta = np.asarray(theta)
    assert theta.shape == (N_PARAMS,)
    out, off = {}, 0
    for name, shape in _SIZES:
        k = int(np.prod(shape))
        out[name] = theta[off:off + k].reshape(shape)
        off += k
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1)
                           for name, _ in _SIZES])


def init_params(seed):
    """He-uniform weights, zero biases except b3 = 0."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.uniform(-1, 1, (N_HID, N_IN)) * np.sqrt(6.0 / N_IN),
         "b1": np.zeros(N_HID),
         "W2": rng.uniform(-1, 1, (N_HID, N_HID)) * np.sqrt(6.0 / N_HID),
         "b2": np.zeros(N_HID),
         "w3": rng.uniform(-1, 1, N_HID) * np.sqrt(6.0 / N_HID),
         "b3": np.zeros(1)}
    return pack(p)


def features(a, e, inc, mu):
    """Network inputs of each object: a, e, i, perigee radius and perigee
    speed, each on a fixed scale.  The perigee speed is the largest speed on a
    Kepler ellipse (the speed bound the boxes use)."""
    a = np.asarray(a, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    inc = np.asarray(inc, dtype=np.float64)
    rp = a * (1.0 - e)
    vmax = np.sqrt(mu * (1.0 + e) / rp)
    return np.stack([a / A_SCALE_KM, e, inc / np.pi, rp / A_SCALE_KM, vmax / V_SCALE_KMS],
                    axis=1)


def forward(theta, X):
    """y[b] for every row of X, plus the intermediate values."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, {"X": X, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def loss(theta, X, target):
    """Mean squared error over the batch."""
    y, _ = forward(theta, X)
    r = y - np.asarray(target, dtype=np.float64)
    return float(np.mean(r * r))


def grad(theta, X, target):
    """Analytic gradient of loss() by the chain rule, layer by layer."""
    p = unpack(theta)
    y, c = forward(theta, X)
    B = y.shape[0]
    dy = 2.0 * (y - np.asarray(target, dtype=np.float64)) / B        # [B]
    g = {"w3": c["h2"].T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, p["w3"]) * (c["z2"] > 0)                       # [B, 64]
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * (c["z1"] > 0)                             # [B, 64]
    g["W1"] = dz1.T @ c["X"]
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def adam(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def decode(y, tick_s, T):
    """Step in ticks from the predicted log2(seconds); 0 where y is not finite
    (the caller then uses its fallback step)."""
    y = np.asarray(y, dtype=np.float64)
    cap = float(max(int(T), 1))
    out = np.zeros(y.shape, dtype=np.uint32)
    ok = np.isfinite(y)
    d = np.floor(np.exp2(np.where(ok, y, 0.0)) / tick_s)
    d = np.clip(d, 1.0, cap)
    out[ok] = d[ok].astype(np.uint32)
    return out


def bf16(x):
    """Round FP32 values to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    r = np.where(np.isnan(f), (u >> 16) | 0x40, r)
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def forward_bf16(theta, X):
    """The network with weights, biases, inputs and hidden activations rounded
    to bfloat16 and sums taken in FP64: the arithmetic of a BF16 inference
    path up to the order and precision of its accumulations."""
    p = {k: bf16(v) for k, v in unpack(theta).items()}
    x = bf16(X)
    h1 = bf16(np.maximum(x @ p["W1"].T + p["b1"], 0.0))
    h2 = bf16(np.maximum(h1 @ p["W2"].T + p["b2"], 0.0))
    return h2 @ p["w3"] + p["b3"][0]
