"""FP64 reference of the learned search-window network (test infrastructure only).

Network 8 -> 64 -> 64 -> 2 with ReLU hidden layers:
    h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), o = W3 h2 + b3.
The two outputs are log scales (log s_t, log s_z) of the tangential and z
residuals of a track's own hit around the propagated prediction.  Training
minimises the Gaussian negative log-likelihood per record
    l = sum_k [ r_k^2 exp(-2 o_k) / 2 + o_k ],
averaged over the batch; the optimiser is Adam (Kingma & Ba, 2015) with
bias-corrected moments.  Parameters are kept in a dict of float64 arrays.

round_bf16 is the bfloat16 format's definition (8 significant bits, round to
nearest, ties to even).  forward_device / grad_device state the network with
the roundings of a bfloat16 matrix-core evaluation written out: weights,
inputs and hidden activations are bfloat16 operands, the backward products
take the output gradient and the pre-activation gradients as bfloat16
operands, biases are float32, sums are exact (float64 here).  With every value
representable in bfloat16 they coincide with forward / grad.
"""
from __future__ import annotations

import numpy as np

SIZES = (8, 64, 64, 2)
NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def n_params():
    return sum(SIZES[i + 1] * SIZES[i] + SIZES[i + 1] for i in range(3))


def init(seed):
    """He-uniform weights, zero biases (seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for i in range(3):
        fan_in, fan_out = SIZES[i], SIZES[i + 1]
        lim = np.sqrt(6.0 / fan_in)
        p[f"W{i + 1}"] = rng.uniform(-lim, lim, (fan_out, fan_in))
        p[f"b{i + 1}"] = np.zeros(fan_out)
    return p


def flatten(p):
    """Parameters as one vector in the order W1, b1, W2, b2, W3, b3 (row-major)."""
    return np.concatenate([p[k].ravel() for k in NAMES])


def unflatten(v):
    p = {}
    off = 0
    for i in range(3):
        fo, fi = SIZES[i + 1], SIZES[i]
        p[f"W{i + 1}"] = v[off:off + fo * fi].reshape(fo, fi)
        off += fo * fi
        p[f"b{i + 1}"] = v[off:off + fo].copy()
        off += fo
    return p


def round_bf16(a):
    """Nearest bfloat16 value of each element (ties to even), returned as float64."""
    a = np.asarray(a, dtype=np.float64)
    _, e = np.frexp(a)  # |a| = m 2^e with 0.5 <= m < 1
    # spacing of bfloat16 values around a: 2^(e-8), and 2^-133 in the subnormal range
    quantum = np.ldexp(1.0, np.maximum(e, -125) - 8)
    with np.errstate(invalid="ignore"):
        out = np.round(a / quantum) * quantum  # numpy rounds halves to even
    return np.where(np.isfinite(a), out, a)


def bf16_params(p):
    """The parameters as the device network holds them: weights in bfloat16, biases in float32."""
    return {k: (round_bf16(v) if k.startswith("W") else v.astype(np.float32).astype(np.float64)) for k, v in p.items()}


def forward(p, X):
    """X (B, 8) -> outputs (B, 2) and the hidden activations."""
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    o = h2 @ p["W3"].T + p["b3"]
    return o, (a1, h1, a2, h2)


def forward_device(p, X):
    """Outputs (B, 2) and (a1, h1b, a2, h2b) of the network with bfloat16 operands (see module doc)."""
    q = bf16_params(p)
    xb = round_bf16(X)
    a1 = xb @ q["W1"].T + q["b1"]
    h1b = round_bf16(np.maximum(a1, 0.0))
    a2 = h1b @ q["W2"].T + q["b2"]
    h2b = round_bf16(np.maximum(a2, 0.0))
    o = h2b @ q["W3"].T + q["b3"]
    return o, (xb, a1, h1b, a2, h2b)


def grad_device(p, X, T):
    """Mean loss and gradient of the network with bfloat16 operands: the output gradient dO and the
    pre-activation gradients dA2, dA1 enter the products as bfloat16; the bias gradients sum the unrounded
    values."""
    B = X.shape[0]
    q = bf16_params(p)
    o, (xb, a1, h1b, a2, h2b) = forward_device(p, X)
    e = T * T * np.exp(-2.0 * o)
    L = float(np.mean(np.sum(0.5 * e + o, axis=1)))
    do = 1.0 - e
    dob = round_bf16(do)
    da2 = (dob @ q["W3"]) * (a2 > 0)
    da2b = round_bf16(da2)
    da1 = (da2b @ q["W2"]) * (a1 > 0)
    da1b = round_bf16(da1)
    g = {"W3": dob.T @ h2b / B, "b3": do.sum(axis=0) / B, "W2": da2b.T @ h1b / B, "b2": da2.sum(axis=0) / B,
         "W1": da1b.T @ xb / B, "b1": da1.sum(axis=0) / B}
    return L, g


def loss(p, X, T):
    o, _ = forward(p, X)
    return float(np.mean(np.sum(0.5 * T * T * np.exp(-2.0 * o) + o, axis=1)))


def grad(p, X, T):
    """Mean loss and its gradient (dict like p), by the chain rule."""
    B = X.shape[0]
    o, (a1, h1, a2, h2) = forward(p, X)
    L = float(np.mean(np.sum(0.5 * T * T * np.exp(-2.0 * o) + o, axis=1)))
    do = (1.0 - T * T * np.exp(-2.0 * o)) / B
    g = {"W3": do.T @ h2, "b3": do.sum(axis=0)}
    dh2 = do @ p["W3"]
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return L, g


def adam_step(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; state = dict(m, v, t) (created if empty)."""
    if not state:
        state.update(m={k: np.zeros_like(v) for k, v in p.items()}, v={k: np.zeros_like(v) for k, v in p.items()},
                     t=0)
    state["t"] += 1
    t = state["t"]
    for k in p:
        state["m"][k] = beta1 * state["m"][k] + (1 - beta1) * g[k]
        state["v"][k] = beta2 * state["v"][k] + (1 - beta2) * g[k] * g[k]
        mh = state["m"][k] / (1 - beta1 ** t)
        vh = state["v"][k] / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p
