"""Pins of the FP64 network oracle (oracle/mlp.py) to facts independent of it:
central finite differences of the loss, the closed-form maximum-likelihood
optimum of a constant output, Adam's first step, and the bfloat16 format."""
import numpy as np

from oracle import mlp
from paper_1705_02876_amd import synth as S


def _params(seed):
    p = mlp.init(seed)
    r = np.random.Generator(np.random.PCG64(seed + 1))
    for k in ("b1", "b2", "b3"):
        p[k] = r.normal(0, 0.1, p[k].shape)
    return p


def test_param_count_and_flat_order():
    assert mlp.n_params() == 4866
    p = _params(3)
    v = mlp.flatten(p)
    assert v.shape == (4866,)
    assert v[0] == p["W1"][0, 0] and v[8] == p["W1"][1, 0] and v[512] == p["b1"][0]
    assert v[576 + 64] == p["W2"][1, 0] and v[4736] == p["W3"][0, 0] and v[4864] == p["b3"][0]
    q = mlp.unflatten(v)
    assert all(np.array_equal(q[k], p[k]) for k in p)


def test_gradient_matches_central_differences():
    x, t = S.window_records(11, 64)
    p = _params(5)
    L, g = mlp.grad(p, x, t)
    assert abs(L - mlp.loss(p, x, t)) < 1e-12
    v = mlp.flatten(p)
    gv = mlp.flatten(g)
    r = np.random.Generator(np.random.PCG64(9))
    # every bias and a sample of every weight matrix
    idx = np.concatenate([np.arange(512, 576), np.arange(4672, 4736), [4864, 4865],
                          r.choice(512, 40, replace=False), 576 + r.choice(4096, 60, replace=False),
                          4736 + r.choice(128, 40, replace=False)])
    h = 1e-6
    for i in idx:
        vp, vm = v.copy(), v.copy()
        vp[i] += h
        vm[i] -= h
        fd = (mlp.loss(mlp.unflatten(vp), x, t) - mlp.loss(mlp.unflatten(vm), x, t)) / (2 * h)
        assert abs(fd - gv[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gv[i])


def test_constant_output_optimum_is_the_gaussian_mle():
    # W3 = 0: o = b3 for every record; the NLL is minimised at exp(2 b3_k) = mean(t_k^2)
    x, t = S.window_records(12, 5000)
    p = _params(6)
    p["W3"][:] = 0.0
    s2 = np.mean(t * t, axis=0)
    p["b3"] = 0.5 * np.log(s2)
    L, g = mlp.grad(p, x, t)
    assert np.abs(g["b3"]).max() < 1e-12
    assert abs(L - np.sum(0.5 + 0.5 * np.log(s2))) < 1e-12
    p["b3"] += 0.01
    assert mlp.loss(p, x, t) > L


def test_adam_first_step_moves_by_lr_times_sign():
    p = _params(7)
    g = {k: np.random.Generator(np.random.PCG64(8)).normal(0, 1, v.shape) for k, v in p.items()}
    p0 = {k: v.copy() for k, v in p.items()}
    st = {}
    mlp.adam_step(p, g, st, lr=1e-3, eps=1e-300)
    for k in p:
        np.testing.assert_allclose(p[k] - p0[k], -1e-3 * np.sign(g[k]), rtol=1e-9, atol=1e-15)
    assert st["t"] == 1


def test_training_reduces_loss_towards_the_generating_widths():
    x, t = S.window_records(13, 4000)
    p = mlp.init(14)
    st = {}
    L0 = mlp.loss(p, x, t)
    for _ in range(300):
        L, g = mlp.grad(p, x, t)
        mlp.adam_step(p, g, st, lr=3e-3)
    L1 = mlp.loss(p, x, t)
    # a constant-width model cannot beat its own MLE
    s2 = np.mean(t * t, axis=0)
    L_const = np.sum(0.5 + 0.5 * np.log(s2))
    assert L1 < L0 and L1 < L_const


def test_bf16_rounding_definition():
    vals = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 1 + 2 ** -7, 3.0, 0.0, 2 ** -130 * 1.5])
    want = np.array([1.0, 1 + 2 ** -6, -1.0, 1 + 2 ** -7, 3.0, 0.0, 2 ** -130 * 1.5])
    np.testing.assert_array_equal(mlp.round_bf16(vals), want)
    r = np.random.Generator(np.random.PCG64(1))
    x = (r.standard_normal(20000) * np.exp(r.uniform(-30, 30, 20000))).astype(np.float32).astype(np.float64)
    y = mlp.round_bf16(x)
    # within half a spacing of 8 significant bits, and idempotent
    assert np.all(np.abs(y - x) <= np.abs(x) * 2.0 ** -8)
    np.testing.assert_array_equal(mlp.round_bf16(y), y)
    _, e = np.frexp(y)
    np.testing.assert_array_equal(np.ldexp(np.round(np.ldexp(np.frexp(y)[0], 8)), e - 8), y)


def _exact_params(seed):
    """Dyadic weights and sparse W2 so that every operand of the network is a bfloat16 value."""
    r = np.random.Generator(np.random.PCG64(seed))
    p = {"W1": r.integers(-2, 3, (64, 8)) * 0.5, "b1": r.integers(-2, 3, 64) * 1.0, "W2": np.zeros((64, 64)),
         "b2": r.integers(-2, 3, 64) * 1.0, "W3": np.zeros((2, 64)), "b3": np.array([0.25, -0.5])}
    for i in range(64):
        p["W2"][i, r.choice(64, 2, replace=False)] = r.integers(-2, 3, 2) * 0.5
    for k in range(2):
        p["W3"][k, r.choice(64, 3, replace=False)] = r.integers(-2, 3, 3) * 0.25
    return p


def test_device_semantics_reduce_to_the_exact_network():
    p = _exact_params(4)
    X = np.random.Generator(np.random.PCG64(5)).integers(-4, 5, (300, 8)) * 0.5
    # targets such that the output gradients are bfloat16 values: t^2 exp(-2 o) = 1 - dO exactly
    o, _ = mlp.forward(p, X)
    d = np.random.Generator(np.random.PCG64(6)).integers(-3, 1, o.shape) * 0.25
    T = np.sqrt((1.0 - d) * np.exp(2.0 * o))
    od, _ = mlp.forward_device(p, X)
    np.testing.assert_array_equal(od, o)
    L, g = mlp.grad(p, X, T)
    Ld, gd = mlp.grad_device(p, X, T)
    assert abs(L - Ld) < 1e-12
    for k in g:
        np.testing.assert_allclose(gd[k], g[k], rtol=1e-9, atol=1e-12)


def test_device_semantics_close_to_the_exact_network():
    # generic parameters: bfloat16 operands move the gradient by a few 2^-9 relative steps
    x, t = S.window_records(21, 4000)
    p = mlp.init(22)
    s2 = np.mean(t * t, axis=0)
    p["b3"] = 0.5 * np.log(s2)
    p["W3"] *= 0.1
    L, g = mlp.grad(p, x, t)
    Ld, gd = mlp.grad_device(p, x, t)
    assert abs(L - Ld) < 2e-2 * max(1.0, abs(L))
    for k in g:
        assert np.abs(gd[k] - g[k]).max() <= 5e-2 * np.abs(g[k]).max(), k
