"""Pins of the oracle's learned search window (a project addition beyond the
paper): the C network and features against independent statements of them,
and the build semantics at the limits where the learned window must reduce to
the plain definition.

  * or_bf16 is bfloat16 rounding (torch's conversion from float32);
  * or_mlp_forward equals the float64 network of oracle/mlp.py exactly when
    every weight, input and hidden activation is representable in bfloat16
    (so the device's roundings are identities);
  * features of a prediction at a hand-placed state are their closed forms;
  * a network with huge scales (window contains everything compatible) and
    one with tiny scales (window never holds a hit, so every candidate falls
    back) both give exactly the plain build;
  * the brute-force and binned scans agree in learned mode too;
  * with a one-sigma window the learned build differs from the plain one and
    falls back where the own hit lies outside.
"""
import numpy as np
import pytest

from oracle import mlp
from paper_1705_02876_amd import synth as S


def test_bf16_matches_torch(orc):
    import torch
    r = np.random.Generator(np.random.PCG64(3))
    x = (r.standard_normal(3000) * np.exp(r.uniform(-20, 20, 3000))).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).double().numpy()
    got = np.array([orc.bf16(float(v)) for v in x])
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(got, mlp.round_bf16(x.astype(np.float64)))


def _exact_params(seed):
    """Parameters whose network is exact in bfloat16: small dyadic weights, sparse W2."""
    r = np.random.Generator(np.random.PCG64(seed))
    p = {"W1": r.integers(-2, 3, (64, 8)) * 0.5, "b1": r.integers(-2, 3, 64) * 1.0,
         "W2": np.zeros((64, 64)), "b2": r.integers(-2, 3, 64) * 1.0,
         "W3": np.zeros((2, 64)), "b3": np.array([0.25, -0.5])}
    for i in range(64):
        j = r.choice(64, 2, replace=False)
        p["W2"][i, j] = r.integers(-2, 3, 2) * 0.5
    for k in range(2):
        j = r.choice(64, 3, replace=False)
        p["W3"][k, j] = r.integers(-2, 3, 3) * 0.25
    return p


def test_mlp_forward_matches_numpy_network_when_exact(orc):
    p = _exact_params(4)
    X = np.random.Generator(np.random.PCG64(5)).integers(-4, 5, (300, 8)) * 0.5
    want, (a1, h1, a2, h2) = mlp.forward(p, X)
    # every intermediate is representable with 8 significant bits
    for a in (X, h1, h2):
        assert np.array_equal(mlp.round_bf16(a), a)
    got = orc.mlp_forward(mlp.flatten(p), X)
    np.testing.assert_array_equal(got, want)
    assert np.abs(want).max() > 0.5  # not a trivial network


def test_mlp_forward_rounds_like_the_device(orc):
    # generic parameters: equals the numpy chain with explicit bfloat16 roundings
    p = mlp.init(6)
    p["b1"] = np.random.Generator(np.random.PCG64(7)).normal(0, 0.1, 64)
    X, _ = S.window_records(8, 200)
    W1, W2, W3 = (mlp.round_bf16(p[k]) for k in ("W1", "W2", "W3"))
    b1, b2, b3 = (S.round_f32(p[k]) for k in ("b1", "b2", "b3"))
    h1 = mlp.round_bf16(np.maximum(mlp.round_bf16(X) @ W1.T + b1, 0))
    h2 = mlp.round_bf16(np.maximum(h1 @ W2.T + b2, 0))
    want = h2 @ W3.T + b3
    got = orc.mlp_forward(mlp.flatten(p), X)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_window_features_closed_form(orc):
    # on the x axis at r = 10, momentum along +y (perpendicular crossing)
    s = np.array([10.0, 0.0, 3.0, 0.0, 2.0, 1.0])
    C = np.diag([1e-4, 4e-4, 9e-4, 1e-3, 1e-3, 1e-3])
    f = orc.window_features(s, C, -1, 4.0, 10.0, 50.0)
    want = [-0.5, 0.5, 3.0 / 50.0, 1.0, 0.04, 0.10, 0.5 * np.log(4e-4), 0.5 * np.log(9e-4)]
    np.testing.assert_allclose(f, want, rtol=1e-14, atol=1e-15)
    # on the y axis, momentum at 30 degrees to the radial direction
    s = np.array([0.0, 10.0, 0.0, -np.sin(np.pi / 6), np.cos(np.pi / 6), 0.0])
    C = np.zeros((6, 6))
    C[0, 0], C[1, 1], C[2, 2] = 2.5e-5, 1e-6, 4e-2
    f = orc.window_features(s, C, 1, 4.0, 10.0, 50.0)
    np.testing.assert_allclose(f[3], 0.5, rtol=1e-14)
    np.testing.assert_allclose(f[6], 0.5 * np.log(2.5e-5), rtol=1e-14)
    np.testing.assert_allclose(f[7], 0.5 * np.log(4e-2), rtol=1e-14)


def _net(b3):
    p = mlp.init(9)
    p["W3"][:] = 0.0
    p["b3"] = np.array(b3, dtype=np.float64)
    return mlp.flatten(p)


@pytest.fixture(scope="module")
def small_build():
    det = S.detector_full()
    prob = S.make_build_problem([300, 500], det, 41)
    return det, prob


def _same(a, b):
    for k in ("n_cands", "cand_hits", "cand_nhits", "cand_status"):
        assert np.array_equal(a[k], b[k]), k
    np.testing.assert_array_equal(a["cand_chi2"], b["cand_chi2"])


def test_huge_and_tiny_windows_reduce_to_plain(orc, small_build):
    det, prob = small_build
    g = orc.geometry(det)
    plain = orc.build(g, prob)
    huge = orc.build(g, prob, mlp_params=_net([30.0, 30.0]))
    _same(plain, huge)
    assert huge["fallbacks"].sum() == 0
    tiny = orc.build(g, prob, mlp_params=_net([-60.0, -60.0]))
    _same(plain, tiny)
    assert tiny["fallbacks"].sum() > 0


def test_learned_binned_equals_brute_force(orc, small_build):
    det, prob = small_build
    g = orc.geometry(det)
    net = _net([np.log(0.02 / 4), np.log(0.15 / 4)])
    a = orc.build(g, prob, mlp_params=net, mode=1)
    b = orc.build(g, prob, mlp_params=net, mode=0)
    _same(a, b)


def test_moderate_window_drops_hits_outside(orc, small_build):
    det, prob = small_build
    g = orc.geometry(det)
    plain = orc.build(g, prob)
    # constant one-sigma scales of the hit resolution: the own hit is often inside, its neighbours not
    net = _net([np.log(0.01), np.log(0.1)])
    lw = orc.build(g, prob, mlp_params=net, learned_nsigma=1.0)
    assert lw["fallbacks"].sum() > 0
    assert not np.array_equal(lw["cand_hits"], plain["cand_hits"])
    assert np.isfinite(lw["margin_window"]).all()
