"""GPU parity of the search-window network (pack, forward, gradient, Adam,
training) against the FP64 oracle in oracle/mlp.py, through the C ABI.

The device network holds its weights in bfloat16 (biases float32) and feeds
bfloat16 operands to the matrix cores with float32 accumulation.  The oracle's
forward_device / grad_device write the same bfloat16 roundings out with exact
(float64) sums; what remains is float32 summation and the rare bfloat16
rounding flip it causes.  Tolerances:
- forward: |d o| <= 2^-8 (|W3| h2 + |W3| |W2| h1), the first-order effect of
  a one-step bfloat16 change of every hidden activation, with a factor 2
  margin (against the float64 network on bfloat16 weights: the device's
  activation roundings included);
- gradient (against grad_device): per parameter block, |d g| <= 1e-2 max |g|;
  mean loss 2e-5 relative (a float32 emulation stays below 2.1e-6);
- Adam: float32 update against float64, a few float32 roundings of the
  parameter plus 1e-5 lr;
- training: 200 full-batch steps from the same start end within 0.02 of the
  oracle's loss.
"""
import numpy as np
import pytest

from oracle import mlp
from paper_1705_02876_amd import synth as S

pytestmark = pytest.mark.gpu

BLOCKS = (("W1", 0, 512), ("b1", 512, 576), ("W2", 576, 4672), ("b2", 4672, 4736), ("W3", 4736, 4864),
          ("b3", 4864, 4866))


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1705_02876_amd import kfmi
    assert torch.cuda.is_available()
    c = kfmi.Context(0)
    yield c
    c.close()


def _dev_params(p):
    import torch
    return torch.from_numpy(mlp.flatten(p).astype(np.float32)).cuda()


def _records_dev(a, ld=None):
    """(n, k) float64 -> (k, ld) float32 device, feature-major, padded with NaN."""
    import torch
    n, k = a.shape
    ld = n if ld is None else ld
    h = np.full((k, ld), np.nan, np.float32)
    h[:, :n] = a.T
    return torch.from_numpy(h).cuda()


def _params(seed):
    p = mlp.init(seed)
    r = np.random.Generator(np.random.PCG64(seed + 7))
    for k in ("b1", "b2", "b3"):
        p[k] = r.normal(0, 0.05, p[k].shape)
    return p


@pytest.mark.parametrize("n,pad", [(4099, 3), (16, 0), (5, 11), (1, 0), (65536, 0)])
def test_forward_parity(ctx, n, pad):
    import torch
    from paper_1705_02876_amd import kfmi_mlp as M
    print(f"[mlp forward n={n} pad={pad}]", flush=True)
    x, _ = S.window_records(300 + n, n)
    p = _params(n)
    packed = M.pack(ctx, _dev_params(p), M.new_packed())
    xd = _records_dev(x, n + pad)
    y = torch.full((2, n + pad), -7.0, dtype=torch.float32, device="cuda")
    M.forward(ctx, xd, packed, y, n=n)
    torch.cuda.synchronize()
    yo = y.cpu().numpy().astype(np.float64)
    assert np.all(yo[:, n:] == -7.0), "wrote beyond n"
    pb = mlp.bf16_params(p)
    o, (a1, h1, a2, h2) = mlp.forward(pb, mlp.round_bf16(S.round_f32(x)))
    bound = 2.0 ** -8 * (h2 @ np.abs(pb["W3"]).T + (h1 @ np.abs(pb["W2"]).T) @ np.abs(pb["W3"]).T) + 1e-5
    err = np.abs(yo[:, :n].T - o)
    assert np.all(err <= bound), f"worst |d o|/bound {np.max(err / bound):.3g}"


def _grad_gpu(ctx, p, x, t, pad=0):
    import torch
    from paper_1705_02876_amd import kfmi_mlp as M
    packed = M.pack(ctx, _dev_params(p), M.new_packed())
    g, loss, count = M.grad(ctx, _records_dev(x, x.shape[0] + pad), _records_dev(t, t.shape[0] + pad), packed,
                            n=x.shape[0])
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64), float(loss.item()), float(count.item())


def _check_grad(g, go):
    for name, a, b in BLOCKS:
        scale = np.abs(go[a:b]).max()
        err = np.abs(g[a:b] - go[a:b]).max()
        assert err <= 1e-2 * scale + 1e-7, f"{name}: max |d g| {err:.3g} vs max |g| {scale:.3g}"


@pytest.mark.parametrize("n,pad", [(20000, 0), (3001, 5), (7, 0), (16 * 1024 + 1, 2)])
def test_grad_parity(ctx, n, pad):
    print(f"[mlp grad n={n} pad={pad}]", flush=True)
    x, t = S.window_records(400 + n, n)
    p = _params(n + 1)
    g, loss, count = _grad_gpu(ctx, p, x, t, pad)
    Lo, go = mlp.grad_device(p, S.round_f32(x), S.round_f32(t))
    assert count == n
    assert abs(loss - Lo) <= 2e-5 * max(1.0, abs(Lo)), (loss, Lo)
    _check_grad(g, mlp.flatten(go))


def test_grad_near_the_exact_gradient(ctx):
    """The device gradient against the exact FP64 gradient of the same network (bfloat16-rounded weights, no
    rounding of activations or gradients), not the oracle's emulation of the device's rounding points.  Every
    operand of the device's products is rounded to bfloat16 once (relative error at most 2^-9, 0.2%); the
    backward products chain a few such roundings per term, so each parameter block stays within 2% of its
    largest gradient (the FP64 emulation of the device's roundings lies within 0.12% of the exact gradient on
    these records) and the mean loss within 1e-3."""
    print("[mlp grad exact]", flush=True)
    n = 20000
    x, t = S.window_records(901, n)
    p = _params(902)
    g, loss, count = _grad_gpu(ctx, p, x, t, 0)
    pq = mlp.bf16_params(p)
    Le, ge = mlp.grad({k: np.asarray(v, np.float64) for k, v in pq.items()}, S.round_f32(x), S.round_f32(t))
    assert count == n
    assert abs(loss - Le) <= 1e-3 * max(1.0, abs(Le)), (loss, Le)
    ge = mlp.flatten(ge)
    for name, a, b in BLOCKS:
        scale = np.abs(ge[a:b]).max()
        err = np.abs(g[a:b] - ge[a:b]).max()
        print(f"[mlp grad exact] {name}: max |d g| / max |g| = {err / scale:.3g}", flush=True)
        assert err <= 2e-2 * scale + 1e-7, f"{name}: max |d g| {err:.3g} vs max |g| {scale:.3g}"


def test_grad_skips_nonfinite_records_and_empty_input(ctx):
    print("[mlp grad nonfinite/empty]", flush=True)
    n = 2000
    x, t = S.window_records(77, n)
    bad = np.zeros(n, bool)
    bad[::17] = True
    xb, tb = x.copy(), t.copy()
    xb[np.flatnonzero(bad)[::2], 3] = np.nan
    tb[np.flatnonzero(bad)[1::2], 1] = np.inf
    p = _params(3)
    g, loss, count = _grad_gpu(ctx, p, xb, tb)
    keep = ~bad
    assert count == keep.sum()
    Lo, go = mlp.grad_device(p, S.round_f32(x[keep]), S.round_f32(t[keep]))
    assert abs(loss - Lo) <= 2e-5 * max(1.0, abs(Lo))
    _check_grad(g, mlp.flatten(go))
    g0, l0, c0 = _grad_gpu(ctx, p, x[:0], t[:0], pad=1)
    assert c0 == 0 and l0 == 0.0 and np.all(g0 == 0.0)


def test_grad_is_deterministic(ctx):
    print("[mlp grad determinism]", flush=True)
    x, t = S.window_records(78, 50000)
    p = _params(4)
    a = _grad_gpu(ctx, p, x, t)
    b = _grad_gpu(ctx, p, x, t)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


def test_adam_step_matches_oracle(ctx):
    import torch
    from paper_1705_02876_amd import kfmi_mlp as M
    print("[mlp adam]", flush=True)
    p = _params(5)
    r = np.random.Generator(np.random.PCG64(6))
    gs = [{k: r.normal(0, 1e-2, v.shape) for k, v in p.items()} for _ in range(3)]
    pd = _dev_params(p)
    md = torch.zeros_like(pd)
    vd = torch.zeros_like(pd)
    packed = M.new_packed()
    st = {}
    po = {k: S.round_f32(v) for k, v in p.items()}
    for i, g in enumerate(gs):
        gd = torch.from_numpy(mlp.flatten(g).astype(np.float32)).cuda()
        M.adam(ctx, pd, gd, md, vd, i + 1, 1e-3, packed)
        mlp.adam_step(po, {k: S.round_f32(v) for k, v in g.items()}, st, lr=1e-3)
    torch.cuda.synchronize()
    want = mlp.flatten(po)
    err = np.abs(pd.cpu().numpy().astype(np.float64) - want)
    # one float32 rounding of the parameter per step, plus the update's own float32 error
    assert np.all(err <= 4 * 2.0 ** -24 * np.abs(want) + 1e-5 * 1e-3), err.max()
    # the packed copy is the repacked new parameters: forward agrees with a fresh pack
    x, _ = S.window_records(79, 100)
    xd = _records_dev(x)
    y1 = M.forward(ctx, xd, packed)
    y2 = M.forward(ctx, xd, M.pack(ctx, pd, M.new_packed()))
    assert torch.equal(y1, y2)


def test_training_follows_the_oracle(ctx):
    import torch
    from paper_1705_02876_amd import kfmi_mlp as M
    print("[mlp training 200 steps]", flush=True)
    x, t = S.window_records(200, 20000)
    p = mlp.init(1)
    tr = M.Trainer(ctx, _dev_params(p), lr=3e-3)
    xd, td = _records_dev(x), _records_dev(t)
    for _ in range(200):
        tr.step(xd, td)
    torch.cuda.synchronize()
    pg = mlp.unflatten(tr.params.cpu().numpy().astype(np.float64))
    po = {k: v.copy() for k, v in p.items()}
    st = {}
    for _ in range(200):
        _, g = mlp.grad(po, x, t)
        mlp.adam_step(po, g, st, lr=3e-3)
    Lg, Lo = mlp.loss(pg, x, t), mlp.loss(po, x, t)
    L_const = np.sum(0.5 + 0.5 * np.log(np.mean(t * t, axis=0)))
    assert abs(Lg - Lo) <= 0.02, (Lg, Lo)
    assert Lg < L_const - 0.5
