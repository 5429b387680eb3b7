"""GPU parity of the smoother (kf_smooth) against the FP64 oracle (through the C ABI).

Every layer's smoothed row is compared with the oracle's at kfutil's
tolerances: state 1e-4 relative, covariance 1e-3 of sqrt(C_ii C_jj) away from
grazing crossings, 1e-2 at them.  Rows after the last hit layer are NaN on both
sides.  A failed fit leaves the filtered rows of the layers it completed.
"""
import dataclasses

import numpy as np
import pytest

from paper_1705_02876_amd import synth as S

from kfutil import GRAZING_COS, check_cov, check_params, fit_inputs_gpu, min_cos_psi, rounded

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1705_02876_amd import kfmi
    assert torch.cuda.is_available()
    c = kfmi.Context(0)
    yield c
    c.close()


def _smooth_gpu(ctx, fp, pad=0, fp64=False, cols=None):
    """Smoothed rows as (n, L, 6) and (n, L, 6, 6) float64 (only the columns `cols` if given)."""
    import torch
    d = fit_inputs_gpu(fp, pad)
    ld, n = d["ld"], d["n"]
    L = fp.hit_idx.shape[0]
    so = torch.full((L, 6, ld), -7.0, dtype=torch.float32, device="cuda")
    co = torch.full((L, 21, ld), -7.0, dtype=torch.float32, device="cuda")
    st = torch.empty(ld, dtype=torch.int32, device="cuda")
    chi2 = torch.empty(ld, dtype=torch.float32, device="cuda")
    nh = torch.empty(ld, dtype=torch.int32, device="cuda")
    ctx.kf_smooth(d["state"], d["cov"], d["q"], d["hidx"], d["hpos"], d["hcov"], so, co, st, chi2_out=chi2,
                  nhits_out=nh, n=n, fp64=fp64)
    torch.cuda.synchronize()
    sel = torch.arange(n, device="cuda") if cols is None else torch.as_tensor(cols, device="cuda")
    s = so[:, :, sel].permute(2, 0, 1).double().cpu().numpy()
    cp = co[:, :, sel].permute(2, 0, 1).double().cpu().numpy()  # (n, L, 21)
    c = S.unpack6(cp.reshape(-1, 21)).reshape(cp.shape[0], L, 6, 6)
    if pad:
        assert (so[:, :, n:] == -7.0).all() and (co[:, :, n:] == -7.0).all()  # padding untouched
    stn = st.cpu().numpy()[:n]
    return s, c, stn, chi2.cpu().numpy()[:n], nh.cpu().numpy()[:n]


def _oracle_smooth(orc, det32, fp):
    g = orc.geometry(det32)
    return orc.smooth(g, rounded(fp.state0), rounded(S.unpack6(S.pack6(fp.cov0))), fp.q, fp.hit_idx,
                      rounded(fp.hit_pos), S.unpack3(rounded(fp.hit_cov)))


def _compare_rows(gs, gc, os_, oc, ok, graz, name):
    """Rows of converged tracks up to their last hit layer; NaN after it."""
    fin = np.isfinite(os_[..., 0])
    assert np.array_equal(fin[ok], np.isfinite(gs[..., 0])[ok]), f"{name}: rows present differ"
    m = fin & ok[:, None]
    w1 = check_params(gs[m], os_[m], f"{name} state")
    mg = fin & (ok & ~graz)[:, None]
    w2 = check_cov(gc[mg], oc[mg], f"{name} cov")
    mgz = fin & (ok & graz)[:, None]
    w3 = check_cov(gc[mgz], oc[mgz], f"{name} cov (grazing)", rel=1e-2) if mgz.any() else 0.0
    assert np.isnan(gs[ok][~fin[ok]]).all() and np.isnan(gc[ok][~fin[ok]]).all()
    return w1, w2, w3


@pytest.mark.parametrize("which,n,pad,fp64", [("small", 1000, 0, False), ("full", 20037, 5, False), ("full", 1, 0, False),
                                             ("full", 255, 1, False), ("small", 1000, 0, True), ("full", 5003, 3, True)])
def test_smooth_parity(ctx, orc, which, n, pad, fp64):
    det = S.detector_small() if which == "small" else S.detector_full()
    det32 = det.as_float32()
    fp = S.make_fit_problem(n, det, 300 + n, p_miss=0.0 if which == "small" else 0.05,
                            min_hits=0 if which == "small" else 6)
    ctx.kf_set_geometry(det32)
    print(f"[smooth parity] {which} n={n} pad={pad} fp64={fp64}", flush=True)
    gs, gc, gst, gchi, gnh = _smooth_gpu(ctx, fp, pad, fp64=fp64)
    os_, oc, ost = _oracle_smooth(orc, det32, fp)
    same = gst == ost
    assert same.mean() >= 0.9995 or (~same).sum() <= 1
    ok = same & (gst == 0)
    graz = min_cos_psi(fp) < GRAZING_COS
    w = _compare_rows(gs, gc, os_, oc, ok, graz, "smooth")
    assert np.array_equal(gnh[ok], (fp.hit_idx >= 0).sum(axis=0)[ok])
    print(f"[smooth parity] worst rel: state {w[0]:.2e} cov {w[1]:.2e} grazing {w[2]:.2e}", flush=True)


def test_smooth_last_row_is_the_fit(ctx):
    """The last hit layer's row is the fit's output, bit for bit (same forward arithmetic)."""
    import torch
    det = S.detector_full()
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    fp = S.make_fit_problem(3000, det, 77, p_miss=0.05, min_hits=6)
    gs, gc, gst, gchi, gnh = _smooth_gpu(ctx, fp)
    d = fit_inputs_gpu(fp)
    so = torch.empty(6, d["ld"], device="cuda")
    co = torch.empty(21, d["ld"], device="cuda")
    chi2 = torch.empty(d["ld"], device="cuda")
    nh = torch.empty(d["ld"], dtype=torch.int32, device="cuda")
    st = torch.empty(d["ld"], dtype=torch.int32, device="cuda")
    ctx.kf_fit(d["state"], d["cov"], d["q"], d["hidx"], d["hpos"], d["hcov"], so, co, chi2, nh, st)
    torch.cuda.synchronize()
    fs = so.double().cpu().numpy().T
    fc = S.unpack6(co.double().cpu().numpy().T)
    ok = gst == 0
    assert np.array_equal(st.cpu().numpy(), gst)
    ar = np.arange(fp.q.size)[ok]
    last = fp.last_layer[ok]
    assert np.array_equal(gs[ar, last], fs[ok]) and np.array_equal(gc[ar, last], fc[ok])
    assert np.array_equal(gchi, chi2.cpu().numpy()) and np.array_equal(gnh, nh.cpu().numpy())


@pytest.mark.parametrize("fp64", [False, True])
def test_smooth_failed_tracks_keep_filtered_rows(ctx, orc, fp64):
    """Fitted with far more energy loss than simulated: slow tracks stop in the
    material; their completed rows are the filtered states, the rest NaN."""
    fp = S.make_fit_problem(3000, S.detector_full(), 31, smear=True, min_hits=6)
    det32 = dataclasses.replace(S.detector_full(), eloss_per_x0=6.0).as_float32()
    ctx.kf_set_geometry(det32)
    gs, gc, gst, gchi, gnh = _smooth_gpu(ctx, fp, fp64=fp64)
    os_, oc, ost = _oracle_smooth(orc, det32, fp)
    stopped = np.nonzero((ost == 16) & (gst == 16))[0]
    print(f"[smooth failures] stopped {stopped.size} of {fp.q.size}", flush=True)
    assert stopped.size >= 20 and (gst == ost).mean() > 0.995
    fin = np.isfinite(os_[stopped, :, 0])
    assert np.array_equal(fin, np.isfinite(gs[stopped, :, 0]))
    check_params(gs[stopped][fin], os_[stopped][fin], "filtered rows of stopped tracks")
    check_cov(gc[stopped][fin], oc[stopped][fin], "filtered rows of stopped tracks", rel=1e-2)
    ok = (gst == 0) & (ost == 0)
    graz = min_cos_psi(fp) < GRAZING_COS
    _compare_rows(gs, gc, os_, oc, ok, graz, "smooth (heavy loss)")


def test_smooth_edge_cases(ctx, orc):
    import torch
    det = S.detector_full()
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    fp = S.make_fit_problem(70, det, 7, p_miss=0.05, min_hits=6)
    fp.hit_idx[:, 3] = -1  # no hits: every row NaN, status 0
    fp.hit_idx[1:, 4] = -1
    fp.hit_idx[0, 4] = max(fp.hit_idx[0, 5], 0)  # one hit on the first layer: one row, the filtered state
    fp.state0[5, 0] = np.nan  # non-finite input
    fp.state0[9, 3:5] = [0.02, 0.0]  # 20 MeV: never reaches the first layer
    gs, gc, gst, gchi, gnh = _smooth_gpu(ctx, fp)
    os_, oc, ost = _oracle_smooth(orc, det32, fp)
    assert gst[3] == 0 and np.isnan(gs[3]).all() and np.isnan(gc[3]).all()
    assert gst[4] == 0 and np.isfinite(gs[4, 0]).all() and np.isnan(gs[4, 1:]).all()
    assert gst[5] == ost[5] == 4 and np.isnan(gs[5]).all()
    assert gst[9] == ost[9] == 1 and np.isnan(gs[9]).all()
    ok = (gst == 0) & (ost == 0)
    _compare_rows(gs, gc, os_, oc, ok, min_cos_psi(fp) < GRAZING_COS, "smooth edge")
    # n = 0 is a no-op; wrong output shapes and flags are refused
    L = det.n_layers
    e = lambda *s, dt=torch.float32: torch.empty(*s, dtype=dt, device="cuda")
    ctx.kf_smooth(e(6, 0), e(21, 0), e(0, dt=torch.int8), e(L, 0, dt=torch.int32), e(3, 1), e(6, 1), e(L, 6, 0),
                  e(L, 21, 0), e(0, dt=torch.int32))
    with pytest.raises(ValueError):
        ctx.kf_smooth(e(6, 4), e(21, 4), e(4, dt=torch.int8), e(L, 4, dt=torch.int32), e(3, 1), e(6, 1), e(6, 4),
                      e(21, 4), e(4, dt=torch.int32))


def test_smooth_full_size_sampled(ctx, orc):
    """2M tracks, 17 layers (the fit's bench workload), the launch the bench times; 1500 sampled tracks
    against the oracle, and properties over all of them."""
    det = S.detector_full()
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    from paper_1705_02876_amd import workloads
    fp = workloads.fit_workload(det, 2_000_000)
    rng = np.random.Generator(np.random.PCG64(19))
    idx = np.sort(rng.choice(fp.state0.shape[0], 1500, replace=False))
    gs, gc, gst, gchi, gnh = _smooth_gpu(ctx, fp, cols=idx)
    sub = S.FitProblem(det, fp.q[idx], fp.state0[idx], fp.cov0[idx], fp.hit_idx[:, idx], fp.hit_pos, fp.hit_cov,
                       fp.truth_state0[idx], fp.truth_last[idx], fp.last_layer[idx],
                       extra=dict(true_pos=fp.extra["true_pos"][:, idx], true_mom=fp.extra["true_mom"][:, idx]))
    os_, oc, ost = _oracle_smooth(orc, det32, sub)
    same = gst[idx] == ost
    assert (~same).sum() <= 1
    ok = same & (ost == 0)
    _compare_rows(gs, gc, os_, oc, ok, min_cos_psi(sub) < GRAZING_COS, "full-size smooth")
    assert (gst == 0).mean() > 0.999


@pytest.mark.parametrize("n_layers", [1, 2])
def test_smooth_few_layers(ctx, orc, n_layers):
    """One layer: the only row is the filtered state (no backward step).  Two layers: one backward step."""
    det = dataclasses.replace(S.detector_full(), radii=tuple(S.detector_full().radii[:n_layers]))
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    fp = S.make_fit_problem(300, det, 900 + n_layers, p_miss=0.0, min_hits=n_layers)
    gs, gc, gst, gchi, gnh = _smooth_gpu(ctx, fp)
    os_, oc, ost = _oracle_smooth(orc, det32, fp)
    ok = (gst == 0) & (ost == 0)
    assert ok.mean() > 0.99
    _compare_rows(gs, gc, os_, oc, ok, min_cos_psi(fp) < GRAZING_COS, f"smooth {n_layers} layers")
