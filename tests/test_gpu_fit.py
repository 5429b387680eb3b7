"""GPU parity of propagate, update and fit against the FP64 oracle (through the C ABI).

Tolerances (kfutil): state 1e-4 relative, chi2 1e-3, covariance 1e-3 of
sqrt(C_ii C_jj).  Both sides see the same float32-rounded inputs; the oracle
computes in double precision.
"""
import numpy as np
import pytest

from paper_1705_02876_amd import synth as S

from kfutil import (GRAZING_COS, check_chi2, check_cov, check_params, fit_inputs_gpu, from_soa_cov, from_soa_state,
                    min_cos_psi, oracle_fit_on_f32, rounded, soa_cov, soa_state, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1705_02876_amd import kfmi
    assert torch.cuda.is_available()
    c = kfmi.Context(0)
    yield c
    c.close()


def _fit_gpu(ctx, fp, pad=0, residuals=False, fp64=False):
    import torch
    d = fit_inputs_gpu(fp, pad)
    ld = d["ld"]
    so = torch.empty(6, ld, dtype=torch.float32, device="cuda")
    co = torch.empty(21, ld, dtype=torch.float32, device="cuda")
    chi2 = torch.empty(ld, dtype=torch.float32, device="cuda")
    nh = torch.empty(ld, dtype=torch.int32, device="cuda")
    st = torch.empty(ld, dtype=torch.int32, device="cuda")
    res = None
    if residuals:
        L = fp.hit_idx.shape[0]
        res = torch.empty(10, d["n"] * (L - 1), dtype=torch.float32, device="cuda")
    ctx.kf_fit(d["state"], d["cov"], d["q"], d["hidx"], d["hpos"], d["hcov"], so, co, chi2, nh, st,
               residual_out=res, n=d["n"], fp64=fp64)
    torch.cuda.synchronize()
    n = d["n"]
    out = (from_soa_state(so, n), from_soa_cov(co, n), chi2.cpu().numpy()[:n].astype(np.float64),
           nh.cpu().numpy()[:n], st.cpu().numpy()[:n])
    if residuals:
        return out, res.cpu().numpy()
    return out


@pytest.mark.parametrize("which,n,pad,fp64", [("small", 1000, 0, False), ("full", 20037, 5, False), ("full", 1, 0, False),
                                             ("full", 255, 1, False), ("small", 1000, 0, True), ("full", 20037, 5, True)])
def test_fit_parity(ctx, orc, which, n, pad, fp64):
    det = S.detector_small() if which == "small" else S.detector_full()
    det32 = det.as_float32()
    fp = S.make_fit_problem(n, det, 100 + n, p_miss=0.0 if which == "small" else 0.05,
                            min_hits=0 if which == "small" else 6)
    ctx.kf_set_geometry(det32)
    gs, gc, gchi, gnh, gst = _fit_gpu(ctx, fp, pad, fp64=fp64)
    os_, oc, ochi, onh, ost = oracle_fit_on_f32(orc, det32, fp)
    print(f"[fit parity] {which} n={n} fp64={fp64}: status gpu {np.bincount(gst)} oracle {np.bincount(ost)}", flush=True)
    # near-tangent loopers may flip between NO_CROSSING and a crossing; they must be rare
    same = gst == ost
    assert same.mean() >= 0.9995 or (~same).sum() <= 1
    ok = same & (gst == 0)
    assert np.array_equal(gnh[ok], onh[ok])
    w1 = check_params(gs[ok], os_[ok], "fit state")
    w2 = check_chi2(gchi[ok], ochi[ok], "fit chi2")
    # covariance: 1e-3 where the track never crosses a layer at a grazing angle; grazing
    # crossings amplify float32 rounding of the state like 1/cos^2 and are held to 1e-2
    graz = min_cos_psi(fp) < GRAZING_COS
    w3 = check_cov(gc[ok & ~graz], oc[ok & ~graz], "fit cov")
    w4 = check_cov(gc[ok & graz], oc[ok & graz], "fit cov (grazing)", rel=1e-2) if (ok & graz).any() else 0.0
    assert graz.mean() < 0.01
    print(f"[fit parity] worst rel: state {w1:.2e} chi2 {w2:.2e} cov {w3:.2e} (grazing {graz.sum()}: {w4:.2e})",
          flush=True)


def test_fit_edge_cases(ctx, orc):
    import torch
    det = S.detector_full()
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    fp = S.make_fit_problem(70, det, 7, p_miss=0.05, min_hits=6)
    fp.hit_idx[:, 3] = -1  # a track without hits: output = input, nhits 0
    fp.state0[5, 0] = np.nan  # non-finite input
    fp.state0[9, 3:5] = [0.02, 0.0]  # pT = 20 MeV: diameter 3.5 cm never reaches r = 4 cm
    gs, gc, gchi, gnh, gst = _fit_gpu(ctx, fp)
    os_, oc, ochi, onh, ost = oracle_fit_on_f32(orc, det32, fp)
    assert gst[3] == 0 and gnh[3] == 0 and np.allclose(gs[3], rounded(fp.state0[3]))
    assert gst[5] == 4 and ost[5] == 4  # NONFINITE
    assert gst[9] == ost[9] == 1
    ok = (gst == 0) & (ost == 0)
    check_params(gs[ok], os_[ok])
    # n = 0 is a no-op
    z = torch.empty(6, 0, device="cuda")
    ctx.kf_fit(z, torch.empty(21, 0, device="cuda"), torch.empty(0, dtype=torch.int8, device="cuda"),
               torch.empty(17, 0, dtype=torch.int32, device="cuda"), torch.empty(3, 1, device="cuda"),
               torch.empty(6, 1, device="cuda"), z, torch.empty(21, 0, device="cuda"), torch.empty(0, device="cuda"),
               torch.empty(0, dtype=torch.int32, device="cuda"), torch.empty(0, dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("fp64", [False, True])
def test_fit_failing_tracks_keep_last_valid_state(ctx, orc, fp64):
    """A track stops at its first failing step and reports the state before it: slow tracks given a hit on
    the outermost layer, which they cannot reach, stop there with the state after the material of the layer
    before; a 20 MeV track stops at the first layer and reports its input."""
    det = S.detector_full()
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    fp = S.make_fit_problem(6000, det, 71, p_miss=0.05, min_hits=6)
    L = det.n_layers
    pt = np.hypot(fp.state0[:, 3], fp.state0[:, 4])
    slow = np.nonzero((fp.hit_idx[L - 1] < 0) & (pt < 0.56))[0]
    donor = int(np.nonzero(fp.hit_idx[L - 1] >= 0)[0][0])
    fp.hit_idx[L - 1, slow] = fp.hit_idx[L - 1, donor]
    first = int(np.nonzero(fp.hit_idx[L - 1] >= 0)[0][1])
    fp.state0[first, 3:5] = [0.02, 0.0]
    gs, gc, gchi, gnh, gst = _fit_gpu(ctx, fp, fp64=fp64)
    os_, oc, ochi, onh, ost = oracle_fit_on_f32(orc, det32, fp)
    stopped = slow[ost[slow] == 1]  # NO_CROSSING on the outermost layer
    print(f"[fit failures] slow tracks {slow.size}, stopped at the last layer {stopped.size}", flush=True)
    assert stopped.size >= 5
    assert np.array_equal(gst[stopped], ost[stopped])
    assert gst[first] == ost[first] == 1 and gnh[first] == 0 and gchi[first] == 0
    assert np.array_equal(gs[first], rounded(fp.state0[first]))
    sel = np.concatenate([stopped, [first]])
    assert np.array_equal(gnh[sel], onh[sel])
    check_params(gs[sel], os_[sel], "last valid state")
    check_chi2(gchi[stopped], ochi[stopped], "chi2 up to the failure")
    check_cov(gc[sel], oc[sel], "last valid covariance", rel=1e-2)
    assert (gst == ost).mean() > 0.999


def test_fit_rejects_bad_arguments(ctx):
    import torch
    from paper_1705_02876_amd import kfmi
    det = S.detector_full()
    ctx.kf_set_geometry(det.as_float32())
    st = torch.zeros(6, 10, device="cuda")
    with pytest.raises(kfmi.KfError):
        ctx.kf_fit(st, torch.zeros(21, 10, device="cuda"), torch.zeros(10, dtype=torch.int8, device="cuda"),
                   torch.zeros(17, 5, dtype=torch.int32, device="cuda"),  # ld_idx < n
                   torch.zeros(3, 10, device="cuda"), torch.zeros(6, 10, device="cuda"), st,
                   torch.zeros(21, 10, device="cuda"), torch.zeros(10, device="cuda"),
                   torch.zeros(10, dtype=torch.int32, device="cuda"), torch.zeros(10, dtype=torch.int32, device="cuda"))
    bad = kfmi.geometry_struct(det)
    bad.r[3] = bad.r[2]
    with pytest.raises(kfmi.KfError):
        ctx.kf_set_geometry(bad)
    ctx.kf_set_geometry(det.as_float32())


def test_propagate_nonfinite_statuses(ctx, orc):
    """Statuses of the propagation for non-finite covariance entries, alone and with a crossing that fails (a
    failed crossing still reports the non-finite input), and for non-finite states, equal to the oracle's."""
    import torch
    det = S.detector_full()
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    g = orc.geometry(det32)
    fp = S.make_fit_problem(40, det, 56)
    tp, tm = fp.extra["true_pos"][3], fp.extra["true_mom"][3]
    ok = np.flatnonzero(np.isfinite(tp[:, 0]))[:8]
    s0 = np.concatenate([tp, tm], axis=1)[ok]
    C0 = fp.cov0[ok].copy()
    q = fp.q[ok]
    C0[0, 4, 2] = C0[0, 2, 4] = np.nan        # non-finite covariance, crossing reached
    C0[1, 5, 5] = np.inf                       # infinite variance, crossing reached
    s0[2, 3:5] = [0.02, 0.0]                   # pT = 20 MeV: no crossing of the outer radius...
    C0[2, 0, 0] = np.nan                       # ...and a non-finite covariance: non-finite wins
    s0[3, 3:5] = [0.02, 0.0]                   # no crossing alone
    s0[4, 1] = np.nan                          # non-finite state
    s0[5, 3:5] = [0.02, 0.0]                   # no crossing with an infinite covariance entry
    C0[5, 3, 1] = C0[5, 1, 3] = -np.inf
    for material_layer in (-1, 3):
        st_d = to_dev(soa_state(s0))
        cv_d = to_dev(soa_cov(C0))
        q_d = to_dev(q.astype(np.int8))
        stat = torch.empty(len(ok), dtype=torch.int32, device="cuda")
        ctx.kf_propagate_to_r(st_d, cv_d, q_d, stat, r_scalar=float(det32.radii[12]), z_half=float(det32.z_half),
                              material_layer=material_layer)
        torch.cuda.synchronize()
        gst = stat.cpu().numpy()
        _, _, ost = orc.propagate(g, rounded(s0), rounded(C0), q, r_scalar=det32.radii[12], z_half=det32.z_half,
                                  material_layer=material_layer)
        print(f"[propagate statuses] material {material_layer}: gpu {gst.tolist()} oracle {ost.tolist()}", flush=True)
        assert np.array_equal(gst, ost)
        assert gst[0] == gst[1] == gst[2] == gst[4] == gst[5] == 4
        assert gst[3] == 1


def test_propagate_parity(ctx, orc):
    import torch
    det = S.detector_full()
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    g = orc.geometry(det32)
    n = 5003
    fp = S.make_fit_problem(n, det, 55)
    # start on layer 3 (truth there) with the workload's prior widths, go to layer 4 with layer-3 material
    tp = fp.extra["true_pos"][3]
    tm = fp.extra["true_mom"][3]
    ok = np.isfinite(tp[:, 0])
    s0 = np.concatenate([tp, tm], axis=1)[ok]
    C0 = fp.cov0[ok]
    q = fp.q[ok]
    m = s0.shape[0]
    st_d = to_dev(soa_state(s0))
    cv_d = to_dev(soa_cov(C0))
    q_d = to_dev(q.astype(np.int8))
    stat = torch.empty(m, dtype=torch.int32, device="cuda")
    ctx.kf_propagate_to_r(st_d, cv_d, q_d, stat, r_scalar=float(det32.radii[4]), z_half=float(det32.z_half),
                          material_layer=3)
    torch.cuda.synchronize()
    gs, gc = from_soa_state(st_d), from_soa_cov(cv_d)
    gst = stat.cpu().numpy()
    os_, oc, ost = orc.propagate(g, rounded(s0), rounded(S.unpack6(S.pack6(C0))), q, r_scalar=det32.radii[4],
                                 z_half=det32.z_half, material_layer=3)
    assert np.array_equal(gst, ost)
    good = gst == 0
    w = check_params(gs[good], os_[good], "propagate state")
    wc = check_cov(gc[good], oc[good], "propagate cov")
    print(f"[propagate parity] n={m} worst state {w:.2e} cov {wc:.2e}", flush=True)
    # exits: steep tracks leave |z| < z_half; soft ones never reach r = 100
    s1 = np.array([[0, 0, 0, 5.0, 0.0, 20.0], [0, 0, 0, 0.3, 0.0, 0.1], [0, 0, 0, 1.0, 1.0, 0.2]])
    st_d = to_dev(soa_state(s1))
    cv_d = to_dev(soa_cov(np.repeat(np.eye(6)[None] * 1e-4, 3, 0)))
    stat = torch.empty(3, dtype=torch.int32, device="cuda")
    ctx.kf_propagate_to_r(st_d, cv_d, to_dev(np.array([1, 1, -1], np.int8)), stat,
                          r_target=to_dev(np.array([20.0, 100.0, 10.0], np.float32)), z_half=50.0)
    assert list(stat.cpu().numpy()) == [2, 1, 0]


def test_update_parity(ctx, orc):
    import torch
    det = S.detector_full()
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    g = orc.geometry(det32)
    fp = S.make_fit_problem(3001, det, 56)
    s1, C1, st = orc.propagate(g, rounded(fp.state0), rounded(S.unpack6(S.pack6(fp.cov0))), fp.q,
                               r_scalar=det32.radii[0])
    assert (st == 0).all()
    hits = fp.hit_pos[fp.hit_idx[0]]
    hc = fp.hit_cov[fp.hit_idx[0]]
    s1r, C1r = rounded(s1), rounded(C1)
    for chi2_only in (True, False):
        st_d = to_dev(soa_state(s1r))
        cv_d = to_dev(soa_cov(C1r))
        chi2 = torch.empty(s1.shape[0], device="cuda")
        stat = torch.empty(s1.shape[0], dtype=torch.int32, device="cuda")
        ctx.kf_update(st_d, cv_d, to_dev(np.ascontiguousarray(rounded(hits).T.astype(np.float32))),
                      to_dev(np.ascontiguousarray(hc.T.astype(np.float32))), chi2, stat, chi2_only=chi2_only)
        torch.cuda.synchronize()
        os_, oc, ochi, ost = orc.update(s1r, C1r, rounded(hits), S.unpack3(rounded(hc)), chi2_only=chi2_only)
        assert np.array_equal(stat.cpu().numpy(), ost)
        check_chi2(chi2.cpu().numpy().astype(np.float64), ochi, "update chi2")
        check_params(from_soa_state(st_d), os_, "update state")
        check_cov(from_soa_cov(cv_d), oc, "update cov")
        if chi2_only:
            assert np.array_equal(from_soa_state(st_d), s1r.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("fp64", [False, True])
def test_fit_full_size_sampled(ctx, orc, fp64):
    """2M tracks, 17 layers (the bench workload and launch); 3000 sampled tracks against the oracle."""
    det = S.detector_full()
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    from paper_1705_02876_amd import workloads
    fp = workloads.fit_workload(det, 2_000_000)
    gs, gc, gchi, gnh, gst = _fit_gpu(ctx, fp, fp64=fp64)
    rng = np.random.Generator(np.random.PCG64(9))
    idx = np.sort(rng.choice(fp.state0.shape[0], 3000, replace=False))
    sub = S.FitProblem(det, fp.q[idx], fp.state0[idx], fp.cov0[idx], fp.hit_idx[:, idx], fp.hit_pos, fp.hit_cov,
                       fp.truth_state0[idx], fp.truth_last[idx], fp.last_layer[idx],
                       extra=dict(true_pos=fp.extra["true_pos"][:, idx], true_mom=fp.extra["true_mom"][:, idx]))
    os_, oc, ochi, onh, ost = oracle_fit_on_f32(orc, det32, sub)
    same = gst[idx] == ost
    assert (~same).sum() <= 1
    ok = same & (ost == 0)
    assert np.array_equal(gnh[idx][ok], onh[ok])
    check_params(gs[idx][ok], os_[ok], "full-size fit state")
    check_chi2(gchi[idx][ok], ochi[ok], "full-size fit chi2")
    graz = min_cos_psi(sub) < GRAZING_COS
    check_cov(gc[idx][ok & ~graz], oc[ok & ~graz], "full-size fit cov")
    # properties over all 2M: finite outputs, nhits = assigned hits for converged tracks
    allok = gst == 0
    assert allok.mean() > 0.999
    assert np.isfinite(gs[allok]).all() and np.isfinite(gchi[allok]).all()
    assert np.array_equal(gnh[allok], (fp.hit_idx >= 0).sum(axis=0)[allok])


def test_residual_emission(ctx, orc):
    det = S.detector_full()
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    fp = S.make_fit_problem(500, det, 58, p_miss=0.05, min_hits=6)
    (gs, gc, gchi, gnh, gst), res = _fit_gpu(ctx, fp, residuals=True)
    L = det.n_layers
    rows = res.reshape(10, 500, L - 1)
    has = fp.hit_idx[1:].T >= 0  # (n, L-1)
    last = fp.last_layer
    finite = np.isfinite(rows[0])
    # a record for every hit on layer >= 1 up to the last one, NaN elsewhere
    assert np.array_equal(finite, has)
    # targets: tangential offsets are O(prediction sigma), z offsets too
    assert np.nanstd(rows[8]) < 0.5 and np.nanstd(rows[9]) < 2.0


def test_fit_and_smoother_64bit_addressing(ctx, orc):
    """Arrays whose extent crosses 2^30 elements take the 64-bit addressing kernels (fit_kernel_i64,
    smooth_fwd_kernel_i64, smooth_bwd_kernel_i64): a covariance array with ld = 51.2 M columns for the fit
    (21 ld > 2^30, rows past 4 GiB) and smoothed rows with ld = 3.1 M for the smoother (17 * 21 ld > 2^30).
    Only the first n columns hold tracks.  The results equal the 32-bit kernels' bit for bit and the
    oracle's at the usual tolerances."""
    import torch
    det = S.detector_full()
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    L = det.n_layers
    n = 3000
    fp = S.make_fit_problem(n, det, 4097, p_miss=0.05, min_hits=6)
    base = fit_inputs_gpu(fp)
    os_, oc, ochi, onh, ost = oracle_fit_on_f32(orc, det32, fp)

    def wide(t, ld):
        w = torch.empty(t.shape[0], ld, dtype=t.dtype, device="cuda")
        w[:, :n] = t[:, :n]
        return w

    # fit: narrow (ld = n) and wide (ld = 51.2 M) launches on the same tracks
    ldw = 51_200_000
    assert 21 * ldw > (1 << 30) and 21 * n < (1 << 30)
    outs = []
    for ld in (n, ldw):
        print(f"[64-bit addressing] fit, ld = {ld}", flush=True)
        st_in, cv_in = (base["state"], base["cov"]) if ld == n else (wide(base["state"], ld), wide(base["cov"], ld))
        so = torch.empty(6, ld, dtype=torch.float32, device="cuda")
        co = torch.empty(21, ld, dtype=torch.float32, device="cuda")
        chi2 = torch.empty(n, dtype=torch.float32, device="cuda")
        nh = torch.empty(n, dtype=torch.int32, device="cuda")
        st = torch.empty(n, dtype=torch.int32, device="cuda")
        ctx.kf_fit(st_in, cv_in, base["q"], base["hidx"], base["hpos"], base["hcov"], so, co, chi2, nh, st, n=n)
        torch.cuda.synchronize()
        outs.append((so[:, :n].cpu().numpy(), co[:, :n].cpu().numpy(), chi2.cpu().numpy(), nh.cpu().numpy(),
                     st.cpu().numpy()))
        del st_in, cv_in, so, co
        torch.cuda.empty_cache()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b, equal_nan=True)
    gs, gc = outs[1][0].T.astype(np.float64), S.unpack6(outs[1][1].T.astype(np.float64))
    gst = outs[1][4]
    ok = (gst == 0) & (ost == 0)
    assert ok.mean() > 0.995
    check_params(gs[ok], os_[ok], "wide fit state")
    check_chi2(outs[1][2][ok].astype(np.float64), ochi[ok], "wide fit chi2")
    graz = min_cos_psi(fp) < GRAZING_COS
    check_cov(gc[ok & ~graz], oc[ok & ~graz], "wide fit cov")

    # smoother: rows (L, 21, ld) with ld = 3.1 M cross 2^30 elements
    lds = 3_100_000
    assert L * 21 * lds > (1 << 30) and L * 21 * n < (1 << 30)
    rows = []
    for ld in (n, lds):
        print(f"[64-bit addressing] smoother, ld = {ld}", flush=True)
        st_in, cv_in = (base["state"], base["cov"]) if ld == n else (wide(base["state"], ld), wide(base["cov"], ld))
        rs = torch.empty(L, 6, ld, dtype=torch.float32, device="cuda")
        rc = torch.empty(L, 21, ld, dtype=torch.float32, device="cuda")
        st = torch.empty(n, dtype=torch.int32, device="cuda")
        ctx.kf_smooth(st_in, cv_in, base["q"], base["hidx"], base["hpos"], base["hcov"], rs, rc, st, n=n)
        torch.cuda.synchronize()
        rows.append((rs[:, :, :n].cpu().numpy(), rc[:, :, :n].cpu().numpy(), st.cpu().numpy()))
        del st_in, cv_in, rs, rc
        torch.cuda.empty_cache()
    for a, b in zip(rows[0], rows[1]):
        assert np.array_equal(a, b, equal_nan=True)
    oss, osc, osst = orc.smooth(orc.geometry(det32), rounded(fp.state0), rounded(S.unpack6(S.pack6(fp.cov0))),
                                fp.q, fp.hit_idx, rounded(fp.hit_pos), S.unpack3(rounded(fp.hit_cov)))
    gss = rows[1][0].transpose(2, 0, 1).astype(np.float64)
    okk = (rows[1][2] == 0) & (osst == 0)
    fin = np.isfinite(oss[..., 0]) & okk[:, None]
    assert np.array_equal(fin, np.isfinite(gss[..., 0]) & okk[:, None])
    check_params(gss[fin], oss[fin], "wide smoothed state")
