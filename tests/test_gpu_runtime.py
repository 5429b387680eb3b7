"""GPU tests of the runtime around the kernels: a HIP graph of binning + building
replays to the eager result (several replays, with eager work and
synchronisation between them, outputs clobbered before each), and the build
autotuner returns a valid launch shape whose results equal the default's,
caches it and round-trips the cache through a file."""
import numpy as np
import pytest

from paper_1705_02876_amd import synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1705_02876_amd import kfmi
    assert torch.cuda.is_available()
    c = kfmi.Context(0)
    yield c
    c.close()


def _tensors(out):
    """The output tensors of a binding result (build() also stores its call arguments under '_' keys)."""
    return {k: v for k, v in out.items() if not k.startswith("_")}


def _host(out):
    return {k: v.cpu().numpy().copy() for k, v in _tensors(out).items()}


def _empty_like_out(out):
    return {k: v.clone() for k, v in _tensors(out).items()}


@pytest.mark.parametrize("mode", [0, 1])
def test_graph_replays_bin_and_build(ctx, mode):
    import torch
    from paper_1705_02876_amd import kfmi, kfmi_build as KB
    print(f"[graph bin+build mode={mode}]", flush=True)
    det = S.detector_full()
    ctx.kf_set_geometry(det.as_float32())
    prob = S.make_build_problem([1500, 2500, 7], det, 68)
    seeds, hits = KB.upload_problem(prob)
    ldh = hits["pos"].shape[1]
    bws = torch.empty(max(kfmi.load_library().kf_bin_hits_workspace_size(ldh, prob.n_events), 4), dtype=torch.uint8,
                      device="cuda")
    cfg = KB.make_cfg(mode=mode)
    wsb = torch.empty(KB.workspace_bytes(cfg, prob.n_events, seeds["n"]), dtype=torch.uint8, device="cuda")
    bins = KB.bin_hits(ctx, hits["layer_offsets"], hits["pos"], hits["cov"], prob.n_events, workspace=bws)
    eager = KB.build(ctx, cfg, seeds, bins, hits["layer_offsets"], prob.n_events, workspace=wsb)
    torch.cuda.synchronize()
    want_bins, want = _host(bins), _host(eager)
    bins_g, out_g = _empty_like_out(bins), _empty_like_out(eager)
    bws_g = torch.empty_like(bws)
    wsb_g = torch.empty_like(wsb)

    def step():
        KB.bin_hits(ctx, hits["layer_offsets"], hits["pos"], hits["cov"], prob.n_events, out=bins_g, workspace=bws_g,
                    check=False)
        KB.build(ctx, cfg, seeds, bins_g, hits["layer_offsets"], prob.n_events, out=out_g, workspace=wsb_g,
                 check=False)

    g = KB.Graph(ctx).capture(step)
    for rep in range(4):
        for v in list(_tensors(bins_g).values()) + list(_tensors(out_g).values()):
            v.fill_(-3)
        # unrelated eager work on the default stream between replays
        eager2 = KB.build(ctx, cfg, seeds, bins, hits["layer_offsets"], prob.n_events, workspace=wsb)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        got_bins, got = _host(bins_g), _host(out_g)
        for k in want_bins:
            assert np.array_equal(got_bins[k], want_bins[k], equal_nan=True), (rep, k)
        S_ = seeds["n"]
        for k in ("n_cands", "cand_chi2", "cand_nhits", "cand_status"):
            assert np.array_equal(got[k][:S_], want[k][:S_], equal_nan=True), (rep, k)
        assert np.array_equal(got["cand_hits"][:, :S_], want["cand_hits"][:, :S_]), rep
        assert np.array_equal(got["best_state"][:, :S_], want["best_state"][:, :S_], equal_nan=True), rep
        del eager2
    g.close()


def test_autotune_picks_valid_shape_and_caches(ctx, tmp_path):
    import time
    import torch
    from paper_1705_02876_amd import kfmi, kfmi_build as KB
    print("[autotune build]", flush=True)
    det = S.detector_full()
    ctx.kf_set_geometry(det.as_float32())
    prob = S.make_build_problem([3000, 4000], det, 69)
    seeds, hits = KB.upload_problem(prob)
    bins = KB.bin_hits(ctx, hits["layer_offsets"], hits["pos"], hits["cov"], prob.n_events)
    cfg = KB.make_cfg(precision=KB.PREC_F32)
    wsb = torch.empty(KB.workspace_bytes(cfg, prob.n_events, seeds["n"]), dtype=torch.uint8, device="cuda")
    ref = _host(KB.build(ctx, cfg, seeds, bins, hits["layer_offsets"], prob.n_events, workspace=wsb))
    out = KB.build(ctx, cfg, seeds, bins, hits["layer_offsets"], prob.n_events, workspace=wsb)
    ms = KB.autotune(ctx, cfg, out, reps=2)
    print(f"[autotune] mode {cfg.mode} waves/block {cfg.waves_per_block} blocks/CU {cfg.blocks_per_cu}: "
          f"{ms:.3f} ms", flush=True)
    assert ms > 0 and cfg.mode in (0, 1) and cfg.waves_per_block in (1, 2, 4) and cfg.blocks_per_cu in (1, 2, 4, 8)
    tuned = _host(KB.build(ctx, cfg, seeds, bins, hits["layer_offsets"], prob.n_events, workspace=wsb))
    torch.cuda.synchronize()
    for k in ref:
        assert np.array_equal(ref[k], tuned[k], equal_nan=True), k
    # cached: same answer without timing
    cfg2 = KB.make_cfg(precision=KB.PREC_F32)
    t0 = time.perf_counter()
    ms2 = KB.autotune(ctx, cfg2, out, reps=50)
    assert time.perf_counter() - t0 < 0.05 and ms2 == ms
    assert (cfg2.mode, cfg2.waves_per_block, cfg2.blocks_per_cu) == (cfg.mode, cfg.waves_per_block, cfg.blocks_per_cu)
    # file round trip into a fresh context
    path = tmp_path / "tune.jsonl"
    KB.autotune_save(ctx, path)
    c2 = kfmi.Context(0)
    c2.kf_set_geometry(det.as_float32())
    KB.autotune_load(c2, path)
    cfg3 = KB.make_cfg(precision=KB.PREC_F32)
    assert KB.autotune(c2, cfg3, out, reps=50) == pytest.approx(ms, rel=1e-5)
    assert (cfg3.mode, cfg3.waves_per_block, cfg3.blocks_per_cu) == (cfg.mode, cfg.waves_per_block, cfg.blocks_per_cu)
    bad = tmp_path / "bad.jsonl"
    bad.write_text('{"key": "x", "mode": 9}\n')
    with pytest.raises(kfmi.KfError):
        KB.autotune_load(c2, bad)
    c2.close()
