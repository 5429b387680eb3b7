"""GPU tests of the runtime around the kernels: a HIP graph of binning + building
replays to the eager result (several replays, with eager work and
synchronisation between them, outputs clobbered before each), and the build
autotuner returns a valid launch shape whose results equal the default's,
caches it and round-trips the cache through a file; cache keys carry the
device architecture and the kernel source digest; the fit autotuner."""
import re

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
    assert ms > 0 and cfg.mode in (0, 1, 2) and cfg.waves_per_block in (1, 2, 4) and cfg.blocks_per_cu in (1, 2, 3, 4, 8, 12, 14)
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


def test_autotune_cache_keyed_by_arch_and_sources(ctx, tmp_path):
    """Cache keys carry the device architecture and the digest of the kernel sources the library was built
    from: an entry whose digest differs is never used."""
    import torch
    from paper_1705_02876_amd import build_lib, kfmi, kfmi_build as KB
    print("[autotune keys]", flush=True)
    det = S.detector_full()
    ctx.kf_set_geometry(det.as_float32())
    prob = S.make_build_problem([1500], det, 70)
    seeds, hits = KB.upload_problem(prob)
    bins = KB.bin_hits(ctx, hits["layer_offsets"], hits["pos"], hits["cov"], prob.n_events)
    cfg = KB.make_cfg(precision=KB.PREC_F32, mode=KB.BUILD_TILED)
    out = KB.build(ctx, cfg, seeds, bins, hits["layer_offsets"], prob.n_events)
    c2 = kfmi.Context(0)
    c2.kf_set_geometry(det.as_float32())
    ms = KB.autotune(c2, cfg, out, reps=1)
    path = tmp_path / "tune.jsonl"
    KB.autotune_save(c2, path)
    lines = path.read_text().splitlines()
    digest = build_lib.source_digest()
    assert lines and all(f"gfx950" in ln and digest in ln for ln in lines), lines
    # the same entry under another digest, with a time no measurement gives: loaded, but never matched
    path2 = tmp_path / "stale.jsonl"
    path2.write_text("\n".join(re.sub(r'"ms": [^}]*', '"ms": 1e9', ln.replace(digest, "0" * 16)) for ln in lines)
                     + "\n")
    c3 = kfmi.Context(0)
    c3.kf_set_geometry(det.as_float32())
    KB.autotune_load(c3, path2)
    cfg3 = KB.make_cfg(precision=KB.PREC_F32, mode=KB.BUILD_TILED)
    ms3 = KB.autotune(c3, cfg3, out, reps=1)
    torch.cuda.synchronize()
    assert ms3 < 1e8 and ms > 0
    c2.close()
    c3.close()


def test_fit_autotune(ctx, tmp_path):
    """kf_fit_autotune picks a block size of 64, 128 or 256 threads; fits launched with it give bit-identical
    outputs (tracks are independent); the entry is cached and survives a save / load round trip."""
    import time
    import torch
    from paper_1705_02876_amd import kfmi
    print("[fit autotune]", flush=True)
    det = S.detector_full()
    ctx.kf_set_geometry(det.as_float32())
    fp = S.make_fit_problem(20000, det, 71, p_miss=0.05, min_hits=6)
    n = fp.state0.shape[0]
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()
    args = [f32(fp.state0.T), f32(S.pack6(fp.cov0).T), torch.from_numpy(fp.q.astype(np.int8)).cuda(),
            torch.from_numpy(np.ascontiguousarray(fp.hit_idx)).cuda(), f32(fp.hit_pos.T), f32(fp.hit_cov.T)]

    def outs():
        return [torch.empty(6, n, device="cuda"), torch.empty(21, n, device="cuda"), torch.empty(n, device="cuda"),
                torch.empty(n, dtype=torch.int32, device="cuda"), torch.empty(n, dtype=torch.int32, device="cuda")]

    c2 = kfmi.Context(0)
    c2.kf_set_geometry(det.as_float32())
    ref = outs()
    c2.kf_fit(*args, *ref)  # default block size
    o = outs()
    block, ms = c2.kf_fit_autotune(*args, *o, reps=3)
    print(f"[fit autotune] block {block}: {ms:.4f} ms", flush=True)
    assert block in (64, 128, 256) and ms > 0
    tuned = outs()
    c2.kf_fit(*args, *tuned)
    torch.cuda.synchronize()
    for a, b in zip(ref, tuned):
        assert torch.equal(a, b) or torch.equal(torch.nan_to_num(a, nan=7.0), torch.nan_to_num(b, nan=7.0))
    t0 = time.perf_counter()
    assert c2.kf_fit_autotune(*args, *o, reps=50) == (block, ms)
    assert time.perf_counter() - t0 < 0.05
    path = tmp_path / "fit.jsonl"
    from paper_1705_02876_amd import kfmi_build as KB
    KB.autotune_save(c2, path)
    assert '"fit_block"' in path.read_text()
    c3 = kfmi.Context(0)
    c3.kf_set_geometry(det.as_float32())
    KB.autotune_load(c3, path)
    b3, ms3 = c3.kf_fit_autotune(*args, *o, reps=50)
    assert b3 == block and ms3 == pytest.approx(ms, rel=1e-5)
    c2.close()
    c3.close()
