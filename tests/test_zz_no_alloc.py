"""kf_build_noalloc (the build entry point that allocates nothing: its work
queue, direction cells and seed order live in the library's static device
scratch) against kf_build with a caller workspace: identical outputs, on two
calls in a row, the second with a smaller problem, in the tiled and the
persistent launch; a problem whose scratch need exceeds the static maximum is
rejected before anything runs."""
import numpy as np
import pytest

from paper_1705_02876_amd import synth as S

pytestmark = pytest.mark.gpu

KEYS = ("n_cands", "cand_hits", "cand_chi2", "cand_nhits", "cand_status", "best_state", "best_cov")


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1705_02876_amd import kfmi
    assert torch.cuda.is_available()
    c = kfmi.Context(0)
    c.kf_set_geometry(S.detector_full().as_float32())
    yield c
    c.close()


def _problem(ctx, sizes, seed):
    from paper_1705_02876_amd import kfmi_build as KB
    prob = S.make_build_problem(sizes, S.detector_full(), seed)
    seeds, hits = KB.upload_problem(prob)
    bins = KB.bin_hits(ctx, hits["layer_offsets"], hits["pos"], hits["cov"], prob.n_events, n_phi=512, n_eta=32)
    return prob, seeds, hits, bins


def _host(out, S_):
    return {k: out[k].cpu().numpy()[..., :S_] if k in ("best_state", "best_cov") else
            (out[k].cpu().numpy()[:, :S_] if k == "cand_hits" else out[k].cpu().numpy()[:S_]) for k in KEYS}


@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_equals_workspace_build(ctx, mode):
    import torch
    from paper_1705_02876_amd import kfmi_build as KB
    big = _problem(ctx, [4000, 2500, 6000], 901)
    small = _problem(ctx, [1200, 700], 902)
    cfg = KB.make_cfg(max_cands=6, mode=mode, precision=KB.PREC_F32, n_phi=512, n_eta=32, waves_per_block=1,
                      blocks_per_cu=2, seed_order=1)
    assert KB.workspace_bytes(cfg, big[0].n_events, big[1]["n"]) > 0
    for tag, (prob, seeds, hits, bins) in (("first call, larger problem", big), ("second call, smaller", small)):
        print(f"[noalloc] mode {mode}: {tag}: {seeds['n']} seeds", flush=True)
        ref = KB.build(ctx, cfg, seeds, bins, hits["layer_offsets"], prob.n_events)
        torch.cuda.synchronize()
        want = _host(ref, seeds["n"])
        got_out = KB.build(ctx, cfg, seeds, bins, hits["layer_offsets"], prob.n_events, noalloc=True)
        torch.cuda.synchronize()
        got = _host(got_out, seeds["n"])
        for k in KEYS:
            assert np.array_equal(got[k], want[k], equal_nan=True), (tag, k)
        assert (want["n_cands"] >= 1).all()


def test_noalloc_rejects_problems_beyond_the_scratch(ctx):
    import ctypes as C
    from paper_1705_02876_amd import kfmi, kfmi_build as KB
    lib = kfmi.load_library()
    cfg = KB.make_cfg(max_cands=6, precision=KB.PREC_F32, seed_order=1)
    n_events, n_seeds = 64, 5_000_000
    need = lib.kf_build_workspace_size(C.byref(cfg), n_events, n_seeds)
    assert need > (16 << 20)
    a = KB.kf_build_args()
    a.n_events, a.n_seeds, a.ld_seed, a.first_layer = n_events, n_seeds, n_seeds, 3
    rc = lib.kf_build_noalloc(ctx.h, C.byref(cfg), C.byref(a))
    assert rc == kfmi.KF_ERR_WORKSPACE
    assert "static maximum" in lib.kf_last_error().decode()
