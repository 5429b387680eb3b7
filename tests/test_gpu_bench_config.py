"""Oracle parity of the build exactly as the benchmark times it.

The batched workload (64 events of log-uniform 1 000 - 50 000 tracks plus 20%
noise hits, 878 k seeds) is binned on the 1024 x 32 grid and built with
N = 6 in single precision with the seed ordering, in every launch shape the
build autotuner can pick (tiled with 1, 2 or 4 waves per block, persistent with
1 or 2 blocks per compute unit).  1 000 seeds sampled from the four largest
events (about 50 000 tracks each, the densest windows) are compared with the
FP64 oracle's binned build on the same events: identical candidate lists on
decision-stable seeds, chi2 within 1e-3 and the best state within 1e-4.

The learned window is checked the same way with a network trained as the
benchmark trains it (residual records of 625 000 fitted tracks, 300 full-batch
Adam steps on the device) at the benchmark's half width of 2.5 network scales.
"""
import numpy as np
import pytest

from paper_1705_02876_amd import synth as S

from kfutil import rounded

from test_gpu_build import _compare

pytestmark = pytest.mark.gpu

N_PHI, N_ETA = 1024, 32
NSIGMA = 2.5


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1705_02876_amd import kfmi
    assert torch.cuda.is_available()
    c = kfmi.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def bench(ctx):
    """The batched workload on the device, binned on the benchmark's grid, and the sampled seeds."""
    from paper_1705_02876_amd import kfmi_build as KB, workloads as W
    print("[bench config] generating the batched workload (64 events)", flush=True)
    det = S.detector_full()
    det32 = det.as_float32()
    prob = W.batched_workload(64, det)
    ctx.kf_set_geometry(det32)
    seeds, hits = KB.upload_problem(prob)
    bins = KB.bin_hits(ctx, hits["layer_offsets"], hits["pos"], hits["cov"], prob.n_events, n_phi=N_PHI, n_eta=N_ETA)
    sizes = np.diff(prob.seed_offsets)
    big = np.argsort(-sizes, kind="stable")[:4]
    rng = np.random.Generator(np.random.PCG64(11))
    sel = np.sort(np.concatenate([rng.choice(np.arange(prob.seed_offsets[e], prob.seed_offsets[e + 1]), 250,
                                             replace=False) for e in big]))
    print(f"[bench config] {prob.seed_state.shape[0]} seeds, {prob.hit_pos.shape[0]} hits; sampled events "
          f"{list(big)} ({list(sizes[big])} seeds)", flush=True)
    return dict(det=det, det32=det32, prob=prob, seeds=seeds, hits=hits, bins=bins, sel=sel)


def _oracle(orc, b, mlp=None):
    prob, det32 = b["prob"], b["det32"]
    print(f"[bench config] oracle build of {b['sel'].size} seeds ({'learned' if mlp is not None else 'plain'})",
          flush=True)
    return orc.build(orc.geometry(det32), prob, max_cands=6, mode=1, hit_pos=rounded(prob.hit_pos),
                     hit_cov_full=S.unpack3(rounded(prob.hit_cov)), seed_state=rounded(prob.seed_state),
                     seed_cov=S.unpack6(rounded(S.pack6(prob.seed_cov))), seeds=b["sel"],
                     mlp_params=None if mlp is None else rounded(mlp), learned_nsigma=float(np.float32(NSIGMA)))


def _gpu(ctx, b, mode, wpb, bpc, packed=None):
    import torch
    from paper_1705_02876_amd import kfmi_build as KB
    cfg = KB.make_cfg(max_cands=6, mode=mode, precision=KB.PREC_F32, n_phi=N_PHI, n_eta=N_ETA, waves_per_block=wpb,
                      blocks_per_cu=bpc, seed_order=1,
                      window_mode=KB.WINDOW_PLAIN if packed is None else KB.WINDOW_LEARNED, learned_nsigma=NSIGMA)
    out = KB.build(ctx, cfg, b["seeds"], b["bins"], b["hits"]["layer_offsets"], b["prob"].n_events,
                   mlp_packed=packed)
    torch.cuda.synchronize()
    sel = torch.as_tensor(b["sel"], device="cuda")
    return dict(n_cands=out["n_cands"][sel].cpu().numpy(),
                cand_hits=out["cand_hits"][:, sel, :].permute(1, 2, 0).cpu().numpy(),  # (S, N, L)
                cand_chi2=out["cand_chi2"][sel].double().cpu().numpy(),
                cand_nhits=out["cand_nhits"][sel].cpu().numpy(),
                cand_status=out["cand_status"][sel].cpu().numpy(),
                best_state=out["best_state"][:, sel].T.double().cpu().numpy())


@pytest.fixture(scope="module")
def oracle_plain(orc, bench):
    return _oracle(orc, bench)


LAUNCHES = [(0, 1, 0), (0, 2, 0), (0, 4, 0), (1, 4, 1), (1, 4, 2), (1, 4, 3)]


@pytest.mark.parametrize("mode,wpb,bpc", LAUNCHES)
def test_bench_build_matches_oracle(ctx, bench, oracle_plain, mode, wpb, bpc):
    print(f"[bench config] plain build mode {mode} waves/block {wpb} blocks/CU {bpc}", flush=True)
    g = _gpu(ctx, bench, mode, wpb, bpc)
    st, n, same = _compare(g, oracle_plain, label=f"bench plain mode={mode} wpb={wpb} bpc={bpc}", min_same=0.9)
    assert st >= 0.5 * n


@pytest.fixture(scope="module")
def trained(ctx, bench):
    """A window network trained like the benchmark's: residual records of 625 000 fitted tracks of the full fit
    workload, 300 Adam steps."""
    import torch
    from paper_1705_02876_amd import window, workloads as W
    from kfutil import fit_inputs_gpu
    print("[bench config] training the window network (625 000 fitted tracks)", flush=True)
    fp = W.fit_workload(bench["det"], 625_000)
    ctx.kf_set_geometry(bench["det32"])
    d = fit_inputs_gpu(fp)
    x, t = window.fit_records(ctx, d, bench["det"].n_layers)
    tr = window.train(ctx, x, t, steps=300)
    torch.cuda.synchronize()
    params = tr.params.detach().cpu().numpy().astype(np.float64)
    del x, t, d
    torch.cuda.empty_cache()
    return tr, params


@pytest.mark.parametrize("mode,wpb,bpc", [(0, 4, 0), (0, 1, 0), (1, 4, 2), (1, 4, 3)])
def test_bench_learned_build_matches_oracle(ctx, orc, bench, trained, mode, wpb, bpc):
    tr, params = trained
    ora = getattr(test_bench_learned_build_matches_oracle, "_ora", None)
    if ora is None:
        ora = _oracle(orc, bench, mlp=params)
        test_bench_learned_build_matches_oracle._ora = ora
    print(f"[bench config] learned build mode {mode} waves/block {wpb} blocks/CU {bpc}; oracle fallbacks "
          f"{int(ora['fallbacks'].sum())}", flush=True)
    assert ora["fallbacks"].sum() > 0
    g = _gpu(ctx, bench, mode, wpb, bpc, packed=tr.packed)
    st, n, same = _compare(g, ora, label=f"bench learned mode={mode} wpb={wpb} bpc={bpc}", min_same=0.85)
    # A seed is decision-stable only if no pair of any layer lies within 1% of its learned box edge; in the four
    # densest events (about 50 000 tracks each) that leaves about 40% of the sampled seeds for exact comparison.
    assert st >= 0.3 * n
