"""The learned search window end to end on the GPU: residual records from
kf_fit, full-batch training with the device kernels, then the learned build
against the plain build on the same events, judged against the simulation
truth (efficiency: the best candidate holds >= 7 hits of its seed's track and
>= 75% of its hits are that track's).

Checks: training lowers the loss below the constant-width model's; the learned
build examines fewer hits; its efficiency is within 0.5 percentage points of
the plain build's.
"""
import numpy as np
import pytest

from paper_1705_02876_amd import synth as S

from kfutil import fit_inputs_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1705_02876_amd import kfmi
    assert torch.cuda.is_available()
    c = kfmi.Context(0)
    yield c
    c.close()


def _build(ctx, prob, det32, packed=None, nsigma=4.0, N=6):
    import torch
    from paper_1705_02876_amd import judge, kfmi_build as KB
    ctx.kf_set_geometry(det32)
    seeds, hits = KB.upload_problem(prob)
    bins = KB.bin_hits(ctx, hits["layer_offsets"], hits["pos"], hits["cov"], prob.n_events)
    cfg = KB.make_cfg(max_cands=N, mode=KB.BUILD_PERSISTENT,
                      window_mode=KB.WINDOW_PLAIN if packed is None else KB.WINDOW_LEARNED, learned_nsigma=nsigma)
    cnt = torch.zeros(KB.BUILD_COUNTERS, dtype=torch.int64, device="cuda")
    out = KB.build(ctx, cfg, seeds, bins, hits["layer_offsets"], prob.n_events, counters=cnt, mlp_packed=packed)
    torch.cuda.synchronize()
    best = out["cand_hits"][:, : seeds["n"], 0].T.cpu().numpy()
    return judge.judge_problem(prob, best), cnt.cpu().numpy()


def test_trained_window_keeps_efficiency_and_examines_fewer_hits(ctx):
    import torch
    from paper_1705_02876_amd import window
    det = S.detector_full()
    det32 = det.as_float32()
    ctx.kf_set_geometry(det32)
    fp = S.make_fit_problem(100000, det, 1705028790, p_miss=0.05, min_hits=6)
    d = fit_inputs_gpu(fp)
    x, t = window.fit_records(ctx, d, det.n_layers)
    losses = []
    tr = window.train(ctx, x, t, steps=300, on_step=lambda i, l: losses.append(l) if i % 50 == 0 else None)
    torch.cuda.synchronize()
    losses = [float(l.item()) for l in losses]
    rms = window.target_rms(t)
    const_loss = float(np.sum(0.5 + np.log(rms)))
    print(f"[window training] loss every 50 steps {np.round(losses, 3)}, constant model {const_loss:.3f}", flush=True)
    assert losses[-1] < const_loss - 0.1
    prob = S.make_build_problem([3000, 6000], det, 1705028791)
    e_plain, c_plain = _build(ctx, prob, det32)
    for nsigma in (5.0, 4.0, 3.0):
        e_l, c_l = _build(ctx, prob, det32, tr.packed, nsigma)
        print(f"[window build] nsigma {nsigma}: eff {e_l['eff']:.4f} vs plain {e_plain['eff']:.4f}; box tests "
              f"{c_l[0]} vs {c_plain[0]}, chi2 {c_l[1]} vs {c_plain[1]}, fallback passes {c_l[5]}", flush=True)
    e_l, c_l = _build(ctx, prob, det32, tr.packed, 4.0)
    assert e_plain["eff"] - e_l["eff"] <= 0.005
    assert c_l[1] < c_plain[1]
