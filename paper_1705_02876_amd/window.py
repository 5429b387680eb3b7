"""Learned search window: training data from the fit, training on the GPU,
and the packed network the builder evaluates (a project addition beyond the
paper; the paper's window is the plain chi2 bound).

Every arithmetic step runs in libkfmi (kf_fit with residual records,
kf_mlp_grad, kf_mlp_adam); this module only allocates buffers and sequences
the calls.  The initial parameters are drawn on the host (He-uniform weights,
zero hidden biases) and the output bias starts at the log of the targets'
root mean square over a sample of records, so that training starts from the
constant-width model.
"""
from __future__ import annotations

import numpy as np

from . import kfmi_mlp as M

SIZES = (8, 64, 64, 2)


def initial_params(seed, out_bias=(0.0, 0.0)):
    """Flat float32 parameter vector (W1, b1, W2, b2, W3, b3) on the host."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for i in range(3):
        fi, fo = SIZES[i], SIZES[i + 1]
        lim = np.sqrt(6.0 / fi)
        w = rng.uniform(-lim, lim, (fo, fi))
        if i == 2:
            w *= 0.1  # start close to the constant model
        parts.append(w.ravel())
        parts.append(np.asarray(out_bias, np.float64) if i == 2 else np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def fit_records(ctx, fit_dev, n_layers, fp64=False):
    """Run kf_fit with residual records on device inputs (kfutil-style dict: state, cov, q, hidx, hpos, hcov, n).
    Returns (x (8, M), t (2, M)) device views of the records; rows without a hit hold NaN (skipped in training)."""
    import torch
    n = fit_dev["n"]
    ld = fit_dev["state"].shape[1]
    dev = fit_dev["state"].device
    res = torch.empty(10, n * (n_layers - 1), dtype=torch.float32, device=dev)
    so = torch.empty(6, ld, dtype=torch.float32, device=dev)
    co = torch.empty(21, ld, dtype=torch.float32, device=dev)
    chi2 = torch.empty(ld, dtype=torch.float32, device=dev)
    nh = torch.empty(ld, dtype=torch.int32, device=dev)
    st = torch.empty(ld, dtype=torch.int32, device=dev)
    ctx.kf_fit(fit_dev["state"], fit_dev["cov"], fit_dev["q"], fit_dev["hidx"], fit_dev["hpos"], fit_dev["hcov"],
               so, co, chi2, nh, st, residual_out=res, n=n, fp64=fp64)
    return res[:8], res[8:10]


def target_rms(t, sample=1 << 16):
    """Root mean square of each target over the finite records of a leading sample (host)."""
    h = t[:, :sample].detach().cpu().numpy().astype(np.float64)
    ok = np.isfinite(h).all(axis=0)
    return np.sqrt(np.mean(h[:, ok] ** 2, axis=1))


def train(ctx, x, t, steps=300, lr=1e-2, lr_final=1e-3, seed=1705, on_step=None):
    """Full-batch Adam on the device-resident records; the learning rate decays
    geometrically from lr to lr_final.  Returns the Trainer (params, packed)."""
    import torch
    rms = target_rms(t)
    p0 = torch.from_numpy(initial_params(seed, np.log(np.maximum(rms, 1e-6)))).cuda()
    tr = M.Trainer(ctx, p0, lr=lr)
    decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1))
    for i in range(steps):
        tr.lr = lr * decay ** i
        loss = tr.step(x, t)
        if on_step is not None:
            on_step(i, loss)
    return tr
