"""Helpers shared by the GPU parity tests: float32 packing of generated inputs,
oracle calls on the same float32-rounded values, and the tolerance checks.

Tolerances: track parameters 1e-4 relative (positions relative to the layer
radius, momentum components relative to |p|), chi2 |d| <= 1e-3 max(chi2, 1),
covariance |dC_ij| <= 1e-3 sqrt(D_i D_j), D = diag(C) with the transverse variance
C_xx + C_yy used for both x and y (positions on a cylinder have a null radial
direction).
"""
from __future__ import annotations

import numpy as np

from paper_1705_02876_amd import synth as S

REL_PARAM = 1e-4
REL_CHI2 = 1e-3
REL_COV = 1e-3


def f32(a):
    return np.asarray(a, dtype=np.float32)


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def soa_state(states):
    """(n,6) -> (6,n) float32."""
    return np.ascontiguousarray(f32(states).T)


def soa_cov(covs):
    """(n,6,6) -> (21,n) float32 packed."""
    return np.ascontiguousarray(f32(S.pack6(np.asarray(covs))).T)


def from_soa_state(t, n=None):
    a = t.detach().cpu().numpy().astype(np.float64)
    return a.T[: (n or a.shape[1])]


def from_soa_cov(t, n=None):
    a = t.detach().cpu().numpy().astype(np.float64).T[: (n or t.shape[1])]
    return S.unpack6(a)


def rounded(a):
    """Float32-rounded values in float64: what the GPU sees, handed to the oracle."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def check_params(gs, os_, name="state", rel=REL_PARAM):
    """gs, os_: (n,6).  Positions relative to |(x,y)| (layer radius), momentum relative to |p|."""
    R = np.maximum(np.hypot(os_[:, 0], os_[:, 1]), 1.0)
    p = np.linalg.norm(os_[:, 3:], axis=1)
    dpos = np.abs(gs[:, :3] - os_[:, :3]) / R[:, None]
    dmom = np.abs(gs[:, 3:] - os_[:, 3:]) / p[:, None]
    worst = max(dpos.max(initial=0), dmom.max(initial=0))
    assert worst <= rel, f"{name}: worst relative error {worst:.3g} (pos {dpos.max(initial=0):.3g}, mom {dmom.max(initial=0):.3g})"
    return worst


def cov_scale(oc):
    """sqrt(D_i D_j) with D = diag(C), except that x and y both use the transverse
    variance C_xx + C_yy: a position on a cylinder has no radial variance, so one
    of C_xx, C_yy vanishes where the radial direction is along an axis."""
    d = np.maximum(np.diagonal(oc, axis1=1, axis2=2), 0.0).copy()
    t = d[:, 0] + d[:, 1]
    d[:, 0] = t
    d[:, 1] = t
    d = np.sqrt(d)
    return d[:, :, None] * d[:, None, :] + 1e-30


def check_cov(gc, oc, name="cov", rel=REL_COV):
    scale = cov_scale(oc)
    err = np.abs(gc - oc) / scale
    worst = err.max(initial=0)
    assert worst <= rel, f"{name}: worst relative covariance error {worst:.3g}"
    return worst


GRAZING_COS = 0.2


def min_cos_psi(fp):
    """Smallest |cos| of the angle between the truth momentum and the layer normal over
    the crossings up to each track's last hit (a conditioning measure: the transported
    covariance grows like 1/cos^2 at grazing crossings)."""
    tp, tm = fp.extra["true_pos"], fp.extra["true_mom"]
    c = np.abs((tp[..., 0] * tm[..., 0] + tp[..., 1] * tm[..., 1]) /
               (np.hypot(tp[..., 0], tp[..., 1]) * np.linalg.norm(tm, axis=2)))
    L = c.shape[0]
    mask = np.arange(L)[:, None] <= fp.last_layer[None, :]
    return np.where(mask & np.isfinite(c), c, np.inf).min(axis=0)


def check_chi2(gc, oc, name="chi2", rel=REL_CHI2):
    err = np.abs(gc - oc) / np.maximum(np.abs(oc), 1.0)
    worst = err.max(initial=0)
    assert worst <= rel, f"{name}: worst chi2 error {worst:.3g}"
    return worst


def fit_inputs_gpu(fp, pad=0):
    """Device tensors of a synth.FitProblem in the kfmi.h layouts (ld = n + pad)."""
    import torch
    n = fp.state0.shape[0]
    ld = n + pad
    st = np.zeros((6, ld), np.float32)
    st[:, :n] = soa_state(fp.state0)
    cv = np.zeros((21, ld), np.float32)
    cv[:, :n] = soa_cov(fp.cov0)
    q = np.zeros(ld, np.int8)
    q[:n] = fp.q.astype(np.int8)
    hidx = np.full((fp.hit_idx.shape[0], ld), -1, np.int32)
    hidx[:, :n] = fp.hit_idx
    return dict(state=to_dev(st), cov=to_dev(cv), q=to_dev(q), hidx=to_dev(hidx),
                hpos=to_dev(np.ascontiguousarray(f32(fp.hit_pos).T)),
                hcov=to_dev(np.ascontiguousarray(f32(fp.hit_cov).T)), n=n, ld=ld)


def oracle_fit_on_f32(orc, det32, fp):
    """Oracle fit on the float32-rounded inputs the GPU sees."""
    g = orc.geometry(det32)
    return orc.fit(g, rounded(fp.state0), rounded(S.unpack6(S.pack6(fp.cov0))), fp.q, fp.hit_idx,
                   rounded(fp.hit_pos), S.unpack3(rounded(fp.hit_cov)))
