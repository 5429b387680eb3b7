"""Pins of the oracle's smoother (Rauch-Tung-Striebel backward pass after the fit).

What fixes the smoother independently of its own code:
  * the pseudo-inverse on the surface is numpy's Moore-Penrose pseudo-inverse;
  * one backward step, chained over a linear Gaussian model, gives the exact
    posterior of the batch least-squares problem over all states at once;
  * without process noise the smoothed trajectory is one deterministic
    trajectory: every layer's smoothed state and covariance is the last
    layer's carried back (reversed momentum and charge, then the energy loss
    undone), exactly when the hits lie on the track;
  * with material the smoothed estimate scatters around the truth with the
    width its covariance claims, the covariance never exceeds the filtered
    one, and the last layer equals the fit.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_1705_02876_amd import synth as S

REV = np.diag([1.0, 1.0, 1.0, -1.0, -1.0, -1.0])


def surface_basis(x):
    """5x6 orthonormal rows (tangent, z, px, py, pz) orthogonal to the radial direction of x."""
    r = np.hypot(x[0], x[1])
    P = np.zeros((5, 6))
    P[0, 0], P[0, 1] = -x[1] / r, x[0] / r
    for k in range(1, 5):
        P[k, k + 1] = 1.0
    return P


def surface_errors(x_ref, C_ref, x, C):
    """Largest state and covariance differences in units of C_ref's surface standard deviations."""
    P = surface_basis(x_ref)
    sg = np.sqrt(np.diag(P @ C_ref @ P.T))
    es = np.abs(P @ (x - x_ref) / sg).max()
    ec = np.abs(P @ (C - C_ref) @ P.T / np.outer(sg, sg)).max()
    return es, ec


def smooth_problem(det, n, seed, **kw):
    fp = S.make_fit_problem(n, det, seed, **kw)
    g = O.geometry(det)
    hc = O.full3(fp.hit_cov)
    so, co, st = O.smooth(g, fp.state0, fp.cov0, fp.q, fp.hit_idx, fp.hit_pos, hc)
    return fp, g, hc, so, co, st


def test_surface_pinv_is_moore_penrose():
    rng = np.random.default_rng(5)
    for _ in range(50):
        phi = rng.uniform(-np.pi, np.pi)
        x = np.array([7.0 * np.cos(phi), 7.0 * np.sin(phi), 1.0, 0.3, -0.2, 0.4])
        P = surface_basis(x)
        A = rng.standard_normal((5, 5))
        M = A @ A.T + 0.1 * np.eye(5)
        D = np.diag(10.0 ** rng.uniform(-1.5, 0.5, 5))
        C = P.T @ D @ M @ D @ P
        got = O.surface_pinv(C, x[0], x[1])
        ref = np.linalg.pinv(C, rcond=1e-13, hermitian=True)
        assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()
        # the four Moore-Penrose conditions
        assert np.allclose(C @ got @ C, C, rtol=0, atol=1e-10 * np.abs(C).max())
        assert np.allclose(got @ C @ got, got, rtol=0, atol=1e-8 * np.abs(got).max())
    # not positive definite on the surface
    C = P.T @ np.diag([1.0, 1.0, -1.0, 1.0, 1.0]) @ P
    assert O.surface_pinv(C, x[0], x[1]) is None


def test_rts_step_gives_the_batch_posterior():
    """Linear Gaussian chain x_{k+1} = F_k x_k + w_k, y_k = H x_k + v_k."""
    rng = np.random.default_rng(11)
    K, n = 7, 6
    H = np.hstack([np.eye(3), np.zeros((3, 3))])

    def spd(d, s):
        A = rng.standard_normal((d, d))
        return s * (A @ A.T + 0.5 * np.eye(d))

    m0, P0 = rng.standard_normal(n), spd(n, 2.0)
    F = [np.eye(n) + 0.3 * rng.standard_normal((n, n)) for _ in range(K - 1)]
    Q = [spd(n, 0.05) for _ in range(K - 1)]
    V = [spd(3, 0.1) for _ in range(K)]
    y = [rng.standard_normal(3) for _ in range(K)]
    # forward Kalman filter (scaffolding that produces the smoother's inputs)
    xf, Cf, xp, Cp = [], [], [m0], [P0]
    for k in range(K):
        if k:
            xp.append(F[k - 1] @ xf[-1])
            Cp.append(F[k - 1] @ Cf[-1] @ F[k - 1].T + Q[k - 1])
        Kg = Cp[k] @ H.T @ np.linalg.inv(H @ Cp[k] @ H.T + V[k])
        xf.append(xp[k] + Kg @ (y[k] - H @ xp[k]))
        Cf.append((np.eye(n) - Kg @ H) @ Cp[k])
    xs, Cs = [None] * K, [None] * K
    xs[-1], Cs[-1] = xf[-1], Cf[-1]
    for k in range(K - 2, -1, -1):
        xs[k], Cs[k] = O.rts_step(xf[k], Cf[k], F[k], xp[k + 1], Cp[k + 1], np.linalg.inv(Cp[k + 1]), xs[k + 1],
                                  Cs[k + 1])
    # batch posterior: information matrix over all K states
    Lam = np.zeros((K * n, K * n))
    eta = np.zeros(K * n)
    blk = lambda k: slice(k * n, (k + 1) * n)
    P0i = np.linalg.inv(P0)
    Lam[blk(0), blk(0)] += P0i
    eta[blk(0)] += P0i @ m0
    for k in range(K):
        Vi = np.linalg.inv(V[k])
        Lam[blk(k), blk(k)] += H.T @ Vi @ H
        eta[blk(k)] += H.T @ Vi @ y[k]
    for k in range(K - 1):
        Qi = np.linalg.inv(Q[k])
        Lam[blk(k), blk(k)] += F[k].T @ Qi @ F[k]
        Lam[blk(k), blk(k + 1)] -= F[k].T @ Qi
        Lam[blk(k + 1), blk(k)] -= Qi @ F[k]
        Lam[blk(k + 1), blk(k + 1)] += Qi
    Sig = np.linalg.inv(Lam)
    mu = Sig @ eta
    for k in range(K):
        assert np.allclose(xs[k], mu[blk(k)], rtol=0, atol=1e-9 * (1 + np.abs(mu).max()))
        assert np.allclose(Cs[k], Sig[blk(k), blk(k)], rtol=0, atol=1e-9 * np.abs(Sig).max())


def test_smoother_without_material_is_the_last_state_carried_back():
    """Hits on the track and a prior at the truth: every residual vanishes, and
    without process noise the smoothed covariance at each layer is the last
    layer's transported inward."""
    det = S.detector_small()
    fp, g, hc, so, co, st = smooth_problem(det, 150, 21, smear=False, min_hits=10, prior_at_truth=True)
    assert (st == 0).all()
    worst = 0.0
    for i in range(fp.q.size):
        last = fp.last_layer[i]
        for l in range(last):
            stt, x, C = O.propagate_one(g, REV @ so[i, last], REV @ co[i, last] @ REV, -fp.q[i], det.radii[l])
            assert stt == 0
            worst = max(worst, *surface_errors(so[i, l], co[i, l], REV @ x, REV @ C @ REV))
    assert worst < 1e-7, worst


def test_smoother_with_measurement_noise_stays_near_the_carried_back_state():
    """Noisy hits: the extended smoother linearises about the filtered states,
    so the carried-back state differs from it only at second order."""
    det = S.detector_small()
    fp, g, hc, so, co, st = smooth_problem(det, 120, 23, smear=True, min_hits=10, prior_at_truth=True)
    errs = []
    for i in range(fp.q.size):
        last = fp.last_layer[i]
        for l in range(last):
            stt, x, C = O.propagate_one(g, REV @ so[i, last], REV @ co[i, last] @ REV, -fp.q[i], det.radii[l])
            errs.append(surface_errors(so[i, l], co[i, l], REV @ x, REV @ C @ REV))
    errs = np.array(errs)
    assert np.median(errs[:, 0]) < 0.05 and np.median(errs[:, 1]) < 0.05, np.median(errs, axis=0)
    assert errs.max() < 1.0


def test_smoother_undoes_deterministic_energy_loss():
    """Material that takes energy but hardly scatters (x/X0 = 1e-8 at 1e6 GeV
    per X0: 0.01 GeV a layer, theta0 below 1e-6): the smoothed trajectory is
    the last state carried back with the energy loss undone (a negative loss
    per X0 is the exact inverse of the forward step)."""
    det = dataclasses.replace(S.detector_small(), x_over_x0=1e-8, eloss_per_x0=1e6)
    gn = O.geometry(dataclasses.replace(det, eloss_per_x0=-1e6))
    fp, g, hc, so, co, st = smooth_problem(det, 120, 13, smear=False, min_hits=10, prior_at_truth=True)
    assert (st == 0).all()
    errs, fs = [], []
    for i in range(fp.q.size):
        last = fp.last_layer[i]
        x, C = so[i, last], co[i, last]
        for l in range(last - 1, -1, -1):
            stt, x, C = O.propagate_one(g, REV @ x, REV @ C @ REV, -fp.q[i], det.radii[l])
            assert stt == 0
            x, C = REV @ x, REV @ C @ REV
            p = np.linalg.norm(x[3:])
            stt, x, C = O.material_one(gn, l, x, C)
            assert stt == 0
            fs.append(p / np.linalg.norm(x[3:]))
            errs.append(surface_errors(so[i, l], co[i, l], x, C))
    errs = np.array(errs)
    assert min(fs) < 0.98  # the loss is large enough to matter
    assert np.median(errs) < 1e-4 and errs.max() < 1e-2, (np.median(errs, axis=0), errs.max(axis=0))


def test_smoother_pulls_covariance_bound_and_last_layer():
    det = S.detector_full()
    n = 2000
    fp, g, hc, so, co, st = smooth_problem(det, n, 7, smear=True, min_hits=8)
    assert (st == 0).mean() > 0.99
    ok = st == 0
    L = det.n_layers
    tp, tm = fp.extra["true_pos"], fp.extra["true_mom"]
    # the last layer has seen every hit: the smoothed state is the fit's
    fs, fc, _, _, fst = O.fit(g, fp.state0, fp.cov0, fp.q, fp.hit_idx, fp.hit_pos, hc)
    ar = np.arange(n)
    assert np.array_equal(so[ar[ok], fp.last_layer[ok]], fs[ok])
    assert np.array_equal(co[ar[ok], fp.last_layer[ok]], fc[ok])
    assert np.array_equal(st, fst)
    # rows after the last hit layer are NaN
    after = np.arange(L)[None, :] > fp.last_layer[:, None]
    assert np.isnan(so[after]).all() and np.isnan(co[after]).all()
    assert np.isfinite(so[~after & ok[:, None]]).all()
    # pulls against the truth in (tangent, z, px, py, pz)
    for l in (0, 4, 9):
        pulls = []
        for i in np.nonzero(ok & (fp.last_layer > l) & fp.extra["has_hit"][l])[0]:
            P = surface_basis(so[i, l])
            t = np.concatenate([tp[l, i], tm[l, i]])
            pulls.append(P @ (so[i, l] - t) / np.sqrt(np.diag(P @ co[i, l] @ P.T)))
        w = np.std(np.array(pulls), axis=0)
        assert (np.abs(w - 1.0) < 0.08).all(), (l, w)
    # smoothed covariance <= filtered covariance (filtered at l = fit over the hits up to l)
    for l in (0, 5):
        hidx = fp.hit_idx.copy()
        hidx[l + 1:] = -1
        sel = ok & fp.extra["has_hit"][l] & (fp.last_layer > l)
        ff, fcl, _, _, fst2 = O.fit(g, fp.state0[sel], fp.cov0[sel], fp.q[sel], hidx[:, sel], fp.hit_pos, hc)
        assert (fst2 == 0).all()
        shrink = []
        for k, i in enumerate(np.nonzero(sel)[0]):
            P = surface_basis(ff[k])
            Df = P @ fcl[k] @ P.T
            D = Df - P @ co[i, l] @ P.T
            sc = np.sqrt(np.diag(Df))
            ev = np.linalg.eigvalsh(D / np.outer(sc, sc))
            assert ev.min() > -1e-9, (l, i, ev)
            shrink.append(np.trace(P @ co[i, l] @ P.T / np.outer(sc, sc)) / 5.0)
        assert np.median(shrink) < 0.9


def test_smoother_failed_track_keeps_filtered_rows():
    """A track that stops in the material is not smoothed: the rows of the
    layers its filter completed are the filtered states and the fit's output is
    the last of them."""
    fp = S.make_fit_problem(400, S.detector_full(), 31, smear=True, min_hits=6)
    # fitted with far more energy loss than the tracks were simulated with
    g = O.geometry(dataclasses.replace(S.detector_full(), eloss_per_x0=6.0))
    hc = O.full3(fp.hit_cov)
    so, co, st = O.smooth(g, fp.state0, fp.cov0, fp.q, fp.hit_idx, fp.hit_pos, hc)
    fs, fc, _, _, fst = O.fit(g, fp.state0, fp.cov0, fp.q, fp.hit_idx, fp.hit_pos, hc)
    assert np.array_equal(st, fst)
    stopped = np.nonzero(st == O.STOPPED)[0]
    assert stopped.size >= 5
    for i in stopped:
        done = int(np.isfinite(so[i, :, 0]).sum())
        assert np.isfinite(so[i, :done]).all() and np.isnan(so[i, done:]).all()
        assert np.array_equal(so[i, done - 1], fs[i]) and np.array_equal(co[i, done - 1], fc[i])
    # the others are smoothed as usual: their last row is the fit
    good = np.nonzero(st == 0)[0]
    assert good.size > 100
    ar = fp.last_layer[good]
    assert np.array_equal(so[good, ar], fs[good])
