"""Seeded synthetic event generator (simulation side only).

This module produces the inputs that both the GPU library and the FP64 oracle
consume: charged-particle tracks in a uniform solenoidal field crossing equally
spaced, fixed-length concentric cylinders, with Gaussian hit smearing, optional
multiple scattering and mean energy loss, random missing hits, uniform noise
hits, and one seed per simulated track carrying its hits on the first three
layers.

Sec. 3.2 describes the workload this stands in for: a detector of equally
spaced concentric cylinders of fixed length, an in-house simulation that
smears hit positions with Gaussians, and one seed per simulated track made
from its first three hits.  Nothing here runs the Kalman filter: the truth
trajectory is stepped with the exact circle/circle intersection of the
track's transverse circle with each layer.  A seed carries its three hits;
its covariance is that of the helix through the vertex and those hits
(finite-difference error propagation of the hit errors), and its state is
drawn around the truth at the third hit from that covariance
(`seed_mode="truth"`, the default), or is the state of a three-hit circle
and helix fit itself (`seed_mode="hits"`, see `seeds_from_hits`).

All arithmetic is float64; callers cast to float32 for the GPU and pass the
float32-rounded values back to the oracle so both sides see identical inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 0.299792458e-2  # GeV / (T cm): pT = C_LIGHT * |B| * radius
M_PION = 0.13957039  # GeV
BASE_SEED = 1705028760


@dataclass(frozen=True)
class Detector:
    """Barrel of concentric cylinders with a uniform field B = (0, 0, bz)."""

    radii: tuple
    z_half: float = 50.0
    x_over_x0: float = 0.0  # thickness per layer at normal incidence
    bz: float = 3.8
    sigma_rphi: float = 0.01
    sigma_z: float = 0.1
    eloss_per_x0: float = 0.0363  # GeV per radiation length (Si, minimum ionising)
    mass: float = M_PION

    @property
    def n_layers(self) -> int:
        return len(self.radii)

    def as_float32(self) -> "Detector":
        """Same detector with every real parameter rounded to float32."""
        f = lambda v: float(np.float32(v))
        return Detector(tuple(f(r) for r in self.radii), f(self.z_half), f(self.x_over_x0), f(self.bz),
                        f(self.sigma_rphi), f(self.sigma_z), f(self.eloss_per_x0), f(self.mass))


def detector_small() -> Detector:
    """10 layers r = 4..40 cm, |z| < 50 cm, 3.8 T, no material."""
    return Detector(radii=tuple(4.0 * (k + 1) for k in range(10)), x_over_x0=0.0)


def detector_full() -> Detector:
    """17 layers r = 4 + 6k cm, |z| < 50 cm, 0.02 X0 per layer."""
    return Detector(radii=tuple(4.0 + 6.0 * k for k in range(17)), x_over_x0=0.02)


# ----------------------------------------------------------------------------
# truth stepping (simulation)
# ----------------------------------------------------------------------------

def _cross(pos, mom, q, R, bz):
    """Exact first crossing of each track's helix with the cylinder of radius R.

    Works on arrays (n,3).  Returns (pos', mom', ok).  Uses the intersection of
    the track's transverse circle with the circle |x| = R, then the turning
    angle around the circle centre; z advances linearly in transverse path.
    """
    n = pos.shape[0]
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    px, py, pz = mom[:, 0], mom[:, 1], mom[:, 2]
    pt = np.hypot(px, py)
    ux, uy = px / pt, py / pt
    a = -q * C_LIGHT * bz
    kappa = a / pt
    newpos = np.full_like(pos, np.nan)
    newmom = np.full_like(mom, np.nan)
    ok = np.zeros(n, dtype=bool)
    r0sq = x * x + y * y

    line = kappa == 0.0
    if np.any(line):
        idx = np.nonzero(line)[0]
        b = x[idx] * ux[idx] + y[idx] * uy[idx]
        disc = b * b + (R * R - r0sq[idx])
        good = disc >= 0
        t = -b + np.sqrt(np.where(good, disc, 0.0))
        good &= t > 0
        gi = idx[good]
        tg = t[good]
        newpos[gi, 0] = x[gi] + ux[gi] * tg
        newpos[gi, 1] = y[gi] + uy[gi] * tg
        newpos[gi, 2] = z[gi] + pz[gi] / pt[gi] * tg
        newmom[gi] = mom[gi]
        ok[gi] = True

    idx = np.nonzero(~line)[0]
    if idx.size:
        k = kappa[idx]
        xi, yi = x[idx], y[idx]
        uxi, uyi = ux[idx], uy[idx]
        # left normal n = (-uy, ux); circle centre c = P0 + n / kappa
        cx = xi - uyi / k
        cy = yi + uxi / k
        rho = 1.0 / np.abs(k)
        d = np.hypot(cx, cy)
        # d^2 - rho^2 = r0^2 + 2 (P0 . n) / kappa, written without cancellation
        an = -xi * uyi + yi * uxi
        d2mr2 = r0sq[idx] + 2.0 * an / k
        xa = (R * R + d2mr2) / (2.0 * d)  # distance of the chord midpoint from the origin along c
        h2 = R * R - xa * xa
        good = h2 >= 0
        h = np.sqrt(np.where(good, h2, 0.0))
        chx, chy = cx / d, cy / d
        best_phi = np.full(idx.size, np.inf)
        v0x, v0y = xi - cx, yi - cy
        for sgn in (1.0, -1.0):
            qx = xa * chx - sgn * h * chy
            qy = xa * chy + sgn * h * chx
            v1x, v1y = qx - cx, qy - cy
            ang = np.arctan2(v0x * v1y - v0y * v1x, v0x * v1x + v0y * v1y)  # (-pi, pi]
            turn = np.where(k > 0, ang, -ang)  # turning in the sense of motion
            turn = np.where(turn <= 1e-300, turn + 2.0 * np.pi, turn)
            best_phi = np.where(good & (turn < best_phi), turn, best_phi)
        good &= np.isfinite(best_phi)
        phi = np.where(good, best_phi * np.sign(k), 0.0)  # signed rotation angle kappa * t
        t = phi / k
        sn, cs = np.sin(phi), np.cos(phi)
        omc = 2.0 * np.sin(0.5 * phi) ** 2
        S = sn / k
        Cc = omc / k
        gi = idx[good]
        sel = good
        newpos[gi, 0] = xi[sel] + S[sel] * uxi[sel] - Cc[sel] * uyi[sel]
        newpos[gi, 1] = yi[sel] + S[sel] * uyi[sel] + Cc[sel] * uxi[sel]
        newpos[gi, 2] = z[gi] + pz[gi] / pt[gi] * t[sel]
        newmom[gi, 0] = px[gi] * cs[sel] - py[gi] * sn[sel]
        newmom[gi, 1] = py[gi] * cs[sel] + px[gi] * sn[sel]
        newmom[gi, 2] = pz[gi]
        ok[gi] = True
    return newpos, newmom, ok


def _scatter(rng, pos, mom, det: Detector, alive):
    """Mean energy loss plus two Gaussian deflections perpendicular to p.

    Thin-scatterer model: thickness x/X0 along the path is the layer's normal
    thickness over |cos| of the angle to the layer normal; the angular width is
    the Highland formula (PDG review of passage of particles through matter)
    evaluated with the incoming momentum.  Returns (mom', alive').
    """
    if det.x_over_x0 <= 0:
        return mom, alive
    p = np.linalg.norm(mom, axis=1)
    u = mom / p[:, None]
    r = np.hypot(pos[:, 0], pos[:, 1])
    cospsi = np.abs(u[:, 0] * pos[:, 0] / r + u[:, 1] * pos[:, 1] / r)
    t = det.x_over_x0 / cospsi
    E = np.sqrt(p * p + det.mass ** 2)
    beta = p / E
    theta0 = 0.0136 / (beta * p) * np.sqrt(t) * (1.0 + 0.038 * np.log(t / (beta * beta)))
    E2 = E - det.eloss_per_x0 * t
    alive2 = alive & (E2 > det.mass)
    p2 = np.sqrt(np.maximum(E2 * E2 - det.mass ** 2, 1e-300))
    # orthonormal pair perpendicular to u: e1 = z x u / |z x u|, e2 = u x e1
    e1 = np.stack([-u[:, 1], u[:, 0], np.zeros_like(p)], axis=1)
    e1 /= np.linalg.norm(e1, axis=1)[:, None]
    e2 = np.cross(u, e1)
    g = rng.standard_normal((p.size, 2))
    un = u + (theta0 * g[:, 0])[:, None] * e1 + (theta0 * g[:, 1])[:, None] * e2
    un /= np.linalg.norm(un, axis=1)[:, None]
    newmom = np.where(alive2[:, None], un * p2[:, None], mom)
    return newmom, alive2


def _truth_kinematics(rng, n, pt_range=(0.5, 10.0), eta_range=(-1.0, 1.0)):
    pt = rng.uniform(pt_range[0], pt_range[1], n)
    eta = rng.uniform(eta_range[0], eta_range[1], n)
    phi = rng.uniform(-np.pi, np.pi, n)
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    mom = np.stack([pt * np.cos(phi), pt * np.sin(phi), pt * np.sinh(eta)], axis=1)
    return mom, q


def simulate(rng, n, det: Detector, p_miss=0.0, force_first=0, pt_range=(0.5, 10.0), eta_range=(-1.0, 1.0),
             smear=True):
    """Simulate n tracks from the origin.

    Returns dict with
      q (n,), mom0 (n,3) truth momentum at the vertex,
      true_pos (L,n,3), true_mom (L,n,3) truth at each crossing (NaN if not reached),
      hit_pos (L,n,3) measured hit (NaN if absent), has_hit (L,n) bool,
      reached (L,n) bool.
    Layers below `force_first` never lose their hit to the missing-hit draw.
    """
    L = det.n_layers
    mom0, q = _truth_kinematics(rng, n, pt_range, eta_range)
    pos = np.zeros((n, 3))
    mom = mom0.copy()
    alive = np.ones(n, dtype=bool)
    true_pos = np.full((L, n, 3), np.nan)
    true_mom = np.full((L, n, 3), np.nan)
    hit_pos = np.full((L, n, 3), np.nan)
    has_hit = np.zeros((L, n), dtype=bool)
    reached = np.zeros((L, n), dtype=bool)
    for l, R in enumerate(det.radii):
        npos, nmom, ok = _cross(pos, mom, q, R, det.bz)
        ok &= alive
        ok &= np.abs(np.where(ok, npos[:, 2], 0.0)) <= det.z_half
        alive = ok
        pos = np.where(ok[:, None], npos, pos)
        mom = np.where(ok[:, None], nmom, mom)
        reached[l] = ok
        true_pos[l][ok] = pos[ok]
        true_mom[l][ok] = mom[ok]
        # Gaussian smearing: r-phi as an angle (hit stays on the cylinder), z linear
        phi_t = np.arctan2(pos[:, 1], pos[:, 0])
        if smear:
            dphi = rng.standard_normal(n) * det.sigma_rphi / R
            dz = rng.standard_normal(n) * det.sigma_z
        else:
            dphi = np.zeros(n)
            dz = np.zeros(n)
        ph = phi_t + dphi
        hp = np.stack([R * np.cos(ph), R * np.sin(ph), pos[:, 2] + dz], axis=1)
        present = ok.copy()
        if p_miss > 0 and l >= force_first:
            present &= rng.random(n) >= p_miss
        has_hit[l] = present
        hit_pos[l][present] = hp[present]
        if not smear:
            hit_pos[l][present] = pos[present]
        mom, alive = _scatter(rng, pos, mom, det, alive)
    return dict(q=q, mom0=mom0, true_pos=true_pos, true_mom=true_mom, hit_pos=hit_pos, has_hit=has_hit,
                reached=reached)


def hit_cov_packed(det: Detector, n):
    """Packed lower-triangle hit covariance (xx, yx, yy, zx, zy, zz), isotropic in x-y."""
    c = np.zeros((n, 6))
    c[:, 0] = det.sigma_rphi ** 2
    c[:, 2] = det.sigma_rphi ** 2
    c[:, 5] = det.sigma_z ** 2
    return c


# ----------------------------------------------------------------------------
# packing helpers
# ----------------------------------------------------------------------------

TRI6 = [(i, j) for i in range(6) for j in range(i + 1)]  # packed index k = i(i+1)/2 + j


def pack6(C):
    """(n,6,6) -> (n,21) lower triangle, k = i(i+1)/2 + j."""
    return np.stack([C[:, i, j] for (i, j) in TRI6], axis=1)


def unpack6(P):
    n = P.shape[0]
    C = np.zeros((n, 6, 6), dtype=P.dtype)
    for k, (i, j) in enumerate(TRI6):
        C[:, i, j] = P[:, k]
        C[:, j, i] = P[:, k]
    return C


def pack3(C):
    return np.stack([C[:, 0, 0], C[:, 1, 0], C[:, 1, 1], C[:, 2, 0], C[:, 2, 1], C[:, 2, 2]], axis=1)


def unpack3(P):
    n = P.shape[0]
    C = np.zeros((n, 3, 3), dtype=P.dtype)
    idx = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
    for k, (i, j) in enumerate(idx):
        C[:, i, j] = P[:, k]
        C[:, j, i] = P[:, k]
    return C


# ----------------------------------------------------------------------------
# fit workloads
# ----------------------------------------------------------------------------

def fit_prior_sigmas(mom0):
    """Diagonal prior sigmas at the vertex: 0.01 cm (x, y), 0.1 cm (z), 2% of pT per momentum component."""
    pt = np.hypot(mom0[:, 0], mom0[:, 1])
    n = mom0.shape[0]
    s = np.empty((n, 6))
    s[:, 0] = 0.01
    s[:, 1] = 0.01
    s[:, 2] = 0.1
    s[:, 3:] = 0.02 * pt[:, None]
    return s


@dataclass
class FitProblem:
    det: Detector
    q: np.ndarray  # (n,) +-1
    state0: np.ndarray  # (n,6) prior mean at the vertex
    cov0: np.ndarray  # (n,6,6) prior covariance
    hit_idx: np.ndarray  # (L,n) int32, -1 = no hit
    hit_pos: np.ndarray  # (H,3)
    hit_cov: np.ndarray  # (H,6) packed
    truth_state0: np.ndarray  # (n,6) truth at the vertex
    truth_last: np.ndarray  # (n,6) truth at the last hit layer (after the crossing, before scattering)
    last_layer: np.ndarray  # (n,)
    extra: dict = field(default_factory=dict)


FIT_CHUNK = 131072


def _fit_chunk(seed, chunk_id, n, det, p_miss, min_hits, smear, prior_at_truth, prior_sigma_scale):
    """One chunk of fit tracks with its own random stream (seed, chunk_id)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(chunk_id)])))
    need = n
    parts = []
    while need > 0:
        m = int(need * 1.02) + 16
        s = simulate(rng, m, det, p_miss=p_miss, smear=smear)
        nh = s["has_hit"].sum(axis=0)
        good = np.nonzero(nh >= max(min_hits, 1))[0][:need]
        parts.append((s["q"][good], s["mom0"][good], s["hit_pos"][:, good], s["has_hit"][:, good],
                      s["true_pos"][:, good], s["true_mom"][:, good]))
        need -= good.size
    q, mom0, hp, has, tp, tm = [np.concatenate([p_[k] for p_ in parts], axis=0 if k < 2 else 1) for k in range(6)]
    sig = fit_prior_sigmas(mom0) * prior_sigma_scale
    truth0 = np.concatenate([np.zeros((n, 3)), mom0], axis=1)
    state0 = truth0.copy() if prior_at_truth else truth0 + rng.standard_normal((n, 6)) * sig
    return q, mom0, hp, has, tp, tm, sig, state0


def make_fit_problem(n, det: Detector, seed, p_miss=0.0, min_hits=0, smear=True, prior_at_truth=False,
                     prior_sigma_scale=1.0, workers=None):
    """Tracks for the fit: hits at the crossed layers, prior = truth + N(0, C0) at the vertex.

    Tracks with fewer than `min_hits` hits are re-drawn until every track qualifies.
    Hits are stored layer-major, in track order within each layer (coalesced gathers).
    Generation runs in chunks of FIT_CHUNK tracks with independent random streams
    derived from (seed, chunk index), on a thread pool; the result depends only on
    (n, seed), not on the number of workers.
    """
    import os
    from concurrent.futures import ThreadPoolExecutor
    L = det.n_layers
    sizes = [min(FIT_CHUNK, n - k) for k in range(0, n, FIT_CHUNK)] or [0]
    args = [(seed, i, sz, det, p_miss, min_hits, smear, prior_at_truth, prior_sigma_scale)
            for i, sz in enumerate(sizes)]
    nw = workers or min(8, os.cpu_count() or 1, len(args))
    if nw > 1:
        with ThreadPoolExecutor(nw) as ex:
            chunks = list(ex.map(lambda a: _fit_chunk(*a), args))
    else:
        chunks = [_fit_chunk(*a) for a in args]
    q = np.concatenate([c[0] for c in chunks])
    mom0 = np.concatenate([c[1] for c in chunks])
    hp = np.concatenate([c[2] for c in chunks], axis=1)
    has = np.concatenate([c[3] for c in chunks], axis=1)
    tp = np.concatenate([c[4] for c in chunks], axis=1)
    tm = np.concatenate([c[5] for c in chunks], axis=1)
    sig = np.concatenate([c[6] for c in chunks])
    state0 = np.concatenate([c[7] for c in chunks])
    hit_idx = np.full((L, n), -1, dtype=np.int32)
    counts = has.sum(axis=1)
    offs = np.concatenate([[0], np.cumsum(counts)])
    H = int(offs[-1])
    hit_pos = np.empty((H, 3))
    for l in range(L):
        idx = np.nonzero(has[l])[0]
        hit_idx[l, idx] = offs[l] + np.arange(idx.size, dtype=np.int32)
        hit_pos[offs[l]:offs[l + 1]] = hp[l, idx]
    hit_cov = hit_cov_packed(det, H)
    truth0 = np.concatenate([np.zeros((n, 3)), mom0], axis=1)
    cov0 = np.zeros((n, 6, 6))
    for i in range(6):
        cov0[:, i, i] = sig[:, i] ** 2
    last = np.where(has.any(axis=0), L - 1 - np.argmax(has[::-1], axis=0), -1)
    ar = np.arange(n)
    truth_last = np.concatenate([tp[last, ar], tm[last, ar]], axis=1)
    return FitProblem(det, q, state0, cov0, hit_idx, hit_pos, hit_cov, truth0, truth_last, last,
                      extra=dict(true_pos=tp, true_mom=tm, has_hit=has))


# ----------------------------------------------------------------------------
# seeds from three hits (vertex-constrained helix, no Kalman filter)
# ----------------------------------------------------------------------------

def _helix3(P0, P1, P2, bz):
    """State (x,y,z,px,py,pz) at P2 and charge of the helix through the vertex and three hits.

    The vertex sits at the origin (no spread), so the transverse circle passes
    through it: in conformal coordinates (u, v) = (x, y) / (x^2 + y^2) such
    circles are the lines 2 a u + 2 b v = 1 (centre (a, b)), fitted to the three
    hits by least squares.  Longitudinal: z = cot(theta) s through the vertex,
    least squares against the transverse arc length s from the vertex.  The
    direction at P2 is the circle's tangent at the hit's angle around the centre.
    """
    pts = [P0, P1, P2]
    us, vs = [], []
    for P in pts:
        r2 = P[:, 0] ** 2 + P[:, 1] ** 2
        us.append(P[:, 0] / r2)
        vs.append(P[:, 1] / r2)
    Suu = sum(u * u for u in us)
    Suv = sum(u * v for u, v in zip(us, vs))
    Svv = sum(v * v for v in vs)
    Su = sum(us)
    Sv = sum(vs)
    det = Suu * Svv - Suv * Suv
    # normal equations of min sum (2a u + 2b v - 1)^2
    a = 0.5 * (Su * Svv - Sv * Suv) / det
    b = 0.5 * (Sv * Suu - Su * Suv) / det
    rho = np.hypot(a, b)
    # direction at the vertex is perpendicular to the centre, pointing to the hits
    u0x, u0y = -b / rho, a / rho
    flip = (u0x * P1[:, 0] + u0y * P1[:, 1]) < 0
    u0x = np.where(flip, -u0x, u0x)
    u0y = np.where(flip, -u0y, u0y)
    # centre = n0 / kappa with n0 = (-u0y, u0x)  =>  sign(kappa) = sign(n0 . c)
    sgn = np.sign(-u0y * a + u0x * b)
    kappa = sgn / rho
    pt = C_LIGHT * abs(bz) * rho
    q = -sgn * np.sign(bz)
    # arc length from the vertex to each hit along the circle
    ang0 = np.arctan2(-b, -a)  # angle of the vertex seen from the centre
    def arclen(P):
        ang = np.arctan2(P[:, 1] - b, P[:, 0] - a)
        return np.mod((ang - ang0) * sgn, 2.0 * np.pi) * rho
    ss = [arclen(P) for P in pts]
    zs = [P[:, 2] for P in pts]
    cot = sum(s_ * z_ for s_, z_ in zip(ss, zs)) / sum(s_ * s_ for s_ in ss)
    # state at P2: position = the hit (x, y), z on the fitted line, tangent direction
    cx, cy = P2[:, 0], P2[:, 1]
    ang2 = np.arctan2(cy - b, cx - a)
    nx = -sgn * np.cos(ang2)  # n = -kappa (P - c) / |kappa (P - c)| on the circle
    ny = -sgn * np.sin(ang2)
    dirx, diry = ny, -nx
    st = np.stack([cx, cy, cot * ss[2], pt * dirx, pt * diry, pt * cot], axis=1)
    return st, q


def seeds_from_hits(hits3, det: Detector, ms_layers=2):
    """Seed state at the third hit and its covariance.

    hits3: (3, n, 3) hit positions on layers 0..2.  The covariance propagates
    the hit errors (sigma_rphi as an angle on each cylinder, sigma_z) through
    the three-point helix by central finite differences, plus the angular
    variance of `ms_layers` thin scatterers on the momentum direction.
    """
    n = hits3.shape[1]
    st, q = _helix3(hits3[0], hits3[1], hits3[2], det.bz)
    C = np.zeros((n, 6, 6))
    for k in range(3):
        R = det.radii[k]
        phik = np.arctan2(hits3[k][:, 1], hits3[k][:, 0])
        for comp, sig in (("phi", det.sigma_rphi / R), ("z", det.sigma_z)):
            h = 1e-3 * sig
            out = []
            for sg in (1.0, -1.0):
                hh = [hits3[0].copy(), hits3[1].copy(), hits3[2].copy()]
                if comp == "phi":
                    ph = phik + sg * h
                    hh[k][:, 0] = R * np.cos(ph)
                    hh[k][:, 1] = R * np.sin(ph)
                else:
                    hh[k][:, 2] = hits3[k][:, 2] + sg * h
                out.append(_helix3(hh[0], hh[1], hh[2], det.bz)[0])
            g = (out[0] - out[1]) / (2.0 * h)
            C += (sig * sig) * g[:, :, None] * g[:, None, :]
    if det.x_over_x0 > 0 and ms_layers > 0:
        p = np.linalg.norm(st[:, 3:], axis=1)
        u = st[:, 3:] / p[:, None]
        E = np.sqrt(p * p + det.mass ** 2)
        beta = p / E
        t = det.x_over_x0
        th = 0.0136 / (beta * p) * math.sqrt(t) * (1.0 + 0.038 * np.log(t / (beta * beta)))
        P = np.eye(3)[None] - u[:, :, None] * u[:, None, :]
        C[:, 3:, 3:] += ms_layers * (p * th)[:, None, None] ** 2 * P
    C = 0.5 * (C + np.transpose(C, (0, 2, 1)))
    return st, C, q


SEED_MAX_REL_MOMENTUM_SIGMA = 0.15


def truth_seeds(rng, sim, det: Detector, draw=True):
    """Seeds at the third hit: covariance from the three-hit fit (seeds_from_hits) with the
    momentum block's eigenvalues capped at (0.15 p)^2, mean = truth at the third layer plus a
    draw from that covariance, charge = truth.

    Realistic seeding is outside the method (the paper reports none); a Gaussian in
    Cartesian momentum cannot describe a curvature that is consistent with zero, so the
    three-hit estimate alone gives meaningless priors for stiff tracks.
    """
    h3 = sim["hit_pos"][0:3]
    _, C, _ = seeds_from_hits(h3, det)
    truth = np.concatenate([sim["true_pos"][2], sim["true_mom"][2]], axis=1)
    p = np.linalg.norm(truth[:, 3:], axis=1)
    w, V = np.linalg.eigh(C[:, 3:, 3:])
    cap = (SEED_MAX_REL_MOMENTUM_SIGMA * p) ** 2
    wc = np.minimum(w, cap[:, None])
    scale = np.sqrt(np.where(w > 0, wc / np.where(w > 0, w, 1.0), 1.0))  # shrink factor per eigen-direction
    # C' = S C S^T with S = I on positions and V diag(scale) V^T on momenta keeps the
    # cross-correlations consistent with the shrunk momentum block
    Sm = np.einsum("nij,nj,nkj->nik", V, scale, V)
    Sfull = np.zeros_like(C)
    Sfull[:, :3, :3] = np.eye(3)
    Sfull[:, 3:, 3:] = Sm
    Cc = Sfull @ C @ np.transpose(Sfull, (0, 2, 1))
    Cc = 0.5 * (Cc + np.transpose(Cc, (0, 2, 1)))
    if not draw:
        return truth.copy(), Cc, sim["q"].copy()
    w2, V2 = np.linalg.eigh(Cc)
    g = rng.standard_normal((truth.shape[0], 6)) * np.sqrt(np.maximum(w2, 0.0))
    st = truth + np.einsum("nij,nj->ni", V2, g)
    return st, Cc, sim["q"].copy()


# ----------------------------------------------------------------------------
# build workloads (events with noise hits, seeds)
# ----------------------------------------------------------------------------

@dataclass
class BuildProblem:
    det: Detector
    n_events: int
    layer_hit_offsets: np.ndarray  # (E*L+1,) int64, hits of (event e, layer l) in [o[e*L+l], o[e*L+l+1])
    hit_pos: np.ndarray  # (H,3)
    hit_cov: np.ndarray  # (H,6) packed
    hit_track: np.ndarray  # (H,) sim track index within the event, -1 = noise
    seed_offsets: np.ndarray  # (E+1,) int64
    seed_state: np.ndarray  # (S,6)
    seed_cov: np.ndarray  # (S,6,6)
    seed_q: np.ndarray  # (S,)
    seed_hits: np.ndarray  # (S,3) global hit indices on layers 0..2
    seed_track: np.ndarray  # (S,) sim track index within its event
    track_nhits: list  # per event: (n_tracks,) number of hits of each sim track
    first_layer: int = 3


def make_build_problem(track_counts, det: Detector, seed, p_miss=0.05, noise_frac=0.2, smear=True,
                       pt_range=(0.5, 10.0), eta_range=(-1.0, 1.0), seed_draw=True, seed_mode="truth"):
    """Events of sim tracks plus `noise_frac * n_tracks` uniform noise hits per layer.

    The first three layers always carry the track's hit; one seed per track.
    Hits inside each (event, layer) are randomly permuted (read-out order is
    unrelated to the track order).  seed_mode "truth": the seed state is drawn
    around the truth at the third hit (truth_seeds); "hits": it is the helix
    through the vertex and the three smeared hits, with that fit's covariance
    (seeds_from_hits), the charge from the turning sense.
    """
    if seed_mode not in ("truth", "hits"):
        raise ValueError(f"unknown seed_mode {seed_mode!r}")
    rng = np.random.Generator(np.random.PCG64(seed))
    L = det.n_layers
    E = len(track_counts)
    offs = [0]
    pos_chunks, trk_chunks = [], []
    seed_state, seed_cov, seed_q, seed_hits, seed_track = [], [], [], [], []
    seed_offsets = [0]
    track_nhits = []
    for e, nt in enumerate(track_counts):
        nt = int(nt)
        sim = simulate(rng, nt, det, p_miss=p_miss, force_first=3, smear=smear, pt_range=pt_range,
                       eta_range=eta_range)
        has = sim["has_hit"]
        track_nhits.append(has.sum(axis=0).astype(np.int32))
        local_index = np.full((L, nt), -1, dtype=np.int64)
        nnoise = int(round(noise_frac * nt))
        for l in range(L):
            R = det.radii[l]
            tidx = np.nonzero(has[l])[0]
            hp = sim["hit_pos"][l, tidx]
            phi = rng.uniform(-np.pi, np.pi, nnoise)
            zz = rng.uniform(-det.z_half, det.z_half, nnoise)
            npos = np.stack([R * np.cos(phi), R * np.sin(phi), zz], axis=1)
            allpos = np.concatenate([hp, npos], axis=0)
            alltrk = np.concatenate([tidx, np.full(nnoise, -1)]).astype(np.int32)
            perm = rng.permutation(allpos.shape[0])
            allpos = allpos[perm]
            alltrk = alltrk[perm]
            inv = np.empty_like(perm)
            inv[perm] = np.arange(perm.size)
            base = offs[-1]
            local_index[l, tidx] = base + inv[: tidx.size]
            pos_chunks.append(allpos)
            trk_chunks.append(alltrk)
            offs.append(base + allpos.shape[0])
        # seeds: one per track, covariance from its layer 0..2 hits, mean drawn around the truth
        if seed_mode == "truth":
            st, C, q = truth_seeds(rng, sim, det, draw=seed_draw)
        else:
            st, C, q = seeds_from_hits(sim["hit_pos"][0:3], det)
        seed_state.append(st)
        seed_cov.append(C)
        seed_q.append(q)
        seed_hits.append(local_index[0:3].T.copy())
        seed_track.append(np.arange(nt, dtype=np.int32))
        seed_offsets.append(seed_offsets[-1] + nt)
    hit_pos = np.concatenate(pos_chunks, axis=0)
    return BuildProblem(
        det=det, n_events=E, layer_hit_offsets=np.asarray(offs, dtype=np.int64), hit_pos=hit_pos,
        hit_cov=hit_cov_packed(det, hit_pos.shape[0]), hit_track=np.concatenate(trk_chunks),
        seed_offsets=np.asarray(seed_offsets, dtype=np.int64), seed_state=np.concatenate(seed_state),
        seed_cov=np.concatenate(seed_cov), seed_q=np.concatenate(seed_q),
        seed_hits=np.concatenate(seed_hits).astype(np.int64), seed_track=np.concatenate(seed_track),
        track_nhits=track_nhits)


def uniform_event_sizes(seed, n_events, lo=5000, hi=20000):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, n_events)


def loguniform_event_sizes(seed, n_events, lo=1000, hi=50000):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), n_events))).astype(np.int64)


def round_f32(x):
    """Round a float64 array to float32 and back (the values both sides see)."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def window_records(seed, n):
    """Synthetic training records for the search-window network: 8 features in the
    ranges a fit prediction produces (q/pT, cot theta, z/z_half, sin of the crossing
    angle, r_from/100, r_to/100, log sigma_t, log sigma_z of the prediction) and two
    Gaussian offsets whose widths grow with the prediction's sigmas and with
    |q/pT| (multiple scattering).  Returns x (n, 8), t (n, 2) float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    qpt = rng.choice([-1.0, 1.0], n) / rng.uniform(0.5, 10.0, n)
    cot = np.sinh(rng.uniform(-1.0, 1.0, n))
    r_from = rng.integers(0, 16, n) * 0.06 + 0.04
    r_to = r_from + 0.06
    z = np.clip(cot * r_to * 100.0 / 50.0, -1.0, 1.0)
    sin_cross = np.clip(0.5 * 0.0114 * r_to * 100.0 * qpt, -1.0, 1.0)
    lst = rng.uniform(-5.5, -2.0, n)
    lsz = rng.uniform(-4.0, -1.5, n)
    x = np.stack([qpt, cot, z, sin_cross, r_from, r_to, lst, lsz], axis=1)
    st = np.sqrt(np.exp(2 * lst) + 0.01 ** 2 + (0.004 * np.abs(qpt)) ** 2)
    sz = np.sqrt(np.exp(2 * lsz) + 0.1 ** 2 / 12 + (0.004 * np.abs(qpt) * np.sqrt(1 + cot ** 2)) ** 2)
    t = np.stack([st * rng.standard_normal(n), sz * rng.standard_normal(n)], axis=1)
    return x, t
