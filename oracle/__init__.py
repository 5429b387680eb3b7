"""FP64 CPU oracle for Kalman-filter track fitting and building.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
baseline timing are the only code allowed to import this package.  It wraps
`liboracle.so` (plain C, built from kf_oracle.c by `oracle.make_lib`) with numpy
arrays in array-of-structures float64 layout; it shares nothing with the GPU
library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
MAX_LAYERS = 32

NO_CROSSING, OUT_OF_Z, NONFINITE, NOT_PD, STOPPED = 1, 2, 4, 8, 16


class Geometry(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int32),
        ("r", C.c_double * MAX_LAYERS),
        ("z_half", C.c_double * MAX_LAYERS),
        ("x_over_x0", C.c_double * MAX_LAYERS),
        ("bz", C.c_double),
        ("eloss_per_x0", C.c_double),
        ("mass", C.c_double),
    ]


class BuildCfg(C.Structure):
    _fields_ = [
        ("max_cands", C.c_int32),
        ("mode", C.c_int32),
        ("chi2_cut", C.c_double),
        ("n_phi", C.c_int32),
        ("n_eta", C.c_int32),
        ("window_margin", C.c_double),
        ("mlp_params", C.c_void_p),
        ("learned_nsigma", C.c_double),
        ("bin_offsets", C.c_void_p),
        ("perm", C.c_void_p),
        ("layer_vmax", C.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import make_lib as _b
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def _declare(L):
    P = C.c_void_p
    L.or_propagate_one.restype = C.c_int32
    L.or_propagate_one.argtypes = [P, P, P, C.c_int32, C.c_double, C.c_double, P, P]
    L.or_material_one.restype = C.c_int32
    L.or_material_one.argtypes = [P, C.c_int32, P, P]
    L.or_update_one.restype = C.c_int32
    L.or_update_one.argtypes = [P, P, P, P, P, C.c_int32]
    L.or_propagate.restype = C.c_int32
    L.or_propagate.argtypes = [P, C.c_int64, P, P, P, P, C.c_double, C.c_double, C.c_int32, P]
    L.or_update.restype = C.c_int32
    L.or_update.argtypes = [C.c_int64, P, P, P, P, P, P, C.c_int32]
    L.or_fit.restype = C.c_int32
    L.or_fit.argtypes = [P, C.c_int64, P, P, P, P, P, P, P, P, P, P, P]
    L.or_bin_hits.restype = C.c_int32
    L.or_smooth.argtypes = [P, C.c_int64, P, P, P, P, P, P, P, P, P]
    L.or_smooth.restype = C.c_int32
    L.or_surface_pinv.argtypes = [P, C.c_double, C.c_double, P]
    L.or_surface_pinv.restype = C.c_int32
    L.or_rts_step.argtypes = [P] * 10
    L.or_rts_step.restype = None
    L.or_bin_hits.argtypes = [P, C.c_int64, P, P, C.c_int32, C.c_int32, P, P, P]
    L.or_layer_vmax.restype = None
    L.or_layer_vmax.argtypes = [P, C.c_int64, P, P, P]
    L.or_build.restype = C.c_int32
    L.or_build.argtypes = [P, P, C.c_int64, P, P, P, C.c_int64, P, P, P, P, P, C.c_int32] + [P] * 12
    L.or_bf16.restype = C.c_double
    L.or_bf16.argtypes = [C.c_double]
    L.or_mlp_forward.restype = None
    L.or_mlp_forward.argtypes = [P, P, P]
    L.or_window_features.restype = None
    L.or_window_features.argtypes = [P, P, C.c_int, C.c_double, C.c_double, C.c_double, P]


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def geometry(det) -> Geometry:
    """Oracle geometry from a synth.Detector (values used exactly as given)."""
    g = Geometry()
    g.n_layers = det.n_layers
    for i, r in enumerate(det.radii):
        g.r[i] = r
        g.z_half[i] = det.z_half
        g.x_over_x0[i] = det.x_over_x0
    g.bz = det.bz
    g.eloss_per_x0 = det.eloss_per_x0
    g.mass = det.mass
    return g


def full3(packed):
    from paper_1705_02876_amd.synth import unpack3
    return unpack3(np.asarray(packed, dtype=np.float64))


def propagate_one(g, s, Cm, q, R, z_half=0.0, want_jacobian=False):
    s = _f64(s, (6,)).copy()
    Cm = _f64(Cm, (6, 6)).copy()
    J = np.zeros((6, 6))
    t = np.zeros(1)
    st = lib().or_propagate_one(C.byref(g), _p(s), _p(Cm), int(q), float(R), float(z_half), _p(J), _p(t))
    if want_jacobian:
        return st, s, Cm, J, float(t[0])
    return st, s, Cm


def material_one(g, layer, s, Cm):
    s = _f64(s, (6,)).copy()
    Cm = _f64(Cm, (6, 6)).copy()
    st = lib().or_material_one(C.byref(g), int(layer), _p(s), _p(Cm))
    return st, s, Cm


def update_one(s, Cm, m, V, chi2_only=False):
    s = _f64(s, (6,)).copy()
    Cm = _f64(Cm, (6, 6)).copy()
    m = _f64(m, (3,))
    V = _f64(V, (3, 3))
    c2 = np.zeros(1)
    st = lib().or_update_one(_p(s), _p(Cm), _p(m), _p(V), _p(c2), int(chi2_only))
    return st, s, Cm, float(c2[0])


def propagate(g, state, cov, q, r=None, r_scalar=0.0, z_half=0.0, material_layer=-1):
    state = _f64(state).copy()
    n = state.shape[0]
    cov = _f64(cov, (n, 6, 6)).copy()
    q8 = np.ascontiguousarray(q, dtype=np.int8)
    rt = None if r is None else _f64(r)
    status = np.zeros(n, dtype=np.int32)
    rc = lib().or_propagate(C.byref(g), n, _p(state), _p(cov), _p(q8), _p(rt), float(r_scalar), float(z_half),
                            int(material_layer), _p(status))
    assert rc == 0
    return state, cov, status


def update(state, cov, hit_pos, hit_cov_full, chi2_only=False):
    state = _f64(state).copy()
    n = state.shape[0]
    cov = _f64(cov, (n, 6, 6)).copy()
    hp = _f64(hit_pos, (n, 3))
    hc = _f64(hit_cov_full, (n, 3, 3))
    chi2 = np.zeros(n)
    status = np.zeros(n, dtype=np.int32)
    rc = lib().or_update(n, _p(state), _p(cov), _p(hp), _p(hc), _p(chi2), _p(status), int(chi2_only))
    assert rc == 0
    return state, cov, chi2, status


def fit(g, state0, cov0, q, hit_idx_LN, hit_pos, hit_cov_full):
    """hit_idx_LN: (L, n) int32 as in the GPU layout; transposed here."""
    state0 = _f64(state0)
    n = state0.shape[0]
    cov0 = _f64(cov0, (n, 6, 6))
    q8 = np.ascontiguousarray(q, dtype=np.int8)
    hidx = np.ascontiguousarray(np.asarray(hit_idx_LN, dtype=np.int32).T)
    hp = _f64(hit_pos)
    hc = _f64(hit_cov_full)
    so = np.zeros((n, 6))
    co = np.zeros((n, 6, 6))
    chi2 = np.zeros(n)
    nh = np.zeros(n, dtype=np.int32)
    st = np.zeros(n, dtype=np.int32)
    rc = lib().or_fit(C.byref(g), n, _p(state0), _p(cov0), _p(q8), _p(hidx), _p(hp), _p(hc), _p(so), _p(co),
                      _p(chi2), _p(nh), _p(st))
    assert rc == 0
    return so, co, chi2, nh, st


def smooth(g, state0, cov0, q, hit_idx_LN, hit_pos, hit_cov_full):
    """Smoothed state (n, L, 6) and covariance (n, L, 6, 6) at every layer up to
    the last hit layer (NaN after it), and the fit status (n,)."""
    state0 = _f64(state0)
    n = state0.shape[0]
    cov0 = _f64(cov0, (n, 6, 6))
    L = g.n_layers
    q8 = np.ascontiguousarray(q, dtype=np.int8)
    hidx = np.ascontiguousarray(np.asarray(hit_idx_LN, dtype=np.int32).T)
    hp = _f64(hit_pos)
    hc = _f64(hit_cov_full)
    so = np.zeros((n, L, 6))
    co = np.zeros((n, L, 6, 6))
    st = np.zeros(n, dtype=np.int32)
    rc = lib().or_smooth(C.byref(g), n, _p(state0), _p(cov0), _p(q8), _p(hidx), _p(hp), _p(hc), _p(so), _p(co),
                         _p(st))
    assert rc == 0
    return so, co, st


def surface_pinv(Cm, x, y):
    Cm = _f64(Cm, (6, 6))
    out = np.zeros((6, 6))
    ok = lib().or_surface_pinv(_p(Cm), float(x), float(y), _p(out))
    return out if ok else None


def rts_step(xf, Cf, F, xp, Cp, Cp_inv, xs_next, Cs_next):
    a = [_f64(v) for v in (xf, Cf, F, xp, Cp, Cp_inv, xs_next, Cs_next)]
    xs = np.zeros(6)
    Cs = np.zeros((6, 6))
    lib().or_rts_step(*[_p(v) for v in a], _p(xs), _p(Cs))
    return xs, Cs


def bin_hits(g, n_events, layer_offsets, hit_pos, n_phi=64, n_eta=16):
    lo = np.ascontiguousarray(layer_offsets, dtype=np.int64)
    hp = _f64(hit_pos)
    H = int(lo[-1])
    L = g.n_layers
    nb = n_phi * n_eta
    bo = np.zeros(n_events * L * (nb + 1), dtype=np.int32)
    perm = np.zeros(max(H, 1), dtype=np.int64)
    bin_of = np.zeros(max(H, 1), dtype=np.int32)
    rc = lib().or_bin_hits(C.byref(g), n_events, _p(lo), _p(hp), n_phi, n_eta, _p(bo), _p(perm), _p(bin_of))
    assert rc == 0
    return bo.reshape(n_events * L, nb + 1), perm[:H], bin_of[:H]


def layer_vmax(g, n_events, layer_offsets, hit_cov_full):
    """Per (event, layer): largest x-y eigenvalue and largest zz entry of the hit covariances, (E*L, 2)."""
    lo = np.ascontiguousarray(layer_offsets, dtype=np.int64)
    hc = _f64(hit_cov_full)
    out = np.zeros((n_events * g.n_layers, 2))
    lib().or_layer_vmax(C.byref(g), int(n_events), _p(lo), _p(hc), _p(out))
    return out


def build(g, prob, max_cands=6, mode=1, chi2_cut=30.0, n_phi=64, n_eta=16, window_margin=0.01, seeds=None,
          hit_pos=None, hit_cov_full=None, seed_state=None, seed_cov=None, mlp_params=None, learned_nsigma=4.0,
          prebinned=None):
    """Run the oracle builder on a synth.BuildProblem (optionally a subset of seeds).
    mlp_params (4866 float64, or None for the plain window) selects the learned window.
    prebinned: optional (bin_offsets, perm, layer_vmax) from bin_hits and layer_vmax on the same hits and
    grid, so that several calls over one set of events bin it once.

    Returns dict of numpy arrays (see kf_oracle.h)."""
    mp = None if mlp_params is None else _f64(mlp_params)
    if mp is not None and mp.size != 4866:
        raise ValueError("mlp_params must hold 4866 values")
    pb = [None, None, None]
    if prebinned is not None:
        bo, pm, vm = prebinned
        pb = [np.ascontiguousarray(bo, dtype=np.int32), np.ascontiguousarray(pm, dtype=np.int64), _f64(vm)]
        if pb[0].size != prob.n_events * g.n_layers * (n_phi * n_eta + 1) or pb[2].size != 2 * prob.n_events * g.n_layers:
            raise ValueError("prebinned arrays do not fit this problem and grid")
    cfg = BuildCfg(max_cands, mode, chi2_cut, n_phi, n_eta, window_margin, None if mp is None else mp.ctypes.data,
                   learned_nsigma, *[None if a is None else a.ctypes.data for a in pb])
    L = g.n_layers
    E = prob.n_events
    hp = _f64(prob.hit_pos if hit_pos is None else hit_pos)
    hc = _f64(full3(prob.hit_cov) if hit_cov_full is None else hit_cov_full)
    seed_event = np.repeat(np.arange(E, dtype=np.int64), np.diff(prob.seed_offsets))
    sel = np.arange(prob.seed_state.shape[0]) if seeds is None else np.asarray(seeds)
    S = sel.size
    ss = _f64((prob.seed_state if seed_state is None else seed_state)[sel])
    sc = _f64((prob.seed_cov if seed_cov is None else seed_cov)[sel], (S, 6, 6))
    sq = np.ascontiguousarray(prob.seed_q[sel], dtype=np.int8)
    sh = np.ascontiguousarray(prob.seed_hits[sel], dtype=np.int64)
    se = np.ascontiguousarray(seed_event[sel])
    N = max_cands
    out = dict(
        n_cands=np.zeros(S, dtype=np.int32), cand_hits=np.zeros((S, N, L), dtype=np.int32),
        cand_chi2=np.zeros((S, N)), cand_nhits=np.zeros((S, N), dtype=np.int32),
        cand_status=np.zeros((S, N), dtype=np.int32), best_state=np.zeros((S, 6)), best_cov=np.zeros((S, 6, 6)),
        margin_cut=np.zeros(S), margin_rank=np.zeros(S), hits_examined=np.zeros(S, dtype=np.int64),
        margin_window=np.zeros(S), fallbacks=np.zeros(S, dtype=np.int64))
    rc = lib().or_build(C.byref(g), C.byref(cfg), E, _p(np.ascontiguousarray(prob.layer_hit_offsets, np.int64)),
                        _p(hp), _p(hc), S, _p(se), _p(ss), _p(sc), _p(sq), _p(sh), prob.first_layer,
                        _p(out["n_cands"]), _p(out["cand_hits"]), _p(out["cand_chi2"]), _p(out["cand_nhits"]),
                        _p(out["cand_status"]), _p(out["best_state"]), _p(out["best_cov"]), _p(out["margin_cut"]),
                        _p(out["margin_rank"]), _p(out["hits_examined"]), _p(out["margin_window"]),
                        _p(out["fallbacks"]))
    assert rc == 0
    return out


def bf16(x):
    return lib().or_bf16(float(x))


def mlp_forward(params, X):
    """Network outputs (n, 2) for features X (n, 8), device arithmetic semantics (see kf_oracle.h)."""
    P = _f64(params)
    X = _f64(X)
    out = np.zeros((X.shape[0], 2))
    o = np.zeros(2)
    for i in range(X.shape[0]):
        xi = np.ascontiguousarray(X[i])
        lib().or_mlp_forward(_p(P), _p(xi), _p(o))
        out[i] = o
    return out


def window_features(state, cov, q, r_from, r_to, zh):
    """Features (8,) of one prediction (state (6,), cov (6,6))."""
    f = np.zeros(8)
    lib().or_window_features(_p(_f64(state)), _p(_f64(cov)), int(q), float(r_from), float(r_to), float(zh), _p(f))
    return f
