"""Thin Python binding of the C ABI in include/kfmi.h (argument marshalling only).

Every function takes torch tensors that live on the GPU and passes their
device pointers and torch's current HIP stream to libkfmi.so.  There is no
fallback: if the library is not built, or a call fails, an exception is
raised.  Layouts are those of kfmi.h: state (6, ld), cov (21, ld),
charge (n,) int8, hits pos (3, ldh) and cov (6, ldh), hit_idx (L, ld_idx).
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkfmi.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "kfmi.h")
MAX_LAYERS = 32

KF_OK = 0
KF_ERR_INVALID_ARG, KF_ERR_GEOMETRY, KF_ERR_DEVICE, KF_ERR_UNSUPPORTED, KF_ERR_WORKSPACE = -1, -2, -3, -4, -5
ST_NO_CROSSING, ST_OUT_OF_Z, ST_NONFINITE, ST_NOT_PD, ST_STOPPED = 1, 2, 4, 8, 16
UPDATE_CHI2_ONLY = 1
FIT_EMIT_RESIDUALS = 1
FIT_FP64 = 2
RES_FEATURES = 8


class KfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kfmi error {code}: {msg}")
        self.code = code


class kf_geometry(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int32),
        ("r", C.c_float * MAX_LAYERS),
        ("z_half", C.c_float * MAX_LAYERS),
        ("x_over_x0", C.c_float * MAX_LAYERS),
        ("bz", C.c_float),
        ("eloss_per_x0", C.c_float),
        ("mass", C.c_float),
    ]


class kf_fit_args(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("ld", C.c_int64),
        ("state_in", C.c_void_p), ("cov_in", C.c_void_p), ("charge", C.c_void_p),
        ("hit_idx", C.c_void_p), ("ld_idx", C.c_int64),
        ("hit_pos", C.c_void_p), ("hit_cov", C.c_void_p), ("ldh", C.c_int64),
        ("state_out", C.c_void_p), ("cov_out", C.c_void_p), ("chi2_out", C.c_void_p),
        ("nhits_out", C.c_void_p), ("status_out", C.c_void_p),
        ("flags", C.c_uint32), ("residual_out", C.c_void_p), ("ld_res", C.c_int64),
        ("stream", C.c_void_p),
    ]


class kf_smooth_args(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("ld", C.c_int64),
        ("state_in", C.c_void_p), ("cov_in", C.c_void_p), ("charge", C.c_void_p),
        ("hit_idx", C.c_void_p), ("ld_idx", C.c_int64),
        ("hit_pos", C.c_void_p), ("hit_cov", C.c_void_p), ("ldh", C.c_int64),
        ("state_out", C.c_void_p), ("cov_out", C.c_void_p), ("chi2_out", C.c_void_p),
        ("nhits_out", C.c_void_p), ("status_out", C.c_void_p),
        ("flags", C.c_uint32), ("stream", C.c_void_p),
    ]


_lib = None


def load_library(path=LIB_PATH):
    """Load libkfmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: the HIP library must be built first (__graft_entry__.build())")
    lib = C.CDLL(path)
    P, I32, I64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    lib.kf_ctx_create.restype = I32
    lib.kf_ctx_create.argtypes = [C.POINTER(P), I32]
    lib.kf_ctx_destroy.restype = None
    lib.kf_ctx_destroy.argtypes = [P]
    lib.kf_last_error.restype = C.c_char_p
    lib.kf_last_error.argtypes = []
    lib.kf_set_geometry.restype = I32
    lib.kf_set_geometry.argtypes = [P, P]
    lib.kf_propagate_to_r.restype = I32
    lib.kf_propagate_to_r.argtypes = [P, I64, I64, P, P, P, P, F, F, I32, P, P]
    lib.kf_update.restype = I32
    lib.kf_update.argtypes = [P, I64, I64, P, P, P, P, I64, P, P, C.c_uint32, P]
    lib.kf_fit.restype = I32
    lib.kf_fit.argtypes = [P, P]
    lib.kf_fit_autotune.restype = I32
    lib.kf_fit_autotune.argtypes = [P, P, I32, C.POINTER(C.c_int32), C.POINTER(C.c_float)]
    lib.kf_smooth.restype = I32
    lib.kf_smooth.argtypes = [P, P]
    _declare_more(lib)
    _lib = lib
    return lib


def _declare_more(lib):
    """Declarations of the building / batching / learned-window calls (see kfmi.h)."""
    from . import kfmi_build, kfmi_mlp
    kfmi_build.declare(lib)
    kfmi_mlp.declare(lib)


def header_symbols(path=HEADER):
    """Names of every function declared in include/kfmi.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(kf_[a-z0-9_]+)\s*\(", txt)))


def _check(rc):
    if rc != KF_OK:
        raise KfError(rc, _lib.kf_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, name):
    import torch
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def geometry_struct(det) -> kf_geometry:
    g = kf_geometry()
    g.n_layers = det.n_layers
    for i, r in enumerate(det.radii):
        g.r[i] = r
        g.z_half[i] = det.z_half
        g.x_over_x0[i] = det.x_over_x0
    g.bz = det.bz
    g.eloss_per_x0 = det.eloss_per_x0
    g.mass = det.mass
    return g


class Context:
    """kf_ctx: device binding plus geometry (host state only)."""

    def __init__(self, device=0):
        lib = load_library()
        h = C.c_void_p()
        _check(lib.kf_ctx_create(C.byref(h), int(device)))
        self.h = h
        self.device = device
        self.n_layers = 0

    def close(self):
        if self.h:
            _lib.kf_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def kf_set_geometry(self, det):
        g = geometry_struct(det) if not isinstance(det, kf_geometry) else det
        _check(_lib.kf_set_geometry(self.h, C.byref(g)))
        self.n_layers = g.n_layers
        self.geom = g

    def kf_propagate_to_r(self, state, cov, charge, status, r_target=None, r_scalar=0.0, z_half=0.0,
                          material_layer=-1, n=None, stream=None):
        import torch
        for t, dt, nm in ((state, torch.float32, "state"), (cov, torch.float32, "cov"), (charge, torch.int8, "charge"),
                          (status, torch.int32, "status"), (r_target, torch.float32, "r_target")):
            _dev(t, dt, nm)
        ld = state.shape[1]
        n = ld if n is None else n
        _check(_lib.kf_propagate_to_r(self.h, n, ld, _ptr(state), _ptr(cov), _ptr(charge), _ptr(r_target),
                                      float(r_scalar), float(z_half), int(material_layer), _ptr(status),
                                      _stream(stream)))

    def kf_update(self, state, cov, hit_pos, hit_cov, chi2, status, chi2_only=False, n=None, stream=None):
        import torch
        for t, dt, nm in ((state, torch.float32, "state"), (cov, torch.float32, "cov"),
                          (hit_pos, torch.float32, "hit_pos"), (hit_cov, torch.float32, "hit_cov"),
                          (chi2, torch.float32, "chi2"), (status, torch.int32, "status")):
            _dev(t, dt, nm)
        ld = state.shape[1]
        n = ld if n is None else n
        _check(_lib.kf_update(self.h, n, ld, _ptr(state), _ptr(cov), _ptr(hit_pos), _ptr(hit_cov), hit_pos.shape[1],
                              _ptr(chi2), _ptr(status), UPDATE_CHI2_ONLY if chi2_only else 0, _stream(stream)))

    def kf_fit(self, state_in, cov_in, charge, hit_idx, hit_pos, hit_cov, state_out, cov_out, chi2_out, nhits_out,
               status_out, residual_out=None, n=None, stream=None, fp64=False):
        a = self._fit_args(state_in, cov_in, charge, hit_idx, hit_pos, hit_cov, state_out, cov_out, chi2_out,
                           nhits_out, status_out, residual_out, n, stream, fp64)
        _check(_lib.kf_fit(self.h, C.byref(a)))

    def kf_fit_autotune(self, state_in, cov_in, charge, hit_idx, hit_pos, hit_cov, state_out, cov_out, chi2_out,
                        nhits_out, status_out, residual_out=None, n=None, stream=None, fp64=False, reps=5):
        """kf_fit_autotune (synchronous): returns (block size, ms per call); later kf_fit calls of this problem
        class launch with that block size."""
        a = self._fit_args(state_in, cov_in, charge, hit_idx, hit_pos, hit_cov, state_out, cov_out, chi2_out,
                           nhits_out, status_out, residual_out, n, stream, fp64)
        block, ms = C.c_int32(0), C.c_float(0.0)
        _check(_lib.kf_fit_autotune(self.h, C.byref(a), int(reps), C.byref(block), C.byref(ms)))
        return block.value, ms.value

    def _fit_args(self, state_in, cov_in, charge, hit_idx, hit_pos, hit_cov, state_out, cov_out, chi2_out, nhits_out,
                  status_out, residual_out, n, stream, fp64):
        import torch
        for t, dt, nm in ((state_in, torch.float32, "state_in"), (cov_in, torch.float32, "cov_in"),
                          (charge, torch.int8, "charge"), (hit_idx, torch.int32, "hit_idx"),
                          (hit_pos, torch.float32, "hit_pos"), (hit_cov, torch.float32, "hit_cov"),
                          (state_out, torch.float32, "state_out"), (cov_out, torch.float32, "cov_out"),
                          (chi2_out, torch.float32, "chi2_out"), (nhits_out, torch.int32, "nhits_out"),
                          (status_out, torch.int32, "status_out"), (residual_out, torch.float32, "residual_out")):
            _dev(t, dt, nm)
        a = kf_fit_args()
        a.ld = state_in.shape[1]
        a.n = a.ld if n is None else n
        a.state_in, a.cov_in, a.charge = _ptr(state_in), _ptr(cov_in), _ptr(charge)
        a.hit_idx, a.ld_idx = _ptr(hit_idx), hit_idx.shape[1]
        a.hit_pos, a.hit_cov, a.ldh = _ptr(hit_pos), _ptr(hit_cov), hit_pos.shape[1]
        a.state_out, a.cov_out, a.chi2_out = _ptr(state_out), _ptr(cov_out), _ptr(chi2_out)
        a.nhits_out, a.status_out = _ptr(nhits_out), _ptr(status_out)
        a.flags = FIT_FP64 if fp64 else 0
        if residual_out is not None:
            a.flags |= FIT_EMIT_RESIDUALS
            a.residual_out = _ptr(residual_out)
            a.ld_res = residual_out.shape[1]
        a.stream = _stream(stream)
        return a

    def kf_smooth(self, state_in, cov_in, charge, hit_idx, hit_pos, hit_cov, state_out, cov_out, status_out,
                  chi2_out=None, nhits_out=None, n=None, stream=None, fp64=False):
        """state_out (n_layers, 6, ld), cov_out (n_layers, 21, ld): smoothed rows per layer."""
        import torch
        for t, dt, nm in ((state_in, torch.float32, "state_in"), (cov_in, torch.float32, "cov_in"),
                          (charge, torch.int8, "charge"), (hit_idx, torch.int32, "hit_idx"),
                          (hit_pos, torch.float32, "hit_pos"), (hit_cov, torch.float32, "hit_cov"),
                          (state_out, torch.float32, "state_out"), (cov_out, torch.float32, "cov_out"),
                          (chi2_out, torch.float32, "chi2_out"), (nhits_out, torch.int32, "nhits_out"),
                          (status_out, torch.int32, "status_out")):
            _dev(t, dt, nm)
        ld = state_in.shape[1]
        L = hit_idx.shape[0]
        if tuple(state_out.shape) != (L, 6, ld) or tuple(cov_out.shape) != (L, 21, ld):
            raise ValueError(f"state_out must be ({L}, 6, {ld}) and cov_out ({L}, 21, {ld})")
        a = kf_smooth_args()
        a.ld = ld
        a.n = ld if n is None else n
        a.state_in, a.cov_in, a.charge = _ptr(state_in), _ptr(cov_in), _ptr(charge)
        a.hit_idx, a.ld_idx = _ptr(hit_idx), hit_idx.shape[1]
        a.hit_pos, a.hit_cov, a.ldh = _ptr(hit_pos), _ptr(hit_cov), hit_pos.shape[1]
        a.state_out, a.cov_out, a.chi2_out = _ptr(state_out), _ptr(cov_out), _ptr(chi2_out)
        a.nhits_out, a.status_out = _ptr(nhits_out), _ptr(status_out)
        a.flags = FIT_FP64 if fp64 else 0
        a.stream = _stream(stream)
        _check(_lib.kf_smooth(self.h, C.byref(a)))
