"""Binding of the hit-binning and building calls of include/kfmi.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C

BINNED_FLOATS = 12
BUILD_TILED, BUILD_PERSISTENT, BUILD_SERIAL = 0, 1, 2
WINDOW_PLAIN, WINDOW_LEARNED = 0, 1
PREC_F32, PREC_F64 = 0, 1
BUILD_COUNTERS = 6  # box tests, chi2 evaluations, compatible hits, candidate-layer steps, updates, fallbacks


class kf_bin_args(C.Structure):
    _fields_ = [
        ("n_events", C.c_int64), ("layer_offsets", C.c_void_p), ("hit_pos", C.c_void_p), ("hit_cov", C.c_void_p),
        ("ldh", C.c_int64), ("n_phi", C.c_int32), ("n_eta", C.c_int32), ("bin_offsets", C.c_void_p),
        ("perm", C.c_void_p), ("binned", C.c_void_p), ("layer_vmax", C.c_void_p), ("workspace", C.c_void_p),
        ("workspace_bytes", C.c_size_t), ("stream", C.c_void_p),
    ]


class kf_build_cfg(C.Structure):
    _fields_ = [
        ("max_cands", C.c_int32), ("chi2_cut", C.c_float), ("n_phi", C.c_int32), ("n_eta", C.c_int32),
        ("window_margin", C.c_float), ("mode", C.c_int32), ("window_mode", C.c_int32),
        ("waves_per_block", C.c_int32), ("blocks_per_cu", C.c_int32), ("precision", C.c_int32),
        ("learned_nsigma", C.c_float), ("seed_order", C.c_int32),
    ]


class kf_build_args(C.Structure):
    _fields_ = [
        ("n_events", C.c_int64), ("n_seeds", C.c_int64), ("ld_seed", C.c_int64), ("first_layer", C.c_int32),
        ("seed_offsets", C.c_void_p), ("seed_state", C.c_void_p), ("seed_cov", C.c_void_p),
        ("seed_charge", C.c_void_p), ("seed_hits", C.c_void_p), ("layer_offsets", C.c_void_p),
        ("bin_offsets", C.c_void_p), ("binned", C.c_void_p), ("layer_vmax", C.c_void_p),
        ("n_cands", C.c_void_p), ("cand_hits", C.c_void_p), ("cand_chi2", C.c_void_p),
        ("cand_nhits", C.c_void_p), ("cand_status", C.c_void_p), ("best_state", C.c_void_p),
        ("best_cov", C.c_void_p), ("counters", C.c_void_p), ("workspace", C.c_void_p),
        ("workspace_bytes", C.c_size_t), ("stream", C.c_void_p), ("mlp_packed", C.c_void_p),
    ]


def declare(lib):
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    lib.kf_bin_hits_workspace_size.restype = C.c_size_t
    lib.kf_bin_hits_workspace_size.argtypes = [I64, I64]
    lib.kf_bin_hits.restype = I32
    lib.kf_bin_hits.argtypes = [P, P]
    lib.kf_build_workspace_size.restype = C.c_size_t
    lib.kf_build_workspace_size.argtypes = [P, I64, I64]
    lib.kf_build.restype = I32
    lib.kf_build.argtypes = [P, P, P]
    lib.kf_build_noalloc.restype = I32
    lib.kf_build_noalloc.argtypes = [P, P, P]
    lib.kf_build_host_workspace_size.restype = C.c_size_t
    lib.kf_build_host_workspace_size.argtypes = [P, P, P]
    lib.kf_build_host.restype = I32
    lib.kf_build_host.argtypes = [P, P, P]
    lib.kf_graph_begin.restype = I32
    lib.kf_graph_begin.argtypes = [P, P]
    lib.kf_graph_end.restype = I32
    lib.kf_graph_end.argtypes = [P, P, C.POINTER(P)]
    lib.kf_graph_launch.restype = I32
    lib.kf_graph_launch.argtypes = [P, P]
    lib.kf_graph_destroy.restype = None
    lib.kf_graph_destroy.argtypes = [P]
    lib.kf_build_autotune.restype = I32
    lib.kf_build_autotune.argtypes = [P, P, P, I32, C.POINTER(C.c_float)]
    lib.kf_autotune_save.restype = I32
    lib.kf_autotune_save.argtypes = [P, C.c_char_p]
    lib.kf_autotune_load.restype = I32
    lib.kf_autotune_load.argtypes = [P, C.c_char_p]
    return lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# The build's rank key and back-pointer records carry a hit's index within its (event, layer) in 24 bits, with
# 2^24 - 1 reserved for "no hit": an (event, layer) may hold at most 2^24 - 2 hits.
MAX_LAYER_HITS = (1 << 24) - 2


def check_offsets(t, count, limit, name, max_run=None):
    """Host check of a device offset array: `count` + 1 ascending int64 values in [0, limit], and consecutive
    differences at most `max_run` when given."""
    import torch
    if t.dtype != torch.int64 or t.numel() < count + 1:
        raise ValueError(f"{name}: need {count + 1} int64 offsets")
    h = t[: count + 1].cpu()
    if int(h[0]) < 0 or int(h[-1]) > limit or bool((h[1:] < h[:-1]).any()):
        raise ValueError(f"{name}: offsets must ascend within [0, {limit}]")
    if max_run is not None and count > 0 and int((h[1:] - h[:-1]).max()) > max_run:
        raise ValueError(f"{name}: a range holds more than {max_run} entries")


def bin_hits(ctx, layer_offsets, hit_pos, hit_cov, n_events, n_phi=64, n_eta=16, out=None, workspace=None,
             stream=None, check=True):
    """kf_bin_hits.  Returns dict(bin_offsets, perm, binned, layer_vmax) of device tensors."""
    import torch
    from . import kfmi
    lib = kfmi.load_library()
    ldh = hit_pos.shape[1]
    L = ctx.n_layers
    dev = hit_pos.device
    if check:
        check_offsets(layer_offsets, n_events * L, ldh, "layer_offsets", max_run=MAX_LAYER_HITS)
    if out is None:
        out = dict(bin_offsets=torch.empty(n_events * L, n_phi * n_eta + 1, dtype=torch.int32, device=dev),
                   perm=torch.empty(max(ldh, 1), dtype=torch.int32, device=dev),
                   binned=torch.empty(max(ldh, 1), BINNED_FLOATS, dtype=torch.float32, device=dev),
                   layer_vmax=torch.empty(n_events * L, 2, dtype=torch.float32, device=dev))
    wsb = lib.kf_bin_hits_workspace_size(ldh, n_events)
    if workspace is None:
        workspace = torch.empty(max(wsb, 4), dtype=torch.uint8, device=dev)
    a = kf_bin_args()
    a.n_events = n_events
    a.layer_offsets = _ptr(layer_offsets)
    a.hit_pos, a.hit_cov, a.ldh = _ptr(hit_pos), _ptr(hit_cov), ldh
    a.n_phi, a.n_eta = n_phi, n_eta
    a.bin_offsets, a.perm, a.binned, a.layer_vmax = (_ptr(out["bin_offsets"]), _ptr(out["perm"]),
                                                       _ptr(out["binned"]), _ptr(out["layer_vmax"]))
    a.workspace, a.workspace_bytes = _ptr(workspace), workspace.numel()
    a.stream = kfmi._stream(stream)
    kfmi._check(lib.kf_bin_hits(ctx.h, C.byref(a)))
    return out


def make_cfg(max_cands=6, chi2_cut=30.0, n_phi=64, n_eta=16, window_margin=0.01, mode=BUILD_TILED,
             window_mode=WINDOW_PLAIN, waves_per_block=0, blocks_per_cu=0, precision=PREC_F64, learned_nsigma=4.0,
             seed_order=1):
    return kf_build_cfg(max_cands, chi2_cut, n_phi, n_eta, window_margin, mode, window_mode, waves_per_block,
                        blocks_per_cu, precision, learned_nsigma, seed_order)


def workspace_bytes(cfg, n_events, n_seeds, serial=False):
    """kf_build_workspace_size for a configuration; the largest over the grouped launch modes (tiled,
    persistent) when the autotuner may switch between them, and over the serial-candidate mode too when
    `serial` or when cfg asks for it (its candidate buffers take about 240 bytes per candidate slot)."""
    from . import kfmi
    lib = kfmi.load_library()
    best = 0
    modes = (BUILD_TILED, BUILD_PERSISTENT) + ((BUILD_SERIAL,) if serial or cfg.mode == BUILD_SERIAL else ())
    for mode in modes:
        c = kf_build_cfg.from_buffer_copy(cfg)
        c.mode = mode
        best = max(best, int(lib.kf_build_workspace_size(C.byref(c), int(n_events), int(n_seeds))))
    return best


def build(ctx, cfg, seeds, bins, layer_offsets, n_events, first_layer=3, out=None, counters=None, workspace=None,
          stream=None, mlp_packed=None, check=True, noalloc=False):
    """kf_build (kf_build_noalloc with noalloc=True: no workspace, the library's static scratch instead).
    seeds: dict(offsets int64 (E+1), state (6,ld), cov (21,ld), charge int8 (S), hits int32 (3,ld), n).

    Returns dict of device tensors (n_cands, cand_hits (L,S,N), cand_chi2 (S,N), cand_nhits, cand_status,
    best_state, best_cov)."""
    import torch
    from . import kfmi
    lib = kfmi.load_library()
    S = seeds["n"]
    ld = seeds["state"].shape[1]
    N = cfg.max_cands
    L = ctx.n_layers
    dev = seeds["state"].device
    nb = cfg.n_phi * cfg.n_eta
    if bins["bin_offsets"].dim() != 2 or bins["bin_offsets"].shape[1] != nb + 1 or \
            bins["bin_offsets"].shape[0] < n_events * L:
        raise ValueError(f"bins were made for another grid or problem: bin_offsets {tuple(bins['bin_offsets'].shape)}, "
                         f"config {cfg.n_phi}x{cfg.n_eta} with {n_events * L} (event, layer) pairs")
    if S > 0 and check:  # host copies of the offsets: not allowed while a graph is being captured
        check_offsets(seeds["offsets"], n_events, S, "seed_offsets")
        if int(seeds["offsets"][n_events].item()) != S or int(seeds["offsets"][0].item()) != 0:
            raise ValueError("seed_offsets must start at 0 and end at n_seeds")
        check_offsets(layer_offsets, n_events * L, bins["binned"].shape[0], "layer_offsets",
                      max_run=MAX_LAYER_HITS)
    if out is None:
        out = dict(n_cands=torch.empty(max(S, 1), dtype=torch.int32, device=dev),
                   cand_hits=torch.empty(L, max(S, 1), N, dtype=torch.int32, device=dev),
                   cand_chi2=torch.empty(max(S, 1), N, dtype=torch.float32, device=dev),
                   cand_nhits=torch.empty(max(S, 1), N, dtype=torch.int32, device=dev),
                   cand_status=torch.empty(max(S, 1), N, dtype=torch.int32, device=dev),
                   best_state=torch.empty(6, ld, dtype=torch.float32, device=dev),
                   best_cov=torch.empty(21, ld, dtype=torch.float32, device=dev))
    wsb = 0 if noalloc else workspace_bytes(cfg, n_events, S)
    if noalloc and workspace is not None:
        raise ValueError("kf_build_noalloc takes no workspace")
    if workspace is None and wsb > 0:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
    if workspace is not None and workspace.numel() < wsb:
        raise ValueError(f"workspace of {workspace.numel()} bytes, {wsb} needed (kfmi_build.workspace_bytes)")
    a = kf_build_args()
    a.n_events, a.n_seeds, a.ld_seed, a.first_layer = n_events, S, ld, first_layer
    a.seed_offsets, a.seed_state, a.seed_cov = _ptr(seeds["offsets"]), _ptr(seeds["state"]), _ptr(seeds["cov"])
    a.seed_charge, a.seed_hits = _ptr(seeds["charge"]), _ptr(seeds["hits"])
    a.layer_offsets = _ptr(layer_offsets)
    a.bin_offsets, a.binned, a.layer_vmax = _ptr(bins["bin_offsets"]), _ptr(bins["binned"]), _ptr(bins["layer_vmax"])
    a.n_cands, a.cand_hits, a.cand_chi2 = _ptr(out["n_cands"]), _ptr(out["cand_hits"]), _ptr(out["cand_chi2"])
    a.cand_nhits, a.cand_status = _ptr(out["cand_nhits"]), _ptr(out["cand_status"])
    a.best_state, a.best_cov = _ptr(out.get("best_state")), _ptr(out.get("best_cov"))
    if counters is not None and (counters.dtype != torch.int64 or counters.numel() < BUILD_COUNTERS):
        raise ValueError(f"counters must hold {BUILD_COUNTERS} int64")
    a.counters = _ptr(counters)
    if cfg.window_mode == WINDOW_LEARNED:
        if mlp_packed is None or mlp_packed.dtype != torch.uint8 or mlp_packed.numel() < 23048:
            raise ValueError("the learned window needs the packed network (uint8, 23048 bytes)")
        a.mlp_packed = _ptr(mlp_packed)
    if workspace is not None:
        a.workspace, a.workspace_bytes = _ptr(workspace), workspace.numel()
    a.stream = kfmi._stream(stream)
    # kept for kf_build_autotune, with every tensor the pointers refer to
    out["_args"] = a
    out["_keep"] = (seeds, bins, layer_offsets, workspace, mlp_packed, counters)
    kfmi._check((lib.kf_build_noalloc if noalloc else lib.kf_build)(ctx.h, C.byref(cfg), C.byref(a)))
    return out


def autotune(ctx, cfg, out, reps=3):
    """kf_build_autotune on the arguments of a previous build() call (its `out`): updates cfg in place and
    returns the best average time in ms."""
    from . import kfmi
    ms = C.c_float(0.0)
    kfmi._check(kfmi.load_library().kf_build_autotune(ctx.h, C.byref(cfg), C.byref(out["_args"]), int(reps),
                                                      C.byref(ms)))
    return ms.value


def autotune_save(ctx, path):
    from . import kfmi
    kfmi._check(kfmi.load_library().kf_autotune_save(ctx.h, str(path).encode()))


def autotune_load(ctx, path):
    from . import kfmi
    kfmi._check(kfmi.load_library().kf_autotune_load(ctx.h, str(path).encode()))


class Graph:
    """A HIP graph of library calls: capture(fn) records every kf_* call fn issues on a side stream;
    launch() replays them."""

    def __init__(self, ctx):
        import torch
        self.ctx = ctx
        self.stream = torch.cuda.Stream()  # default priority
        self.h = None

    def capture(self, fn):
        import torch
        from . import kfmi
        lib = kfmi.load_library()
        torch.cuda.synchronize()
        kfmi._check(lib.kf_graph_begin(self.ctx.h, C.c_void_p(self.stream.cuda_stream)))
        err = None
        try:
            with torch.cuda.stream(self.stream):
                fn()
        except Exception as e:  # the capture must be ended in any case
            err = e
        h = C.c_void_p()
        rc = lib.kf_graph_end(self.ctx.h, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if err is not None:
            if h.value:
                lib.kf_graph_destroy(h)
            raise err
        kfmi._check(rc)
        self.h = h
        return self

    def launch(self, stream=None):
        from . import kfmi
        kfmi._check(kfmi.load_library().kf_graph_launch(self.h, kfmi._stream(stream)))

    def close(self):
        if self.h:
            from . import kfmi
            kfmi.load_library().kf_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def upload_problem(prob, dtype_note=None):
    """Device tensors of a synth.BuildProblem in the kfmi.h layouts (float32)."""
    import numpy as np
    import torch
    from . import synth as S
    dev = "cuda"
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).to(dev)
    seeds = dict(
        offsets=torch.from_numpy(np.asarray(prob.seed_offsets, np.int64)).to(dev),
        state=f32(prob.seed_state.T), cov=f32(S.pack6(prob.seed_cov).T),
        charge=torch.from_numpy(prob.seed_q.astype(np.int8)).to(dev),
        hits=torch.from_numpy(np.ascontiguousarray(prob.seed_hits.T.astype(np.int32))).to(dev),
        n=prob.seed_state.shape[0])
    hits = dict(layer_offsets=torch.from_numpy(np.asarray(prob.layer_hit_offsets, np.int64)).to(dev),
                pos=f32(prob.hit_pos.T), cov=f32(prob.hit_cov.T))
    return seeds, hits


class kf_build_host_args(C.Structure):
    _fields_ = [
        ("n_events", C.c_int64), ("n_seeds", C.c_int64), ("n_hits", C.c_int64), ("first_layer", C.c_int32),
        ("n_chunks", C.c_int32), ("n_slots", C.c_int32),
        ("layer_offsets", C.c_void_p), ("hit_pos", C.c_void_p), ("hit_cov", C.c_void_p),
        ("seed_offsets", C.c_void_p), ("seed_state", C.c_void_p), ("seed_cov", C.c_void_p),
        ("seed_charge", C.c_void_p), ("seed_hits", C.c_void_p),
        ("n_cands", C.c_void_p), ("cand_hits", C.c_void_p), ("cand_chi2", C.c_void_p),
        ("cand_nhits", C.c_void_p), ("cand_status", C.c_void_p), ("best_state", C.c_void_p),
        ("best_cov", C.c_void_p), ("counters", C.c_void_p), ("mlp_packed", C.c_void_p),
        ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t), ("stream", C.c_void_p),
    ]


def host_problem(prob, pin=True):
    """Host (page-locked when pin) tensors of a synth.BuildProblem in the kfmi.h layouts, for build_host."""
    import numpy as np
    import torch
    from . import synth as S
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=dt)))
    d = dict(layer_offsets=t(prob.layer_hit_offsets, np.int64), pos=t(prob.hit_pos.T, np.float32),
             cov=t(prob.hit_cov.T, np.float32), seed_offsets=t(prob.seed_offsets, np.int64),
             state=t(prob.seed_state.T, np.float32), scov=t(S.pack6(prob.seed_cov).T, np.float32),
             charge=t(prob.seed_q, np.int8), hits=t(prob.seed_hits.T, np.int32))
    if pin:
        d = {k: v.pin_memory() for k, v in d.items()}
    d["n_events"], d["n_seeds"], d["n_hits"] = prob.n_events, prob.seed_state.shape[0], prob.hit_pos.shape[0]
    return d


def _host_args(ctx, cfg, hp, out, n_chunks, n_slots, first_layer, counters, mlp_packed, workspace, stream):
    import torch
    from . import kfmi
    for k in ("layer_offsets", "pos", "cov", "seed_offsets", "state", "scov", "charge", "hits"):
        if hp[k].is_cuda or not hp[k].is_contiguous():
            raise ValueError(f"{k} must be a contiguous host tensor")
    a = kf_build_host_args()
    a.n_events, a.n_seeds, a.n_hits = hp["n_events"], hp["n_seeds"], hp["n_hits"]
    a.first_layer, a.n_chunks, a.n_slots = first_layer, n_chunks, n_slots
    a.layer_offsets, a.hit_pos, a.hit_cov = _ptr(hp["layer_offsets"]), _ptr(hp["pos"]), _ptr(hp["cov"])
    a.seed_offsets, a.seed_state, a.seed_cov = _ptr(hp["seed_offsets"]), _ptr(hp["state"]), _ptr(hp["scov"])
    a.seed_charge, a.seed_hits = _ptr(hp["charge"]), _ptr(hp["hits"])
    if out is not None:
        for k, v in out.items():
            if k.startswith("_"):
                continue
            if v is not None and (v.is_cuda or not v.is_contiguous()):
                raise ValueError(f"output {k} must be a contiguous host tensor")
        a.n_cands, a.cand_hits, a.cand_chi2 = _ptr(out["n_cands"]), _ptr(out["cand_hits"]), _ptr(out["cand_chi2"])
        a.cand_nhits, a.cand_status = _ptr(out["cand_nhits"]), _ptr(out["cand_status"])
        a.best_state, a.best_cov = _ptr(out.get("best_state")), _ptr(out.get("best_cov"))
    if counters is not None and (counters.dtype != torch.int64 or counters.numel() < BUILD_COUNTERS or
                                 not counters.is_cuda):
        raise ValueError(f"counters must be a device tensor of {BUILD_COUNTERS} int64")
    a.counters = _ptr(counters)
    if cfg.window_mode == WINDOW_LEARNED:
        if mlp_packed is None or mlp_packed.dtype != torch.uint8 or mlp_packed.numel() < 23048:
            raise ValueError("the learned window needs the packed network (uint8, 23048 bytes)")
        a.mlp_packed = _ptr(mlp_packed)
    if workspace is not None:
        a.workspace, a.workspace_bytes = _ptr(workspace), workspace.numel()
    a.stream = kfmi._stream(stream)
    return a


def build_host_workspace_bytes(ctx, cfg, hp, n_chunks=4, n_slots=4, first_layer=3):
    """kf_build_host_workspace_size for this problem (host tensors from host_problem) and chunking."""
    from . import kfmi
    a = _host_args(ctx, cfg, hp, None, n_chunks, n_slots, first_layer, None, None, None, None)
    n = int(kfmi.load_library().kf_build_host_workspace_size(ctx.h, C.byref(cfg), C.byref(a)))
    if n == 0:
        raise ValueError("invalid problem for kf_build_host (offsets or chunking)")
    return n


def build_host(ctx, cfg, hp, n_chunks=4, n_slots=4, out=None, workspace=None, counters=None, mlp_packed=None,
               first_layer=3, stream=None):
    """kf_build_host: binning and building from host memory with overlapped copies.  hp from host_problem.
    Returns the host output tensors (page-locked; complete once `stream` is synchronised)."""
    import torch
    from . import kfmi
    S, N, L = hp["n_seeds"], cfg.max_cands, ctx.n_layers
    if out is None:
        e = lambda shape, dt: torch.empty(shape, dtype=dt).pin_memory()
        out = dict(n_cands=e((S,), torch.int32), cand_hits=e((L, S, N), torch.int32),
                   cand_chi2=e((S, N), torch.float32), cand_nhits=e((S, N), torch.int32),
                   cand_status=e((S, N), torch.int32), best_state=e((6, S), torch.float32),
                   best_cov=e((21, S), torch.float32))
    if workspace is None:
        workspace = torch.empty(build_host_workspace_bytes(ctx, cfg, hp, n_chunks, n_slots, first_layer),
                                dtype=torch.uint8, device="cuda")
    a = _host_args(ctx, cfg, hp, out, n_chunks, n_slots, first_layer, counters, mlp_packed, workspace, stream)
    kfmi._check(kfmi.load_library().kf_build_host(ctx.h, C.byref(cfg), C.byref(a)))
    out["_keep"] = (hp, workspace, counters, mlp_packed)
    return out
