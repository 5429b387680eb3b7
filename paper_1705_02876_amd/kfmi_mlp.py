"""Binding of the learned-window network calls of include/kfmi.h (argument marshalling only).

Tensors are float32 on the GPU; records are feature-major, x (8, ldx), targets
t (2, ldt), outputs y (2, ldy).  Parameters are one vector of MLP_PARAMS values
in the order W1 [64][8], b1, W2 [64][64], b2, W3 [2][64], b3.
"""
from __future__ import annotations

import ctypes as C

MLP_PARAMS = 4866
MLP_PACKED_BYTES = 23048


def declare(lib):
    P, I32, I64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    lib.kf_mlp_pack.restype = I32
    lib.kf_mlp_pack.argtypes = [P, P, P, P]
    lib.kf_mlp_forward.restype = I32
    lib.kf_mlp_forward.argtypes = [P, I64, P, I64, P, P, I64, P]
    lib.kf_mlp_grad_workspace_size.restype = C.c_size_t
    lib.kf_mlp_grad_workspace_size.argtypes = []
    lib.kf_mlp_grad.restype = I32
    lib.kf_mlp_grad.argtypes = [P, I64, P, I64, P, I64, P, P, P, P, P, C.c_size_t, P]
    lib.kf_mlp_adam.restype = I32
    lib.kf_mlp_adam.argtypes = [P, P, P, P, P, I32, F, F, F, F, P, P]
    return lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, dtype, name, min_numel=None):
    if t is None or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} GPU tensor")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name} needs at least {min_numel} elements")


def _records(x, rows, name):
    import torch
    _need(x, torch.float32, name)
    if x.dim() != 2 or x.shape[0] != rows:
        raise ValueError(f"{name} must be ({rows}, ld)")
    return x.shape[1]


def new_packed(device="cuda"):
    import torch
    return torch.empty(MLP_PACKED_BYTES, dtype=torch.uint8, device=device)


def pack(ctx, params, packed, stream=None):
    """kf_mlp_pack: float32 parameters -> the kernels' bf16 tile layout."""
    import torch
    from . import kfmi
    _need(params, torch.float32, "params", MLP_PARAMS)
    _need(packed, torch.uint8, "packed", MLP_PACKED_BYTES)
    kfmi._check(kfmi.load_library().kf_mlp_pack(ctx.h, _ptr(params), _ptr(packed), kfmi._stream(stream)))
    return packed


def forward(ctx, x, packed, y=None, n=None, stream=None):
    """kf_mlp_forward: outputs (log s_t, log s_z) as a (2, n) tensor."""
    import torch
    from . import kfmi
    ldx = _records(x, 8, "x")
    n = ldx if n is None else n
    if y is None:
        y = torch.empty(2, n, dtype=torch.float32, device=x.device)
    ldy = _records(y, 2, "y")
    _need(packed, torch.uint8, "packed", MLP_PACKED_BYTES)
    kfmi._check(kfmi.load_library().kf_mlp_forward(ctx.h, n, _ptr(x), ldx, _ptr(packed), _ptr(y), ldy,
                                                   kfmi._stream(stream)))
    return y


def workspace_bytes():
    from . import kfmi
    return int(kfmi.load_library().kf_mlp_grad_workspace_size())


def grad(ctx, x, t, packed, grad_out=None, workspace=None, n=None, stream=None):
    """kf_mlp_grad: returns (grad, loss, count) device tensors (mean over the used records)."""
    import torch
    from . import kfmi
    ldx = _records(x, 8, "x")
    ldt = _records(t, 2, "t")
    n = min(ldx, ldt) if n is None else n
    dev = x.device
    if grad_out is None:
        grad_out = torch.empty(MLP_PARAMS + 2, dtype=torch.float32, device=dev)
    _need(grad_out, torch.float32, "grad_out", MLP_PARAMS + 2)
    if workspace is None:
        workspace = torch.empty(workspace_bytes(), dtype=torch.uint8, device=dev)
    g = grad_out[:MLP_PARAMS]
    loss = grad_out[MLP_PARAMS:MLP_PARAMS + 1]
    count = grad_out[MLP_PARAMS + 1:MLP_PARAMS + 2]
    kfmi._check(kfmi.load_library().kf_mlp_grad(ctx.h, n, _ptr(x), ldx, _ptr(t), ldt, _ptr(packed), _ptr(g),
                                                _ptr(loss), _ptr(count), _ptr(workspace), workspace.numel(),
                                                kfmi._stream(stream)))
    return g, loss, count


def adam(ctx, params, g, m, v, step, lr, packed, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """kf_mlp_adam: one bias-corrected Adam step on params (in place), then repack."""
    import torch
    from . import kfmi
    for a, nm in ((params, "params"), (g, "grad"), (m, "m"), (v, "v")):
        _need(a, torch.float32, nm, MLP_PARAMS)
    _need(packed, torch.uint8, "packed", MLP_PACKED_BYTES)
    kfmi._check(kfmi.load_library().kf_mlp_adam(ctx.h, _ptr(params), _ptr(g), _ptr(m), _ptr(v), int(step),
                                                float(lr), float(beta1), float(beta2), float(eps), _ptr(packed),
                                                kfmi._stream(stream)))


class Trainer:
    """Adam training of the window network on device-resident records; every
    step (forward, backward, reduction, update, repack) runs in the library."""

    def __init__(self, ctx, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        self.ctx = ctx
        self.params = params.detach().to(device="cuda", dtype=torch.float32).contiguous().clone()
        dev = self.params.device
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.packed = pack(ctx, self.params, new_packed(dev))
        self.buf = torch.empty(MLP_PARAMS + 2, dtype=torch.float32, device=dev)
        self.ws = torch.empty(workspace_bytes(), dtype=torch.uint8, device=dev)
        self.step_no = 0
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps

    def step(self, x, t, n=None):
        """One full-batch step on (x, t); returns the device loss of the batch before the update."""
        g, loss, _ = grad(self.ctx, x, t, self.packed, self.buf, self.ws, n=n)
        self.step_no += 1
        adam(self.ctx, self.params, g, self.m, self.v, self.step_no, self.lr, self.packed, self.beta1, self.beta2,
             self.eps)
        return loss
