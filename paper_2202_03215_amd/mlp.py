"""Python front-end of the closure network kernels (include/pc_mlp.h).

Device memory comes from torch tensors; every computation runs in the HIP
kernels of libpc.so (argument marshalling only here).  Parameters are the
flat FP32 master vector of include/pc_mlp.h; inputs are float32 [n, 5] and
targets / outputs float32 [n, 2], already normalised by the caller.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import native as N

N_PARAMS = 8834


class pc_mlp_sizes(C.Structure):
    _fields_ = [("params", C.c_int64), ("packed_bytes", C.c_int64), ("scratch_bytes", C.c_int64)]


def _lib():
    L = N.lib()
    if not getattr(L, "_mlp_sig", False):
        P, I64 = C.c_void_p, C.c_int64
        sig = {
            "pc_mlp_query": [I64, C.POINTER(pc_mlp_sizes)],
            "pc_mlp_pack": [P, P, P],
            "pc_mlp_forward": [P, P, I64, P, P, P],
            "pc_mlp_grad": [P, P, P, I64, P, P, P, C.c_size_t, P],
            "pc_mlp_grad_noalloc": [P, P, P, I64, P, P, P],
            "pc_mlp_adam": [P, P, P, P, I64, C.c_double, C.c_double, C.c_double, C.c_double, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32
        L.pc_mlp_last_error.argtypes = []
        L.pc_mlp_last_error.restype = C.c_char_p
        L._mlp_sig = True
    return L


def _check(status: int) -> None:
    if status != 0:
        raise N.PcError(status, _lib().pc_mlp_last_error().decode(errors="replace"))


def _ptr(t):
    return None if t is None else t.data_ptr()


class ClosureNet:
    """Parameters, Adam state and packed operands of one network on a device."""

    def __init__(self, params=None, device="cuda:0", max_batch: int = 1 << 16):
        self.device = torch.device(device)
        sz = pc_mlp_sizes()
        _check(_lib().pc_mlp_query(int(max_batch), C.byref(sz)))
        self.max_batch = int(max_batch)
        if params is None:
            params = np.zeros(N_PARAMS, dtype=np.float32)
        self.master = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(self.device).contiguous()
        if self.master.numel() != N_PARAMS:
            raise ValueError(f"expected {N_PARAMS} parameters")
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.packed = torch.empty(int(sz.packed_bytes), dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(int(sz.scratch_bytes), dtype=torch.uint8, device=self.device)
        self.step_count = 0
        self.pack()

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def pack(self) -> None:
        _check(_lib().pc_mlp_pack(_ptr(self.master), _ptr(self.packed), self._stream()))

    def set_params(self, params) -> None:
        self.master.copy_(torch.as_tensor(np.asarray(params, dtype=np.float32)))
        self.pack()

    def params(self) -> np.ndarray:
        return self.master.cpu().numpy().astype(np.float64)

    def forward(self, x: torch.Tensor, hidden: bool = False):
        x = x.to(self.device, torch.float32).contiguous()
        n = x.shape[0]
        y = torch.empty((n, 2), dtype=torch.float32, device=self.device)
        h = torch.empty((3, n, 64), dtype=torch.int16, device=self.device) if hidden else None
        _check(_lib().pc_mlp_forward(_ptr(self.packed), _ptr(x), n, _ptr(y), _ptr(h), self._stream()))
        return (y, h) if hidden else y

    def grad_loss(self, x: torch.Tensor, t: torch.Tensor):
        """Gradient (device float32 [8834]) and loss of the mean squared error."""
        x = x.to(self.device, torch.float32).contiguous()
        t = t.to(self.device, torch.float32).contiguous()
        n = x.shape[0]
        if n > self.max_batch:
            raise ValueError("batch larger than max_batch")
        _check(_lib().pc_mlp_grad(_ptr(self.packed), _ptr(x), _ptr(t), n, _ptr(self.grad), _ptr(self.loss),
                                  _ptr(self.scratch), self.scratch.numel(), self._stream()))
        return self.grad, self.loss

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        self.step_count += 1
        _check(_lib().pc_mlp_adam(_ptr(self.master), _ptr(self.m), _ptr(self.v), _ptr(self.grad),
                                  self.step_count, lr, beta1, beta2, eps, _ptr(self.packed), self._stream()))

    def train(self, x: torch.Tensor, t: torch.Tensor, steps: int, lr: float, batch: int | None = None,
              seed: int = 0):
        """Adam on minibatches (sampled without replacement per epoch with a
        seeded generator); returns the per-step losses."""
        x = x.to(self.device, torch.float32).contiguous()
        t = t.to(self.device, torch.float32).contiguous()
        n = x.shape[0]
        b = min(batch or n, self.max_batch, n)
        g = torch.Generator(device="cpu").manual_seed(seed)
        perm = torch.randperm(n, generator=g).to(self.device)
        pos = 0
        losses = torch.empty(steps, dtype=torch.float32, device=self.device)
        for k in range(steps):
            if pos + b > n:
                perm = torch.randperm(n, generator=g).to(self.device)
                pos = 0
            idx = perm[pos:pos + b]
            pos += b
            xb = x if b == n else x.index_select(0, idx).contiguous()
            tb = t if b == n else t.index_select(0, idx).contiguous()
            self.grad_loss(xb, tb)
            losses[k] = self.loss[0]
            self.adam(lr)
        return losses.cpu().numpy()


def glorot_params(seed: int = 0) -> np.ndarray:
    """Initial parameters: Glorot-uniform weights, zero biases (flat layout of
    include/pc_mlp.h), from a seeded generator."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((5, 64), (64, 64), (64, 64), (64, 2)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-lim, lim, size=fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def bf16_bits_to_float(h: torch.Tensor) -> np.ndarray:
    """BF16 bit patterns (int16 tensor) -> float64 numpy array."""
    u = h.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)
