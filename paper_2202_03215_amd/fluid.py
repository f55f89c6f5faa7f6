"""Python front-end of the batched fluid column (include/pc_fluid.h).

Device memory comes from torch; every step runs in the HIP kernels of
libpc.so (argument marshalling only).  Columns share the cell count, the
time step and the transport table; each has its own length, gas density,
imposed field, radial loss frequency and ion mobility.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import native as N


class pc_fluid_column(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("L", "Ngas", "E0", "nu_w", "muiN")]


class pc_fluid_config(C.Structure):
    _fields_ = [("n_columns", C.c_int32), ("n_cells", C.c_int32), ("table_len", C.c_int32),
                ("pad", C.c_int32), ("dt", C.c_double), ("T_min", C.c_double), ("T_step", C.c_double),
                ("n_floor", C.c_double)]


def _lib():
    L = N.lib()
    if not getattr(L, "_fluid_sig", False):
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "pc_fluid_query": [C.POINTER(pc_fluid_config), C.POINTER(I64)],
            "pc_fluid_init": [C.POINTER(pc_fluid_config), C.POINTER(pc_fluid_column), C.POINTER(C.c_double),
                              P, C.c_size_t, P, C.POINTER(P)],
            "pc_fluid_set_state": [P, P, P],
            "pc_fluid_get_state": [P, P, P],
            "pc_fluid_set_closure": [P, P, C.POINTER(C.c_float)],
            "pc_fluid_set_closure_multipliers": [P, P, C.POINTER(C.c_float)],
            "pc_fluid_step": [P, I64],
            "pc_fluid_get_faces": [P, P, P, P],
            "pc_cyclic_tridiag": [P, P, P, P, I32, I32, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32
        L.pc_fluid_destroy.argtypes = [P]
        L.pc_fluid_destroy.restype = None
        L.pc_fluid_last_error.argtypes = []
        L.pc_fluid_last_error.restype = C.c_char_p
        L._fluid_sig = True
    return L


def _check(status: int) -> None:
    if status != 0:
        raise N.PcError(status, _lib().pc_fluid_last_error().decode(errors="replace"))


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def cyclic_tridiag(a: torch.Tensor, b: torch.Tensor, c: torch.Tensor, d: torch.Tensor) -> torch.Tensor:
    """Solve the cyclic tridiagonal systems [ns, n] on the GPU; returns x."""
    a, b, c = (t.to(torch.float64).contiguous() for t in (a, b, c))
    x = d.to(torch.float64).clone().contiguous()
    ns, n = x.shape
    _check(_lib().pc_cyclic_tridiag(a.data_ptr(), b.data_ptr(), c.data_ptr(), x.data_ptr(), ns, n,
                                    _stream(x.device)))
    return x


class FluidBatch:
    def __init__(self, columns: list, n_cells: int, dt: float, table: np.ndarray, T_min: float,
                 T_step: float, n_floor: float = 1.0e6, device="cuda:0"):
        self.device = torch.device(device)
        self.n_cells = int(n_cells)
        self.n_columns = len(columns)
        tab = np.ascontiguousarray(np.asarray(table, dtype=np.float64))
        self.cfg = pc_fluid_config(self.n_columns, self.n_cells, tab.shape[0], 0, dt, T_min, T_step, n_floor)
        cols = (pc_fluid_column * self.n_columns)(
            *[pc_fluid_column(c["L"], c["Ngas"], c["E0"], c["nu_w"], c["muiN"]) for c in columns])
        nbytes = C.c_int64()
        _check(_lib().pc_fluid_query(C.byref(self.cfg), C.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(_lib().pc_fluid_init(C.byref(self.cfg), cols, tab.ctypes.data_as(C.POINTER(C.c_double)),
                                    self.workspace.data_ptr(), int(nbytes.value), _stream(self.device),
                                    C.byref(h)))
        self.h = h
        self._net = None
        self._destroy = _lib().pc_fluid_destroy   # held: module globals may be gone at interpreter exit

    def __del__(self):
        h = getattr(self, "h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self.h = None

    def set_state(self, n, w) -> None:
        n = torch.as_tensor(np.asarray(n, dtype=np.float32)).to(self.device).contiguous()
        w = torch.as_tensor(np.asarray(w, dtype=np.float32)).to(self.device).contiguous()
        _check(_lib().pc_fluid_set_state(self.h, n.data_ptr(), w.data_ptr()))
        torch.cuda.synchronize(self.device)

    def get_state(self):
        n = torch.empty((self.n_columns, self.n_cells), dtype=torch.float32, device=self.device)
        w = torch.empty_like(n)
        _check(_lib().pc_fluid_get_state(self.h, n.data_ptr(), w.data_ptr()))
        return n, w

    def set_closure(self, net=None, norm=None, multipliers: bool = False) -> None:
        """net: a ClosureNet (packed operands used) or None for the table
        closure; multipliers: the network answers multipliers (m_D, m_eps) of
        the tabulated coefficients instead of the fluxes."""
        self._net = net
        self._fluxes_stored = net is None or multipliers
        arr = (C.c_float * 14)(*([float(v) for v in norm] if norm is not None else [0.0] * 14))
        if multipliers:
            if net is None:
                raise ValueError("the multiplier closure needs a network")
            _check(_lib().pc_fluid_set_closure_multipliers(self.h, net.packed.data_ptr(), arr))
        else:
            _check(_lib().pc_fluid_set_closure(self.h, net.packed.data_ptr() if net is not None else None, arr))

    def step(self, n: int = 1) -> None:
        _check(_lib().pc_fluid_step(self.h, int(n)))

    def faces(self):
        E = torch.empty((self.n_columns, self.n_cells), dtype=torch.float32, device=self.device)
        if getattr(self, "_fluxes_stored", True):
            g = torch.empty_like(E)
            H = torch.empty_like(E)
            _check(_lib().pc_fluid_get_faces(self.h, g.data_ptr(), H.data_ptr(), E.data_ptr()))
            return g, H, E
        _check(_lib().pc_fluid_get_faces(self.h, None, None, E.data_ptr()))
        return None, None, E
