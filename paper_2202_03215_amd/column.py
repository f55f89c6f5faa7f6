"""Python front-end of one PIC-MCC column on the GPU.

PyTorch supplies device memory (one workspace tensor plus caller-side output
tensors) and the HIP stream; the C ABI (include/pc.h) does the work.  Method
names follow the C entry points: init_column (the constructor), step,
deposit, solve_field, moments, get_state / set_state, get_field / set_field,
set_counters, set_events, counts, sync.

Each column runs on its own default-priority stream (so that the library can
replay whole step periods as a HIP graph); every method orders that stream
against torch's current stream in both directions.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import native as N


def _ptr(t: torch.Tensor | None) -> int | None:
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


class Column:
    """A column created by pc_init_column in a torch-owned workspace."""

    def __init__(self, cfg: dict, device: str | torch.device = "cuda:0",
                 stream: torch.cuda.Stream | None = None):
        self.cfg = dict(cfg)
        self.device = torch.device(device)
        self._c = N.make_config(cfg)
        self.sizes = N.pc_sizes()
        N.check(N.lib().pc_query_sizes(C.byref(self._c), C.byref(self.sizes)))
        self.nn = int(self.sizes.n_nodes)
        self.nc = int(self.sizes.n_cells)
        self.capacity = int(self.sizes.capacity)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.workspace = torch.empty(int(self.sizes.workspace_bytes), dtype=torch.uint8,
                                         device=self.device)
        h = C.c_void_p()
        self._in()
        N.check(N.lib().pc_init_column(C.byref(self._c), self.workspace.data_ptr(),
                                       int(self.sizes.workspace_bytes),
                                       C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self._events = None
        self._destroy = N.lib().pc_destroy   # held: module globals may be gone at interpreter exit

    @classmethod
    def _member(cls, owner: "Batch", index: int, cfg: dict) -> "Column":
        """Borrowed view of column `index` of a batch (shares its stream)."""
        self = cls.__new__(cls)
        self.cfg = dict(cfg)
        self.device = owner.device
        self._c = N.make_config(cfg)
        self.sizes = N.pc_sizes()
        N.check(N.lib().pc_query_sizes(C.byref(self._c), C.byref(self.sizes)))
        self.nn = int(self.sizes.n_nodes)
        self.nc = int(self.sizes.n_cells)
        self.capacity = int(self.sizes.capacity)
        self.stream = owner.stream
        self._owner = owner
        h = C.c_void_p()
        N.check(N.lib().pc_batch_column(owner.h, int(index), C.byref(h)))
        self.h = h
        self._events = None
        return self

    def __del__(self):
        if getattr(self, "_owner", None) is not None:
            return   # batch members are freed with their batch
        h = getattr(self, "h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self.h = None

    # ------------------------------------------------------- stream order
    def _in(self, *tensors):
        """Column stream waits for torch's stream (inputs produced there)."""
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)

    def _out(self):
        """Torch's stream waits for the column stream (outputs written there)."""
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    # ------------------------------------------------------------ stepping
    def step(self, n: int = 1) -> None:
        self._in()
        N.check(N.lib().pc_step(self.h, int(n)))
        self._out()

    def prepare_graphs(self, n: int) -> None:
        """Capture the graphs a following step(n) replays (nothing executes)."""
        N.check(N.lib().pc_prepare_graphs(self.h, int(n)))

    def sync(self) -> None:
        N.check(N.lib().pc_sync(self.h))

    def counts(self) -> dict:
        c = N.pc_counts()
        N.check(N.lib().pc_get_counts(self.h, C.byref(c)))
        return dict(n=(int(c.n[0]), int(c.n[1])), next_id=(int(c.next_id[0]), int(c.next_id[1])),
                    step=int(c.step), errors=int(c.errors),
                    balance=(int(c.births_last), int(c.births_since_ion)),
                    circuit=(float(c.V_anode), int(c.vsum_ion), float(c.emit_carry)),
                    J_cond=float(c.J_cond))

    # ------------------------------------------------------ stand-alone ops
    def _empty(self, n, dtype):
        return torch.empty(n, dtype=dtype, device=self.device)

    def deposit(self, x: torch.Tensor) -> torch.Tensor:
        x = x.to(self.device, torch.float64).contiguous()
        rho = self._empty(self.nn, torch.int64)
        self._in(x, rho)
        N.check(N.lib().pc_deposit(self.h, _ptr(x), x.numel(), _ptr(rho)))
        self._out()
        return rho

    def solve_field(self, rho_e: torch.Tensor, rho_i: torch.Tensor, want_phi: bool = True):
        re = rho_e.to(self.device, torch.int64).contiguous()
        ri = rho_i.to(self.device, torch.int64).contiguous()
        E = self._empty(self.nn, torch.float64)
        phi = self._empty(self.nn, torch.float64) if want_phi else None
        self._in(re, ri, E, phi)
        N.check(N.lib().pc_solve_field(self.h, _ptr(re), _ptr(ri), _ptr(phi), _ptr(E)))
        self._out()
        return phi, E

    def moments(self, cells_per_group: int = 1, reset_iz: bool = False) -> torch.Tensor:
        ng = (self.nc + cells_per_group - 1) // cells_per_group
        out = self._empty(7 * self.nc + ng * 240, torch.int64)
        self._in(out)
        N.check(N.lib().pc_moments(self.h, int(cells_per_group), int(reset_iz), _ptr(out)))
        self._out()
        return out

    # ------------------------------------------------------------ state I/O
    def get_state(self, species: int):
        n = self.counts()["n"][species]
        x, vx, vy, vz = (self._empty(n, torch.float64) for _ in range(4))
        ids = self._empty(n, torch.int32)
        self._in(x, vx, vy, vz, ids)
        N.check(N.lib().pc_get_state(self.h, int(species), _ptr(x), _ptr(vx), _ptr(vy), _ptr(vz),
                                     _ptr(ids), n))
        self._out()
        return x, vx, vy, vz, ids

    def set_state(self, species: int, x, vx, vy, vz, ids) -> None:
        ts = [torch.as_tensor(a).to(self.device, torch.float64).contiguous() for a in (x, vx, vy, vz)]
        it = torch.as_tensor(ids).to(torch.int64).to(torch.int32).to(self.device).contiguous()
        self._in(*ts, it)
        N.check(N.lib().pc_set_state(self.h, int(species), it.numel(), *[_ptr(t) for t in ts],
                                     _ptr(it)))
        torch.cuda.synchronize(self.device)

    def set_counters(self, step: int, next_e: int, next_i: int) -> None:
        N.check(N.lib().pc_set_counters(self.h, int(step), int(next_e), int(next_i)))

    def set_balance(self, births_last: int, births_since_ion: int) -> None:
        N.check(N.lib().pc_set_balance(self.h, int(births_last), int(births_since_ion)))

    def set_circuit(self, V_anode: float, vsum_ion: int, emit_carry: float) -> None:
        """Anode potential, ions' held v_x sum and emission carry (section V)."""
        N.check(N.lib().pc_set_circuit(self.h, float(V_anode), int(vsum_ion), float(emit_carry)))

    def get_field(self):
        E = self._empty(self.nn, torch.float64)
        re = self._empty(self.nn, torch.int64)
        ri = self._empty(self.nn, torch.int64)
        self._in(E, re, ri)
        N.check(N.lib().pc_get_field(self.h, _ptr(E), _ptr(re), _ptr(ri)))
        self._out()
        return E, re, ri

    def set_field(self, E) -> None:
        e = torch.as_tensor(E).to(self.device, torch.float64).contiguous()
        self._in(e)
        N.check(N.lib().pc_set_field(self.h, _ptr(e)))
        torch.cuda.synchronize(self.device)

    def set_events(self, len_e: int, len_i: int):
        """Allocate per-id event buffers (uint8) that each step fills."""
        ev_e = torch.zeros(len_e, dtype=torch.uint8, device=self.device)
        ev_i = torch.zeros(len_i, dtype=torch.uint8, device=self.device)
        self._in(ev_e, ev_i)
        N.check(N.lib().pc_set_events(self.h, _ptr(ev_e), len_e, _ptr(ev_i), len_i))
        self._events = (ev_e, ev_i)
        return self._events

    def timer_enable(self, max_launches: int) -> None:
        N.check(N.lib().pc_timer_enable(self.h, int(max_launches)))

    def timer_read(self):
        """(summed duration in ms, launches) of the timed electron-advance launches."""
        ms = C.c_double()
        n = C.c_int64()
        N.check(N.lib().pc_timer_read(self.h, C.byref(ms), C.byref(n)))
        return float(ms.value), int(n.value)

    def clear_events(self) -> None:
        N.check(N.lib().pc_set_events(self.h, None, 0, None, 0))
        self._events = None


class Batch:
    """Many columns advanced together by pc_init_batch / pc_batch_step in one
    torch-owned workspace; column(c) gives a Column view of member c."""

    def __init__(self, cfgs: list, device: str | torch.device = "cuda:0",
                 stream: torch.cuda.Stream | None = None):
        self.cfgs = [dict(c) for c in cfgs]
        self.device = torch.device(device)
        n = len(self.cfgs)
        self._arr = (N.pc_config * n)(*[N.make_config(c) for c in self.cfgs])
        nbytes = C.c_int64()
        N.check(N.lib().pc_query_batch_sizes(self._arr, n, C.byref(nbytes)))
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        N.check(N.lib().pc_init_batch(self._arr, n, self.workspace.data_ptr(), int(nbytes.value),
                                      C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self._views = {}
        self._destroy = N.lib().pc_batch_destroy   # held: module globals may be gone at interpreter exit

    def __len__(self) -> int:
        return len(self.cfgs)

    def __del__(self):
        h = getattr(self, "h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self.h = None

    def column(self, c: int) -> Column:
        if c not in self._views:
            self._views[c] = Column._member(self, c, self.cfgs[c])
        return self._views[c]

    def step(self, n: int = 1) -> None:
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        N.check(N.lib().pc_batch_step(self.h, int(n)))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def sync(self) -> None:
        N.check(N.lib().pc_batch_sync(self.h))

    def tune(self, trial_steps: int = 80) -> dict:
        t = N.pc_tuning()
        N.check(N.lib().pc_batch_tune(self.h, int(trial_steps), C.byref(t)))
        return dict(chunk=t.chunk, sort_interval=t.sort_interval, n_items_e=t.n_items_e,
                    n_items_i=t.n_items_i, us_per_step=t.us_per_step)

    def tuning(self) -> dict:
        t = N.pc_tuning()
        N.check(N.lib().pc_batch_get_tuning(self.h, C.byref(t)))
        return dict(chunk=t.chunk, sort_interval=t.sort_interval, n_items_e=t.n_items_e,
                    n_items_i=t.n_items_i)

    def set_tuning(self, chunk: int, sort_interval: int) -> None:
        N.check(N.lib().pc_batch_set_tuning(self.h, int(chunk), int(sort_interval)))

    def timer_enable(self, max_launches: int) -> None:
        N.check(N.lib().pc_batch_timer_enable(self.h, int(max_launches)))

    def timer_read(self):
        ms = C.c_double()
        n = C.c_int64()
        N.check(N.lib().pc_batch_timer_read(self.h, C.byref(ms), C.byref(n)))
        return float(ms.value), int(n.value)


def stream_probe(src: torch.Tensor, dst: torch.Tensor, blocks: int = 0) -> None:
    """dst = src (FP64 device tensors) by the library's stream-probe kernel
    on torch's current stream (pc_stream_probe)."""
    if src.dtype != torch.float64 or dst.dtype != torch.float64 or src.numel() != dst.numel():
        raise ValueError("stream probe: two FP64 tensors of one size")
    st = torch.cuda.current_stream(src.device)
    N.check(N.lib().pc_stream_probe(_ptr(src), _ptr(dst), int(src.numel()), int(blocks),
                                    C.c_void_p(st.cuda_stream)))
