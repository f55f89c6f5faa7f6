"""ctypes binding of libpc.so (the gfx950 HIP library declared in include/pc.h).

Argument marshalling only: every step of the particle path runs in the HIP
kernels.  Importing this module does not touch the GPU; loading fails loudly
if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpc.so")

PC_OK = 0
STATUS = {
    -1: "PC_ERR_INVALID_ARG", -2: "PC_ERR_UNSTABLE_CONFIG", -3: "PC_ERR_CAPACITY",
    -4: "PC_ERR_NONFINITE", -5: "PC_ERR_ECAP", -6: "PC_ERR_GCAP", -7: "PC_ERR_HIP",
    -8: "PC_ERR_POISONED", -9: "PC_ERR_WORKSPACE", -10: "PC_ERR_IDS",
}
ELECTRON, ION = 0, 1

# every exported symbol of include/*.h
EXPORTS = ("pc_query_sizes", "pc_init_column", "pc_step", "pc_prepare_graphs", "pc_deposit", "pc_solve_field",
           "pc_moments", "pc_get_counts", "pc_get_state", "pc_set_state", "pc_set_counters", "pc_set_balance",
           "pc_set_circuit",
           "pc_get_field", "pc_set_field", "pc_set_events", "pc_timer_enable",
           "pc_timer_read", "pc_sync", "pc_destroy",
           "pc_query_batch_sizes", "pc_init_batch", "pc_batch_step", "pc_batch_column",
           "pc_batch_tune", "pc_batch_get_tuning", "pc_batch_set_tuning",
           "pc_batch_timer_enable", "pc_batch_timer_read", "pc_batch_sync", "pc_batch_destroy",
           "pc_stream_probe", "pc_status_string", "pc_last_error",
           "pc_mlp_query", "pc_mlp_pack", "pc_mlp_forward", "pc_mlp_grad", "pc_mlp_grad_noalloc", "pc_mlp_adam",
           "pc_mlp_last_error",
           "pc_fluid_query", "pc_fluid_init", "pc_fluid_set_state", "pc_fluid_get_state",
           "pc_fluid_set_closure", "pc_fluid_set_closure_multipliers", "pc_fluid_step", "pc_fluid_get_faces", "pc_cyclic_tridiag",
           "pc_fluid_destroy", "pc_fluid_last_error")


class PcError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status


class pc_config(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("bc", "n_cells", "ppc", "ion_subcycle", "wall_mode",
                                         "energy_sharing", "poisson", "sort_interval",
                                         "launch_blocks", "precision", "pad1", "pad2")] + \
        [(k, C.c_double) for k in ("L", "V", "p_torr", "Tg", "n0", "Te0_eV", "Ti0_K", "nu_w",
                                   "dt", "eps_cap", "g_cap", "capacity", "M_amu", "el_A",
                                   "el_B", "el_p", "ex_U", "ex_smax", "iz_U", "iz_smax",
                                   "cx_sigma", "opb_w", "emit_J", "emit_T", "circuit_R")] + \
        [("seed", C.c_uint64)]


class pc_sizes(C.Structure):
    _fields_ = [("workspace_bytes", C.c_int64), ("capacity", C.c_int64),
                ("max_births", C.c_int64), ("max_losses", C.c_int64),
                ("n_nodes", C.c_int32), ("n_cells", C.c_int32),
                ("nu_max", C.c_double), ("p_null", C.c_double), ("p_cx", C.c_double)]


class pc_counts(C.Structure):
    _fields_ = [("n", C.c_int64 * 2), ("next_id", C.c_int64 * 2), ("step", C.c_int64),
                ("errors", C.c_uint32), ("pad", C.c_uint32), ("births_last", C.c_int64),
                ("births_since_ion", C.c_int64), ("V_anode", C.c_double), ("J_cond", C.c_double),
                ("vsum_ion", C.c_int64), ("emit_carry", C.c_double)]


class pc_tuning(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("sort_interval", C.c_int32), ("n_items_e", C.c_int32),
                ("n_items_i", C.c_int32), ("us_per_step", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """Load libpc.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2202_03215_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    P, I64, I32 = C.c_void_p, C.c_int64, C.c_int32
    sig = {
        "pc_query_sizes": [C.POINTER(pc_config), C.POINTER(pc_sizes)],
        "pc_init_column": [C.POINTER(pc_config), P, C.c_size_t, P, C.POINTER(P)],
        "pc_step": [P, I64],
        "pc_prepare_graphs": [P, I64],
        "pc_deposit": [P, P, I64, P],
        "pc_solve_field": [P, P, P, P, P],
        "pc_moments": [P, I32, I32, P],
        "pc_get_counts": [P, C.POINTER(pc_counts)],
        "pc_get_state": [P, I32, P, P, P, P, P, I64],
        "pc_set_state": [P, I32, I64, P, P, P, P, P],
        "pc_set_counters": [P, I64, I64, I64],
        "pc_set_balance": [P, I64, I64],
        "pc_set_circuit": [P, C.c_double, I64, C.c_double],
        "pc_get_field": [P, P, P, P],
        "pc_set_field": [P, P],
        "pc_set_events": [P, P, I64, P, I64],
        "pc_timer_enable": [P, I64],
        "pc_timer_read": [P, C.POINTER(C.c_double), C.POINTER(I64)],
        "pc_sync": [P],
        "pc_query_batch_sizes": [C.POINTER(pc_config), I32, C.POINTER(I64)],
        "pc_init_batch": [C.POINTER(pc_config), I32, P, C.c_size_t, P, C.POINTER(P)],
        "pc_batch_step": [P, I64],
        "pc_batch_column": [P, I32, C.POINTER(P)],
        "pc_batch_tune": [P, I32, C.POINTER(pc_tuning)],
        "pc_batch_get_tuning": [P, C.POINTER(pc_tuning)],
        "pc_batch_set_tuning": [P, I32, I32],
        "pc_batch_timer_enable": [P, I64],
        "pc_batch_timer_read": [P, C.POINTER(C.c_double), C.POINTER(I64)],
        "pc_batch_sync": [P],
        "pc_stream_probe": [P, P, I64, I32, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int32
    L.pc_destroy.argtypes = [P]
    L.pc_destroy.restype = None
    L.pc_batch_destroy.argtypes = [P]
    L.pc_batch_destroy.restype = None
    L.pc_status_string.argtypes = [C.c_int32]
    L.pc_status_string.restype = C.c_char_p
    L.pc_last_error.argtypes = []
    L.pc_last_error.restype = C.c_char_p
    _lib = L
    return L


def check(status: int) -> None:
    if status != PC_OK:
        detail = lib().pc_last_error().decode(errors="replace")
        raise PcError(status, detail)


def make_config(cfg: dict) -> pc_config:
    s = pc_config()
    s.bc = {"bounded": 0, "periodic": 1}[cfg["bc"]]
    s.n_cells = int(cfg["n_cells"])
    s.ppc = int(cfg["ppc"])
    s.ion_subcycle = int(cfg["ion_subcycle"])
    s.wall_mode = {"off": 0, "fixed": 1, "balanced": 2, "pair": 3}[cfg["wall_mode"]]
    s.energy_sharing = {"opb": 0, "equal": 1}[cfg["energy_sharing"]]
    s.poisson = int(cfg["poisson"])
    s.sort_interval = int(cfg.get("sort_interval", 0))
    s.launch_blocks = int(cfg.get("launch_blocks", 0))
    s.precision = {"fp64": 0, "fp32": 1}[cfg.get("precision", "fp64")]
    for k in ("L", "V", "p_torr", "Tg", "n0", "Te0_eV", "Ti0_K", "nu_w", "dt", "eps_cap",
              "g_cap", "M_amu", "el_A", "el_B", "el_p", "ex_U", "ex_smax", "iz_U", "iz_smax",
              "cx_sigma", "opb_w"):
        setattr(s, k, float(cfg[k]))
    s.capacity = float(cfg.get("capacity", 1.25))
    s.emit_J = float(cfg.get("emit_J", 0.0))
    s.emit_T = float(cfg.get("emit_T", 0.5))
    s.circuit_R = float(cfg.get("circuit_R", 0.0))
    s.seed = int(cfg["seed"])
    return s


def query_sizes(cfg: dict) -> pc_sizes:
    c = make_config(cfg)
    out = pc_sizes()
    check(lib().pc_query_sizes(C.byref(c), C.byref(out)))
    return out


def query_batch_sizes(cfgs: list) -> int:
    arr = (pc_config * len(cfgs))(*[make_config(c) for c in cfgs])
    out = C.c_int64()
    check(lib().pc_query_batch_sizes(arr, len(cfgs), C.byref(out)))
    return int(out.value)
