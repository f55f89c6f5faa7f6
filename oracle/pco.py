"""ctypes front-end of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this module.  It converts a workload config dict into the oracle's own
``pco_config`` struct; it shares no code with the GPU library or its binding.
"""
from __future__ import annotations

import ctypes as C
import numpy as np

from . import build as _build

ELECTRON, ION = 0, 1
EV_NONE, EV_ELASTIC, EV_EXCITE, EV_IONIZE, EV_WALL, EV_ABSORB, EV_CX, EV_NULL = range(8)
ERR_ECAP, ERR_GCAP, ERR_NUMAX, ERR_IDS, ERR_RANGE = 1, 2, 4, 8, 16
EEPF_BINS = 240


class pco_config(C.Structure):
    _fields_ = [("bc", C.c_int32), ("n_cells", C.c_int32), ("ppc", C.c_int32),
                ("ion_subcycle", C.c_int32), ("wall_mode", C.c_int32),
                ("energy_sharing", C.c_int32), ("poisson", C.c_int32), ("pad0", C.c_int32)] + \
        [(k, C.c_double) for k in ("L", "V", "p_torr", "Tg", "n0", "Te0_eV", "Ti0_K", "nu_w",
                                   "dt", "eps_cap", "g_cap", "M_amu", "el_A", "el_B", "el_p",
                                   "ex_U", "ex_smax", "iz_U", "iz_smax", "cx_sigma", "opb_w",
                                   "emit_J", "emit_T", "circuit_R")] + \
        [("seed", C.c_uint64)]


_libs = {}


def lib(omp: bool = False):
    """The serial oracle library (parity reference), or with omp=True its
    OpenMP timing build (same results, all host cores)."""
    if omp not in _libs:
        path = _build.ensure(omp)
        L = C.CDLL(path)
        P = C.c_void_p
        d = C.POINTER(C.c_double)
        i64 = C.POINTER(C.c_int64)
        u32 = C.POINTER(C.c_uint32)
        u8 = C.POINTER(C.c_uint8)
        L.pco_philox4x32_10.argtypes = [u32, u32, u32]
        L.pco_philox4x32_10.restype = None
        L.pco_create.argtypes = [C.POINTER(pco_config)]
        L.pco_create.restype = P
        L.pco_destroy.argtypes = [P]
        L.pco_destroy.restype = None
        L.pco_init_column.argtypes = [P]
        L.pco_step.argtypes = [P, C.c_int64]
        L.pco_deposit.argtypes = [P, d, C.c_int64, i64]
        L.pco_solve_field.argtypes = [P, i64, i64, d, d]
        L.pco_n_nodes.argtypes = [P]
        L.pco_count.argtypes = [P, C.c_int]
        L.pco_count.restype = C.c_int64
        L.pco_step_index.argtypes = [P]
        L.pco_step_index.restype = C.c_int64
        L.pco_next_id.argtypes = [P, C.c_int]
        L.pco_next_id.restype = C.c_int64
        L.pco_errors.argtypes = [P]
        L.pco_errors.restype = C.c_uint32
        L.pco_constant.argtypes = [P, C.c_int]
        L.pco_constant.restype = C.c_double
        L.pco_get_state.argtypes = [P, C.c_int, d, d, d, d, u32]
        L.pco_set_state.argtypes = [P, C.c_int, C.c_int64, d, d, d, d, u32]
        L.pco_set_counters.argtypes = [P, C.c_int64, C.c_int64, C.c_int64]
        L.pco_set_balance.argtypes = [P, C.c_int64, C.c_int64]
        L.pco_get_balance.argtypes = [P, i64]
        L.pco_get_victims.argtypes = [P, C.c_int, u32, C.c_int64]
        L.pco_set_circuit.argtypes = [P, C.c_double, C.c_int64, C.c_double]
        L.pco_get_circuit.argtypes = [P, d, i64]
        L.pco_get_victims.restype = C.c_int64
        L.pco_get_field.argtypes = [P, d, i64, i64]
        L.pco_set_field.argtypes = [P, d]
        L.pco_get_events.argtypes = [P, C.c_int, u8, C.c_int64]
        L.pco_moments.argtypes = [P, C.c_int32, C.c_int32, i64]
        L.pco_threads.argtypes = [C.c_int]
        L.pco_threads.restype = C.c_int
        _libs[omp] = L
    return _libs[omp]


def threads(n: int = 0) -> int:
    """Threads of the OpenMP timing build (n > 0 sets them)."""
    return int(lib(True).pco_threads(int(n)))


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().pco_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def make_config(cfg: dict) -> pco_config:
    s = pco_config()
    s.bc = {"bounded": 0, "periodic": 1}[cfg["bc"]]
    s.n_cells = int(cfg["n_cells"])
    s.ppc = int(cfg["ppc"])
    s.ion_subcycle = int(cfg["ion_subcycle"])
    s.wall_mode = {"off": 0, "fixed": 1, "balanced": 2, "pair": 3}[cfg["wall_mode"]]
    s.energy_sharing = {"opb": 0, "equal": 1}[cfg["energy_sharing"]]
    s.poisson = int(cfg["poisson"])
    for k in ("L", "V", "p_torr", "Tg", "n0", "Te0_eV", "Ti0_K", "nu_w", "dt", "eps_cap",
              "g_cap", "M_amu", "el_A", "el_B", "el_p", "ex_U", "ex_smax", "iz_U", "iz_smax",
              "cx_sigma", "opb_w"):
        setattr(s, k, float(cfg[k]))
    s.emit_J = float(cfg.get("emit_J", 0.0))
    s.emit_T = float(cfg.get("emit_T", 0.5))
    s.circuit_R = float(cfg.get("circuit_R", 0.0))
    s.seed = int(cfg["seed"])
    return s


class Oracle:
    """One oracle column on host memory."""

    def __init__(self, cfg: dict, init: bool = True, omp: bool = False):
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        self._L = lib(omp)
        self.h = self._L.pco_create(C.byref(self._c))
        if not self.h:
            raise ValueError("oracle rejected the config")
        self.nc = int(cfg["n_cells"])
        self.nn = self._L.pco_n_nodes(self.h)
        if init:
            self._chk(self._L.pco_init_column(self.h))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self._L.pco_destroy(h)
            self.h = None

    @staticmethod
    def _chk(rc):
        if rc != 0:
            raise RuntimeError(f"oracle call failed with {rc}")

    def step(self, n: int = 1):
        self._chk(self._L.pco_step(self.h, int(n)))

    def deposit(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        rho = np.zeros(self.nn, dtype=np.int64)
        self._chk(self._L.pco_deposit(self.h, _ptr(x, C.c_double), x.size, _ptr(rho, C.c_int64)))
        return rho

    def solve_field(self, rho_e: np.ndarray, rho_i: np.ndarray):
        re = np.ascontiguousarray(rho_e, dtype=np.int64)
        ri = np.ascontiguousarray(rho_i, dtype=np.int64)
        phi = np.zeros(self.nn)
        E = np.zeros(self.nn)
        self._chk(self._L.pco_solve_field(self.h, _ptr(re, C.c_int64), _ptr(ri, C.c_int64),
                                        _ptr(phi, C.c_double), _ptr(E, C.c_double)))
        return phi, E

    def count(self, s: int) -> int:
        return int(self._L.pco_count(self.h, s))

    @property
    def step_index(self) -> int:
        return int(self._L.pco_step_index(self.h))

    def next_id(self, s: int) -> int:
        return int(self._L.pco_next_id(self.h, s))

    @property
    def errors(self) -> int:
        return int(self._L.pco_errors(self.h))

    def constant(self, name: str) -> float:
        idx = {"dx": 0, "nu_max": 1, "P_null": 2, "W": 3, "Ng": 4, "P_cx": 5}[name]
        return float(self._L.pco_constant(self.h, idx))

    def state(self, s: int):
        n = self.count(s)
        x, vx, vy, vz = (np.zeros(n) for _ in range(4))
        ids = np.zeros(n, dtype=np.uint32)
        self._chk(self._L.pco_get_state(self.h, s, _ptr(x, C.c_double), _ptr(vx, C.c_double),
                                      _ptr(vy, C.c_double), _ptr(vz, C.c_double),
                                      _ptr(ids, C.c_uint32)))
        return x, vx, vy, vz, ids

    def set_state(self, s: int, x, vx, vy, vz, ids):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, vx, vy, vz)]
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        self._chk(self._L.pco_set_state(self.h, s, ids.size,
                                      *[_ptr(a, C.c_double) for a in arrs],
                                      _ptr(ids, C.c_uint32)))

    def set_counters(self, step: int, next_e: int, next_i: int):
        self._chk(self._L.pco_set_counters(self.h, int(step), int(next_e), int(next_i)))

    def set_balance(self, births_last: int, births_since_ion: int):
        self._chk(self._L.pco_set_balance(self.h, int(births_last), int(births_since_ion)))

    def balance(self):
        out = np.zeros(2, dtype=np.int64)
        self._chk(self._L.pco_get_balance(self.h, _ptr(out, C.c_int64)))
        return int(out[0]), int(out[1])

    def set_circuit(self, V_anode: float, vsum_ion: int, emit_carry: float):
        self._chk(self._L.pco_set_circuit(self.h, float(V_anode), int(vsum_ion), float(emit_carry)))

    def circuit(self) -> dict:
        """Section V state: anode potential, last conduction current density,
        emission carry and the ions' held v_x sum."""
        out = np.zeros(3)
        vs = np.zeros(1, dtype=np.int64)
        self._chk(self._L.pco_get_circuit(self.h, _ptr(out, C.c_double), _ptr(vs, C.c_int64)))
        return dict(V_anode=float(out[0]), J_cond=float(out[1]), emit_carry=float(out[2]), vsum_ion=int(vs[0]))

    def victims(self, species: int) -> np.ndarray:
        """Pair sink: ids removed by the last step, in ionization-rank order."""
        m = int(self._L.pco_get_victims(self.h, species, None, 0))
        out = np.zeros(max(m, 1), dtype=np.uint32)
        self._L.pco_get_victims(self.h, species, _ptr(out, C.c_uint32), m)
        return out[:m]

    def field(self):
        E = np.zeros(self.nn)
        re = np.zeros(self.nn, dtype=np.int64)
        ri = np.zeros(self.nn, dtype=np.int64)
        self._chk(self._L.pco_get_field(self.h, _ptr(E, C.c_double), _ptr(re, C.c_int64),
                                      _ptr(ri, C.c_int64)))
        return E, re, ri

    def set_field(self, E: np.ndarray):
        E = np.ascontiguousarray(E, dtype=np.float64)
        self._chk(self._L.pco_set_field(self.h, _ptr(E, C.c_double)))

    def events(self, s: int, length: int | None = None) -> np.ndarray:
        n = self.next_id(s) if length is None else length
        ev = np.zeros(n, dtype=np.uint8)
        self._chk(self._L.pco_get_events(self.h, s, _ptr(ev, C.c_uint8), n))
        return ev

    def moments(self, cells_per_group: int = 1, reset_iz: bool = False) -> np.ndarray:
        ng = (self.nc + cells_per_group - 1) // cells_per_group
        out = np.zeros(7 * self.nc + ng * EEPF_BINS, dtype=np.int64)
        self._chk(self._L.pco_moments(self.h, cells_per_group, int(reset_iz),
                                    _ptr(out, C.c_int64)))
        return out
