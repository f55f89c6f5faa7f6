"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the bench.

This module holds *data only*: gas parameters, the synthetic cross-section
constants, the column configurations and seeded random particle arrays.  It
contains none of the method's arithmetic (no push, no collision, no field
solve); each backend turns a config dict into its own native struct and
derives every physical quantity itself.

Config keys (all SI unless noted):
  gas           "Ne" | "Ar" (label only; masses and cross sections are explicit)
  M_amu         atom / ion mass in atomic mass units
  el_A, el_B    elastic cross section sigma_el = A + B * (eps/1 eV)**el_p  [m^2]
  el_p          +0.5 or -0.5 (so that only sqrt is needed)
  ex_U, ex_smax lumped excitation: threshold [eV], peak sigma [m^2] (Thomson-like
                shape 4 smax (U/eps)(1 - U/eps), peak at eps = 2U)
  iz_U, iz_smax ionization: threshold [eV], peak sigma [m^2] (same shape)
  cx_sigma      constant ion-atom charge-exchange cross section [m^2]
  opb_w         energy-sharing width of the ionization split [eV]
  bc            "bounded" (grounded x=0, anode phi(L)=V, absorbing walls) |
                "periodic" (reinjection, imposed mean field E0 = V/L)
  n_cells, L    grid cells and column length [m]
  V             anode voltage (bounded) or E0*L (periodic) [V]
  p_torr, Tg    gas pressure [Torr] and temperature [K]
  n0            initial plasma density [m^-3]
  ppc           macroparticles per cell per species at t=0
  Te0_eV, Ti0_K initial electron temperature [eV] and ion temperature [K]
  wall_mode     "off" | "fixed": radial-loss sink with frequency nu_w [s^-1] |
                "balanced": removal probability = ionizations since the species'
                previous step / its count (constant particle number on average) |
                "pair": per ionization one random electron and one random ion
                removed, the products take their ids (constant counts; periodic)
  dt            electron time step [s]; ions advance every ion_subcycle steps
  eps_cap       energy [eV] up to which the null-collision bound is taken
  g_cap         relative-speed bound [m/s] of the ion null-collision method
  energy_sharing "opb" | "equal" split of the ionization excess energy
  poisson       1 = self-consistent field, 0 = imposed field only (swarm mode)
  sort_interval steps between counting sorts (0 = never; no effect on physics)
  emit_J, emit_T bounded columns: cathode emission current density [A/m^2]
                and temperature of the emitted electrons [eV] (section V)
  circuit_R     bounded columns: series resistance [ohm m^2] between the
                source V and the anode (0 = anode held at V)
  capacity      particle-array capacity as a multiple of the initial count
  precision     "fp64" | "fp32" particle state on the GPU (the oracle is FP64)
  seed          Philox key
"""
from __future__ import annotations

import copy
import numpy as np

# Synthetic cross-section sets.  The forms follow the lumped-level description of
# the paper (one excitation level, one ionization channel, constant ion charge
# exchange); the numbers are this project's own order-of-magnitude choices, not
# tabulated data.
NEON = dict(gas="Ne", M_amu=20.1797,
            el_A=1.0e-21, el_B=4.0e-21, el_p=0.5,
            ex_U=16.6, ex_smax=1.6e-21,
            iz_U=21.56, iz_smax=6.0e-21,
            cx_sigma=4.0e-19, opb_w=24.0)

ARGON = dict(gas="Ar", M_amu=39.948,
             el_A=1.0e-21, el_B=2.0e-20, el_p=0.5,
             ex_U=11.5, ex_smax=1.0e-20,
             iz_U=15.76, iz_smax=2.5e-20,
             cx_sigma=5.0e-19, opb_w=10.0)

_COMMON = dict(p_torr=1.0, Tg=300.0, Te0_eV=2.0, Ti0_K=300.0,
               wall_mode="fixed", nu_w=1.0e5, dt=1.0e-11, ion_subcycle=20,
               eps_cap=100.0, g_cap=1.0e4, energy_sharing="opb", poisson=1,
               sort_interval=20, capacity=1.25, emit_J=0.0, emit_T=0.5, circuit_R=0.0, seed=1)


def _mk(gas: dict, **kw) -> dict:
    c = dict(_COMMON)
    c.update(gas)
    c.update(kw)
    return c


# Radial loss frequency nu_w = (2.405 / R)^2 D_a of eq. (2), D_a = mu_i D_e / mu_e,
# for a 1 cm tube radius: D_e / mu_e from the two-term solution of the synthetic
# neon set at the column's E/N and mu_i N = 4e21 /(V m s); evaluated once and
# frozen here (tests/test_boltzmann_cpu.py recomputes them).
NU_W_NE_1TORR_10VCM = 6.05e4     # D_e / mu_e = 8.42 V
NU_W_NE_05TORR_10VCM = 1.43e5    # D_e / mu_e = 9.96 V


def small_bounded(seed: int = 1) -> dict:
    """Neon, 1 Torr, 4 cm, 400 cells, grounded cathode / 40 V anode (~10 V/cm),
    n0 = 1e14 m^-3, 50 particles per cell per species (20k + 20k), radial sink
    of eq. (2) for a 1 cm radius, dt = 1e-11 s, ions every 20 steps, 2000 steps."""
    return _mk(NEON, bc="bounded", n_cells=400, L=0.04, V=40.0, n0=1.0e14,
               ppc=50, nu_w=NU_W_NE_1TORR_10VCM, seed=seed)


def hot_cathode_15cm(seed: int = 1, ppc: int = 100) -> dict:
    """The bounded column of section V: neon, 1 Torr, 15 cm gap, source 270 V
    through a 10 ohm m^2 resistor, hot cathode emitting 10 A/m^2 (electrons at
    0.5 eV), fixed radial loss frequency 1e6 /s; 1500 cells, n0 = 1e15 m^-3
    (near the density the discharge settles at), 100 per cell per species
    (150k + 150k).  Ions cross the cathode sheath fast: g_cap 5e4 m/s with
    ions every 10 steps keeps their null-collision probability below 0.1."""
    return _mk(NEON, bc="bounded", n_cells=1500, L=0.15, V=270.0, n0=1.0e15, ppc=ppc,
               nu_w=1.0e6, emit_J=10.0, emit_T=0.5, circuit_R=10.0, capacity=3.0, g_cap=5.0e4,
               ion_subcycle=10, seed=seed)


def column_20cm(seed: int = 1, ppc: int = 200) -> dict:
    """Neon, 1 Torr, periodic 20 cm column, 2000 cells, 200 per cell per species
    (400k + 400k), E0 = 10 V/cm, n0 = 1e15 m^-3, radial sink of eq. (2)."""
    return _mk(NEON, bc="periodic", n_cells=2000, L=0.20, V=0.20 * 1000.0,
               n0=1.0e15, ppc=ppc, nu_w=NU_W_NE_1TORR_10VCM, seed=seed)


def column_50cm(seed: int = 1, ppc: int = 1000) -> dict:
    """Neon, 0.5 Torr, periodic 50 cm column, 5000 cells, 1000 per cell per
    species (5M + 5M), E0 = 10 V/cm, n0 = 1e15 m^-3, radial sink of eq. (2)."""
    return _mk(NEON, bc="periodic", n_cells=5000, L=0.50, V=0.50 * 1000.0,
               p_torr=0.5, n0=1.0e15, ppc=ppc, nu_w=NU_W_NE_05TORR_10VCM, seed=seed)


def argon_scan(n_columns: int = 64, seed: int = 1, precision: str = "fp32") -> list:
    """Parameter scan of uneven argon columns for one batched job: periodic
    columns of 5-40 cm at 50 um cells (1000-8000 cells), pressures 0.5-4 Torr
    log-uniform, imposed fields with E/p log-uniform over 2-20 V/(cm Torr)
    (a tenfold span of drift current at equal density), 100-400 particles per
    cell per species, n0 = 1e15 m^-3, Te0 = 2 eV.  The time step scales as
    1/p (2 ps at 1 Torr) so that every column has the same null-collision
    probability per step.  Radial sink: eq. (2) gives 0.9-6.9e4 /s over these
    columns (1 cm radius); all take its median, 3.2e4 /s.  Column c uses
    seed + c."""
    rng = np.random.default_rng(1000 + seed)
    cols = []
    for c in range(n_columns):
        cells = int(rng.integers(1000, 8001))
        L = cells * 50.0e-6
        p = float(np.exp(rng.uniform(np.log(0.5), np.log(4.0))))
        e_over_p = float(np.exp(rng.uniform(np.log(2.0), np.log(20.0))))   # V/(cm Torr)
        E0 = e_over_p * p * 100.0                                          # V/m
        ppc = int(rng.integers(100, 401))
        cols.append(_mk(ARGON, bc="periodic", n_cells=cells, L=L, V=E0 * L, p_torr=p,
                        n0=1.0e15, ppc=ppc, dt=2.0e-12 / p, precision=precision, nu_w=3.2e4,
                        seed=seed + c))
    return cols


def tiny(bc: str = "periodic", seed: int = 3, **kw) -> dict:
    """Small column for oracle pins and fast parity cases (several tiles, ragged)."""
    c = _mk(NEON, bc=bc, n_cells=kw.pop("n_cells", 37), L=kw.pop("L", 0.0037),
            V=kw.pop("V", 3.7), n0=kw.pop("n0", 1.0e14), ppc=kw.pop("ppc", 29),
            seed=seed)
    c.update(kw)
    return c


def with_(cfg: dict, **kw) -> dict:
    c = copy.deepcopy(cfg)
    c.update(kw)
    return c


def random_positions(n: int, L: float, seed: int) -> np.ndarray:
    """Uniform positions in [0, L) from a seeded numpy generator."""
    rng = np.random.default_rng(seed)
    x = rng.random(n) * L
    x[x >= L] = 0.0
    return x


def random_state(n: int, L: float, sigma_v: float, seed: int, id0: int = 0):
    """Seeded particle arrays (x, vx, vy, vz, id) for parity cases."""
    rng = np.random.default_rng(seed)
    x = rng.random(n) * L
    x[x >= L] = 0.0
    v = rng.normal(0.0, sigma_v, size=(3, n))
    ids = (np.arange(n, dtype=np.uint64) + id0).astype(np.uint32)
    perm = rng.permutation(n)
    return x[perm], v[0][perm].copy(), v[1][perm].copy(), v[2][perm].copy(), ids[perm]


def charge_profile(n_nodes: int, seed: int, scale: int = 1 << 36):
    """Seeded int64 fixed-point node charges for field-solve cases."""
    rng = np.random.default_rng(seed)
    re = rng.integers(0, scale, size=n_nodes, dtype=np.int64)
    ri = rng.integers(0, scale, size=n_nodes, dtype=np.int64)
    return re, ri


# ------------------------------------------------------------ fluid column
# Transport tables of the fluid model on a uniform temperature grid, columns
# (mu_e N, D_e N, mu_eps N, D_eps N, k_iz, L/N); see include/pc_fluid.h.
FLUID_T_MIN, FLUID_T_STEP, FLUID_T_LEN = 0.5, 0.125, 120   # 0.5 .. 15.375 eV


def fluid_table_flat(Ngas: float = 3.2e22, nu_w: float = 1.0e5, D_eps_ratio: float = 1.0):
    """Temperature-independent coefficients (closed-form checks): mu_e N =
    1e24, D_e N = 3e24, mu_eps N = 5/3 mu_e N, D_eps N = D_eps_ratio 5/3 D_e N,
    k_iz = nu_w / Ngas, L / N = 4e-15."""
    t = np.empty((FLUID_T_LEN, 6))
    t[:, 0] = 1.0e24
    t[:, 1] = 3.0e24
    t[:, 2] = 5.0 / 3.0 * 1.0e24
    t[:, 3] = D_eps_ratio * 5.0 / 3.0 * 3.0e24
    t[:, 4] = nu_w / Ngas
    t[:, 5] = 4.0e-15
    return t


def fluid_table_ne():
    """Two-term table of the synthetic neon cross sections (the striated
    column's gas) on the fluid grid, written by make_fluid_table.py (E/N
    0.1-300 Td; below the lowest solved temperature, 0.87 eV, the first
    solved row)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "fluid_table_ne_1torr.json")) as f:
        d = json.load(f)
    assert d["T_min"] == FLUID_T_MIN and d["T_step"] == FLUID_T_STEP
    return np.asarray(d["table"], dtype=np.float64)


def fluid_table_smooth():
    """Smooth synthetic temperature dependence of the right orders of magnitude
    for a rare gas (mobility falling and diffusion rising with T, Arrhenius
    ionisation, D_eps below 5/3 D_e so that the chi coefficient is negative)."""
    T = FLUID_T_MIN + FLUID_T_STEP * np.arange(FLUID_T_LEN)
    t = np.empty((FLUID_T_LEN, 6))
    t[:, 0] = 1.2e24 / (1.0 + 0.08 * T)
    t[:, 1] = t[:, 0] * T * (1.0 + 0.15 * np.tanh((T - 4.0) / 2.0))
    t[:, 2] = 5.0 / 3.0 * t[:, 0] * (1.0 - 0.05 * np.tanh((T - 5.0) / 3.0))
    t[:, 3] = 0.9 * 5.0 / 3.0 * t[:, 1]
    t[:, 4] = 2.0e-13 * np.exp(-18.0 / T)
    t[:, 5] = 2.0e-14 * np.exp(-9.0 / T) + 1.0e-16 * T
    return t
