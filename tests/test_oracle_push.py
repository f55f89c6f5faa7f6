"""Pins of the oracle's gather + leapfrog push and its coupling to deposit and
Poisson (paper section II: trajectories under the self-consistent field,
standard electrostatic PIC after Birdsall and Langdon).

- free flight: x_n = x_0 + n v dt, wrapped into [0, L);
- uniform field: leapfrog started with the half-step velocity is exact for
  constant acceleration, x_n = x_0 + v_0 t_n + a t_n^2 / 2;
- cold plasma oscillation of a long-wavelength mode: leapfrog dispersion
  sin(w dt / 2) = w_pe dt / 2.
"""
import numpy as np
import pytest

import workloads as W
from oracle.pco import Oracle, ELECTRON, ION

QE = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12

NO_COLL = dict(el_A=0.0, el_B=0.0, ex_smax=0.0, iz_smax=0.0, cx_sigma=0.0, wall_mode="off")


def test_free_flight_periodic_wrap():
    L = 0.0037
    cfg = W.tiny("periodic", V=0.0, poisson=0, Te0_eV=2.0, **NO_COLL)
    o = Oracle(cfg)
    x0, vx0, vy0, vz0, ids = o.state(ELECTRON)
    n = 57
    o.step(n)
    x, vx, vy, vz, ids2 = o.state(ELECTRON)
    assert np.array_equal(ids, ids2)
    assert np.array_equal(vx, vx0) and np.array_equal(vy, vy0) and np.array_equal(vz, vz0)
    ref = np.mod(x0 + n * vx0 * 1e-11, L)
    d = np.abs(x - ref)
    d = np.minimum(d, L - d)
    assert d.max() <= 1e-12 * L


def test_uniform_field_leapfrog_is_exact():
    # electrons and ions in the imposed field only; wide column so nothing wraps
    E0 = 500.0
    L = 40.0
    cfg = W.tiny("periodic", n_cells=40, L=L, V=E0 * L, poisson=0, ppc=20,
                 Te0_eV=0.05, Ti0_K=300.0, n0=1e6, **NO_COLL)
    o = Oracle(cfg, init=False)
    rng = np.random.default_rng(4)
    n = 600
    x0 = 15.0 + 10.0 * rng.random(n)
    v0 = rng.normal(0.0, 1e5, n)
    a = -QE * (-E0) / ME          # electron acceleration in E = -E0 (towards +x)
    dt = 1e-11
    vhalf = v0 - a * dt / 2       # leapfrog start
    o.set_state(ELECTRON, x0, vhalf, np.zeros(n), np.zeros(n), np.arange(n, dtype=np.uint32))
    o.set_state(ION, x0[:1], np.zeros(1), np.zeros(1), np.zeros(1), np.zeros(1, dtype=np.uint32))
    o.set_counters(1, n, 1)       # start at a non-ion step
    E = np.full(o.nn, -E0)
    o.set_field(E)
    steps = 300
    o.step(steps)
    x, vx, *_ , ids = o.state(ELECTRON)
    order = np.argsort(ids)
    t = steps * dt
    ref = x0 + v0 * t + 0.5 * a * t * t
    assert np.abs(x[order] - ref).max() <= 1e-12 * L
    vref = v0 + a * (t - dt / 2)
    assert np.abs(vx[order] - vref).max() <= 1e-9 * np.abs(vref).max()


def test_cold_plasma_oscillation_frequency():
    # quiet start: ions and electrons on the same uniform lattice, electrons
    # displaced by d cos(kx); the mode oscillates at w with
    # sin(w dt/2) = w_pe dt/2 (long wavelength: k dx = 2 pi / 64)
    nc, L = 64, 0.0064
    ppc = 32
    n0 = 1e14
    dt = 1e-10
    cfg = W.tiny("periodic", n_cells=nc, L=L, V=0.0, ppc=ppc, n0=n0, dt=dt,
                 ion_subcycle=1_000_000, **NO_COLL)
    cfg["M_amu"] = 1.0e9          # immobile ions
    o = Oracle(cfg, init=False)
    n = nc * ppc
    xi = (np.arange(n) + 0.5) * (L / n)
    k = 2 * np.pi / L
    d = 1e-6
    xe = np.mod(xi + d * np.cos(k * xi), L)
    z = np.zeros(n)
    ids = np.arange(n, dtype=np.uint32)
    o.set_state(ION, xi, z, z, z, ids)
    o.set_state(ELECTRON, xe, z, z, z, ids)
    o.set_counters(1, n, n)
    # field of the displaced state (self-consistent start, v^{-1/2} = 0 is
    # the turning point to O(dt^2))
    re = o.deposit(xe)
    ri = o.deposit(xi)
    _, E = o.solve_field(re, ri)
    o.set_field(E)
    wpe = np.sqrt(n0 * QE * QE / (EPS0 * ME))
    w = 2.0 / dt * np.arcsin(wpe * dt / 2)
    T = 2 * np.pi / w
    nsteps = int(3.2 * T / dt)
    amp = []
    for _ in range(nsteps):
        o.step(1)
        x, *_ , idd = o.state(ELECTRON)
        xs = x[np.argsort(idd)]
        disp = (xs - xi + L / 2) % L - L / 2
        amp.append(2.0 / n * np.sum(disp * np.cos(k * xi)))
    amp = np.array(amp)
    # zero crossings -> half periods
    s = np.sign(amp)
    idx = np.where(s[:-1] * s[1:] < 0)[0]
    tc = []
    for i in idx:
        f = amp[i] / (amp[i] - amp[i + 1])
        tc.append((i + 1 + f) * dt)
    tc = np.array(tc)
    half = np.diff(tc).mean()
    w_meas = np.pi / half
    # finite k dx lowers the CIC grid response slightly (Birdsall & Langdon)
    assert abs(w_meas / w - 1) < 5e-3
    assert np.abs(amp).max() < 1.5 * d
