"""Pins of the oracle's moments accumulator (the diagnostics of section III:
densities, mean energy and T_e = 2/3 of it (section II), particle and energy
fluxes, ionization counts, and the EEPF histogram normalised as in
section III.C).

Every case places particles by hand -- chosen cells, chosen energies and
velocities -- so the expected integers are known by construction, not by
repeating the accumulator's arithmetic: e.g. seven electrons of 5.3 eV in
cell 3 must add 7 * floor(5.3 * 2^20) to the energy slot of cell 3 and seven
counts to EEPF bin 21 (0.25 eV bins) of the group holding cell 3.  Energies
are chosen away from the truncation boundaries of every fixed-point scale,
velocities of both signs check truncation towards zero, and each case is
built so that a wrong scale (2^20, 2^10, 2^4), bin width, group index
(cell // cells_per_group), species slot or sign fails it.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle.pco import Oracle, ELECTRON, ION

QE = 1.602176634e-19
ME = 9.1093837015e-31
C_EPS = 0.5 * ME / QE           # eV per (m/s)^2 of an electron


def _column(n_cells=40, L=0.004):
    cfg = W.tiny("periodic", n_cells=n_cells, L=L, V=0.0, ppc=1, wall_mode="off")
    return cfg, Oracle(cfg, init=False)


def _put(o, species, xs, vxs, vys=None, vzs=None, id0=0):
    n = len(xs)
    z = np.zeros(n)
    vy = z if vys is None else np.asarray(vys, dtype=np.float64)
    vz = z if vzs is None else np.asarray(vzs, dtype=np.float64)
    o.set_state(species, np.asarray(xs, dtype=np.float64), np.asarray(vxs, dtype=np.float64), vy, vz,
                np.arange(id0, id0 + n, dtype=np.uint32))


def _blocks(mom, nc, cpg):
    ng = (nc + cpg - 1) // cpg
    assert mom.size == 7 * nc + 240 * ng
    return [mom[k * nc:(k + 1) * nc] for k in range(7)] + [mom[7 * nc:].reshape(ng, 240)]


def _cell_centre(cfg, j):
    return (j + 0.5) * cfg["L"] / cfg["n_cells"]


def test_single_cell_monoenergetic_electrons():
    cfg, o = _column()
    nc = cfg["n_cells"]
    # 5.3 eV along +x: 5.3 * 2^20 = 5557452.8, so each electron adds 5557452
    v = math.sqrt(5.3 / C_EPS)                   # 1.3654e6 m/s
    _put(o, ELECTRON, [_cell_centre(cfg, 3)] * 7, [v] * 7)
    _put(o, ION, [], [])
    cnt, eps, vx, epsvx, ni, vxi, iz, eepf = _blocks(o.moments(1), nc, 1)
    assert cnt[3] == 7 and cnt.sum() == 7
    assert eps[3] == 7 * 5557452 and eps.sum() == eps[3]
    assert vx[3] == 7 * math.floor(v * 1024.0) and vx.sum() == vx[3]
    assert epsvx[3] == 7 * math.floor(5.3 * v * 16.0)
    assert ni.sum() == 0 and vxi.sum() == 0 and iz.sum() == 0
    assert eepf[3, 21] == 7 and eepf.sum() == 7           # 5.3 eV / 0.25 eV = 21.2


def test_negative_velocity_truncates_towards_zero():
    cfg, o = _column()
    nc = cfg["n_cells"]
    # the same 5.3 eV electron moving along -x: -1398205.6 -> -1398205 (not -1398206)
    v = math.sqrt(5.3 / C_EPS)
    _put(o, ELECTRON, [_cell_centre(cfg, 11)], [-v])
    _put(o, ION, [_cell_centre(cfg, 11)], [-123.4567])
    cnt, eps, vx, epsvx, ni, vxi, iz, eepf = _blocks(o.moments(1), nc, 1)
    assert vx[11] == -math.floor(v * 1024.0)
    assert epsvx[11] == -math.floor(5.3 * v * 16.0)
    assert eps[11] == 5557452                              # energy does not depend on the sign
    assert ni[11] == 1 and vxi[11] == -126419              # -123.4567 * 1024 = -126419.66


def test_energy_from_all_three_components():
    cfg, o = _column()
    nc = cfg["n_cells"]
    # 2 + 3 + 4.7 eV in x, y, z: 9.7 eV in total (bin 38), flux from v_x only
    vx, vy, vz = (math.sqrt(e / C_EPS) for e in (2.0, 3.0, 4.7))
    _put(o, ELECTRON, [_cell_centre(cfg, 0)], [vx], [vy], [-vz])
    _put(o, ION, [], [])
    cnt, eps, svx, epsvx, *_, eepf = _blocks(o.moments(1), nc, 1)
    assert eps[0] == math.floor(9.7 * 2 ** 20)             # 10171187.2
    assert svx[0] == math.floor(vx * 1024.0)
    assert epsvx[0] == math.floor(9.7 * vx * 16.0)
    assert eepf[0, 38] == 1


@pytest.mark.parametrize("cpg", [1, 4, 7, 40])
def test_eepf_bins_and_cell_groups(cpg):
    cfg, o = _column()
    nc = cfg["n_cells"]
    # (cell, energy [eV], expected bin): bin edges every 0.25 eV on [0, 60)
    cases = [(0, 0.1, 0), (0, 0.3, 1), (5, 1.12, 4), (6, 1.13, 4), (13, 7.9, 31), (27, 30.05, 120),
             (39, 59.9, 239), (39, 12.6, 50), (20, 61.3, None), (21, 75.0, None)]
    xs = [_cell_centre(cfg, j) for j, _, _ in cases]
    vs = [math.sqrt(e / C_EPS) for _, e, _ in cases]
    _put(o, ELECTRON, xs, vs)
    _put(o, ION, [], [])
    cnt, eps, *_, eepf = _blocks(o.moments(cpg), nc, cpg)
    ng = (nc + cpg - 1) // cpg
    want = np.zeros((ng, 240), dtype=np.int64)
    for j, _, b in cases:
        if b is not None:
            want[j // cpg, b] += 1
    assert np.array_equal(eepf, want)
    # energies above 60 eV leave the histogram but stay in the counts and sums
    assert cnt[20] == 1 and eps[20] == math.floor(61.3 * 2 ** 20)
    assert cnt.sum() == len(cases)


def test_species_slots_and_cells_at_the_edges():
    cfg, o = _column()
    nc, dx = cfg["n_cells"], cfg["L"] / cfg["n_cells"]
    # electrons at the very start of cells 0 and 39 and just below L; ions elsewhere
    _put(o, ELECTRON, [0.0, 39.001 * dx, cfg["L"] * (1 - 1e-12)], [10.0, 20.0, 30.0])
    _put(o, ION, [5.5 * dx, 5.5 * dx, 17.25 * dx], [1.0, 2.0, 3.0], id0=100)
    cnt, eps, vx, epsvx, ni, vxi, iz, eepf = _blocks(o.moments(1), nc, 1)
    assert cnt[0] == 1 and cnt[39] == 2 and cnt.sum() == 3
    assert vx[0] == 10240 and vx[39] == 20480 + 30720
    assert ni[5] == 2 and ni[17] == 1 and ni.sum() == 3
    assert vxi[5] == 1024 + 2048 and vxi[17] == 3072
    assert eps.sum() == 0                                # 10-30 m/s: below 2^-20 eV each
    assert eepf[0, 0] == 1 and eepf[39, 0] == 2


def test_mean_energy_temperature_and_eepf_normalisation():
    """Host analysis on pinned moments: T_e = 2/3 of the mean energy
    (section II) and the EEPF integral of eps^(1/2) F over energy equal to 1
    (section III.C), for a constructed two-energy population."""
    from paper_2202_03215_amd import analysis as A
    cfg, o = _column()
    nc = cfg["n_cells"]
    e1, e2 = 3.3, 8.8
    xs = [_cell_centre(cfg, 9)] * 12
    vs = [math.sqrt(e1 / C_EPS)] * 4 + [math.sqrt(e2 / C_EPS)] * 8
    _put(o, ELECTRON, xs, vs)
    _put(o, ION, [], [])
    mom = o.moments(nc)
    parts = A.split(mom, nc, nc)
    mean = (4 * e1 + 8 * e2) / 12
    assert abs(A.mean_energy(parts)[9] - mean) < 2e-6
    assert abs(A.electron_temperature(parts)[9] - 2.0 / 3.0 * mean) < 2e-6
    e, F = A.eepf(parts["eepf"][0])
    assert abs(np.sum(np.sqrt(e) * F) * A.EEPF_DE - 1.0) < 1e-12
    # the two populations sit in bins 13 (3.3 eV) and 35 (8.8 eV) with weights 1/3, 2/3
    f = np.sqrt(e) * F * A.EEPF_DE
    assert abs(f[13] - 1.0 / 3.0) < 1e-12 and abs(f[35] - 2.0 / 3.0) < 1e-12


def test_ionization_counts_accumulate_and_reset():
    cfg = W.tiny("periodic", V=0.0037 * 8000.0, wall_mode="off", ppc=60, eps_cap=100.0)
    o = Oracle(cfg)
    nc = cfg["n_cells"]
    tot = 0
    for _ in range(3):
        o.step(40)
        iz = o.moments(1)[6 * nc:7 * nc]
        assert iz.sum() >= tot
        tot = iz.sum()
    assert tot > 0
    assert o.moments(1, reset_iz=True)[6 * nc:7 * nc].sum() == tot
    assert o.moments(1)[6 * nc:7 * nc].sum() == 0
