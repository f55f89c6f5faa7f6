"""Pins of the host analysis (section III diagnostics) on synthetic profiles
with known answers."""
import math

import numpy as np

from paper_2202_03215_amd import analysis as A


def test_wavelength_of_a_pure_mode():
    L = 0.2
    x = (np.arange(2000) + 0.5) * L / 2000
    for m in (1, 7, 13):
        prof = 1e15 * (1 + 0.3 * np.sin(2 * np.pi * m * x / L + 0.4))
        assert A.dominant_mode(prof) == m
        assert abs(A.wavelength(prof, L) - L / m) < 1e-15


def test_phase_velocity_of_a_travelling_wave():
    L, m = 0.1, 5
    x = (np.arange(1000) + 0.5) * L / 1000
    v = -700.0                              # towards the cathode
    t = np.linspace(0.0, 2e-5, 41)          # less than half a period between samples
    snaps = np.array([1 + 0.5 * np.cos(2 * np.pi * m * (x - v * tt) / L) for tt in t])
    assert abs(A.phase_velocity(snaps, t, L) / v - 1) < 1e-9
    assert A.dominant_mode_of_snapshots(snaps) == m
    # over many periods the mean profile is flat but the mean spectrum is not
    t2 = np.linspace(0.0, 1e-3, 400)
    s2 = np.array([1 + 0.5 * np.cos(2 * np.pi * m * (x - v * tt) / L) for tt in t2])
    assert A.dominant_mode_of_snapshots(s2) == m
    # frequency identity of section III.D: F = v / lambda
    assert abs(abs(v) / (L / m) - 35000.0) < 1e-6


def test_potential_drop_eq1():
    # 6 V/cm and 2 cm give 12 V (the section III.C/D example)
    assert abs(A.potential_drop_per_striation(600.0, 0.02) - 12.0) < 1e-12


def test_eepf_of_a_maxwellian_histogram():
    # f(eps) = 2 sqrt(eps/pi) T^-3/2 exp(-eps/T): F = f / sqrt(eps) is
    # exp(-eps/T) times a constant, so ln F is linear with slope -1/T
    T = 3.0
    de = A.EEPF_DE
    edges = np.arange(A.EEPF_BINS + 1) * de
    from scipy.special import gammainc
    cdf = gammainc(1.5, edges / T)
    counts = np.round(1e12 * np.diff(cdf))
    eps, F = A.eepf(counts, de)
    assert abs(np.sum(np.sqrt(eps) * F * de) - 1) < 1e-12
    sel = (eps > 1) & (eps < 20)
    slope = np.polyfit(eps[sel], np.log(F[sel]), 1)[0]
    assert abs(slope * T + 1) < 2e-3


def test_moment_blocks_and_temperature():
    nc, cpg = 10, 5
    ng = 2
    m = np.zeros(7 * nc + ng * 240, dtype=np.int64)
    m[:nc] = 100
    m[nc:2 * nc] = int(100 * 4.5 * A.EPS_SCALE)
    p = A.split(m, nc, cpg)
    assert np.allclose(A.mean_energy(p), 4.5)
    assert np.allclose(A.electron_temperature(p), 3.0)
    ne, ni = A.densities(p, weight=2e8, dx=1e-4)
    assert np.allclose(ne, 100 * 2e8 / 1e-4)
