"""Host-side analysis of column moments (the diagnostics of section III).

Inputs are the integer cell moments written by pc_moments (layout in
include/pc.h); outputs are physical profiles and striation properties:

- densities n_e, n_i per cell and mean energy / T_e = (2/3) mean energy
  (section II: the electron "temperature" is 2/3 of the mean energy);
- EEPF F(eps) = f(eps) / sqrt(eps), normalised so that the integral of
  eps^(1/2) F over energy is 1 (section III.C);
- striation wavelength lambda = L / m* from the dominant Fourier mode of the
  time-averaged electron density, its phase velocity from the phase of that
  mode between snapshots (section III.D: waves move towards the cathode, i.e.
  negative velocity), and the potential drop per striation delta_phi =
  E0 * lambda (eq. (1)).
"""
from __future__ import annotations

import numpy as np

EEPF_BINS = 240
EEPF_DE = 0.25          # eV per bin
EPS_SCALE = 2.0 ** 20   # fixed-point scale of the energy sums (eV)
V_SCALE = 2.0 ** 10     # fixed-point scale of the velocity sums (m/s)


def split(mom: np.ndarray, n_cells: int, cells_per_group: int = 1) -> dict:
    """Split the flat int64 moments vector into named blocks."""
    nc = n_cells
    ng = (nc + cells_per_group - 1) // cells_per_group
    m = np.asarray(mom, dtype=np.int64)
    if m.size != 7 * nc + ng * EEPF_BINS:
        raise ValueError("moments vector has the wrong length")
    return {
        "ne": m[0:nc], "eps": m[nc:2 * nc], "vx": m[2 * nc:3 * nc], "epsvx": m[3 * nc:4 * nc],
        "ni": m[4 * nc:5 * nc], "vxi": m[5 * nc:6 * nc], "iz": m[6 * nc:7 * nc],
        "eepf": m[7 * nc:].reshape(ng, EEPF_BINS),
    }


def densities(parts: dict, weight: float, dx: float):
    """Cell densities [m^-3] from macroparticle counts (weight = real
    particles per m^2 per macroparticle)."""
    return parts["ne"] * weight / dx, parts["ni"] * weight / dx


def mean_energy(parts: dict) -> np.ndarray:
    """Mean electron energy per cell [eV] (NaN in empty cells)."""
    n = parts["ne"].astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        return parts["eps"] / EPS_SCALE / n


def electron_temperature(parts: dict) -> np.ndarray:
    return 2.0 / 3.0 * mean_energy(parts)


def eepf(counts: np.ndarray, de: float = EEPF_DE):
    """Normalised EEPF of histogram counts on bins [k de, (k+1) de):
    returns (bin centres, F) with sum(sqrt(eps) F de) = 1."""
    c = np.asarray(counts, dtype=np.float64)
    eps = (np.arange(c.size) + 0.5) * de
    tot = c.sum()
    if tot <= 0:
        return eps, np.zeros_like(c)
    f = c / (tot * de)                 # EEDF: integral f deps = 1
    return eps, f / np.sqrt(eps)


def dominant_mode(profile: np.ndarray) -> int:
    """Index m* >= 1 of the largest Fourier amplitude of a periodic profile."""
    p = np.asarray(profile, dtype=np.float64)
    spec = np.abs(np.fft.rfft(p - p.mean()))
    spec[0] = 0.0
    return int(np.argmax(spec))


def wavelength(profile: np.ndarray, L: float) -> float:
    """Striation wavelength L / m* of a periodic profile on [0, L)."""
    return L / dominant_mode(profile)


def dominant_mode_of_snapshots(snapshots: np.ndarray) -> int:
    """Mode with the largest time-averaged Fourier amplitude of snapshots[t, x]
    (moving striations wash out of a time-averaged profile, not of its
    amplitude spectrum)."""
    s = np.asarray(snapshots, dtype=np.float64)
    spec = np.abs(np.fft.rfft(s - s.mean(axis=1, keepdims=True), axis=1)).mean(axis=0)
    spec[0] = 0.0
    return int(np.argmax(spec))


def phase_velocity(snapshots: np.ndarray, times: np.ndarray, L: float, m: int | None = None) -> float:
    """Phase velocity of mode m (default: the dominant mode of the snapshots)
    from snapshots[t, x]: least-squares slope of the unwrapped phase, divided
    by the wave number.  For n ~ cos(k x - k v t) the forward transform's
    coefficient of mode m has phase -k v t, so v = -d(phase)/dt / k."""
    s = np.asarray(snapshots, dtype=np.float64)
    if m is None:
        m = dominant_mode_of_snapshots(s)
    k = 2.0 * np.pi * m / L
    ph = np.unwrap(np.angle(np.fft.rfft(s - s.mean(axis=1, keepdims=True), axis=1)[:, m]))
    t = np.asarray(times, dtype=np.float64)
    slope = np.polyfit(t, ph, 1)[0]
    return -slope / k


def potential_drop_per_striation(E0: float, lam: float) -> float:
    """Eq. (1): the potential drop over one striation is E0 * lambda."""
    return E0 * lam


def mode_amplitudes(coef: np.ndarray) -> np.ndarray:
    """Relative amplitudes 2 |c_m| / c_0 of modes m >= 1 from Fourier
    coefficients coef[t, m] of cell counts (c_0 = the total count)."""
    c = np.asarray(coef)
    return 2.0 * np.abs(c[:, 1:]) / c[:, 0].real[:, None]


def striation_statistics(coef: np.ndarray, times: np.ndarray, L: float, t_from: float,
                         lo: float = 1e-2, hi: float = 1e-1, onset: float = 0.1, nprof: int = 32) -> dict:
    """Statistics of a free run from the Fourier coefficients coef[t, m]
    (m = 0..M) of its electron cell counts at `times`:

    - mode: the dominant mode over t >= t_from (largest mean amplitude),
      wavelength L / mode (section III) and its mean relative amplitude
      (modulation);
    - first: the first mode whose amplitude exceeds `onset`, the onset time,
      and its linear growth rate (slope of ln amplitude while it lies in
      (lo, hi));
    - phase velocity of the dominant mode over t >= t_from (negative: towards
      the cathode, x = 0 being the cathode side of the imposed field);
    - profile: the time-averaged density over one wavelength in the frame of
      the wave (harmonics h * mode <= M, each rotated by h times the phase of
      the dominant mode, averaged, summed), relative to the mean, on nprof
      points."""
    c = np.asarray(coef)
    t = np.asarray(times, dtype=np.float64)
    A = mode_amplitudes(c)
    sel = t >= t_from
    m = int(np.argmax(A[sel].mean(axis=0))) + 1
    over = np.argwhere(A > onset)
    first, t_on, growth = -1, float("nan"), float("nan")
    if over.size:
        k0 = over[0, 0]
        cand = over[over[:, 0] == k0][:, 1]
        first = int(cand[np.argmax(A[k0, cand])]) + 1
        t_on = float(t[k0])
        a = A[:, first - 1]
        g = (a > lo) & (a < hi) & (t <= t_on)
        if g.sum() >= 3:
            growth = float(np.polyfit(t[g], np.log(a[g]), 1)[0])
    k = 2.0 * np.pi * m / L
    ph = np.unwrap(np.angle(c[sel, m]))
    vph = float(-np.polyfit(t[sel], ph, 1)[0] / k)
    M = c.shape[1] - 1
    theta = np.angle(c[sel, m])
    xs = (np.arange(nprof) + 0.5) / nprof
    prof = np.zeros(nprof)
    n0 = c[sel, 0].real.mean()
    for h in range(1, M // m + 1):
        ch = (c[sel, h * m] * np.exp(-1j * h * theta)).mean()
        prof += 2.0 * np.real(ch * np.exp(2j * np.pi * h * xs)) / n0
    return dict(mode=m, wavelength=L / m, modulation=float(A[sel, m - 1].mean()), first=first, onset=t_on,
                growth=growth, phase_velocity=vph, profile=prof)
