"""Linear stability of the homogeneous quasi-neutral column (section IV.F).

Small perturbations (dn, dT) ~ exp(-i Omega t + i k x), Omega = omega + i
gamma, of the steady homogeneous state (n0, T0, E0) of the fluid equations
(3)-(4), with the fluxes (12)-(13) and the field (17), obey the 2x2 system
(18).  Setting its determinant to zero gives the angular frequency (19) and
the growth rate (20); the maximum of (20) over k is (21) at the wave number
(22), with

    alpha = chi nu_i' / (D_a K),  beta = L' / K,  delta = 2 L nu_i' / (D_a K),

K = kappa / n0; the column is unstable iff (23) holds, i.e. iff gamma_max > 0.
The phase velocity at the maximum growth rate is omega(k_max) / k_max.

Coefficients at T0 come from a transport table in the fluid kernels' layout
(columns mu_e N, D_e N, mu_eps N, D_eps N, k_iz, L/N on a uniform T grid,
include/pc_fluid.h), evaluated as the fluid kernels evaluate them: linear
interpolation, d/dT from the slope of the same segment.  Eq. (9) is read as
beta_e = 3/2 T mu_eps and G_e = 3/2 T D_eps; kappa (15) and chi (16) follow;
D_a = mu_i D_e / mu_e; nu_i = N k_iz; the steady field balances heating and
loss, mu_e E0^2 = L (eq. (5) with the drift flux).

Sign convention: the fluid one (E0 > 0 along +x, electrons drifting to -x);
omega / k > 0 is a wave moving against the electron drift, towards the
cathode, as the striations of section III.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Coefficients:
    T0: float        # electron temperature [eV]
    E0: float        # steady field [V/m]
    mu_e: float      # electron mobility [m^2/(V s)]
    D_e: float       # electron diffusion [m^2/s]
    D_a: float       # ambipolar diffusion mu_i D_e / mu_e [m^2/s]
    chi: float       # eq. (16) [eV m^2/s]
    K: float         # kappa / n0, eq. (15) [m^2/s]
    nu_p: float      # d nu_i / dT [1/(s eV)]
    L: float         # energy loss rate per electron [eV/s]
    L_p: float       # dL / dT [1/s]


def _row(table: np.ndarray, T_min: float, T_step: float, T: float):
    K = table.shape[0]
    u = (min(max(T, T_min), T_min + (K - 1) * T_step) - T_min) / T_step
    k = min(int(np.floor(u)), K - 2)
    f = u - k
    lo, hi = table[k], table[k + 1]
    return lo + f * (hi - lo), (hi - lo) / T_step


def coefficients(table, T_min: float, T_step: float, Ngas: float, muiN: float, T0: float) -> Coefficients:
    """Coefficients of eqs. (18)-(23) at T0."""
    table = np.asarray(table, dtype=np.float64)
    v, s = _row(table, T_min, T_step, T0)
    N = Ngas
    mu, D, mu_eps, D_eps = v[0] / N, v[1] / N, v[2] / N, v[3] / N
    dD, dD_eps = s[1] / N, s[3] / N
    beta = 1.5 * T0 * mu_eps
    G = 1.5 * T0 * D_eps
    dG = 1.5 * D_eps + 1.5 * T0 * dD_eps
    L = N * v[5]
    return Coefficients(T0=T0, E0=float(np.sqrt(L / mu)), mu_e=mu, D_e=D, D_a=(muiN / N) * D / mu,
                        chi=G - beta / mu * D, K=dG - beta / mu * dD, nu_p=N * s[4], L=L, L_p=N * s[5])


def frequency(k, c: Coefficients):
    """Eq. (19)."""
    k = np.asarray(k, dtype=np.float64)
    return k * c.nu_p * c.E0 * c.D_e / (k * k * c.K + c.L_p)


def growth(k, c: Coefficients):
    """Eq. (20)."""
    k = np.asarray(k, dtype=np.float64)
    return -c.D_a * k * k - c.nu_p * (2.0 * c.L + c.chi * k * k) / (k * k * c.K + c.L_p)


def maximum(c: Coefficients) -> dict:
    """Eqs. (21)-(23): gamma_max, k_max, the instability condition, and the
    phase velocity omega(k_max) / k_max.  Without an interior maximum (k_max^2
    of eq. (22) not positive) gamma decreases from k = 0: then k_max is nan
    and gamma_max is gamma(0) = -2 L nu_i' / L'."""
    alpha = c.chi * c.nu_p / (c.D_a * c.K)
    beta = c.L_p / c.K
    delta = 2.0 * c.L * c.nu_p / (c.D_a * c.K)
    root = np.sqrt(delta - alpha * beta) if delta - alpha * beta >= 0.0 else np.nan
    k2 = -beta + root
    if k2 > 0.0:
        k_max = float(np.sqrt(k2))
        g_max = c.D_a * (beta - alpha - 2.0 * root)
    else:
        k_max = np.nan
        g_max = float(growth(0.0, c))
    bound = -(c.D_a * c.L_p + np.sqrt(8.0 * c.D_a * c.K * c.L * c.nu_p)) / c.nu_p
    return dict(alpha=alpha, beta=beta, delta=delta, gamma_max=float(g_max), k_max=k_max,
                wavelength=2.0 * np.pi / k_max if k_max == k_max else np.nan,
                unstable=bool(c.chi < bound), chi_bound=float(bound),
                v_ph=float(frequency(k_max, c) / k_max) if k_max == k_max else np.nan)


def _bisect(f, lo: float, hi: float) -> float:
    flo = f(lo)
    if flo * f(hi) > 0:
        raise ValueError("no root in the tabulated temperature range")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        fm = f(mid)
        if flo * fm <= 0:
            hi = mid
        else:
            lo, flo = mid, fm
    return 0.5 * (lo + hi)


def temperature_for_loss(table, T_min: float, T_step: float, Ngas: float, nu_w: float) -> float:
    """T0 with nu_i(T0) = nu_w (the homogeneous steady state of section IV)."""
    table = np.asarray(table, dtype=np.float64)
    hi = T_min + (table.shape[0] - 1) * T_step
    return _bisect(lambda T: Ngas * _row(table, T_min, T_step, T)[0][4] - nu_w, T_min, hi)


def temperature_for_field(table, T_min: float, T_step: float, Ngas: float, E0: float) -> float:
    """T0 whose balancing field sqrt(L / mu_e) equals E0 (the paper's control
    parameter E0 / p)."""
    table = np.asarray(table, dtype=np.float64)
    hi = T_min + (table.shape[0] - 1) * T_step

    def f(T):
        v, _ = _row(table, T_min, T_step, T)
        return np.sqrt((Ngas * v[5]) / (v[0] / Ngas)) - E0
    return _bisect(f, T_min, hi)


def scan(table, T_min: float, T_step: float, Ngas: float, muiN: float, E0_values) -> dict:
    """gamma_max, lambda = 2 pi / k_max and v_ph against the mean field (the
    fluid-model curves of Figs. 14, 15 and 17)."""
    rows = []
    for E0 in E0_values:
        T0 = temperature_for_field(table, T_min, T_step, Ngas, float(E0))
        m = maximum(coefficients(table, T_min, T_step, Ngas, muiN, T0))
        rows.append((float(E0), T0, m["gamma_max"], m["wavelength"], m["v_ph"], m["unstable"]))
    a = np.array(rows, dtype=np.float64)
    return dict(E0=a[:, 0], T0=a[:, 1], gamma_max=a[:, 2], wavelength=a[:, 3], v_ph=a[:, 4],
                unstable=a[:, 5].astype(bool))


def threshold(table, T_min: float, T_step: float, Ngas: float, muiN: float, E_lo: float, E_hi: float) -> float:
    """Mean field [V/m] at which gamma_max changes sign (bisection between a
    stable E_lo and an unstable E_hi)."""
    def g(E0):
        T0 = temperature_for_field(table, T_min, T_step, Ngas, E0)
        return maximum(coefficients(table, T_min, T_step, Ngas, muiN, T0))["gamma_max"]
    return _bisect(g, E_lo, E_hi)


def main(argv=None) -> int:
    """python -m paper_2202_03215_amd.stability [--gas neon|argon] [--muiN X]
    Fluid-model predictions against E0/p at 1 Torr, 300 K (gamma_max,
    lambda = 2 pi / k_max, v_ph) from two-term tables of the synthetic cross
    sections, and the instability threshold."""
    import argparse
    import json
    import workloads as W
    from . import closure as CL
    ap = argparse.ArgumentParser()
    ap.add_argument("--gas", default="neon", choices=["neon", "argon"])
    ap.add_argument("--muiN", type=float, default=4.0e21)
    a = ap.parse_args(argv)
    cfg = W.column_20cm() if a.gas == "neon" else W.argon_scan(1)[0]
    Ngas = 133.322368 / (1.380649e-23 * 300.0)
    T, cols = CL.transport_table(cfg, np.geomspace(2e-21, 4e-19, 80), Ngas)
    tab = CL.resample_uniform(T, cols, W.FLUID_T_MIN, W.FLUID_T_STEP, W.FLUID_T_LEN)
    E = np.array([1.0, 1.5, 2.0, 3.0, 5.0, 7.5, 10.0, 15.0, 20.0, 30.0]) * 100.0
    out = scan(tab, W.FLUID_T_MIN, W.FLUID_T_STEP, Ngas, a.muiN, E)
    stable = E[~out["unstable"]]
    unstable = E[out["unstable"]]
    thr = (threshold(tab, W.FLUID_T_MIN, W.FLUID_T_STEP, Ngas, a.muiN, stable.max(), unstable.min())
           if stable.size and unstable.size else None)
    print(json.dumps({"gas": a.gas, "E0_over_p_V_cm_Torr": (E / 100.0).tolist(), "T0_eV": out["T0"].tolist(),
                      "gamma_max_per_s": out["gamma_max"].tolist(), "wavelength_cm": (out["wavelength"] * 100).tolist(),
                      "v_ph_m_s": out["v_ph"].tolist(),
                      "threshold_V_cm_Torr": None if thr is None else thr / 100.0}))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
