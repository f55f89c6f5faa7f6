"""Two-term steady homogeneous Boltzmann solver for the electron energy
distribution in a DC field (CPU, offline).

The paper uses a 0D Boltzmann solver to relate the reduced field E0/p to the
electron temperature, the ionization frequency and the transport
coefficients that enter eq. (2) and the fluid model of section IV
(mu_e, D_e, mu_eps, D_eps, nu_i, energy loss).  This is the project's own
solver for the synthetic cross sections: the isotropic part f0(eps) of the
distribution (normalised so that the integral of eps^(1/2) f0 is 1, as the
EEPF of section III.C) obeys, per gas atom,

    d/deps [ W f0 - D df0/deps ] = S_inel(eps)
    W = -g eps^2 (2m/M) s_m                               (elastic cooling)
    D = (g/3) (E/N)^2 eps / s_m + g (k T_g / e) eps^2 (2m/M) s_m
    S = sum_k [ -g eps s_k(eps) f0(eps) + g (eps+U_k) s_k(eps+U_k) f0(eps+U_k) ]

with g = sqrt(2e/m) and energies in eV.  Excitation and ionization both
remove their threshold (ionization without electron growth; the ejected
electron is not followed).  Finite volumes on a uniform energy grid with
Scharfetter-Gummel fluxes; the non-local gain term is interpolated linearly.

Closed-form checks (tests): constant collision frequency gives a Maxwellian
with kT = kT_g + (E/N)^2 / (6 (m/M) C^2) for s_m = C eps^-1/2; constant
cross section gives the Druyvesteyn law exp(-3 (m/M) s^2 eps^2 / (E/N)^2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

QE = 1.602176634e-19
ME = 9.1093837015e-31
AMU = 1.66053906660e-27
KB = 1.380649e-23
GAMMA = math.sqrt(2.0 * QE / ME)   # m/s per sqrt(eV)


def sigma_elastic(cfg: dict, eps: np.ndarray) -> np.ndarray:
    e = np.maximum(eps, 1e-300)
    if cfg["el_p"] > 0:
        return cfg["el_A"] + cfg["el_B"] * np.sqrt(e)
    return cfg["el_A"] + cfg["el_B"] / np.sqrt(e)


def sigma_thomson(eps: np.ndarray, U: float, smax: float) -> np.ndarray:
    e = np.asarray(eps, dtype=np.float64)
    out = np.zeros_like(e)
    m = e > U
    t = U / e[m]
    out[m] = 4.0 * smax * t * (1.0 - t)
    return out


@dataclass
class Swarm:
    EN: float            # reduced field [V m^2]
    eps_mean: float      # mean energy [eV]
    Te: float            # (2/3) mean energy [eV]
    muN: float           # mobility x N [1/(V m s)]
    DN: float            # diffusion x N [1/(m s)]
    mu_epsN: float       # energy mobility x N
    D_epsN: float        # energy diffusion x N
    k_ex: float          # rate coefficients [m^3/s]
    k_iz: float
    w: float             # drift velocity [m/s]
    eps: np.ndarray      # grid (cell centres) [eV]
    f0: np.ndarray       # EEPF [eV^-3/2]


def solve(cfg: dict, EN: float, eps_max: float = 100.0, n: int = 4000,
          include_inelastic: bool = True, collision_scale: float = 1.0) -> Swarm:
    """Two-term solution for the cross sections of a workload config at the
    reduced field EN = E/N [V m^2].  collision_scale multiplies every cross
    section (e.g. the per-step sampling factor of a discrete-time collision
    method when comparing with it)."""
    if collision_scale != 1.0:
        cfg = dict(cfg)
        for k in ("el_A", "el_B", "ex_smax", "iz_smax"):
            cfg[k] = cfg[k] * collision_scale
    M = cfg["M_amu"] * AMU
    mr = ME / M
    kTg = KB * cfg["Tg"] / QE
    de = eps_max / n
    ec = (np.arange(n) + 0.5) * de          # cell centres
    ef = (np.arange(n + 1)) * de            # faces
    sm_f = sigma_elastic(cfg, ef)
    with np.errstate(divide="ignore", invalid="ignore"):
        W = -GAMMA * ef ** 2 * 2.0 * mr * sm_f
        D = GAMMA / 3.0 * EN ** 2 * ef / sm_f + GAMMA * kTg * ef ** 2 * 2.0 * mr * sm_f
    # Scharfetter-Gummel flux at interior faces k = 1..n-1:
    #   G_k = a_k F_{k-1} - b_k F_k
    a = np.zeros(n + 1)
    b = np.zeros(n + 1)
    for k in range(1, n):
        z = W[k] * de / D[k]
        if abs(z) < 1e-8:
            a[k] = D[k] / de + 0.5 * W[k]
            b[k] = D[k] / de - 0.5 * W[k]
        else:
            ez = math.exp(z) if z < 700 else math.inf
            if math.isinf(ez):
                a[k], b[k] = W[k], 0.0
            else:
                a[k] = W[k] * ez / (ez - 1.0)
                b[k] = W[k] / (ez - 1.0)
    # (G_{i+1} - G_i)/de = S_i
    rows, cols, vals = [], [], []

    def put(i, j, v):
        rows.append(i)
        cols.append(j)
        vals.append(v)

    for i in range(n):
        if i + 1 <= n - 1:                       # G_{i+1} = a F_i - b F_{i+1}
            put(i, i, a[i + 1] / de)
            put(i, i + 1, -b[i + 1] / de)
        if i >= 1:                               # - G_i
            put(i, i - 1, -a[i] / de)
            put(i, i, b[i] / de)
    chans = []
    if include_inelastic:
        for U, smax in ((cfg["ex_U"], cfg["ex_smax"]), (cfg["iz_U"], cfg["iz_smax"])):
            if smax > 0:
                chans.append((U, smax))
    for U, smax in chans:
        sk = sigma_thomson(ec, U, smax)
        for i in range(n):
            if sk[i] > 0:                        # loss at eps_i: -g eps s f
                put(i, i, GAMMA * ec[i] * sk[i])
            eu = ec[i] + U                       # gain from eps_i + U
            if eu < ec[-1]:
                x = eu / de - 0.5
                j = int(math.floor(x))
                t = x - j
                s_up = sigma_thomson(np.array([eu]), U, smax)[0]
                g = GAMMA * eu * s_up
                if g > 0:
                    put(i, j, -g * (1.0 - t))
                    put(i, j + 1, -g * t)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n)).tolil()
    # normalisation replaces the last equation: sum sqrt(eps) F de = 1
    A[n - 1, :] = np.sqrt(ec) * de
    rhs = np.zeros(n)
    rhs[n - 1] = 1.0
    F = spla.spsolve(A.tocsr(), rhs)
    F = np.maximum(F, 0.0)
    F /= np.sum(np.sqrt(ec) * F * de)
    # moments
    dF = np.gradient(F, de)
    smc = sigma_elastic(cfg, ec)
    eps_mean = float(np.sum(ec ** 1.5 * F * de))
    muN = float(-GAMMA / 3.0 * np.sum(ec / smc * dF * de))
    DN = float(GAMMA / 3.0 * np.sum(ec / smc * F * de))
    mu_epsN = float(-GAMMA / (3.0 * eps_mean) * np.sum(ec ** 2 / smc * dF * de))
    D_epsN = float(GAMMA / (3.0 * eps_mean) * np.sum(ec ** 2 / smc * F * de))
    k_ex = float(GAMMA * np.sum(ec * sigma_thomson(ec, cfg["ex_U"], cfg["ex_smax"]) * F * de))
    k_iz = float(GAMMA * np.sum(ec * sigma_thomson(ec, cfg["iz_U"], cfg["iz_smax"]) * F * de))
    return Swarm(EN=EN, eps_mean=eps_mean, Te=2.0 / 3.0 * eps_mean, muN=muN, DN=DN,
                 mu_epsN=mu_epsN, D_epsN=D_epsN, k_ex=k_ex, k_iz=k_iz, w=muN * EN,
                 eps=ec, f0=F)


def table(cfg: dict, EN_values, **kw):
    """Transport table over reduced fields: arrays keyed by Swarm fields."""
    rows = [solve(cfg, float(en), **kw) for en in EN_values]
    keys = ("EN", "eps_mean", "Te", "muN", "DN", "mu_epsN", "D_epsN", "k_ex", "k_iz", "w")
    return {k: np.array([getattr(r, k) for r in rows]) for k in keys}
