"""Plain FP64 oracle of the quasi-neutral fluid column (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this module; it shares no code with the GPU library.

Model: section IV of the paper.  Electron continuity (3) and energy (4)
equations with the heating (5), drift-diffusion fluxes (12)-(13) whose
coefficients (14)-(16) follow from temperature-dependent transport
coefficients, and the quasi-neutral field (17).  Reading of eq. (9): the
thermoelectric and heat diffusion coefficients are beta = 3/2 T mu_eps and
G = 3/2 T D_eps.  The column is periodic with an imposed mean field E0, which
fixes the constant total flux Gamma_T at every step.

Discrete scheme (written out here and in the design notes; the GPU follows
the same steps):
  cells j = 0..N-1 (periodic), faces f = j + 1/2 between j and j+1
  T_j = w_j / (1.5 n_j), w the energy density 3/2 n T [eV m^-3]
  coefficients from a table on a uniform T grid, linear interpolation, T
  clamped to the table; slopes d/dT from the same linear segments
  face state: n_f, T_f = means of the two cells; coefficients at T_f
  dn_f = (n_{j+1} - n_j)/dx, dT_f likewise
  Phi_j = n_j D_e(T_j)/mu_e(T_j)
  A_f = (Phi_{j+1} - Phi_j)/(dx n_f),  B_f = 1/(n_f (mu_e,f + mu_i))
  Gamma_T = (E0 + mean A) / mean B,  E_f = -A_f + Gamma_T B_f         (17)
  closure (time level k): either the table form
    Gamma_f = -D_a dn - eta dT - mu_e/(mu_e+mu_i) Gamma_T               (12)
    H_f     = -chi dn - kappa dT - beta/(mu_e+mu_i) Gamma_T             (13)
  with D_a = mu_i D_e/mu_e, eta = n (mu_i/mu_e) D_e', beta = 1.5 T mu_eps,
  G = 1.5 T D_eps, kappa = n (G' - beta D_e'/mu_e), chi = G - beta D_e/mu_e,
  or a closure network fed (n_f, 1.5 T_f, E_f, dn_f, 1.5 dT_f) (normalised),
  or the table form with multipliers from a network fed the same features:
    m_D multiplies D_e, its slope and A_f (the diffusion of eq. (17) at the
    face), m_eps multiplies mu_eps, D_eps and the slope of D_eps, both
    clamped to [1/4, 4]; the multipliers of step k are the network's answer
    to the features of step k - 1 (1 on the first step)
  sources: S_n = n_j (nu_i(T_j) - nu_w); heating P_j = -(Gamma E)_{j-1/2,j+1/2}
  mean; S_w = P_j - n_j L(T_j)
  implicit step (backward Euler on the diffusion parts, the rest explicit):
    Gamma'_f = Gamma_f - D_a (dn'_f - dn_f),  n' from the cyclic tridiagonal
    system  n' + dt div Gamma' = n + dt S_n
    H'_f = H_f - kappa (dT'_f - dT_f) with T' = w'/(1.5 n'),  w' from
    w' + dt div H' = w + dt S_w
  floors: n' >= n_floor, w' >= 1.5 n' T_min.

Table columns (per reduced unit of gas density N where marked):
  0 mu_e N, 1 D_e N, 2 mu_eps N, 3 D_eps N, 4 k_iz (nu_i = N k_iz),
  5 L / N (energy loss rate per electron per unit N, eV m^3 / s)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

N_TABLE_COLS = 6


@dataclass
class FluidColumn:
    n_cells: int
    L: float
    Ngas: float          # gas density [m^-3]
    E0: float            # imposed mean field [V/m]
    nu_w: float          # radial loss frequency [1/s]
    muiN: float          # ion mobility x N [1/(V m s)]
    dt: float
    T_min: float         # table grid [eV]
    T_step: float
    table: np.ndarray    # [K, 6]
    n_floor: float = 1.0e6
    # closure network hook: f(features[M, 5]) -> (Gamma[M], H[M]) in physical units
    closure: object = None
    # multiplier network hook: f(features[M, 5]) -> (m_D[M], m_eps[M]) before clamping;
    # m holds the multipliers of the next step (None: all 1)
    multipliers: object = None
    m: object = None
    diag: dict = field(default_factory=dict)


def interp(col: FluidColumn, T):
    """Coefficient rows at temperatures T (clamped), and their slopes d/dT."""
    K = col.table.shape[0]
    u = (np.clip(T, col.T_min, col.T_min + (K - 1) * col.T_step) - col.T_min) / col.T_step
    k = np.minimum(np.floor(u).astype(np.int64), K - 2)
    f = u - k
    lo = col.table[k]
    hi = col.table[k + 1]
    val = lo + f[:, None] * (hi - lo)
    slope = (hi - lo) / col.T_step
    return val, slope


M_MIN, M_MAX = 0.25, 4.0


def faces(col: FluidColumn, n, w):
    """Face quantities of the current state (time level k)."""
    N = col.n_cells
    dx = col.L / N
    Ng = col.Ngas
    mui = col.muiN / Ng
    T = w / (1.5 * n)
    cv, _ = interp(col, T)
    mue_c = cv[:, 0] / Ng
    De_c = cv[:, 1] / Ng
    Phi = n * De_c / mue_c
    nr = np.roll(n, -1)
    Tr = np.roll(T, -1)
    nf = 0.5 * (n + nr)
    Tf = 0.5 * (T + Tr)
    fv, fs = interp(col, Tf)
    mue, De, mueps, Deps = fv[:, 0] / Ng, fv[:, 1] / Ng, fv[:, 2] / Ng, fv[:, 3] / Ng
    dDe, dDeps = fs[:, 1] / Ng, fs[:, 3] / Ng
    dn = (nr - n) / dx
    dT = (Tr - T) / dx
    A = (np.roll(Phi, -1) - Phi) / (dx * nf)
    if col.multipliers is not None and col.m is not None:
        mD, mE = col.m
        A, De, dDe = mD * A, mD * De, mD * dDe
        mueps, Deps, dDeps = mE * mueps, mE * Deps, mE * dDeps
    B = 1.0 / (nf * (mue + mui))
    GT = (col.E0 + A.mean()) / B.mean()
    E = -A + GT * B
    Da = mui * De / mue
    beta = 1.5 * Tf * mueps
    G = 1.5 * Tf * Deps
    dG = 1.5 * Deps + 1.5 * Tf * dDeps
    kappa = nf * (dG - beta * dDe / mue)
    if col.closure is None:
        eta = nf * (mui / mue) * dDe
        chi = G - beta * De / mue
        Gam = -Da * dn - eta * dT - mue / (mue + mui) * GT
        H = -chi * dn - kappa * dT - beta / (mue + mui) * GT
        if col.multipliers is not None:   # the next step's multipliers
            mD, mE = col.multipliers(np.stack([nf, 1.5 * Tf, E, dn, 1.5 * dT], axis=1))
            col.m = (np.clip(mD, M_MIN, M_MAX), np.clip(mE, M_MIN, M_MAX))
    else:
        feats = np.stack([nf, 1.5 * Tf, E, dn, 1.5 * dT], axis=1)
        Gam, H = col.closure(feats)
    return dict(T=T, cv=cv, nf=nf, Tf=Tf, dn=dn, dT=dT, E=E, GT=GT, Da=Da, kappa=kappa, Gam=Gam, H=H)


def cyclic_solve(a, b, c, d):
    """Solve a_j x_{j-1} + b_j x_j + c_j x_{j+1} = d_j (indices mod N) by a
    sparse LU factorisation of the assembled matrix (scipy)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    N = b.size
    i = np.arange(N)
    M = sp.coo_matrix((np.concatenate([b, a, c]),
                       (np.concatenate([i, i, i]), np.concatenate([i, (i - 1) % N, (i + 1) % N]))),
                      shape=(N, N)).tocsc()
    return spla.spsolve(M, d)


def step(col: FluidColumn, n, w):
    """One time step; returns (n', w')."""
    N = col.n_cells
    dx = col.L / N
    dt = col.dt
    F = faces(col, n, w)
    cv = F["cv"]
    nu_i = col.Ngas * cv[:, 4]
    Lrate = col.Ngas * cv[:, 5]
    Gam, H, E = F["Gam"], F["H"], F["E"]
    Sn = n * (nu_i - col.nu_w)
    P = -0.5 * (np.roll(Gam * E, 1) + Gam * E)
    Sw = P - n * Lrate
    r = dt / (dx * dx)
    # density: faces f = j+1/2 (index j) and j-1/2 (index j-1)
    Dp = F["Da"]
    Dm = np.roll(Dp, 1)
    Ge = Gam + Dp * F["dn"]                    # explicit remainder of Gamma
    rhs = n + dt * Sn - dt / dx * (Ge - np.roll(Ge, 1))
    n1 = cyclic_solve(-r * Dm, 1.0 + r * (Dm + Dp), -r * Dp, rhs)
    n1 = np.maximum(n1, col.n_floor)
    # energy density with T' = w'/(1.5 n')
    Kp = F["kappa"]
    Km = np.roll(Kp, 1)
    m = 1.5 * n1
    He = H + Kp * F["dT"]
    rhs = w + dt * Sw - dt / dx * (He - np.roll(He, 1))
    w1 = cyclic_solve(-r * Km / np.roll(m, 1), 1.0 + r * (Km + Kp) / m, -r * Kp / np.roll(m, -1), rhs)
    w1 = np.maximum(w1, 1.5 * n1 * col.T_min)
    col.diag = F
    return n1, w1


def run(col: FluidColumn, n, w, steps: int):
    for _ in range(steps):
        n, w = step(col, n, w)
    return n, w


def steady_temperature(col: FluidColumn):
    """T0 with nu_i(T0) = nu_w on the table (bisection on the interpolant;
    the section IV homogeneous condition), and the balancing field
    E0 = sqrt(L(T0)/mu_e(T0)) (heating n mu_e E0^2 equals loss n L)."""
    K = col.table.shape[0]
    lo, hi = col.T_min, col.T_min + (K - 1) * col.T_step
    f = lambda T: col.Ngas * interp(col, np.array([T]))[0][0, 4] - col.nu_w
    if f(lo) * f(hi) > 0:
        raise ValueError("nu_w outside the tabulated ionisation frequencies")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(lo) * f(mid) <= 0:
            hi = mid
        else:
            lo = mid
    T0 = 0.5 * (lo + hi)
    cv = interp(col, np.array([T0]))[0][0]
    E0 = np.sqrt((col.Ngas * cv[5]) / (cv[0] / col.Ngas))
    return T0, E0
