"""Plain oracle of the linear stability analysis of section IV.F (test
infrastructure only: tests, the smoke check and the CPU baseline use it).

Instead of the closed forms (19)-(22), it works from the 2x2 system (18)
itself: for each k the determinant of the matrix is affine in Omega, so it is
evaluated at two values of Omega and its root taken; the maximum growth rate
is then found numerically over k (logarithmic scan and golden-section
refinement).  The coefficients at T0 are evaluated with the fluid oracle's
table interpolant (oracle.fluid.interp) and the definitions (9), (14)-(16)
(eq. (9) read as beta = 3/2 T mu_eps, G = 3/2 T D_eps).
"""
from __future__ import annotations

import numpy as np

from . import fluid as F


def coefficients(table, T_min, T_step, Ngas, muiN, T0) -> dict:
    col = F.FluidColumn(n_cells=2, L=1.0, Ngas=Ngas, E0=0.0, nu_w=0.0, muiN=muiN, dt=1.0,
                        T_min=T_min, T_step=T_step, table=np.asarray(table, dtype=np.float64))
    v, s = F.interp(col, np.array([T0]))
    v, s = v[0] / Ngas, s[0] / Ngas
    mu, D, mu_eps, D_eps = v[0], v[1], v[2], v[3]
    beta = 1.5 * T0 * mu_eps                       # eq. (9)
    G = 1.5 * T0 * D_eps
    dG_dT = 1.5 * D_eps + 1.5 * T0 * s[3]
    L = Ngas * Ngas * v[5]                         # table holds L / N
    return dict(E0=np.sqrt(L / mu), D_e=D, D_a=(muiN / Ngas) * D / mu,
                chi=G - (beta / mu) * D,             # eq. (16)
                K=dG_dT - (beta / mu) * s[1],        # eq. (15) over n0
                nu_p=Ngas * Ngas * s[4], L=L, L_p=Ngas * Ngas * s[5])


def matrix(Omega: complex, k: float, c: dict, n0: float = 1.0) -> np.ndarray:
    """The matrix of eq. (18) acting on (dn / n0, dT)."""
    return np.array([[-1j * Omega + c["D_a"] * k * k, -n0 * c["nu_p"]],
                     [c["chi"] * k * k + 2.0 * c["L"] + 1j * k * c["E0"] * c["D_e"],
                      n0 * c["K"] * k * k + n0 * c["L_p"]]], dtype=np.complex128)


def det(M: np.ndarray) -> complex:
    return complex(M[0, 0] * M[1, 1] - M[0, 1] * M[1, 0])


def omega(k: float, c: dict) -> complex:
    """Omega = omega + i gamma with det(matrix) = 0.  The determinant is
    affine in Omega: its value at 0 and its slope give the root; the slope is
    the difference quotient between Omega = +S and -S with S large enough
    that the value at 0 does not round it away."""
    d0 = det(matrix(0.0, k, c))
    S = 1.0e15
    slope = (det(matrix(S, k, c)) - det(matrix(-S, k, c))) / (2.0 * S)
    return complex(-d0 / slope)


def max_growth(c: dict, k_lo: float = 1.0, k_hi: float = 1.0e5) -> tuple[float, float]:
    """(gamma_max, k_max) by scanning gamma(k) on a log grid and refining the
    best bracket by golden sections."""
    ks = np.geomspace(k_lo, k_hi, 2001)
    g = np.array([omega(k, c).imag for k in ks])
    i = int(np.argmax(g))
    a, b = ks[max(i - 1, 0)], ks[min(i + 1, ks.size - 1)]
    r = (np.sqrt(5.0) - 1.0) / 2.0
    for _ in range(200):
        x1, x2 = b - r * (b - a), a + r * (b - a)
        if omega(x1, c).imag < omega(x2, c).imag:
            a = x1
        else:
            b = x2
    k = 0.5 * (a + b)
    return omega(k, c).imag, k
