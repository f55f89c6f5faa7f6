"""Pins of the oracle's charge deposit and Poisson solve.

Deposit (linear weighting of particle positions onto the grid, paper section
II) is checked against exact rational arithmetic, conservation and order
independence.  The field solve (Poisson's equation by the Thomas algorithm,
section II) is checked against closed-form discrete solutions, an FFT solve of
the periodic system, scipy's banded solver and Gauss's law.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle.pco import Oracle

QE = 1.602176634e-19
EPS0 = 8.8541878128e-12
FIX = 1 << 25


def _col(bc, n_cells=37, L=0.0037, **kw):
    return Oracle(W.tiny(bc=bc, n_cells=n_cells, L=L, **kw), init=False)


@pytest.mark.parametrize("bc", ["bounded", "periodic"])
def test_deposit_total_charge_exact(bc):
    o = _col(bc)
    x = W.random_positions(10007, 0.0037, seed=11)
    rho = o.deposit(x)
    assert rho.sum() == 10007 * FIX
    assert (rho >= 0).all()


@pytest.mark.parametrize("bc", ["bounded", "periodic"])
def test_deposit_matches_exact_rational_weights(bc):
    # brute force: node j+1 receives floor(frac(x/dx) 2^25) up to one unit
    # (the oracle forms x/dx as x * (n/L) in double)
    nc, L = 37, 0.0037
    o = _col(bc, n_cells=nc, L=L)
    x = W.random_positions(300, L, seed=5)
    nn = nc if bc == "periodic" else nc + 1
    for xi in x:
        s = Fraction(xi) * nc / Fraction(L)
        j = int(s)
        a = int((s - j) * FIX)
        ref = np.zeros(nn, dtype=np.int64)
        ref[j] += FIX - a
        ref[(j + 1) % nc if bc == "periodic" else j + 1] += a
        got = o.deposit(np.array([xi]))
        assert np.abs(got - ref).max() <= 1
        assert got.sum() == FIX


def test_deposit_on_node_goes_to_that_node_only():
    o = _col("bounded", n_cells=16, L=1.0)   # dx = 1/16 exactly
    for j in range(16):
        rho = o.deposit(np.array([j / 16.0]))
        ref = np.zeros(17, dtype=np.int64)
        ref[j] = FIX
        assert np.array_equal(rho, ref)


def test_deposit_order_independent_and_mirror():
    o = _col("bounded", n_cells=16, L=1.0)
    rng = np.random.default_rng(2)
    # dyadic positions: x*16 has at most 20 fractional bits, so f*2^25 is exact
    x = rng.integers(0, 16 << 20, size=4000) / float(16 << 20)
    r1 = o.deposit(x)
    r2 = o.deposit(x[rng.permutation(x.size)])
    assert np.array_equal(r1, r2)
    xm = 1.0 - x
    keep = xm < 1.0
    rm = o.deposit(xm[keep])
    r1k = o.deposit(x[keep])
    assert np.array_equal(rm, r1k[::-1])


def test_deposit_rejects_out_of_range():
    o = _col("periodic")
    with pytest.raises(RuntimeError):
        o.deposit(np.array([0.0037]))
    with pytest.raises(RuntimeError):
        o.deposit(np.array([-1e-12]))


# ---------------------------------------------------------------- field

def _fpc(o):
    return QE * o.constant("W") / FIX / EPS0


def test_field_zero_charge_bounded_is_uniform():
    o = _col("bounded", n_cells=400, L=0.04, V=40.0)
    z = np.zeros(401, dtype=np.int64)
    phi, E = o.solve_field(z, z)
    x = np.arange(401) * 0.04 / 400
    assert np.abs(phi - 40.0 * x / 0.04).max() <= 1e-12 * 40.0
    assert np.abs(E + 1000.0).max() <= 1e-12 * 1000.0


def test_field_uniform_charge_bounded_parabola():
    # constant interior charge density: the 3-point scheme is exact for the
    # parabola phi = V x/L + rho x (L - x) / (2 eps0)
    nc, L, V = 200, 0.02, 7.0
    o = _col("bounded", n_cells=nc, L=L, V=V)
    q = np.full(nc + 1, 3 << 26, dtype=np.int64)
    z = np.zeros(nc + 1, dtype=np.int64)
    phi, E = o.solve_field(z, q)
    dx = L / nc
    rho = QE * o.constant("W") * (3 << 26) / FIX / dx
    x = np.arange(nc + 1) * dx
    ref = V * x / L + rho * x * (L - x) / (2 * EPS0)
    assert np.abs(phi - ref).max() <= 1e-11 * np.abs(ref).max()
    Eref = -(V / L + rho * (L - 2 * x) / (2 * EPS0))
    # interior nodes: centred difference of a parabola is exact
    assert np.abs(E[1:-1] - Eref[1:-1]).max() <= 1e-10 * np.abs(Eref).max()


@pytest.mark.parametrize("m", [1, 3, 7])
def test_field_periodic_sinusoid_closed_form(m):
    nc, L, E0L = 256, 0.0256, 2.56
    o = _col("periodic", n_cells=nc, L=L, V=E0L)
    j = np.arange(nc)
    amp = float(1 << 40)
    q = np.rint(amp * np.sin(2 * np.pi * m * j / nc)).astype(np.int64)
    base = np.full(nc, 1 << 42, dtype=np.int64)
    phi, E = o.solve_field(base, base + q)
    dx = L / nc
    k = 2 * np.pi * m / L
    rho = QE * o.constant("W") * q / FIX / dx
    phi_ref = rho * dx * dx / (EPS0 * (2 - 2 * np.cos(k * dx)))
    phi_ref -= phi_ref[0]                     # gauge phi_0 = 0
    assert np.abs(phi - phi_ref).max() <= 1e-9 * np.abs(phi_ref).max()
    Esp = (np.roll(phi_ref, 1) - np.roll(phi_ref, -1)) / (2 * dx)
    assert np.abs(E - (-E0L / L + Esp)).max() <= 1e-9 * np.abs(Esp).max()


def _fft_periodic(q, dx, fpc):
    """Independent periodic solve: spectral inversion of the 3-point Laplacian."""
    n = q.size
    b = fpc * dx * (q - q.mean())
    bh = np.fft.fft(b)
    lam = 2 - 2 * np.cos(2 * np.pi * np.arange(n) / n)
    ph = np.zeros_like(bh)
    ph[1:] = bh[1:] / lam[1:]
    phi = np.real(np.fft.ifft(ph))
    return phi - phi[0]


@pytest.mark.parametrize("nc", [37, 400, 2000])
def test_field_periodic_random_vs_fft(nc):
    L = nc * 1e-4
    o = _col("periodic", n_cells=nc, L=L, V=L * 1000.0)
    re, ri = W.charge_profile(nc, seed=nc)
    phi, E = o.solve_field(re, ri)
    ref = _fft_periodic((ri - re).astype(np.float64), L / nc, _fpc(o))
    assert np.abs(phi - ref).max() <= 1e-10 * np.abs(ref).max()
    # mean space-charge field vanishes, node-0 equation holds
    Esp = E + 1000.0
    assert abs(Esp.mean()) <= 1e-9 * np.abs(Esp).max()


@pytest.mark.parametrize("nc", [37, 400, 2000])
def test_field_bounded_random_vs_banded_and_gauss(nc):
    L, V = nc * 1e-4, 33.0
    o = _col("bounded", n_cells=nc, L=L, V=V)
    re, ri = W.charge_profile(nc + 1, seed=nc + 1)
    phi, E = o.solve_field(re, ri)
    dx = L / nc
    fpc = _fpc(o)
    b = fpc * dx * (ri - re)[1:nc].astype(np.float64)
    b[-1] += V
    ab = np.zeros((3, nc - 1))
    ab[0, 1:] = -1.0
    ab[1, :] = 2.0
    ab[2, :-1] = -1.0
    ref = scipy.linalg.solve_banded((1, 1), ab, b)
    assert np.abs(phi[1:nc] - ref).max() <= 1e-12 * max(np.abs(ref).max(), V)
    assert phi[0] == 0.0 and phi[nc] == V
    # Gauss's law over the whole column: eps0 (E_N - E_0) = total charge
    tot = fpc * float((ri - re).sum())
    assert abs((E[nc] - E[0]) - tot) <= 1e-9 * max(abs(tot), np.abs(E).max())


def _exact_gauss_field(o, bc, re, ri, V):
    """Exact rational solution of the three-point system, written as Gauss's
    law over half cells (independent of the Thomas sweeps being pinned)."""
    from fractions import Fraction as Fr
    nc = o.nc
    L = Fr(o.cfg["L"])
    fpc = Fr(_fpc(o))
    Q = [int(a) - int(b) for a, b in zip(ri, re)]
    T = [0] * nc
    for j in range(1, nc):
        T[j] = T[j - 1] + Q[j]
    if bc == "bounded":
        eh0 = -Fr(V) / L - fpc * Fr(sum(T), nc)
        Eh = [eh0 + fpc * t for t in T]
        E = [Eh[0] - fpc * Q[0]] + [(Eh[j - 1] + Eh[j]) / 2 for j in range(1, nc)] + \
            [Eh[nc - 1] + fpc * Q[nc]]
    else:
        qt = sum(Q)
        Tp = [Fr(T[j]) - Fr(j * qt, nc) for j in range(nc)]
        eh0 = -fpc * sum(Tp) / nc
        Eh = [eh0 + fpc * t for t in Tp]
        E = [-Fr(V) / L + (Eh[j - 1] + Eh[j]) / 2 for j in range(nc)]
    return np.array([float(v) for v in E])


@pytest.mark.parametrize("bc", ["bounded", "periodic"])
@pytest.mark.parametrize("nc", [2000, 8000])
def test_field_matches_exact_rational_solution(bc, nc):
    # the Thomas reference must be far tighter than the 1e-12 parity bar
    L = nc * 1e-4
    o = _col(bc, n_cells=nc, L=L, V=L * 1000.0)
    re, ri = W.charge_profile(o.nn, seed=1 + nc)
    _, E = o.solve_field(re, ri)
    Ex = _exact_gauss_field(o, bc, re, ri, L * 1000.0)
    assert np.abs(E - Ex).max() <= 2e-14 * np.abs(Ex).max()
