"""Pins of the fluid-column oracle (oracle/fluid.py) against closed forms of
the discrete scheme: with temperature-independent coefficients a density or
temperature sinusoid decays by exactly 1/(1 + dt D (2 - 2 cos(k dx))/dx^2)
per backward-Euler step (D = D_a for the density, D_eps for the
temperature); the homogeneous steady state of section IV (nu_i(T0) = nu_w,
heating equal to loss) is preserved; particles are conserved when
ionisation balances the losses."""
import numpy as np
import pytest

import workloads as W
from oracle import fluid as F


def _col(table, N=64, L=0.02, Ngas=3.2e22, nu_w=1.0e5, dt=2e-9, E0=None):
    c = F.FluidColumn(n_cells=N, L=L, Ngas=Ngas, E0=0.0, nu_w=nu_w, muiN=4.0e21, dt=dt,
                      T_min=W.FLUID_T_MIN, T_step=W.FLUID_T_STEP, table=table)
    if E0 is None:
        T0, E0 = F.steady_temperature(c) if np.ptp(table[:, 4]) > 0 else (4.0, None)
        if E0 is None:
            cv = F.interp(c, np.array([T0]))[0][0]
            E0 = np.sqrt(Ngas * cv[5] / (cv[0] / Ngas))
    c.E0 = E0
    return c


def test_cyclic_solve_matches_definition():
    rng = np.random.default_rng(0)
    N = 50
    a, c = rng.normal(size=N), rng.normal(size=N)
    b = 4.0 + rng.random(N)
    d = rng.normal(size=N)
    x = F.cyclic_solve(a, b, c, d)
    r = a * np.roll(x, 1) + b * x + c * np.roll(x, -1) - d
    assert np.abs(r).max() < 1e-13


def test_density_sinusoid_decays_at_the_discrete_rate():
    col = _col(W.fluid_table_flat())
    N, m = col.n_cells, 3
    x = (np.arange(N) + 0.5) / N
    n0 = 1e15 * (1.0 + 1e-6 * np.cos(2 * np.pi * m * x))
    w0 = 1.5 * n0 * 4.0
    Ng = col.Ngas
    Da = (col.muiN / Ng) * (3.0e24 / Ng) / (1.0e24 / Ng)
    dx = col.L / N
    g = 1.0 / (1.0 + col.dt * Da * (2 - 2 * np.cos(2 * np.pi * m / N)) / dx ** 2)
    n, w = n0, w0
    for k in range(1, 21):
        n, w = F.step(col, n, w)
        amp = (n - n.mean()) / 1e15
        expect = 1e-6 * g ** k * np.cos(2 * np.pi * m * x)
        assert np.abs(amp - expect).max() < 1e-6 * 1e-8, k
    assert abs(n.sum() - n0.sum()) < 1e-12 * n0.sum()      # conservation (nu_i = nu_w)


def test_temperature_sinusoid_decays_at_the_discrete_rate():
    # n uniform, flat tables, balanced field: the energy equation reduces to
    # dT/dt = D_eps T'' + mu_eps E T' (heat conduction and convection by the
    # energy drift, eq. (13)); per step a mode T^ e^{ikx} is multiplied by
    # (1 + i dt mu_eps E sin(k dx)/dx) / (1 + dt D_eps (2 - 2 cos(k dx))/dx^2)
    col = _col(W.fluid_table_flat())
    N, m = col.n_cells, 2
    x = (np.arange(N) + 0.5) / N
    n0 = np.full(N, 1e15)
    ph = 2 * np.pi * m * x
    T0 = 4.0 * (1.0 + 1e-6 * np.sin(ph))
    Deps = 5.0 / 3.0 * 3.0e24 / col.Ngas
    mueps = 5.0 / 3.0 * 1.0e24 / col.Ngas
    dx = col.L / N
    kdx = 2 * np.pi * m / N
    g = (1.0 + 1j * col.dt * mueps * col.E0 * np.sin(kdx) / dx) / \
        (1.0 + col.dt * Deps * (2 - 2 * np.cos(kdx)) / dx ** 2)
    n, w = n0, 1.5 * n0 * T0
    for k in range(1, 21):
        n, w = F.step(col, n, w)
        T = w / (1.5 * n)
        expect = 4.0 * 1e-6 * np.imag(g ** k * np.exp(1j * ph))
        assert np.abs(n - 1e15).max() < 1e-12 * 1e15
        assert np.abs((T - 4.0) - expect).max() < 4.0 * 1e-6 * 1e-8, k
    assert abs(np.angle(g)) > 1e-3        # the convection term is exercised


def test_homogeneous_steady_state_is_preserved():
    col = _col(W.fluid_table_smooth())
    T0, E0 = F.steady_temperature(col)
    assert 1.0 < T0 < 10.0
    n = np.full(col.n_cells, 1e15)
    w = 1.5 * n * T0
    n1, w1 = F.run(col, n, w, 50)
    assert np.abs(n1 / n - 1).max() < 1e-9
    assert np.abs(w1 / w - 1).max() < 1e-9
    d = col.diag
    assert np.allclose(d["E"], E0, rtol=1e-12, atol=0)        # eq. (17) gives back the imposed field


def test_perturbed_column_stays_positive_and_finite():
    col = _col(W.fluid_table_smooth(), N=128, L=0.05)
    T0, _ = F.steady_temperature(col)
    rng = np.random.default_rng(3)
    n = 1e15 * (1.0 + 0.05 * rng.normal(size=col.n_cells))
    w = 1.5 * n * T0
    n, w = F.run(col, n, w, 200)
    assert np.all(np.isfinite(n)) and np.all(np.isfinite(w)) and n.min() > 0


def _perturbed(col, seed, amp=0.05):
    T0, _ = F.steady_temperature(col)
    rng = np.random.default_rng(seed)
    n = 1e15 * (1.0 + amp * rng.normal(size=col.n_cells))
    w = 1.5 * n * T0 * (1.0 + amp * rng.normal(size=col.n_cells))
    return n, w


def test_constant_multipliers_equal_scaled_tables():
    """Multiplier closure with constant answers (m_D, m_eps): the first step
    is the table closure itself (no multipliers before the network has
    answered), every later step the table closure on a table whose D_e column
    is scaled by m_D and whose mu_eps and D_eps columns by m_eps (the
    multipliers act on the coefficients, the gradient term of eq. (17) and
    the slopes alike).  A multiplier outside [1/4, 4] acts as its bound."""
    for mD, mE, eD, eE in ((1.3, 0.7, 1.3, 0.7), (9.0, 0.1, 4.0, 0.25)):
        col = _col(W.fluid_table_smooth(), N=64, L=0.03)
        n0, w0 = _perturbed(col, 5)
        col.multipliers = lambda f: (np.full(f.shape[0], mD), np.full(f.shape[0], mE))
        n1, w1 = F.step(col, n0, w0)
        ref = _col(W.fluid_table_smooth(), N=64, L=0.03)
        r1, s1 = F.step(ref, n0, w0)
        assert np.array_equal(n1, r1) and np.array_equal(w1, s1)
        n, w = F.run(col, n1, w1, 5)
        tab = W.fluid_table_smooth().copy()
        tab[:, 1] *= eD
        tab[:, 2:4] *= eE
        sc = _col(tab, N=64, L=0.03)
        sc.E0 = col.E0
        r, s = F.run(sc, r1, s1, 5)
        assert np.allclose(n, r, rtol=1e-12, atol=0) and np.allclose(w, s, rtol=1e-12, atol=0)
        assert not np.allclose(n, F.run(ref, r1, s1, 5)[0], rtol=1e-6)   # the multipliers changed the run


def test_multipliers_follow_the_previous_step_features():
    """The multipliers applied at step k are the network's answer to the face
    features of step k - 1 (features n_f, 3/2 T_f, E_f, dn_f, 3/2 dT_f): a
    hook recording its inputs sees at each call exactly the features of the
    table closure's diagnostics of the same step."""
    col = _col(W.fluid_table_smooth(), N=32, L=0.02)
    n, w = _perturbed(col, 9)
    seen = []

    def hook(f):
        seen.append(f.copy())
        return 1.0 + 0.1 * np.tanh(f[:, 3] / np.abs(f[:, 3]).max()), np.full(f.shape[0], 1.2)

    col.multipliers = hook
    for k in range(3):
        n, w = F.step(col, n, w)
        d = col.diag
        feats = np.stack([d["nf"], 1.5 * d["Tf"], d["E"], d["dn"], 1.5 * d["dT"]], axis=1)
        assert np.array_equal(seen[k], feats)
    assert len(seen) == 3 and col.m[1].max() == 1.2
