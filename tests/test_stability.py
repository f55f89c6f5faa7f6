"""Linear stability of the homogeneous column (section IV.F): the closed forms
(19)-(23) of paper_2202_03215_amd.stability against the oracle, which works
from the matrix of eq. (18) directly, and against the fluid model itself.

Pins of the oracle (independent of the closed forms):
- the root Omega(k) annuls the determinant of (18) (to 1e-12 of its terms);
- gamma(-k) = gamma(k), omega(-k) = -omega(k);
- at k = 0 the matrix reduces to -i Omega L' + 2 L nu_i' = 0;
- the numerical maximum is a maximum (neighbours lower).
Closed forms against the oracle on random coefficient sets: (19)-(20) to
1e-10, (21) to 1e-9, (22) to 1e-4 (flat maximum), (23) <=> gamma_max > 0.
Against the fluid model (FP64 oracle of eqs. (3)-(17), 256 cells, dt 0.25
ns, two-term tables of the synthetic neon): the growth rate of a 1e-4
density perturbation at k_max / 2, k_max and 3 k_max / 2 agrees with eq.
(20) within 3 %, the frequency with eq. (19) within 25 % (the paper's
approximations -- no dT in dE, no time derivative in the energy equation --
act mostly on omega).
"""
import numpy as np
import pytest

import workloads as W
from oracle import fluid as F
from oracle import stability as OS
from paper_2202_03215_amd import stability as S

KEYS = ("E0", "D_e", "D_a", "chi", "K", "nu_p", "L", "L_p")


def _random_sets(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        yield dict(E0=10 ** rng.uniform(2, 3.7), D_e=10 ** rng.uniform(2, 3.7), D_a=10 ** rng.uniform(-1, 1),
                   chi=-10 ** rng.uniform(2, 4.2) if rng.random() < 0.8 else 10 ** rng.uniform(1, 3),
                   K=10 ** rng.uniform(2.7, 3.7), nu_p=10 ** rng.uniform(5, 7), L=10 ** rng.uniform(7, 9),
                   L_p=10 ** rng.uniform(7, 9))


def _product(c):
    return S.Coefficients(T0=0.0, mu_e=1.0, **c)


def test_oracle_root_annuls_the_determinant():
    for c in _random_sets(50, 1):
        for k in (10.0, 300.0, 3000.0):
            Om = OS.omega(k, c)
            M = OS.matrix(Om, k, c)
            d = OS.det(M)
            scale = abs(M[0, 0] * M[1, 1]) + abs(M[0, 1] * M[1, 0])    # the two products that cancel
            assert abs(d) <= 1e-12 * scale
            Om_m = OS.omega(-k, c)
            assert abs(Om_m.imag - Om.imag) <= 1e-12 * abs(Om)
            assert abs(Om_m.real + Om.real) <= 1e-12 * abs(Om)


def test_oracle_long_wave_limit():
    for c in _random_sets(20, 2):
        Om = OS.omega(0.0, c)
        assert abs(Om.real) <= 1e-9 * abs(Om)
        assert abs(Om.imag - (-2.0 * c["L"] * c["nu_p"] / c["L_p"])) <= 1e-12 * abs(Om.imag)


def test_closed_forms_against_the_oracle():
    n_unstable = 0
    for c in _random_sets(200, 3):
        p = _product(c)
        for k in (30.0, 500.0, 4000.0):
            Om = OS.omega(k, c)
            assert abs(S.frequency(k, p) - Om.real) <= 1e-10 * abs(Om)
            assert abs(S.growth(k, p) - Om.imag) <= 1e-10 * abs(Om)
        m = S.maximum(p)
        g_num, k_num = OS.max_growth(c, 1e-1, 1e6)
        if m["k_max"] == m["k_max"]:                    # interior maximum
            assert abs(m["gamma_max"] - g_num) <= 1e-9 * abs(g_num) + 1e-9
            assert abs(m["k_max"] - k_num) <= 1e-4 * m["k_max"]
            assert abs(S.growth(m["k_max"], p) - m["gamma_max"]) <= 1e-9 * abs(m["gamma_max"])
        assert m["unstable"] == (g_num > 0.0)
        n_unstable += m["unstable"]
    assert 40 <= n_unstable <= 160


def test_numerical_maximum_is_a_maximum():
    for c in _random_sets(20, 4):
        g, k = OS.max_growth(c, 1e-1, 1e6)
        for f in (0.99, 1.01):
            assert OS.omega(k * f, c).imag <= g


def _neon_table():
    from paper_2202_03215_amd import closure as CL
    cfg = W.column_20cm()
    Ng = cfg["p_torr"] * 133.322368 / (1.380649e-23 * cfg["Tg"])
    T, cols = CL.transport_table(cfg, np.geomspace(5e-21, 2e-19, 60), Ng)
    return CL.resample_uniform(T, cols, W.FLUID_T_MIN, W.FLUID_T_STEP, W.FLUID_T_LEN), Ng


@pytest.fixture(scope="module")
def neon():
    tab, Ng = _neon_table()
    T0 = S.temperature_for_field(tab, W.FLUID_T_MIN, W.FLUID_T_STEP, Ng, 1000.0)
    return tab, Ng, T0


def test_coefficients_and_steady_state(neon):
    tab, Ng, T0 = neon
    muiN = 4.0e21
    p = S.coefficients(tab, W.FLUID_T_MIN, W.FLUID_T_STEP, Ng, muiN, T0)
    o = OS.coefficients(tab, W.FLUID_T_MIN, W.FLUID_T_STEP, Ng, muiN, T0)
    for k in KEYS:
        assert abs(getattr(p, k) - o[k]) <= 1e-12 * abs(o[k]), k
    assert abs(p.E0 - 1000.0) <= 1e-9 * 1000.0
    nu_w = Ng * F.interp(F.FluidColumn(2, 1.0, Ng, 0.0, 0.0, muiN, 1.0, W.FLUID_T_MIN, W.FLUID_T_STEP, tab),
                         np.array([T0]))[0][0, 4]
    assert abs(S.temperature_for_loss(tab, W.FLUID_T_MIN, W.FLUID_T_STEP, Ng, nu_w) - T0) <= 1e-9 * T0
    m = S.maximum(p)
    assert m["unstable"] and m["gamma_max"] > 0 and m["v_ph"] > 0


@pytest.mark.parametrize("ratio", [0.5, 1.0, 1.5])
def test_fluid_model_growth_matches_eq20(neon, ratio):
    tab, Ng, T0 = neon
    muiN = 4.0e21
    c = S.coefficients(tab, W.FLUID_T_MIN, W.FLUID_T_STEP, Ng, muiN, T0)
    k = ratio * S.maximum(c)["k_max"]
    Lc, N, dt, steps = 4 * 2 * np.pi / k, 256, 2.5e-10, 1600
    nu_w = Ng * F.interp(F.FluidColumn(2, 1.0, Ng, 0.0, 0.0, muiN, 1.0, W.FLUID_T_MIN, W.FLUID_T_STEP, tab),
                         np.array([T0]))[0][0, 4]
    col = F.FluidColumn(n_cells=N, L=Lc, Ngas=Ng, E0=c.E0, nu_w=nu_w, muiN=muiN, dt=dt,
                        T_min=W.FLUID_T_MIN, T_step=W.FLUID_T_STEP, table=tab)
    x = (np.arange(N) + 0.5) / N * Lc
    n = 1e15 * (1.0 + 1e-4 * np.cos(k * x))
    w = 1.5 * n * T0
    ts, amps = [], []
    for s in range(steps + 1):
        if s % 40 == 0:
            ts.append(s * dt)
            amps.append(np.fft.rfft(n / 1e15 - 1.0)[4] * 2.0 / N)
        if s < steps:
            n, w = F.step(col, n, w)
    ts, amps = np.array(ts)[20:], np.array(amps)[20:]
    gamma = np.polyfit(ts, np.log(np.abs(amps)), 1)[0]
    omega = -np.polyfit(ts, np.unwrap(np.angle(amps)), 1)[0]
    print(f"k = {ratio} k_max: fluid gamma {gamma:.4e} omega {omega:.4e}; "
          f"eq. (20) {S.growth(k, c):.4e}, eq. (19) {S.frequency(k, c):.4e}")
    assert abs(gamma - S.growth(k, c)) <= 0.03 * S.growth(k, c)
    assert abs(omega - S.frequency(k, c)) <= 0.25 * S.frequency(k, c)
