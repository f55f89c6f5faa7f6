"""Pins of the two-term Boltzmann solver, and the uniform-field check of the
oracle's PIC-MCC swarm against it (the paper validates its PIC-MCC code the
same way: under a uniform field it reproduces the 0D Boltzmann EEPF and
ionization rate, section III.B/C)."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import workloads as W
from paper_2202_03215_amd import boltzmann as B
from oracle.pco import Oracle, ELECTRON, ION

MR_NE = B.ME / (20.1797 * B.AMU)


def test_constant_frequency_gives_maxwellian():
    # s_m = C eps^-1/2: f0 Maxwellian with kT = kT_g + (E/N)^2 / (6 (m/M) C^2);
    # mobility is exact: mu N = e / (m g C)
    EN = 3e-21
    C = EN / math.sqrt(6 * MR_NE * 3.0)
    cfg = W.tiny(el_A=0.0, el_B=C, el_p=-0.5, ex_smax=0.0, iz_smax=0.0, Tg=300.0)
    s = B.solve(cfg, EN, eps_max=60.0, n=3000)
    kT = B.KB * 300.0 / B.QE + EN ** 2 / (6 * MR_NE * C ** 2)
    assert abs(s.eps_mean / (1.5 * kT) - 1) < 2e-4
    sel = (s.eps > 0.5) & (s.eps < 20)
    assert abs(np.polyfit(s.eps[sel], np.log(s.f0[sel]), 1)[0] * kT + 1) < 1e-6
    assert abs(s.muN / (B.QE / (B.ME * B.GAMMA * C)) - 1) < 2e-4


def test_constant_cross_section_gives_druyvesteyn():
    EN = 30e-21
    sig = 1e-20
    cfg = W.tiny(el_A=sig, el_B=0.0, el_p=0.5, ex_smax=0.0, iz_smax=0.0, Tg=0.0)
    s = B.solve(cfg, EN, eps_max=60.0, n=3000)
    a = 3 * MR_NE * sig ** 2 / EN ** 2
    num = quad(lambda e: e ** 1.5 * math.exp(-a * e * e), 0, 60)[0]
    den = quad(lambda e: e ** 0.5 * math.exp(-a * e * e), 0, 60)[0]
    assert abs(s.eps_mean / (num / den) - 1) < 1e-5


@pytest.mark.parametrize("EN", [10e-21, 30e-21])
def test_energy_balance_with_inelastic_channels(EN):
    # field power per electron equals elastic plus inelastic losses (cold gas)
    cfg = W.tiny(Tg=0.0)
    s = B.solve(cfg, EN)
    de = s.eps[1] - s.eps[0]
    M = cfg["M_amu"] * B.AMU
    elastic = B.GAMMA * np.sum(2 * B.ME / M * B.sigma_elastic(cfg, s.eps) * s.eps ** 2 * s.f0 * de)
    loss = elastic + cfg["ex_U"] * s.k_ex + cfg["iz_U"] * s.k_iz
    gain = EN * s.w
    assert abs(loss / gain - 1) < 5e-3


def test_oracle_swarm_matches_two_term():
    # uniform field, elastic + excitation, light test atoms (M = 200 m_e) so
    # that the energy relaxes within ~1e5 steps; drift from the mean
    # displacement, mean energy averaged over the measurement window.  The
    # null-collision method samples collisions at (1 - exp(-nu_max dt)) /
    # (nu_max dt) of the continuous rate per step; the two-term solve uses the
    # same factor.
    EN = 10e-21
    M_amu = 200 * B.ME / B.AMU
    cfg = W.tiny("periodic", n_cells=10, L=1.0, poisson=0, wall_mode="off", iz_smax=0.0,
                 cx_sigma=0.0, M_amu=M_amu, eps_cap=40.0, ppc=1)
    Ng = cfg["p_torr"] * (101325 / 760) / (B.KB * cfg["Tg"])
    cfg["V"] = EN * Ng * cfg["L"]
    o = Oracle(cfg, init=False)
    c = o.constant("P_null") / (o.constant("nu_max") * cfg["dt"])
    s = B.solve(cfg, EN, collision_scale=c)
    n = 2000
    rng = np.random.default_rng(1)
    sv = math.sqrt(2 / 3 * s.eps_mean * B.QE / B.ME)
    o.set_state(ELECTRON, 0.3 + 0.01 * rng.random(n), *rng.normal(0, sv, (3, n)),
                np.arange(n, dtype=np.uint32))
    o.set_state(ION, np.array([0.0005]), *np.zeros((3, 1)), np.zeros(1, dtype=np.uint32))
    o.set_counters(1, n, 1)
    nu = Ng * (cfg["el_A"] + cfg["el_B"] * math.sqrt(s.eps_mean)) * math.sqrt(2 * s.eps_mean * B.QE / B.ME)
    relax = 1 / (nu * 2 * B.ME / (M_amu * B.AMU))
    warm, chunk = int(2.5 * relax / cfg["dt"]), int(3 * relax / cfg["dt"]) // 100
    o.step(warm)
    x0 = o.state(ELECTRON)[0].mean()
    es = []
    for _ in range(100):
        o.step(chunk)
        _, vx, vy, vz, _ = o.state(ELECTRON)
        es.append((0.5 * B.ME * (vx ** 2 + vy ** 2 + vz ** 2)).mean() / B.QE)
    w = (o.state(ELECTRON)[0].mean() - x0) / (100 * chunk * cfg["dt"])
    assert o.errors == 0
    assert abs(w / s.w - 1) < 0.03
    assert abs(np.mean(es) / s.eps_mean - 1) < 0.03


@pytest.mark.parametrize("p_torr, frozen", [(1.0, W.NU_W_NE_1TORR_10VCM), (0.5, W.NU_W_NE_05TORR_10VCM)])
def test_workload_wall_frequency_is_eq2(p_torr, frozen):
    # eq. (2): nu_w = (2.405 / R)^2 D_a with D_a = mu_i D_e / mu_e (the
    # ambipolar diffusion of section II), R = 1 cm, mu_i N = 4e21 /(V m s),
    # D_e / mu_e from the two-term solution at E0 = 10 V/cm: the value the
    # neon workloads freeze in their configs
    cfg = W.with_(W.column_20cm(), p_torr=p_torr)
    N = p_torr * (101325.0 / 760.0) / (B.KB * cfg["Tg"])
    s = B.solve(cfg, 1000.0 / N)
    Da = 4.0e21 / N * s.DN / s.muN
    nu = (2.405 / 0.01) ** 2 * Da
    assert abs(nu / frozen - 1) < 0.01, (nu, frozen)
    for wl in (W.small_bounded(), W.column_20cm(), W.column_50cm()):
        if wl["p_torr"] == p_torr:
            assert wl["nu_w"] == frozen
