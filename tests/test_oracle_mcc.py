"""Pins of the oracle's Monte Carlo collisions, radial sink, ionization
bookkeeping and initial load (paper section II).

Each check compares a statistic with what the method fixes exactly: binomial
counts with the null-collision probability, branching ratios, per-collision
energy bookkeeping, isotropy, the energy-sharing law, the charge-exchange
acceptance bias, relaxation to the gas temperature, exponential survival under
the sink, and the constant-frequency swarm's momentum and energy balance.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.stats

import workloads as W
from oracle.pco import (Oracle, ELECTRON, ION, EV_ELASTIC, EV_EXCITE, EV_IONIZE, EV_WALL,
                        EV_CX, EV_NULL, EV_NONE)

QE = 1.602176634e-19
ME = 9.1093837015e-31
AMU = 1.66053906660e-27
KB = 1.380649e-23
TORR = 101325.0 / 760.0
C_EPS = 0.5 * ME / QE

NO_COLL = dict(el_A=0.0, el_B=0.0, ex_smax=0.0, iz_smax=0.0, cx_sigma=0.0, wall_mode="off")


def _binom_ok(k, n, p, z=5.0):
    mu = n * p
    sd = math.sqrt(n * p * (1 - p))
    return abs(k - mu) <= z * sd + 1


def _beam(o, n, eps_eV, L, rng, species=ELECTRON):
    v = math.sqrt(eps_eV / C_EPS)
    x = rng.random(n) * L
    z = np.zeros(n)
    o.set_state(species, x, np.full(n, v), z, z, np.arange(n, dtype=np.uint32))


def _sigmas(cfg, eps):
    se = cfg["el_A"] + cfg["el_B"] * (math.sqrt(eps) if cfg["el_p"] > 0 else 1 / math.sqrt(eps))

    def th(U, s):
        return 4 * s * (U / eps) * (1 - U / eps) if eps > U else 0.0
    return se, th(cfg["ex_U"], cfg["ex_smax"]), th(cfg["iz_U"], cfg["iz_smax"])


def _field_free(**kw):
    base = dict(V=0.0, poisson=0, wall_mode="off", cx_sigma=0.0)
    base.update(kw)
    return W.tiny("periodic", **base)


def test_constant_frequency_collision_count():
    # sigma = B / sqrt(eps): nu = Ng B sqrt(2e/m) for every energy, so each
    # step's real-collision count is Binomial(N, P_null nu / nu_max)
    cfg = _field_free(el_A=0.0, el_B=3e-20, el_p=-0.5, ex_smax=0.0, iz_smax=0.0, ppc=400)
    o = Oracle(cfg)
    n = o.count(ELECTRON)
    Ng = cfg["p_torr"] * TORR / (KB * cfg["Tg"])
    nu = Ng * 3e-20 / math.sqrt(C_EPS)
    p = o.constant("P_null") * nu / o.constant("nu_max")
    tot = 0
    steps = 30
    for _ in range(steps):
        o.step(1)
        tot += int((o.events(ELECTRON) == EV_ELASTIC).sum())
    assert _binom_ok(tot, n * steps, p)
    assert abs(o.constant("nu_max") / nu - 1.001) < 1e-9


def test_branching_ratios_and_energy_bookkeeping():
    cfg = _field_free(ppc=2000, eps_cap=100.0)
    o = Oracle(cfg, init=False)
    rng = np.random.default_rng(7)
    n = 60000
    eps0 = 60.0
    _beam(o, n, eps0, cfg["L"], rng)
    o.set_state(ION, np.array([0.001]), *np.zeros((3, 1)), np.zeros(1, dtype=np.uint32))
    o.set_counters(1, n, 1)
    x0, vx0, vy0, vz0, id0 = o.state(ELECTRON)
    o.step(1)
    ev = o.events(ELECTRON, n)
    x, vx, vy, vz, ids = o.state(ELECTRON)
    Ng = cfg["p_torr"] * TORR / (KB * cfg["Tg"])
    v0 = math.sqrt(eps0 / C_EPS)
    s = _sigmas(cfg, eps0)
    pn, numax = o.constant("P_null"), o.constant("nu_max")
    for code, sk in zip((EV_ELASTIC, EV_EXCITE, EV_IONIZE), s):
        assert _binom_ok(int((ev == code).sum()), n, pn * Ng * sk * v0 / numax)
    assert _binom_ok(int((ev == EV_NULL).sum()), n, pn * (1 - Ng * sum(s) * v0 / numax))
    assert int((ev == EV_NONE).sum()) + int((ev > 0).sum()) == n

    byid = {int(i): k for k, i in enumerate(ids)}
    eps = C_EPS * (vx * vx + vy * vy + vz * vz)
    M = cfg["M_amu"] * AMU
    # elastic: |v'|^2 / |v|^2 = 1 - (2m/M)(1 - cos chi) with cos chi from the
    # pre- and post-collision directions
    for i in np.where(ev == EV_ELASTIC)[0][:500]:
        k = byid[i]
        cosx = vx[k] / math.sqrt(vx[k] ** 2 + vy[k] ** 2 + vz[k] ** 2)
        assert abs(eps[k] / eps0 - (1 - 2 * ME / M * (1 - cosx))) < 1e-12
    # excitation: exactly the threshold is lost
    exc = np.where(ev == EV_EXCITE)[0]
    assert len(exc) > 10
    for i in exc:
        assert abs(eps[byid[i]] - (eps0 - cfg["ex_U"])) < 1e-12 * eps0
    # ionization: scattered + ejected = eps - U_iz, one new pair per event
    iz = np.sort(np.where(ev == EV_IONIZE)[0])
    assert len(iz) > 10
    assert o.count(ELECTRON) == n + len(iz)
    assert o.count(ION) == 1 + len(iz)
    assert o.next_id(ELECTRON) == n + len(iz)
    xi, vxi, vyi, vzi, idi = o.state(ION)
    ibyid = {int(i): k for k, i in enumerate(idi)}
    M_ = cfg["M_amu"] * AMU
    vi2 = []
    for r, pid in enumerate(iz):
        kp = byid[pid]
        kn = byid[n + r]                 # ejected electron id = next id + rank
        assert x[kn] == x[kp]
        assert abs(eps[kp] + eps[kn] - (eps0 - cfg["iz_U"])) < 1e-12 * eps0
        assert eps[kn] <= 0.5 * (eps0 - cfg["iz_U"]) * (1 + 1e-12)
        ki = ibyid[1 + r]                # new ion id = next ion id + rank
        assert xi[ki] == x[kp]
        vi2.append(vxi[ki] ** 2 + vyi[ki] ** 2 + vzi[ki] ** 2)
    # new ions are at the gas temperature: <v^2> = 3 kT / M
    t = np.mean(vi2) * M_ / (3 * KB)
    assert abs(t / cfg["Tg"] - 1) < 5 * math.sqrt(2 / 3 / len(vi2)) + 0.02


def test_isotropic_scattering_and_energy_sharing_law():
    cfg = _field_free(ppc=2000, eps_cap=100.0, ex_smax=0.0, el_A=0.0, el_B=1e-21,
                      iz_smax=3e-20)
    o = Oracle(cfg, init=False)
    rng = np.random.default_rng(8)
    n = 200000
    eps0 = 70.0
    _beam(o, n, eps0, cfg["L"], rng)
    o.set_state(ION, np.array([0.001]), *np.zeros((3, 1)), np.zeros(1, dtype=np.uint32))
    o.set_counters(1, n, 1)
    o.step(1)
    ev = o.events(ELECTRON, n)
    x, vx, vy, vz, ids = o.state(ELECTRON)
    sel = np.isin(ids, np.where(ev > 0)[0][np.isin(ev[ev > 0], [EV_ELASTIC, EV_IONIZE])])
    v = np.sqrt(vx[sel] ** 2 + vy[sel] ** 2 + vz[sel] ** 2)
    m = sel.sum()
    assert m > 2000
    for comp in (vx[sel], vy[sel], vz[sel]):
        c = comp / v
        assert abs(c.mean()) < 5 / math.sqrt(3 * m)
        assert abs((c * c).mean() - 1 / 3) < 5 * math.sqrt(4 / 45 / m)
    # ejected energies follow the Opal-Peterson-Beaty law truncated at er/2
    new = ids >= n
    ej = C_EPS * (vx[new] ** 2 + vy[new] ** 2 + vz[new] ** 2)
    w = cfg["opb_w"]
    er = eps0 - cfg["iz_U"]
    cdf = lambda e: np.arctan(np.asarray(e) / w) / math.atan(er / (2 * w))
    assert ej.size > 200
    assert scipy.stats.kstest(ej, cdf).pvalue > 1e-4


def test_equal_energy_sharing_mode():
    cfg = _field_free(ppc=100, energy_sharing="equal", el_A=0.0, el_B=0.0, ex_smax=0.0,
                      iz_smax=3e-20)
    o = Oracle(cfg, init=False)
    rng = np.random.default_rng(9)
    n = 20000
    _beam(o, n, 50.0, cfg["L"], rng)
    o.set_state(ION, np.array([0.001]), *np.zeros((3, 1)), np.zeros(1, dtype=np.uint32))
    o.set_counters(1, n, 1)
    o.step(1)
    x, vx, vy, vz, ids = o.state(ELECTRON)
    ev = o.events(ELECTRON, n)
    eps = C_EPS * (vx * vx + vy * vy + vz * vz)
    iz_ids = set(np.where(ev == EV_IONIZE)[0].tolist())
    half = 0.5 * (50.0 - cfg["iz_U"])
    touched = np.array([int(i) in iz_ids or i >= n for i in ids])
    assert touched.sum() > 20
    assert np.abs(eps[touched] - half).max() < 1e-12 * 50


def test_charge_exchange_rate_and_acceptance_bias():
    # ions at rest: g = |v_atom|, so P(CX) = P_cx <|v_a|> / g_cap and the
    # accepted atoms are speed-weighted: <|v|^2> = <v^3>/<v> = 4 kT / M
    cfg = _field_free(ppc=100, el_A=0.0, el_B=0.0, ex_smax=0.0, iz_smax=0.0,
                      cx_sigma=4e-19, g_cap=2000.0)
    o = Oracle(cfg, init=False)
    n = 200000
    rng = np.random.default_rng(10)
    z = np.zeros(n)
    o.set_state(ION, rng.random(n) * cfg["L"], z, z, z, np.arange(n, dtype=np.uint32))
    o.set_state(ELECTRON, np.array([0.001]), *np.zeros((3, 1)), np.zeros(1, dtype=np.uint32))
    o.set_counters(0, 1, n)
    o.step(1)
    ev = o.events(ION, n)
    M = cfg["M_amu"] * AMU
    kT = KB * cfg["Tg"]
    mean_speed = math.sqrt(8 * kT / (math.pi * M))
    p = o.constant("P_cx") * mean_speed / cfg["g_cap"]
    k = int((ev == EV_CX).sum())
    assert _binom_ok(k, n, p)
    assert o.errors == 0
    x, vx, vy, vz, ids = o.state(ION)
    cx = np.isin(ids, np.where(ev == EV_CX)[0])
    v2 = (vx[cx] ** 2 + vy[cx] ** 2 + vz[cx] ** 2).mean()
    # relative sd of v^2 under the speed-weighted law: <v^5>/<v> / (4kT/M)^2 - 1 = 1
    assert abs(v2 / (4 * kT / M) - 1) < 5 / math.sqrt(k)


def test_charge_exchange_relaxes_to_gas_temperature():
    cfg = _field_free(ppc=100, el_A=0.0, el_B=0.0, ex_smax=0.0, iz_smax=0.0,
                      cx_sigma=3e-17, g_cap=12000.0, ion_subcycle=1, Ti0_K=3000.0)
    o = Oracle(cfg, init=False)
    n = 20000
    M = cfg["M_amu"] * AMU
    rng = np.random.default_rng(12)
    s = math.sqrt(KB * 3000.0 / M)
    o.set_state(ION, rng.random(n) * cfg["L"], *rng.normal(0, s, (3, n)),
                np.arange(n, dtype=np.uint32))
    o.set_state(ELECTRON, np.array([0.001]), *np.zeros((3, 1)), np.zeros(1, dtype=np.uint32))
    o.set_counters(0, 1, n)
    o.step(1000)
    assert o.errors == 0
    x, vx, vy, vz, ids = o.state(ION)
    T = M * (vx ** 2 + vy ** 2 + vz ** 2).mean() / (3 * KB)
    assert abs(T / cfg["Tg"] - 1) < 0.03


def test_radial_sink_survival():
    nu_w = 1e8
    cfg = W.tiny("periodic", V=0.0, poisson=0, ppc=400, nu_w=nu_w, wall_mode="fixed",
                 **{k: 0.0 for k in ("el_A", "el_B", "ex_smax", "iz_smax", "cx_sigma")})
    o = Oracle(cfg)
    n0e, n0i = o.count(ELECTRON), o.count(ION)
    o.step(200)
    p = math.exp(-nu_w * 200 * cfg["dt"])
    assert _binom_ok(n0e - o.count(ELECTRON), n0e, 1 - p)
    # ions are tested on their 10 subcycle steps with dt_i = 20 dt
    assert _binom_ok(n0i - o.count(ION), n0i, 1 - p)


def test_pair_creation_balance_without_losses():
    cfg = W.tiny("periodic", V=0.0037 * 8000.0, wall_mode="off", ppc=60, eps_cap=100.0)
    o = Oracle(cfg)
    ne0, ni0 = o.count(ELECTRON), o.count(ION)
    niz = 0
    for _ in range(150):
        o.step(1)
        niz += int((o.events(ELECTRON) == EV_IONIZE).sum())
    assert o.errors == 0
    assert o.count(ELECTRON) - ne0 == niz
    assert o.count(ION) - ni0 == niz
    assert o.next_id(ELECTRON) == ne0 + niz and o.next_id(ION) == ni0 + niz
    mom = o.moments(reset_iz=True)
    nc = cfg["n_cells"]
    assert mom[6 * nc:7 * nc].sum() == niz
    assert mom[:nc].sum() == o.count(ELECTRON) and mom[4 * nc:5 * nc].sum() == o.count(ION)


def test_initial_load_uniform_and_maxwellian():
    cfg = W.tiny("periodic", ppc=400)
    o = Oracle(cfg)
    x, vx, vy, vz, ids = o.state(ELECTRON)
    assert np.array_equal(ids, np.arange(ids.size, dtype=np.uint32))
    assert scipy.stats.kstest(x / cfg["L"], "uniform").pvalue > 1e-4
    s = math.sqrt(cfg["Te0_eV"] * QE / ME)
    for comp in (vy, vz):
        assert scipy.stats.kstest(comp / s, "norm").pvalue > 1e-4
    xi, vxi, vyi, vzi, idi = o.state(ION)
    si = math.sqrt(KB * cfg["Ti0_K"] / (cfg["M_amu"] * AMU))
    assert scipy.stats.kstest(vyi / si, "norm").pvalue > 1e-4
    assert not np.array_equal(x, xi)


def test_constant_frequency_swarm_balance():
    # elastic-only, constant frequency, light "atoms" (delta = 2m/M = 0.04).
    # Per step: push (v_x += a dt), then a real collision with probability p
    # replaces v by a vector of mean r v, r = mean over isotropic c of
    # sqrt(1 - delta(1-c)) c, and scales the energy by (1 - delta(1-c)).
    # Stationary means of the post-step state therefore satisfy
    #   w = (1 - p(1-r)) (w + a dt)
    #   <eps> = (1 - p delta) (<eps> + m a dt w + m a^2 dt^2 / 2)
    # (momentum and energy balance of the discrete scheme).
    M_amu = 50 * ME / AMU
    delta = 2 * ME / (M_amu * AMU)
    B = 1.0e-19
    E = 4000.0
    dt = 1e-11
    cfg = W.tiny("periodic", n_cells=10, L=0.001, V=E * 0.001, poisson=0, wall_mode="off",
                 el_A=0.0, el_B=B, el_p=-0.5, ex_smax=0.0, iz_smax=0.0, cx_sigma=0.0,
                 M_amu=M_amu, eps_cap=400.0, ppc=1, dt=dt)
    o = Oracle(cfg, init=False)
    Ng = cfg["p_torr"] * TORR / (KB * cfg["Tg"])
    nu = Ng * B / math.sqrt(C_EPS)
    p = o.constant("P_null") * nu / o.constant("nu_max")
    r = 0.5 * scipy.integrate.quad(lambda c: math.sqrt(1 - delta * (1 - c)) * c, -1, 1)[0]
    a = QE * E / ME
    q = p * (1 - r)
    w = a * dt / q - a * dt
    eps_J = (1 - p * delta) * (ME * a * dt * w + 0.5 * ME * (a * dt) ** 2) / (p * delta)
    n = 20000
    rng = np.random.default_rng(13)
    s = math.sqrt(2 / 3 * eps_J / ME)
    o.set_state(ELECTRON, rng.random(n) * 0.001, *rng.normal(0, s, (3, n)),
                np.arange(n, dtype=np.uint32))
    o.set_state(ION, np.array([0.0005]), *np.zeros((3, 1)), np.zeros(1, dtype=np.uint32))
    o.set_counters(1, n, 1)
    o.step(2000)
    ws, es = [], []
    for _ in range(200):
        o.step(10)
        _, vx, vy, vz, _ = o.state(ELECTRON)
        ws.append(vx.mean())
        es.append(0.5 * ME * (vx ** 2 + vy ** 2 + vz ** 2).mean())
    assert o.errors == 0
    assert abs(np.mean(ws) / w - 1) < 0.025
    assert abs(np.mean(es) / eps_J - 1) < 0.025


def test_balanced_sink_keeps_the_particle_number():
    """Balanced sink: a particle is removed with probability (ionizations
    since its species' previous step) / (count), so removals match births on
    average (the paper's constant particle number).  Over 400 steps of an
    ionizing column the counts stay within a few standard deviations of
    sqrt(total births) of the start, while the fixed sink lets them grow."""
    import workloads as W
    from oracle.pco import Oracle
    base = dict(n_cells=101, L=0.0101, V=0.0101 * 6.0e3, ppc=40, Te0_eV=8.0, ion_subcycle=4)
    o = Oracle(W.tiny("periodic", wall_mode="balanced", **base))
    n0 = (o.count(0), o.count(1))
    births = 0
    for _ in range(400):
        b0 = o.next_id(0)
        o.step(1)
        births += o.next_id(0) - b0
        bl, bs = o.balance()
        assert bl == o.next_id(0) - b0            # tally of the step just taken
    assert o.errors == 0 and births > 500
    tol = 5.0 * births ** 0.5
    assert abs(o.count(0) - n0[0]) <= tol, (o.count(0), n0, births)
    assert abs(o.count(1) - n0[1]) <= tol + births / 100, (o.count(1), n0, births)
    f = Oracle(W.tiny("periodic", wall_mode="fixed", nu_w=1e5, **base))
    for _ in range(400):
        f.step(1)
    assert f.count(0) - n0[0] > 0.5 * births
