"""Pins of the oracle's bounded column of section V: cathode emission and the
external circuit.

- An empty gap (no particles) with a resistor is an RC circuit: the backward-
  Euler recurrence V' (1 + a) = U + a V, a = R eps0 / (L dt), has the closed
  form V_n = U + (V_0 - U) (a / (1 + a))^n, and the field of the empty gap is
  the Laplace field -V_n / L.
- With R = 0 the anode stays at U.
- Emission: J dt / (e W) electrons per step on average (the carried
  fraction makes the total exact to within one); v_x follows the Rayleigh
  law of a flux-weighted half-Maxwellian at T_c (Kolmogorov-Smirnov), v_y and
  v_z are normal with variance e T_c / m, and each starts in [0, v_x dt).
"""
import math

import numpy as np
from scipy import stats

import workloads as W
from oracle.pco import Oracle

QE, ME, EPS0 = 1.602176634e-19, 9.1093837015e-31, 8.8541878128e-12


def _empty(cfg):
    o = Oracle(cfg)
    z = np.zeros(0)
    for s in (0, 1):
        o.set_state(s, z, z, z, z, np.zeros(0, dtype=np.uint32))
    return o


def test_empty_gap_relaxes_as_an_rc_circuit():
    cfg = W.with_(W.small_bounded(), circuit_R=2.0)
    o = _empty(cfg)
    V0 = 5.0
    o.set_circuit(V0, 0, 0.0)
    a = cfg["circuit_R"] * EPS0 / (cfg["L"] * cfg["dt"])
    U = cfg["V"]
    for n in range(1, 301):
        o.step(1)
        V = o.circuit()["V_anode"]
        expect = U + (V0 - U) * (a / (1.0 + a)) ** n
        assert abs(V - expect) <= 1e-12 * U, (n, V, expect)
        assert o.circuit()["J_cond"] == 0.0
    E, _, _ = o.field()
    assert np.abs(E + V / cfg["L"]).max() <= 1e-12 * V / cfg["L"]
    assert abs(V - U) < 0.3 * abs(V0 - U)           # a few time constants R eps0 / L


def test_without_resistor_the_anode_stays_at_the_source():
    cfg = W.with_(W.small_bounded(), emit_J=10.0)
    o = Oracle(cfg)
    o.step(30)
    assert o.circuit()["V_anode"] == cfg["V"]


def test_emission_count_and_velocity_distribution():
    cfg = W.with_(W.small_bounded(), emit_J=40.0, emit_T=0.5, nu_w=0.0, wall_mode="off")
    o = Oracle(cfg)
    W_ = cfg["n0"] * (cfg["L"] / cfg["n_cells"]) / cfg["ppc"]
    per_step = cfg["emit_J"] * cfg["dt"] / (QE * W_)
    sig = math.sqrt(QE * cfg["emit_T"] / ME)
    vx, vy, vz, x0 = [], [], [], []
    total = 0
    steps = 300
    for _ in range(steps):
        before = o.next_id(0)
        o.step(1)
        ev = o.events(0, before)
        births = int(np.sum(ev == 3))
        x, ux, uy, uz, ids = o.state(0)
        new = ids >= before + births                  # emitted: ids after the products'
        total += int(new.sum())
        vx.append(ux[new]); vy.append(uy[new]); vz.append(uz[new]); x0.append(x[new])
    assert abs(total - steps * per_step) < 1.0 + 1e-9 * steps * per_step, (total, steps * per_step)
    vx, vy, vz, x0 = (np.concatenate(a) for a in (vx, vy, vz, x0))
    assert vx.size > 2000
    assert stats.kstest(vx / sig, "rayleigh").pvalue > 1e-3
    for v in (vy, vz):
        assert stats.kstest(v / sig, "norm").pvalue > 1e-3
    assert np.all(x0 >= 0.0) and np.all(x0 < vx * cfg["dt"])
