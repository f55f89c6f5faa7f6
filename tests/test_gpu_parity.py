"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

- deposit: int64 fixed-point charge bitwise identical, in any particle order;
- field solve: |dE| <= 1e-12 max|E|, |dphi| <= 1e-12 max(max|phi|, V);
- initial load: positions, ids and charges bitwise, velocities to 1e-12;
- full step from a shared state (the oracle is given the GPU state before
  every step): identical event per particle id, identical id sets, positions
  within 1e-12 L, velocities within 1e-12 (|v| + v_th), charges bitwise,
  field to 1e-12.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle.pco import Oracle
from tests.gpu_helpers import (ELECTRON, ION, by_id, compare_states, copy_gpu_to_oracle,
                               field_close, gpu_state)

pytestmark = pytest.mark.gpu

QE = 1.602176634e-19
ME = 9.1093837015e-31
AMU = 1.66053906660e-27
KB = 1.380649e-23


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _column(cfg):
    from paper_2202_03215_amd.column import Column
    return Column(cfg)


def _vth(cfg):
    return (math.sqrt(max(cfg["Te0_eV"], 1.0) * QE / ME),
            math.sqrt(KB * cfg["Tg"] / (cfg["M_amu"] * AMU)))


# ------------------------------------------------------------------ deposit
@pytest.mark.parametrize("bc", ["bounded", "periodic"])
@pytest.mark.parametrize("n", [0, 1, 63, 1000, 100_003])
def test_deposit_bitwise(torch_cuda, bc, n):
    torch = torch_cuda
    cfg = W.tiny(bc=bc, n_cells=400, L=0.04, V=40.0)
    col = _column(cfg)
    orc = Oracle(cfg, init=False)
    x = W.random_positions(n, cfg["L"], seed=n + 7)
    g = col.deposit(torch.from_numpy(x)).cpu().numpy()
    o = orc.deposit(x)
    assert np.array_equal(g, o)
    if n > 1:
        perm = np.random.default_rng(1).permutation(n)
        g2 = col.deposit(torch.from_numpy(x[perm])).cpu().numpy()
        assert np.array_equal(g2, o)
    assert g.sum() == n << 25


# -------------------------------------------------------------- field solve
@pytest.mark.parametrize("bc", ["bounded", "periodic"])
@pytest.mark.parametrize("nc", [37, 400, 2000, 5000, 8000, 8191])   # 8191: 8192 bounded nodes, the maximum
def test_field_solve(torch_cuda, bc, nc):
    torch = torch_cuda
    L = nc * 1e-4
    cfg = W.tiny(bc=bc, n_cells=nc, L=L, V=L * 1000.0, ppc=2)
    col = _column(cfg)
    orc = Oracle(cfg, init=False)
    nn = col.nn
    for seed in (1, 2):
        re, ri = W.charge_profile(nn, seed=seed + nc)
        phi_g, E_g = col.solve_field(torch.from_numpy(re), torch.from_numpy(ri))
        phi_o, E_o = orc.solve_field(re, ri)
        E_g = E_g.cpu().numpy()
        phi_g = phi_g.cpu().numpy()
        assert np.abs(E_g - E_o).max() <= 1e-12 * np.abs(E_o).max()
        scale = max(np.abs(phi_o).max(), abs(cfg["V"]))
        assert np.abs(phi_g - phi_o).max() <= 1e-12 * scale


@pytest.mark.parametrize("bc", ["bounded", "periodic"])
@pytest.mark.parametrize("one_signed", [False, True])
def test_field_solve_large_charges(torch_cuda, bc, one_signed):
    # node charges up to 2^45 units on the 8192-node maximum: the potential
    # constant's weighted sum (n_c - k) Q_k reaches 2^58 per term, beyond the
    # 53-bit mantissa, and the integer prefix sums reach 2^58; one-signed: a
    # net charge of 2^58 units (a column of electrons only)
    torch = torch_cuda
    nc = 8191
    L = nc * 1e-4
    cfg = W.tiny(bc=bc, n_cells=nc, L=L, V=L * 1000.0, ppc=2)
    col = _column(cfg)
    orc = Oracle(cfg, init=False)
    re, ri = W.charge_profile(col.nn, seed=5, scale=1 << 45)
    if one_signed:
        ri = np.zeros_like(ri)
    phi_g, E_g = col.solve_field(torch.from_numpy(re), torch.from_numpy(ri))
    phi_o, E_o = orc.solve_field(re, ri)
    E_g = E_g.cpu().numpy()
    phi_g = phi_g.cpu().numpy()
    assert np.abs(E_g - E_o).max() <= 1e-12 * np.abs(E_o).max()
    scale = max(np.abs(phi_o).max(), abs(cfg["V"]))
    assert np.abs(phi_g - phi_o).max() <= 1e-12 * scale


@pytest.mark.parametrize("bc", ["bounded", "periodic"])
def test_field_zero_charge(torch_cuda, bc):
    torch = torch_cuda
    cfg = W.tiny(bc=bc, n_cells=400, L=0.04, V=40.0, ppc=2)
    col = _column(cfg)
    z = torch.zeros(col.nn, dtype=torch.int64)
    phi, E = col.solve_field(z, z)
    assert np.abs(E.cpu().numpy() + 1000.0).max() <= 1e-12 * 1000.0


# --------------------------------------------------------------- init / load
@pytest.mark.parametrize("cfg", [W.small_bounded(), W.tiny("periodic")],
                         ids=["small_bounded", "tiny_periodic"])
def test_initial_load(torch_cuda, cfg):
    col = _column(cfg)
    orc = Oracle(cfg)
    c = col.counts()
    assert c["n"] == (orc.count(0), orc.count(1))
    assert c["step"] == 0 and c["errors"] == 0
    compare_states(col, orc, cfg["L"], _vth(cfg))
    for s in (ELECTRON, ION):
        g = gpu_state(col, s)
        o = by_id(orc.state(s))
        assert np.array_equal(g[0], o[0])            # positions: no transcendental
    Eg, reg, rig = col.get_field()
    Eo, reo, rio = orc.field()
    assert np.array_equal(reg.cpu().numpy(), reo) and np.array_equal(rig.cpu().numpy(), rio)
    assert field_close(Eg.cpu().numpy(), Eo)


# ------------------------------------------------------- per-step parity (P5)
def _run_shared_state(torch, cfg, steps, min_events=None, setup=None, check=None):
    col = _column(cfg)
    orc = Oracle(cfg, init=False)
    if setup is not None:
        setup(col)
    cap = col.capacity
    ev_e, ev_i = col.set_events(4 * cap, 4 * cap)
    tot = np.zeros(8, dtype=np.int64)
    vth = _vth(cfg)
    for k in range(steps):
        copy_gpu_to_oracle(col, orc)
        ev_e.zero_()
        ev_i.zero_()
        col.step(1)
        orc.step(1)
        c = col.counts()
        assert c["errors"] == 0, f"device error bits {c['errors']} at step {k}"
        assert orc.errors == 0
        assert c["n"] == (orc.count(0), orc.count(1)), f"step {k}"
        assert c["next_id"] == (orc.next_id(0), orc.next_id(1)), f"step {k}"
        for s, ev in ((ELECTRON, ev_e), (ION, ev_i)):
            n = orc.next_id(s)
            ge = ev[:n].cpu().numpy()
            oe = orc.events(s, n)
            bad = np.where(ge != oe)[0]
            assert bad.size == 0, f"step {k} species {s}: events differ at ids {bad[:10]}"
            if s == ELECTRON:
                tot += np.bincount(oe, minlength=8)
        compare_states(col, orc, cfg["L"], vth)
        Eg, reg, rig = col.get_field()
        Eo, reo, rio = orc.field()
        assert np.array_equal(reg.cpu().numpy(), reo), f"step {k}: electron charge"
        assert np.array_equal(rig.cpu().numpy(), rio), f"step {k}: ion charge"
        assert field_close(Eg.cpu().numpy(), Eo), f"step {k}: field"
        if check is not None:
            check(col, orc, k)
    if min_events:
        for code, m in min_events.items():
            assert tot[code] >= m, f"only {tot[code]} events of type {code}: {tot}"
    return tot


def test_step_parity_column_20cm_full_size(torch_cuda):
    # the bench's workload in the bench's launch grid (400k + 400k particles,
    # 2000 cells, one initial particle per thread): 38 steps on the GPU alone
    # (births, losses, the sort and ion step at 20), then steps 38-40 from the
    # shared state (the sort after step 39, the ion step 40), every particle
    # compared
    cfg = W.column_20cm()
    _run_shared_state(torch_cuda, cfg, steps=3, setup=lambda col: col.step(38), min_events={1: 1000, 7: 10000})


def test_step_parity_column_50cm_full_size(torch_cuda):
    # the large column (5M + 5M particles, 5000 cells, 4096 blocks of about
    # five tiles, the finish with 768 threads): steps 19 and 20 from the
    # shared state after 19 steps alone (step 19 ends with the sort, step 20
    # is an ion step)
    cfg = W.column_50cm()
    _run_shared_state(torch_cuda, cfg, steps=2, setup=lambda col: col.step(19), min_events={1: 1000, 7: 50000})


def test_step_parity_small_bounded_all_2000_steps(torch_cuda):
    # the small workload's whole run (neon, 4 cm, 400 cells, 50 per cell,
    # grounded cathode / 40 V anode, 2000 steps): every step from the shared
    # state, every particle, event, charge and the field
    tot = _run_shared_state(torch_cuda, W.small_bounded(), steps=2000,
                            min_events={1: 100000, 2: 50, 3: 5, 4: 10, 5: 2000})
    print("events over 2000 steps", tot)


def test_step_parity_periodic_ionizing(torch_cuda):
    # strong field: many excitations and ionizations; fast sink: many losses
    cfg = W.tiny("periodic", n_cells=101, L=0.0101, V=0.0101 * 6.0e3, ppc=40,
                 Te0_eV=8.0, nu_w=2e8, eps_cap=100.0, sort_interval=3)
    _run_shared_state(torch_cuda, cfg, steps=45, min_events={1: 20, 2: 5, 3: 5, 4: 5})


@pytest.mark.parametrize("nc", [5000, 7000])
def test_step_parity_many_nodes(torch_cuda, nc):
    # long grids: the finish kernel runs with 768 (5000 nodes) and 1024 (7000
    # nodes) threads, more than the 512 of the shorter columns
    # (6 eV: no electron of the initial 20k-28k reaches the 100 eV cap)
    cfg = W.tiny("periodic", n_cells=nc, L=nc * 1e-4, V=nc * 1e-4 * 6.0e3, ppc=4,
                 Te0_eV=6.0, nu_w=2e8, eps_cap=100.0, sort_interval=3)
    _run_shared_state(torch_cuda, cfg, steps=8, min_events={1: 20, 3: 3, 4: 3})


def test_step_parity_equal_sharing_and_ions(torch_cuda):
    cfg = W.tiny("bounded", n_cells=64, L=0.0064, V=40.0, ppc=50, Te0_eV=8.0,
                 energy_sharing="equal", ion_subcycle=2, nu_w=5e7, Ti0_K=3000.0,
                 sort_interval=5)
    _run_shared_state(torch_cuda, cfg, steps=30, min_events={3: 3, 5: 3})


def test_step_parity_balanced_sink(torch_cuda):
    # removal probability from the previous step's ionizations (electrons) and
    # from those since the last ion step (ions, subcycle 3)
    cfg = W.tiny("periodic", n_cells=101, L=0.0101, V=0.0101 * 6.0e3, ppc=40, Te0_eV=8.0,
                 wall_mode="balanced", ion_subcycle=3, sort_interval=4)
    tot = _run_shared_state(torch_cuda, cfg, steps=40, min_events={3: 20, 4: 20})
    assert tot[4] > 0


def test_step_parity_pair_sink(torch_cuda):
    # the paper's own sink: per ionization a random electron and ion leave
    # and the products take their slots and ids; the GPU arrays are first
    # stored in a shuffled order (the id -> slot map is rebuilt from them)
    cfg = W.tiny("periodic", n_cells=101, L=0.0101, V=0.0101 * 6.0e3, ppc=40, Te0_eV=6.0,
                 wall_mode="pair", ion_subcycle=3, sort_interval=4)

    def setup(col):
        rng = np.random.default_rng(2)
        for s in (ELECTRON, ION):
            x, vx, vy, vz, ids = (a.cpu().numpy() for a in col.get_state(s))
            p = rng.permutation(x.size)
            col.set_state(s, x[p], vx[p], vy[p], vz[p], ids[p])

    tot = _run_shared_state(torch_cuda, cfg, steps=40, setup=setup, min_events={1: 50, 3: 20})
    assert tot[4] == 0


def test_step_parity_hot_cathode_and_circuit(torch_cuda):
    # section V: cathode emission (10 A/m^2, about 3 electrons per step) and
    # a 10 ohm m^2 series resistor; ions every 4 steps (their held current)
    cfg = W.with_(W.small_bounded(), emit_J=10.0, emit_T=0.5, circuit_R=10.0, nu_w=1.0e6, ion_subcycle=4)
    seen = []

    def check(col, orc, k):
        g = col.counts()
        o = orc.circuit()
        V, vs, carry = g["circuit"]
        assert abs(V - o["V_anode"]) <= 1e-12 * abs(cfg["V"]), (k, V, o["V_anode"])
        assert abs(g["J_cond"] - o["J_cond"]) <= 1e-12 * max(abs(o["J_cond"]), 1.0), k
        assert vs == o["vsum_ion"] and carry == o["emit_carry"], k
        seen.append((g["next_id"][0], V))

    _run_shared_state(torch_cuda, cfg, steps=40, check=check, min_events={1: 20})
    assert seen[-1][0] - seen[0][0] >= 100               # emitted electrons took new ids
    assert abs(seen[-1][1] - cfg["V"]) > 0.01             # the resistor moved the anode potential


def test_step_parity_full_size_pair_sink_and_hot_cathode(torch_cuda):
    # the bench's pair-sink leg (the 20 cm column with the paper's pair
    # removal, 400k + 400k) and its section V leg (the 15 cm bounded column
    # with emission and the series resistor, 150k + 150k): three shared-state
    # steps each after 38 steps alone, every particle compared
    cfg = W.with_(W.column_20cm(), wall_mode="pair")
    _run_shared_state(torch_cuda, cfg, steps=3, setup=lambda col: col.step(38), min_events={1: 1000})
    hc = W.hot_cathode_15cm()

    def check(col, orc, k):
        g = col.counts()
        o = orc.circuit()
        assert abs(g["circuit"][0] - o["V_anode"]) <= 1e-12 * abs(hc["V"]), k
        assert g["circuit"][1] == o["vsum_ion"] and g["circuit"][2] == o["emit_carry"], k

    _run_shared_state(torch_cuda, hc, steps=3, setup=lambda col: col.step(38), check=check, min_events={1: 100})


@pytest.mark.parametrize("bc", ["bounded", "periodic"])
def test_empty_column_steps(torch_cuda, bc):
    # no particles at all: every kernel sees empty chunks; the field is the
    # Laplace field of the gap (bounded: the anode relaxes through the series
    # resistor as an RC circuit, V_n = U + (V_0 - U) (a / (1 + a))^n)
    cfg = W.tiny(bc, n_cells=400, L=0.04, V=40.0, ppc=2,
                 **({"circuit_R": 2.0} if bc == "bounded" else {}))
    col = _column(cfg)
    orc = Oracle(cfg, init=False)
    z = np.zeros(0)
    zi = np.zeros(0, dtype=np.uint32)
    for s in (ELECTRON, ION):
        col.set_state(s, z, z, z, z, zi)
        orc.set_state(s, z, z, z, z, zi)
    V0 = 5.0 if bc == "bounded" else cfg["V"]
    col.set_circuit(V0, 0, 0.0)
    orc.set_circuit(V0, 0, 0.0)
    a = cfg.get("circuit_R", 0.0) * 8.8541878128e-12 / (cfg["L"] * cfg["dt"])
    for n in range(1, 51):
        col.step(1)
        orc.step(1)
        c = col.counts()
        assert c["errors"] == 0 and c["n"] == (0, 0)
        Eg = col.get_field()[0].cpu().numpy()
        Eo = orc.field()[0]
        assert np.abs(Eg - Eo).max() <= 1e-12 * np.abs(Eo).max()
        if bc == "bounded":
            V = c["circuit"][0]
            expect = cfg["V"] + (V0 - cfg["V"]) * (a / (1.0 + a)) ** n
            assert abs(V - expect) <= 1e-12 * cfg["V"] and abs(V - orc.circuit()["V_anode"]) <= 1e-13 * cfg["V"]
            assert np.abs(Eg[:col.nn] + V / cfg["L"]).max() <= 1e-12 * V / cfg["L"]
        else:
            assert np.abs(Eg[:col.nn] + cfg["V"] / cfg["L"]).max() <= 1e-12 * cfg["V"] / cfg["L"]


def test_step_parity_long_loss_and_birth_lists(torch_cuda):
    # more than 2048 losses and ionizations in one step: the finish kernel
    # takes its global-scratch paths instead of the LDS lists
    torch = torch_cuda
    n = 80_000
    cfg = W.tiny("periodic", n_cells=200, L=0.02, V=0.0, poisson=0, ppc=600, Te0_eV=2.0,
                 nu_w=3e9, ion_subcycle=1, iz_smax=3.2e-20, el_B=1e-21, eps_cap=100.0,
                 capacity=2.0, sort_interval=2)

    def setup(col):
        rng = np.random.default_rng(5)
        v = math.sqrt(85.0 * QE / ME * 2.0)
        d = rng.normal(size=(3, n))
        d /= np.linalg.norm(d, axis=0)
        x = rng.random(n) * cfg["L"]
        col.set_state(ELECTRON, x, v * d[0], v * d[1], v * d[2], np.arange(n))
        s = math.sqrt(KB * 300.0 / (cfg["M_amu"] * AMU))
        xi = rng.random(n) * cfg["L"]
        col.set_state(ION, xi, *rng.normal(0.0, s, (3, n)), np.arange(n))
        col.set_counters(1, n, n)
        col.set_field(np.zeros(col.nn))

    tot = _run_shared_state(torch, cfg, steps=2, setup=setup)
    assert tot[3] > 2 * 2048, tot      # ionizations over the two steps
    assert tot[4] > 2 * 2048, tot      # radial losses


# ---------------------------------------------------------------- moments
def test_moments_bitwise(torch_cuda):
    # cell moments (counts, energy / flux sums, EEPF histogram, ionization
    # counts) of the same state are integers: identical on both sides
    cfg = W.tiny("periodic", n_cells=101, L=0.0101, V=0.0101 * 6.0e3, ppc=60, Te0_eV=8.0,
                 nu_w=5e7, eps_cap=100.0, sort_interval=3)
    col = _column(cfg)
    orc = Oracle(cfg, init=False)
    col.step(25)
    col.moments(cells_per_group=4, reset_iz=True)
    for k in range(3):
        copy_gpu_to_oracle(col, orc)
        orc.moments(reset_iz=True)
        col.step(1)
        orc.step(1)
        for cpg in (1, 4, 101):
            g = col.moments(cells_per_group=cpg).cpu().numpy()
            o = orc.moments(cells_per_group=cpg)
            nc = cfg["n_cells"]
            assert np.array_equal(g[:6 * nc], o[:6 * nc])
            assert np.array_equal(g[7 * nc:], o[7 * nc:])
            assert np.array_equal(g[6 * nc:7 * nc], o[6 * nc:7 * nc])
        col.moments(cells_per_group=1, reset_iz=True)
    assert g[:nc].sum() == col.counts()["n"][0]
