"""Checkpoint/resume and device-error handling through the C ABI (GPU).

- Resume: a column stepped 2N steps equals, bit for bit, a column stepped N
  steps whose state (particles, field E^n, step index, next ids, sink
  tallies) is then copied into a freshly initialised column that steps N
  more.  Counter-based draws keyed by (id, step) and order-free integer
  charges make the particle order of the restored arrays irrelevant.  (FP32
  columns exchange their state as FP64 positions and velocities, so their
  restart goes through a conversion and is not covered here.)
- Errors: an electron above the collision bound eps_cap sets a device error
  bit; pc_sync maps it to PC_ERR_ECAP and poisons the handle, pc_step then
  returns PC_ERR_POISONED, and pc_set_state with a valid state clears it.
  A position outside [0, L) is refused by pc_set_state itself.  Every
  kernel runs to completion in these cases (the checks are flags, not traps).
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import ELECTRON, ION, gpu_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _snap(col):
    c = col.counts()
    E, re, ri = col.get_field()
    return c, [gpu_state(col, s) for s in (ELECTRON, ION)], E.cpu().numpy(), ri.cpu().numpy()


def _restore(src, dst, torch):
    c = src.counts()
    for s in (ELECTRON, ION):
        x, vx, vy, vz, ids = src.get_state(s)
        dst.set_state(s, x, vx, vy, vz, ids)
    E, _, _ = src.get_field()
    dst.set_field(E)
    dst.set_counters(c["step"], c["next_id"][0], c["next_id"][1])
    dst.set_balance(*c["balance"])
    dst.set_circuit(*c["circuit"])


@pytest.mark.parametrize("case", ["balanced", "pair", "section_v"])
def test_resume_is_bitwise(torch_cuda, case):
    from paper_2202_03215_amd.column import Column
    base = dict(bc="periodic", n_cells=101, L=0.0101, V=0.0101 * 6.0e3, ppc=60, Te0_eV=8.0, eps_cap=100.0,
                sort_interval=7)
    if case == "section_v":
        cfg = W.with_(W.hot_cathode_15cm(ppc=20), n_cells=150, L=0.015, V=60.0)
    else:
        cfg = W.tiny(**base, wall_mode="pair" if case == "pair" else "balanced")
    N = 150
    a = Column(cfg)
    a.step(2 * N)
    b = Column(cfg)
    b.step(N)
    c = Column(cfg)
    _restore(b, c, torch_cuda)
    c.step(N)
    sa, sc = _snap(a), _snap(c)
    assert sa[0]["errors"] == 0 and sc[0]["errors"] == 0
    for k in ("n", "next_id", "step", "balance"):
        assert sa[0][k] == sc[0][k], k
    assert sa[0]["circuit"] == sc[0]["circuit"]
    for s in (ELECTRON, ION):
        for k in range(5):
            assert np.array_equal(sa[1][s][k], sc[1][s][k]), (case, s, k)
    assert np.array_equal(sa[2], sc[2]) and np.array_equal(sa[3], sc[3])


def test_device_error_poisons_and_set_state_clears(torch_cuda):
    from paper_2202_03215_amd import native as N
    from paper_2202_03215_amd.column import Column
    torch = torch_cuda
    cfg = W.tiny("periodic", n_cells=37, L=0.0037, V=0.0, ppc=29, wall_mode="off", eps_cap=100.0)
    col = Column(cfg)
    col.step(3)
    col.sync()
    x, vx, vy, vz, ids = col.get_state(ELECTRON)
    # every electron at 400 eV (eps_cap is 100 eV): the collision candidates flag it
    hot = torch.full_like(vx, (400.0 / (0.5 * 9.1093837015e-31 / 1.602176634e-19)) ** 0.5)
    z = torch.zeros_like(vx)
    col.set_state(ELECTRON, x, hot, z, z, ids)
    col.step(20)
    with pytest.raises(N.PcError) as e:
        col.sync()
    assert e.value.status == -5                     # PC_ERR_ECAP
    with pytest.raises(N.PcError) as e:
        col.step(1)
    assert e.value.status == -8                     # PC_ERR_POISONED
    col.set_state(ELECTRON, x, vx, vy, vz, ids)     # a valid state clears the handle
    col.step(10)
    col.sync()
    assert col.counts()["errors"] == 0


def test_set_state_refuses_positions_outside_the_column(torch_cuda):
    from paper_2202_03215_amd import native as N
    from paper_2202_03215_amd.column import Column
    cfg = W.tiny("periodic", n_cells=37, L=0.0037, V=0.0, ppc=29, wall_mode="off")
    col = Column(cfg)
    x, vx, vy, vz, ids = col.get_state(ELECTRON)
    bad = x.clone()
    bad[5] = cfg["L"] * 1.5
    with pytest.raises(N.PcError):
        col.set_state(ELECTRON, bad, vx, vy, vz, ids)
    with pytest.raises(N.PcError) as e:
        col.step(1)
    assert e.value.status == -8
    col.set_state(ELECTRON, x, vx, vy, vz, ids)
    col.step(5)
    col.sync()
