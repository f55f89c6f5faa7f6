"""Determinism of the HIP path (race detection by bitwise comparison).

Charges are integer sums and every random draw is keyed by (id, step), so a
column's state as a set of particles is a function of the config alone: it
must not depend on the launch grid, the sort interval, graph replay versus
eager launches, or particle order.  Any race in the deposit, compaction,
birth or sort kernels shows up as a bitwise difference here.
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


def _run(cfg, steps, events=False):
    from paper_2202_03215_amd.column import Column
    col = Column(cfg)
    if events:
        col.set_events(4 * col.capacity, 4 * col.capacity)
    col.step(steps)
    c = col.counts()
    assert c["errors"] == 0
    states = [gpu_state(col, s) for s in (ELECTRON, ION)]
    E, re, ri = col.get_field()
    return c, states, E.cpu().numpy(), re.cpu().numpy(), ri.cpu().numpy()


def _same(a, b):
    ca, sa, Ea, rea, ria = a
    cb, sb, Eb, reb, rib = b
    assert ca["n"] == cb["n"] and ca["next_id"] == cb["next_id"] and ca["step"] == cb["step"]
    for s in (ELECTRON, ION):
        for k in range(5):
            assert np.array_equal(sa[s][k], sb[s][k]), (s, k)
    assert np.array_equal(rea, reb) and np.array_equal(ria, rib)
    assert np.array_equal(Ea, Eb)


BASE = dict(bc="periodic", n_cells=101, L=0.0101, V=0.0101 * 6.0e3, ppc=60, Te0_eV=8.0,
            nu_w=5e7, eps_cap=100.0)


def test_graph_replay_equals_eager_launches(torch_cuda):
    cfg = W.tiny(**BASE, sort_interval=3)           # graph period lcm(2, 40, 6) = 120
    a = _run(cfg, 240)
    b = _run(cfg, 240, events=True)                 # event recording forces eager launches
    assert a[0]["n"][0] != cfg["ppc"] * cfg["n_cells"]   # births / losses happened
    _same(a, b)


@pytest.mark.parametrize("variant", [dict(launch_blocks=7), dict(launch_blocks=333),
                                     dict(sort_interval=0), dict(sort_interval=1)])
def test_launch_grid_and_sort_interval_invariance(torch_cuda, variant):
    cfg = W.tiny(**BASE, sort_interval=10)
    ref = _run(cfg, 160)
    alt = _run(W.with_(cfg, **variant), 160)
    _same(ref, alt)


def test_bounded_column_repeatable(torch_cuda):
    cfg = W.small_bounded()
    _same(_run(cfg, 200), _run(cfg, 200))


def test_remainder_graphs_equal_eager_launches(torch_cuda):
    """Step counts that are not whole graph periods replay a graph per
    (phase, length), some captured ahead by prepare_graphs: bitwise the same
    as eager launches."""
    from paper_2202_03215_amd.column import Column
    cfg = W.tiny(**BASE, sort_interval=3)           # graph period 120
    col = Column(cfg)
    col.prepare_graphs(37)
    for n in (37, 5, 1, 1, 130, 77, 37):            # 288 steps in pieces
        col.step(n)
    c = col.counts()
    assert c["errors"] == 0
    E, re, ri = col.get_field()
    a = (c, [gpu_state(col, s) for s in (ELECTRON, ION)], E.cpu().numpy(), re.cpu().numpy(), ri.cpu().numpy())
    _same(a, _run(cfg, 288, events=True))
