"""Pins of the oracle's pair sink (section II: for every ionization one
electron and one ion, chosen at random over the column, are removed, so that
the particle numbers stay constant).

- the counts stay at N0 and the ids stay a permutation of 0..N0-1 (products
  take over the victims' ids), with the exact charge sum of N0 particles;
- one victim per ionization and species, all distinct within a step;
- victims are uniform over the ids (chi-square over bins) and over the
  column (left and right halves, binomial);
- the choice depends on ids only: the same state stored in another array
  order gives the same victims and the same particles by id.
"""
import numpy as np

import workloads as W
from oracle.pco import Oracle

def _cfg(**kw):
    base = dict(n_cells=101, L=0.0101, V=0.0101 * 6.0e3, ppc=40, Te0_eV=8.0, eps_cap=100.0,
                wall_mode="pair", sort_interval=3)
    base.update(kw)
    return W.tiny("periodic", **base)


def _by_id(o, s):
    x, vx, vy, vz, ids = o.state(s)
    order = np.argsort(ids)
    return ids[order], np.stack([x, vx, vy, vz])[:, order]


def test_counts_ids_and_charge_stay_fixed():
    cfg = _cfg()
    o = Oracle(cfg)
    n0 = o.count(0)
    births = 0
    for _ in range(60):
        o.step(1)
        ev = o.events(0, o.next_id(0))
        nb = int(np.sum(ev == 3))
        births += nb
        for s in (0, 1):
            assert o.count(s) == n0 and o.next_id(s) == n0
            ids, _ = _by_id(o, s)
            assert np.array_equal(ids, np.arange(n0, dtype=ids.dtype))
            v = o.victims(s)
            assert v.size == nb and np.unique(v).size == nb
        _, re, ri = o.field()
        assert re.sum() == n0 << 25 and ri.sum() == n0 << 25
    assert o.errors == 0 and births >= 50


def test_victims_uniform_over_ids_and_column():
    cfg = _cfg(seed=7, Te0_eV=6.0)      # 6 eV: no electron reaches the 100 eV cap in 1500 steps
    o = Oracle(cfg)
    n0 = o.count(0)
    vic, left, total = [], 0, 0
    for _ in range(1500):
        # ion positions by id before the step (ions move only on subcycle
        # steps, and then by far less than a cell)
        x, _, _, _, ids = o.state(1)
        pos = np.empty(n0)
        pos[ids] = x
        o.step(1)
        v = o.victims(1)
        vic.append(v)
        left += int(np.sum(pos[v] < 0.5 * cfg["L"]))
        total += v.size
    ids = np.concatenate(vic).astype(np.int64)
    assert ids.size >= 1500 and o.errors == 0
    counts = np.bincount(ids * 10 // n0, minlength=10)
    expect = ids.size / 10.0
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    assert chi2 < 27.9, (chi2, counts)           # chi-square, 9 dof, p = 0.001
    # ions at rest between subcycle steps: left-half share binomial(total, ~1/2)
    assert abs(left - 0.5 * total) < 4.0 * np.sqrt(0.25 * total), (left, total)


def test_choice_independent_of_array_order():
    cfg = _cfg(seed=11)
    a = Oracle(cfg)
    a.step(5)
    b = Oracle(cfg, init=False)
    rng = np.random.default_rng(3)
    for s in (0, 1):
        x, vx, vy, vz, ids = a.state(s)
        p = rng.permutation(x.size)
        b.set_state(s, x[p], vx[p], vy[p], vz[p], ids[p])
    b.set_counters(a.step_index, a.next_id(0), a.next_id(1))
    E, _, _ = a.field()
    b.set_field(E)
    b.set_balance(*a.balance())
    for _ in range(20):
        a.step(1)
        b.step(1)
        for s in (0, 1):
            assert np.array_equal(a.victims(s), b.victims(s))
            ia, sa = _by_id(a, s)
            ib, sb = _by_id(b, s)
            assert np.array_equal(ia, ib) and np.array_equal(sa, sb)
