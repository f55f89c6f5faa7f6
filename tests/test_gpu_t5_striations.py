"""Long free runs in the striated regime against the oracle (section III),
statistically.

The oracle's golden runs (tests/golden/oracle_striations_*.json, written by
make_oracle_striations.py with the oracle only) hold the Fourier
coefficients of the electron cell counts every 1000 or 2000 steps over 2e5
steps, the EEPF summed over the second half and its energy sum.  The GPU
runs the same columns from the same seeded loads with the plain FP64 path
(FP32 against FP64: test_gpu_striations.py).  Trajectories diverge after the
first ulp difference (transcendentals of the collision kinematics), and in
the striated regime the divergence grows with the instability, so a GPU run
and the oracle run of one seed are two realizations of one random process;
what must agree are its statistics, computed identically on both sides
(analysis.striation_statistics).

The columns are multistable: the 20 cm column (neon, 1 Torr, 10 V/cm,
400k + 400k) saturates in mode 16, 17 or 18 depending on the realization
(GPU FP64, seeds 1-12: 16 eight times, 17 three times, 18 once), the 4 cm
column (40k + 40k) in mode 3 or 4, and a single realization's saturated
modulation -- with it its EEDF and mean energy -- differs from another's by
more than 3 % (two oracle seeds of the 20 cm column: depth 0.57 and 0.48,
EEDFs 4.4 % apart in L1, mean energies 3.5 %).  So the comparison is over
the ensemble of seeds on each side: a statistic that averages over the
whole column (EEDF, mean energy) or over the seeds (wavelength) must agree
within 3 %, and every statistic within three standard errors of the two
ensembles' means (seed-to-seed spread on both sides).
"""
import json
import os

import numpy as np
import pytest

from tests.gpu_helpers import striation_run

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")
E0 = 1000.0          # V/m
SEEDS_20CM = (1, 2, 3, 4, 5, 6, 7, 8)
SEEDS_4CM = (1, 2, 3, 4)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _have(column, seed):
    return os.path.exists(os.path.join(GOLD, f"oracle_striations_{column}_seed{seed}.json"))


def _eedf(counts):
    from paper_2202_03215_amd import analysis as A
    e, F = A.eepf(np.asarray(counts, dtype=np.float64))
    return F * np.sqrt(e) * A.EEPF_DE       # histogram normalised to 1


def _oracle_stats(column, seed):
    from paper_2202_03215_amd import analysis as A
    g = json.load(open(os.path.join(GOLD, f"oracle_striations_{column}_seed{seed}.json")))
    assert g["errors"] == 0
    coef = np.array(g["fourier_re"]) + 1j * np.array(g["fourier_im"])
    t = np.array(g["steps_at"]) * g["dt"]
    st = A.striation_statistics(coef, t, g["L"], 0.5 * g["steps"] * g["dt"])
    st.update(eedf=_eedf(g["eepf_counts"]), mean_energy=g["energy_sum_2p20"] / 2 ** 20 / g["energy_count"])
    return g, st


def _gpu_stats(column, seed, g):
    from paper_2202_03215_amd import analysis as A
    r = striation_run(column, seed, "fp64", steps=g["steps"], every=g["every"], modes=g["modes"])
    assert r["cfg"]["n_cells"] == g["n_cells"] and r["cfg"]["L"] == g["L"]
    st = A.striation_statistics(r["coef"], r["times"], g["L"], 0.5 * g["steps"] * g["dt"])
    st.update(eedf=_eedf(r["eepf"]), mean_energy=r["energy_sum"] / 2 ** 20 / r["energy_count"])
    return st


def _within_se(a, b, k=3.0):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    se = np.sqrt(a.var(axis=0, ddof=1) / len(a) + b.var(axis=0, ddof=1) / len(b))
    return np.abs(a.mean(axis=0) - b.mean(axis=0)) <= k * se + 1e-12 * np.abs(b.mean(axis=0))


def _ensembles(column, seeds):
    so, sg = [], []
    for seed in seeds:
        g, o = _oracle_stats(column, seed)
        so.append(o)
        sg.append(_gpu_stats(column, seed, g))
    for k, (o, s) in enumerate(zip(so, sg)):
        print(column, seeds[k], "oracle", o["mode"], o["first"], round(o["growth"] / 1e6, 3),
              round(o["phase_velocity"]), round(o["modulation"], 3), round(o["mean_energy"], 3),
              "| gpu", s["mode"], s["first"], round(s["growth"] / 1e6, 3), round(s["phase_velocity"]),
              round(s["modulation"], 3), round(s["mean_energy"], 3))
    return so, sg


def test_striated_20cm_column_matches_oracle(torch_cuda):
    seeds = [s for s in SEEDS_20CM if _have("20cm", s)]
    assert len(seeds) >= 4, seeds
    so, sg = _ensembles("20cm", seeds)
    assert all(s["modulation"] > 0.3 for s in so + sg)                 # striated
    assert all(s["phase_velocity"] < 0 for s in so + sg)               # towards the cathode
    lo = np.array([s["wavelength"] for s in so])
    lg = np.array([s["wavelength"] for s in sg])
    print("mean wavelength", lg.mean(), lo.mean(), "potential drop", E0 * lg.mean(), E0 * lo.mean())
    # wavelength and potential drop per striation, eq. (1): delta_phi = E0 lambda
    assert abs(lg.mean() / lo.mean() - 1.0) <= 0.03
    assert abs(E0 * lg.mean() - E0 * lo.mean()) <= 0.03 * E0 * lo.mean()
    assert _within_se(lg, lo)
    for key in ("growth", "phase_velocity", "modulation", "mean_energy"):
        a, b = [s[key] for s in sg], [s[key] for s in so]
        print(key, np.mean(a), np.mean(b))
        assert _within_se(a, b), key
    fo = np.mean([s["eedf"] for s in so], axis=0)
    fg = np.mean([s["eedf"] for s in sg], axis=0)
    l1 = float(np.abs(fg - fo).sum())
    mo = np.mean([s["mean_energy"] for s in so])
    mg = np.mean([s["mean_energy"] for s in sg])
    print("EEDF L1", l1, "mean energy", mg, mo)
    assert l1 <= 0.03, l1
    assert abs(mg / mo - 1.0) <= 0.03, (mg, mo)
    po = np.array([s["profile"] for s in so])
    pg = np.array([s["profile"] for s in sg])
    assert np.all(_within_se(pg, po)), (pg.mean(axis=0), po.mean(axis=0))


def test_striated_4cm_column_matches_oracle(torch_cuda):
    so, sg = _ensembles("4cm", SEEDS_4CM)
    assert all(s["modulation"] > 0.3 for s in so + sg)
    assert all(3 <= s["mode"] <= 5 for s in so + sg)
    for key in ("wavelength", "growth", "mean_energy"):
        a, b = [s[key] for s in sg], [s[key] for s in so]
        print(key, np.mean(a), np.mean(b))
        assert _within_se(a, b), key
