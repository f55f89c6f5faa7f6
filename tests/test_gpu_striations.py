"""Moving striations in the 20 cm neon column (section III), FP32 against
FP64 particles (free runs, compared statistically).

Both precisions start from the same seeded loads and run 2e5 steps (2 us)
with the balanced sink (constant particle number, as the paper's pair
removal).  The ionization wave grows from noise (~6e6 /s) towards a
saturated modulation moving towards the cathode; the saturated mode depends
on the realization, so the two precisions are compared over eight seeds.

The paper's own sink (one random electron and one random ion removed per
ionization) against the balanced sink, FP64, same length: the particle
numbers stay exactly constant, and the striations have the same dominant
mode, growth rates within 10 % and phase velocities within 15 %.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


SEEDS = (1, 2, 3, 4, 5, 6, 7, 8)


def test_fp32_striations_match_fp64(torch_cuda):
    """FP32 against FP64 particles over seeds 1-8 (same seeded loads, 2e5
    steps each).  The column saturates in mode 15-18 depending on the
    realization on either path (FP64, seeds 1-12: 16 eight times, 17 three,
    18 once; FP32: 17 eight times, 16 and 15 twice each), so single runs
    do not share a mode and the wavelength is compared over the seeds: the
    mean wavelength and potential drop per striation (eq. (1)) within 3 %,
    and the mean wavelength, growth rate, phase velocity and modulation within
    three standard errors of the two ensembles (their seed-to-seed spread)."""
    from paper_2202_03215_amd import analysis as A
    from tests.gpu_helpers import striation_run
    st = {"fp64": [], "fp32": []}
    for seed in SEEDS:
        for prec in ("fp64", "fp32"):
            r = striation_run("20cm", seed, prec)
            assert abs(r["counts"][-1][0] - 400_000) < 0.05 * 400_000
            s = A.striation_statistics(r["coef"], r["times"], 0.20, 1.0e-6)
            st[prec].append(s)
            print(prec, seed, s["mode"], s["first"], round(s["growth"] / 1e6, 3), round(s["phase_velocity"]),
                  round(s["modulation"], 3))
    a, b = st["fp64"], st["fp32"]
    assert all(s["modulation"] > 0.3 and s["phase_velocity"] < 0 for s in a + b)
    la = np.array([s["wavelength"] for s in a])
    lb = np.array([s["wavelength"] for s in b])
    print("mean wavelength fp64", la.mean(), "fp32", lb.mean())
    assert abs(lb.mean() / la.mean() - 1.0) <= 0.03
    E0 = 1000.0
    assert abs(E0 * lb.mean() - E0 * la.mean()) <= 0.03 * E0 * la.mean()
    for key in ("wavelength", "growth", "phase_velocity", "modulation"):
        x = np.array([s[key] for s in a])
        y = np.array([s[key] for s in b])
        se = np.sqrt(x.var(ddof=1) / x.size + y.var(ddof=1) / y.size)
        print(key, x.mean(), y.mean(), se)
        assert abs(x.mean() - y.mean()) <= 3.0 * se, key


def test_pair_sink_striations_match_balanced_sink(torch_cuda):
    from paper_2202_03215_amd import physics as PH
    steps, every = 200_000, 1000
    out = {}
    for wm in ("pair", "balanced"):
        cfg = W.with_(W.column_20cm(), wall_mode=wm)
        res = PH.run(cfg, steps, every)
        s = PH.striation_summary(res, cfg, 0.75 * steps * cfg["dt"])
        s["growth"] = PH.growth_rate(res, s["mode"])
        print(wm, s)
        out[wm] = (s, res["counts"])
    (a, counts), (b, _) = out["pair"], out["balanced"]
    assert np.all(counts == 400_000), counts.min()
    assert a["modulation"] > 0.3 and b["modulation"] > 0.3
    assert a["mode"] == b["mode"]
    assert a["phase_velocity"] < 0 and abs(a["phase_velocity"] - b["phase_velocity"]) <= 0.15 * abs(b["phase_velocity"])
    assert a["growth"] > 0 and abs(a["growth"] - b["growth"]) <= 0.10 * b["growth"]
