"""Long free runs on the GPU against the oracle, statistically.

A stationary neon column (E0 = 3 V/cm, below the striation threshold) runs
2e5 steps from the same seeded load on the GPU (FP64 and FP32 particles) as
the oracle's golden run (tests/golden/oracle_eedf_4cm_3Vcm.json, written by
make_oracle_eedf_4cm.py with the oracle only).  Trajectories diverge after
the first ulp difference, so only statistics are compared: the
time-averaged EEDF (L1 distance of the normalised distributions, 0.25 eV
bins) within 3 % and the mean energy within 3 % (observed: 0.6 % and 0.1 %).
"""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _eedf(counts):
    from paper_2202_03215_amd import analysis as A
    e, F = A.eepf(np.asarray(counts, dtype=np.float64))
    f = F * np.sqrt(e)
    return e, f, float(np.sum(e * f) * A.EEPF_DE)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_stationary_column_eedf_matches_oracle(torch_cuda, precision):
    from paper_2202_03215_amd import analysis as A
    from paper_2202_03215_amd import physics as PH
    gold = json.load(open(os.path.join(HERE, "golden", "oracle_eedf_4cm_3Vcm.json")))
    assert gold["errors"] == 0
    cfg = W.with_(W.column_20cm(), n_cells=400, L=0.04, V=0.04 * 300.0, ppc=100, wall_mode="balanced",
                  seed=1, precision=precision)
    r = PH.run(cfg, gold["steps"], gold["every"], eepf_from=gold["steps"] // 2)
    e, fg, mg = _eedf(r["eepf"])
    _, fo, mo = _eedf(gold["eepf_counts"])
    l1 = float(np.sum(np.abs(fg - fo)) * A.EEPF_DE)
    print(precision, "EEDF L1", l1, "mean energy", mg, mo)
    assert l1 <= 0.03, l1
    assert abs(mg / mo - 1.0) <= 0.03, (mg, mo)
    # no striations: the density spectrum stays at the noise level
    ne = r["ne"][len(r["ne"]) // 2:]
    spec = np.abs(np.fft.rfft(ne - ne.mean(1, keepdims=True), axis=1))
    assert (2 * spec[:, 1:] / ne.shape[1] / ne.mean(1)[:, None]).max() < 0.1
