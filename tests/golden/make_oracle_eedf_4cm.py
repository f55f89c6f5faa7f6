"""Writes oracle_eedf_4cm_3Vcm.json: the time-averaged EEDF and mean energy
of a long free run of the CPU oracle (calls oracle/ only).

Column: neon 1 Torr, periodic 4 cm, 400 cells, 100 electrons and ions per
cell, E0 = 3 V/cm (below the striation threshold, a stationary column),
balanced sink, dt = 1e-11 s, seed 1; 2e5 steps, EEPF counts (0.25 eV bins
on [0, 60) eV, whole column) summed every 1000 steps over the second half.
Run time ~7 min (serial).  Usage: python tests/golden/make_oracle_eedf_4cm.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle.pco import Oracle  # noqa: E402


def config():
    return W.with_(W.column_20cm(), n_cells=400, L=0.04, V=0.04 * 300.0, ppc=100, wall_mode="balanced", seed=1)


def main():
    cfg = config()
    steps, every = 200_000, 1000
    o = Oracle(cfg)
    nc = cfg["n_cells"]
    eepf = np.zeros(240, dtype=np.int64)
    for k in range(steps // every):
        o.step(every)
        if (k + 1) * every >= steps // 2:
            m = o.moments(nc, 0)
            eepf += m[7 * nc:7 * nc + 240]
    out = dict(config="neon 1 Torr, periodic 4 cm, 400 cells, 100/cell, E0 = 3 V/cm, balanced sink, seed 1",
               steps=steps, every=every, eepf_counts=eepf.tolist(), errors=int(o.errors),
               counts=[o.count(0), o.count(1)])
    with open(os.path.join(HERE, "oracle_eedf_4cm_3Vcm.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
