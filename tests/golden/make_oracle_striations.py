"""Writes oracle_striations_<column>_seed<k>.json: free runs of the CPU oracle
in the striated regime (section III), for the statistical comparison of long
GPU runs with the oracle.  Calls oracle/ only (numpy's FFT turns the oracle's
cell counts into Fourier coefficients; nothing else is computed here).

Columns (neon, 1 Torr, 300 K, periodic, E0 = 10 V/cm, n0 = 1e15 m^-3,
balanced sink, dt = 1e-11 s, ions every 20 steps; section III's runs use
neon at 1 Torr and a few V/cm above the striation threshold):
  4cm   400 cells, 100 electrons and ions per cell (40k + 40k)
  20cm  2000 cells, 200 per cell (400k + 400k)
Each run: 2e5 steps from the seeded initial load; every `every` steps the
oracle's electron cell counts are Fourier transformed and modes 0..M kept
(complex, 5 significant digits), and over the second half the EEPF counts
(0.25 eV bins on [0, 60) eV, whole column) and the energy sum and count are
accumulated for the time-averaged EEDF and mean energy.

Usage: python tests/golden/make_oracle_striations.py {4cm|20cm} SEED [--threads N]
(--threads uses the OpenMP build of the oracle, which computes bit for bit
what the serial build computes).  Run times: 4cm ~3 min serial, 20cm ~20 min
on 8 threads.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import pco  # noqa: E402

STEPS = 200_000
SETUP = {
    "4cm": dict(n_cells=400, L=0.04, ppc=100, every=1000, modes=32),
    "20cm": dict(n_cells=2000, L=0.20, ppc=200, every=2000, modes=64),
}


def config(column: str, seed: int) -> dict:
    s = SETUP[column]
    return W.with_(W.column_20cm(), n_cells=s["n_cells"], L=s["L"], V=s["L"] * 1000.0, ppc=s["ppc"],
                   wall_mode="balanced", seed=seed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("column", choices=sorted(SETUP))
    ap.add_argument("seed", type=int)
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    s = SETUP[a.column]
    cfg = config(a.column, a.seed)
    omp = a.threads > 0
    if omp:
        pco.threads(a.threads)
    o = pco.Oracle(cfg, omp=omp)
    nc, every, M = cfg["n_cells"], s["every"], s["modes"]
    re, im, steps_at, counts = [], [], [], []
    eepf = np.zeros(240, dtype=np.int64)
    esum, ecount = 0, 0
    t0 = time.time()
    for k in range(STEPS // every):
        o.step(every)
        done = (k + 1) * every
        m = o.moments(nc, 0)
        ne = m[:nc].astype(np.float64)
        c = np.fft.rfft(ne)[:M + 1]
        re.append([float(f"{v:.5g}") for v in c.real])
        im.append([float(f"{v:.5g}") for v in c.imag])
        steps_at.append(done)
        counts.append([o.count(0), o.count(1)])
        if done > STEPS // 2:
            eepf += m[7 * nc:7 * nc + 240]
            esum += int(m[nc:2 * nc].sum())
            ecount += int(m[:nc].sum())
        if done % 20_000 == 0:
            print(f"[golden] {a.column} seed {a.seed}: step {done} ({time.time() - t0:.0f} s)", flush=True)
    out = dict(config=f"neon 1 Torr, periodic {a.column}, {nc} cells, {cfg['ppc']} per cell, E0 = 10 V/cm, "
                      f"balanced sink, dt = 1e-11 s, seed {a.seed}",
               column=a.column, seed=a.seed, steps=STEPS, every=every, dt=cfg["dt"], L=cfg["L"],
               n_cells=nc, modes=M, steps_at=steps_at, fourier_re=re, fourier_im=im,
               eepf_counts=eepf.tolist(), energy_sum_2p20=esum, energy_count=ecount,
               counts=counts, errors=int(o.errors))
    with open(os.path.join(HERE, f"oracle_striations_{a.column}_seed{a.seed}.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))


if __name__ == "__main__":
    main()
