"""Long free runs of a GPU column and the striation diagnostics of section III
(wavelength, phase velocity, potential drop per striation, EEPF).

`run` advances a column and records electron-density snapshots (cell counts
from pc_moments, every `every` steps) plus time-averaged EEPF counts; the
analysis functions of analysis.py turn them into lambda = L / m*, v_ph and
delta_phi = E0 lambda (eq. (1)).
"""
from __future__ import annotations

import numpy as np
import torch

from . import analysis as A


def run(cfg: dict, steps: int, every: int, eepf_from: int = 0, progress=None):
    """Returns dict(times [s], ne [snapshots, cells] (counts), eepf (summed
    counts over snapshots at or after eepf_from steps), energy_sum (their
    summed energy moment, 2^-20 eV units) and energy_count (their summed
    electron counts), counts (n_e, n_i) per snapshot)."""
    from .column import Column
    col = Column(cfg)
    nc = int(cfg["n_cells"])
    snaps, times, counts = [], [], []
    eepf = np.zeros(A.EEPF_BINS)
    esum = ecount = 0
    done = 0
    while done < steps:
        k = min(every, steps - done)
        col.step(k)
        done += k
        mom = col.moments(nc).cpu().numpy()          # one EEPF group for the whole column
        parts = A.split(mom, nc, nc)
        snaps.append(parts["ne"].astype(np.float64))
        times.append(done * cfg["dt"])
        c = col.counts()
        counts.append(c["n"])
        if done >= eepf_from:
            eepf += parts["eepf"][0]
            esum += int(parts["eps"].sum())
            ecount += int(parts["ne"].sum())
        if progress is not None:
            progress(done)
    col.sync()
    return dict(times=np.array(times), ne=np.array(snaps), eepf=eepf, counts=np.array(counts),
                energy_sum=esum, energy_count=ecount)


def bounded_run(cfg: dict, steps: int, every: int, snap_every: int = 10, progress=None):
    """Free run of a bounded column with cathode emission and a series
    resistor (section V).  Returns dict(times [s], V (anode potential), J
    (conduction current density [A/m^2]), E_anode (field at the anode node
    [V/m], the anode sheath), counts, ne [snapshots, cells] every
    snap_every records)."""
    from .column import Column
    col = Column(cfg)
    nc = int(cfg["n_cells"])
    rec, snaps, counts = [], [], []
    done = 0
    while done < steps:
        k = min(every, steps - done)
        col.step(k)
        done += k
        c = col.counts()
        E, _, _ = col.get_field()
        rec.append((done * cfg["dt"], c["circuit"][0], c["J_cond"], float(E[-1])))
        counts.append(c["n"])
        if len(rec) % snap_every == 0:
            mom = col.moments(nc).cpu().numpy()
            snaps.append(A.split(mom, nc, nc)["ne"].astype(np.float64))
        if progress is not None:
            progress(done)
    col.sync()
    r = np.array(rec)
    return dict(times=r[:, 0], V=r[:, 1], J=r[:, 2], E_anode=r[:, 3], counts=np.array(counts),
                ne=np.array(snaps))


def striation_summary(res: dict, cfg: dict, t_from: float) -> dict:
    """Dominant mode, wavelength, phase velocity and potential drop per
    striation of the snapshots after t_from, plus the modulation depth."""
    sel = res["times"] >= t_from
    ne = res["ne"][sel]
    t = res["times"][sel]
    L = cfg["L"]
    m = A.dominant_mode_of_snapshots(ne)
    lam = L / m
    vph = A.phase_velocity(ne, t, L, m)
    E0 = cfg["V"] / cfg["L"]
    spec = np.abs(np.fft.rfft(ne - ne.mean(axis=1, keepdims=True), axis=1))
    depth = float(np.mean(2.0 * spec[:, m] / ne.shape[1] / ne.mean(axis=1)))
    return dict(mode=int(m), wavelength=float(lam), phase_velocity=float(vph),
                potential_drop=float(A.potential_drop_per_striation(E0, lam)), modulation=depth)


def growth_rate(res: dict, mode: int, lo: float = 1e-2, hi: float = 1e-1) -> float:
    """Growth rate [1/s] of a mode: slope of ln(relative amplitude) while the
    amplitude is between lo and hi (linear stage of the instability)."""
    ne = res["ne"]
    spec = np.abs(np.fft.rfft(ne - ne.mean(axis=1, keepdims=True), axis=1))
    amp = 2.0 * spec[:, mode] / ne.shape[1] / ne.mean(axis=1)
    sel = (amp > lo) & (amp < hi)
    if sel.sum() < 3:
        return float("nan")
    return float(np.polyfit(res["times"][sel], np.log(amp[sel]), 1)[0])


def main(argv=None) -> int:
    """python -m paper_2202_03215_amd.physics [--steps N] [--every K] [--precision fp64 fp32]
    Free run of the 20 cm neon column (balanced sink) with striation summaries."""
    import argparse
    import json
    import sys
    import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=1_000_000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--precision", nargs="+", default=["fp64", "fp32"])
    a = ap.parse_args(argv)
    for prec in a.precision:
        cfg = W.with_(W.column_20cm(), precision=prec, wall_mode="balanced")
        res = run(cfg, a.steps, a.every, eepf_from=a.steps // 2,
                  progress=lambda d: print(f"[physics] {prec} step {d}", file=sys.stderr, flush=True)
                  if d % 100_000 == 0 else None)
        s = striation_summary(res, cfg, 0.5 * a.steps * cfg["dt"])
        s["growth_rate"] = growth_rate(res, s["mode"])
        s["counts_end"] = res["counts"][-1].tolist()
        print(json.dumps({"precision": prec, "steps": a.steps, **s}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
