"""Throughput benchmark of the GPU PIC-MCC column step.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu] ...

Prints one JSON line.  A step is one full time step of the column (electron
advance with collisions and fused deposit, ion advance on subcycle steps,
compaction, ionization products, field solve, periodic sort).  `value` is
particle-steps per second of the plain FP64 step on the headline workload
(column_50cm: neon 0.5 Torr, 50 cm, 5000 cells, 5M + 5M particles):
electrons advanced plus ions advanced (ions only on their subcycle steps),
over exactly K timed steps with the state resident in device memory, all K
replayed from HIP graphs captured beforehand.  `roofline` reports the
electron advance kernel (the dominant kernel) against the HBM peak and the
stream probe's rate, its duration measured with HIP events that take the
start and end timestamps of each launch on the library's stream
(hipExtLaunchKernelGGL), in an eager window of the same length after the
graph-replayed one; `traffic` is the kernel's hardware-counter HBM traffic
from the committed counter profile when that profile was taken on the
current kernel sources, else null.  `cpu_baseline` times the FP64 CPU oracle
(serial parity build and OpenMP all-core build) on bounded samples.
Further objects: `fp32` (the same workload with FP32 particles),
`column_20cm` (the 400k + 400k column, FP64 and FP32), `pair_sink` (20 cm
column with the paper's own loss model: a random electron and ion removed
per ionization), `section_v` (the bounded 15 cm column with a hot cathode and
a series resistor), `batched` (64-column argon scan, FP32) and `fluid`
(256 x 4096 fluid columns).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
METRIC = "particle-steps/s at 1 GPU (plain FP64 vs batched FP32) + % HBM peak"

WORKLOADS = {
    # Ne 0.5 Torr, periodic 50 cm, 5000 cells, 1000 per cell per species (5M + 5M)
    "column_50cm": lambda: W.column_50cm(),
    # Ne 1 Torr, periodic 20 cm, 2000 cells, 200 per cell per species (400k + 400k)
    "column_20cm": lambda: W.column_20cm(),
    # Ne 1 Torr, bounded 4 cm, 400 cells, 50 per cell per species (20k + 20k)
    "small_bounded": lambda: W.small_bounded(),
}

# sources and build flags of the particle kernels: a counter profile is valid
# for the build it was taken on
KERNEL_SOURCES = ("paper_2202_03215_amd/csrc/kernels.hip", "paper_2202_03215_amd/csrc/device.h",
                  "paper_2202_03215_amd/build.py")


def kernel_source_sha16() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(workload: str, precision: str, electrons: float = 0.0) -> tuple:
    """HBM bytes per launch of the electron advance kernel from the committed
    counter profile (profiles/hbm_counters_push_<workload>_<precision>.md):
    FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the same
    counter reads for the stream-probe copy of known size, and by the ratio
    of this run's electrons per launch to the profile run's when the record
    holds that count.  Null when there is no profile or when it was taken on
    other kernel sources or build flags."""
    path = os.path.join(ROOT, "profiles", f"hbm_counters_push_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None, f"no counter profile for {workload} {precision}"
    m = re.search(r"```json\s*(\{.*?\})\s*```", open(path).read(), re.S)
    if not m:
        return None, f"{os.path.relpath(path, ROOT)} holds no counter record"
    rec = json.loads(m.group(1))
    if rec.get("source_sha16") != kernel_source_sha16():
        return None, (f"{os.path.relpath(path, ROOT)} was taken on kernel sources {rec.get('source_sha16')}, "
                      f"not the current {kernel_source_sha16()}")
    t = rec["fetch_kib"] * 1024.0 * rec["fetch_factor"] + rec["write_kib"] * 1024.0 * rec["write_factor"]
    note = f"{os.path.relpath(path, ROOT)} (kernel sources {rec['source_sha16']})"
    if electrons > 0 and rec.get("electrons_per_launch"):
        t *= electrons / float(rec["electrons_per_launch"])
        note += f", scaled from {rec['electrons_per_launch']:.0f} to {electrons:.0f} electrons per launch"
    return t, note


def electron_bytes_per_step(p_null: float, fp32: bool = False) -> float:
    """Algorithmic HBM bytes per electron per step of the electron advance
    kernel.  FP64: read x, vx (8 B each) and id (4 B), write x, vx; a
    collision candidate (fraction p_null) also reads and writes vy, vz:
    36 + 32 p_null.  FP32: read cell, offset, vx, id, write cell, offset, vx
    (4 B each); candidates read and write vy, vz: 28 + 16 p_null."""
    if fp32:
        return 28 + 16 * p_null
    return 36 + 32 * p_null


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Host cores this process may use: the OpenMP thread setting of the
    environment if there is one, else the CPUs of its affinity mask."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(env))) if env.isdigit() and int(env) > 0 else n


def oracle_rate(cfg: dict, steps: int, threads: int) -> dict:
    """Particle-steps/s of the FP64 oracle over `steps` steps from the initial
    load (serial parity build for threads == 1, else the OpenMP build)."""
    from oracle import pco
    omp = threads > 1
    if omp:
        pco.threads(threads)
    o = pco.Oracle(cfg, omp=omp)
    n0e, n0i = o.count(0), o.count(1)
    S = int(cfg["ion_subcycle"])
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    ne = 0.5 * (n0e + o.count(0)) * steps
    ion_steps = sum(1 for k in range(steps) if k % S == 0)
    ni = 0.5 * (n0i + o.count(1)) * ion_steps
    used = pco.threads() if omp else 1
    del o
    return {"value": (ne + ni) / dt, "seconds": dt, "steps": steps, "cores": used}


def cpu_baseline(cfg: dict, workload: str, steps_serial: int, steps_omp: int) -> dict:
    threads = host_threads()
    print(f"[bench] cpu baseline: oracle {workload}, {steps_serial} steps serial, {steps_omp} steps on "
          f"{threads} threads", file=sys.stderr, flush=True)
    ser = oracle_rate(cfg, steps_serial, 1)
    allc = oracle_rate(cfg, steps_omp, threads) if threads > 1 else ser
    small = W.small_bounded()
    m1s = oracle_rate(small, 2000, 1)
    m1a = oracle_rate(small, 2000, threads) if threads > 1 else m1s
    return {"value": allc["value"], "unit": "particle-steps/s", "cores": allc["cores"], "kind": "oracle",
            "sample": f"{allc['steps']} steps of {workload} from its initial load, OpenMP build of the FP64 "
                      f"oracle on {allc['cores']} threads ({allc['seconds']:.1f} s)",
            "serial": {"value": ser["value"], "cores": 1,
                       "sample": f"{ser['steps']} steps of {workload}, serial parity build ({ser['seconds']:.1f} s)"},
            "small_bounded_2000_steps": {"serial": m1s["value"], "all_cores": m1a["value"],
                                         "cores": m1a["cores"]},
            "host": {"cpu_model": cpu_model(), "cpus": os.cpu_count(),
                     "affinity": len(os.sched_getaffinity(0)), "threads_used": allc["cores"]}}


def measure(cfg: dict, args, tag: str, workload: str) -> dict:
    """Graph-replayed timed window (throughput; the graphs are captured
    before it) then an eager event-timed window of the same length (electron
    advance kernel duration)."""
    import torch
    from paper_2202_03215_amd.column import Column

    print(f"[bench] {tag}: init", file=sys.stderr, flush=True)
    col = Column(cfg)
    S = int(cfg["ion_subcycle"])
    col.step(args.warmup)
    col.sync()
    c0 = col.counts()
    col.prepare_graphs(args.steps)
    print(f"[bench] {tag}: warmup {args.warmup} done, n = {c0['n']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    col.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c1 = col.counts()
    col.sync()
    elapsed = t1 - t0
    step0 = c0["step"]
    ion_steps = sum(1 for k in range(step0, step0 + args.steps) if k % S == 0)
    ne_avg = 0.5 * (c0["n"][0] + c1["n"][0])
    ni_avg = 0.5 * (c0["n"][1] + c1["n"][1])
    value = (ne_avg * args.steps + ni_avg * ion_steps) / elapsed
    # second timed window: every electron-advance launch carries start/end
    # events of its own on the column's stream (eager launches: events
    # recorded by graph nodes carry no readable time on this runtime)
    col.timer_enable(args.steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    col.step(args.steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ker_ms, launches = col.timer_read()
    col.timer_enable(0)
    c2 = col.counts()
    col.sync()
    ne_avg2 = 0.5 * (c1["n"][0] + c2["n"][0])
    fp32 = cfg.get("precision", "fp64") == "fp32"
    p_null = float(col.sizes.p_null)
    bpe = electron_bytes_per_step(p_null, fp32)
    bytes_per_launch = ne_avg2 * bpe
    avg_s = ker_ms * 1e-3 / max(launches, 1)
    achieved = bytes_per_launch / avg_s / 1e9
    print(f"[bench] {tag}: {args.steps} steps in {elapsed:.4f} s (graphs), {t3 - t2:.4f} s (eager, "
          f"timed); push kernel avg {avg_s * 1e6:.2f} us over {launches} launches",
          file=sys.stderr, flush=True)
    traffic, tnote = counter_traffic(workload, "fp32" if fp32 else "fp64", ne_avg2)
    moments_us = None
    if args.moments:
        # diagnostics on demand (cell moments of both species and the EEPF
        # histogram): host-timed calls, each with its output clear and copy-out
        col.moments()
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        for _ in range(20):
            col.moments()
        torch.cuda.synchronize()
        moments_us = (time.perf_counter() - t4) * 1e6 / 20
    del col
    torch.cuda.empty_cache()
    return {"value": value, "elapsed": elapsed, "ne": ne_avg, "ni": ni_avg, "ion_steps": ion_steps,
            "moments_us_per_call": moments_us,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": tnote,
                         "kernel": "k_push_e<false, Soa32>" if fp32 else "k_push_e<false, Soa>",
                         "avg_us": avg_s * 1e6, "launches": launches,
                         "bytes_per_electron": bpe, "p_null": p_null,
                         "bytes_per_launch": bytes_per_launch,
                         "window": "eager timed window of the same length after the graph window",
                         "ms_per_step_eager": (t3 - t2) * 1e3 / args.steps}}


def stream_probe(mib: int = 2048, reps: int = 10) -> dict:
    """Achievable copy rate of the particle kernels' access form: the
    library's stream-probe kernel (one 8-byte element per lane) copying
    `mib` MiB, timed with events over `reps` launches."""
    import torch
    from paper_2202_03215_amd.column import stream_probe as probe
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        probe(src, dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        probe(src, dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ok = bool(torch.equal(src, dst))
    del src, dst
    torch.cuda.empty_cache()
    gbs = 2.0 * n * 8 * reps / (ms * 1e-3) / 1e9
    print(f"[bench] stream probe: {gbs:.0f} GB/s ({mib} MiB copy)", file=sys.stderr, flush=True)
    return {"GB_s": gbs, "bytes_per_launch": 2.0 * n * 8, "launches": reps, "copy_ok": ok,
            "kernel": "k_stream_copy (one 8-byte element per lane, 4096 blocks)"}


def measure_sequential(cfgs: list, steps: int = 160, warmup: int = 160) -> dict:
    """The same columns as plain FP64 single columns, one after the other
    (each graph-replayed on its own): the baseline the batched FP32 launch
    is compared with."""
    import torch
    from paper_2202_03215_amd.column import Column
    work = 0.0
    elapsed = 0.0
    for cfg in cfgs:
        c = W.with_(cfg, precision="fp64")
        col = Column(c)
        col.step(warmup)
        col.sync()
        n0 = col.counts()
        col.prepare_graphs(steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        col.step(steps)
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        n1 = col.counts()
        col.sync()
        S = int(c["ion_subcycle"])
        ion_steps = sum(1 for k in range(n0["step"], n0["step"] + steps) if k % S == 0)
        work += 0.5 * (n0["n"][0] + n1["n"][0]) * steps + 0.5 * (n0["n"][1] + n1["n"][1]) * ion_steps
        del col
    torch.cuda.empty_cache()
    print(f"[bench] sequential fp64 columns: {len(cfgs)} x {steps} steps in {elapsed:.3f} s",
          file=sys.stderr, flush=True)
    return {"value": work / elapsed, "steps_per_column": steps, "dtype": "f64"}


def measure_batch(cfgs: list, args) -> dict:
    """Batched columns: autotune, warm up, then a graph-replayed timed window
    (throughput of every column together) and an eager event-timed window of
    the batched electron launch (roofline)."""
    import torch
    from paper_2202_03215_amd.column import Batch

    print(f"[bench] batch: init {len(cfgs)} columns", file=sys.stderr, flush=True)
    b = Batch(cfgs)
    tuning = b.tune(trial_steps=40) if not args.no_tune else b.tuning()
    print(f"[bench] batch: tuning {tuning}", file=sys.stderr, flush=True)
    b.step(args.batch_warmup)
    b.sync()

    def totals():
        ne = ni = 0
        for k in range(len(cfgs)):
            c = b.column(k).counts()
            ne += c["n"][0]
            ni += c["n"][1]
        return ne, ni

    S = int(cfgs[0]["ion_subcycle"])
    step0 = b.column(0).counts()["step"]
    ne0, ni0 = totals()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(args.batch_steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    b.sync()
    ne1, ni1 = totals()
    elapsed = t1 - t0
    ion_steps = sum(1 for k in range(step0, step0 + args.batch_steps) if k % S == 0)
    value = (0.5 * (ne0 + ne1) * args.batch_steps + 0.5 * (ni0 + ni1) * ion_steps) / elapsed
    b.timer_enable(args.batch_steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    b.step(args.batch_steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ker_ms, launches = b.timer_read()
    b.timer_enable(0)
    b.sync()
    ne2, _ = totals()
    from paper_2202_03215_amd import native as N
    p_null = [float(N.query_sizes(c).p_null) for c in cfgs]
    bpe = electron_bytes_per_step(max(p_null), True)
    bytes_per_launch = 0.5 * (ne1 + ne2) * bpe
    avg_s = ker_ms * 1e-3 / max(launches, 1)
    achieved = bytes_per_launch / avg_s / 1e9
    print(f"[bench] batch: {args.batch_steps} steps in {elapsed:.3f} s (graphs), {t3 - t2:.3f} s "
          f"(eager); batched electron launch avg {avg_s * 1e6:.1f} us", file=sys.stderr, flush=True)
    del b
    torch.cuda.empty_cache()
    return {"value": value, "ms_per_step": elapsed * 1e3 / args.batch_steps,
            "steps": args.batch_steps, "warmup": args.batch_warmup, "electrons": int(0.5 * (ne0 + ne1)),
            "ions": int(0.5 * (ni0 + ni1)), "tuning": tuning,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k_batch_push_e<Soa32>", "avg_us": avg_s * 1e6, "launches": launches,
                         "bytes_per_electron": bpe, "bytes_per_launch": bytes_per_launch,
                         "window": "eager timed window of the same length after the graph window"}}


CLOSURE_WEIGHTS = "workloads/closure_multipliers_ne_20cm.npz"


def measure_fluid(args, pic_ms_per_step: float, pic_dt: float, batch=None) -> dict:
    """Batched quasi-neutral fluid columns (section IV): 256 neon columns of
    20 cm and 4096 cells at 1 Torr and 10 V/cm (the striated PIC column's
    conditions, two-term table), each its own realization (1e-3 density
    noise), with the table closure and with the learned multiplier closure
    (network trained on the striated PIC column, weights in
    workloads/closure_multipliers_ne_20cm.npz, BF16 matrix cores in the
    loop).  Per closure: time per step over a timed window, then a free run
    to 40 us of simulated time: striated fraction and ensemble wavelength."""
    import numpy as np
    from paper_2202_03215_amd import closure as CL
    from paper_2202_03215_amd.mlp import ClosureNet

    ncol, ncell, dt, L, E0 = args.fluid_columns, 4096, 1.0e-9, 0.20, 1000.0
    Ngas = 1.0 * 133.322368 / (1.380649e-23 * 300.0)
    table = W.fluid_table_ne()
    wpath = os.path.join(ROOT, CLOSURE_WEIGHTS)
    if not os.path.exists(wpath):
        raise FileNotFoundError(f"{CLOSURE_WEIGHTS} missing (python -m paper_2202_03215_amd.closure OUT.npz)")
    d = np.load(wpath)
    net = ClosureNet(d["theta"].astype(np.float64), max_batch=1024)
    out = {}
    for name, kw in (("table", {}), ("learned_multipliers", dict(net=net, norm=d["norm"], multipliers=True))):
        r = CL.fluid_ensemble(table, W.FLUID_T_MIN, W.FLUID_T_STEP, Ngas, E0, L, ncell, dt, args.fluid_run_steps,
                              ncol, snapshots=10, timed=(args.fluid_warmup, args.fluid_steps), **kw)
        lam = r["wavelength"]
        ok = np.isfinite(lam)
        us = r["us_per_step"]
        out[name] = {"us_per_step": us, "cell_steps_per_s": ncol * ncell / (us * 1e-6),
                     "striated_fraction": float(ok.mean()),
                     "wavelength_mean_cm": float(lam[ok].mean() * 100) if ok.any() else None,
                     "wavelength_se_cm": float(lam[ok].std(ddof=1) / np.sqrt(ok.sum()) * 100) if ok.sum() > 1
                     else None,
                     "modulation_mean": float(r["modulation"].mean())}
        print(f"[bench] fluid {name}: {us:.1f} us per step ({ncol} x {ncell} cells); striated "
              f"{ok.mean():.2f}, lambda {out[name]['wavelength_mean_cm']} cm", file=sys.stderr, flush=True)
    # wall time per simulated microsecond of one column
    fluid_s = out["learned_multipliers"]["us_per_step"] * 1e-6 / dt * 1e-6 / ncol
    pic_s = pic_ms_per_step * 1e-3 / pic_dt * 1e-6
    res = {"workload": f"fluid_ne_20cm_{ncol}x{ncell}", "columns": ncol, "cells": ncell, "dt": dt, "E0": E0,
           "free_run_us": args.fluid_run_steps * dt * 1e6,
           "dtype": "f32 state, f64 tridiagonal, bf16 network", **out,
           "wall_s_per_simulated_us_per_column": fluid_s,
           "pic_wall_s_per_simulated_us_per_column": pic_s,
           "wall_time_ratio_pic_over_fluid": pic_s / fluid_s}
    if batch is not None:
        bs = batch["ms_per_step"] * 1e-3 / (batch["dt_sum"] * 1e6)   # columns advance their own dt per step
        res["batched_pic_wall_s_per_simulated_us_per_column"] = bs
        res["wall_time_ratio_batched_pic_over_fluid"] = bs / fluid_s
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="column_50cm", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps of the headline workload (0 = 40 serial, 100 all-core)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 variant")
    ap.add_argument("--no-20cm", action="store_true", help="skip the 20 cm column legs")
    ap.add_argument("--no-pair", action="store_true", help="skip the pair-sink variant")
    ap.add_argument("--no-section-v", action="store_true",
                    help="skip the bounded hot-cathode column with the external circuit")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched argon scan")
    ap.add_argument("--no-tune", action="store_true", help="batched scan without the autotuner")
    ap.add_argument("--batch-columns", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=320)
    ap.add_argument("--batch-warmup", type=int, default=40)
    ap.add_argument("--no-fluid", action="store_true", help="skip the batched fluid columns")
    ap.add_argument("--fluid-columns", type=int, default=256)
    ap.add_argument("--fluid-steps", type=int, default=200)
    ap.add_argument("--fluid-run-steps", type=int, default=40_000,
                    help="free-run length of the fluid ensembles (steps of 1 ns)")
    ap.add_argument("--fluid-warmup", type=int, default=20)
    ap.add_argument("--no-probe", action="store_true", help="skip the stream probe")
    ap.add_argument("--probe-mib", type=int, default=2048)
    ap.add_argument("--no-moments", dest="moments", action="store_false",
                    help="skip the on-demand moments timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the engine runs a column on exactly one GPU (no sharding or "
                                   "collectives); run with --gpus 1"}))
        return 2

    cfg = WORKLOADS[args.workload]()
    r64 = measure(cfg, args, "fp64", args.workload)
    value, elapsed, ne_avg, ni_avg = r64["value"], r64["elapsed"], r64["ne"], r64["ni"]
    S = int(cfg["ion_subcycle"])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "gas": cfg["gas"], "bc": cfg["bc"], "p_torr": cfg["p_torr"],
                   "L_m": cfg["L"], "n_cells": cfg["n_cells"], "particles_per_cell": cfg["ppc"],
                   "electrons": int(ne_avg), "ions": int(ni_avg), "dt": cfg["dt"],
                   "ion_subcycle": S, "sort_interval": cfg["sort_interval"], "precision": "fp64",
                   "graph_replayed": True},
        "roofline": r64["roofline"],
        "electron_steps_per_s": ne_avg * args.steps / elapsed,
        "ion_steps_per_s": ni_avg * r64["ion_steps"] / elapsed,
    }
    if r64["moments_us_per_call"] is not None:
        out["moments"] = {"us_per_call": r64["moments_us_per_call"],
                          "what": "cell moments of both species and the EEPF histogram, on demand, host-timed"}
    if not args.no_probe:
        probe = stream_probe(args.probe_mib)
        out["stream_probe"] = probe
        out["roofline"]["peak_measured_copy"] = probe["GB_s"]
        out["roofline"]["frac_of_measured_copy"] = out["roofline"]["achieved"] / probe["GB_s"]
    if not args.no_fp32:
        r32 = measure(W.with_(cfg, precision="fp32"), args, "fp32", args.workload)
        out["fp32"] = {"value": r32["value"], "ms_per_step": r32["elapsed"] * 1e3 / args.steps,
                       "dtype": "f32 particles, f64 field", "roofline": r32["roofline"],
                       "speedup_vs_fp64": r32["value"] / value}
    if not args.no_20cm and args.workload != "column_20cm":
        c20 = W.column_20cm()
        a = measure(c20, args, "20cm fp64", "column_20cm")
        leg = {"workload": "column_20cm", "value": a["value"], "ms_per_step": a["elapsed"] * 1e3 / args.steps,
               "dtype": "f64", "electrons": int(a["ne"]), "ions": int(a["ni"]), "roofline": a["roofline"]}
        if not args.no_fp32:
            b = measure(W.with_(c20, precision="fp32"), args, "20cm fp32", "column_20cm")
            leg["fp32"] = {"value": b["value"], "ms_per_step": b["elapsed"] * 1e3 / args.steps,
                           "roofline": b["roofline"], "speedup_vs_fp64": b["value"] / a["value"]}
        out["column_20cm"] = leg
    if not args.no_pair:
        # the paper's own sink (a random electron and ion removed per ionization)
        c20 = W.column_20cm()
        base = out.get("column_20cm", {}).get("value") if args.workload != "column_20cm" else value
        rp = measure(W.with_(c20, wall_mode="pair"), args, "pair", "column_20cm")
        out["pair_sink"] = {"workload": "column_20cm", "value": rp["value"],
                            "ms_per_step": rp["elapsed"] * 1e3 / args.steps, "dtype": "f64", "wall_mode": "pair",
                            "roofline": rp["roofline"],
                            "relative_to_fixed_sink": rp["value"] / base if base else None}
    if not args.no_section_v:
        hc = W.hot_cathode_15cm()
        rv = measure(hc, args, "section_v", "hot_cathode_15cm")
        out["section_v"] = {"workload": "hot_cathode_15cm", "value": rv["value"],
                            "ms_per_step": rv["elapsed"] * 1e3 / args.steps, "dtype": "f64",
                            "electrons": int(rv["ne"]), "ions": int(rv["ni"]), "roofline": rv["roofline"]}
    if not args.no_batch:
        cfgs = W.argon_scan(args.batch_columns)
        rb = measure_batch(cfgs, args)
        rs = measure_sequential(cfgs)
        out["batched"] = {"workload": f"argon_scan_{args.batch_columns}", "columns": len(cfgs),
                          "cells": [min(c["n_cells"] for c in cfgs), max(c["n_cells"] for c in cfgs)],
                          "dtype": "f32 particles, f64 field", **rb,
                          "speedup_vs_plain_fp64": rb["value"] / value,
                          "sequential_fp64_columns": rs,
                          "speedup_vs_sequential_fp64_columns": rb["value"] / rs["value"]}
    if not args.no_fluid:
        ref = out.get("column_20cm")
        pic_ms = ref["ms_per_step"] if ref else elapsed * 1e3 / args.steps
        bt = None
        if "batched" in out:
            bt = {"ms_per_step": out["batched"]["ms_per_step"],
                  "dt_sum": float(sum(c["dt"] for c in W.argon_scan(args.batch_columns)))}
        out["fluid"] = measure_fluid(args, pic_ms, float(W.column_20cm()["dt"]), bt)
    if not args.no_cpu:
        ss = args.cpu_steps or 40
        sa = args.cpu_steps or 100
        out["cpu_baseline"] = cpu_baseline(cfg, args.workload, ss, sa)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
