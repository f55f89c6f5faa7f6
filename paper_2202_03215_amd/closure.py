"""Learned closure of the fluid model: training data from PIC-MCC moments,
the table (drift-diffusion) closure it is compared with, normalisation and
GPU training (section IV of the paper: the fluid equations (3)-(4) need the
electron flux and energy flux; eqs. (7)-(8) give them in drift-diffusion
form with coefficients from 0D Boltzmann tables).

Sign convention of the samples: the fluid model's, i.e. a positive mean
field E0 along +x (the PIC column imposes E = -E0 + E_sp, so PIC samples are
mirrored, x -> -x: E, the gradients and both fluxes change sign).

Samples per cell group and time window (moments of the GPU column, summed
every `every` steps over `window` steps):
  features (n [m^-3], mean energy [eV], E [V/m], dn/dx, d(mean energy)/dx)
  targets  (Gamma_e [m^-2 s^-1], H_e [eV m^-2 s^-1])
"""
from __future__ import annotations

import numpy as np
import torch

from . import analysis as A


def modulated_state(cfg: dict, amp_n: float, mode: int, amp_T: float, seed: int):
    """Seeded particles with density n0 (1 + amp_n cos(k x)) for both species
    (quasi-neutral) and electron temperature Te0 (1 + amp_T sin(k x))."""
    rng = np.random.default_rng(seed)
    L = cfg["L"]
    n_part = int(cfg["ppc"]) * int(cfg["n_cells"])
    k = 2.0 * np.pi * mode / L

    def positions(n):
        out = np.empty(0)
        while out.size < n:
            x = rng.random(2 * n) * L
            keep = rng.random(2 * n) * (1.0 + abs(amp_n)) < 1.0 + amp_n * np.cos(k * x)
            out = np.concatenate([out, x[keep]])
        return out[:n]

    qe, me, amu, kb = 1.602176634e-19, 9.1093837015e-31, 1.66053906660e-27, 1.380649e-23
    xe = positions(n_part)
    Te = cfg["Te0_eV"] * (1.0 + amp_T * np.sin(k * xe))
    ve = rng.normal(size=(3, n_part)) * np.sqrt(Te * qe / me)
    xi = positions(n_part)
    vi = rng.normal(size=(3, n_part)) * np.sqrt(kb * cfg["Ti0_K"] / (cfg["M_amu"] * amu))
    ids = np.arange(n_part)
    return (xe, ve[0], ve[1], ve[2], ids), (xi, vi[0], vi[1], vi[2], ids)


def _window_samples(col, cfg: dict, steps: int, every: int, window: int, group: int):
    """Advance a GPU column by `steps` and return its samples (X, Y) in the
    fluid sign convention: moments summed every `every` steps over windows
    of `window` steps and groups of `group` cells."""
    Xs, Ys = [], []
    nc, L = int(cfg["n_cells"]), float(cfg["L"])
    ng = nc // group
    dxg = L / ng
    wmac = cfg["n0"] / cfg["ppc"]                   # real electrons per macroparticle per cell length
    acc = None
    nacc = 0
    for s in range(steps // every):
        col.step(every)
        mom = col.moments(1).to(torch.float64)
        E, _, _ = col.get_field()
        Ec = 0.5 * (E + torch.roll(E, -1))          # cell average (periodic nodes)
        part = torch.stack([mom[0:nc], mom[nc:2 * nc], mom[2 * nc:3 * nc], mom[3 * nc:4 * nc], Ec])
        acc = part if acc is None else acc + part
        nacc += 1
        if (s + 1) * every % window == 0:
            a = acc.cpu().numpy()
            g = a.reshape(5, ng, group).sum(axis=2)
            cnt = g[0] / nacc
            n = cnt * wmac / group
            eps = g[1] / A.EPS_SCALE / np.maximum(g[0], 1)
            gam = g[2] / A.V_SCALE / nacc * wmac / group
            H = g[3] / 16.0 / nacc * wmac / group
            Eg = g[4] / (nacc * group)
            dn = (np.roll(n, -1) - np.roll(n, 1)) / (2 * dxg)
            de = (np.roll(eps, -1) - np.roll(eps, 1)) / (2 * dxg)
            # mirror x -> -x into the fluid convention
            Xs.append(np.stack([n, eps, -Eg, -dn, -de], axis=1))
            Ys.append(np.stack([-gam, -H], axis=1))
            acc = None
            nacc = 0
    return np.concatenate(Xs), np.concatenate(Ys)


def pic_samples(cfgs: list, steps: int, every: int, window: int, group: int, amp_n=0.3, amp_T=0.2,
                mode=2, seed=0):
    """Run each column on the GPU from a modulated state and return samples
    (X [M, 5], Y [M, 2]) in the fluid sign convention, plus the column index
    of every sample."""
    from .column import Column
    Xs, Ys, cols = [], [], []
    for c, cfg in enumerate(cfgs):
        col = Column(cfg)
        e, i = modulated_state(cfg, amp_n, mode, amp_T, seed + c)
        col.set_state(0, *e)
        col.set_state(1, *i)
        col.set_counters(0, e[0].size, i[0].size)
        X, Y = _window_samples(col, cfg, steps, every, window, group)
        Xs.append(X)
        Ys.append(Y)
        cols.append(np.full(X.shape[0], c))
        col.sync()
        del col
    return np.concatenate(Xs), np.concatenate(Ys), np.concatenate(cols)


def striated_samples(cfgs: list, warm: int, steps: int, every: int, window: int, group: int):
    """Samples of columns in their saturated striated state: each column
    starts from its own seeded load, runs `warm` steps until the ionization
    wave has saturated, then is sampled over `steps` steps.  Returns
    (X, Y, column index)."""
    from .column import Column
    Xs, Ys, cols = [], [], []
    for c, cfg in enumerate(cfgs):
        col = Column(cfg)
        col.step(warm)
        X, Y = _window_samples(col, cfg, steps, every, window, group)
        Xs.append(X)
        Ys.append(Y)
        cols.append(np.full(X.shape[0], c))
        col.sync()
        del col
    return np.concatenate(Xs), np.concatenate(Ys), np.concatenate(cols)


def transport_table(gas_cfg: dict, EN_values, Ngas: float):
    """Two-term tables for the fluid model and the table closure: rows sorted
    by T_e = 2/3 mean energy (columns of include/pc_fluid.h: mu_e N, D_e N,
    mu_eps N, D_eps N, k_iz, L/N) and the T grid."""
    from . import boltzmann
    t = boltzmann.table(gas_cfg, EN_values)
    o = np.argsort(t["Te"])
    T = t["Te"][o]
    Lrate = t["EN"][o] * t["w"][o]                    # heating per electron per N equals the loss
    cols = np.stack([t["muN"][o], t["DN"][o], t["mu_epsN"][o], t["D_epsN"][o], t["k_iz"][o], Lrate], axis=1)
    return T, cols


def resample_uniform(T, cols, T_min, T_step, K):
    """Linear resampling of a table onto the uniform grid T_min + k T_step."""
    Tg = T_min + T_step * np.arange(K)
    return np.stack([np.interp(Tg, T, cols[:, q]) for q in range(cols.shape[1])], axis=1)


def table_fluxes(X, T, cols, Ngas):
    """Local drift-diffusion fluxes (eqs. (7)-(8), coefficients from the
    table at T = 2/3 mean energy, eq. (9) read as beta = 3/2 T mu_eps,
    G = 3/2 T D_eps): Gamma = -n mu_e E - d(n D_e)/dx, H = -n beta E - d(n G)/dx."""
    n, eps, E, dn, de = X.T
    Te = 2.0 / 3.0 * eps
    dT = 2.0 / 3.0 * de
    c = [np.interp(Te, T, cols[:, q]) / Ngas for q in range(4)]
    mue, De, mueps, Deps = c
    h = 1e-3
    dDe = (np.interp(Te + h, T, cols[:, 1]) - np.interp(Te - h, T, cols[:, 1])) / (2 * h) / Ngas
    G = 1.5 * Te * Deps
    dG = (1.5 * (Te + h) * np.interp(Te + h, T, cols[:, 3]) - 1.5 * (Te - h) * np.interp(Te - h, T, cols[:, 3])) \
        / (2 * h) / Ngas
    beta = 1.5 * Te * mueps
    gam = -n * mue * E - De * dn - n * dDe * dT
    H = -n * beta * E - G * dn - n * dG * dT
    return np.stack([gam, H], axis=1)


def table_terms(X, T, cols, Ngas):
    """The parts of the drift-diffusion fluxes of eqs. (7)-(8) that the
    multiplier closure scales: electron drift -n mu_e E and diffusion
    -(D_e dn + n D_e' dT) (scaled by m_D), energy flux H (all of it scaled by
    m_eps, since beta and G are 3/2 T mu_eps and 3/2 T D_eps)."""
    n, eps, E, dn, de = X.T
    Te = 2.0 / 3.0 * eps
    dT = 2.0 / 3.0 * de
    mue = np.interp(Te, T, cols[:, 0]) / Ngas
    De = np.interp(Te, T, cols[:, 1]) / Ngas
    h = 1e-3
    dDe = (np.interp(Te + h, T, cols[:, 1]) - np.interp(Te - h, T, cols[:, 1])) / (2 * h) / Ngas
    drift = -n * mue * E
    diff = -(De * dn + n * dDe * dT)
    H = table_fluxes(X, T, cols, Ngas)[:, 1]
    return drift, diff, H


def multiplier_targets(X, Y, T, cols, Ngas, k: int = 64, lo: float = 0.25, hi: float = 4.0):
    """Targets (m_D, m_eps) of the multiplier closure at every sample: the
    least-squares multipliers over the sample's k nearest neighbours in
    normalised feature space, m_D = sum a r / sum a^2 with a the table's
    diffusive electron flux and r = Gamma - (table drift flux), m_eps =
    sum H_table H / sum H_table^2 (one sample alone is too noisy where the
    table flux is small), clipped to [lo, hi]."""
    from scipy.spatial import cKDTree
    drift, diff, Ht = table_terms(X, T, cols, Ngas)
    r = Y[:, 0] - drift
    Z = (X - X.mean(0)) / (X.std(0) + 1e-30)
    _, nb = cKDTree(Z).query(Z, k=k)
    mD = (diff[nb] * r[nb]).sum(1) / np.maximum((diff[nb] ** 2).sum(1), 1e-300)
    mE = (Ht[nb] * Y[nb, 1]).sum(1) / np.maximum((Ht[nb] ** 2).sum(1), 1e-300)
    return np.stack([np.clip(mD, lo, hi), np.clip(mE, lo, hi)], axis=1)


def normalisation(X, Y):
    """(v - mean) / std inputs, std * y + mean outputs: the 14 numbers of
    include/pc_fluid.h."""
    mx, sx = X.mean(0), X.std(0) + 1e-30
    my, sy = Y.mean(0), Y.std(0) + 1e-30
    return np.concatenate([mx, 1.0 / sx, sy, my]).astype(np.float32)


def normalise(X, Y, norm):
    xn = (X - norm[:5]) * norm[5:10]
    yn = None if Y is None else (Y - norm[12:14]) / norm[10:12]
    return xn.astype(np.float32), (None if yn is None else yn.astype(np.float32))


def train(X, Y, steps=2000, lr=2e-3, batch=4096, seed=0, norm=None):
    """Train a closure network on the GPU (the library's forward, backward
    and Adam kernels) on normalised samples; returns (net, norm, losses)."""
    from .mlp import ClosureNet, glorot_params
    if norm is None:
        norm = normalisation(X, Y)
    xn, yn = normalise(X, Y, norm)
    net = ClosureNet(glorot_params(seed), max_batch=max(batch, 1024))
    losses = net.train(torch.from_numpy(xn), torch.from_numpy(yn), steps=steps, lr=lr, batch=batch, seed=seed)
    return net, norm, losses


def predict(net, X, norm):
    """Fluxes (physical units) predicted by a trained network."""
    xn, _ = normalise(X, None, norm)
    y = net.forward(torch.from_numpy(xn)).cpu().numpy().astype(np.float64)
    return y * norm[10:12] + norm[12:14]


def fluid_striations(table, T_min: float, T_step: float, Ngas: float, E0: float, L: float, n_cells: int,
                     dt: float, steps: int, every: int = 100, net=None, norm=None, muiN: float = 4.0e21,
                     seed: int = 1, multipliers: bool = False):
    """Free run of GPU fluid columns (two identical columns) at the mean field
    E0 from the homogeneous steady state of the table (nu_w = nu_i(T0)) with a
    1e-3 density noise, with the table closure or, given (net, norm), the
    learned one (fluxes, or with `multipliers` the multiplier form).  Returns (times, dominant mode, its modulation) of column 0
    every `every` steps: lambda = L / mode, to set against the PIC column."""
    from . import stability as S
    from .fluid import FluidBatch
    T0 = S.temperature_for_field(table, T_min, T_step, Ngas, E0)
    nu_w = Ngas * S._row(np.asarray(table, dtype=np.float64), T_min, T_step, T0)[0][4]
    fb = FluidBatch([dict(L=L, Ngas=Ngas, E0=E0, nu_w=nu_w, muiN=muiN)] * 2, n_cells, dt, table, T_min, T_step)
    if net is not None:
        fb.set_closure(net, norm, multipliers=multipliers)
    rng = np.random.default_rng(seed)
    n0 = 1e15 * (1.0 + 1e-3 * rng.normal(size=(2, n_cells)))
    fb.set_state(n0, 1.5 * n0 * T0)
    out = []
    for s in range(steps // every):
        fb.step(every)
        n, _ = (t.cpu().numpy().astype(np.float64) for t in fb.get_state())
        sp = np.abs(np.fft.rfft(n[0] - n[0].mean()))
        m = int(np.argmax(sp[1:]) + 1)
        out.append(((s + 1) * every * dt, m, 2.0 * sp[m] / n_cells / n[0].mean()))
    a = np.array(out)
    return a[:, 0], a[:, 1].astype(int), a[:, 2]


def fluid_ensemble(table, T_min: float, T_step: float, Ngas: float, E0: float, L: float, n_cells: int,
                   dt: float, steps: int, n_columns: int, snapshots: int = 10, net=None, norm=None,
                   multipliers: bool = False, muiN: float = 4.0e21, seed: int = 1, timed=None):
    """Free runs of n_columns identical fluid columns in one batch, each from
    the table's homogeneous steady state (nu_w = nu_i(T0)) with its own 1e-3
    density noise: every column is one realization.  The dominant mode and
    its modulation are taken from `snapshots` states spread over the second
    half of the run.  timed = (warmup, n): also time n steps after `warmup`
    (microseconds per step).  Returns dict(wavelength [m] per column (nan
    where the column did not striate: mean modulation <= 0.2), modulation,
    us_per_step)."""
    import time
    from . import stability as S
    from .fluid import FluidBatch
    T0 = S.temperature_for_field(table, T_min, T_step, Ngas, E0)
    nu_w = Ngas * S._row(np.asarray(table, dtype=np.float64), T_min, T_step, T0)[0][4]
    fb = FluidBatch([dict(L=L, Ngas=Ngas, E0=E0, nu_w=nu_w, muiN=muiN)] * n_columns, n_cells, dt, table,
                    T_min, T_step)
    if net is not None:
        fb.set_closure(net, norm, multipliers=multipliers)
    rng = np.random.default_rng(seed)
    n0 = 1e15 * (1.0 + 1e-3 * rng.normal(size=(n_columns, n_cells)))
    fb.set_state(n0, 1.5 * n0 * T0)
    done, us = 0, None
    if timed is not None:
        fb.step(timed[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fb.step(timed[1])
        torch.cuda.synchronize()
        us = (time.perf_counter() - t0) * 1e6 / timed[1]
        done = timed[0] + timed[1]
    marks = [steps // 2 + (steps - steps // 2) * (k + 1) // snapshots for k in range(snapshots)]
    modes, mods = [], []
    for m in marks:
        if m > done:
            fb.step(m - done)
            done = m
        n = fb.get_state()[0].cpu().numpy().astype(np.float64)
        sp = np.abs(np.fft.rfft(n - n.mean(axis=1, keepdims=True), axis=1))
        k = np.argmax(sp[:, 1:], axis=1) + 1
        modes.append(k)
        mods.append(2.0 * sp[np.arange(n_columns), k] / n_cells / n.mean(axis=1))
    modes, mods = np.array(modes), np.array(mods)
    mod = mods.mean(axis=0)
    lam = np.where(mod > 0.2, (L / modes).mean(axis=0), np.nan)
    return dict(wavelength=lam, modulation=mod, us_per_step=us, steps=steps, T0=T0, nu_w=nu_w)


def train_multipliers(seeds=(1, 2, 3, 4), warm: int = 100_000, steps: int = 100_000, train_steps: int = 4000,
                      table=None, k: int = 64):
    """The multiplier closure of the striated neon column: samples of the
    20 cm column (1 Torr, 10 V/cm, 400k + 400k) in its saturated striated
    state for each seed, local least-squares targets (multiplier_targets)
    against the two-term table, GPU training.  Returns (net, norm, info)."""
    import workloads as W
    cfgs = [W.with_(W.column_20cm(), n_cells=2000, L=0.20, V=200.0, ppc=200, wall_mode="balanced", seed=s)
            for s in seeds]
    X, Y, col = striated_samples(cfgs, warm=warm, steps=steps, every=5, window=500, group=4)
    Ngas = float(cfgs[0]["p_torr"]) * 133.322368 / (1.380649e-23 * float(cfgs[0]["Tg"]))
    if table is None:
        T, cols = transport_table(cfgs[0], np.geomspace(1e-22, 3e-19, 200), Ngas)
    else:
        T, cols = table
    M = multiplier_targets(X, Y, T, cols, Ngas, k=k)
    net, norm, losses = train(X, M, steps=train_steps, lr=2e-3, batch=4096, seed=0)
    drift, diff, Ht = table_terms(X, T, cols, Ngas)
    r = Y[:, 0] - drift
    info = dict(samples=int(X.shape[0]), m_D_global=float((diff * r).sum() / (diff ** 2).sum()),
                m_eps_global=float((Ht * Y[:, 1]).sum() / (Ht ** 2).sum()),
                m_D_median=float(np.median(M[:, 0])), m_eps_median=float(np.median(M[:, 1])),
                loss_first=float(losses[:10].mean()), loss_last=float(losses[-100:].mean()))
    return net, norm, info


if __name__ == "__main__":
    # python -m paper_2202_03215_amd.closure OUT.npz: train the multiplier
    # closure of the striated neon column on the GPU and store its weights
    import json
    import sys
    net, norm, info = train_multipliers()
    np.savez(sys.argv[1], theta=net.params().astype(np.float32), norm=norm.astype(np.float32))
    print(json.dumps(info))
