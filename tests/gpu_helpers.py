"""Shared helpers of the GPU parity tests (HIP path through the C ABI versus
the CPU oracle on the same seeded inputs)."""
from __future__ import annotations

import numpy as np

ELECTRON, ION = 0, 1

# per-step parity tolerances (see the parity contract in the design notes)
TOL_E = 1e-12        # field: max |dE| <= TOL_E * max |E|
TOL_PHI = 1e-12      # potential: max |dphi| <= TOL_PHI * max(max |phi|, V)
TOL_X = 1e-12        # positions: |dx| <= TOL_X * L
TOL_V = 1e-12        # velocities: |dv| <= TOL_V * (|v| + v_th)


def by_id(state):
    """Sort a (x, vx, vy, vz, id) tuple by id; returns numpy arrays."""
    arrs = [a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a) for a in state]
    ids = arrs[4].astype(np.uint32)
    o = np.argsort(ids, kind="stable")
    return [a[o] for a in arrs[:4]] + [ids[o]]


def gpu_state(col, s):
    return by_id(col.get_state(s))


def copy_gpu_to_oracle(col, orc):
    """Give the oracle the GPU column's exact state: particles, field E^n,
    step index and next ids."""
    c = col.counts()
    for s in (ELECTRON, ION):
        x, vx, vy, vz, ids = gpu_state(col, s)
        orc.set_state(s, x, vx, vy, vz, ids)
    E, _, _ = col.get_field()
    orc.set_field(E.cpu().numpy())
    orc.set_counters(c["step"], c["next_id"][0], c["next_id"][1])
    orc.set_balance(*c["balance"])
    orc.set_circuit(*c["circuit"])


def compare_states(col, orc, L, vth, exact_v=False):
    """Compare GPU and oracle particle sets by id; returns a dict of maxima."""
    out = {}
    for s in (ELECTRON, ION):
        g = gpu_state(col, s)
        o = by_id(orc.state(s))
        assert g[4].size == o[4].size, f"species {s}: {g[4].size} vs {o[4].size} particles"
        assert np.array_equal(g[4], o[4]), f"species {s}: id sets differ"
        dx = np.abs(g[0] - o[0]).max(initial=0.0)
        assert dx <= TOL_X * L, f"species {s}: max |dx| = {dx}"
        for k in (1, 2, 3):
            scale = np.abs(o[k]) + vth[s]
            dv = (np.abs(g[k] - o[k]) / scale).max(initial=0.0)
            assert dv <= TOL_V, f"species {s} component {k}: max rel dv = {dv}"
            if exact_v:
                assert np.array_equal(g[k], o[k])
        out[s] = dx
    return out


def field_close(Eg, Eo):
    Eg = np.asarray(Eg)
    Eo = np.asarray(Eo)
    return np.abs(Eg - Eo).max() <= TOL_E * np.abs(Eo).max()


# ------------------------------------------- striated free runs (shared)
_STRIATION_RUNS = {}


def striation_config(column, seed, precision="fp64"):
    """The striated neon columns of the long-run tests and of the oracle's
    golden runs (1 Torr, periodic, E0 = 10 V/cm, balanced sink)."""
    import workloads as W
    s = {"4cm": dict(n_cells=400, L=0.04, ppc=100), "20cm": dict(n_cells=2000, L=0.20, ppc=200)}[column]
    return W.with_(W.column_20cm(), n_cells=s["n_cells"], L=s["L"], V=s["L"] * 1000.0, ppc=s["ppc"],
                   wall_mode="balanced", seed=seed, precision=precision)


def striation_run(column, seed, precision, steps=200_000, every=None, modes=None):
    """GPU free run of a striated column (2e5 steps), cached per process:
    Fourier coefficients of the electron cell counts (modes 0..M) every
    `every` steps, their times, the EEPF counts and energy sums over the
    second half."""
    from paper_2202_03215_amd import physics as PH
    every = every or (1000 if column == "4cm" else 2000)
    modes = modes or (32 if column == "4cm" else 64)
    key = (column, seed, precision, steps, every, modes)
    if key not in _STRIATION_RUNS:
        cfg = striation_config(column, seed, precision)
        r = PH.run(cfg, steps, every, eepf_from=steps // 2 + every)
        coef = np.fft.rfft(r["ne"], axis=1)[:, :modes + 1]
        _STRIATION_RUNS[key] = dict(coef=coef, times=r["times"], eepf=r["eepf"], energy_sum=r["energy_sum"],
                                    energy_count=r["energy_count"], counts=r["counts"], cfg=cfg)
    return _STRIATION_RUNS[key]
