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
