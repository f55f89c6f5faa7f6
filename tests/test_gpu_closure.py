"""What the learned closure gains over the table closure, on PIC-MCC data.

Samples come from GPU PIC-MCC neon columns started from density and
temperature modulations (so that gradients and non-local transport are
present): time- and cell-group-averaged moments give (n, mean energy, E,
gradients) -> (electron flux, energy flux).  The closure network is trained
on the GPU on some columns and evaluated on held-out columns, next to the
drift-diffusion closure of eqs. (7)-(8) with coefficients from the two-term
Boltzmann tables of the same cross sections (the method without the
network).  The network must predict the held-out PIC fluxes with a clearly
smaller error.
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


def _columns():
    cols = []
    for k, (ev, mode, seed) in enumerate(((6.0, 2, 1), (9.0, 3, 2), (12.0, 2, 3), (15.0, 4, 4),
                                          (7.5, 3, 5), (13.5, 2, 6), (10.5, 3, 7), (8.0, 4, 8))):
        cols.append(W.tiny("periodic", n_cells=400, L=0.02, V=0.02 * ev * 100.0, ppc=300, n0=1.0e15,
                           Te0_eV=3.0, nu_w=4.0e6, capacity=2.0, seed=seed, sort_interval=20))
    return cols


def _nmse(p, y):
    return float(np.mean([np.mean((p[:, k] - y[:, k]) ** 2) / np.var(y[:, k]) for k in range(2)]))


def test_learned_closure_beats_table_closure_on_held_out_pic_columns(torch_cuda):
    from paper_2202_03215_amd import closure as CL
    cfgs = _columns()
    X, Y, col = CL.pic_samples(cfgs, steps=5000, every=5, window=500, group=4, amp_n=0.35, amp_T=0.3, seed=11)
    keep = np.isin(np.arange(X.shape[0]) // 100 % 10, np.arange(2, 10))   # drop the first two windows
    X, Y, col = X[keep], Y[keep], col[keep]
    test = col >= 6
    assert test.sum() >= 1600 and (~test).sum() >= 4800
    Ngas = 1.0 * 133.322368 / (1.380649e-23 * 300.0)
    T, tab = CL.transport_table(W.tiny(), np.geomspace(2e-21, 4e-19, 40), Ngas)
    pt = CL.table_fluxes(X[test], T, tab, Ngas)
    net, norm, losses = CL.train(X[~test], Y[~test], steps=3000, lr=2e-3, batch=2048, seed=0)
    assert np.all(np.isfinite(losses)) and losses[-100:].mean() < losses[:10].mean()
    pm = CL.predict(net, X[test], norm)
    e_table = _nmse(pt, Y[test])
    e_net = _nmse(pm, Y[test])
    print(f"normalised MSE on held-out columns: table closure {e_table:.4f}, network {e_net:.4f}")
    assert e_net < 0.7 * e_table, (e_net, e_table)


def test_sample_pipeline_against_table_closure_in_a_uniform_column(torch_cuda):
    """Control of units and signs: without modulation the column is a swarm
    in a uniform field, where the drift-diffusion closure with two-term
    coefficients holds (its drift velocity and mean energy agree with the
    oracle swarm within 3 %): mean fluxes must agree within 10 %."""
    from paper_2202_03215_amd import closure as CL
    cfg = W.tiny("periodic", n_cells=400, L=0.02, V=0.02 * 1000.0, ppc=300, n0=1.0e15, Te0_eV=3.0,
                 nu_w=4.0e6, capacity=2.0, seed=21, sort_interval=20)
    X, Y, _ = CL.pic_samples([cfg], steps=5000, every=5, window=500, group=4, amp_n=0.0, amp_T=0.0, seed=3)
    X, Y = X[400:], Y[400:]                                   # after four windows of relaxation
    Ngas = 1.0 * 133.322368 / (1.380649e-23 * 300.0)
    T, tab = CL.transport_table(W.tiny(), np.geomspace(2e-21, 4e-19, 40), Ngas)
    pt = CL.table_fluxes(X, T, tab, Ngas)
    assert X[:, 2].mean() > 0 and Y[:, 0].mean() < 0         # fluid convention: E0 > 0, electrons drift to -x
    for k in range(2):
        r = Y[:, k].mean() / pt[:, k].mean()
        print(f"uniform column, output {k}: PIC / table = {r:.3f}")
        assert abs(r - 1.0) < 0.10, (k, r)


def test_multiplier_closure_on_striated_pic_columns(torch_cuda):
    """The learned closure in multiplier form (network answers m_D for the
    electron diffusion and m_eps for the energy transport of the two-term
    table) trained on the striated 20 cm neon column (1 Torr, 10 V/cm,
    saturated ionization wave), evaluated on a held-out realization.

    What it gains: the table's local drift-diffusion fluxes at the PIC
    column's own field and gradients miss the PIC fluxes by far (normalised
    MSE in the hundreds for the electron flux); the learned multipliers
    bring it down by more than 10x, and the energy flux error below 0.8x.
    What it finds (recorded reading, not a goal): the PIC's effective
    electron diffusion is a fraction of the local two-term value (global
    least-squares m_D below 0.6), and a fluid column carrying these
    multipliers does not striate at this field (the fluid model's own
    instability needs the local-field diffusion), while the table closure
    does."""
    import workloads as W
    from paper_2202_03215_amd import closure as CL
    from tests.gpu_helpers import striation_config
    cfgs = [striation_config("20cm", s) for s in (1, 2)]
    X, Y, col = CL.striated_samples(cfgs, warm=100_000, steps=50_000, every=5, window=500, group=4)
    Ngas = 1.0 * 133.322368 / (1.380649e-23 * 300.0)
    T = W.FLUID_T_MIN + W.FLUID_T_STEP * np.arange(W.FLUID_T_LEN)
    tab = W.fluid_table_ne()
    tr, te = col == 0, col == 1
    M = CL.multiplier_targets(X[tr], Y[tr], T, tab, Ngas, k=64)
    net, norm, losses = CL.train(X[tr], M, steps=2000, lr=2e-3, batch=4096, seed=0)
    assert np.all(np.isfinite(losses)) and losses[-100:].mean() < losses[:10].mean()
    drift, diff, Ht = CL.table_terms(X[te], T, tab, Ngas)
    m = np.clip(CL.predict(net, X[te], norm), 0.25, 4.0)
    pt = CL.table_fluxes(X[te], T, tab, Ngas)
    pm = np.stack([drift + m[:, 0] * diff, m[:, 1] * Ht], axis=1)
    e_table = [np.mean((pt[:, k] - Y[te, k]) ** 2) / np.var(Y[te, k]) for k in range(2)]
    e_net = [np.mean((pm[:, k] - Y[te, k]) ** 2) / np.var(Y[te, k]) for k in range(2)]
    dr, df, _ = CL.table_terms(X[tr], T, tab, Ngas)
    mD = float((df * (Y[tr, 0] - dr)).sum() / (df ** 2).sum())
    print(f"held-out normalised MSE: electron flux table {e_table[0]:.1f} / learned {e_net[0]:.2f}, energy flux "
          f"table {e_table[1]:.3f} / learned {e_net[1]:.3f}; global m_D {mD:.3f}")
    assert e_net[0] < 0.1 * e_table[0] and e_net[1] < 0.8 * e_table[1]
    assert mD < 0.6
    runs = {}
    for name, kw in (("table", {}), ("learned", dict(net=net, norm=norm, multipliers=True))):
        r = CL.fluid_ensemble(tab, W.FLUID_T_MIN, W.FLUID_T_STEP, Ngas, 1000.0, 0.2, 1024, 1e-9, 20_000, 16, **kw)
        runs[name] = r
        print(name, "striated fraction", np.isfinite(r["wavelength"]).mean(), "modulation",
              np.round(r["modulation"], 2).tolist())
    assert np.isfinite(runs["table"]["wavelength"]).mean() >= 0.5
    assert np.isfinite(runs["learned"]["wavelength"]).mean() == 0.0    # no column reaches modulation 0.2
