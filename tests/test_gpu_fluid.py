"""Batched fluid column on the GPU against the FP64 fluid oracle.

- cyclic tridiagonal solve (cyclic reduction in LDS, FP64) against a sparse
  LU solve: residual-level agreement (<= 1e-12 relative), on random
  diagonally dominant systems and on weakly dominant backward-Euler
  diffusion systems (r = 50);
- one step from a shared state, table closure: FP32 state and fluxes, FP64
  solves.  The differences come from FP32 rounding of the explicit terms
  (single precision, 6e-8, amplified by differences such as Phi_{j+1} -
  Phi_j in the field); the bound 2e-5 relative on n and T holds with a wide
  margin at the cell counts tested;
- 40 steps: 2e-4 relative (the FP32 differences of each step, carried);
- network closure: one step within 2e-3 relative (BF16 inputs and weights
  make the fluxes differ where FP32 and FP64 inputs round to different
  BF16 values).
"""
import numpy as np
import pytest

import workloads as W
from oracle import fluid as F
from oracle import mlp as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("n,weak", [(8, False), (32, False), (64, False), (128, True), (1024, False),
                                    (4096, False), (4096, True)])
def test_cyclic_tridiagonal_solve(torch_cuda, n, weak):
    from paper_2202_03215_amd.fluid import cyclic_tridiag
    torch = torch_cuda
    rng = np.random.default_rng(n)
    ns = 3
    if weak:   # backward-Euler diffusion at r = 50: 1 + r (D_- + D_+) on the diagonal
        D = 0.5 + rng.random((ns, n))
        a = -50.0 * np.roll(D, 1, axis=1)
        c = -50.0 * D
        b = 1.0 - a - c
    else:
        a = -rng.random((ns, n))
        c = -rng.random((ns, n))
        b = 1.0 + np.abs(a) + np.abs(c) + rng.random((ns, n))
    d = rng.normal(size=(ns, n))
    x = cyclic_tridiag(*(torch.from_numpy(v).cuda() for v in (a, b, c, d))).cpu().numpy()
    for s in range(ns):
        ref = F.cyclic_solve(a[s], b[s], c[s], d[s])
        assert np.abs(x[s] - ref).max() <= 1e-12 * np.abs(ref).max()


def _columns(n_cells, table, dt, T_step=W.FLUID_T_STEP):
    cols = []
    for k, (L, p, dE) in enumerate(((0.05, 1.0, 1.0), (0.08, 0.7, 1.15), (0.03, 1.5, 0.9))):
        Ng = 3.22e22 * p
        c = F.FluidColumn(n_cells=n_cells, L=L, Ngas=Ng, E0=0.0, nu_w=2.0e4 / p, muiN=4.0e21, dt=dt,
                          T_min=W.FLUID_T_MIN, T_step=T_step, table=table)
        T0, E0 = F.steady_temperature(c)
        c.E0 = E0 * dE
        cols.append((c, T0))
    return cols


def _state(cols, n_cells, seed):
    rng = np.random.default_rng(seed)
    ns, ws = [], []
    for c, T0 in cols:
        x = (np.arange(n_cells) + 0.5) / n_cells
        n = 1e15 * (1.0 + 0.1 * np.cos(2 * np.pi * 3 * x) + 0.02 * rng.normal(size=n_cells))
        T = T0 * (1.0 + 0.05 * np.sin(2 * np.pi * 2 * x))
        ns.append(n)
        ws.append(1.5 * n * T)
    return np.array(ns), np.array(ws)


def _batch(cols, n_cells, dt, table, T_step=W.FLUID_T_STEP):
    from paper_2202_03215_amd.fluid import FluidBatch
    spec = [dict(L=c.L, Ngas=c.Ngas, E0=c.E0, nu_w=c.nu_w, muiN=c.muiN) for c, _ in cols]
    return FluidBatch(spec, n_cells, dt, table, W.FLUID_T_MIN, T_step)


@pytest.mark.parametrize("n_cells,steps,tol", [(64, 1, 2e-5), (512, 1, 2e-5), (4096, 1, 2e-5), (256, 40, 2e-4)])
def test_fluid_steps_against_oracle(torch_cuda, n_cells, steps, tol):
    table = W.fluid_table_smooth()
    dt = 2e-9
    cols = _columns(n_cells, table, dt)
    n0, w0 = _state(cols, n_cells, n_cells)
    n0 = n0.astype(np.float32).astype(np.float64)
    w0 = w0.astype(np.float32).astype(np.float64)
    fb = _batch(cols, n_cells, dt, table)
    fb.set_state(n0, w0)
    fb.step(steps)
    ng, wg = (t.cpu().numpy().astype(np.float64) for t in fb.get_state())
    for k, (c, _) in enumerate(cols):
        n, w = F.run(c, n0[k], w0[k], steps)
        Tg, To = wg[k] / (1.5 * ng[k]), w / (1.5 * n)
        assert np.abs(ng[k] - n).max() <= tol * n.mean(), (k, np.abs(ng[k] - n).max() / n.mean())
        assert np.abs(Tg - To).max() <= tol * To.mean(), (k, np.abs(Tg - To).max() / To.mean())
    if steps == 1:
        g, H, E = (t.cpu().numpy().astype(np.float64) for t in fb.faces())
        d = cols[0][0].diag
        assert np.abs(E[0] - d["E"]).max() <= 1e-4 * np.abs(d["E"]).max()


def test_fluid_step_longest_table_against_oracle(torch_cuda):
    """The kernels stage the table in LDS, at most 1024 rows: the smooth
    table resampled on a T grid of 1024 rows over the same range, one step
    of 4096 cells against the oracle on the same table (bound as above)."""
    base = np.asarray(W.fluid_table_smooth(), dtype=np.float64)
    K = 1024
    T_base = W.FLUID_T_MIN + W.FLUID_T_STEP * np.arange(len(base))
    T_step = (T_base[-1] - W.FLUID_T_MIN) / (K - 1)
    T_new = W.FLUID_T_MIN + T_step * np.arange(K)
    table = np.stack([np.interp(T_new, T_base, base[:, q]) for q in range(base.shape[1])], axis=1)
    n_cells, dt = 4096, 2e-9
    cols = _columns(n_cells, table, dt, T_step)
    n0, w0 = _state(cols, n_cells, 7)
    n0 = n0.astype(np.float32).astype(np.float64)
    w0 = w0.astype(np.float32).astype(np.float64)
    fb = _batch(cols, n_cells, dt, table, T_step)
    fb.set_state(n0, w0)
    fb.step(1)
    ng, wg = (t.cpu().numpy().astype(np.float64) for t in fb.get_state())
    for k, (c, _) in enumerate(cols):
        n, w = F.run(c, n0[k], w0[k], 1)
        Tg, To = wg[k] / (1.5 * ng[k]), w / (1.5 * n)
        assert np.abs(ng[k] - n).max() <= 2e-5 * n.mean(), (k, np.abs(ng[k] - n).max() / n.mean())
        assert np.abs(Tg - To).max() <= 2e-5 * To.mean(), (k, np.abs(Tg - To).max() / To.mean())


def test_fluid_full_size_against_oracle(torch_cuda):
    # the bench's fluid workload: 256 columns x 4096 cells (20 cm, pressures
    # 0.5-2 Torr, 5 % density modulations), table closure, one launch per
    # kernel for all columns; after 4 steps columns 0, 127 and 255 against
    # the oracle
    table = W.fluid_table_smooth()
    ncol, ncell, dt, L, steps = 256, 4096, 2.0e-9, 0.20, 4
    rng = np.random.default_rng(5)
    spec = []
    for c in range(ncol):
        p = float(np.exp(rng.uniform(np.log(0.5), np.log(2.0))))
        spec.append(dict(L=L, Ngas=3.22e22 * p, E0=300.0 * p * float(rng.uniform(0.9, 1.3)), nu_w=2.0e4 / p,
                         muiN=4.0e21))
    x = (np.arange(ncell) + 0.5) / ncell
    n0 = np.array([1e15 * (1.0 + 0.05 * np.cos(2 * np.pi * (2 + c % 5) * x)) for c in range(ncol)])
    w0 = 1.5 * n0 * 3.0
    n0 = n0.astype(np.float32).astype(np.float64)
    w0 = w0.astype(np.float32).astype(np.float64)
    from paper_2202_03215_amd.fluid import FluidBatch
    fb = FluidBatch(spec, ncell, dt, table, W.FLUID_T_MIN, W.FLUID_T_STEP)
    fb.set_state(n0, w0)
    fb.step(steps)
    ng, wg = (t.cpu().numpy().astype(np.float64) for t in fb.get_state())
    for k in (0, 127, 255):
        c = F.FluidColumn(n_cells=ncell, T_min=W.FLUID_T_MIN, T_step=W.FLUID_T_STEP, table=table, dt=dt,
                          **spec[k])
        n, w = F.run(c, n0[k], w0[k], steps)
        Tg, To = wg[k] / (1.5 * ng[k]), w / (1.5 * n)
        assert np.abs(ng[k] - n).max() <= 1e-4 * n.mean(), (k, np.abs(ng[k] - n).max() / n.mean())
        assert np.abs(Tg - To).max() <= 1e-4 * To.mean(), (k, np.abs(Tg - To).max() / To.mean())


def test_fluid_network_closure_against_oracle(torch_cuda):
    from paper_2202_03215_amd.mlp import ClosureNet
    n_cells = 256
    table = W.fluid_table_smooth()
    dt = 1e-9
    cols = _columns(n_cells, table, dt)
    n0, w0 = _state(cols, n_cells, 5)
    n0 = n0.astype(np.float32).astype(np.float64)
    w0 = w0.astype(np.float32).astype(np.float64)
    # a network with small outputs around the drift fluxes of the column
    rng = np.random.default_rng(0)
    th = O.init_params(4)
    W1, b1, W2, b2, W3, b3, W4, b4 = O.unpack(th)
    th = O.pack([W1, b1, W2, b2, W3, b3, W4 * 0.05, rng.normal(0, 0.02, 2)]).astype(np.float32).astype(np.float64)
    norm = np.array([1e15, 6.0, 500.0, 0.0, 0.0,            # input offsets
                     1e-15, 0.3, 2e-3, 1e-17, 3e-3,          # input scales
                     -3e19, -2e20, -1.0e20, -6e20], dtype=np.float32)   # output scales, offsets
    nz = norm.astype(np.float64)

    def closure(feats):
        x = (feats - nz[:5]) * nz[5:10]
        y, _ = O.forward(th, x, emulate=True)
        return y[:, 0] * nz[10] + nz[12], y[:, 1] * nz[11] + nz[13]

    net = ClosureNet(th)
    fb = _batch(cols, n_cells, dt, table)
    fb.set_closure(net, norm)
    fb.set_state(n0, w0)
    fb.step(1)
    ng, wg = (t.cpu().numpy().astype(np.float64) for t in fb.get_state())
    for k, (c, _) in enumerate(cols):
        c.closure = closure
        n, w = F.step(c, n0[k], w0[k])
        Tg, To = wg[k] / (1.5 * ng[k]), w / (1.5 * n)
        assert np.abs(ng[k] - n).max() <= 2e-3 * n.mean(), (k, np.abs(ng[k] - n).max() / n.mean())
        assert np.abs(Tg - To).max() <= 2e-3 * To.mean(), (k, np.abs(Tg - To).max() / To.mean())
        assert np.abs(ng[k] - n0[k]).max() > 1e-4 * n.mean()      # the closure moved the state


def test_fluid_multiplier_closure_against_oracle(torch_cuda):
    """Multiplier closure: the network answers (m_D, m_eps) multipliers of
    the tabulated coefficients.  Step 1 uses no multipliers and must equal
    the table closure's step bit for bit; 40 steps against the oracle with
    the same network (BF16 emulated): within 2e-3 relative (inputs rounding
    to different BF16 values on the two sides move a multiplier by at most
    about one BF16 ulp of its input's influence, each step)."""
    from paper_2202_03215_amd.mlp import ClosureNet
    torch = torch_cuda
    n_cells, dt = 256, 2e-9
    table = W.fluid_table_smooth()
    cols = _columns(n_cells, table, dt)
    n0, w0 = _state(cols, n_cells, 7)
    n0 = n0.astype(np.float32).astype(np.float64)
    w0 = w0.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(1)
    th = O.init_params(6)
    W1, b1, W2, b2, W3, b3, W4, b4 = O.unpack(th)
    th = O.pack([W1, b1, W2, b2, W3, b3, W4 * 0.3, rng.normal(0, 0.1, 2)]).astype(np.float32).astype(np.float64)
    norm = np.array([1e15, 6.0, 500.0, 0.0, 0.0,
                     1e-15, 0.3, 2e-3, 1e-17, 3e-3,
                     0.3, 0.4, 1.0, 1.1], dtype=np.float32)          # m_D = 0.3 y0 + 1, m_eps = 0.4 y1 + 1.1
    nz = norm.astype(np.float64)

    def mult(feats):
        x = (feats - nz[:5]) * nz[5:10]
        y, _ = O.forward(th, x, emulate=True)
        return y[:, 0] * nz[10] + nz[12], y[:, 1] * nz[11] + nz[13]

    net = ClosureNet(th)
    fb = _batch(cols, n_cells, dt, table)
    fb.set_closure(net, norm, multipliers=True)
    fb.set_state(n0, w0)
    fb.step(1)
    n1, w1 = (t.cpu().numpy().copy() for t in fb.get_state())
    ft = _batch(cols, n_cells, dt, table)
    ft.set_state(n0, w0)
    ft.step(1)
    t1, s1 = (t.cpu().numpy() for t in ft.get_state())
    assert np.array_equal(n1, t1) and np.array_equal(w1, s1)
    fb.step(39)
    ng, wg = (t.cpu().numpy().astype(np.float64) for t in fb.get_state())
    ft.step(39)
    nt = ft.get_state()[0].cpu().numpy().astype(np.float64)
    for k, (c, _) in enumerate(cols):
        c.multipliers, c.m = mult, None
        n, w = F.run(c, n0[k], w0[k], 40)
        Tg, To = wg[k] / (1.5 * ng[k]), w / (1.5 * n)
        en = np.abs(ng[k] - n).max() / n.mean()
        eT = np.abs(Tg - To).max() / To.mean()
        print(f"column {k}: 40 steps, |dn| {en:.2e}, |dT| {eT:.2e}; multipliers m_D {c.m[0].min():.3f}..{c.m[0].max():.3f}, "
              f"m_eps {c.m[1].min():.3f}..{c.m[1].max():.3f}; off the table run by {np.abs(nt[k] - n).max() / n.mean():.2e}")
        assert en <= 2e-3 and eT <= 2e-3, (k, en, eT)
        assert np.abs(nt[k] - n).max() > 10 * np.abs(ng[k] - n).max()   # the multipliers moved the run
