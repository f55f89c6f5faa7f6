"""The bounded column of section V on the GPU: 15 cm neon gap at 1 Torr, a
hot cathode emitting 10 A/m^2, a 270 V source behind a 10 ohm m^2 resistor,
fixed radial loss frequency 1e6 /s; 1.5e6 steps (15 us) of FP64 particles.

- The circuit settles where the source voltage minus the resistor drop holds
  the anode: mean V_anode = V + R <J> within 1 % of V (the displacement
  current averages out), with an electron current towards the anode (J < 0).
- The column body (2 cm away from either electrode) striates: modulation
  above 0.3, waves moving towards the cathode.
- The anode sheath field changes sign (electron and ion sheaths alternate)
  at the frequency of the ionization wave: the dominant frequency of E at the
  anode node is v_ph / lambda within one and a half frequency bins (the
  paper reports the anode sheath oscillating in phase with the wave).
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


def test_hot_cathode_column_circuit_sheath_and_striations(torch_cuda):
    from paper_2202_03215_amd import physics as PH
    cfg = W.hot_cathode_15cm()
    res = PH.bounded_run(cfg, 1_500_000, 1000, snap_every=10)
    t = res["times"]
    late = t > 5e-6
    V, J, Ea = res["V"][late], res["J"][late], res["E_anode"][late]
    print(f"V {V.mean():.2f} +- {V.std():.2f} V, J {J.mean():.3f} A/m^2, counts {res['counts'][-1]}")
    assert J.mean() < 0.0
    assert abs(V.mean() - (cfg["V"] + cfg["circuit_R"] * J.mean())) <= 0.01 * cfg["V"]
    # striations in the body of the column
    nc, L = cfg["n_cells"], cfg["L"]
    lo, hi = int(0.02 / L * nc), int(0.13 / L * nc)
    ne = res["ne"][res["ne"].shape[0] // 2:, lo:hi]
    ts = t[9::10][res["ne"].shape[0] // 2:]
    prof = ne - ne.mean(axis=1, keepdims=True)
    spec = np.abs(np.fft.rfft(prof, axis=1))
    m = int(np.argmax(spec.mean(axis=0)[1:]) + 1)
    seg = (hi - lo) * L / nc
    lam = seg / m
    mod = float(np.mean(2.0 * spec[:, m] / prof.shape[1] / ne.mean(axis=1)))
    phase = np.unwrap(np.angle(np.fft.rfft(prof, axis=1)[:, m]))
    v_ph = -np.polyfit(ts, phase, 1)[0] / (2.0 * np.pi / lam)
    f_wave = abs(v_ph) / lam
    ea = Ea - Ea.mean()
    freqs = np.fft.rfftfreq(ea.size, t[1] - t[0])
    f_sheath = freqs[int(np.argmax(np.abs(np.fft.rfft(ea))[1:]) + 1)]
    print(f"mode {m}: lambda {lam * 100:.2f} cm, modulation {mod:.2f}, v_ph {v_ph:.0f} m/s, "
          f"wave {f_wave / 1e3:.0f} kHz, anode sheath {f_sheath / 1e3:.0f} kHz")
    assert mod > 0.3 and v_ph < 0.0
    assert Ea.min() < 0.0 < Ea.max()
    assert abs(f_sheath - f_wave) <= 1.5 * freqs[1]
