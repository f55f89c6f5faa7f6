"""The oracle's two other builds (CPU only).

- The OpenMP timing build (libpco_omp.so, all host cores) must compute bit
  for bit what the serial parity build computes: positions, velocities, ids,
  charges, field, counts and per-id events after the whole 2000-step run of
  the 4 cm bounded neon column (20k + 20k, the small workload), and after
  shorter runs with the pair sink and with cathode emission and the series
  resistor (section V).  Its parallel loops only add integers and or bits
  into shared data, and the ionizations are sorted by parent id before use,
  so any thread schedule gives the serial result.
- The pins of the particle oracle run again against an AddressSanitizer +
  UndefinedBehaviorSanitizer build (libpco_asan.so, host code only) in a
  child process; any out-of-bounds access, use after free or undefined
  operation aborts it.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads as W
from oracle import pco

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _snapshot(o):
    st = [o.state(s) for s in (0, 1)]
    E, re, ri = o.field()
    ev = [o.events(s) for s in (0, 1)]
    return st, (E, re, ri), ev, (o.count(0), o.count(1), o.next_id(0), o.next_id(1), o.errors)


def _equal(a, b):
    (sa, fa, ea, ca), (sb, fb, eb, cb) = a, b
    assert ca == cb
    for s in (0, 1):
        for u, v in zip(sa[s], sb[s]):
            assert np.array_equal(u, v)
        assert np.array_equal(ea[s], eb[s])
    for u, v in zip(fa, fb):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("case", ["small_bounded", "pair", "hot_cathode"])
def test_openmp_build_matches_serial_build(case):
    if case == "small_bounded":
        cfg, steps = W.small_bounded(), 2000
    elif case == "pair":
        cfg, steps = W.tiny("periodic", V=0.0037 * 6000.0, wall_mode="pair", ppc=60), 300
    else:
        cfg, steps = W.with_(W.hot_cathode_15cm(ppc=20), n_cells=150, L=0.015, V=60.0), 300
    pco.threads(4)
    out = []
    for omp in (False, True):
        o = pco.Oracle(cfg, omp=omp)
        o.step(steps)
        out.append(_snapshot(o))
    assert out[0][3][4] == 0
    _equal(out[0], out[1])


def test_oracle_pins_under_address_and_undefined_sanitizers():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.exists(asan):
        pytest.skip("no libasan in this toolchain")
    env = dict(os.environ)
    env.update(PCO_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    files = ["test_oracle_push.py", "test_oracle_deposit_field.py", "test_oracle_mcc.py",
             "test_oracle_moments.py", "test_oracle_pair.py", "test_oracle_circuit.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider"] +
                       [os.path.join(ROOT, "tests", f) for f in files],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-3000:] + r.stderr[-3000:])
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert os.path.exists(os.path.join(ROOT, "oracle", "libpco_asan.so"))
