"""Pins of the oracle's Philox4x32-10 and of its uniform-variate conversion.

Philox4x32-10 is defined in Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11).  The oracle's implementation is checked
against an independent one: rocRAND's header-only device/host generator,
compiled here for the host and run as a black box.  rocRAND maps
rocrand_init(seed, subsequence, offset) to key = seed and counter =
(offset/4 low, offset/4 high, subsequence low, subsequence high).
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle.pco import philox4x32_10

KAT_SRC = r"""
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
  unsigned long long seeds[4] = {0ull, 1ull, 0x123456789abcdef0ull, 0xffffffffffffffffull};
  unsigned long long subs[3] = {0ull, 5ull, 0xfedcba9876543210ull};
  unsigned long long blocks[3] = {0ull, 7ull, (3ull << 32) | 11ull};
  for (int a = 0; a < 4; ++a) for (int b = 0; b < 3; ++b) for (int c = 0; c < 3; ++c) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seeds[a], subs[b], 4ull * blocks[c], &st);
    uint4 r = rocrand4(&st);
    printf("%llu %llu %llu %u %u %u %u\n", seeds[a], subs[b], blocks[c], r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


def _hipcc():
    for p in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if p and os.path.exists(p):
            return p
    return None


@pytest.fixture(scope="module")
def rocrand_kat():
    hipcc = _hipcc()
    if hipcc is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tempfile.mkdtemp()
    try:
        src = os.path.join(d, "kat.cpp")
        exe = os.path.join(d, "kat")
        with open(src, "w") as f:
            f.write(KAT_SRC)
        subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    finally:
        shutil.rmtree(d, ignore_errors=True)
    rows = []
    for line in out.strip().splitlines():
        s, q, b, *r = (int(t) for t in line.split())
        rows.append((s, q, b, r))
    return rows


def test_philox_matches_rocrand(rocrand_kat):
    assert len(rocrand_kat) == 36
    for s, q, b, ref in rocrand_kat:
        ctr = [b & 0xFFFFFFFF, b >> 32, q & 0xFFFFFFFF, q >> 32]
        key = [s & 0xFFFFFFFF, s >> 32]
        assert list(philox4x32_10(ctr, key)) == ref, (s, q, b)


def test_philox_is_counter_sensitive():
    base = philox4x32_10([1, 2, 3, 4], [5, 6])
    for k in range(4):
        c = [1, 2, 3, 4]
        c[k] ^= 1
        assert not np.array_equal(philox4x32_10(c, [5, 6]), base)
    assert not np.array_equal(philox4x32_10([1, 2, 3, 4], [5, 7]), base)


def test_philox_bits_uniform():
    # 4096 blocks -> 16384 words: each of the 32 bit positions is set with p = 1/2
    words = np.concatenate([philox4x32_10([i, 17, 0, 3], [1, 0]) for i in range(4096)])
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.float64)
    frac = bits.mean(axis=0)
    sd = math.sqrt(0.25 / words.size)
    assert np.all(np.abs(frac - 0.5) < 5 * sd)
    # chi-square of the top byte over 256 bins
    h = np.bincount(words >> 24, minlength=256)
    e = words.size / 256
    chi2 = ((h - e) ** 2 / e).sum()
    assert 180 < chi2 < 340   # 255 dof, ~ +-3.5 sigma
