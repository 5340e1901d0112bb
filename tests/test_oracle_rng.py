"""Pins of the oracle's random numbers (Section 5, RNG discussion: Philox).

The oracle's Philox4x32-10 is checked bit for bit against rocRAND's
independent implementation of the same published generator (host-compiled
from its header); the uniform map is checked against its exact definition
and for uniformity.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long offset = 4ULL * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
    rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
"""


def _rocrand_probe(tmp_path):
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr) or shutil.which("g++") is None:
        pytest.skip("rocRAND header or g++ not available")
    src = tmp_path / "probe.cpp"
    exe = tmp_path / "probe"
    src.write_text(PROBE)
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", str(src),
                    "-o", str(exe)], check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, tmp_path):
    exe = _rocrand_probe(tmp_path)
    rng = np.random.default_rng(1)
    cases = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    # rocRAND's engine takes the counter's words 0-1 as a 64-bit element offset
    # times 4, so word 1 must stay below 2^30 for that offset not to wrap.
    cases[:, 3] >>= 2
    cases[0] = 0
    cases[1] = 2**32 - 1
    cases[1, 3] = 2**30 - 1
    cases[2] = [0x01234567, 0x89ABCDEF, 7, 1, (1 << 24) | 3, 5]
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                   dtype=np.uint64)
    mine = np.array([orc.philox(c[2:6].astype(np.uint32), c[0:2].astype(np.uint32))
                     for c in cases], dtype=np.uint64)
    assert np.array_equal(mine, ref)


def test_words_layout(orc):
    """orc_words puts (index, sweep, tag<<24|round, chain) in the counter and the seed in the key."""
    seed = 0x0000000500000009
    w = orc.words(seed, 17, 3, orc.TAG_Z, 2, 4)
    ref = orc.philox(np.array([17, 3, (orc.TAG_Z << 24) | 2, 4], np.uint32),
                     np.array([9, 5], np.uint32))
    assert np.array_equal(w, ref)


def test_uniform_exact_values(orc):
    assert orc.uniform(0) == 2.0 ** -24
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert orc.uniform(0x80000000) == 0.5 + 2.0 ** -24
    for w in [0, 1, 511, 512, 0x12345678, 0xFFFFFFFF]:
        u = orc.uniform(w)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u  # exactly representable in float32
        assert u == (2 * (w >> 9) + 1) / 2**24


def test_uniform_distribution(orc):
    # 4 words per call; 50k calls -> 200k uniforms
    us = np.array([[orc.uniform(int(v)) for v in orc.words(42, i, 1, orc.TAG_Z, 0, 0)]
                   for i in range(50_000)]).ravel()
    assert abs(us.mean() - 0.5) < 5 * np.sqrt(1 / 12 / us.size)
    counts, _ = np.histogram(us, bins=64, range=(0, 1))
    chi2 = ((counts - us.size / 64) ** 2 / (us.size / 64)).sum()
    assert stats.chi2.sf(chi2, 63) > 1e-4
    # lag-1 correlation across consecutive counters
    r = np.corrcoef(us[:-1], us[1:])[0, 1]
    assert abs(r) < 5 / np.sqrt(us.size)
