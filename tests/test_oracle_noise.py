"""Pins of the oracle's noise stream (Philox4x32-10 + Box-Muller).

The noise of Eq. (8)-(9) is N(0, 2 eps) per parameter.  The oracle draws it
from Philox4x32-10 (Salmon et al., SC'11).  Pins:
  * raw 128-bit blocks equal the generator's published known-answer vectors
    (tests/golden/philox4x32_10_kat.txt) and agree bit for bit with an
    independent implementation, rocRAND's Philox4x32-10 engine, run as a
    black box on the host;
  * the uniforms are in (0, 1) and the normals pass mean / variance /
    Kolmogorov-Smirnov tests against N(0, 1), with adjacent counters
    uncorrelated.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import oracle
from parity import philox_kat

ROCRAND_PROBE = r"""
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
// Reads lines "c0 c1 c2 c3 k0 k1" and prints the Philox4x32-10 block.
// rocRAND seeds key = seed, counter words 2,3 = subsequence, words 0,1 =
// offset / 4; next4() at substate 0 returns the block of that counter.
int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
"""


def _cases(n=64, seed=5):
    rng = np.random.default_rng(seed)
    # rocRAND takes counter words 0-1 as a 64-bit offset times 4, so word 1
    # stays below 2^30 here (the sampler's word 1 is a row/column index).
    top = np.array([0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF],
                   dtype=np.uint32)
    cases = [np.zeros(6, dtype=np.uint32), top]
    for _ in range(n):
        c = rng.integers(0, 2**32, 6, dtype=np.uint64).astype(np.uint32)
        c[1] &= 0x3FFFFFFF
        cases.append(c)
    # counters of the form the sampler uses: (quad, index, t, stream)
    cases += [np.array([q, idx, t, s, 1234, 0], dtype=np.uint32)
              for q, idx, t, s in [(0, 0, 0, 0), (12, 69999, 999, 1), (3, 5, 7, 0)]]
    return cases


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_engine():
    cases = _cases()
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.cpp")
        exe = os.path.join(d, "probe")
        open(src, "w").write(ROCRAND_PROBE)
        subprocess.run(["hipcc", "-O1", "-x", "hip", "--offload-arch=gfx950", src, "-o", exe],
                       check=True, capture_output=True)
        inp = "\n".join(" ".join(str(int(x)) for x in c) for c in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    got = np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()],
                   dtype=np.uint64)
    for c, g in zip(cases, got):
        mine = oracle.philox4x32_10(c[:4], c[4:])
        assert np.array_equal(mine.astype(np.uint64), g), (c, mine, g)


def test_philox_known_answer_vectors():
    inp, expect = philox_kat()
    for c, e in zip(inp, expect):
        assert np.array_equal(oracle.philox4x32_10(c[:4], c[4:]), e), (c, e)


def test_normals_are_standard_gaussian():
    K = 64
    z = np.concatenate([oracle.normals(77, t, s, idx, K)[0]
                        for t in range(4) for s in (0, 1) for idx in range(400)])
    assert len(z) == 4 * 2 * 400 * K
    assert abs(z.mean()) < 5 / np.sqrt(len(z))
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / len(z))
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # Box-Muller radius bounds |z| and the tail is cut at sqrt(48 ln 2)
    zz, rr = oracle.normals(3, 1, 0, 11, 4096)
    assert np.all(np.abs(zz) <= rr + 1e-15)
    assert rr.max() <= np.sqrt(48 * np.log(2)) + 1e-12


def test_adjacent_counters_uncorrelated():
    K = 256
    a = np.stack([oracle.normals(9, 0, 0, i, K)[0] for i in range(300)])
    b = np.stack([oracle.normals(9, 1, 0, i, K)[0] for i in range(300)])      # next t
    c = np.stack([oracle.normals(9, 0, 1, i, K)[0] for i in range(300)])      # other stream
    n = a.size
    for x, y in [(a, b), (a, c), (a[:-1], a[1:]), (a[:, :-1], a[:, 1:])]:
        r = np.corrcoef(x.ravel(), y.ravel())[0, 1]
        assert abs(r) < 5 / np.sqrt(n)


def test_uniform_map_open_interval_and_box_muller_form():
    # Philox words -> u = (2 (r >> 9) + 1) / 2^24 in (0, 1); z from (u0,u1),(u2,u3).
    seed, t, stream, idx = 42, 3, 1, 17
    r = oracle.philox4x32_10([0, idx, t, stream], [seed & 0xFFFFFFFF, seed >> 32])
    u = (2.0 * (r.astype(np.float64) // 512) + 1.0) / 2**24
    assert np.all((u > 0) & (u < 1))
    rad = np.sqrt(-2 * np.log(u[[0, 2]]))
    expect = np.array([rad[0] * np.cos(2 * np.pi * u[1]), rad[0] * np.sin(2 * np.pi * u[1]),
                       rad[1] * np.cos(2 * np.pi * u[3]), rad[1] * np.sin(2 * np.pi * u[3])])
    z, _ = oracle.normals(seed, t, stream, idx, 4)
    np.testing.assert_allclose(z, expect, rtol=1e-14, atol=1e-14)
