"""Pins of the oracle's ray directions (section 2.1: uniform points on the sphere).

Philox4x32-10 is checked word for word against rocRAND's independent implementation
(its header is C++ source; compiled here for the host with g++).  The Marsaglia
directions are checked statistically (moments, octant balance) and for unit length.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROCRAND = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"

PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    rocrand_state_philox4x32_10 st;
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    rocrand_init(seed, ((unsigned long long)c3 << 32) | c2,
                 (((unsigned long long)c1 << 32) | c0) * 4ULL, &st);
    unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
}
"""


@pytest.mark.skipif(not (os.path.exists(ROCRAND) and shutil.which("g++")), reason="rocRAND header or g++ missing")
def test_philox_matches_rocrand(orc):
    rng = np.random.default_rng(11)
    cases = rng.integers(0, 2 ** 32, size=(300, 6), dtype=np.uint64)
    # rocRAND takes the counter's low 64 bits as offset/4, so word 1 must stay below 2^30
    cases[:, 1] %= 2 ** 30
    cases[:4] = [[0, 0, 0, 0, 0, 0], [2 ** 32 - 1, 2 ** 30 - 1] + [2 ** 32 - 1] * 4, [1, 2, 3, 4, 5, 6],
                 [0, 0, 0, 255, 7, 0]]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "p.cpp"), os.path.join(d, "p")
        open(src, "w").write(PROG)
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                               src, "-o", exe])
        inp = "\n".join(" ".join(str(int(x)) for x in row) for row in cases) + "\n"
        res = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(x) for x in line.split()] for line in res.strip().splitlines()], np.uint64)
    for row, r in zip(cases, ref):
        got = orc.philox(row[:4].astype(np.uint32), row[4:].astype(np.uint32))
        assert np.array_equal(got.astype(np.uint64), r)


def test_direction_statistics(orc):
    n = 60000
    w = np.empty((n, 3), np.float64)
    calls = np.empty(n, np.int64)
    for i in range(n):
        d, c = orc.direction(0x1234, i % 997, i // 997, 3, 0)
        w[i] = d
        calls[i] = c
    norm = np.linalg.norm(w, axis=1)
    assert np.abs(norm - 1).max() < 4e-7
    sig = np.sqrt(1.0 / 3.0 / n)
    assert (np.abs(w.mean(0)) < 4.5 * sig).all()
    # E[w_i^2] = 1/3, Var[w_i^2] = 1/5 - 1/9
    sig2 = np.sqrt((1 / 5 - 1 / 9) / n)
    assert (np.abs((w ** 2).mean(0) - 1 / 3) < 4.5 * sig2).all()
    # octants equally likely (chi-square, 7 dof; 99.9% quantile 24.3)
    oct_ = (w[:, 0] > 0) + 2 * (w[:, 1] > 0) + 4 * (w[:, 2] > 0)
    cnt = np.bincount(oct_, minlength=8)
    chi2 = ((cnt - n / 8) ** 2 / (n / 8)).sum()
    assert chi2 < 24.3
    # one Philox call suffices with probability 1 - (1 - pi/4)^2
    p1 = 1 - (1 - np.pi / 4) ** 2
    assert abs((calls == 1).mean() - p1) < 4.5 * np.sqrt(p1 * (1 - p1) / n)


def test_direction_depends_on_every_counter_word(orc):
    base, _ = orc.direction(5, 10, 2, 3, 4)
    for args in [(6, 10, 2, 3, 4), (5, 11, 2, 3, 4), (5, 10, 3, 3, 4), (5, 10, 2, 4, 4), (5, 10, 2, 3, 5)]:
        other, _ = orc.direction(*args)
        assert not np.array_equal(base, other)
