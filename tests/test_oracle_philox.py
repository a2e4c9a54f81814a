"""Pins of the oracle's Philox4x32-10 generator and normal transform.

* The bijection is checked word for word against rocRAND's open-source Philox4x32-10 engine
  (the library routine, compiled for the host from its installed header): with seed = key,
  subsequence = counter words (2, 3) and the engine advanced by counter words (0, 1), its
  next4() is the bijection applied to (counter, key).
* Box-Muller: z0^2 + z1^2 = -2 ln u0 and atan2(z1, z0) = 2 pi u1 (mod 2 pi) exactly up to
  rounding; mean 0, variance 1 and a Kolmogorov-Smirnov test on 10^6 draws.
* The coordinate / particle / level / point layout of the streams.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import philox

ROCRAND_HEADER = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"

_HOST_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    /* discard() counts numbers (four per counter step) in 64 bits, so counter word 1 is
       advanced in steps of 2^29 for its top two bits */
    unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)(c1 & 0x3FFFFFFFu) << 32));
    rocrand_device::philox4x32_10_engine e(seed, subseq, off);
    for (unsigned i = 0; i < 2u * (c1 >> 30); ++i) e.discard(1ull << 63);
    uint4 r = e.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_host(tmp_path_factory):
    if not os.path.exists(ROCRAND_HEADER) or shutil.which("g++") is None:
        pytest.skip("rocRAND header or g++ not available")
    d = tmp_path_factory.mktemp("rocrand")
    src = d / "philox_host.cpp"
    src.write_text(_HOST_SRC)
    exe = d / "philox_host"
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", str(src),
                    "-o", str(exe)], check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand_engine(rocrand_host):
    rng = np.random.default_rng(123)
    n = 400
    words = rng.integers(0, 2 ** 32, size=(n, 6), dtype=np.uint64)
    words[:4] = [[0, 0, 0, 0, 0, 0], [2 ** 32 - 1] * 6, [1, 2, 3, 4, 5, 6],
                 [0xFFFFFFFF, 0, 0xFFFFFFFF, 0, 0xFFFFFFFF, 0]]
    text = "\n".join(" ".join(str(int(v)) for v in row) for row in words) + "\n"
    out = subprocess.run([str(rocrand_host)], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(x) for x in line.split()] for line in out.stdout.strip().splitlines()],
                   dtype=np.uint64)
    got = np.stack(philox.philox4x32_10(*[words[:, i] for i in range(6)]), axis=1).astype(np.uint64)
    assert ref.shape == got.shape
    assert np.array_equal(ref, got)


def test_box_muller_identities():
    rng = np.random.default_rng(5)
    w = rng.integers(0, 2 ** 32, size=(20000, 4), dtype=np.uint64).astype(np.uint32)
    w[0] = [0, 0, 0, 0]
    w[1] = [2 ** 32 - 1] * 4
    z = philox.box_muller(w)
    u = philox.uniforms(w)
    assert np.all(u > 0.0) and np.all(u < 1.0)
    np.testing.assert_allclose(z[:, 0] ** 2 + z[:, 1] ** 2, -2.0 * np.log(u[:, 0]), rtol=1e-14, atol=1e-300)
    np.testing.assert_allclose(z[:, 2] ** 2 + z[:, 3] ** 2, -2.0 * np.log(u[:, 2]), rtol=1e-14, atol=1e-300)
    ang = np.mod(np.arctan2(z[:, 1], z[:, 0]), 2 * np.pi)
    ref = np.mod(2 * np.pi * u[:, 1], 2 * np.pi)
    diff = np.abs(ang - ref)
    diff = np.minimum(diff, 2 * np.pi - diff)
    assert diff.max() < 1e-12


def test_normals_statistics():
    z = philox.normals(seed=7, instance=0, stream=3, k=0, M=2500, d=400).ravel()
    assert z.size == 10 ** 6
    assert abs(z.mean()) < 5.0 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # independent coordinates: the four members of one Philox call are uncorrelated
    g = z.reshape(-1, 4)
    c = np.corrcoef(g.T)
    assert np.abs(c - np.eye(4)).max() < 5.0 / np.sqrt(g.shape[0])


def test_stream_layout():
    seed, inst, stream, k, M, d = (0x1234_5678_9ABC_DEF0, 5, 77, 3, 6, 10)
    z = philox.normals(seed, inst, stream, k, M, d)
    k0 = seed & 0xFFFFFFFF
    k1 = (seed >> 32) ^ inst
    for j in range(M):
        for i in range(d):
            wd = philox.philox4x32_10(i // 4, j, k, stream, k0, k1)
            ref = philox.box_muller(np.array([[int(x) for x in wd]], dtype=np.uint32))[0, i % 4]
            assert z[j, i] == ref
    # a different level, particle, point or instance gives different words
    base = philox.raw_words(seed, inst, stream, k, [0], 3)
    for args in [(seed, inst, stream, k + 1), (seed, inst, stream + 1, k), (seed, inst + 1, stream, k)]:
        assert not np.array_equal(philox.raw_words(*args[:2], args[2], args[3], [0], 3), base)
    assert not np.array_equal(philox.raw_words(seed, inst, stream, k, [1], 3), base)
