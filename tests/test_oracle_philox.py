"""Pins of the oracle's Philox4x32-10 and Box-Muller normals.

* Bitwise agreement with an independent implementation: PyTorch's open-source
  header ATen/core/PhiloxRNGEngine.h, compiled here into a tiny probe (its
  engine(seed, subsequence, offset) maps to key = seed, counter =
  (offset_lo, offset_hi, subsequence_lo, subsequence_hi)).
* Uniform mapping end points; moments and independence of the normals.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import philox

PROBE_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  for (int a = 1; a + 2 < argc; a += 3) {
    unsigned long long seed = strtoull(argv[a], 0, 0);
    unsigned long long sub = strtoull(argv[a + 1], 0, 0);
    unsigned long long off = strtoull(argv[a + 2], 0, 0);
    at::Philox4_32 e(seed, sub, off);
    for (int i = 0; i < 4; i++) printf("%u ", e());
    printf("\n");
  }
  return 0;
}
"""


def _torch_include():
    try:
        import torch
    except Exception:
        return None
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    return inc if os.path.exists(os.path.join(inc, "ATen/core/PhiloxRNGEngine.h")) else None


@pytest.fixture(scope="module")
def torch_probe(tmp_path_factory):
    inc = _torch_include()
    gxx = shutil.which("g++")
    if inc is None or gxx is None:
        pytest.skip("torch headers or g++ not available")
    d = tmp_path_factory.mktemp("philox_probe")
    src = d / "probe.cpp"
    src.write_text(PROBE_SRC)
    exe = d / "probe"
    subprocess.check_call([gxx, "-O1", "-std=c++17", "-I", inc, str(src), "-o", str(exe)])
    return str(exe)


def test_philox_matches_torch_header(torch_probe):
    rng = np.random.default_rng(123)
    cases = []
    for _ in range(64):
        c = rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)
        k = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)
        cases.append((c, k))
    cases.append((np.zeros(4, np.uint64), np.zeros(2, np.uint64)))
    cases.append((np.full(4, 2 ** 32 - 1, np.uint64), np.full(2, 2 ** 32 - 1, np.uint64)))
    args = []
    for c, k in cases:
        seed = int(k[0]) | (int(k[1]) << 32)
        sub = int(c[2]) | (int(c[3]) << 32)
        off = int(c[0]) | (int(c[1]) << 32)
        args += [str(seed), str(sub), str(off)]
    out = subprocess.check_output([torch_probe] + args).decode().split("\n")
    for (c, k), line in zip(cases, out):
        ref = [int(v) for v in line.split()]
        got = philox.philox4x32_10(c[0], c[1], c[2], c[3], k[0], k[1])
        assert [int(v) for v in got] == ref


def test_philox_vectorised_equals_scalar():
    ids = np.arange(100)
    vec = philox.blocks(0x1234_5678_9ABC, 7, 3, 2, ids)
    for b in (0, 1, 57, 99):
        one = philox.blocks(0x1234_5678_9ABC, 7, 3, 2, [b])[0]
        assert np.array_equal(vec[b], one)


def test_uniform_end_points():
    u = philox.to_uniform(np.array([0, 2 ** 32 - 1], dtype=np.uint32))
    assert u[0] == 2.0 ** -33
    assert u[1] == 1.0 - 2.0 ** -33
    assert 0.0 < u[0] < u[1] < 1.0


def test_normal_moments_and_independence():
    blk = philox.blocks(0, 0, 0, 5, np.arange(250_000))
    z = philox.normals_of_block(blk).reshape(-1)
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    kurt = np.mean(z ** 4) / np.mean(z ** 2) ** 2
    assert abs(kurt - 3.0) < 5 * np.sqrt(24.0 / n)
    zz = philox.normals_of_block(blk)
    for a, b in ((0, 1), (0, 2), (1, 3), (2, 3)):
        corr = np.corrcoef(zz[:, a], zz[:, b])[0, 1]
        assert abs(corr) < 5 / np.sqrt(zz.shape[0])


def test_box_muller_special_values():
    # u0 = e^-1/2 gives radius 1; u1 = 1/4 points along the second axis.
    z0, z1 = philox.box_muller(np.array([np.exp(-0.5)]), np.array([0.25]))
    assert abs(z0[0]) < 1e-15 and abs(z1[0] - 1.0) < 1e-15
