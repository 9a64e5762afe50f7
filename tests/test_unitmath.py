"""Accuracy of the device's short logarithm and sine/cosine of pi x (the
Box-Muller steps of the noise, csrc/unitmath.hpp), compiled for the CPU from
the same header and compared with 60-digit references (mpmath) on the
arguments the sampler produces: u = (k + 1/2) 2^-32 and x = 2 u, random k and
the extreme and branch-boundary ones.  Bound: 4 units in the last place for
log u and for sin/cos of pi x (the references' own rounding included); the
normals they make differ from exact ones by about 1e-15 relative, far inside
the sampler's 1e-11 parity in log k.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

HERE = os.path.dirname(os.path.abspath(__file__))
HDR = os.path.join(os.path.dirname(HERE), "paper_1506_04694_amd", "csrc", "unitmath.hpp")

SRC = r'''
#include "%s"
extern "C" double um_log(double u) { return mlmc::log_unit(u); }
extern "C" void um_sincospi(double x, double* s, double* c) { mlmc::sincospi_unit(x, s, c); }
'''


def _has_fma():
    try:
        with open("/proc/cpuinfo") as f:
            return " fma " in f.read().replace("\n", " ")
    except OSError:
        return False


# the device contracts a * b + c into fused multiply-adds; both roundings are
# checked (fused only where the host has FMA instructions)
MODES = ["-ffp-contract=off"] + (["-ffp-contract=fast -mfma"] if _has_fma() else [])


@pytest.fixture(scope="module", params=MODES)
def um(request, tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    d = tmp_path_factory.mktemp("unitmath")
    src, lib = d / "um.cpp", d / "libum.so"
    src.write_text(SRC % HDR)
    subprocess.run([gxx, "-O2"] + request.param.split() + ["-shared", "-fPIC", "-o", str(lib),
                                                           str(src)], check=True)
    so = ctypes.CDLL(str(lib))
    so.um_log.restype = ctypes.c_double
    so.um_log.argtypes = [ctypes.c_double]
    so.um_sincospi.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double)]
    return so


def _arguments():
    rng = np.random.default_rng(11)
    k = list(rng.integers(0, 2 ** 32, size=4000))
    k += [0, 1, 2, 3, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 1, 2 ** 32 - 2]
    # log's branch at m = sqrt(1/2) and sincospi's quadrant edges (2x near an integer)
    for e in range(0, 32):
        c = int(round(2 ** 32 * 2 ** -e * 0.7071067811865476))
        k += [c - 1, c, c + 1]
    for q in range(0, 5):
        c = int(round(q * 2 ** 30))
        k += [c - 1, c, c + 1] if 0 < c < 2 ** 32 else []
    k = [int(v) for v in k if 0 <= v < 2 ** 32]
    return [(v + 0.5) * 2.0 ** -32 for v in k]


def _ulps(got, ref):
    r = float(ref)
    if r == 0.0:
        return abs(got) / np.spacing(np.float64(0.0))
    return abs(got - r) / np.spacing(np.float64(abs(r)))


def test_log_unit_is_within_four_ulps(um):
    mp.mp.dps = 60
    worst = 0.0
    for u in _arguments():
        ref = mp.log(mp.mpf(u))
        worst = max(worst, _ulps(um.um_log(u), ref))
    assert worst <= 4.0, worst


def test_sincospi_unit_is_within_four_ulps(um):
    mp.mp.dps = 60
    s, c = ctypes.c_double(), ctypes.c_double()
    worst_s = worst_c = 0.0
    for u in _arguments():
        x = 2.0 * u                      # exact
        um.um_sincospi(x, ctypes.byref(s), ctypes.byref(c))
        rs, rc = mp.sinpi(mp.mpf(x)), mp.cospi(mp.mpf(x))
        # far from zeros the relative ulps; near a zero (|value| < 1e-3) the
        # absolute error against the ulp of 1
        ws = _ulps(s.value, rs) if abs(rs) > 1e-3 else abs(s.value - float(rs)) / 2.0 ** -52
        wc = _ulps(c.value, rc) if abs(rc) > 1e-3 else abs(c.value - float(rc)) / 2.0 ** -52
        worst_s, worst_c = max(worst_s, ws), max(worst_c, wc)
    assert worst_s <= 4.0 and worst_c <= 4.0, (worst_s, worst_c)


def test_box_muller_pairs_match_the_definition(um):
    """z0 = sqrt(-2 log u0) cos(2 pi u1), z1 = ... sin(2 pi u1) to 1e-15
    relative of the pair's radius."""
    mp.mp.dps = 40
    s, c = ctypes.c_double(), ctypes.c_double()
    args = _arguments()
    for u0, u1 in zip(args[::2], args[1::2]):
        r = np.sqrt(-2.0 * um.um_log(u0))
        um.um_sincospi(2.0 * u1, ctypes.byref(s), ctypes.byref(c))
        rr = mp.sqrt(-2 * mp.log(mp.mpf(u0)))
        z0 = rr * mp.cospi(2 * mp.mpf(u1))
        z1 = rr * mp.sinpi(2 * mp.mpf(u1))
        assert abs(r * c.value - float(z0)) <= 1e-15 * float(rr)
        assert abs(r * s.value - float(z1)) <= 1e-15 * float(rr)
