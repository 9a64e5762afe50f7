"""The colour-split order of 3-D level vectors (csrc/cs3.hpp), compiled for
the CPU from the same header: on every even side the kernels use (2 to 20 and
a 64 sample of cells), the index is a bijection onto [0, m^3) that puts the
red cells ((i + j + l) even) first, row by row in order of i; cs3_cell
inverts it; and every neighbour that exists in the natural order is found at
the offset cs3_neighbours gives, inside the other colour's block.
"""
import ctypes
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HDR = os.path.join(os.path.dirname(HERE), "paper_1506_04694_amd", "csrc", "cs3.hpp")

SRC = r'''
#include "%s"
extern "C" long long cs_index(int m, int i, int j, int l) { return mlmc::cs3_index(m, i, j, l); }
extern "C" void cs_cell(int m, long long e, int* ijl) {
  mlmc::cs3_cell(m, e, ijl[0], ijl[1], ijl[2]);
}
extern "C" void cs_nb(int m, int i, int j, int l, long long* out) {
  const mlmc::Cs3Nb nb = mlmc::cs3_neighbours(m, i, j, l);
  out[0] = nb.other;
  out[1] = nb.de; out[2] = nb.dw; out[3] = nb.dn; out[4] = nb.ds; out[5] = nb.du; out[6] = nb.dd;
}
'''


@pytest.fixture(scope="module")
def cs(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    d = tmp_path_factory.mktemp("cs3")
    src, lib = d / "cs.cpp", d / "libcs.so"
    src.write_text(SRC % HDR)
    subprocess.run([gxx, "-O1", "-shared", "-fPIC", "-o", str(lib), str(src)], check=True)
    so = ctypes.CDLL(str(lib))
    so.cs_index.restype = ctypes.c_longlong
    so.cs_index.argtypes = [ctypes.c_int] * 4
    so.cs_cell.argtypes = [ctypes.c_int, ctypes.c_longlong, ctypes.POINTER(ctypes.c_int)]
    so.cs_nb.argtypes = [ctypes.c_int] * 4 + [ctypes.POINTER(ctypes.c_longlong)]
    return so


def _expected_order(m):
    """Cells in the colour-split order, from its definition."""
    order = []
    for col in (0, 1):
        for l in range(m):
            for j in range(m):
                for i in range(m):
                    if (i + j + l) % 2 == col:
                        order.append((i, j, l))
    return order


def _cells(m, rng):
    if m <= 20:
        return list(itertools.product(range(m), repeat=3))
    edge = [0, 1, m - 2, m - 1]
    cells = list(itertools.product(edge, repeat=3))
    cells += [tuple(int(v) for v in rng.integers(0, m, 3)) for _ in range(3000)]
    return cells


@pytest.mark.parametrize("m", [2, 4, 6, 8, 10, 12, 16, 20])
def test_index_is_the_defined_order(cs, m):
    for e, (i, j, l) in enumerate(_expected_order(m)):
        assert cs.cs_index(m, i, j, l) == e


@pytest.mark.parametrize("m", [2, 4, 8, 12, 20, 64])
def test_cell_inverts_index(cs, m):
    rng = np.random.default_rng(m)
    buf = (ctypes.c_int * 3)()
    seen = set()
    for (i, j, l) in _cells(m, rng):
        e = cs.cs_index(m, i, j, l)
        assert 0 <= e < m ** 3
        cs.cs_cell(m, e, buf)
        assert tuple(buf) == (i, j, l)
        seen.add(e)
    if m <= 20:
        assert len(seen) == m ** 3


@pytest.mark.parametrize("m", [2, 4, 6, 8, 16, 64])
def test_neighbour_offsets(cs, m):
    rng = np.random.default_rng(100 + m)
    out = (ctypes.c_longlong * 7)()
    half = m ** 3 // 2
    for (i, j, l) in _cells(m, rng):
        cs.cs_nb(m, i, j, l, out)
        other = out[0]
        col = (i + j + l) % 2
        assert (1 - col) * half <= other < (2 - col) * half
        steps = [((1, 0, 0), out[1]), ((-1, 0, 0), out[2]), ((0, 1, 0), out[3]),
                 ((0, -1, 0), out[4]), ((0, 0, 1), out[5]), ((0, 0, -1), out[6])]
        for (di, dj, dl), off in steps:
            ii, jj, ll = i + di, j + dj, l + dl
            if 0 <= ii < m and 0 <= jj < m and 0 <= ll < m:
                assert other + off == cs.cs_index(m, ii, jj, ll), ((i, j, l), (di, dj, dl))
