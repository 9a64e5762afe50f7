// Colour-split order of the vectors of a 3-D grid level with an even side m.
//
// The red cells ((i + j + l) even) come first, then the black ones; within a
// colour, row (l, j) holds its m/2 cells in order of i.  Cell (i, j, l) sits at
//
//   ((i + j + l) & 1) m^3/2 + (l m + j) m/2 + i/2.
//
// A red-black half-sweep then reads the swept colour's r and the other
// colour's z, and writes the swept colour's z, as contiguous runs, where the
// natural order (x1 fastest) uses every other word of each line it touches.
// The faces stay in the natural order.
//
// Neighbours: the six neighbours of a cell have the other colour.  For
// i = 2h + o in row (l, j), the x1-neighbours i - 1 and i + 1 are at h - 1 + o
// and h + o of the other colour's row (l, j); the x2- and x3-neighbours are at
// h in the rows (l, j -+ 1) and (l -+ 1, j), a row of m/2 and a plane of m^2/2
// entries away.  A neighbour exists under the same conditions as in the
// natural order (0 <= i +- 1 < m, ...).
//
// Plain C++ (host and device), so the CPU tests compile this header as it is.
#pragma once

#if defined(__HIPCC__)
#define MLMC_CS_HD __host__ __device__
#else
#define MLMC_CS_HD
#endif

namespace mlmc {

// Colour-split index of cell (i, j, l) of an m^3 level (m even).
MLMC_CS_HD inline long long cs3_index(int m, int i, int j, int l) {
  const int half = m >> 1;
  return (long long)((i + j + l) & 1) * ((long long)m * m * half) +
         ((long long)l * m + j) * half + (i >> 1);
}

// Cell (i, j, l) at colour-split index e, 0 <= e < m^3 < 2^31.
MLMC_CS_HD inline void cs3_cell(int m, long long e, int& i, int& j, int& l) {
  const unsigned half = (unsigned)m >> 1;
  const unsigned nh = (unsigned)m * (unsigned)m * half;
  const unsigned ue = (unsigned)e;
  const unsigned col = ue >= nh ? 1u : 0u;
  const unsigned rem = ue - col * nh;
  const unsigned row = rem / half;
  const unsigned h = rem - row * half;
  l = (int)(row / (unsigned)m);
  j = (int)(row - (unsigned)l * (unsigned)m);
  i = (int)(2u * h + (((unsigned)(j + l) + col) & 1u));
}

// The other colour's entry at h in the cell's own row, and the offsets from
// it of the six neighbours: east (i + 1), west (i - 1), north (j + 1),
// south (j - 1), up (l + 1), down (l - 1).
struct Cs3Nb {
  long long other;
  int de, dw, dn, ds, du, dd;
};

MLMC_CS_HD inline Cs3Nb cs3_neighbours(int m, int i, int j, int l) {
  const int half = m >> 1;
  Cs3Nb r;
  r.other = (long long)(1 - ((i + j + l) & 1)) * ((long long)m * m * half) +
            ((long long)l * m + j) * half + (i >> 1);
  r.de = i & 1;
  r.dw = (i & 1) - 1;
  r.dn = half;
  r.ds = -half;
  r.du = m * half;
  r.dd = -m * half;
  return r;
}

}  // namespace mlmc
