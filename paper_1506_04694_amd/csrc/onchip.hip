// Whole multigrid-preconditioned CG solve of one 64 x 64 sample in one
// workgroup (Section 3.5 with the cycle of the tiled kernels): the sample's
// vectors, operator and grid hierarchy live in LDS and registers, so a solve
// reads T, tb and b and writes p once, instead of streaming every vector
// through HBM in each of its ~9 iterations.  This is the form for the grids
// whose whole state fits on one CU (the 64^2 level and the 64^2 companions of
// the 128^2 level); larger grids use the tiled kernels.
//
// Layout: the smoothing levels 64^2, 32^2, 16^2 and 8^2 keep z in LDS split by
// colour.  A "pair" is the red and the black cell of columns 2c and 2c + 1 of
// row j (red at i = 2c + (j & 1)); both sit at split index c of their colour's
// plane, a (m + 2) x (m / 2 + 2) array with a zero frame.  A half-sweep of one
// colour reads only the other plane, at contiguous split indices across the
// lanes, and every lane of a working wave has a cell of the swept colour.
// Thread t owns pairs t + 1024 s.  On 64^2 the east and north faces sit in
// colour-split planes too (a cell's west / south face is its neighbour's east /
// north face, read at the neighbour's position; the frame holds the boundary
// faces), and the reciprocal diagonal, r, x and p in registers; 32^2 keeps its
// cells in registers (threads < 512), 16^2 and 8^2 in LDS; the coarsest 4^2
// grid is solved with its precomputed inverse (staged in LDS).
//
// Arithmetic follows the tiled path step for step (same sweeps, residuals,
// restriction, prolongation with over-correction omega, W on the levels with
// two visits, V-cycle restart after a breakdown); only the summation order of
// the dot products differs, so results agree with it to rounding.
#include <cfloat>

#include "common.hpp"
#include "kernels.hpp"

namespace mlmc {
namespace {

constexpr int kOcT = 1024;  // threads per workgroup
constexpr int kOcLevels = 4;  // smoothing levels 64, 32, 16, 8; then the 4^2 inverse

__host__ __device__ constexpr int oc_m(int L) { return 64 >> L; }
__host__ __device__ constexpr int oc_w(int L) { return oc_m(L) / 2; }  // pairs per row
__host__ __device__ constexpr int oc_P(int L) { return oc_w(L) + 2; }  // padded plane pitch
__host__ __device__ constexpr int oc_plane(int L) { return (oc_m(L) + 2) * oc_P(L); }
__host__ __device__ constexpr int oc_zoff(int L) {
  return L == 0 ? 0 : oc_zoff(L - 1) + 2 * oc_plane(L - 1);
}
// LDS map (doubles)
constexpr int kOcFace = oc_zoff(kOcLevels);      // 64^2 east faces (red, black), north faces (red, black)
constexpr int kOcSres = kOcFace + 4 * oc_plane(0);  // red residuals of the level being restricted
constexpr int kOcCell = kOcSres + 64 * 32;       // levels 2, 3: six arrays of m^2 each
__host__ __device__ constexpr int oc_celloff(int L) { return kOcCell + (L == 2 ? 0 : 6 * 256); }
constexpr int kOcVec = kOcCell + 6 * (256 + 64);  // coarsest right-hand side
constexpr int kOcZ4 = kOcVec + 16;                 // coarsest solution
constexpr int kOcAinv = kOcZ4 + 16;                // coarsest inverse
constexpr int kOcRed = kOcAinv + 256;              // wave partials of a dot product
constexpr int kOcWords = kOcRed + kOcT / kWave;

struct OcCell {
  double te, tw, tn, ts, di, r;
};

__device__ __forceinline__ int oc_zi(int P, int j, int c) { return (j + 1) * P + (c + 1); }

// Element i of a per-sample array with a workgroup-uniform base: the byte
// offset is an unsigned 32-bit value, so the load takes its base from scalar
// registers and a single offset VGPR.
__device__ __forceinline__ double oc_ld(const double* p, unsigned i) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(p) + (size_t)(i * 8u));
}

// faces of cell (i, j) of an m x m level with operator Ts / tbs (global)
__device__ __forceinline__ void oc_load(OcCell& c, const double* __restrict__ Ts,
                                        const double* __restrict__ tbs, int m, int i, int j) {
  const unsigned n = m * m, q = j * m + i;
  c.te = oc_ld(Ts, q);
  c.tn = oc_ld(Ts, n + q);
  c.tw = i > 0 ? oc_ld(Ts, q - 1) : oc_ld(tbs, j);
  c.ts = j > 0 ? oc_ld(Ts, n + q - m) : oc_ld(tbs, m + i);
  c.di = 1.0 / (c.te + c.tw + c.tn + c.ts);
  c.r = 0.0;
}

// Neighbour sum of the cell of colour `col` of pair (j, c): reads the other
// colour's plane `o` (pitch P).
__device__ __forceinline__ double oc_nsum(const OcCell& c, const double* o, int P, int j, int cp,
                                          int col) {
  const int sh = col == 0 ? (j & 1) : 1 - (j & 1);
  const int row = (j + 1) * P + 1;
  return c.te * o[row + cp + sh] + c.tw * o[row + cp - 1 + sh] + c.tn * o[row + P + cp] +
         c.ts * o[row - P + cp];
}

// Register-held cell data: level 0 keeps the reciprocal diagonal and r of its
// four cells ([pair slot][colour]), level 1 whole cells (threads < 512).
struct OcRegs {
  double di0[2][2], r0[2][2];
  OcCell c1[2];
};

template <int L, int COL>
__device__ __forceinline__ OcCell oc_cell(const OcRegs& g, const double* lds, int s, int j,
                                          int cp) {
  if constexpr (L == 0) {
    constexpr int P = oc_P(0), pl = oc_plane(0);
    const double* te = lds + kOcFace;
    const double* tn = te + 2 * pl;
    const int sh = COL == 0 ? (j & 1) : 1 - (j & 1);
    const int f = oc_zi(P, j, cp);
    return OcCell{te[COL * pl + f], te[(1 - COL) * pl + f - 1 + sh], tn[COL * pl + f],
                  tn[(1 - COL) * pl + f - P], g.di0[s][COL], g.r0[s][COL]};
  } else if constexpr (L == 1) {
    return g.c1[COL];
  } else {
    constexpr int m = oc_m(L), n = m * m;
    const int i = 2 * cp + (COL == 0 ? (j & 1) : 1 - (j & 1));
    const double* a = lds + oc_celloff(L);
    const int q = j * m + i;
    return OcCell{a[q], a[n + q], a[2 * n + q], a[3 * n + q], a[4 * n + q], a[5 * n + q]};
  }
}

template <int L>
__device__ __forceinline__ constexpr int oc_slots() {
  return (oc_m(L) * oc_w(L) + kOcT - 1) / kOcT;
}

__host__ __device__ constexpr int oc_log2(int v) { return v <= 1 ? 0 : 1 + oc_log2(v / 2); }

// The thread index as a value the compiler cannot see through.  Every phase
// starts from it, so the LDS addresses a phase derives from it live only in
// that phase: otherwise common-subexpression elimination keeps hundreds of
// them alive across the whole unrolled cycle and the kernel spills.
__device__ __forceinline__ int oc_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Pair pr of level L: row j and split index cp (w is a power of two).
template <int L>
__device__ __forceinline__ void oc_pair(int pr, int& j, int& cp) {
  j = (int)((unsigned)pr >> oc_log2(oc_w(L)));
  cp = (int)((unsigned)pr & (unsigned)(oc_w(L) - 1));
}

// Whether slot s of thread t holds a pair of level L (always, when the pairs
// fill every slot).
template <int L>
__device__ __forceinline__ bool oc_has(int pr) {
  constexpr int npairs = oc_m(L) * oc_w(L);
  if constexpr (npairs % kOcT == 0) return true;
  return pr < npairs;
}

// One colour (COL: 0 red, 1 black) of a Gauss-Seidel sweep on level L (ZERO:
// from z = 0).  Colours are compile-time so that register-held cell data are
// selected statically.
template <int L, int COL, bool ZERO>
__device__ __forceinline__ void oc_smooth(const OcRegs& g, double* lds, int) {
  const int t = oc_tid();
  constexpr int P = oc_P(L);
  double* own = lds + oc_zoff(L) + COL * oc_plane(L);
  const double* oth = lds + oc_zoff(L) + (1 - COL) * oc_plane(L);
#pragma unroll
  for (int s = 0; s < oc_slots<L>(); ++s) {
    const int pr = t + s * kOcT;
    if (oc_has<L>(pr)) {
      int j, cp;
      oc_pair<L>(pr, j, cp);
      const OcCell c = oc_cell<L, COL>(g, lds, s, j, cp);
      own[oc_zi(P, j, cp)] = ZERO ? c.r * c.di : (c.r + oc_nsum(c, oth, P, j, cp, COL)) * c.di;
    }
  }
  __syncthreads();
}

// Red-cell residuals of level L into sres[j * w + c] (black residuals vanish
// after a black sweep).  first: the zero-guess pre-smoothing just ran, whose
// red values are r / D, so the residual is the neighbour sum.
template <int L>
__device__ __forceinline__ void oc_residual(const OcRegs& g, double* lds, int, bool first) {
  const int t = oc_tid();
  constexpr int P = oc_P(L);
  const double* red = lds + oc_zoff(L);
  const double* blk = red + oc_plane(L);
  double* sres = lds + kOcSres;
#pragma unroll
  for (int s = 0; s < oc_slots<L>(); ++s) {
    const int pr = t + s * kOcT;
    if (oc_has<L>(pr)) {
      int j, cp;
      oc_pair<L>(pr, j, cp);
      const OcCell c = oc_cell<L, 0>(g, lds, s, j, cp);
      const double nb = oc_nsum(c, blk, P, j, cp, 0);
      sres[pr] = first ? nb : c.r - (c.te + c.tw + c.tn + c.ts) * red[oc_zi(P, j, cp)] + nb;
    }
  }
  __syncthreads();
}

// Right-hand side of level L + 1: coarse cell (I, J) gathers the red residuals
// of fine cells (2I, 2J) and (2I + 1, 2J + 1), both at split index I.
template <int L>
__device__ __forceinline__ double oc_gather(const double* lds, int I, int J) {
  constexpr int w = oc_w(L);
  const double* sres = lds + kOcSres;
  return sres[(2 * J) * w + I] + sres[(2 * J + 1) * w + I];
}

template <int L>
__device__ __forceinline__ void oc_restrict(OcRegs& g, double* lds, int) {
  const int t = oc_tid();
  constexpr int Lc = L + 1, mc = oc_m(Lc);
  if constexpr (Lc == kOcLevels) {
    if (t < mc * mc) {
      const int J = t / mc, I = t - J * mc;
      lds[kOcVec + t] = oc_gather<L>(lds, I, J);
    }
  } else {
    constexpr int wc = oc_w(Lc), npairs = mc * wc;
    if (t < npairs) {  // one pair per thread on levels >= 1
      int J, cp;
      oc_pair<Lc>(t, J, cp);
#pragma unroll
      for (int col = 0; col < 2; ++col) {
        const int I = 2 * cp + (col == 0 ? (J & 1) : 1 - (J & 1));
        const double v = oc_gather<L>(lds, I, J);
        if constexpr (Lc == 1) {
          g.c1[col].r = v;
        } else {
          lds[oc_celloff(Lc) + 5 * mc * mc + J * mc + I] = v;
        }
      }
    }
  }
  __syncthreads();
}

// z_L += omega P z_{L+1} (piecewise constant prolongation) on every cell.
template <int L>
__device__ __forceinline__ void oc_prolong(double* lds, int, double omega) {
  const int t = oc_tid();
  constexpr int P = oc_P(L);
  double* red = lds + oc_zoff(L);
  double* blk = red + oc_plane(L);
#pragma unroll
  for (int s = 0; s < oc_slots<L>(); ++s) {
    const int pr = t + s * kOcT;
    if (oc_has<L>(pr)) {
      int j, cp;
      oc_pair<L>(pr, j, cp);
      const int J = j >> 1, I = cp;  // both cells of the pair lie in coarse cell (cp, j / 2)
      double e;
      if constexpr (L + 1 == kOcLevels) {
        e = lds[kOcZ4 + J * oc_m(L + 1) + I];
      } else {
        constexpr int Pc = oc_P(L + 1);
        const int colc = (I + J) & 1;
        e = lds[oc_zoff(L + 1) + colc * oc_plane(L + 1) + oc_zi(Pc, J, I >> 1)];
      }
      const int f = oc_zi(P, j, cp);
      red[f] += omega * e;
      blk[f] += omega * e;
    }
  }
  __syncthreads();
}

// gamma-cycle on level L from a zero guess: z_L ~ A_L^{-1} r_L.  WMASK bit L:
// level L takes two coarse visits (compile-time, so every loop unrolls).
template <int L, unsigned WMASK>
__device__ __forceinline__ void oc_cycle(OcRegs& g, double* lds, int t, double omega) {
  if constexpr (L == kOcLevels) {
    if (t < 16) {
      const double* A = lds + kOcAinv;
      const double* v = lds + kOcVec;
      double acc = 0.0;
      for (int q = 0; q < 16; ++q) acc += A[t * 16 + q] * v[q];
      lds[kOcZ4 + t] = acc;
    }
    __syncthreads();
  } else {
    constexpr int nv = (WMASK >> L) & 1u ? 2 : 1;
    oc_smooth<L, 0, true>(g, lds, t);
    oc_smooth<L, 1, false>(g, lds, t);
#pragma unroll
    for (int v = 0; v < nv; ++v) {
      oc_residual<L>(g, lds, t, L == 0 && v == 0);
      oc_restrict<L>(g, lds, t);
      oc_cycle<L + 1, WMASK>(g, lds, t, omega);
      oc_prolong<L>(lds, t, omega);
      oc_smooth<L, 1, false>(g, lds, t);
      oc_smooth<L, 0, false>(g, lds, t);
      if (v + 1 < nv) oc_smooth<L, 1, false>(g, lds, t);
    }
  }
}

// Writes a level-0 vector held by the threads (two pairs each) into the planes.
__device__ __forceinline__ void oc_write0(const double (&v)[2][2], double* lds, int) {
  const int t = oc_tid();
  constexpr int w = oc_w(0), P = oc_P(0);
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int pr = t + sl * kOcT;
    int j, cp;
    oc_pair<0>(pr, j, cp);
    lds[oc_zi(P, j, cp)] = v[sl][0];
    lds[oc_plane(0) + oc_zi(P, j, cp)] = v[sl][1];
  }
  __syncthreads();
}

// q = A v on this thread's level-0 cells (v already written to the planes).
__device__ __forceinline__ void oc_apply0(const OcRegs& g, const double (&v)[2][2],
                                          double (&q)[2][2], const double* lds, int) {
  const int t = oc_tid();
  constexpr int w = oc_w(0), P = oc_P(0);
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int pr = t + sl * kOcT;
    int j, cp;
    oc_pair<0>(pr, j, cp);
    {
      const OcCell c = oc_cell<0, 0>(g, lds, sl, j, cp);
      q[sl][0] = (c.te + c.tw + c.tn + c.ts) * v[sl][0] -
                 oc_nsum(c, lds + oc_plane(0), P, j, cp, 0);
    }
    {
      const OcCell c = oc_cell<0, 1>(g, lds, sl, j, cp);
      q[sl][1] = (c.te + c.tw + c.tn + c.ts) * v[sl][1] - oc_nsum(c, lds, P, j, cp, 1);
    }
  }
}

// Fixed-order dot product over the workgroup; every thread returns the sum.
__device__ __forceinline__ double oc_dot(double v, double* lds, int t) {
  v = wave_sum(v);
  double* red = lds + kOcRed;
  if ((t & (kWave - 1)) == 0) red[t / kWave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kOcT / kWave; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Set-up of one sample's hierarchy in LDS and registers: the 64^2 faces into
// their planes (boundary faces into the frames), the reciprocal diagonals and
// the right-hand side rhs (64^2, [j][i]) into registers, 32^2 cells into
// registers, 16^2 and 8^2 cells into LDS, the 4^2 inverse into LDS.
__device__ __forceinline__ void oc_setup(OcRegs& g, double* lds, const OcHierarchy& h,
                                         const double* __restrict__ rhs,
                                         const double* __restrict__ Ainv, int s, int t) {
  constexpr int m = 64, n = m * m;
  for (int q = t; q < kOcSres; q += kOcT) lds[q] = 0.0;  // zero frames of every plane
  __syncthreads();
  {
    const double* Ts = h.T[0] + (long long)s * 2 * n;
    const double* tbs = h.tb[0] + (long long)s * 2 * m;
    constexpr int P = oc_P(0), pl = oc_plane(0);
    double* te = lds + kOcFace;
    double* tn = te + 2 * pl;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int pr = t + sl * kOcT;
      int j, cp;
      oc_pair<0>(pr, j, cp);
#pragma unroll
      for (int col = 0; col < 2; ++col) {
        const int i = 2 * cp + (col == 0 ? (j & 1) : 1 - (j & 1));
        OcCell c;
        oc_load(c, Ts, tbs, m, i, j);
        const int f = oc_zi(P, j, cp);
        te[col * pl + f] = c.te;
        tn[col * pl + f] = c.tn;
        // boundary faces go to the frame position a neighbour would occupy
        if (i == 0) te[(1 - col) * pl + f - 1] = c.tw;
        if (j == 0) tn[(1 - col) * pl + f - P] = c.ts;
        g.di0[sl][col] = c.di;
        g.r0[sl][col] = oc_ld(rhs, j * m + i);
      }
    }
  }
  if (t < 512) {
    constexpr int m1 = 32;
    const double* Ts = h.T[1] + (long long)s * 2 * m1 * m1;
    const double* tbs = h.tb[1] + (long long)s * 2 * m1;
    const int j = t / 16, cp = t - j * 16;
    oc_load(g.c1[0], Ts, tbs, m1, 2 * cp + (j & 1), j);
    oc_load(g.c1[1], Ts, tbs, m1, 2 * cp + 1 - (j & 1), j);
  }
#pragma unroll
  for (int L = 2; L < kOcLevels; ++L) {
    const int ml = 64 >> L, nl = ml * ml;
    const double* Ts = h.T[L] + (long long)s * 2 * nl;
    const double* tbs = h.tb[L] + (long long)s * 2 * ml;
    double* a = lds + kOcCell + (L == 2 ? 0 : 6 * 256);
    if (t < nl) {
      OcCell c;
      oc_load(c, Ts, tbs, ml, t % ml, t / ml);
      a[t] = c.te;
      a[nl + t] = c.tw;
      a[2 * nl + t] = c.tn;
      a[3 * nl + t] = c.ts;
      a[4 * nl + t] = c.di;
      a[5 * nl + t] = 0.0;
    }
  }
  if (t < 256) lds[kOcAinv + t] = oc_ld(Ainv + (long long)s * 256, t);
  __syncthreads();
}

}  // namespace

// One workgroup per sample.  h: operators of the levels 64, 32, 16, 8, 4
// (Galerkin); Ainv: inverse of each sample's 4^2 operator; b, x: [batch][64^2].
template <unsigned WMASK>
__global__ void __launch_bounds__(kOcT)
k_pcg_onchip64(OcHierarchy h, const double* __restrict__ b, double* __restrict__ x,
               const double* __restrict__ Ainv, double tol, int maxit, double omega,
               int32_t* __restrict__ status, int32_t* __restrict__ iters,
               double* __restrict__ relres) {
  __shared__ double lds[kOcWords];
  const int t = threadIdx.x;
  const int s = blockIdx.x;
  constexpr int m = 64, n = m * m, w = 32;
  OcRegs g;
  const double* bs = b + (long long)s * n;
  oc_setup(g, lds, h, bs, Ainv, s, t);
  double xr[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, pr_[2][2] = {{0.0, 0.0}, {0.0, 0.0}};

  // r0 = b (x0 = 0)
  double acc = 0.0;
#pragma unroll
  for (int sl = 0; sl < 2; ++sl)
#pragma unroll
    for (int col = 0; col < 2; ++col) acc += g.r0[sl][col] * g.r0[sl][col];
  const double r0sq = oc_dot(acc, lds, t);
  int st = MLMC_SAMPLE_OK, it = 0, carried = 0;
  double* zR = lds;  // level-0 planes
  double* zB = lds + oc_plane(0);
  constexpr int P0 = oc_P(0);
  if (!(r0sq > 0.0) || !isfinite(r0sq)) {
    if (!isfinite(r0sq)) st = MLMC_SAMPLE_BREAKDOWN;
  } else {
    // pass 0 with the W mask of (gamma, gamma_levels); after a breakdown of
    // the W-preconditioned iteration, pass 1 from x0 = 0 with the V-cycle
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1) {
        carried = it;
        it = 0;
        st = MLMC_SAMPLE_OK;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
          const int pr = t + sl * kOcT;
    int j, cp;
    oc_pair<0>(pr, j, cp);
#pragma unroll
          for (int col = 0; col < 2; ++col) {
            const int i = 2 * cp + (col == 0 ? (j & 1) : 1 - (j & 1));
            g.r0[sl][col] = oc_ld(bs, j * m + i);
            xr[sl][col] = 0.0;
          }
        }
      }
      double rho = 0.0;
      bool broke = false;
      for (;;) {
        // z = M r, rho = r^T z, beta
        if (pass == 0) oc_cycle<0, WMASK>(g, lds, t, omega);
        else oc_cycle<0, 0u>(g, lds, t, omega);
        acc = 0.0;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
          const int pr = t + sl * kOcT;
    int j, cp;
    oc_pair<0>(pr, j, cp);
          acc += g.r0[sl][0] * zR[oc_zi(P0, j, cp)];
          acc += g.r0[sl][1] * zB[oc_zi(P0, j, cp)];
        }
        const double rho_new = oc_dot(acc, lds, t);
        if (!(rho_new > 0.0) || !isfinite(rho_new)) {
          broke = true;
          break;
        }
        const double beta = it == 0 ? 0.0 : rho_new / rho;
        rho = rho_new;
        ++it;
        // p = z + beta p, q = A p, p^T q
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
          const int pr = t + sl * kOcT;
    int j, cp;
    oc_pair<0>(pr, j, cp);
          const double z0 = zR[oc_zi(P0, j, cp)], z1 = zB[oc_zi(P0, j, cp)];
          pr_[sl][0] = it == 1 ? z0 : z0 + beta * pr_[sl][0];
          pr_[sl][1] = it == 1 ? z1 : z1 + beta * pr_[sl][1];
        }
        oc_write0(pr_, lds, t);
        double qv[2][2];
        oc_apply0(g, pr_, qv, lds, t);
        acc = 0.0;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl)
#pragma unroll
          for (int col = 0; col < 2; ++col) acc += pr_[sl][col] * qv[sl][col];
        const double pq = oc_dot(acc, lds, t);
        if (!(pq > 0.0) || !isfinite(pq)) {
          --it;  // the iteration did not complete
          broke = true;
          break;
        }
        const double alpha = rho / pq;
        acc = 0.0;
#pragma unroll
        for (int sl = 0; sl < 2; ++sl)
#pragma unroll
          for (int col = 0; col < 2; ++col) {
            xr[sl][col] += alpha * pr_[sl][col];
            g.r0[sl][col] -= alpha * qv[sl][col];
            acc += g.r0[sl][col] * g.r0[sl][col];
          }
        const double rr = oc_dot(acc, lds, t);
        if (!isfinite(rr)) {
          broke = true;
          break;
        }
        if (sqrt(rr / r0sq) < tol) {
          st = MLMC_SAMPLE_OK;
          break;
        }
        if (it >= maxit) {
          st = MLMC_SAMPLE_NOCONV;
          break;
        }
      }
      if (broke) st = MLMC_SAMPLE_BREAKDOWN;
      if (!(broke && WMASK != 0u && pass == 0)) break;
    }
    it += carried;
  }
  // true residual ||b - A x|| / ||b||, and the solution
  oc_write0(xr, lds, t);
  double qv[2][2];
  oc_apply0(g, xr, qv, lds, t);
  acc = 0.0;
  double* xs = x + (long long)s * n;
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int pr = t + sl * kOcT;
    int j, cp;
    oc_pair<0>(pr, j, cp);
#pragma unroll
    for (int col = 0; col < 2; ++col) {
      const int i = 2 * cp + (col == 0 ? (j & 1) : 1 - (j & 1));
      const double rv = oc_ld(bs, j * m + i) - qv[sl][col];
      acc += rv * rv;
      xs[j * m + i] = xr[sl][col];
    }
  }
  const double v = oc_dot(acc, lds, t);
  if (t == 0) {
    status[s] = st;
    iters[s] = it;
    relres[s] = r0sq > 0.0 ? sqrt(v / r0sq) : 0.0;
  }
}

// The W/V cycle of a 64^2 level that is not the finest of its solve, in one
// workgroup per sample: z = M_64 r for the levels 64, 32, 16, 8 and the 4^2
// inverse, the same cycle as the tiled down / mid / up kernels and the
// coarse-grid kernel, in one launch per visit instead of five.  r, z:
// [batch][64^2]; inactive samples are skipped.
template <unsigned WMASK>
__global__ void __launch_bounds__(kOcT)
k_cycle_onchip64(OcHierarchy h, const double* __restrict__ r, double* __restrict__ z,
                 const double* __restrict__ Ainv, double omega,
                 const int32_t* __restrict__ active) {
  __shared__ double lds[kOcWords];
  const int t = threadIdx.x;
  const int s = blockIdx.x;
  if (!active[s]) return;
  constexpr int m = 64, n = m * m;
  OcRegs g;
  oc_setup(g, lds, h, r + (long long)s * n, Ainv, s, t);
  oc_cycle<0, WMASK>(g, lds, t, omega);
  constexpr int P = oc_P(0);
  double* zs = z + (long long)s * n;
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int pr = t + sl * kOcT;
    int j, cp;
    oc_pair<0>(pr, j, cp);
    zs[j * m + 2 * cp + (j & 1)] = lds[oc_zi(P, j, cp)];
    zs[j * m + 2 * cp + 1 - (j & 1)] = lds[oc_plane(0) + oc_zi(P, j, cp)];
  }
}

void launch_cycle_onchip64(hipStream_t st, int batch, const OcHierarchy& h, const double* r,
                           double* z, const double* Ainv, double omega, unsigned wmask,
                           const int32_t* active) {
#define OC_LAUNCH(M)                                                                          \
  hipLaunchKernelGGL(k_cycle_onchip64<M>, dim3(batch), dim3(kOcT), 0, st, h, r, z, Ainv, omega, \
                     active)
  switch (wmask & 15u) {
    case 0u: OC_LAUNCH(0u); break;
    case 1u: OC_LAUNCH(1u); break;
    case 3u: OC_LAUNCH(3u); break;
    case 7u: OC_LAUNCH(7u); break;
    default: OC_LAUNCH(15u); break;
  }
#undef OC_LAUNCH
}

void launch_pcg_onchip64(hipStream_t st, int batch, const OcHierarchy& h, const double* b,
                         double* x, const double* Ainv, double tol, int maxit, double omega,
                         int gamma, int gamma_levels, int32_t* status, int32_t* iters,
                         double* relres) {
  unsigned wmask = 0;
  for (int L = 0; L < kOcLevels; ++L)
    if (gamma == 2 && (gamma_levels == 0 || L < gamma_levels)) wmask |= 1u << L;
#define OC_LAUNCH(M)                                                                       \
  hipLaunchKernelGGL(k_pcg_onchip64<M>, dim3(batch), dim3(kOcT), 0, st, h, b, x, Ainv, tol, \
                     maxit, omega, status, iters, relres)
  switch (wmask) {
    case 0u: OC_LAUNCH(0u); break;
    case 1u: OC_LAUNCH(1u); break;
    case 3u: OC_LAUNCH(3u); break;
    case 7u: OC_LAUNCH(7u); break;
    default: OC_LAUNCH(15u); break;
  }
#undef OC_LAUNCH
}

}  // namespace mlmc
