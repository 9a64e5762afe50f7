// Fused, LDS-tiled multigrid kernels for the symmetric V(1,1)-cycle on gfx950.
//
// The V-cycle of mg_pcg.hip does, on each level with a zero initial guess,
//   red sweep, black sweep, residual, 2x2 restriction  (down), and after the
//   coarse correction: prolongation, black sweep, red sweep (up).
// Launching each step separately streams the level's arrays through HBM six
// times.  Here the down and up halves are each one kernel over 2-D tiles held
// in LDS with a halo, so each level reads its operator once per half:
//
// down: with z = 0 the red sweep gives z_red = r / D; the black sweep gives
//   z_black = (r + N(z_red)) / D, where N(x)_P = sum over neighbours T_PQ x_Q.
//   After it the residual r - A z vanishes on black cells and equals N(z_black)
//   on red cells (D z_red = r), so the restricted residual of a 2x2 block is
//   the sum of N(z_black) over its two red cells.  A tile needs r and D two
//   cells beyond its edge (black halo cells use red values one further out)
//   and faces three cells beyond on the low side.
// up: z' = z + omega P z_c on the tile and two halo cells, a black sweep on the
//   tile and one halo cell, then a red sweep on the tile.  It reads the down
//   result from one buffer and writes the final z to another, because its halo
//   cells belong to tiles that other workgroups update in the same launch.
//
// Precision: every kernel is a template on the storage type S of the
// multigrid hierarchy (operators T, intermediate z, restricted residuals):
// double (FP64 arithmetic), float or bf16 (FP32 arithmetic).  On the finest
// level (TOP) the residual r read and the correction z written are FP64, as is
// the r^T z partial sum; the coarsest-grid solve runs in FP64 in any case.
//
// Levels of 32 x 32 cells or fewer are handled by k_mg_coarse_cycle: one
// workgroup per sample runs the remaining V-cycle entirely in LDS and applies
// the coarsest inverse (a dense matrix-vector product).
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace mlmc {

// ------------------------------------------------------------------ storage types
template <class S>
struct Prec;
template <>
struct Prec<double> {
  using C = double;
  __device__ static __forceinline__ double ld(const double* p, long long i) { return p[i]; }
  __device__ static __forceinline__ void st(double* p, long long i, double v) { p[i] = v; }
};
template <>
struct Prec<float> {
  using C = float;
  __device__ static __forceinline__ float ld(const float* p, long long i) { return p[i]; }
  __device__ static __forceinline__ void st(float* p, long long i, float v) { p[i] = v; }
};
template <>
struct Prec<bf16_t> {
  using C = float;
  __device__ static __forceinline__ float ld(const bf16_t* p, long long i) {
    return __uint_as_float((uint32_t)p[i].bits << 16);
  }
  // round to nearest, ties to even
  __device__ static __forceinline__ void st(bf16_t* p, long long i, float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    p[i].bits = (uint16_t)(u >> 16);
  }
};

// Type of the finest-level residual / correction: FP64; coarser levels: S.
template <class S, bool TOP>
using VecT = typename std::conditional<TOP, double, S>::type;

template <class V>
__device__ __forceinline__ typename Prec<V>::C ldv(const V* p, long long i) {
  return Prec<V>::ld(p, i);
}

// Load element i (< 2^32 / sizeof(V)) of a per-sample array whose base is
// uniform across the workgroup: the byte offset is an unsigned 32-bit value,
// so the load takes the base from scalar registers and one VGPR of offset
// instead of a 64-bit VGPR address.
template <class V>
__device__ __forceinline__ typename Prec<V>::C ldo(const V* p, unsigned i) {
  const V* q = reinterpret_cast<const V*>(reinterpret_cast<const char*>(p) +
                                          (size_t)(i * (unsigned)sizeof(V)));
  return Prec<V>::ld(q, 0);
}

// ------------------------------------------------------------------ fixed-tile helpers
// Tiles of compile-time size TX x TY (used when TX and TY divide m).  Each
// thread owns fixed frame cells in every phase and keeps their faces,
// reciprocal diagonal and right-hand side in registers; LDS holds z, which is
// what neighbours read.  All loads use clamped, always-valid addresses and are
// resolved by selects, so a thread's loads are issued back to back.  Tiles of
// one sample run on one XCD, so the halo re-reads hit that XCD's L2.
constexpr int kMgThreads = 512;

__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
  const int x = bid & 7, q = bid >> 3;
  const int per = nblocks >> 3, rem = nblocks & 7;
  return x * per + (x < rem ? x : rem) + q;
}

template <class C>
struct CellFaces {
  C te, tw, tn, ts;
  int c;    // clamped linear index of the cell in its sample
  bool in;  // inside the domain
};

// Faces of frame cells in two steps.  own_faces loads a cell's east and north
// faces from T (0 outside the domain); the caller writes them to two frame
// arrays in LDS, synchronises, and adjacent_faces takes the west and south
// faces from the neighbours' copies there, or from the boundary arrays on the
// domain's west / south edge.  Two global loads per frame cell instead of four
// (plus the boundary arrays only where a lane is on that edge).
template <class S>
__device__ __forceinline__ CellFaces<typename Prec<S>::C> own_faces(const S* __restrict__ Ts, int m,
                                                                    int i, int j) {
  using C = typename Prec<S>::C;
  CellFaces<C> v;
  const int ic = min(max(i, 0), m - 1), jc = min(max(j, 0), m - 1);
  v.c = jc * m + ic;
  v.in = i >= 0 && i < m && j >= 0 && j < m;
  const C te = ldo(Ts, (unsigned)v.c), tn = ldo(Ts, (unsigned)(m * m + v.c));
  v.te = v.in ? te : C(0);
  v.tn = v.in ? tn : C(0);
  v.tw = C(0);
  v.ts = C(0);
  return v;
}

// valid: f is a cell of the frame (fi, fj its column and row, W the pitch).
// Cells on the frame's own west column / south row (not on the domain edge)
// load the neighbour's face from T.
template <class S, class C>
__device__ __forceinline__ void adjacent_faces(CellFaces<C>& v, const C* se, const C* sn,
                                               const S* __restrict__ Ts,
                                               const S* __restrict__ tbs, int m, int i, int j,
                                               int f, int fi, int fj, int W, bool valid) {
  if (!valid || !v.in) return;
  if (i == 0) v.tw = ldv(tbs, j);
  else if (fi > 0) v.tw = se[f - 1];
  else v.tw = ldv(Ts, v.c - 1);
  if (j == 0) v.ts = ldv(tbs, m + i);
  else if (fj > 0) v.ts = sn[f - W];
  else v.ts = ldv(Ts, m * m + v.c - m);
}

template <class C>
__device__ __forceinline__ C inv_diag(const CellFaces<C>& f) {
  return f.in ? C(1) / (f.te + f.tw + f.tn + f.ts) : C(0);
}

template <class C>
__device__ __forceinline__ C nsum_lds(const CellFaces<C>& f, const C* sz, int fr, int W) {
  return f.te * sz[fr + 1] + f.tw * sz[fr - 1] + f.tn * sz[fr + W] + f.ts * sz[fr - W];
}

// ------------------------------------------------------------------ colour-split tile kernels
// The down / mid / up steps of the fixed-tile kernels above, with the frame
// split by colour: a thread owns "pairs" of horizontally adjacent frame cells
// (columns 2q and 2q + 1 of a row; one red, one black), keeps both cells'
// faces, reciprocal diagonals and right-hand sides in registers, and z lives
// in two zero-padded LDS planes, one per colour, indexed by (row, q).  In a
// half-sweep every lane then updates a cell of the swept colour (instead of
// half the lanes idling), and its four neighbours -- all of the other colour
// -- sit at contiguous plane addresses across the lanes:
//   red cell of pair (fj, q):   west/east other-plane q - 1 + (fj & 1), q + (fj & 1),
//                               north/south q in rows fj +- 1;
//   black cell of pair (fj, q): west/east q - (fj & 1), q + 1 - (fj & 1), north/south q.
// A pair's loads are 2-element vector loads (16 B in FP64); its west face is
// the east face of the cell to its left (one scalar load), its south faces the
// north faces of the row below.  The arithmetic and its order are those of the
// kernels above, so the results are the same bit for bit (the r^T z partial of
// up sums the cells in another order).
template <class V>
struct PairLd;
template <>
struct PairLd<double> {
  __device__ static __forceinline__ void ld(const double* p, unsigned i, double& a, double& b) {
    const double2 v = *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(p) +
                                                        (size_t)(i * 8u));
    a = v.x;
    b = v.y;
  }
  __device__ static __forceinline__ void st(double* p, long long i, double a, double b) {
    *reinterpret_cast<double2*>(p + i) = make_double2(a, b);
  }
};
template <>
struct PairLd<float> {
  __device__ static __forceinline__ void ld(const float* p, unsigned i, float& a, float& b) {
    const float2 v = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(p) +
                                                      (size_t)(i * 4u));
    a = v.x;
    b = v.y;
  }
  __device__ static __forceinline__ void st(float* p, long long i, float a, float b) {
    *reinterpret_cast<float2*>(p + i) = make_float2(a, b);
  }
};
template <>
struct PairLd<bf16_t> {
  __device__ static __forceinline__ void ld(const bf16_t* p, unsigned i, float& a, float& b) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(p) +
                                                          (size_t)(i * 2u));
    a = __uint_as_float(w << 16);
    b = __uint_as_float(w & 0xFFFF0000u);
  }
  __device__ static __forceinline__ void st(bf16_t* p, long long i, float a, float b) {
    uint32_t ua = __float_as_uint(a), ub = __float_as_uint(b);
    ua += 0x7FFFu + ((ua >> 16) & 1u);
    ub += 0x7FFFu + ((ub >> 16) & 1u);
    *reinterpret_cast<uint32_t*>(p + i) = (ua >> 16) | (ub & 0xFFFF0000u);
  }
};

template <class C>
struct PCell {
  C te, tw, tn, ts, di, rv;
};

// Geometry of a colour-split frame: tile TX x TY, HALO cells around it.
template <int TX, int TY, int HALO, int NT>
struct PGeom {
  static constexpr int W = TX + 2 * HALO, H = TY + 2 * HALO;
  static constexpr int P = W / 2, NP = P * H;          // pairs per row, pairs
  static constexpr int PP = P + 2, PL = PP * (H + 2);  // padded plane pitch, plane size
  static constexpr int K = (NP + NT - 1) / NT;         // pair slots per thread
  static_assert(K <= 4, "one flag byte per slot");
  static_assert(HALO % 2 == 0 && TX % 2 == 0, "pairs start on even columns");
  // plane index of pair (fj, q)
  __device__ static __forceinline__ int at(int fj, int q) { return (fj + 1) * PP + q + 1; }
};

// Zero the padding ring of both planes (interior cells are written by their owners).
template <class G, class C>
__device__ __forceinline__ void zero_padding(C* zR, C* zB, int nt) {
  for (int e = threadIdx.x; e < 2 * G::PP + 2 * G::H; e += nt) {
    const int o = e < G::PP       ? e
                  : e < 2 * G::PP ? (G::H + 1) * G::PP + e - G::PP
                                  : (1 + (e - 2 * G::PP) / 2) * G::PP + ((e & 1) ? G::PP - 1 : 0);
    zR[o] = C(0);
    zB[o] = C(0);
  }
}

// Operator rows and right-hand sides of the two cells of pair (fj, q) of the
// frame whose cell (0, 0) is the global cell (X0 - HALO, Y0 - HALO): red and
// black cell in that order, zero outside the domain (in = false).  Also the
// clamped linear index c of the pair's first cell, for further pair loads.
template <class S, class R, int HALO>
__device__ __forceinline__ void pair_rows(const S* __restrict__ Ts, const S* __restrict__ tbs,
                                          const R* __restrict__ rs, int m, int X0, int Y0, int fj,
                                          int q, bool valid,
                                          PCell<typename Prec<S>::C>& red,
                                          PCell<typename Prec<S>::C>& black, bool& in,
                                          unsigned& c, int& ic, int& jc, double (&rd)[2]) {
  using C = typename Prec<S>::C;
  const int i0 = X0 - HALO + 2 * q, j = Y0 - HALO + fj;
  in = valid && i0 >= 0 && i0 < m && j >= 0 && j < m;  // m even: both cells or neither
  ic = min(max(i0, 0), m - 2);
  jc = min(max(j, 0), m - 1);
  c = (unsigned)(jc * m + ic);
  const unsigned mm = (unsigned)(m * m);
  C te0, te1, tn0, tn1, tst0, tst1, tsb0, tsb1;
  PairLd<S>::ld(Ts, c, te0, te1);
  PairLd<S>::ld(Ts, mm + c, tn0, tn1);
  PairLd<S>::ld(Ts, mm + (c >= (unsigned)m ? c - (unsigned)m : 0u), tst0, tst1);
  PairLd<S>::ld(tbs, (unsigned)(m + ic), tsb0, tsb1);
  const C twt = ldo(Ts, c > 0u ? c - 1u : 0u), twb = ldo(tbs, (unsigned)jc);
  double r0, r1;
  {
    typename Prec<R>::C a, b;
    PairLd<R>::ld(rs, c, a, b);
    r0 = (double)a;
    r1 = (double)b;
  }
  PCell<C> c0{te0, i0 == 0 ? twb : twt, tn0, j == 0 ? tsb0 : tst0, C(0), (C)r0};
  PCell<C> c1{te1, te0, tn1, j == 0 ? tsb1 : tst1, C(0), (C)r1};
  if (in) {
    c0.di = C(1) / (c0.te + c0.tw + c0.tn + c0.ts);
    c1.di = C(1) / (c1.te + c1.tw + c1.tn + c1.ts);
  } else {
    c0 = PCell<C>{C(0), C(0), C(0), C(0), C(0), C(0)};
    c1 = c0;
    r0 = r1 = 0.0;
  }
  const bool odd = fj & 1;  // red is the cell with even global i + j
  red = odd ? c1 : c0;
  black = odd ? c0 : c1;
  rd[0] = odd ? r1 : r0;  // FP64 right-hand side, red then black
  rd[1] = odd ? r0 : r1;
}

// Flag byte of a pair: bit 0 in the domain, bit e (e = 1..3) red cell at least
// e cells inside the frame edge, bit 3 + e the same for the black cell, bit 7
// pair on the tile.
template <class G, int HALO>
__device__ __forceinline__ unsigned pair_flags(int fj, int q, bool in) {
  unsigned b = in ? 1u : 0u;
  const int cR = 2 * q + (fj & 1), cB = 2 * q + 1 - (fj & 1);
#pragma unroll
  for (int e = 1; e < HALO; ++e) {
    const bool row = fj >= e && fj < G::H - e;
    if (row && cR >= e && cR < G::W - e) b |= 1u << e;
    if (row && cB >= e && cB < G::W - e) b |= 1u << (3 + e);
  }
  if (fj >= HALO && fj < G::H - HALO && q >= HALO / 2 && q < G::P - HALO / 2) b |= 128u;
  return b;
}

// N(z) of the red / black cell of pair (fj, q) from the other colour's plane.
template <class G, class C>
__device__ __forceinline__ C nsum_red(const PCell<C>& c, const C* zB, int o, int par) {
  const int w = o - 1 + par;
  return c.te * zB[w + 1] + c.tw * zB[w] + c.tn * zB[o + G::PP] + c.ts * zB[o - G::PP];
}
template <class G, class C>
__device__ __forceinline__ C nsum_black(const PCell<C>& c, const C* zR, int o, int par) {
  const int w = o - par;
  return c.te * zR[w + 1] + c.tw * zR[w] + c.tn * zR[o + G::PP] + c.ts * zR[o - G::PP];
}

// One half-sweep over the pairs whose flags contain `want` (red or black cells).
template <class G, int NT, bool RED, class C>
__device__ __forceinline__ void pair_sweep(const PCell<C> (&cr)[G::K], const PCell<C> (&cb)[G::K],
                                           unsigned fl, unsigned want, C* zR, C* zB) {
#pragma unroll
  for (int k = 0; k < G::K; ++k) {
    if (((fl >> (8 * k)) & want) == want) {
      int g = threadIdx.x + k * NT;
      asm volatile("" : "+v"(g));  // keep the index math local to the sweep
      const int fj = g / G::P, q = g - fj * G::P;
      const int o = G::at(fj, q), par = fj & 1;
      if (RED) zR[o] = (cr[k].rv + nsum_red<G>(cr[k], zB, o, par)) * cr[k].di;
      else zB[o] = (cb[k].rv + nsum_black<G>(cb[k], zR, o, par)) * cb[k].di;
    }
  }
}

// Restriction: the coarse residual of each 2 x 2 block of the tile is the sum
// of the residuals of its two red cells, stored in place of their red z.
template <class G, int NT, int HALO, class S, class C>
__device__ __forceinline__ void pair_restrict(const C* zR, S* __restrict__ rcs, int mc, int X0,
                                              int Y0) {
  constexpr int HX = (G::W - 2 * HALO) / 2, HY = (G::H - 2 * HALO) / 2;
  for (int c = threadIdx.x; c < HX * HY; c += NT) {
    const int cj = c / HX, ci = c - cj * HX;
    // rows HALO + 2cj (red at column 2q) and HALO + 2cj + 1 (red at 2q + 1), q = HALO/2 + ci
    const int o = G::at(HALO + 2 * cj, HALO / 2 + ci);
    Prec<S>::st(rcs, (Y0 / 2 + cj) * mc + X0 / 2 + ci, zR[o] + zR[o + G::PP]);
  }
}

// down: red sweep from z = 0 (z_red = r / D), black sweep, store, restricted residual.
template <int TX, int TY, int NT, class S, bool TOP>
__global__ void __launch_bounds__(NT)
k_mg_down_p(int m, const S* __restrict__ T, const S* __restrict__ tb,
            const VecT<S, TOP>* __restrict__ r, S* __restrict__ z, S* __restrict__ rc,
            const int32_t* __restrict__ active) {
  using C = typename Prec<S>::C;
  using G = PGeom<TX, TY, 2, NT>;
  __shared__ C zR[G::PL];
  __shared__ C zB[G::PL];
  const int ntx = m / TX, tps = ntx * (m / TY);
  const int bid = xcd_tile(blockIdx.x, gridDim.x);
  const long long s = bid / tps;
  if (!active[s]) return;
  const int tile = bid - (int)(s * tps);
  const int X0 = (tile % ntx) * TX, Y0 = (tile / ntx) * TY;
  const long long n = (long long)m * m;
  const S* Ts = T + s * 2 * n;
  const S* tbs = tb + s * 2 * m;
  zero_padding<G>(zR, zB, NT);
  PCell<C> cr[G::K], cb[G::K];
  unsigned fl = 0;
#pragma unroll
  for (int k = 0; k < G::K; ++k) {
    const int g = threadIdx.x + k * NT;
    const int fj = g / G::P, q = g - fj * G::P;
    bool in;
    unsigned c;
    int ic, jc;
    double rd[2];
    pair_rows<S, VecT<S, TOP>, 2>(Ts, tbs, r + s * n, m, X0, Y0, fj, q, g < G::NP, cr[k], cb[k],
                                  in, c, ic, jc, rd);
    if (g < G::NP) {
      const int o = G::at(fj, q);
      zR[o] = in ? cr[k].rv * cr[k].di : C(0);
      zB[o] = C(0);
    }
    fl |= pair_flags<G, 2>(fj, q, in) << (8 * k);
  }
  __syncthreads();
  pair_sweep<G, NT, false>(cr, cb, fl, 1u | 16u, zR, zB);  // black on the frame less one ring
  __syncthreads();
  S* zs = z + s * n;
#pragma unroll
  for (int k = 0; k < G::K; ++k) {
    if ((fl >> (8 * k)) & 128u) {
      int g = threadIdx.x + k * NT;
      asm volatile("" : "+v"(g));
      const int fj = g / G::P, q = g - fj * G::P;
      const int o = G::at(fj, q), par = fj & 1;
      const C zr = zR[o], zb = zB[o];
      PairLd<S>::st(zs, (long long)(Y0 - 2 + fj) * m + (X0 - 2 + 2 * q), par ? zb : zr,
                    par ? zr : zb);
      // red residual r - D z_red + N(z) = N(z_black) (z_red = r / D)
      zR[o] = nsum_red<G>(cr[k], zB, o, par);
    }
  }
  __syncthreads();
  pair_restrict<G, NT, 2>(zR, rc + s * (long long)(m / 2) * (m / 2), m / 2, X0, Y0);
}

// mid: the second coarse correction of a W-cycle level (see k_mg_mid_t).
template <int TX, int TY, int NT, class S, bool TOP>
__global__ void __launch_bounds__(NT)
k_mg_mid_p(int m, const S* __restrict__ T, const S* __restrict__ tb,
           const VecT<S, TOP>* __restrict__ r, const S* __restrict__ zpre, S* __restrict__ z,
           const S* __restrict__ zc, double omega, S* __restrict__ rc,
           const int32_t* __restrict__ active) {
  using C = typename Prec<S>::C;
  using G = PGeom<TX, TY, 4, NT>;
  __shared__ C zR[G::PL];
  __shared__ C zB[G::PL];
  const int ntx = m / TX, tps = ntx * (m / TY);
  const int bid = xcd_tile(blockIdx.x, gridDim.x);
  const long long s = bid / tps;
  if (!active[s]) return;
  const int tile = bid - (int)(s * tps);
  const int X0 = (tile % ntx) * TX, Y0 = (tile / ntx) * TY;
  const long long n = (long long)m * m;
  const int mc = m / 2;
  const S* Ts = T + s * 2 * n;
  const S* tbs = tb + s * 2 * m;
  const S* zps = zpre + s * n;
  const S* zcs = zc + s * (long long)mc * mc;
  const C om = (C)omega;
  zero_padding<G>(zR, zB, NT);
  PCell<C> cr[G::K], cb[G::K];
  unsigned fl = 0;
#pragma unroll
  for (int k = 0; k < G::K; ++k) {
    const int g = threadIdx.x + k * NT;
    const int fj = g / G::P, q = g - fj * G::P;
    bool in;
    unsigned c;
    int ic, jc;
    double rd[2];
    pair_rows<S, VecT<S, TOP>, 4>(Ts, tbs, r + s * n, m, X0, Y0, fj, q, g < G::NP, cr[k], cb[k],
                                  in, c, ic, jc, rd);
    C zp0, zp1;
    PairLd<S>::ld(zps, c, zp0, zp1);
    const C zcv = ldo(zcs, (unsigned)((jc >> 1) * mc + (ic >> 1)));
    if (g < G::NP) {
      const int o = G::at(fj, q);
      const C z0 = in ? zp0 + om * zcv : C(0), z1 = in ? zp1 + om * zcv : C(0);
      zR[o] = (fj & 1) ? z1 : z0;
      zB[o] = (fj & 1) ? z0 : z1;
    }
    fl |= pair_flags<G, 4>(fj, q, in) << (8 * k);
  }
  __syncthreads();
  pair_sweep<G, NT, false>(cr, cb, fl, 1u | (1u << 4), zR, zB);  // black, 1 cell in
  __syncthreads();
  pair_sweep<G, NT, true>(cr, cb, fl, 1u | (1u << 2), zR, zB);   // red, 2 cells in
  __syncthreads();
  pair_sweep<G, NT, false>(cr, cb, fl, 1u | (1u << 6), zR, zB);  // black, 3 cells in
  __syncthreads();
  S* zs = z + s * n;
#pragma unroll
  for (int k = 0; k < G::K; ++k) {
    if ((fl >> (8 * k)) & 128u) {
      int g = threadIdx.x + k * NT;
      asm volatile("" : "+v"(g));
      const int fj = g / G::P, q = g - fj * G::P;
      const int o = G::at(fj, q), par = fj & 1;
      const C zr = zR[o], zb = zB[o];
      PairLd<S>::st(zs, (long long)(Y0 - 4 + fj) * m + (X0 - 4 + 2 * q), par ? zb : zr,
                    par ? zr : zb);
      const PCell<C>& c = cr[k];
      const C dd = c.te + c.tw + c.tn + c.ts;
      zR[o] = c.rv - dd * zr + nsum_red<G>(c, zB, o, par);  // black residuals vanish
    }
  }
  __syncthreads();
  pair_restrict<G, NT, 4>(zR, rc + s * (long long)mc * mc, mc, X0, Y0);
}

// up: z = z_in + omega P e, black sweep, red sweep on the tile, store and, on
// the finest level, the per-tile partial of r^T z.
template <int TX, int TY, int NT, class S, bool TOP>
__global__ void __launch_bounds__(NT)
k_mg_up_p(int m, const S* __restrict__ T, const S* __restrict__ tb,
          const VecT<S, TOP>* __restrict__ r, const S* __restrict__ zpre,
          VecT<S, TOP>* __restrict__ z, const S* __restrict__ zc, double omega,
          const int32_t* __restrict__ active, double* __restrict__ rz_partial) {
  using C = typename Prec<S>::C;
  using G = PGeom<TX, TY, 2, NT>;
  __shared__ C zR[G::PL];
  __shared__ C zB[G::PL];
  __shared__ double red[(NT + kWave - 1) / kWave];
  const int ntx = m / TX, tps = ntx * (m / TY);
  const int bid = xcd_tile(blockIdx.x, gridDim.x);
  const long long s = bid / tps;
  if (!active[s]) return;
  const int tile = bid - (int)(s * tps);
  const int X0 = (tile % ntx) * TX, Y0 = (tile / ntx) * TY;
  const long long n = (long long)m * m;
  const int mc = m / 2;
  const S* Ts = T + s * 2 * n;
  const S* tbs = tb + s * 2 * m;
  const S* zps = zpre + s * n;
  const S* zcs = zc + s * (long long)mc * mc;
  const C om = (C)omega;
  zero_padding<G>(zR, zB, NT);
  PCell<C> cr[G::K], cb[G::K];
  double rdr[G::K], rdb[G::K];  // FP64 right-hand sides for r^T z (finest level)
  unsigned fl = 0;
#pragma unroll
  for (int k = 0; k < G::K; ++k) {
    const int g = threadIdx.x + k * NT;
    const int fj = g / G::P, q = g - fj * G::P;
    bool in;
    unsigned c;
    int ic, jc;
    double rd[2];
    pair_rows<S, VecT<S, TOP>, 2>(Ts, tbs, r + s * n, m, X0, Y0, fj, q, g < G::NP, cr[k], cb[k],
                                  in, c, ic, jc, rd);
    rdr[k] = rd[0];
    rdb[k] = rd[1];
    C zp0, zp1;
    PairLd<S>::ld(zps, c, zp0, zp1);
    const C zcv = ldo(zcs, (unsigned)((jc >> 1) * mc + (ic >> 1)));
    if (g < G::NP) {
      const int o = G::at(fj, q);
      const C z0 = in ? zp0 + om * zcv : C(0), z1 = in ? zp1 + om * zcv : C(0);
      zR[o] = (fj & 1) ? z1 : z0;
      zB[o] = (fj & 1) ? z0 : z1;
    }
    fl |= pair_flags<G, 2>(fj, q, in) << (8 * k);
  }
  __syncthreads();
  pair_sweep<G, NT, false>(cr, cb, fl, 1u | 16u, zR, zB);  // black on the frame less one ring
  __syncthreads();
  using Z = VecT<S, TOP>;
  Z* zs = z + s * n;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < G::K; ++k) {
    if ((fl >> (8 * k)) & 128u) {
      int g = threadIdx.x + k * NT;
      asm volatile("" : "+v"(g));
      const int fj = g / G::P, q = g - fj * G::P;
      const int o = G::at(fj, q), par = fj & 1;
      const C zb = zB[o];
      const C zr = (cr[k].rv + nsum_red<G>(cr[k], zB, o, par)) * cr[k].di;  // red sweep
      PairLd<Z>::st(zs, (long long)(Y0 - 2 + fj) * m + (X0 - 2 + 2 * q), par ? zb : zr,
                    par ? zr : zb);
      if (TOP) acc += rdr[k] * (double)zr + rdb[k] * (double)zb;
    }
  }
  if (TOP && rz_partial) {
    acc = wave_sum(acc);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < (NT + kWave - 1) / kWave; ++w) t += red[w];
      rz_partial[s * tps + tile] = t;
    }
  }
}

// ------------------------------------------------------------------ CG direction + operator
// One conjugate-gradient step's p = z + beta p_old (p = z on the first step)
// and q = A p with the partial sums of p^T q per tile, over tiles of TX x TY
// cells with a one-cell halo: halo values of p are recomputed from z and p_old
// (the same formula the neighbouring tile uses), so p_new goes to a buffer
// other than p_old.  All FP64, operator of the finest level.
template <int TX, int TY>
__global__ void __launch_bounds__(kMgThreads)
k_cg_direction_t(int m, const double* __restrict__ T, const double* __restrict__ tb,
                 const double* __restrict__ z, const double* __restrict__ pold,
                 double* __restrict__ pnew, double* __restrict__ q,
                 const double* __restrict__ beta, int first, double* __restrict__ partial,
                 const int32_t* __restrict__ active) {
  constexpr int W = TX + 2, H = TY + 2, F = W * H;
  constexpr int K = (F + kMgThreads - 1) / kMgThreads;
  __shared__ double sp[F];
  __shared__ double sn[F];
  __shared__ double red[kMgThreads / kWave];
  const int ntx = m / TX, tps = ntx * (m / TY);
  const int bid = xcd_tile(blockIdx.x, gridDim.x);
  const long long s = bid / tps;
  if (!active[s]) return;
  const int tile = bid - (int)(s * tps);
  const int X0 = (tile % ntx) * TX, Y0 = (tile / ntx) * TY;
  const long long n = (long long)m * m;
  const double* Ts = T + s * 2 * n;
  const double* tbs = tb + s * 2 * m;
  const double* zs = z + s * n;
  const double* ps = pold + s * n;
  const double bt = first ? 0.0 : beta[s];
  CellFaces<double> cf[K];
  double pv[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    const int i = X0 - 1 + fi, j = Y0 - 1 + fj;
    cf[k] = own_faces(Ts, m, i, j);
    const double zv = zs[cf[k].c], po = ps[cf[k].c];
    pv[k] = cf[k].in ? (first ? zv : zv + bt * po) : 0.0;
    if (f < F) {
      sp[f] = cf[k].te;
      sn[f] = cf[k].tn;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    adjacent_faces(cf[k], sp, sn, Ts, tbs, m, X0 - 1 + fi, Y0 - 1 + fj, f, fi, fj, W, f < F);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    if (f < F) sp[f] = pv[k];
  }
  __syncthreads();
  double* pn = pnew + s * n;
  double* qs = q + s * n;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    if (f < F && fi >= 1 && fi <= TX && fj >= 1 && fj <= TY) {
      const double d = cf[k].te + cf[k].tw + cf[k].tn + cf[k].ts;
      const double qv = d * pv[k] - (cf[k].te * sp[f + 1] + cf[k].tw * sp[f - 1] +
                                     cf[k].tn * sp[f + W] + cf[k].ts * sp[f - W]);
      pn[cf[k].c] = pv[k];
      qs[cf[k].c] = qv;
      acc += pv[k] * qv;
    }
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kMgThreads / kWave; ++w) t += red[w];
    partial[s * tps + tile] = t;
  }
}

// ------------------------------------------------------------------ runtime-tile kernels
// Same algorithm for sizes the fixed tiles do not divide (tx, ty: even
// divisors of m), 256 threads, all four frame arrays in LDS.
struct FrameGeom {
  int m, tx, ty, W, H;  // level size, tile size, frame width/height
  int X0, Y0;           // tile origin (global cell indices)
  __device__ __forceinline__ int gi(int fi) const { return X0 - 3 + fi; }
  __device__ __forceinline__ int gj(int fj) const { return Y0 - 3 + fj; }
  __device__ __forceinline__ bool inside(int i, int j) const {
    return i >= 0 && i < m && j >= 0 && j < m;
  }
};

__device__ __forceinline__ FrameGeom frame_of(int m, int tx, int ty, int tile) {
  FrameGeom g;
  g.m = m;
  g.tx = tx;
  g.ty = ty;
  g.W = tx + 5;
  g.H = ty + 5;
  const int ntx = m / tx;
  g.X0 = (tile % ntx) * tx;
  g.Y0 = (tile / ntx) * ty;
  return g;
}

// Face of cell (i, j) along x1 in the extended sense: i = -1 is the west
// boundary face of row j; faces outside the domain are 0.
template <class S>
__device__ __forceinline__ typename Prec<S>::C load_te(const S* Ts, const S* tbs, int m, int i,
                                                       int j) {
  using C = typename Prec<S>::C;
  if (j < 0 || j >= m) return C(0);
  if (i == -1) return ldv(tbs, j);
  if (i < 0 || i >= m) return C(0);
  return ldv(Ts, j * m + i);
}

template <class S>
__device__ __forceinline__ typename Prec<S>::C load_tn(const S* Ts, const S* tbs, int m, int i,
                                                       int j) {
  using C = typename Prec<S>::C;
  if (i < 0 || i >= m) return C(0);
  if (j == -1) return ldv(tbs, m + i);
  if (j < 0 || j >= m) return C(0);
  return ldv(Ts, m * m + j * m + i);
}

template <class C>
struct Lds {
  C* te;
  C* tn;
  C* r;
  C* z;
};

template <class C>
__device__ __forceinline__ C diag_at(const Lds<C>& s, int W, int f) {
  return s.te[f] + s.te[f - 1] + s.tn[f] + s.tn[f - W];
}

template <class C>
__device__ __forceinline__ C nsum_at(const Lds<C>& s, int W, int f) {
  return s.te[f] * s.z[f + 1] + s.te[f - 1] * s.z[f - 1] + s.tn[f] * s.z[f + W] +
         s.tn[f - W] * s.z[f - W];
}

template <class S, bool TOP>
__global__ void __launch_bounds__(kBlock)
k_mg_down(int m, int tx, int ty, int tiles_per_sample, const S* __restrict__ T,
          const S* __restrict__ tb, const VecT<S, TOP>* __restrict__ r, S* __restrict__ z,
          S* __restrict__ rc, const int32_t* __restrict__ active) {
  using C = typename Prec<S>::C;
  extern __shared__ double lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const long long s = blockIdx.x / tiles_per_sample;
  if (!active[s]) return;
  const FrameGeom g = frame_of(m, tx, ty, blockIdx.x - (int)(s * tiles_per_sample));
  const int W = g.W, H = g.H, F = W * H;
  Lds<C> L{lds, lds + F, lds + 2 * F, lds + 3 * F};
  const long long n = (long long)m * m;
  const S* Ts = T + s * 2 * n;
  const S* tbs = tb + s * 2 * m;
  const VecT<S, TOP>* rs = r + s * n;
  for (int f = threadIdx.x; f < F; f += kBlock) {
    const int fj = f / W, fi = f - fj * W;
    const int i = g.gi(fi), j = g.gj(fj);
    L.te[f] = load_te(Ts, tbs, m, i, j);
    L.tn[f] = load_tn(Ts, tbs, m, i, j);
    L.r[f] = g.inside(i, j) ? (C)ldv(rs, j * m + i) : C(0);
  }
  __syncthreads();
  for (int f = threadIdx.x; f < F; f += kBlock) {
    const int fj = f / W, fi = f - fj * W;
    const int i = g.gi(fi), j = g.gj(fj);
    C v = C(0);
    if (fi >= 1 && fj >= 1 && g.inside(i, j) && ((i + j) & 1) == 0) v = L.r[f] / diag_at(L, W, f);
    L.z[f] = v;
  }
  __syncthreads();
  for (int f = threadIdx.x; f < F; f += kBlock) {
    const int fj = f / W, fi = f - fj * W;
    if (fi < 2 || fi >= W - 1 || fj < 2 || fj >= H - 1) continue;
    const int i = g.gi(fi), j = g.gj(fj);
    if (!g.inside(i, j) || ((i + j) & 1) == 0) continue;
    L.z[f] = (L.r[f] + nsum_at(L, W, f)) / diag_at(L, W, f);
  }
  __syncthreads();
  S* zs = z + s * n;
  const int tcells = tx * ty;
  for (int c = threadIdx.x; c < tcells; c += kBlock) {
    const int cj = c / tx, ci = c - cj * tx;
    Prec<S>::st(zs, (g.Y0 + cj) * m + g.X0 + ci, L.z[(cj + 3) * W + ci + 3]);
  }
  const int mc = m / 2, hx = tx / 2, hy = ty / 2;
  S* rcs = rc + s * (long long)mc * mc;
  for (int c = threadIdx.x; c < hx * hy; c += kBlock) {
    const int cj = c / hx, ci = c - cj * hx;
    const int fi0 = 3 + 2 * ci, fj0 = 3 + 2 * cj;
    // (X0 + 2ci, Y0 + 2cj) has even i + j: the block's red cells are (0,0) and (1,1)
    const int fa = fj0 * W + fi0, fb = (fj0 + 1) * W + fi0 + 1;
    Prec<S>::st(rcs, (g.Y0 / 2 + cj) * mc + g.X0 / 2 + ci, nsum_at(L, W, fa) + nsum_at(L, W, fb));
  }
}

template <class S, bool TOP>
__global__ void __launch_bounds__(kBlock)
k_mg_up(int m, int tx, int ty, int tiles_per_sample, const S* __restrict__ T,
        const S* __restrict__ tb, const VecT<S, TOP>* __restrict__ r, const S* __restrict__ zpre,
        VecT<S, TOP>* __restrict__ z, const S* __restrict__ zc, double omega,
        const int32_t* __restrict__ active, double* __restrict__ rz_partial) {
  using C = typename Prec<S>::C;
  extern __shared__ double lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const long long s = blockIdx.x / tiles_per_sample;
  if (!active[s]) return;
  const FrameGeom g = frame_of(m, tx, ty, blockIdx.x - (int)(s * tiles_per_sample));
  const int W = g.W, H = g.H, F = W * H;
  Lds<C> L{lds, lds + F, lds + 2 * F, lds + 3 * F};
  const long long n = (long long)m * m;
  const int mc = m / 2;
  const S* Ts = T + s * 2 * n;
  const S* tbs = tb + s * 2 * m;
  const VecT<S, TOP>* rs = r + s * n;
  const S* zps = zpre + s * n;
  VecT<S, TOP>* zs = z + s * n;
  const S* zcs = zc + s * (long long)mc * mc;
  const C om = (C)omega;
  for (int f = threadIdx.x; f < F; f += kBlock) {
    const int fj = f / W, fi = f - fj * W;
    const int i = g.gi(fi), j = g.gj(fj);
    L.te[f] = load_te(Ts, tbs, m, i, j);
    L.tn[f] = load_tn(Ts, tbs, m, i, j);
    const bool in = g.inside(i, j);
    L.r[f] = in ? (C)ldv(rs, j * m + i) : C(0);
    L.z[f] = in ? ldv(zps, j * m + i) + om * ldv(zcs, (j >> 1) * mc + (i >> 1)) : C(0);
  }
  __syncthreads();
  for (int f = threadIdx.x; f < F; f += kBlock) {
    const int fj = f / W, fi = f - fj * W;
    if (fi < 2 || fi >= W - 1 || fj < 2 || fj >= H - 1) continue;
    const int i = g.gi(fi), j = g.gj(fj);
    if (!g.inside(i, j) || ((i + j) & 1) == 0) continue;
    L.z[f] = (L.r[f] + nsum_at(L, W, f)) / diag_at(L, W, f);
  }
  __syncthreads();
  const int tcells = tx * ty;
  for (int c = threadIdx.x; c < tcells; c += kBlock) {
    const int cj = c / tx, ci = c - cj * tx;
    const int f = (cj + 3) * W + ci + 3;
    const int i = g.X0 + ci, j = g.Y0 + cj;
    if (((i + j) & 1) == 0) L.z[f] = (L.r[f] + nsum_at(L, W, f)) / diag_at(L, W, f);
  }
  __syncthreads();
  double acc = 0.0;
  for (int c = threadIdx.x; c < tcells; c += kBlock) {
    const int cj = c / tx, ci = c - cj * tx;
    const int f = (cj + 3) * W + ci + 3;
    const long long e = (g.Y0 + cj) * m + g.X0 + ci;
    Prec<VecT<S, TOP>>::st(zs, e, L.z[f]);
    if (TOP) acc += (double)ldv(rs, e) * (double)L.z[f];
  }
  if (TOP && rz_partial) {
    __shared__ double red[kBlock / kWave];
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) rz_partial[blockIdx.x] = t;
  }
}

// Runtime-tile form of the mid kernel: the frame reaches four cells around the
// tile; the restriction computes each coarse cell's two red residuals directly.
template <class S, bool TOP>
__global__ void __launch_bounds__(kBlock)
k_mg_mid(int m, int tx, int ty, int tiles_per_sample, const S* __restrict__ T,
         const S* __restrict__ tb, const VecT<S, TOP>* __restrict__ r, const S* __restrict__ zpre,
         S* __restrict__ z, const S* __restrict__ zc, double omega, S* __restrict__ rc,
         const int32_t* __restrict__ active) {
  using C = typename Prec<S>::C;
  extern __shared__ double lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const long long s = blockIdx.x / tiles_per_sample;
  if (!active[s]) return;
  const int tile = blockIdx.x - (int)(s * tiles_per_sample);
  const int ntx = m / tx;
  const int X0 = (tile % ntx) * tx, Y0 = (tile / ntx) * ty;
  const int W = tx + 8, H = ty + 8, F = W * H;
  Lds<C> L{lds, lds + F, lds + 2 * F, lds + 3 * F};
  const long long n = (long long)m * m;
  const int mc = m / 2;
  const S* Ts = T + s * 2 * n;
  const S* tbs = tb + s * 2 * m;
  const VecT<S, TOP>* rs = r + s * n;
  const S* zps = zpre + s * n;
  const S* zcs = zc + s * (long long)mc * mc;
  const C om = (C)omega;
  for (int f = threadIdx.x; f < F; f += kBlock) {
    const int fj = f / W, fi = f - fj * W;
    const int i = X0 - 4 + fi, j = Y0 - 4 + fj;
    L.te[f] = load_te(Ts, tbs, m, i, j);
    L.tn[f] = load_tn(Ts, tbs, m, i, j);
    const bool in = i >= 0 && i < m && j >= 0 && j < m;
    L.r[f] = in ? (C)ldv(rs, j * m + i) : C(0);
    L.z[f] = in ? ldv(zps, j * m + i) + om * ldv(zcs, (j >> 1) * mc + (i >> 1)) : C(0);
  }
  __syncthreads();
  for (int pass = 0; pass < 3; ++pass) {
    const int d = 3 - pass, col = (pass == 1) ? 0 : 1;
    for (int f = threadIdx.x; f < F; f += kBlock) {
      const int fj = f / W, fi = f - fj * W;
      if (fi < 4 - d || fi >= W - 4 + d || fj < 4 - d || fj >= H - 4 + d) continue;
      const int i = X0 - 4 + fi, j = Y0 - 4 + fj;
      if (i < 0 || i >= m || j < 0 || j >= m || ((i + j) & 1) != col) continue;
      L.z[f] = (L.r[f] + nsum_at(L, W, f)) / diag_at(L, W, f);
    }
    __syncthreads();
  }
  S* zs = z + s * n;
  for (int c = threadIdx.x; c < tx * ty; c += kBlock) {
    const int cj = c / tx, ci = c - cj * tx;
    Prec<S>::st(zs, (Y0 + cj) * m + X0 + ci, L.z[(cj + 4) * W + ci + 4]);
  }
  const int hx = tx / 2, hy = ty / 2;
  S* rcs = rc + s * (long long)mc * mc;
  for (int c = threadIdx.x; c < hx * hy; c += kBlock) {
    const int cj = c / hx, ci = c - cj * hx;
    // (X0 + 2ci, Y0 + 2cj) has even i + j: the block's red cells are (0,0) and (1,1)
    const int fa = (4 + 2 * cj) * W + 4 + 2 * ci, fb = fa + W + 1;
    const C ra = L.r[fa] - diag_at(L, W, fa) * L.z[fa] + nsum_at(L, W, fa);
    const C rb = L.r[fb] - diag_at(L, W, fb) * L.z[fb] + nsum_at(L, W, fb);
    Prec<S>::st(rcs, (Y0 / 2 + cj) * mc + X0 / 2 + ci, ra + rb);
  }
}

// ------------------------------------------------------------------ coarse cycle in LDS
// One workgroup per sample runs the V- or W-cycle on levels l0..L (m_l0 <= 32)
// in FP64 with every level's operator and vectors in LDS, whatever the
// storage type of the hierarchy.  Level arrays use a padded (m + 2)^2 layout
// with a one-cell ring: ring cells hold z = 0 and the boundary faces (west
// face in column -1, south face in row -1), so the stencil needs no branches.
struct CoarseLevel {
  int m, P, off;  // size, padded pitch (m + 2), offset of the level's arrays in LDS
};

__device__ __forceinline__ int pidx(int P, int i, int j) { return (j + 1) * P + (i + 1); }

__device__ void cc_sweep(double* te, double* tn, double* r, double* z, int m, int P, int color,
                         bool zero) {
  const int half = m / 2 > 0 ? m / 2 : 1;
  const int cnt = m * half;
  for (int c = threadIdx.x; c < cnt; c += kBlock) {
    const int j = c / half;
    int i = 2 * (c - j * half) + ((j + color) & 1);
    if (i >= m) continue;
    const int f = pidx(P, i, j);
    const double d = te[f] + te[f - 1] + tn[f] + tn[f - P];
    z[f] = zero ? r[f] / d
                : (r[f] + te[f] * z[f + 1] + te[f - 1] * z[f - 1] + tn[f] * z[f + P] +
                   tn[f - P] * z[f - P]) / d;
  }
  __syncthreads();
}

template <class S, bool TOP>
__global__ void __launch_bounds__(kBlock)
k_mg_coarse_cycle(int nlev, CoarseDesc desc, const VecT<S, TOP>* __restrict__ r0,
                  VecT<S, TOP>* __restrict__ z0, const double* __restrict__ Ainv, double omega,
                  unsigned wmask, const int32_t* __restrict__ active,
                  double* __restrict__ rz_partial) {
  extern __shared__ double lds[];
  const int s = blockIdx.x;
  if (!active[s]) return;
  // the level table in LDS: the cycle indexes it by the running level, a
  // per-thread array would live in scratch memory
  __shared__ CoarseLevel lv[kMaxCoarseLevels];
  int off = 0;
  for (int l = 0; l < nlev; ++l) {
    const int P = desc.m[l] + 2;
    if (threadIdx.x == 0) lv[l] = CoarseLevel{desc.m[l], P, off};
    off += 4 * P * P;
  }
  __syncthreads();
  double* vec = lds + off;  // coarsest right-hand side (n_c doubles)
  for (int l = 0; l < nlev; ++l) {
    const int m = lv[l].m, P = lv[l].P, PP = P * P;
    double* te = lds + lv[l].off;
    double* tn = te + PP;
    double* rr = tn + PP;
    double* zz = rr + PP;
    const long long n = (long long)m * m;
    const S* Ts = static_cast<const S*>(desc.T[l]) + (long long)s * 2 * n;
    const S* tbs = static_cast<const S*>(desc.tb[l]) + (long long)s * 2 * m;
    for (int f = threadIdx.x; f < PP; f += kBlock) {
      const int j = f / P - 1, i = f % P - 1;
      te[f] = (double)load_te(Ts, tbs, m, i, j);
      tn[f] = (double)load_tn(Ts, tbs, m, i, j);
      rr[f] = (l == 0 && i >= 0 && i < m && j >= 0 && j < m)
                  ? (double)ldv(r0, (long long)s * n + j * m + i)
                  : 0.0;
      zz[f] = 0.0;
    }
  }
  __syncthreads();
  // V/W-cycle without recursion (bit l of wmask: level l takes two coarse
  // visits).  Entering a level downwards (r set, z = 0): red and black sweeps
  // from zero, restrict the residual, go down.  Coming back up: add the
  // prolonged correction, black and red sweeps; then leave upwards, or, on a
  // W level after its first visit, pre-smooth again (its red sweep would repeat
  // the one just done, so only the black sweep) and go down again.
  unsigned once = 0;  // bit l: level l has had its first coarse visit
  int l = 0;
  bool descending = true;
  for (;;) {
    const int m = lv[l].m, P = lv[l].P, PP = P * P;
    double* te = lds + lv[l].off;
    double* tn = te + PP;
    double* rr = tn + PP;
    double* zz = rr + PP;
    if (l == nlev - 1) {
      const int nc = m * m;
      for (int q = threadIdx.x; q < nc; q += kBlock) vec[q] = rr[pidx(P, q % m, q / m)];
      __syncthreads();
      const double* A = Ainv + (long long)s * nc * nc;
      for (int q = threadIdx.x; q < nc; q += kBlock) {
        double acc = 0.0;
        for (int p = 0; p < nc; ++p) acc += A[q * nc + p] * vec[p];
        zz[pidx(P, q % m, q / m)] = acc;
      }
      __syncthreads();
      if (l == 0) break;
      --l;
      descending = false;
      continue;
    }
    if (descending) {
      cc_sweep(te, tn, rr, zz, m, P, 0, true);
      cc_sweep(te, tn, rr, zz, m, P, 1, false);
    } else {
      const int Pc = lv[l + 1].P, PPc = Pc * Pc;
      const double* zc = lds + lv[l + 1].off + 3 * PPc;
      for (int c = threadIdx.x; c < m * m; c += kBlock) {
        const int j = c / m, i = c - j * m;
        zz[pidx(P, i, j)] += omega * zc[pidx(Pc, i / 2, j / 2)];
      }
      __syncthreads();
      cc_sweep(te, tn, rr, zz, m, P, 1, false);
      cc_sweep(te, tn, rr, zz, m, P, 0, false);
      if (!(wmask >> l & 1u) || (once >> l & 1u)) {
        once &= ~(1u << l);
        if (l == 0) break;
        --l;
        continue;
      }
      once |= 1u << l;
      cc_sweep(te, tn, rr, zz, m, P, 1, false);
    }
    const int mc = lv[l + 1].m, Pc = lv[l + 1].P, PPc = Pc * Pc;
    double* rc = lds + lv[l + 1].off + 2 * PPc;
    for (int c = threadIdx.x; c < mc * mc; c += kBlock) {
      const int J = c / mc, I = c - J * mc;
      double acc = 0.0;
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          const int f = pidx(P, 2 * I + a, 2 * J + b);
          const double d = te[f] + te[f - 1] + tn[f] + tn[f - P];
          acc += rr[f] - d * zz[f] + te[f] * zz[f + 1] + te[f - 1] * zz[f - 1] + tn[f] * zz[f + P] +
                 tn[f - P] * zz[f - P];
        }
      rc[pidx(Pc, I, J)] = acc;
    }
    __syncthreads();
    ++l;
    descending = true;
  }
  {
    const int m = lv[0].m, P = lv[0].P, PP = P * P;
    const double* rr = lds + lv[0].off + 2 * PP;
    const double* zz = rr + PP;
    double acc = 0.0;
    for (int c = threadIdx.x; c < m * m; c += kBlock) {
      const int f = pidx(P, c % m, c / m);
      Prec<VecT<S, TOP>>::st(z0, (long long)s * m * m + c, zz[f]);
      acc += rr[f] * zz[f];
    }
    if (TOP && rz_partial) {
      __shared__ double red[kBlock / kWave];
      const double t = block_sum(acc, red);
      if (threadIdx.x == 0) rz_partial[s] = t;
    }
  }
}

// V-cycle form of the coarse cycle (optionally W at its finest level) with
// the operator in registers.  One
// workgroup of 512 threads per sample; thread t owns cells t and t + 512 of
// level l0 (m <= 32) and cell t of every coarser smoothing level, with their
// faces, reciprocal diagonal, right-hand side and z in registers.  LDS holds
// only z of every level (padded (m + 2)^2 layout, zero ring), the residual
// the restriction gathers, and the coarsest right-hand side.  NL = number of
// smoothing levels (the coarsest, solved with its dense inverse, is level NL).
constexpr int kCcThreads = 512;
constexpr int kCcMaxSmooth = 5;
constexpr int kCcLdsInv = 16;

struct CcCell {
  double te, tw, tn, ts, di, r, z;
  int cell, f;  // linear index in the level, index in the padded z array
  bool in;      // the slot holds a cell of the level
  bool red;
};

template <class S>
__device__ __forceinline__ void cc_load(CcCell& c, const S* __restrict__ Ts,
                                        const S* __restrict__ tbs, int m, int cell) {
  const int n = m * m;
  c.in = cell < n;
  const int q = c.in ? cell : 0;
  const int j = q / m, i = q - j * m;
  c.cell = q;
  c.f = pidx(m + 2, i, j);
  c.red = ((i + j) & 1) == 0;
  const double te = (double)ldv(Ts, q), tn = (double)ldv(Ts, n + q);
  const double tw = (double)(i > 0 ? ldv(Ts, q - 1) : ldv(tbs, j));
  const double ts = (double)(j > 0 ? ldv(Ts, n + q - m) : ldv(tbs, m + i));
  c.te = te;
  c.tn = tn;
  c.tw = tw;
  c.ts = ts;
  c.di = c.in ? 1.0 / (te + tw + tn + ts) : 0.0;
  c.r = 0.0;
  c.z = 0.0;
}

__device__ __forceinline__ double cc_nsum(const CcCell& c, const double* z, int P) {
  return c.te * z[c.f + 1] + c.tw * z[c.f - 1] + c.tn * z[c.f + P] + c.ts * z[c.f - P];
}

// One colour of a Gauss-Seidel sweep over a thread's slots (zero: z = 0 before).
template <int K>
__device__ __forceinline__ void cc_smooth(CcCell* c, double* z, int P, bool red, bool zero) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (c[k].in && c[k].red == red) {
      c[k].z = zero ? c[k].r * c[k].di : (c[k].r + cc_nsum(c[k], z, P)) * c[k].di;
      z[c[k].f] = c[k].z;
    }
  }
  __syncthreads();
}

// Restriction of the red-cell residuals held in sres (level of size m) to the
// coarse level: coarse cell t gathers fine cells (2I, 2J) and (2I + 1, 2J + 1).
__device__ __forceinline__ double cc_gather(const double* sres, int m, int mc, int t) {
  if (t >= mc * mc) return 0.0;
  const int J = t / mc, I = t - J * mc;
  return sres[(2 * J) * m + 2 * I] + sres[(2 * J + 1) * m + 2 * I + 1];
}

__device__ __forceinline__ void cc_residual(const CcCell& c, const double* z, int P, double* sres) {
  if (c.in && c.red)
    sres[c.cell] = c.r - (c.te + c.tw + c.tn + c.ts) * c.z + cc_nsum(c, z, P);
}

__device__ __forceinline__ void cc_prolong(CcCell& c, double* z, const double* zc, int m, int Pc,
                                           double omega) {
  if (c.in) {
    const int j = c.cell / m, i = c.cell - j * m;
    c.z += omega * zc[pidx(Pc, i >> 1, j >> 1)];
    z[c.f] = c.z;
  }
}

// The levels below l0 keep their cells' faces, reciprocal diagonal and
// right-hand side in LDS (six arrays of m_l^2 words per level); thread t owns
// cell t of such a level.  Same arithmetic, in the same order, as a CcCell.
struct CcLds {
  double *te, *tw, *tn, *ts, *di, *r;
};

__device__ __forceinline__ CcLds ccl_at(double* base, int n) {
  return CcLds{base, base + n, base + 2 * n, base + 3 * n, base + 4 * n, base + 5 * n};
}

template <class S>
__device__ __forceinline__ void ccl_load(const CcLds& a, const S* __restrict__ Ts,
                                         const S* __restrict__ tbs, int m, int t) {
  const int n = m * m;
  if (t >= n) return;
  const int j = t / m, i = t - j * m;
  const double te = (double)ldv(Ts, t), tn = (double)ldv(Ts, n + t);
  const double tw = (double)(i > 0 ? ldv(Ts, t - 1) : ldv(tbs, j));
  const double ts = (double)(j > 0 ? ldv(Ts, n + t - m) : ldv(tbs, m + i));
  a.te[t] = te;
  a.tw[t] = tw;
  a.tn[t] = tn;
  a.ts[t] = ts;
  a.di[t] = 1.0 / (te + tw + tn + ts);
  a.r[t] = 0.0;
}

__device__ __forceinline__ double ccl_nsum(const CcLds& a, const double* z, int t, int f, int P) {
  return a.te[t] * z[f + 1] + a.tw[t] * z[f - 1] + a.tn[t] * z[f + P] + a.ts[t] * z[f - P];
}

__device__ __forceinline__ void ccl_smooth(const CcLds& a, double* z, int m, int t, bool red,
                                           bool zero) {
  if (t < m * m) {
    const int j = t / m, i = t - j * m;
    if ((((i + j) & 1) == 0) == red) {
      const int P = m + 2, f = pidx(P, i, j);
      z[f] = zero ? a.r[t] * a.di[t] : (a.r[t] + ccl_nsum(a, z, t, f, P)) * a.di[t];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void ccl_residual(const CcLds& a, const double* z, int m, int t,
                                             double* sres) {
  if (t < m * m) {
    const int j = t / m, i = t - j * m;
    if (((i + j) & 1) == 0) {
      const int P = m + 2, f = pidx(P, i, j);
      sres[t] = a.r[t] - (a.te[t] + a.tw[t] + a.tn[t] + a.ts[t]) * z[f] + ccl_nsum(a, z, t, f, P);
    }
  }
}

__device__ __forceinline__ void ccl_prolong(double* z, const double* zc, int m, int Pc, int t,
                                            double omega) {
  if (t < m * m) {
    const int j = t / m, i = t - j * m;
    z[pidx(m + 2, i, j)] += omega * zc[pidx(Pc, i >> 1, j >> 1)];
  }
}

// W0: level l0 takes two coarse visits (W), the levels below one (V).
template <class S, bool TOP, int NL, bool W0>
__global__ void __launch_bounds__(kCcThreads)
k_mg_coarse_v(CoarseDesc desc, const VecT<S, TOP>* __restrict__ r0, VecT<S, TOP>* __restrict__ z0,
              const double* __restrict__ Ainv, double omega, const int32_t* __restrict__ active,
              double* __restrict__ rz_partial) {
  extern __shared__ double lds[];
  const int s = blockIdx.x;
  if (!active[s]) return;
  const int t = threadIdx.x;
  int zoff[NL + 1];
  int off = 0;
#pragma unroll
  for (int l = 0; l <= NL; ++l) {
    zoff[l] = off;
    off += (desc.m[l] + 2) * (desc.m[l] + 2);
  }
  double* sres = lds + off;                        // m0^2 residuals of the level being restricted
  double* vec = sres + desc.m[0] * desc.m[0];      // coarsest right-hand side
  CcLds cl[NL > 1 ? NL - 1 : 1];                   // levels 1 .. NL - 1, after vec
  const int nLc = desc.m[NL] * desc.m[NL];
  // the coarsest inverse is staged in LDS when it is small (<= kCcLdsInv
  // unknowns): its global loads then overlap the set-up instead of lying on
  // the cycle's critical path at every visit
  const double* Ag = Ainv + (long long)s * nLc * nLc;
  const double* A = Ag;
  {
    double* p = vec + nLc;
#pragma unroll
    for (int l = 1; l < NL; ++l) {
      cl[l - 1] = ccl_at(p, desc.m[l] * desc.m[l]);
      p += 6 * desc.m[l] * desc.m[l];
    }
    if (nLc <= kCcLdsInv) {
      for (int q = t; q < nLc * nLc; q += kCcThreads) p[q] = Ag[q];
      A = p;
    }
  }
  for (int q = t; q < off; q += kCcThreads) lds[q] = 0.0;
  // level l0: two slots per thread, in registers
  CcCell c0[2];
  const int m0 = desc.m[0];
  const long long n0 = (long long)m0 * m0;
  {
    const S* Ts = static_cast<const S*>(desc.T[0]) + (long long)s * 2 * n0;
    const S* tbs = static_cast<const S*>(desc.tb[0]) + (long long)s * 2 * m0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      cc_load(c0[k], Ts, tbs, m0, t + k * kCcThreads);
      const double rr = (double)ldv(r0, (long long)s * n0 + c0[k].cell);
      c0[k].r = c0[k].in ? rr : 0.0;
    }
  }
#pragma unroll
  for (int l = 1; l < NL; ++l) {
    const int m = desc.m[l];
    const long long n = (long long)m * m;
    ccl_load(cl[l - 1], static_cast<const S*>(desc.T[l]) + (long long)s * 2 * n,
             static_cast<const S*>(desc.tb[l]) + (long long)s * 2 * m, m, t);
  }
  __syncthreads();
  const int mL = desc.m[NL], nL = mL * mL;
  if (NL == 0) {
    // the coarsest level is level l0: dense inverse only
    for (int q = t; q < nL; q += kCcThreads) vec[q] = (double)ldv(r0, (long long)s * nL + q);
    __syncthreads();
    double acc = 0.0;
    if (t < nL) {
      for (int p = 0; p < nL; ++p) acc += A[t * nL + p] * vec[p];
      Prec<VecT<S, TOP>>::st(z0, (long long)s * nL + t, acc);
      acc *= vec[t];
    }
    if (TOP && rz_partial) {
      __shared__ double red[kCcThreads / kWave];
      acc = wave_sum(acc);
      if ((t & (kWave - 1)) == 0) red[t / kWave] = acc;
      __syncthreads();
      if (t == 0) {
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < kCcThreads / kWave; ++w) sum += red[w];
        rz_partial[s] = sum;
      }
    }
    return;
  }
  // right-hand side of level 1 (or of the coarsest) from the red residuals in sres
  auto hand_down = [&](int l) {
    const double rc = cc_gather(sres, desc.m[l], desc.m[l + 1], t);
    if (l + 1 < NL) {
#pragma unroll
      for (int q = 1; q < NL; ++q)
        if (q == l + 1 && t < desc.m[q] * desc.m[q]) cl[q - 1].r[t] = rc;
    } else if (t < nL) {
      vec[t] = rc;
    }
    __syncthreads();
  };
  // ---- level l0 pre-smoothing: red from zero, black, residual
  {
    double* z = lds + zoff[0];
    const int P = m0 + 2;
    cc_smooth<2>(c0, z, P, true, true);
    cc_smooth<2>(c0, z, P, false, false);
    cc_residual(c0[0], z, P, sres);
    cc_residual(c0[1], z, P, sres);
    __syncthreads();
    hand_down(0);
  }
  for (int visit = 0; visit < (W0 ? 2 : 1); ++visit) {
    if (visit > 0) {
      // second visit: pre-smoothing from the current z (its red sweep would
      // repeat the last one, so only black), residual
      double* z = lds + zoff[0];
      const int P = m0 + 2;
      cc_smooth<2>(c0, z, P, false, false);
      cc_residual(c0[0], z, P, sres);
      cc_residual(c0[1], z, P, sres);
      __syncthreads();
      hand_down(0);
    }
    // ---- V-cycle on levels 1 .. NL - 1 from z = 0
#pragma unroll
    for (int l = 1; l < NL; ++l) {
      const int m = desc.m[l];
      double* z = lds + zoff[l];
      const CcLds& c = cl[l - 1];
      ccl_smooth(c, z, m, t, true, true);
      ccl_smooth(c, z, m, t, false, false);
      ccl_residual(c, z, m, t, sres);
      __syncthreads();
      hand_down(l);
    }
    // ---- coarsest level: dense inverse
    {
      double* z = lds + zoff[NL];
      if (t < nL) {
        double acc = 0.0;
        for (int p = 0; p < nL; ++p) acc += A[t * nL + p] * vec[p];
        z[pidx(mL + 2, t % mL, t / mL)] = acc;
      }
      __syncthreads();
    }
#pragma unroll
    for (int l = NL - 1; l >= 1; --l) {
      const int m = desc.m[l], Pc = desc.m[l + 1] + 2;
      double* z = lds + zoff[l];
      const CcLds& c = cl[l - 1];
      ccl_prolong(z, lds + zoff[l + 1], m, Pc, t, omega);
      __syncthreads();
      ccl_smooth(c, z, m, t, false, false);
      ccl_smooth(c, z, m, t, true, false);
    }
    // ---- level l0: correction and post-smoothing (black, red)
    {
      double* z = lds + zoff[0];
      const int P = m0 + 2, Pc = desc.m[1] + 2;
      cc_prolong(c0[0], z, lds + zoff[1], m0, Pc, omega);
      cc_prolong(c0[1], z, lds + zoff[1], m0, Pc, omega);
      __syncthreads();
      cc_smooth<2>(c0, z, P, false, false);
      cc_smooth<2>(c0, z, P, true, false);
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k)
    if (c0[k].in) {
      Prec<VecT<S, TOP>>::st(z0, (long long)s * n0 + c0[k].cell, c0[k].z);
      acc += c0[k].r * c0[k].z;
    }
  if (TOP && rz_partial) {
    __shared__ double red[kCcThreads / kWave];
    acc = wave_sum(acc);
    if ((t & (kWave - 1)) == 0) red[t / kWave] = acc;
    __syncthreads();
    if (t == 0) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < kCcThreads / kWave; ++w) sum += red[w];
      rz_partial[s] = sum;
    }
  }
}

// ------------------------------------------------------------------ conversions
template <class S>
__global__ void k_convert(long long count, const double* __restrict__ x, S* __restrict__ y) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < count) Prec<S>::st(y, g, (typename Prec<S>::C)x[g]);
}

// ------------------------------------------------------------------ launchers
// Largest even divisor of m that is <= cap.
static int tile_dim(int m, int cap) {
  for (int t = cap < m ? cap : m; t >= 2; --t)
    if (m % t == 0 && (t % 2) == 0) return t;
  return 2;
}

template <class C>
static size_t frame_bytes(int tx, int ty) {
  return (size_t)4 * (tx + 5) * (ty + 5) * sizeof(C);
}

static bool fixed_tile(int m) { return m % kTileX == 0 && m % kTileY == 0; }

// Tile shapes of the colour-split kernels: the fastest of the shapes measured
// per kernel and hierarchy precision on the 512 x 512 level with 64 samples
// (FP64: down 64 x 32 on 768 threads, mid 64 x 32 on 768, up 128 x 16 on 768
// where 128 divides m, else 64 x 16 on 384; FP32 and bfloat16: down and up
// 64 x 32 on 640 threads, mid 64 x 64 on 1024).  Every shape divides each m
// that is a multiple of 64 (fixed_tile), except up's 128 x 16.
// shape = 1 selects an alternative set for the autotuner to try (FP64: down
// and up 64 x 16 on 384 threads, mid 64 x 64 on 1024; FP32 and bfloat16: down
// and up 64 x 16 on 704, mid 64 x 32 on 768).
static bool up_wide(int m) { return m % 128 == 0; }

int mg_rz_parts(int m, int prec, int shape) {
  if (fixed_tile(m)) {
    if (shape == 1) return (m / 64) * (m / 16);
    if (prec == MLMC_PREC_FP64) return up_wide(m) ? (m / 128) * (m / 16) : (m / 64) * (m / 16);
    return (m / 64) * (m / 32);
  }
  const int tx = tile_dim(m, kTileX), ty = tile_dim(m, kTileY);
  return (m / tx) * (m / ty);
}

int cg_dir_parts(int m) { return (m / kTileX) * (m / kTileY); }

template <int TX, int TY, int NT, class S, bool TOP>
static void down_p(hipStream_t st, int m, int batch, const void* T, const void* tb, const void* r,
                   void* z, void* rc, const int32_t* active) {
  using R = VecT<S, TOP>;
  launch_k((k_mg_down_p<TX, TY, NT, S, TOP>), dim3(batch * (m / TX) * (m / TY)),
                     dim3(NT), 0, st, m, (const S*)T, (const S*)tb, (const R*)r, (S*)z, (S*)rc,
                     active);
}

template <int TX, int TY, int NT, class S, bool TOP>
static void up_p(hipStream_t st, int m, int batch, const void* T, const void* tb, const void* r,
                 const void* zpre, void* z, const void* zc, double omega, const int32_t* active,
                 double* rz_partial) {
  using R = VecT<S, TOP>;
  launch_k((k_mg_up_p<TX, TY, NT, S, TOP>), dim3(batch * (m / TX) * (m / TY)), dim3(NT),
                     0, st, m, (const S*)T, (const S*)tb, (const R*)r, (const S*)zpre, (R*)z,
                     (const S*)zc, omega, active, rz_partial);
}

template <int TX, int TY, int NT, class S, bool TOP>
static void mid_p(hipStream_t st, int m, int batch, const void* T, const void* tb, const void* r,
                  const void* zpre, void* z, const void* zc, double omega, void* rc,
                  const int32_t* active) {
  using R = VecT<S, TOP>;
  launch_k((k_mg_mid_p<TX, TY, NT, S, TOP>), dim3(batch * (m / TX) * (m / TY)),
                     dim3(NT), 0, st, m, (const S*)T, (const S*)tb, (const R*)r, (const S*)zpre,
                     (S*)z, (const S*)zc, omega, (S*)rc, active);
}

template <class S, bool TOP>
static void down_impl(int shape, hipStream_t st, int m, int batch, const void* T, const void* tb,
                      const void* r, void* z, void* rc, const int32_t* active) {
  using R = VecT<S, TOP>;
  if (fixed_tile(m)) {
    if (shape == 1) {
      if constexpr (std::is_same<S, double>::value)
        down_p<64, 16, 384, S, TOP>(st, m, batch, T, tb, r, z, rc, active);
      else down_p<64, 16, 704, S, TOP>(st, m, batch, T, tb, r, z, rc, active);
    } else if constexpr (std::is_same<S, double>::value)
      down_p<64, 32, 768, S, TOP>(st, m, batch, T, tb, r, z, rc, active);
    else down_p<64, 32, 640, S, TOP>(st, m, batch, T, tb, r, z, rc, active);
    return;
  }
  using C = typename Prec<S>::C;
  const int tx = tile_dim(m, kTileX), ty = tile_dim(m, kTileY);
  const int tps = (m / tx) * (m / ty);
  launch_k((k_mg_down<S, TOP>), dim3(batch * tps), dim3(kBlock), frame_bytes<C>(tx, ty),
                     st, m, tx, ty, tps, (const S*)T, (const S*)tb, (const R*)r, (S*)z, (S*)rc,
                     active);
}

template <class S, bool TOP>
static void up_impl(int shape, hipStream_t st, int m, int batch, const void* T, const void* tb,
                    const void* r, const void* zpre, void* z, const void* zc, double omega,
                    const int32_t* active, double* rz_partial) {
  using R = VecT<S, TOP>;
  if (fixed_tile(m)) {
    if (shape == 1) {
      if constexpr (std::is_same<S, double>::value)
        up_p<64, 16, 384, S, TOP>(st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
      else up_p<64, 16, 704, S, TOP>(st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
    } else if constexpr (!std::is_same<S, double>::value)
      up_p<64, 32, 640, S, TOP>(st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
    else if (up_wide(m))
      up_p<128, 16, 768, S, TOP>(st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
    else up_p<64, 16, 384, S, TOP>(st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
    return;
  }
  using C = typename Prec<S>::C;
  const int tx = tile_dim(m, kTileX), ty = tile_dim(m, kTileY);
  const int tps = (m / tx) * (m / ty);
  launch_k((k_mg_up<S, TOP>), dim3(batch * tps), dim3(kBlock), frame_bytes<C>(tx, ty), st,
                     m, tx, ty, tps, (const S*)T, (const S*)tb, (const R*)r, (const S*)zpre, (R*)z,
                     (const S*)zc, omega, active, rz_partial);
}

template <class S, bool TOP>
static void mid_impl(int shape, hipStream_t st, int m, int batch, const void* T, const void* tb,
                     const void* r, const void* zpre, void* z, const void* zc, double omega,
                     void* rc, const int32_t* active) {
  using R = VecT<S, TOP>;
  if (fixed_tile(m)) {
    if (shape == 1) {
      if constexpr (std::is_same<S, double>::value)
        mid_p<64, 64, 1024, S, TOP>(st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
      else mid_p<64, 32, 768, S, TOP>(st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
    } else if constexpr (std::is_same<S, double>::value)
      mid_p<64, 32, 768, S, TOP>(st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
    else mid_p<64, 64, 1024, S, TOP>(st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
    return;
  }
  using C = typename Prec<S>::C;
  const int tx = tile_dim(m, kTileX), ty = tile_dim(m, kTileY);
  const int tps = (m / tx) * (m / ty);
  const size_t lds = (size_t)4 * (tx + 8) * (ty + 8) * sizeof(C);
  launch_k((k_mg_mid<S, TOP>), dim3(batch * tps), dim3(kBlock), lds, st, m, tx, ty, tps,
                     (const S*)T, (const S*)tb, (const R*)r, (const S*)zpre, (S*)z, (const S*)zc,
                     omega, (S*)rc, active);
}

template <class S>
static void mid_any(int shape, bool top, hipStream_t st, int m, int batch, const void* T,
                    const void* tb, const void* r, const void* zpre, void* z, const void* zc,
                    double omega, void* rc, const int32_t* active) {
  if (top) mid_impl<S, true>(shape, st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
  else mid_impl<S, false>(shape, st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
}

void launch_mg_mid(hipStream_t st, int prec, int shape, bool top, int m, int batch, const void* T,
                   const void* tb, const void* r, const void* zpre, void* z, const void* zc,
                   double omega, void* rc, const int32_t* active) {
  if (prec == MLMC_PREC_FP64)
    mid_any<double>(shape, top, st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
  else if (prec == MLMC_PREC_FP32)
    mid_any<float>(shape, top, st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
  else mid_any<bf16_t>(shape, top, st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
}

template <class S>
static void down_any(int shape, bool top, hipStream_t st, int m, int batch, const void* T,
                     const void* tb, const void* r, void* z, void* rc, const int32_t* active) {
  if (top) down_impl<S, true>(shape, st, m, batch, T, tb, r, z, rc, active);
  else down_impl<S, false>(shape, st, m, batch, T, tb, r, z, rc, active);
}

template <class S>
static void up_any(int shape, bool top, hipStream_t st, int m, int batch, const void* T,
                   const void* tb, const void* r, const void* zpre, void* z, const void* zc,
                   double omega, const int32_t* active, double* rz_partial) {
  if (top) up_impl<S, true>(shape, st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
  else up_impl<S, false>(shape, st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
}

template <class S, bool TOP, int NL, bool W0>
static void coarse_v_impl(hipStream_t st, int batch, const CoarseDesc& desc, const void* r0,
                          void* z0, const double* Ainv, double omega, const int32_t* active,
                          double* rz_partial) {
  using R = VecT<S, TOP>;
  size_t words = 0;
  for (int l = 0; l <= NL; ++l) words += (size_t)(desc.m[l] + 2) * (desc.m[l] + 2);
  words += (size_t)desc.m[0] * desc.m[0] + (size_t)desc.m[NL] * desc.m[NL];
  for (int l = 1; l < NL; ++l) words += 6 * (size_t)desc.m[l] * desc.m[l];
  const size_t nLc = (size_t)desc.m[NL] * desc.m[NL];
  if (nLc <= (size_t)kCcLdsInv) words += nLc * nLc;
  hipLaunchKernelGGL((k_mg_coarse_v<S, TOP, NL, W0>), dim3(batch), dim3(kCcThreads),
                     words * sizeof(double), st, desc, (const R*)r0, (R*)z0, Ainv, omega, active,
                     rz_partial);
}

template <class S, bool TOP, bool W0>
static void coarse_v_nl(hipStream_t st, int batch, int nlev, const CoarseDesc& desc,
                        const void* r0, void* z0, const double* Ainv, double omega,
                        const int32_t* active, double* rz_partial) {
#define CCV(NL) coarse_v_impl<S, TOP, NL, W0>(st, batch, desc, r0, z0, Ainv, omega, active, rz_partial)
  switch (nlev - 1) {
    case 0: CCV(0); break;
    case 1: CCV(1); break;
    case 2: CCV(2); break;
    case 3: CCV(3); break;
    case 4: CCV(4); break;
    default: CCV(5); break;
  }
#undef CCV
}

template <class S, bool TOP>
static void coarse_v_any(hipStream_t st, int batch, int nlev, const CoarseDesc& desc,
                         const void* r0, void* z0, const double* Ainv, double omega, bool w0,
                         const int32_t* active, double* rz_partial) {
  if (w0) coarse_v_nl<S, TOP, true>(st, batch, nlev, desc, r0, z0, Ainv, omega, active, rz_partial);
  else coarse_v_nl<S, TOP, false>(st, batch, nlev, desc, r0, z0, Ainv, omega, active, rz_partial);
}

template <class S>
static void coarse_any(bool top, hipStream_t st, int batch, int nlev, const CoarseDesc& desc,
                       const void* r0, void* z0, const double* Ainv, double omega, unsigned wmask,
                       const int32_t* active, double* rz_partial) {
  if ((wmask & ~1u) == 0 && nlev - 1 <= kCcMaxSmooth && desc.m[0] <= 32) {
    const bool w0 = (wmask & 1u) && nlev > 1;
    if (top)
      coarse_v_any<S, true>(st, batch, nlev, desc, r0, z0, Ainv, omega, w0, active, rz_partial);
    else
      coarse_v_any<S, false>(st, batch, nlev, desc, r0, z0, Ainv, omega, w0, active, rz_partial);
    return;
  }
  const size_t lds = coarse_cycle_lds_bytes(desc, nlev);
  if (top)
    hipLaunchKernelGGL((k_mg_coarse_cycle<S, true>), dim3(batch), dim3(kBlock), lds, st, nlev, desc,
                       (const double*)r0, (double*)z0, Ainv, omega, wmask, active, rz_partial);
  else
    hipLaunchKernelGGL((k_mg_coarse_cycle<S, false>), dim3(batch), dim3(kBlock), lds, st, nlev,
                       desc, (const S*)r0, (S*)z0, Ainv, omega, wmask, active, rz_partial);
}

template <class S>
static void convert_any(hipStream_t st, long long count, const double* x, void* y) {
  hipLaunchKernelGGL((k_convert<S>), dim3(blocks_for(count)), dim3(kBlock), 0, st, count, x,
                     (S*)y);
}

void launch_mg_down(hipStream_t st, int prec, int shape, bool top, int m, int batch,
                    const void* T, const void* tb, const void* r, void* z, void* rc,
                    const int32_t* active) {
  if (prec == MLMC_PREC_FP64) down_any<double>(shape, top, st, m, batch, T, tb, r, z, rc, active);
  else if (prec == MLMC_PREC_FP32) down_any<float>(shape, top, st, m, batch, T, tb, r, z, rc, active);
  else down_any<bf16_t>(shape, top, st, m, batch, T, tb, r, z, rc, active);
}

void launch_mg_up(hipStream_t st, int prec, int shape, bool top, int m, int batch, const void* T,
                  const void* tb, const void* r, const void* zpre, void* z, const void* zc,
                  double omega, const int32_t* active, double* rz_partial) {
  if (prec == MLMC_PREC_FP64)
    up_any<double>(shape, top, st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
  else if (prec == MLMC_PREC_FP32)
    up_any<float>(shape, top, st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
  else up_any<bf16_t>(shape, top, st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
}

size_t coarse_cycle_lds_bytes(const CoarseDesc& d, int nlev) {
  size_t words = 0;
  for (int l = 0; l < nlev; ++l) words += 4 * (size_t)(d.m[l] + 2) * (d.m[l] + 2);
  words += (size_t)d.m[nlev - 1] * d.m[nlev - 1];
  return words * sizeof(double);
}

void launch_mg_coarse_cycle(hipStream_t st, int prec, bool top, int batch, int nlev,
                            const CoarseDesc& desc, const void* r0, void* z0, const double* Ainv,
                            double omega, unsigned wmask, const int32_t* active,
                            double* rz_partial) {
  if (prec == MLMC_PREC_FP64)
    coarse_any<double>(top, st, batch, nlev, desc, r0, z0, Ainv, omega, wmask, active, rz_partial);
  else if (prec == MLMC_PREC_FP32)
    coarse_any<float>(top, st, batch, nlev, desc, r0, z0, Ainv, omega, wmask, active, rz_partial);
  else
    coarse_any<bf16_t>(top, st, batch, nlev, desc, r0, z0, Ainv, omega, wmask, active, rz_partial);
}

void launch_convert(hipStream_t st, int prec, long long count, const double* x, void* y) {
  if (prec == MLMC_PREC_FP64) convert_any<double>(st, count, x, y);
  else if (prec == MLMC_PREC_FP32) convert_any<float>(st, count, x, y);
  else convert_any<bf16_t>(st, count, x, y);
}

bool cg_direction_fused(int m) { return fixed_tile(m); }

void launch_cg_direction(hipStream_t st, int m, int batch, const double* T, const double* tb,
                         const double* z, const double* pold, double* pnew, double* q,
                         const double* beta, int first, double* partial, const int32_t* active) {
  const int nb = batch * (m / kTileX) * (m / kTileY);
  launch_k((k_cg_direction_t<kTileX, kTileY>), dim3(nb), dim3(kMgThreads), 0, st, m, T,
                     tb, z, pold, pnew, q, beta, first, partial, active);
}

size_t prec_bytes(int prec) {
  return prec == MLMC_PREC_FP64 ? 8 : (prec == MLMC_PREC_FP32 ? 4 : 2);
}

}  // namespace mlmc
