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

// ------------------------------------------------------------------ fixed-tile kernels
// Tiles of compile-time size TX x TY (used when TX and TY divide m).  Each of
// the 512 threads owns the frame cells f = tid + 512 k in every phase and
// keeps their four faces, reciprocal diagonal, right-hand side and z in
// registers; LDS holds z, which is what neighbours read, and the residuals the
// restriction sums.  All loads use clamped, always-valid addresses and are
// resolved by selects, so a thread's loads are issued back to back.  Tiles of
// one sample run on one XCD, so the halo re-reads hit that XCD's L2.  The
// down/up frame reaches two cells around the tile ((TX + 4) x (TY + 4)), the
// mid frame four.
constexpr int kMgThreads = 512;
// The mid kernel's frame reaches four cells around the tile: a taller tile
// (64 x 32, 1.41x halo overhead instead of 1.69x) on 1024 threads, measured
// 6% (FP64) and 15% (FP32) faster than 64 x 16 on 512 threads.
constexpr int kMidThreads = 1024;
constexpr int kMidTileY = 32;

template <int TX, int TY, int HALO>
struct Tile {
  static constexpr int W = TX + 2 * HALO, H = TY + 2 * HALO, F = W * H;
  static constexpr int K = (F + kMgThreads - 1) / kMgThreads;
};

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

// down: pre-smoothing from z = 0 (red, then black) and the restricted residual.
template <int TX, int TY, class S, bool TOP>
__global__ void __launch_bounds__(kMgThreads, 8)
k_mg_down_t(int m, const S* __restrict__ T, const S* __restrict__ tb,
            const VecT<S, TOP>* __restrict__ r, S* __restrict__ z, S* __restrict__ rc,
            const int32_t* __restrict__ active) {
  using C = typename Prec<S>::C;
  using G = Tile<TX, TY, 2>;
  constexpr int W = G::W, H = G::H, F = G::F, K = G::K;
  __shared__ C sz[F];
  __shared__ C sres[F];
  const int ntx = m / TX, tps = ntx * (m / TY);
  const int bid = xcd_tile(blockIdx.x, gridDim.x);
  const long long s = bid / tps;
  if (!active[s]) return;
  const int tile = bid - (int)(s * tps);
  const int X0 = (tile % ntx) * TX, Y0 = (tile / ntx) * TY;
  const long long n = (long long)m * m;
  const S* Ts = T + s * 2 * n;
  const S* tbs = tb + s * 2 * m;
  const VecT<S, TOP>* rs = r + s * n;
  // z lives in LDS only; flags per slot: bit 0 a frame cell inside the domain,
  // bit 1 inside the ring of the black sweep, bit 4 black, bit 5 on the tile.
  CellFaces<C> cf[K];
  C rv[K], di[K];
  unsigned fl[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    cf[k] = own_faces(Ts, m, X0 - 2 + fi, Y0 - 2 + fj);
    const C rr = (C)ldv(rs, cf[k].c);
    rv[k] = cf[k].in ? rr : C(0);
    if (f < F) {
      sz[f] = cf[k].te;
      sres[f] = cf[k].tn;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    adjacent_faces(cf[k], sz, sres, Ts, tbs, m, X0 - 2 + fi, Y0 - 2 + fj, f, fi, fj, W, f < F);
    di[k] = inv_diag(cf[k]);
    unsigned b = (f < F && cf[k].in) ? 1u : 0u;
    if (fi >= 1 && fi < W - 1 && fj >= 1 && fj < H - 1) b |= 2u;
    if ((fi + fj) & 1) b |= 16u;
    if (fi >= 2 && fi < 2 + TX && fj >= 2 && fj < 2 + TY) b |= 32u;
    fl[k] = b;
  }
  __syncthreads();
  // red cells of the frame: z = r / D; black cells start at 0
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    if (f < F) sz[f] = (fl[k] & 16u) ? C(0) : rv[k] * di[k];
  }
  __syncthreads();
  // black cells of R1
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    if ((fl[k] & 19u) == 19u) sz[f] = (rv[k] + nsum_lds(cf[k], sz, f, W)) * di[k];
  }
  __syncthreads();
  // store the tile; residual of its red cells (black residuals vanish)
  S* zs = z + s * n;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    if (fl[k] & 32u) {
      const int fj = f / W, fi = f - fj * W;
      Prec<S>::st(zs, (long long)(Y0 - 2 + fj) * m + (X0 - 2 + fi), sz[f]);
      if (!(fl[k] & 16u)) sres[f] = nsum_lds(cf[k], sz, f, W);
    }
  }
  __syncthreads();
  const int mc = m / 2;
  S* rcs = rc + s * (long long)mc * mc;
  constexpr int HX = TX / 2, HY = TY / 2;
  for (int c = threadIdx.x; c < HX * HY; c += kMgThreads) {
    const int cj = c / HX, ci = c - cj * HX;
    // (X0 + 2ci, Y0 + 2cj) has even i + j: the block's red cells are (0,0) and (1,1)
    const int fa = (2 + 2 * cj) * W + 2 + 2 * ci;
    Prec<S>::st(rcs, (Y0 / 2 + cj) * mc + X0 / 2 + ci, sres[fa] + sres[fa + W + 1]);
  }
}

// mid: the second coarse correction of a W-cycle level.  From z1 (the down
// result) and the first correction e1: z = z1 + omega P e1, then black, red
// and black sweeps (the post-smoothing of the first correction, black then
// red, followed by the pre-smoothing of the second, red then black, whose red
// sweep repeats the one just done and is dropped), then the restricted
// residual as in down.  Halo: the residual on the tile needs the last black
// sweep one cell out, that sweep the red sweep two cells out, that one the
// first black sweep three cells out, which needs z four cells out.
template <int TX, int TY, class S, bool TOP>
__global__ void __launch_bounds__(kMidThreads, 8)
k_mg_mid_t(int m, const S* __restrict__ T, const S* __restrict__ tb,
           const VecT<S, TOP>* __restrict__ r, const S* __restrict__ zpre, S* __restrict__ z,
           const S* __restrict__ zc, double omega, S* __restrict__ rc,
           const int32_t* __restrict__ active) {
  using C = typename Prec<S>::C;
  using G = Tile<TX, TY, 4>;
  constexpr int W = G::W, H = G::H, F = G::F, K = (F + kMidThreads - 1) / kMidThreads;
  __shared__ C sz[F];
  __shared__ C sres[F];
  __shared__ C ste[F];
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
  // z of the frame lives in LDS only (sz, written as soon as it is loaded; the
  // east / north faces are exchanged through ste / sres); registers hold each
  // cell's faces, reciprocal diagonal and right-hand side, which keeps the
  // kernel within 64 VGPRs: two workgroups per CU, so one's loads overlap the
  // other's sweeps.
  // Per slot, one byte of flags (byte k of fl for slot k): bit 0 a frame cell
  // inside the domain, bits 1-3 inside the rings swept by the three passes (R3,
  // R2, R1), bit 4 black, bit 5 on the tile.
  CellFaces<C> cf[K];
  C rv[K], di[K];
  static_assert(K <= 4, "one flag byte per slot");
  unsigned fl = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMidThreads;
    const int fj = f / W, fi = f - fj * W;
    const int i = X0 - 4 + fi, j = Y0 - 4 + fj;
    cf[k] = own_faces(Ts, m, i, j);
    const int ic = min(max(i, 0), m - 1), jc = min(max(j, 0), m - 1);
    const C rr = (C)ldo(r + s * n, (unsigned)cf[k].c);
    const C zp = ldo(zps, (unsigned)cf[k].c), zcv = ldo(zcs, (unsigned)((jc >> 1) * mc + (ic >> 1)));
    rv[k] = cf[k].in ? rr : C(0);
    if (f < F) {
      sz[f] = cf[k].in ? zp + om * zcv : C(0);
      ste[f] = cf[k].te;
      sres[f] = cf[k].tn;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMidThreads;
    const int fj = f / W, fi = f - fj * W;
    adjacent_faces(cf[k], ste, sres, Ts, tbs, m, X0 - 4 + fi, Y0 - 4 + fj, f, fi, fj, W, f < F);
    di[k] = inv_diag(cf[k]);
    unsigned b = (f < F && cf[k].in) ? 1u : 0u;
#pragma unroll
    for (int d = 3; d >= 1; --d)
      if (fi >= 4 - d && fi < W - 4 + d && fj >= 4 - d && fj < H - 4 + d) b |= 2u << (3 - d);
    if ((fi + fj) & 1) b |= 16u;
    if (fi >= 4 && fi < 4 + TX && fj >= 4 && fj < 4 + TY) b |= 32u;
    fl |= b << (8 * k);
  }
  __syncthreads();
  // black on R3, red on R2, black on R1
#pragma unroll
  for (int pass = 0; pass < 3; ++pass) {
    const unsigned want = 1u | (2u << pass) | (pass == 1 ? 0u : 16u);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int f = threadIdx.x + k * kMidThreads;
      if (((fl >> (8 * k)) & (17u | (2u << pass))) == want)
        sz[f] = (rv[k] + nsum_lds(cf[k], sz, f, W)) * di[k];
    }
    __syncthreads();
  }
  // store the tile; residual of its red cells (black residuals vanish after the black sweep)
  S* zs = z + s * n;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int f = threadIdx.x + k * kMidThreads;
    // recomputed here rather than kept from the start (an empty asm makes the
    // index opaque), which keeps the kernel within 64 VGPRs without a spill
    asm volatile("" : "+v"(f));
    if ((fl >> (8 * k)) & 32u) {
      const int fj = f / W, fi = f - fj * W;
      const C zf = sz[f];
      Prec<S>::st(zs, (long long)(Y0 - 4 + fj) * m + (X0 - 4 + fi), zf);
      if (!((fl >> (8 * k)) & 16u)) {
        const C dd = cf[k].te + cf[k].tw + cf[k].tn + cf[k].ts;
        sres[f] = rv[k] - dd * zf + nsum_lds(cf[k], sz, f, W);
      }
    }
  }
  __syncthreads();
  S* rcs = rc + s * (long long)mc * mc;
  constexpr int HX = TX / 2, HY = TY / 2;
  for (int c = threadIdx.x; c < HX * HY; c += kMidThreads) {
    const int cj = c / HX, ci = c - cj * HX;
    const int fa = (4 + 2 * cj) * W + 4 + 2 * ci;
    Prec<S>::st(rcs, (Y0 / 2 + cj) * mc + X0 / 2 + ci, sres[fa] + sres[fa + W + 1]);
  }
}

// up: z = z_in + omega P e, post-smoothing (black, then red) and, on the finest
// level, the per-tile partial of r^T z.
template <int TX, int TY, class S, bool TOP>
__global__ void __launch_bounds__(kMgThreads, 8)
k_mg_up_t(int m, const S* __restrict__ T, const S* __restrict__ tb,
          const VecT<S, TOP>* __restrict__ r, const S* __restrict__ zpre,
          VecT<S, TOP>* __restrict__ z, const S* __restrict__ zc, double omega,
          const int32_t* __restrict__ active, double* __restrict__ rz_partial) {
  using C = typename Prec<S>::C;
  using G = Tile<TX, TY, 2>;
  constexpr int W = G::W, H = G::H, F = G::F, K = G::K;
  __shared__ C sz[F];
  __shared__ C sn[F];
  __shared__ C se[F];
  __shared__ double red[kMgThreads / kWave];
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
  const VecT<S, TOP>* rs = r + s * n;
  const S* zps = zpre + s * n;
  const S* zcs = zc + s * (long long)mc * mc;
  const C om = (C)omega;
  // z lives in LDS only (written as soon as it is loaded; east / north faces
  // are exchanged through se / sn); flags per slot: bit 0 a frame cell inside
  // the domain, bit 1 inside the ring of the black sweep, bit 4 black, bit 5 on
  // the tile.
  CellFaces<C> cf[K];
  C rv[K], di[K];
  double rd[K];  // FP64 residual for the r^T z sum (finest level only)
  unsigned fl[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    const int i = X0 - 2 + fi, j = Y0 - 2 + fj;
    cf[k] = own_faces(Ts, m, i, j);
    const int ic = min(max(i, 0), m - 1), jc = min(max(j, 0), m - 1);
    const double rr = (double)ldv(rs, cf[k].c);
    const C zp = ldv(zps, cf[k].c), zcv = ldv(zcs, (jc >> 1) * mc + (ic >> 1));
    rd[k] = cf[k].in ? rr : 0.0;
    rv[k] = (C)rd[k];
    if (f < F) {
      sz[f] = cf[k].in ? zp + om * zcv : C(0);
      se[f] = cf[k].te;
      sn[f] = cf[k].tn;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    adjacent_faces(cf[k], se, sn, Ts, tbs, m, X0 - 2 + fi, Y0 - 2 + fj, f, fi, fj, W, f < F);
    di[k] = inv_diag(cf[k]);
    unsigned b = (f < F && cf[k].in) ? 1u : 0u;
    if (fi >= 1 && fi < W - 1 && fj >= 1 && fj < H - 1) b |= 2u;
    if ((fi + fj) & 1) b |= 16u;
    if (fi >= 2 && fi < 2 + TX && fj >= 2 && fj < 2 + TY) b |= 32u;
    fl[k] = b;
  }
  __syncthreads();
  // black sweep on R1
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    if ((fl[k] & 19u) == 19u) sz[f] = (rv[k] + nsum_lds(cf[k], sz, f, W)) * di[k];
  }
  __syncthreads();
  // red sweep on the tile, store, r^T z
  VecT<S, TOP>* zs = z + s * n;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    if (fl[k] & 32u) {
      const int fj = f / W, fi = f - fj * W;
      const C zf = (fl[k] & 16u) ? sz[f] : (rv[k] + nsum_lds(cf[k], sz, f, W)) * di[k];
      Prec<VecT<S, TOP>>::st(zs, (long long)(Y0 - 2 + fj) * m + (X0 - 2 + fi), zf);
      if (TOP) acc += rd[k] * (double)zf;
    }
  }
  if (TOP && rz_partial) {
    acc = wave_sum(acc);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kMgThreads / kWave; ++w) t += red[w];
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
  CoarseLevel lv[kMaxCoarseLevels];
  int off = 0;
  for (int l = 0; l < nlev; ++l) {
    lv[l].m = desc.m[l];
    lv[l].P = desc.m[l] + 2;
    lv[l].off = off;
    off += 4 * lv[l].P * lv[l].P;
  }
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

int mg_tiles_per_sample(int m) {
  if (fixed_tile(m)) return (m / kTileX) * (m / kTileY);
  const int tx = tile_dim(m, kTileX), ty = tile_dim(m, kTileY);
  return (m / tx) * (m / ty);
}

template <class S, bool TOP>
static void down_impl(hipStream_t st, int m, int batch, const void* T, const void* tb,
                      const void* r, void* z, void* rc, const int32_t* active) {
  using R = VecT<S, TOP>;
  if (fixed_tile(m)) {
    const int nb = batch * (m / kTileX) * (m / kTileY);
    hipLaunchKernelGGL((k_mg_down_t<kTileX, kTileY, S, TOP>), dim3(nb), dim3(kMgThreads), 0, st,
                       m, (const S*)T, (const S*)tb, (const R*)r, (S*)z, (S*)rc, active);
    return;
  }
  using C = typename Prec<S>::C;
  const int tx = tile_dim(m, kTileX), ty = tile_dim(m, kTileY);
  const int tps = (m / tx) * (m / ty);
  hipLaunchKernelGGL((k_mg_down<S, TOP>), dim3(batch * tps), dim3(kBlock), frame_bytes<C>(tx, ty),
                     st, m, tx, ty, tps, (const S*)T, (const S*)tb, (const R*)r, (S*)z, (S*)rc,
                     active);
}

template <class S, bool TOP>
static void up_impl(hipStream_t st, int m, int batch, const void* T, const void* tb,
                    const void* r, const void* zpre, void* z, const void* zc, double omega,
                    const int32_t* active, double* rz_partial) {
  using R = VecT<S, TOP>;
  if (fixed_tile(m)) {
    const int nb = batch * (m / kTileX) * (m / kTileY);
    hipLaunchKernelGGL((k_mg_up_t<kTileX, kTileY, S, TOP>), dim3(nb), dim3(kMgThreads), 0, st, m,
                       (const S*)T, (const S*)tb, (const R*)r, (const S*)zpre, (R*)z,
                       (const S*)zc, omega, active, rz_partial);
    return;
  }
  using C = typename Prec<S>::C;
  const int tx = tile_dim(m, kTileX), ty = tile_dim(m, kTileY);
  const int tps = (m / tx) * (m / ty);
  hipLaunchKernelGGL((k_mg_up<S, TOP>), dim3(batch * tps), dim3(kBlock), frame_bytes<C>(tx, ty), st,
                     m, tx, ty, tps, (const S*)T, (const S*)tb, (const R*)r, (const S*)zpre, (R*)z,
                     (const S*)zc, omega, active, rz_partial);
}

template <class S, bool TOP>
static void mid_impl(hipStream_t st, int m, int batch, const void* T, const void* tb, const void* r,
                     const void* zpre, void* z, const void* zc, double omega, void* rc,
                     const int32_t* active) {
  using R = VecT<S, TOP>;
  if (fixed_tile(m)) {
    const int nb = batch * (m / kTileX) * (m / kMidTileY);
    hipLaunchKernelGGL((k_mg_mid_t<kTileX, kMidTileY, S, TOP>), dim3(nb), dim3(kMidThreads), 0, st, m,
                       (const S*)T, (const S*)tb, (const R*)r, (const S*)zpre, (S*)z,
                       (const S*)zc, omega, (S*)rc, active);
    return;
  }
  using C = typename Prec<S>::C;
  const int tx = tile_dim(m, kTileX), ty = tile_dim(m, kTileY);
  const int tps = (m / tx) * (m / ty);
  const size_t lds = (size_t)4 * (tx + 8) * (ty + 8) * sizeof(C);
  hipLaunchKernelGGL((k_mg_mid<S, TOP>), dim3(batch * tps), dim3(kBlock), lds, st, m, tx, ty, tps,
                     (const S*)T, (const S*)tb, (const R*)r, (const S*)zpre, (S*)z, (const S*)zc,
                     omega, (S*)rc, active);
}

template <class S>
static void mid_any(bool top, hipStream_t st, int m, int batch, const void* T, const void* tb,
                    const void* r, const void* zpre, void* z, const void* zc, double omega,
                    void* rc, const int32_t* active) {
  if (top) mid_impl<S, true>(st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
  else mid_impl<S, false>(st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
}

void launch_mg_mid(hipStream_t st, int prec, bool top, int m, int batch, const void* T,
                   const void* tb, const void* r, const void* zpre, void* z, const void* zc,
                   double omega, void* rc, const int32_t* active) {
  if (prec == MLMC_PREC_FP64) mid_any<double>(top, st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
  else if (prec == MLMC_PREC_FP32) mid_any<float>(top, st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
  else mid_any<bf16_t>(top, st, m, batch, T, tb, r, zpre, z, zc, omega, rc, active);
}

template <class S>
static void down_any(bool top, hipStream_t st, int m, int batch, const void* T, const void* tb,
                     const void* r, void* z, void* rc, const int32_t* active) {
  if (top) down_impl<S, true>(st, m, batch, T, tb, r, z, rc, active);
  else down_impl<S, false>(st, m, batch, T, tb, r, z, rc, active);
}

template <class S>
static void up_any(bool top, hipStream_t st, int m, int batch, const void* T, const void* tb,
                   const void* r, const void* zpre, void* z, const void* zc, double omega,
                   const int32_t* active, double* rz_partial) {
  if (top) up_impl<S, true>(st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
  else up_impl<S, false>(st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
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

void launch_mg_down(hipStream_t st, int prec, bool top, int m, int batch, const void* T,
                    const void* tb, const void* r, void* z, void* rc, const int32_t* active) {
  if (prec == MLMC_PREC_FP64) down_any<double>(top, st, m, batch, T, tb, r, z, rc, active);
  else if (prec == MLMC_PREC_FP32) down_any<float>(top, st, m, batch, T, tb, r, z, rc, active);
  else down_any<bf16_t>(top, st, m, batch, T, tb, r, z, rc, active);
}

void launch_mg_up(hipStream_t st, int prec, bool top, int m, int batch, const void* T,
                  const void* tb, const void* r, const void* zpre, void* z, const void* zc,
                  double omega, const int32_t* active, double* rz_partial) {
  if (prec == MLMC_PREC_FP64)
    up_any<double>(top, st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
  else if (prec == MLMC_PREC_FP32)
    up_any<float>(top, st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
  else up_any<bf16_t>(top, st, m, batch, T, tb, r, zpre, z, zc, omega, active, rz_partial);
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
  hipLaunchKernelGGL((k_cg_direction_t<kTileX, kTileY>), dim3(nb), dim3(kMgThreads), 0, st, m, T,
                     tb, z, pold, pnew, q, beta, first, partial, active);
}

size_t prec_bytes(int prec) {
  return prec == MLMC_PREC_FP64 ? 8 : (prec == MLMC_PREC_FP32 ? 4 : 2);
}

}  // namespace mlmc
