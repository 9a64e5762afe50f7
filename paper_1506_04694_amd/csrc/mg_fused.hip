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
// Tiles are tx x ty cells (even, dividing m); the LDS frame starts three cells
// below/left of the tile and spans (tx + 5) x (ty + 5) cells.  Outside the
// domain z = 0 and faces are 0, except that the frame holds the west boundary
// face in column i = -1 and the south boundary face in row j = -1, so every
// cell's diagonal is Te(i) + Te(i-1) + Tn(j) + Tn(j-1) without branches.
//
// Levels of 32 x 32 cells or fewer are handled by k_mg_coarse_cycle: one
// workgroup per sample runs the remaining V-cycle entirely in LDS and applies
// the coarsest inverse (a dense matrix-vector product).
#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

namespace mlmc {

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
__device__ __forceinline__ double load_te(const double* Ts, const double* tbs, int m, int i,
                                          int j) {
  if (j < 0 || j >= m) return 0.0;
  if (i == -1) return tbs[j];
  if (i < 0 || i >= m) return 0.0;
  return Ts[j * m + i];
}

__device__ __forceinline__ double load_tn(const double* Ts, const double* tbs, int m, int i,
                                          int j) {
  if (i < 0 || i >= m) return 0.0;
  if (j == -1) return tbs[m + i];
  if (j < 0 || j >= m) return 0.0;
  return Ts[m * m + j * m + i];
}

struct Lds {
  double* te;
  double* tn;
  double* r;
  double* z;
};

__device__ __forceinline__ double diag_at(const Lds& s, int W, int f) {
  return s.te[f] + s.te[f - 1] + s.tn[f] + s.tn[f - W];
}

__device__ __forceinline__ double nsum_at(const Lds& s, int W, int f) {
  return s.te[f] * s.z[f + 1] + s.te[f - 1] * s.z[f - 1] + s.tn[f] * s.z[f + W] +
         s.tn[f - W] * s.z[f - W];
}

// ------------------------------------------------------------------ down
__global__ void __launch_bounds__(kBlock)
k_mg_down(int m, int tx, int ty, int tiles_per_sample, const double* __restrict__ T,
          const double* __restrict__ tb, const double* __restrict__ r, double* __restrict__ z,
          double* __restrict__ rc, const int32_t* __restrict__ active) {
  extern __shared__ double lds[];
  const long long s = blockIdx.x / tiles_per_sample;
  if (!active[s]) return;
  const FrameGeom g = frame_of(m, tx, ty, blockIdx.x - (int)(s * tiles_per_sample));
  const int W = g.W, H = g.H, F = W * H;
  Lds L{lds, lds + F, lds + 2 * F, lds + 3 * F};
  const long long n = (long long)m * m;
  const double* Ts = T + s * 2 * n;
  const double* tbs = tb + s * 2 * m;
  const double* rs = r + s * n;
  for (int f = threadIdx.x; f < F; f += kBlock) {
    const int fj = f / W, fi = f - fj * W;
    const int i = g.gi(fi), j = g.gj(fj);
    L.te[f] = load_te(Ts, tbs, m, i, j);
    L.tn[f] = load_tn(Ts, tbs, m, i, j);
    L.r[f] = g.inside(i, j) ? rs[j * m + i] : 0.0;
  }
  __syncthreads();
  // red cells of R2 (frame [1, W) x [1, H)): z = r / D; everything else 0
  for (int f = threadIdx.x; f < F; f += kBlock) {
    const int fj = f / W, fi = f - fj * W;
    const int i = g.gi(fi), j = g.gj(fj);
    double v = 0.0;
    if (fi >= 1 && fj >= 1 && g.inside(i, j) && ((i + j) & 1) == 0) v = L.r[f] / diag_at(L, W, f);
    L.z[f] = v;
  }
  __syncthreads();
  // black cells of R1 (frame [2, W-1) x [2, H-1))
  for (int f = threadIdx.x; f < F; f += kBlock) {
    const int fj = f / W, fi = f - fj * W;
    if (fi < 2 || fi >= W - 1 || fj < 2 || fj >= H - 1) continue;
    const int i = g.gi(fi), j = g.gj(fj);
    if (!g.inside(i, j) || ((i + j) & 1) == 0) continue;
    L.z[f] = (L.r[f] + nsum_at(L, W, f)) / diag_at(L, W, f);
  }
  __syncthreads();
  double* zs = z + s * n;
  const int tcells = tx * ty;
  for (int c = threadIdx.x; c < tcells; c += kBlock) {
    const int cj = c / tx, ci = c - cj * tx;
    zs[(g.Y0 + cj) * m + g.X0 + ci] = L.z[(cj + 3) * W + ci + 3];
  }
  // restriction: sum of N(z_black) over the two red cells of each 2x2 block
  const int mc = m / 2, hx = tx / 2, hy = ty / 2;
  double* rcs = rc + s * (long long)mc * mc;
  for (int c = threadIdx.x; c < hx * hy; c += kBlock) {
    const int cj = c / hx, ci = c - cj * hx;
    const int fi0 = 3 + 2 * ci, fj0 = 3 + 2 * cj;     // frame index of the block's (0,0) cell
    // global (X0 + 2ci, Y0 + 2cj) has even i + j (X0, Y0 even): red cells are (0,0) and (1,1)
    const int fa = fj0 * W + fi0, fb = (fj0 + 1) * W + fi0 + 1;
    rcs[(g.Y0 / 2 + cj) * mc + g.X0 / 2 + ci] = nsum_at(L, W, fa) + nsum_at(L, W, fb);
  }
}

// ------------------------------------------------------------------ up
__global__ void __launch_bounds__(kBlock)
k_mg_up(int m, int tx, int ty, int tiles_per_sample, const double* __restrict__ T,
        const double* __restrict__ tb, const double* __restrict__ r,
        const double* __restrict__ zpre, double* __restrict__ z, const double* __restrict__ zc,
        double omega, const int32_t* __restrict__ active, double* __restrict__ rz_partial) {
  extern __shared__ double lds[];
  const long long s = blockIdx.x / tiles_per_sample;
  if (!active[s]) return;
  const FrameGeom g = frame_of(m, tx, ty, blockIdx.x - (int)(s * tiles_per_sample));
  const int W = g.W, H = g.H, F = W * H;
  Lds L{lds, lds + F, lds + 2 * F, lds + 3 * F};
  const long long n = (long long)m * m;
  const int mc = m / 2;
  const double* Ts = T + s * 2 * n;
  const double* tbs = tb + s * 2 * m;
  const double* rs = r + s * n;
  const double* zps = zpre + s * n;  // down-sweep result; read-only here (other tiles' halos)
  double* zs = z + s * n;
  const double* zcs = zc + s * (long long)mc * mc;
  for (int f = threadIdx.x; f < F; f += kBlock) {
    const int fj = f / W, fi = f - fj * W;
    const int i = g.gi(fi), j = g.gj(fj);
    L.te[f] = load_te(Ts, tbs, m, i, j);
    L.tn[f] = load_tn(Ts, tbs, m, i, j);
    const bool in = g.inside(i, j);
    L.r[f] = in ? rs[j * m + i] : 0.0;
    L.z[f] = in ? zps[j * m + i] + omega * zcs[(j >> 1) * mc + (i >> 1)] : 0.0;
  }
  __syncthreads();
  // black sweep on R1
  for (int f = threadIdx.x; f < F; f += kBlock) {
    const int fj = f / W, fi = f - fj * W;
    if (fi < 2 || fi >= W - 1 || fj < 2 || fj >= H - 1) continue;
    const int i = g.gi(fi), j = g.gj(fj);
    if (!g.inside(i, j) || ((i + j) & 1) == 0) continue;
    L.z[f] = (L.r[f] + nsum_at(L, W, f)) / diag_at(L, W, f);
  }
  __syncthreads();
  // red sweep on the tile, then store the tile
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
    zs[(g.Y0 + cj) * m + g.X0 + ci] = L.z[f];
    acc += L.r[f] * L.z[f];
  }
  if (rz_partial) {
    __shared__ double red[kBlock / kWave];
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) rz_partial[blockIdx.x] = t;
  }
}

// Branch-free load of one frame cell: every address is clamped into the
// sample's arrays, so all loads of a thread are issued back to back and the
// out-of-domain cases are resolved by selects afterwards.
struct FrameLoad {
  double te, tn;
  int c, ic, jc;
  bool in;
};

__device__ __forceinline__ FrameLoad frame_load(const double* __restrict__ Ts,
                                                const double* __restrict__ tbs, int m, int i,
                                                int j) {
  FrameLoad v;
  v.ic = min(max(i, 0), m - 1);
  v.jc = min(max(j, 0), m - 1);
  v.c = v.jc * m + v.ic;
  const bool iin = i >= 0 && i < m, jin = j >= 0 && j < m;
  v.in = iin && jin;
  const double te = Ts[v.c];
  const double tn = Ts[m * m + v.c];
  const double tw = tbs[v.jc];
  const double ts = tbs[m + v.ic];
  v.te = v.in ? te : ((i == -1 && jin) ? tw : 0.0);
  v.tn = v.in ? tn : ((j == -1 && iin) ? ts : 0.0);
  return v;
}

// ------------------------------------------------------------------ fixed-tile variants
// Same algorithm as k_mg_down / k_mg_up for tiles of compile-time size TX x TY
// (used when TX and TY divide m), organised for occupancy: each of the 512
// threads owns the frame cells f = tid + 512 k in every phase and keeps their
// four faces, right-hand side and z in registers; LDS holds only z, which is
// what neighbours read.  All loads use clamped, always-valid addresses and are
// resolved by selects, so a thread's loads are issued back to back.  Tiles of
// one sample run on one XCD, so the halo re-reads hit that XCD's L2.
constexpr int kMgThreads = 512;

template <int TX, int TY>
struct Tile {
  static constexpr int W = TX + 5, H = TY + 5, F = W * H;
  static constexpr int K = (F + kMgThreads - 1) / kMgThreads;
};

__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
  const int x = bid & 7, q = bid >> 3;
  const int per = nblocks >> 3, rem = nblocks & 7;
  return x * per + (x < rem ? x : rem) + q;
}

struct CellFaces {
  double te, tw, tn, ts;
  int c;      // clamped linear index of the cell in its sample
  bool in;    // inside the domain
};

// Faces of cell (i, j): east/north from T, west/south from the neighbour's
// east/north face or from the boundary arrays; everything 0 outside.
__device__ __forceinline__ CellFaces cell_faces(const double* __restrict__ Ts,
                                                const double* __restrict__ tbs, int m, int i,
                                                int j) {
  CellFaces v;
  const int ic = min(max(i, 0), m - 1), jc = min(max(j, 0), m - 1);
  const int iw = max(ic - 1, 0), js = max(jc - 1, 0);
  const int n = m * m;
  v.c = jc * m + ic;
  v.in = i >= 0 && i < m && j >= 0 && j < m;
  const double te = Ts[v.c], tn = Ts[n + v.c];
  const double tw = Ts[jc * m + iw], ts = Ts[n + js * m + ic];
  const double twb = tbs[jc], tsb = tbs[m + ic];
  v.te = v.in ? te : 0.0;
  v.tn = v.in ? tn : 0.0;
  v.tw = v.in ? (i > 0 ? tw : twb) : 0.0;
  v.ts = v.in ? (j > 0 ? ts : tsb) : 0.0;
  return v;
}

template <int TX, int TY>
__global__ void __launch_bounds__(kMgThreads)
k_mg_down_t(int m, const double* __restrict__ T, const double* __restrict__ tb,
            const double* __restrict__ r, double* __restrict__ z, double* __restrict__ rc,
            const int32_t* __restrict__ active) {
  using G = Tile<TX, TY>;
  constexpr int W = G::W, H = G::H, F = G::F, K = G::K;
  __shared__ double sz[F];
  const int ntx = m / TX, tps = ntx * (m / TY);
  const int bid = xcd_tile(blockIdx.x, gridDim.x);
  const long long s = bid / tps;
  if (!active[s]) return;
  const int tile = bid - (int)(s * tps);
  const int X0 = (tile % ntx) * TX, Y0 = (tile / ntx) * TY;
  const long long n = (long long)m * m;
  const double* Ts = T + s * 2 * n;
  const double* tbs = tb + s * 2 * m;
  const double* rs = r + s * n;
  CellFaces cf[K];
  double rv[K], zv[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    cf[k] = cell_faces(Ts, tbs, m, X0 - 3 + fi, Y0 - 3 + fj);
    const double rr = rs[cf[k].c];
    rv[k] = cf[k].in ? rr : 0.0;
  }
  // red cells of R2: z = r / D; all other cells start at 0
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    const double d = cf[k].te + cf[k].tw + cf[k].tn + cf[k].ts;
    zv[k] = (cf[k].in && fi >= 1 && fj >= 1 && ((fi + fj) & 1) == 0) ? rv[k] / d : 0.0;
    if (f < F) sz[f] = zv[k];
  }
  __syncthreads();
  // black cells of R1
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    if (f < F && cf[k].in && fi >= 2 && fi < W - 1 && fj >= 2 && fj < H - 1 && ((fi + fj) & 1)) {
      const double d = cf[k].te + cf[k].tw + cf[k].tn + cf[k].ts;
      zv[k] = (rv[k] + cf[k].te * sz[f + 1] + cf[k].tw * sz[f - 1] + cf[k].tn * sz[f + W] +
               cf[k].ts * sz[f - W]) / d;
      sz[f] = zv[k];
    }
  }
  __syncthreads();
  // store the tile; residual of its red cells (black residuals vanish)
  double* zs = z + s * n;
  double res[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    res[k] = 0.0;
    if (f < F && fi >= 3 && fi < 3 + TX && fj >= 3 && fj < 3 + TY) {
      zs[cf[k].c] = zv[k];
      if (((fi + fj) & 1) == 0)
        res[k] = cf[k].te * sz[f + 1] + cf[k].tw * sz[f - 1] + cf[k].tn * sz[f + W] +
                 cf[k].ts * sz[f - W];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    if (f < F) sz[f] = res[k];
  }
  __syncthreads();
  const int mc = m / 2;
  double* rcs = rc + s * (long long)mc * mc;
  constexpr int HX = TX / 2, HY = TY / 2;
  for (int c = threadIdx.x; c < HX * HY; c += kMgThreads) {
    const int cj = c / HX, ci = c - cj * HX;
    const int fa = (3 + 2 * cj) * W + 3 + 2 * ci;
    rcs[(Y0 / 2 + cj) * mc + X0 / 2 + ci] = sz[fa] + sz[fa + W + 1];
  }
}

template <int TX, int TY>
__global__ void __launch_bounds__(kMgThreads)
k_mg_up_t(int m, const double* __restrict__ T, const double* __restrict__ tb,
          const double* __restrict__ r, const double* __restrict__ zpre, double* __restrict__ z,
          const double* __restrict__ zc, double omega, const int32_t* __restrict__ active,
          double* __restrict__ rz_partial) {
  using G = Tile<TX, TY>;
  constexpr int W = G::W, H = G::H, F = G::F, K = G::K;
  __shared__ double sz[F];
  __shared__ double red[kMgThreads / kWave];
  const int ntx = m / TX, tps = ntx * (m / TY);
  const int bid = xcd_tile(blockIdx.x, gridDim.x);
  const long long s = bid / tps;
  if (!active[s]) return;
  const int tile = bid - (int)(s * tps);
  const int X0 = (tile % ntx) * TX, Y0 = (tile / ntx) * TY;
  const long long n = (long long)m * m;
  const int mc = m / 2;
  const double* Ts = T + s * 2 * n;
  const double* tbs = tb + s * 2 * m;
  const double* rs = r + s * n;
  const double* zps = zpre + s * n;
  const double* zcs = zc + s * (long long)mc * mc;
  CellFaces cf[K];
  double rv[K], zv[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    const int i = X0 - 3 + fi, j = Y0 - 3 + fj;
    cf[k] = cell_faces(Ts, tbs, m, i, j);
    const int ic = min(max(i, 0), m - 1), jc = min(max(j, 0), m - 1);
    const double rr = rs[cf[k].c], zp = zps[cf[k].c], zcv = zcs[(jc >> 1) * mc + (ic >> 1)];
    rv[k] = cf[k].in ? rr : 0.0;
    zv[k] = cf[k].in ? zp + omega * zcv : 0.0;
    if (f < F) sz[f] = zv[k];
  }
  __syncthreads();
  // black sweep on R1
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    if (f < F && cf[k].in && fi >= 2 && fi < W - 1 && fj >= 2 && fj < H - 1 && ((fi + fj) & 1)) {
      const double d = cf[k].te + cf[k].tw + cf[k].tn + cf[k].ts;
      zv[k] = (rv[k] + cf[k].te * sz[f + 1] + cf[k].tw * sz[f - 1] + cf[k].tn * sz[f + W] +
               cf[k].ts * sz[f - W]) / d;
      sz[f] = zv[k];
    }
  }
  __syncthreads();
  // red sweep on the tile, store, r^T z
  double* zs = z + s * n;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int f = threadIdx.x + k * kMgThreads;
    const int fj = f / W, fi = f - fj * W;
    if (f < F && fi >= 3 && fi < 3 + TX && fj >= 3 && fj < 3 + TY) {
      if (((fi + fj) & 1) == 0) {
        const double d = cf[k].te + cf[k].tw + cf[k].tn + cf[k].ts;
        zv[k] = (rv[k] + cf[k].te * sz[f + 1] + cf[k].tw * sz[f - 1] + cf[k].tn * sz[f + W] +
                 cf[k].ts * sz[f - W]) / d;
      }
      zs[cf[k].c] = zv[k];
      acc += rv[k] * zv[k];
    }
  }
  if (rz_partial) {
    // fixed-order block sum over the 8 waves
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

static int g_tile_y = -1;
static int tile_y() {
  if (g_tile_y < 0) {
    const char* e = getenv("MLMC_TILE_Y");
    g_tile_y = (e && atoi(e) == 16) ? 16 : 32;
  }
  return g_tile_y;
}

// Largest even divisor of m that is <= cap.
static int tile_dim(int m, int cap) {
  for (int t = cap < m ? cap : m; t >= 2; --t)
    if (m % t == 0 && (t % 2) == 0) return t;
  return 2;
}

static size_t frame_bytes(int tx, int ty) { return (size_t)4 * (tx + 5) * (ty + 5) * sizeof(double); }

void launch_mg_down(hipStream_t st, int m, int batch, const double* T, const double* tb,
                    const double* r, double* z, double* rc, const int32_t* active) {
  if (m % 64 == 0 && m % tile_y() == 0) {
    if (tile_y() == 32)
      hipLaunchKernelGGL((k_mg_down_t<64, 32>), dim3(batch * (m / 64) * (m / 32)),
                         dim3(kMgThreads), 0, st, m, T, tb, r, z, rc, active);
    else
      hipLaunchKernelGGL((k_mg_down_t<64, 16>), dim3(batch * (m / 64) * (m / 16)),
                         dim3(kMgThreads), 0, st, m, T, tb, r, z, rc, active);
    return;
  }
  const int tx = tile_dim(m, kTileX), ty = tile_dim(m, kTileY);
  const int tps = (m / tx) * (m / ty);
  hipLaunchKernelGGL(k_mg_down, dim3(batch * tps), dim3(kBlock), frame_bytes(tx, ty), st, m, tx,
                     ty, tps, T, tb, r, z, rc, active);
}

int mg_tiles_per_sample(int m) {
  if (m % 64 == 0 && m % tile_y() == 0) return (m / 64) * (m / tile_y());
  const int tx = tile_dim(m, kTileX), ty = tile_dim(m, kTileY);
  return (m / tx) * (m / ty);
}

void launch_mg_up(hipStream_t st, int m, int batch, const double* T, const double* tb,
                  const double* r, const double* zpre, double* z, const double* zc, double omega,
                  const int32_t* active, double* rz_partial) {
  if (m % 64 == 0 && m % tile_y() == 0) {
    if (tile_y() == 32)
      hipLaunchKernelGGL((k_mg_up_t<64, 32>), dim3(batch * (m / 64) * (m / 32)),
                         dim3(kMgThreads), 0, st, m, T, tb, r, zpre, z, zc, omega, active,
                         rz_partial);
    else
      hipLaunchKernelGGL((k_mg_up_t<64, 16>), dim3(batch * (m / 64) * (m / 16)),
                         dim3(kMgThreads), 0, st, m, T, tb, r, zpre, z, zc, omega, active,
                         rz_partial);
    return;
  }
  const int tx = tile_dim(m, kTileX), ty = tile_dim(m, kTileY);
  const int tps = (m / tx) * (m / ty);
  hipLaunchKernelGGL(k_mg_up, dim3(batch * tps), dim3(kBlock), frame_bytes(tx, ty), st, m, tx, ty,
                     tps, T, tb, r, zpre, z, zc, omega, active, rz_partial);
}

// ------------------------------------------------------------------ coarse cycle in LDS
// One workgroup per sample runs the V(1,1)-cycle on levels l0..L (m_l0 <= 32)
// with every level's operator and vectors in LDS.  Level arrays use a padded
// (m + 2)^2 layout with a one-cell ring: ring cells hold z = 0 and the
// boundary faces (west face in column -1, south face in row -1), so the
// stencil needs no branches.
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

__global__ void __launch_bounds__(kBlock)
k_mg_coarse_cycle(int nlev, CoarseDesc desc, const double* __restrict__ r0,
                  double* __restrict__ z0, const double* __restrict__ Ainv, double omega,
                  const int32_t* __restrict__ active, double* __restrict__ rz_partial) {
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
  double* vec = lds + off;  // coarsest right-hand side / solution scratch (n_c doubles)
  // load operators (levels are stored in global memory with the library layout)
  for (int l = 0; l < nlev; ++l) {
    const int m = lv[l].m, P = lv[l].P, PP = P * P;
    double* te = lds + lv[l].off;
    double* tn = te + PP;
    double* rr = tn + PP;
    double* zz = rr + PP;
    const long long n = (long long)m * m;
    const double* Ts = desc.T[l] + (long long)s * 2 * n;
    const double* tbs = desc.tb[l] + (long long)s * 2 * m;
    for (int f = threadIdx.x; f < PP; f += kBlock) {
      const int j = f / P - 1, i = f % P - 1;
      te[f] = load_te(Ts, tbs, m, i, j);
      tn[f] = load_tn(Ts, tbs, m, i, j);
      rr[f] = (l == 0 && i >= 0 && i < m && j >= 0 && j < m) ? r0[(long long)s * n + j * m + i] : 0.0;
      zz[f] = 0.0;
    }
  }
  __syncthreads();
  // descend
  for (int l = 0; l < nlev - 1; ++l) {
    const int m = lv[l].m, P = lv[l].P, PP = P * P;
    double* te = lds + lv[l].off;
    double* tn = te + PP;
    double* rr = tn + PP;
    double* zz = rr + PP;
    cc_sweep(te, tn, rr, zz, m, P, 0, true);
    cc_sweep(te, tn, rr, zz, m, P, 1, false);
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
  }
  // coarsest: z = Ainv r
  {
    const int l = nlev - 1;
    const int m = lv[l].m, P = lv[l].P, PP = P * P, nc = m * m;
    double* rr = lds + lv[l].off + 2 * PP;
    double* zz = rr + PP;
    for (int q = threadIdx.x; q < nc; q += kBlock) vec[q] = rr[pidx(P, q % m, q / m)];
    __syncthreads();
    const double* A = Ainv + (long long)s * nc * nc;
    for (int q = threadIdx.x; q < nc; q += kBlock) {
      double acc = 0.0;
      for (int p = 0; p < nc; ++p) acc += A[q * nc + p] * vec[p];
      zz[pidx(P, q % m, q / m)] = acc;
    }
    __syncthreads();
  }
  // ascend
  for (int l = nlev - 2; l >= 0; --l) {
    const int m = lv[l].m, P = lv[l].P, PP = P * P;
    double* te = lds + lv[l].off;
    double* tn = te + PP;
    double* rr = tn + PP;
    double* zz = rr + PP;
    const int Pc = lv[l + 1].P, PPc = Pc * Pc;
    const double* zc = lds + lv[l + 1].off + 3 * PPc;
    for (int c = threadIdx.x; c < m * m; c += kBlock) {
      const int j = c / m, i = c - j * m;
      zz[pidx(P, i, j)] += omega * zc[pidx(Pc, i / 2, j / 2)];
    }
    __syncthreads();
    cc_sweep(te, tn, rr, zz, m, P, 1, false);
    cc_sweep(te, tn, rr, zz, m, P, 0, false);
  }
  // store level l0's correction
  {
    const int m = lv[0].m, P = lv[0].P, PP = P * P;
    const double* rr = lds + lv[0].off + 2 * PP;
    const double* zz = rr + PP;
    double acc = 0.0;
    for (int c = threadIdx.x; c < m * m; c += kBlock) {
      const int f = pidx(P, c % m, c / m);
      z0[(long long)s * m * m + c] = zz[f];
      acc += rr[f] * zz[f];
    }
    if (rz_partial) {
      __shared__ double red[kBlock / kWave];
      const double t = block_sum(acc, red);
      if (threadIdx.x == 0) rz_partial[s] = t;
    }
  }
}

size_t coarse_cycle_lds_bytes(const CoarseDesc& d, int nlev) {
  size_t words = 0;
  for (int l = 0; l < nlev; ++l) words += 4 * (size_t)(d.m[l] + 2) * (d.m[l] + 2);
  words += (size_t)d.m[nlev - 1] * d.m[nlev - 1];
  return words * sizeof(double);
}

void launch_mg_coarse_cycle(hipStream_t st, int batch, int nlev, const CoarseDesc& desc,
                            const double* r0, double* z0, const double* Ainv, double omega,
                            const int32_t* active, double* rz_partial) {
  hipLaunchKernelGGL(k_mg_coarse_cycle, dim3(batch), dim3(kBlock),
                     coarse_cycle_lds_bytes(desc, nlev), st, nlev, desc, r0, z0, Ainv, omega,
                     active, rz_partial);
}

}  // namespace mlmc
