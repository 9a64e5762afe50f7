// The 3-D path: sample, assemble, multigrid-preconditioned CG and QoI on
// m x m x m grids (Sections 2, 3.1, 3.4 and 3.5 with d = 3).
//
// Layout per sample s (n = m^3 cells, c = (l m + j) m + i, x1 fastest):
//   k[s][l][j][i];
//   T[s][0][c] face x1 = (i+1)h (i = m-1: the Dirichlet face at x1 = 1),
//   T[s][1][c] face x2 = (j+1)h, T[s][2][c] face x3 = (l+1)h (0 on the top);
//   tb[s][0][l m + j] face x1 = 0 of cell (0, j, l) (Dirichlet, p = 1),
//   tb[s][1][l m + i] face x2 = 0, tb[s][2][j m + i] face x3 = 0 (no flow: 0);
//   (A x)_c = (sum of the six face T) x_c - sum over interior faces T x_nb.
// A face between cells P and Q has T = h^(d-2) 2 k_P k_Q / (k_P + k_Q) = h
// times the harmonic mean; a Dirichlet face T = 2 k_P h (half-cell distance).
//
// The multigrid is the same as in 2-D with 2 x 2 x 2 aggregation (the
// Galerkin coarse face is the sum of the four fine faces it covers): on the
// larger grids one launch per colour half-sweep, one for residual and
// restriction, and the prolongation folded into the next black half-sweep;
// the levels from side 8 (FP64) or 16 (FP32) down in one in-LDS launch per
// visit; the dense inverse on the coarsest grid (<= 4^3 unknowns).
//
// The vectors (z, r and, on the finest level, the CG's x, r, p, q) and the
// faces T of every level swept by the per-sweep kernels are stored in
// colour-split order (cs3.hpp), the faces as a copy in the hierarchy's type;
// k, b, the caller's T and the solution handed back stay in the natural
// order, and so do the in-LDS and the dense coarsest levels.
#include <cfloat>

#include "common.hpp"
#include "cs3.hpp"
#include "fft.hpp"
#include "kernels.hpp"

namespace mlmc {

// Faces of a cell in the storage type S of the operator (double, or float for
// a reduced-precision multigrid hierarchy; the arithmetic is done in S).
template <class S>
struct Faces3T {
  S te, tw, tn, ts, tu, td;
};
using Faces3 = Faces3T<double>;

template <class S>
__device__ __forceinline__ Faces3T<S> load_faces3(const S* __restrict__ Ts,
                                                  const S* __restrict__ tbs, int m, int i, int j,
                                                  int l) {
  const long long n = (long long)m * m * m;
  const int mm = m * m;
  const long long c = ((long long)l * m + j) * m + i;
  Faces3T<S> f;
  f.te = Ts[c];
  f.tw = i > 0 ? Ts[c - 1] : tbs[l * m + j];
  f.tn = Ts[n + c];
  f.ts = j > 0 ? Ts[n + c - m] : tbs[mm + l * m + i];
  f.tu = Ts[2 * n + c];
  f.td = l > 0 ? Ts[2 * n + c - mm] : tbs[2 * mm + j * m + i];
  return f;
}

// The same faces from face arrays in colour-split order (T[a] entry of a cell
// at its colour-split index): the east, north and up faces at the cell's own
// index `own`, the west, south and down ones at its neighbours' (nb).
template <class S>
__device__ __forceinline__ Faces3T<S> load_faces3_cs(const S* __restrict__ Ts,
                                                     const S* __restrict__ tbs, int m, int i,
                                                     int j, int l, long long own,
                                                     const Cs3Nb& nb) {
  const long long n = (long long)m * m * m;
  const int mm = m * m;
  Faces3T<S> f;
  f.te = Ts[own];
  f.tw = i > 0 ? Ts[nb.other + nb.dw] : tbs[l * m + j];
  f.tn = Ts[n + own];
  f.ts = j > 0 ? Ts[n + nb.other + nb.ds] : tbs[mm + l * m + i];
  f.tu = Ts[2 * n + own];
  f.td = l > 0 ? Ts[2 * n + nb.other + nb.dd] : tbs[2 * mm + j * m + i];
  return f;
}

// Neighbour sum over the interior faces, x of type X (the level's vector
// type), accumulated in the operator's type S.
template <class S, class X>
__device__ __forceinline__ S nsum3(const X* __restrict__ x, int m, int i, int j, int l,
                                   const Faces3T<S>& f) {
  const long long c = ((long long)l * m + j) * m + i;
  const long long mm = (long long)m * m;
  S o = S(0);
  if (i < m - 1) o += f.te * (S)x[c + 1];
  if (i > 0) o += f.tw * (S)x[c - 1];
  if (j < m - 1) o += f.tn * (S)x[c + m];
  if (j > 0) o += f.ts * (S)x[c - m];
  if (l < m - 1) o += f.tu * (S)x[c + mm];
  if (l > 0) o += f.td * (S)x[c - mm];
  return o;
}

// The same sum, in the same order, over a level vector xs (one sample) in
// colour-split order.
template <class S, class X>
__device__ __forceinline__ S nsum3_cs(const X* __restrict__ xs, int m, int i, int j, int l,
                                      const Faces3T<S>& f) {
  const Cs3Nb nb = cs3_neighbours(m, i, j, l);
  const X* xo = xs + nb.other;
  S o = S(0);
  if (i < m - 1) o += f.te * (S)xo[nb.de];
  if (i > 0) o += f.tw * (S)xo[nb.dw];
  if (j < m - 1) o += f.tn * (S)xo[nb.dn];
  if (j > 0) o += f.ts * (S)xo[nb.ds];
  if (l < m - 1) o += f.tu * (S)xo[nb.du];
  if (l > 0) o += f.td * (S)xo[nb.dd];
  return o;
}

template <class S>
__device__ __forceinline__ S diag3(const Faces3T<S>& f) {
  return f.te + f.tw + f.tn + f.ts + f.tu + f.td;
}

__device__ __forceinline__ void cell_of(long long rem, int m, int& i, int& j, int& l) {
  l = (int)(rem / ((long long)m * m));
  const int r2 = (int)(rem - (long long)l * m * m);
  j = r2 / m;
  i = r2 - j * m;
}

// Quotient n / d for 0 <= n < 2^32 and a divisor 1 <= d < 2^31 fixed per launch,
// through a multiply-high (Granlund and Montgomery, PLDI 1994, round-up
// method): with l = ceil(log2 d) and mul = floor(2^32 (2^l - d) / d) + 1,
// t = mulhi(n, mul) and q = (t + ((n - t) >> 1)) >> (l - 1) (l = 0: q = n).
// The per-sweep kernels index their cells with it instead of 64-bit divisions.
struct FastDiv {
  uint32_t d, mul, s1, s2;
};

inline FastDiv make_fastdiv(uint32_t d) {
  d = d > 0 ? d : 1u;  // (empty grids)
  FastDiv f{d, 1u, 0u, 0u};
  int l = 0;
  while ((1ull << l) < d) ++l;
  f.mul = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d + 1) & 0xFFFFFFFFull);
  f.s1 = l > 0 ? 1u : 0u;
  f.s2 = l > 0 ? (uint32_t)(l - 1) : 0u;
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  const uint32_t t = __umulhi(n, f.mul);
  return (t + ((n - t) >> f.s1)) >> f.s2;
}

// Cell (i, j, l) and sample s of flat index g = s n + (l a + j) b + i, where n is
// the per-sample count, mm.d = a b and m.d = b (a = b = m for a whole grid),
// through three FastDivs, or 64-bit divisions when the launch has 2^32 or more
// threads (fast = false).
struct CellDiv {
  FastDiv per, mm, m;
  int fast;
};

inline CellDiv make_celldiv(long long total, long long per, int m) {
  CellDiv c;
  c.fast = total < (1ll << 32) && per < (1ll << 31);
  c.per = make_fastdiv(c.fast ? (uint32_t)per : 1u);
  c.mm = make_fastdiv((uint32_t)m * (uint32_t)m);
  c.m = make_fastdiv((uint32_t)m);
  return c;
}

__device__ __forceinline__ long long split_cell(long long g, long long per, const CellDiv& cd,
                                                int& i, int& j, int& l) {
  if (cd.fast) {
    const uint32_t gg = (uint32_t)g;
    const uint32_t s = fdiv(gg, cd.per);
    const uint32_t rem = gg - s * cd.per.d;
    l = (int)fdiv(rem, cd.mm);
    const uint32_t r2 = rem - (uint32_t)l * cd.mm.d;
    j = (int)fdiv(r2, cd.m);
    i = (int)(r2 - (uint32_t)j * cd.m.d);
    return (long long)s;
  }
  const long long s = g / per;
  const long long rem = g - s * per;
  l = (int)(rem / (long long)cd.mm.d);
  const long long r2 = rem - (long long)l * cd.mm.d;
  j = (int)(r2 / (long long)cd.m.d);
  i = (int)(r2 - (long long)j * cd.m.d);
  return s;
}

// ------------------------------------------------------------------ assembly
// Model Problem 2 as in 2-D, with T scaled by the face area / centre distance
// h^2 / h = h; Model Problem 1: every boundary face Dirichlet (T = 2 k h),
// b = f h^3 = h^3.
__global__ void k_assemble3(int problem, int m, long long total, const double* __restrict__ k,
                            double* __restrict__ T, double* __restrict__ tb,
                            double* __restrict__ b) {
  const long long g = (long long)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long long n = (long long)m * m * m;
  const int mm = m * m;
  const long long s = g / n;
  const long long c = g - s * n;
  int i, j, l;
  cell_of(c, m, i, j, l);
  const double h = 1.0 / (double)m;
  const double* ks = k + s * n;
  const double kc = ks[c];
  double* Ts = T + s * 3 * n;
  const bool mp1 = problem == MLMC_PROBLEM_MEAN_PRESSURE;
  const double tw = 2.0 * kc * h;
  const double side = mp1 ? tw : 0.0;  // faces x2 = 0, 1 and x3 = 0, 1
  Ts[c] = i < m - 1 ? h * (2.0 * kc * ks[c + 1] / (kc + ks[c + 1])) : tw;
  Ts[n + c] = j < m - 1 ? h * (2.0 * kc * ks[c + m] / (kc + ks[c + m])) : side;
  Ts[2 * n + c] = l < m - 1 ? h * (2.0 * kc * ks[c + mm] / (kc + ks[c + mm])) : side;
  double* tbs = tb + s * 3 * mm;
  if (i == 0) tbs[l * m + j] = tw;
  if (j == 0) tbs[mm + l * m + i] = side;
  if (l == 0) tbs[2 * mm + j * m + i] = side;
  b[g] = mp1 ? h * h * h : (i == 0 ? tw : 0.0);
}

void launch_assemble3(hipStream_t st, int problem, int m, int batch, const double* k, double* T,
                      double* tb, double* b) {
  const long long total = (long long)batch * m * m * m;
  hipLaunchKernelGGL(k_assemble3, dim3(blocks_for(total)), dim3(kBlock), 0, st, problem, m, total,
                     k, T, tb, b);
}

// ------------------------------------------------------------------ QoI
// Q_out = sum over the x1 = 1 faces of 2 k h p, Q_in = sum over x1 = 0 of
// 2 k h (1 - p); one wave per sample, fixed-order sums.
// Outflow (and inflow) of each sample in two steps: kQoi3Parts workgroups per
// sample sum fixed, contiguous ranges of the m^2 boundary rows (q = l m + j)
// into partials; one wave per sample adds its partials in order.  The sums do
// not depend on the launch's timing.
constexpr int kQoi3Parts = 32;
__global__ void k_qoi3_parts(int m, int batch, const double* __restrict__ k,
                             const double* __restrict__ p, double* __restrict__ part) {
  const int s = blockIdx.x / kQoi3Parts;
  const int g = blockIdx.x - s * kQoi3Parts;
  if (s >= batch) return;
  const long long n = (long long)m * m * m;
  const long long base = (long long)s * n;
  const double h = 1.0 / (double)m;
  const int rows = m * m;
  const int per = (rows + kQoi3Parts - 1) / kQoi3Parts;
  const int q0 = g * per, q1 = min(rows, q0 + per);
  double so = 0.0, si = 0.0;
  for (int q = q0 + threadIdx.x; q < q1; q += kBlock) {
    const long long row = base + (long long)q * m;
    so += 2.0 * k[row + m - 1] * h * p[row + m - 1];
    si += 2.0 * k[row] * h * (1.0 - p[row]);
  }
  __shared__ double sho[kBlock / kWave], shi[kBlock / kWave];
  so = block_sum(so, sho);
  si = block_sum(si, shi);
  if (threadIdx.x == 0) {
    part[2 * (long long)blockIdx.x] = so;
    part[2 * (long long)blockIdx.x + 1] = si;
  }
}

__global__ void k_qoi3_final(int batch, const double* __restrict__ part, double* __restrict__ qout,
                             double* __restrict__ qin) {
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (wave >= batch) return;
  const double* ps = part + 2 * wave * kQoi3Parts;
  double so = lane < kQoi3Parts ? ps[2 * lane] : 0.0;
  double si = lane < kQoi3Parts ? ps[2 * lane + 1] : 0.0;
  so = wave_sum(so);
  si = wave_sum(si);
  if (lane == 0) {
    qout[wave] = so;
    if (qin) qin[wave] = si;
  }
}

size_t qoi3_parts_size(int batch) { return (size_t)batch * kQoi3Parts * 2; }

void launch_qoi3(hipStream_t st, int m, int batch, const double* k, const double* p, double* part,
                 double* qout, double* qin) {
  hipLaunchKernelGGL(k_qoi3_parts, dim3(batch * kQoi3Parts), dim3(kBlock), 0, st, m, batch, k, p,
                     part);
  const long long threads = (long long)batch * kWave;
  hipLaunchKernelGGL(k_qoi3_final, dim3(blocks_for(threads)), dim3(kBlock), 0, st, batch, part,
                     qout, qin);
}

// ------------------------------------------------------------------ hierarchy
__global__ void k_coarsen3(int m, long long total, const double* __restrict__ T,
                           const double* __restrict__ tb, double* __restrict__ Tc,
                           double* __restrict__ tbc) {
  const long long g = (long long)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int mc = m / 2;
  const long long nc = (long long)mc * mc * mc, n = (long long)m * m * m;
  const long long s = g / nc;
  const long long rem = g - s * nc;
  int I, J, L;
  cell_of(rem, mc, I, J, L);
  const double* Ts = T + s * 3 * n;
  double* Tcs = Tc + s * 3 * nc;
  const int i = 2 * I, j = 2 * J, l = 2 * L;
  auto at = [&](int a, int bb, int cc) { return ((long long)cc * m + bb) * m + a; };
  Tcs[rem] = Ts[at(i + 1, j, l)] + Ts[at(i + 1, j + 1, l)] + Ts[at(i + 1, j, l + 1)] +
             Ts[at(i + 1, j + 1, l + 1)];
  Tcs[nc + rem] = Ts[n + at(i, j + 1, l)] + Ts[n + at(i + 1, j + 1, l)] +
                  Ts[n + at(i, j + 1, l + 1)] + Ts[n + at(i + 1, j + 1, l + 1)];
  Tcs[2 * nc + rem] = Ts[2 * n + at(i, j, l + 1)] + Ts[2 * n + at(i + 1, j, l + 1)] +
                      Ts[2 * n + at(i, j + 1, l + 1)] + Ts[2 * n + at(i + 1, j + 1, l + 1)];
  const int mm = m * m, mmc = mc * mc;
  const double* tbs = tb + s * 3 * mm;
  double* tbcs = tbc + s * 3 * mmc;
  if (I == 0)
    tbcs[L * mc + J] = tbs[l * m + j] + tbs[l * m + j + 1] + tbs[(l + 1) * m + j] +
                       tbs[(l + 1) * m + j + 1];
  if (J == 0)
    tbcs[mmc + L * mc + I] = tbs[mm + l * m + i] + tbs[mm + l * m + i + 1] +
                             tbs[mm + (l + 1) * m + i] + tbs[mm + (l + 1) * m + i + 1];
  if (L == 0)
    tbcs[2 * mmc + J * mc + I] = tbs[2 * mm + j * m + i] + tbs[2 * mm + j * m + i + 1] +
                                 tbs[2 * mm + (j + 1) * m + i] + tbs[2 * mm + (j + 1) * m + i + 1];
}

void launch_coarsen3(hipStream_t st, int m, int batch, const double* T, const double* tb,
                     double* Tc, double* tbc) {
  const long long total = (long long)batch * (m / 2) * (m / 2) * (m / 2);
  hipLaunchKernelGGL(k_coarsen3, dim3(blocks_for(total)), dim3(kBlock), 0, st, m, total, T, tb,
                     Tc, tbc);
}

// ------------------------------------------------------------------ smoother
// One thread per cell of the colour ((i + j + l) % 2 == color); m even; T, z
// and r in colour-split order, so thread g of sample s reads r and writes z
// at color m^3/2 + (g - s m^3/2).
// S: operator storage and arithmetic type; V: type of the level's z and r
// (double on the finest level, whose z and r are the CG's).
template <class S, class V>
__global__ void k_rbgs3(int m, long long total, const S* __restrict__ T,
                        const S* __restrict__ tb, V* __restrict__ z,
                        const V* __restrict__ r, const int32_t* __restrict__ active,
                        int color, int zero_init, CellDiv cd) {
  // rows of a sample that share z and face lines run on one XCD
  const long long g = (long long)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int half = m / 2;
  const long long per = (long long)m * m * half;
  // (sample, l, j, h) of g as a cell of an m x m x half grid: the red or black
  // cell of column pair h in row (l, j)
  int h, j, l;
  const long long s = split_cell(g, per, cd, h, j, l);
  if (!active[s]) return;
  const int i = 2 * h + ((j + l + color) & 1);
  const long long n = (long long)m * m * m;
  V* zs = z + s * n;
  const long long e = (long long)color * per + (g - s * per);
  const Faces3T<S> f = load_faces3_cs(T + s * 3 * n, tb + s * 3 * m * m, m, i, j, l, e,
                                      cs3_neighbours(m, i, j, l));
  const S rv = (S)r[s * n + e];
  zs[e] = (V)(zero_init ? rv / diag3(f) : (rv + nsum3_cs(zs, m, i, j, l, f)) / diag3(f));
}

template <class S, class V>
static void rbgs3_t(hipStream_t st, int m, int batch, const void* T, const void* tb, void* z,
                    const void* r, const int32_t* active, int color, int zero_init) {
  const long long total = (long long)batch * m * m * (m / 2);
  // split_cell's rows are (l, j) pairs of m x m, the fastest index a column pair
  CellDiv cd = make_celldiv(total, (long long)m * m * (m / 2), m);
  cd.mm = make_fastdiv((uint32_t)m * (uint32_t)(m / 2));
  cd.m = make_fastdiv((uint32_t)(m / 2));
  launch_k((k_rbgs3<S, V>), dim3(blocks_for(total)), dim3(kBlock), 0, st, m, total,
                     (const S*)T, (const S*)tb, (V*)z, (const V*)r, active, color, zero_init, cd);
}

void launch_rbgs3_p(hipStream_t st, bool f32, bool top, int m, int batch, const void* T,
                    const void* tb, void* z, const void* r, const int32_t* active, int color,
                    int zero_init) {
  if (!f32) rbgs3_t<double, double>(st, m, batch, T, tb, z, r, active, color, zero_init);
  else if (top) rbgs3_t<float, double>(st, m, batch, T, tb, z, r, active, color, zero_init);
  else rbgs3_t<float, float>(st, m, batch, T, tb, z, r, active, color, zero_init);
}

// Prolongation fused into the first half-sweep of post-smoothing.  After
// z += omega P zc the black half-sweep replaces every black value, and the red
// half-sweep after it replaces every red one, so the prolonged values are
// only ever read as the black cells' red neighbours: the kernel updates the
// black cells (one thread each) from neighbours z_n + omega zc(parent of n),
// formed as the prolongation forms them (in V), and writes nothing else: the
// arithmetic of a separate prolongation pass followed by k_rbgs3 on the black
// cells.  T, z and r in colour-split order; zc in colour-split order when csc
// is set (the coarse level is swept per launch too), else natural.
template <class S, class V>
__global__ void k_prolong_black3(int m, long long total, const S* __restrict__ T,
                                 const S* __restrict__ tb, V* __restrict__ z,
                                 const V* __restrict__ r, const S* __restrict__ zc,
                                 double omega, const int32_t* __restrict__ active, int csc,
                                 CellDiv cd) {
  // rows of a sample that share z and face lines run on one XCD
  const long long g = (long long)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int half = m / 2;
  const long long per = (long long)m * m * half;
  int h, j, l;
  const long long s = split_cell(g, per, cd, h, j, l);
  if (!active[s]) return;
  const int i = 2 * h + ((j + l + 1) & 1);
  const long long n = (long long)m * m * m;
  const int mc = m / 2;
  const long long e = per + (g - s * per);  // black block
  const Cs3Nb nb = cs3_neighbours(m, i, j, l);
  const Faces3T<S> f = load_faces3_cs(T + s * 3 * n, tb + s * 3 * m * m, m, i, j, l, e, nb);
  V* zs = z + s * n;
  const S* zcs = zc + s * (long long)mc * mc * mc;
  const V w = (V)omega;
  // The six red neighbours lie in four coarse cells: the cell's own parent
  // (I, J, L) and, along each axis, the parent one step towards the
  // neighbour across the parent's face (I + dx with dx = +1 for odd i, -1 for
  // even i; likewise in x2 and x3).  That parent exists exactly when that
  // neighbour does.  Coarse indices in 32 bits (mc^3 < 2^31).
  const int I = i >> 1, J = j >> 1, L = l >> 1;
  const int dx = (i & 1) ? 1 : -1, dy = (j & 1) ? 1 : -1, dz = (l & 1) ? 1 : -1;
  const int hc = mc / 2, nch = mc * mc * hc;
  auto cidx = [&](int a, int b, int c) -> int {
    return csc ? ((a + b + c) & 1) * nch + (c * mc + b) * hc + (a >> 1) : (c * mc + b) * mc + a;
  };
  const S c0 = zcs[cidx(I, J, L)];
  const bool hx = (unsigned)(I + dx) < (unsigned)mc, hy = (unsigned)(J + dy) < (unsigned)mc,
             hz = (unsigned)(L + dz) < (unsigned)mc;
  const S cx = hx ? zcs[cidx(I + dx, J, L)] : S(0);
  const S cy = hy ? zcs[cidx(I, J + dy, L)] : S(0);
  const S cz = hz ? zcs[cidx(I, J, L + dz)] : S(0);
  // the red neighbour at offset d of the red row entry, prolonged from the
  // coarse value zcv of the cell holding it
  const V* zo = zs + nb.other;
  auto pz = [&](int d, S zcv) -> S { return (S)(zo[d] + w * (V)zcv); };
  S o = S(0);
  if (i < m - 1) o += f.te * pz(nb.de, (i & 1) ? cx : c0);
  if (i > 0) o += f.tw * pz(nb.dw, (i & 1) ? c0 : cx);
  if (j < m - 1) o += f.tn * pz(nb.dn, (j & 1) ? cy : c0);
  if (j > 0) o += f.ts * pz(nb.ds, (j & 1) ? c0 : cy);
  if (l < m - 1) o += f.tu * pz(nb.du, (l & 1) ? cz : c0);
  if (l > 0) o += f.td * pz(nb.dd, (l & 1) ? c0 : cz);
  const S rv = (S)r[s * n + e];
  zs[e] = (V)((rv + o) / diag3(f));
}

template <class S, class V>
static void prolong_black3_t(hipStream_t st, int m, int batch, const void* T, const void* tb,
                             void* z, const void* r, const void* zc, double omega,
                             const int32_t* active, int csc) {
  const long long total = (long long)batch * m * m * (m / 2);
  CellDiv cd = make_celldiv(total, (long long)m * m * (m / 2), m);
  cd.mm = make_fastdiv((uint32_t)m * (uint32_t)(m / 2));
  cd.m = make_fastdiv((uint32_t)(m / 2));
  hipLaunchKernelGGL((k_prolong_black3<S, V>), dim3(blocks_for(total)), dim3(kBlock), 0, st, m,
                     total, (const S*)T, (const S*)tb, (V*)z, (const V*)r, (const S*)zc, omega,
                     active, csc, cd);
}

void launch_prolong_black3_p(hipStream_t st, bool f32, bool top, int m, int batch, const void* T,
                             const void* tb, void* z, const void* r, const void* zc,
                             double omega, const int32_t* active, bool coarse_split) {
  const int csc = coarse_split ? 1 : 0;
  if (!f32) prolong_black3_t<double, double>(st, m, batch, T, tb, z, r, zc, omega, active, csc);
  else if (top)
    prolong_black3_t<float, double>(st, m, batch, T, tb, z, r, zc, omega, active, csc);
  else prolong_black3_t<float, float>(st, m, batch, T, tb, z, r, zc, omega, active, csc);
}

// rc(I, J, L) = sum over the 2 x 2 x 2 fine cells of (r - A z); rc in S.
// T, z and r in colour-split order (one thread per coarse cell, taken in natural
// order: the fine cells 2I and 2I + 1 of a row sit at I in the red and the
// black row); rc in colour-split order when csc is set, else natural.  Each
// value the eight residuals use is loaded once: z and the faces of the block's
// four rows, z of the eight rows beside it in x2 and x3, the faces below and
// south of it, and z and the east face west of it; the sums are those of
// nsum3_cs and diag3, term by term.
template <class S, class V>
__global__ void __launch_bounds__(kBlock) k_resid_restrict3(int m, long long total, const S* __restrict__ T,
                                  const S* __restrict__ tb, const V* __restrict__ z,
                                  const V* __restrict__ r, S* __restrict__ rc,
                                  const int32_t* __restrict__ active, int csc, CellDiv cd) {
  // rows of a sample that share z and face lines run on one XCD
  const long long g = (long long)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int mc = m / 2, half = m / 2;
  const long long nc = (long long)mc * mc * mc, n = (long long)m * m * m;
  int I, J, L;
  const long long s = split_cell(g, nc, cd, I, J, L);
  if (!active[s]) return;
  const S* Te = T + s * 3 * n;  // east, north and up faces
  const S* Tn = Te + n;
  const S* Tu = Tn + n;
  const S* tbs = tb + s * 3 * m * m;
  const V* zs = z + s * n;
  const V* rs = r + s * n;
  const int nh = (int)(n / 2), mm = m * m;
  // colour-split position of cell 2I + a of row (jj, ll); 2I - 1 sits one
  // before that of 2I + 1, 2I + 2 one after that of 2I
  auto pos = [&](int a, int jj, int ll) -> int {
    return ((a + jj + ll) & 1) * nh + (ll * m + jj) * half + I;
  };
  const int j0 = 2 * J, l0 = 2 * L;
  const bool hasW = I > 0, hasE = I < mc - 1, hasS = J > 0, hasN = J < mc - 1, hasD = L > 0,
             hasU = L < mc - 1;
  // rows by (dl, dj) = (ll - l0 + 1, jj - j0 + 1): the block's rows are 1..2 in
  // both, the rows beside it 0 and 3 in one of them
  V zv[4][4][2], rv[2][2][2], zw[2][2], ze[2][2];
  S te[4][4][2], tn[4][4][2], tu[4][4][2], tew[2][2];
#pragma unroll
  for (int cc = 0; cc < 2; ++cc)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      const int jj = j0 + bb, ll = l0 + cc;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int q = pos(a, jj, ll);
        zv[cc + 1][bb + 1][a] = zs[q];
        rv[cc][bb][a] = rs[q];
        te[cc + 1][bb + 1][a] = Te[q];
        tn[cc + 1][bb + 1][a] = Tn[q];
        tu[cc + 1][bb + 1][a] = Tu[q];
      }
      zw[cc][bb] = hasW ? zs[pos(1, jj, ll) - 1] : V(0);
      tew[cc][bb] = hasW ? Te[pos(1, jj, ll) - 1] : S(0);
      ze[cc][bb] = hasE ? zs[pos(0, jj, ll) + 1] : V(0);
    }
#pragma unroll
  for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      zv[c2 + 1][0][a] = hasS ? zs[pos(a, j0 - 1, l0 + c2)] : V(0);
      tn[c2 + 1][0][a] = hasS ? Tn[pos(a, j0 - 1, l0 + c2)] : S(0);
      zv[c2 + 1][3][a] = hasN ? zs[pos(a, j0 + 2, l0 + c2)] : V(0);
      zv[0][c2 + 1][a] = hasD ? zs[pos(a, j0 + c2, l0 - 1)] : V(0);
      tu[0][c2 + 1][a] = hasD ? Tu[pos(a, j0 + c2, l0 - 1)] : S(0);
      zv[3][c2 + 1][a] = hasU ? zs[pos(a, j0 + c2, l0 + 2)] : V(0);
    }
  S acc = S(0);
#pragma unroll
  for (int cc = 0; cc < 2; ++cc)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int dl = cc + 1, dj = bb + 1;
        const int i = 2 * I + a, j = j0 + bb, l = l0 + cc;
        Faces3T<S> f;
        f.te = te[dl][dj][a];
        f.tw = a == 1 ? te[dl][dj][0] : (hasW ? tew[cc][bb] : tbs[l * m + j]);
        f.tn = tn[dl][dj][a];
        f.ts = (bb == 1 || hasS) ? tn[dl][dj - 1][a] : tbs[mm + l * m + i];
        f.tu = tu[dl][dj][a];
        f.td = (cc == 1 || hasD) ? tu[dl - 1][dj][a] : tbs[2 * mm + j * m + i];
        S o = S(0);
        if (i < m - 1) o += f.te * (S)(a == 0 ? zv[dl][dj][1] : ze[cc][bb]);
        if (i > 0) o += f.tw * (S)(a == 1 ? zv[dl][dj][0] : zw[cc][bb]);
        if (j < m - 1) o += f.tn * (S)zv[dl][dj + 1][a];
        if (j > 0) o += f.ts * (S)zv[dl][dj - 1][a];
        if (l < m - 1) o += f.tu * (S)zv[dl + 1][dj][a];
        if (l > 0) o += f.td * (S)zv[dl - 1][dj][a];
        acc += (S)rv[cc][bb][a] - (diag3(f) * (S)zv[dl][dj][a] - o);
      }
  rc[csc ? s * nc + cs3_index(mc, I, J, L) : g] = acc;
}

template <class S, class V>
static void resid_restrict3_t(hipStream_t st, int m, int batch, const void* T, const void* tb,
                              const void* z, const void* r, void* rc, const int32_t* active,
                              int csc) {
  const long long total = (long long)batch * (m / 2) * (m / 2) * (m / 2);
  const CellDiv cd = make_celldiv(total, (long long)(m / 2) * (m / 2) * (m / 2), m / 2);
  hipLaunchKernelGGL((k_resid_restrict3<S, V>), dim3(blocks_for(total)), dim3(kBlock), 0, st, m,
                     total, (const S*)T, (const S*)tb, (const V*)z, (const V*)r, (S*)rc, active,
                     csc, cd);
}

void launch_resid_restrict3_p(hipStream_t st, bool f32, bool top, int m, int batch,
                              const void* T, const void* tb, const void* z, const void* r,
                              void* rc, const int32_t* active, bool coarse_split) {
  const int csc = coarse_split ? 1 : 0;
  if (!f32) resid_restrict3_t<double, double>(st, m, batch, T, tb, z, r, rc, active, csc);
  else if (top) resid_restrict3_t<float, double>(st, m, batch, T, tb, z, r, rc, active, csc);
  else resid_restrict3_t<float, float>(st, m, batch, T, tb, z, r, rc, active, csc);
}

// z = A^-1 r on the coarsest grid for vectors of a reduced-precision
// hierarchy: FP64 inverse and sums, r and z in float.
__global__ void k_dense_apply3f(int n, long long total, const double* __restrict__ Ainv,
                                const float* __restrict__ r, float* __restrict__ z,
                                const int32_t* __restrict__ active) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long long s = g / n;
  if (!active[s]) return;
  const int q = (int)(g - s * n);
  const double* A = Ainv + s * n * n + (long long)q * n;
  const float* rs = r + s * n;
  double acc = 0.0;
  for (int p = 0; p < n; ++p) acc += A[p] * (double)rs[p];
  z[g] = (float)acc;
}

void launch_dense_apply3f(hipStream_t st, int n, int batch, const double* Ainv, const float* r,
                          float* z, const int32_t* active) {
  const long long total = (long long)batch * n;
  hipLaunchKernelGGL(k_dense_apply3f, dim3(blocks_for(total)), dim3(kBlock), 0, st, n, total,
                     Ainv, r, z, active);
}

// ------------------------------------------------------------------ coarse cycle in LDS
// One workgroup per sample runs the V- or W-cycle on the levels l0..L of a
// 3-D hierarchy with every level's operator and vectors in LDS, instead of one
// launch per sweep on these small grids.  FP64 hierarchy: levels of side <= 8
// in FP64 (about 53 KB), 256 threads.  FP32 hierarchy: levels of side <= 16
// in FP32, the arithmetic of its per-sweep kernels (about 143 KB, one
// workgroup per CU, so 1024 threads cost no occupancy: two cells per thread
// and sweep at 16^3).  Level arrays use a padded (m + 2)^3 layout
// with a one-cell ring: ring cells hold z = 0 and the boundary faces (west face
// at i = -1, south face at j = -1, bottom face at l = -1), so the stencil needs
// no branches.  Same steps and order as the per-sweep cycle.
template <class E>
struct Lds3Cfg;
template <>
struct Lds3Cfg<double> {
  static constexpr int kMax = 8, kThreads = 256;
  // 5 (m + 2)^3 words for m = 8, 4, 2, 1
  static constexpr int kWords = 5 * (1000 + 216 + 64 + 27);
};
template <>
struct Lds3Cfg<float> {
  static constexpr int kMax = 16, kThreads = 1024;
  static constexpr int kWords = 5 * (5832 + 1000 + 216 + 64 + 27);
};

struct Lds3Level {
  int m, P, off;  // size, padded pitch (m + 2), offset of the level's arrays
  float inv_m, inv_half;  // 1 / m and 1 / max(m / 2, 1), the divisors of div_small
};

__device__ __forceinline__ int pidx3(int P, int i, int j, int l) {
  return ((l + 1) * P + (j + 1)) * P + (i + 1);
}

// arrays of a level: te, tn, tu, r, z, each P^3 words
template <class E, int NT>
__device__ void c3_sweep(E* a, const Lds3Level& lq, int color, bool zero) {
  const int m = lq.m, P = lq.P;
  const int PPP = P * P * P, PP = P * P;
  E* te = a;
  E* tn = a + PPP;
  E* tu = a + 2 * PPP;
  E* rr = a + 3 * PPP;
  E* zz = a + 4 * PPP;
  const int half = m / 2 > 0 ? m / 2 : 1;
  const int cnt = m * m * half;
  // quotients through one FP32 multiply (exact for these small operands)
  for (int c = threadIdx.x; c < cnt; c += NT) {
    const int row = div_small(c, lq.inv_half);  // row = l m + j
    const int l = div_small(row, lq.inv_m), j = row - l * m;
    const int i = 2 * (c - row * half) + ((j + l + color) & 1);
    if (i >= m) continue;
    const int f = pidx3(P, i, j, l);
    const E d = te[f] + te[f - 1] + tn[f] + tn[f - P] + tu[f] + tu[f - PP];
    if (zero) {
      zz[f] = rr[f] / d;
    } else {
      const E ns = te[f] * zz[f + 1] + te[f - 1] * zz[f - 1] + tn[f] * zz[f + P] +
                   tn[f - P] * zz[f - P] + tu[f] * zz[f + PP] + tu[f - PP] * zz[f - PP];
      zz[f] = (rr[f] + ns) / d;
    }
  }
  __syncthreads();
}

// Padded operator image of the in-LDS levels, built once per solve: per
// sample and level q the arrays te, tn, tu of the kernel's LDS layout ((m + 2)^3
// words each, boundary faces on the ring, zeros elsewhere), so that each cycle
// launch copies them linearly instead of gathering from the hierarchy.
int coarse3_image_words(int nlev, const int* ms) {
  int w = 0;
  for (int q = 0; q < nlev; ++q) w += 3 * (ms[q] + 2) * (ms[q] + 2) * (ms[q] + 2);
  return w;
}

template <class S, class E>
__global__ void k_coarse3_image(int nlev, CoarseDesc desc, long long total, int words,
                                E* __restrict__ img) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long long s = g / words;
  int w = (int)(g - s * words);
  int q = 0, P = desc.m[0] + 2;
  while (w >= 3 * P * P * P) {
    w -= 3 * P * P * P;
    ++q;
    P = desc.m[q] + 2;
  }
  const int m = desc.m[q], PPP = P * P * P, mm = m * m;
  const int arr = w / PPP, f = w - arr * PPP;
  const int row = f / P, lp = row / P;  // row = (l + 1) P + (j + 1)
  const int i = f - row * P - 1, j = row - lp * P - 1, l = lp - 1;
  const bool ii = i >= 0 && i < m, jj = j >= 0 && j < m, ll = l >= 0 && l < m;
  const long long n = (long long)mm * m;
  const long long c = ((long long)l * m + j) * m + i;
  const S* Ts = static_cast<const S*>(desc.T[q]) + s * 3 * n;
  const S* tbs = static_cast<const S*>(desc.tb[q]) + s * 3 * mm;
  E v = E(0);
  if (arr == 0 && jj && ll) v = i == -1 ? (E)tbs[l * m + j] : (ii ? (E)Ts[c] : E(0));
  if (arr == 1 && ii && ll) v = j == -1 ? (E)tbs[mm + l * m + i] : (jj ? (E)Ts[n + c] : E(0));
  if (arr == 2 && ii && jj) v = l == -1 ? (E)tbs[2 * mm + j * m + i] : (ll ? (E)Ts[2 * n + c] : E(0));
  img[g] = v;
}

void launch_coarse3_image(hipStream_t st, bool f32, int batch, int nlev, const CoarseDesc& desc,
                          void* img) {
  const int words = coarse3_image_words(nlev, desc.m);
  const long long total = (long long)batch * words;
  if (f32)
    hipLaunchKernelGGL((k_coarse3_image<float, float>), dim3(blocks_for(total)), dim3(kBlock), 0,
                       st, nlev, desc, total, words, (float*)img);
  else
    hipLaunchKernelGGL((k_coarse3_image<double, double>), dim3(blocks_for(total)), dim3(kBlock),
                       0, st, nlev, desc, total, words, (double*)img);
}

// S: storage type of the hierarchy; V: type of the first level's r and z;
// E: LDS and arithmetic type.
template <class S, class V, class E>
__global__ void __launch_bounds__(Lds3Cfg<E>::kThreads)
k_coarse3_cycle(int nlev, CoarseDesc desc, const E* __restrict__ img, int img_words,
                const V* __restrict__ r0, V* __restrict__ z0,
                const double* __restrict__ Ainv, double omega, unsigned wmask,
                const int32_t* __restrict__ active) {
  constexpr int NT = Lds3Cfg<E>::kThreads;
  __shared__ E lds[Lds3Cfg<E>::kWords];
  const int s = blockIdx.x;
  if (!active[s]) return;
  // the level table in LDS: the loops below index it by the running level, a
  // per-thread array would live in scratch memory
  __shared__ Lds3Level lv[kMaxCoarseLevels];
  // One phase before the cycle: the level table (thread 0), the operators from
  // the image (linear copy), z zero (its frame is read as the boundary cells'
  // neighbours), and r of the first level from r0.  The frame of r is never
  // read, and the restriction writes the interior of a coarser level's r
  // before it is read, so r is not cleared.  Each thread issues its global
  // loads in groups of kCopyU before storing any of them, so a group costs one
  // memory latency instead of one per word (one workgroup per CU: nothing else
  // hides that latency).
  constexpr int kCopyU = 8;
  const E* im = img + (long long)s * img_words;
  int off = 0;
  for (int q = 0; q < nlev; ++q) {
    const int mq = desc.m[q], P = mq + 2, PPP = P * P * P;
    if (threadIdx.x == 0)
      lv[q] = Lds3Level{mq, P, off, 1.0f / (float)mq, 1.0f / (float)(mq / 2 > 0 ? mq / 2 : 1)};
    E* a = lds + off;
    for (int w0 = threadIdx.x; w0 < 3 * PPP; w0 += kCopyU * NT) {
      E v[kCopyU];
#pragma unroll
      for (int u = 0; u < kCopyU; ++u) {
        const int w = w0 + u * NT;
        v[u] = w < 3 * PPP ? im[w] : E(0);
      }
#pragma unroll
      for (int u = 0; u < kCopyU; ++u) {
        const int w = w0 + u * NT;
        if (w < 3 * PPP) a[w] = v[u];
      }
    }
    for (int w = threadIdx.x; w < PPP; w += NT) a[4 * PPP + w] = E(0);
    im += 3 * PPP;
    off += 5 * PPP;
  }
  {
    const int m = desc.m[0], P = m + 2, PPP = P * P * P;
    E* rr = lds + 3 * PPP;  // level 0 sits at offset 0
    const int n = m * m * m;
    const float inv_m = 1.0f / (float)m;
    for (int c0 = threadIdx.x; c0 < n; c0 += kCopyU * NT) {
      V v[kCopyU];
#pragma unroll
      for (int u = 0; u < kCopyU; ++u) {
        const int c = c0 + u * NT;
        v[u] = c < n ? r0[(long long)s * n + c] : V(0);
      }
#pragma unroll
      for (int u = 0; u < kCopyU; ++u) {
        const int c = c0 + u * NT;
        if (c < n) {
          const int row = div_small(c, inv_m), i = c - row * m;  // row = l m + j
          const int l = div_small(row, inv_m), j = row - l * m;
          rr[pidx3(P, i, j, l)] = (E)v[u];
        }
      }
    }
  }
  __syncthreads();
  // V/W-cycle without recursion, as in 2-D (bit q of wmask: level q takes two
  // coarse visits; a second visit re-smooths with a black sweep only).
  unsigned once = 0;
  int q = 0;
  bool descending = true;
  for (;;) {
    const int m = lv[q].m, P = lv[q].P, PPP = P * P * P, PP = P * P;
    E* a = lds + lv[q].off;
    E* te = a;
    E* tn = a + PPP;
    E* tu = a + 2 * PPP;
    E* rr = a + 3 * PPP;
    E* zz = a + 4 * PPP;
    if (q == nlev - 1) {
      const int nc = m * m * m;
      // row c of the inverse by the 16 lanes t = 16 c + k (entries k, k + 16, ...),
      // summed over the lane group; groups never straddle the loop bound
      // (nc <= 64: at most four entries per lane, loaded before the sum)
      const double* A = Ainv + (long long)s * nc * nc;
      for (int t = threadIdx.x; t < 16 * nc; t += NT) {
        const int c = t >> 4, k = t & 15;
        double av[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          av[u] = k + 16 * u < nc ? A[(long long)c * nc + k + 16 * u] : 0.0;
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int p2 = k + 16 * u;
          if (p2 < nc) acc += av[u] * (double)rr[pidx3(P, p2 % m, (p2 / m) % m, p2 / (m * m))];
        }
        acc += __shfl_xor(acc, 8, 16);
        acc += __shfl_xor(acc, 4, 16);
        acc += __shfl_xor(acc, 2, 16);
        acc += __shfl_xor(acc, 1, 16);
        if (k == 0) zz[pidx3(P, c % m, (c / m) % m, c / (m * m))] = (E)acc;
      }
      __syncthreads();
      if (q == 0) break;
      --q;
      descending = false;
      continue;
    }
    if (descending) {
      c3_sweep<E, NT>(a, lv[q], 0, true);
      c3_sweep<E, NT>(a, lv[q], 1, false);
    } else {
      const int Pc = lv[q + 1].P, PPPc = Pc * Pc * Pc;
      const E* zc = lds + lv[q + 1].off + 4 * PPPc;
      const E om = (E)omega;
      const float inv_m = lv[q].inv_m;
      for (int c = threadIdx.x; c < m * m * m; c += NT) {
        const int row = div_small(c, inv_m), i = c - row * m;  // row = l m + j
        const int l = div_small(row, inv_m), j = row - l * m;
        zz[pidx3(P, i, j, l)] += om * zc[pidx3(Pc, i / 2, j / 2, l / 2)];
      }
      __syncthreads();
      c3_sweep<E, NT>(a, lv[q], 1, false);
      c3_sweep<E, NT>(a, lv[q], 0, false);
      if (!(wmask >> q & 1u) || (once >> q & 1u)) {
        once &= ~(1u << q);
        if (q == 0) break;
        --q;
        continue;
      }
      once |= 1u << q;
      c3_sweep<E, NT>(a, lv[q], 1, false);
    }
    // residual, restricted to the next level (sum over the 2 x 2 x 2 block)
    const int mc = lv[q + 1].m, Pc = lv[q + 1].P, PPPc = Pc * Pc * Pc;
    E* rc = lds + lv[q + 1].off + 3 * PPPc;
    // one fine cell per lane, t = 8 c + (aa + 2 bb + 4 cc), summed over the
    // 8-lane group of coarse cell c (groups never straddle the loop bound)
    const float inv_mc = lv[q + 1].inv_m;
    for (int t = threadIdx.x; t < 8 * mc * mc * mc; t += NT) {
      const int c = t >> 3, k = t & 7;
      const int row = div_small(c, inv_mc), I = c - row * mc;  // row = L mc + J
      const int L = div_small(row, inv_mc), J = row - L * mc;
      const int f = pidx3(P, 2 * I + (k & 1), 2 * J + ((k >> 1) & 1), 2 * L + (k >> 2));
      const E d = te[f] + te[f - 1] + tn[f] + tn[f - P] + tu[f] + tu[f - PP];
      E v = rr[f] - (d * zz[f] - (te[f] * zz[f + 1] + te[f - 1] * zz[f - 1] + tn[f] * zz[f + P] +
                                  tn[f - P] * zz[f - P] + tu[f] * zz[f + PP] +
                                  tu[f - PP] * zz[f - PP]));
      v += __shfl_xor(v, 4, 8);
      v += __shfl_xor(v, 2, 8);
      v += __shfl_xor(v, 1, 8);
      if (k == 0) rc[pidx3(Pc, I, J, L)] = v;
    }
    __syncthreads();
    ++q;
    descending = true;
  }
  {
    const int m = lv[0].m, P = lv[0].P, PPP = P * P * P;
    const E* zz = lds + lv[0].off + 4 * PPP;
    const long long n = (long long)m * m * m;
    for (int c = threadIdx.x; c < n; c += NT)
      z0[(long long)s * n + c] = (V)zz[pidx3(P, c % m, (c / m) % m, c / (m * m))];
  }
}

int coarse3_max_side(bool f32) { return f32 ? Lds3Cfg<float>::kMax : Lds3Cfg<double>::kMax; }

void launch_coarse3_cycle(hipStream_t st, bool f32, bool top, int batch, int nlev,
                          const CoarseDesc& desc, const void* img, const void* r0, void* z0,
                          const double* Ainv, double omega, unsigned wmask,
                          const int32_t* active) {
  const int words = coarse3_image_words(nlev, desc.m);
  if (!f32)
    hipLaunchKernelGGL((k_coarse3_cycle<double, double, double>), dim3(batch),
                       dim3(Lds3Cfg<double>::kThreads), 0, st, nlev, desc, (const double*)img,
                       words, (const double*)r0, (double*)z0, Ainv, omega, wmask, active);
  else if (top)
    hipLaunchKernelGGL((k_coarse3_cycle<float, double, float>), dim3(batch),
                       dim3(Lds3Cfg<float>::kThreads), 0, st, nlev, desc, (const float*)img,
                       words, (const double*)r0, (double*)z0, Ainv, omega, wmask, active);
  else
    hipLaunchKernelGGL((k_coarse3_cycle<float, float, float>), dim3(batch),
                       dim3(Lds3Cfg<float>::kThreads), 0, st, nlev, desc, (const float*)img,
                       words, (const float*)r0, (float*)z0, Ainv, omega, wmask, active);
}

// ------------------------------------------------------------------ coarsest grid
// Explicit inverse of each sample's coarsest matrix (n = m^3 <= 64) by
// Gauss-Jordan elimination without pivoting (SPD), as in 2-D.  256 threads
// per sample; thread t holds column j = t mod n of the rows t / n + q P
// (P = 256 / n rows per pass, at most 16 entries) in registers.  Step k
// publishes column k and the scaled pivot row in LDS, then every thread
// updates its entries: no index division inside the elimination.
constexpr int kDenseThreads3 = 256;
__global__ void __launch_bounds__(kDenseThreads3)
k_dense_factor3(int m, int batch, const double* __restrict__ T, const double* __restrict__ tb,
                double* __restrict__ Ainv) {
  __shared__ double A[64 * 64];
  __shared__ double col[64], prow[64];
  const int s = blockIdx.x;
  if (s >= batch) return;
  const int n = m * m * m, mm = m * m;
  const double* Ts = T + (long long)s * 3 * n;
  const double* tbs = tb + (long long)s * 3 * mm;
  for (int q = threadIdx.x; q < n * n; q += kDenseThreads3) A[q] = 0.0;
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += kDenseThreads3) {
    int i, j, l;
    cell_of(c, m, i, j, l);
    const Faces3 f = load_faces3(Ts, tbs, m, i, j, l);
    A[c * n + c] = diag3(f);
    if (i < m - 1) A[c * n + c + 1] = A[(c + 1) * n + c] = -f.te;
    if (j < m - 1) A[c * n + c + m] = A[(c + m) * n + c] = -f.tn;
    if (l < m - 1) A[c * n + c + mm] = A[(c + mm) * n + c] = -f.tu;
  }
  __syncthreads();
  constexpr int kMaxRows = 16;
  const int P = kDenseThreads3 / n;                   // rows per pass (n <= 64: P >= 4)
  const int t = threadIdx.x;
  const bool on = t < P * n;
  const int j = on ? t % n : 0, i0 = on ? t / n : 0;
  double a[kMaxRows];
#pragma unroll
  for (int q = 0; q < kMaxRows; ++q) {
    const int i = i0 + q * P;
    a[q] = (on && i < n) ? A[i * n + j] : 0.0;
  }
  for (int k = 0; k < n; ++k) {
    // column k of the current matrix
    if (on && j == k) {
#pragma unroll
      for (int q = 0; q < kMaxRows; ++q)
        if (i0 + q * P < n) col[i0 + q * P] = a[q];
    }
    __syncthreads();
    const double piv = col[k];
    // row k divided by the pivot (its column-k entry becomes 1 / piv)
    if (on && i0 == k % P) {
      const int q = k / P;
#pragma unroll
      for (int qq = 0; qq < kMaxRows; ++qq)
        if (qq == q) prow[j] = (j == k ? 1.0 : a[qq]) / piv;
    }
    __syncthreads();
    if (on) {
      const double pk = prow[j];
#pragma unroll
      for (int q = 0; q < kMaxRows; ++q) {
        const int i = i0 + q * P;
        if (i < n) a[q] = i == k ? pk : (j == k ? 0.0 : a[q]) - col[i] * pk;
      }
    }
    __syncthreads();
  }
  double* X = Ainv + (long long)s * n * n;
  if (on) {
#pragma unroll
    for (int q = 0; q < kMaxRows; ++q) {
      const int i = i0 + q * P;
      if (i < n) X[i * n + j] = a[q];
    }
  }
}

void launch_dense_factor3(hipStream_t st, int m, int batch, const double* T, const double* tb,
                          double* Ainv) {
  hipLaunchKernelGGL(k_dense_factor3, dim3(batch), dim3(kDenseThreads3), 0, st, m, batch, T, tb,
                     Ainv);
}

// ------------------------------------------------------------------ PCG stencil kernels
// Block b of sample s (blockIdx.x = s * bps + b) owns cells b*1024 + t + 256 c of
// the sample in natural order, with the faces in natural order; p and q in
// colour-split order when CS is set (each wave then reads and writes two
// half-wave runs, one per colour, and every face line is used by both colours
// at once).
template <bool CS>
__global__ void __launch_bounds__(kBlock)
k_spmv3_dot(int m, const double* __restrict__ T, const double* __restrict__ tb,
            const double* __restrict__ p, double* __restrict__ q, double* __restrict__ partial,
            int bps, const int32_t* __restrict__ active) {
  __shared__ double sh[kBlock / kWave];
  // blocks of neighbouring rows and planes run on one XCD
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const long long s = lb / bps;
  const int blk = lb - (int)(s * bps);
  if (!active[s]) return;
  const long long n = (long long)m * m * m;
  const double* Ts = T + s * 3 * n;
  const double* tbs = tb + s * 3 * m * m;
  const double* ps = p + s * n;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < kCellsPerThread; ++c) {
    const long long cell = (long long)blk * kCellsPerBlock + threadIdx.x + c * kBlock;
    if (cell < n) {
      int i, j, l;
      // entry e of p and q
      cell_of(cell, m, i, j, l);
      const long long e = CS ? cs3_index(m, i, j, l) : cell;
      const Faces3 f = load_faces3(Ts, tbs, m, i, j, l);
      const double v =
          diag3(f) * ps[e] - (CS ? nsum3_cs(ps, m, i, j, l, f) : nsum3(ps, m, i, j, l, f));
      q[s * n + e] = v;
      acc += ps[e] * v;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[lb] = t;
}

void launch_spmv3_dot(hipStream_t st, int m, int batch, const double* T, const double* tb,
                      const double* p, double* q, double* partial, int bps,
                      const int32_t* active, bool split) {
  if (split)
    hipLaunchKernelGGL(k_spmv3_dot<true>, dim3(batch * bps), dim3(kBlock), 0, st, m, T, tb, p, q,
                       partial, bps, active);
  else
    hipLaunchKernelGGL(k_spmv3_dot<false>, dim3(batch * bps), dim3(kBlock), 0, st, m, T, tb, p,
                       q, partial, bps, active);
}

// Ts (colour-split order, type S) = T (natural order, FP64), the three face
// arrays of each sample; one thread per destination entry.
template <class S>
__global__ void k_faces_split3(int m, long long total, const double* __restrict__ T,
                               S* __restrict__ Ts) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long long n = (long long)m * m * m;
  const long long a = g / n;  // sample * 3 + face array
  const long long e = g - a * n;
  int i, j, l;
  cs3_cell(m, e, i, j, l);
  Ts[g] = (S)T[a * n + ((long long)l * m + j) * m + i];
}

void launch_faces_split3(hipStream_t st, bool f32, int m, int batch, const double* T, void* Ts) {
  const long long total = (long long)batch * 3 * m * m * m;
  if (f32)
    hipLaunchKernelGGL(k_faces_split3<float>, dim3(blocks_for(total)), dim3(kBlock), 0, st, m,
                       total, T, (float*)Ts);
  else
    hipLaunchKernelGGL(k_faces_split3<double>, dim3(blocks_for(total)), dim3(kBlock), 0, st, m,
                       total, T, (double*)Ts);
}

// x = 0 and r = b with r in colour-split order (b natural), and the partial
// sums of b^2 per block, as k_pcg_init does in the natural order (only: the
// samples to start, or null for all).
__global__ void __launch_bounds__(kBlock)
k_pcg_init3_split(int m, const double* __restrict__ b, double* __restrict__ x,
                  double* __restrict__ r, double* __restrict__ partial, int bps,
                  const int32_t* __restrict__ only) {
  __shared__ double sh[kBlock / kWave];
  // blocks of neighbouring rows and planes run on one XCD
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const long long s = lb / bps;
  const int blk = lb - (int)(s * bps);
  if (only && !only[s]) return;
  const long long n = (long long)m * m * m;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < kCellsPerThread; ++c) {
    const long long e = (long long)blk * kCellsPerBlock + threadIdx.x + c * kBlock;
    if (e < n) {
      int i, j, l;
      cs3_cell(m, e, i, j, l);
      const double v = b[s * n + ((long long)l * m + j) * m + i];
      x[s * n + e] = 0.0;
      r[s * n + e] = v;
      acc += v * v;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[lb] = t;
}

void launch_pcg_init3_split(hipStream_t st, int m, int batch, const double* b, double* x,
                            double* r, double* partial, int bps, const int32_t* only) {
  hipLaunchKernelGGL(k_pcg_init3_split, dim3(batch * bps), dim3(kBlock), 0, st, m, b, x, r,
                     partial, bps, only);
}

// out (natural order) = in (colour-split order), one thread per cell.
__global__ void k_from_split3(int m, long long total, const double* __restrict__ in,
                              double* __restrict__ out, CellDiv cd) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long long n = (long long)m * m * m;
  int i, j, l;
  const long long s = split_cell(g, n, cd, i, j, l);
  out[g] = in[s * n + cs3_index(m, i, j, l)];
}

void launch_from_split3(hipStream_t st, int m, int batch, const double* in, double* out) {
  const long long n = (long long)m * m * m, total = (long long)batch * n;
  const CellDiv cd = make_celldiv(total, n, m);
  hipLaunchKernelGGL(k_from_split3, dim3(blocks_for(total)), dim3(kBlock), 0, st, m, total, in,
                     out, cd);
}

__global__ void __launch_bounds__(kBlock)
k_true_residual3(int m, const double* __restrict__ T, const double* __restrict__ tb,
                 const double* __restrict__ b, const double* __restrict__ x,
                 double* __restrict__ partial, int bps) {
  __shared__ double sh[kBlock / kWave];
  // blocks of neighbouring rows and planes run on one XCD
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const long long s = lb / bps;
  const int blk = lb - (int)(s * bps);
  const long long n = (long long)m * m * m;
  const double* Ts = T + s * 3 * n;
  const double* tbs = tb + s * 3 * m * m;
  const double* xs = x + s * n;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < kCellsPerThread; ++c) {
    const long long cell = (long long)blk * kCellsPerBlock + threadIdx.x + c * kBlock;
    if (cell < n) {
      int i, j, l;
      cell_of(cell, m, i, j, l);
      const Faces3 f = load_faces3(Ts, tbs, m, i, j, l);
      const double rv = b[s * n + cell] - (diag3(f) * xs[cell] - nsum3(xs, m, i, j, l, f));
      acc += rv * rv;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[lb] = t;
}

void launch_true_residual3(hipStream_t st, int m, int batch, const double* T, const double* tb,
                           const double* b, const double* x, double* partial, int bps) {
  hipLaunchKernelGGL(k_true_residual3, dim3(batch * bps), dim3(kBlock), 0, st, m, T, tb, b, x,
                     partial, bps);
}

// ------------------------------------------------------------------ fields
// Example 1 (piecewise constant layers) on the m^3 centres.
__global__ void k_field_pc3(int kind, int n_nodes, int m, long long total,
                            const double* __restrict__ params, double* __restrict__ k) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long long n = (long long)m * m * m;
  const long long s = g / n;
  int i, j, l;
  cell_of(g - s * n, m, i, j, l);
  const double* prm = params + s * kParamStride;
  const int ly = layer_of3(kind, n_nodes, prm, centre(i, m), centre(j, m), centre(l, m));
  k[g] = exp(prm[8 + ly]);
}

void launch_field_pc3(hipStream_t st, const mlmc_model& mdl, int m, int batch,
                      const double* params, double* k) {
  const long long total = (long long)batch * m * m * m;
  hipLaunchKernelGGL(k_field_pc3, dim3(blocks_for(total)), dim3(kBlock), 0, st,
                     mdl.interface_kind, mdl.n_nodes, m, total, params, k);
}

// ---- circulant embedding in 3-D: c, Lambda = FFT3(c), sqrt(Lambda / n^3)
// c[a3][a2][a1] = sigma2 exp(-||(d1, d2, d3)||_r / lambda), d = min(a, n - a) h  (eq. (2.3))
__global__ void k_ce_first_row3(int n, int m, double sigma2, double lambda, int norm_r,
                                double2* __restrict__ c) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nn = (long long)n * n;
  if (g >= nn * n) return;
  const int a3 = (int)(g / nn);
  const int r2 = (int)(g - (long long)a3 * nn);
  const int a2 = r2 / n, a1 = r2 - a2 * n;
  const double h = 1.0 / (double)m;
  const double d1 = (double)min(a1, n - a1) * h;
  const double d2 = (double)min(a2, n - a2) * h;
  const double d3 = (double)min(a3, n - a3) * h;
  const double dist = norm_r == 1 ? d1 + d2 + d3 : sqrt(d1 * d1 + d2 * d2 + d3 * d3);
  c[g] = make_double2(sigma2 * exp(-dist / lambda), 0.0);
}

void launch_ce_first_row3(hipStream_t st, int n, int m, double sigma2, double lambda, int norm_r,
                          double2* c) {
  const long long total = (long long)n * n * n;
  hipLaunchKernelGGL(k_ce_first_row3, dim3(blocks_for(total)), dim3(kBlock), 0, st, n, m, sigma2,
                     lambda, norm_r, c);
}

__global__ void k_ce_sqrt3(const double2* __restrict__ lam, long long count, double n3,
                           double* __restrict__ sq) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  sq[g] = sqrt(fmax(lam[g].x, 0.0) / n3);
}

void launch_ce_sqrt3(hipStream_t st, const double2* lam, int n, double* sq) {
  const long long total = (long long)n * n * n;
  const double n3 = (double)n * (double)n * (double)n;
  hipLaunchKernelGGL(k_ce_sqrt3, dim3(blocks_for(total)), dim3(kBlock), 0, st, lam, total, n3,
                     sq);
}

// Pass A: L consecutive noise rows r = k3 n + k2 (lines along x1) of one
// sample: xi(k1) = (z0, z1) of Philox block (r/2) n + k1 for even r, (z2, z3)
// for odd r; scaled by sqrt(Lambda / n^3); FFT along x1; the first m outputs
// to u1[s][r][j1].  P: L is even (so r0 is), and a thread draws one block for
// the row pair (r, r + 1) and fills both lines; otherwise each row draws its
// own block and keeps half of it.  C = 0: one line per workgroup, fft_line
// (T = kBlock); otherwise fft_lines<C, T>.
template <int C, int T, bool P>
__global__ void __launch_bounds__(T)
k_ce3_pass_a(uint64_t seed, uint32_t tag, uint32_t level, uint64_t first,
             const uint32_t* __restrict__ ids,
             int m, const double* __restrict__ sq, const double2* __restrict__ tw, FftPlan pl,
             int L, int groups, double2* __restrict__ u1) {
  extern __shared__ double lds[];
  const int n = pl.n;
  double* sre = lds;
  double* sim = lds + L * n;
  const int s = blockIdx.x / groups;
  const int r0 = (blockIdx.x - s * groups) * L;
  const int rows = n * n;
  const int lines = min(L, rows - r0);
  const uint32_t sample = ids ? ids[s] : (uint32_t)(first + (uint64_t)s);
  const float inv_n = 1.0f / (float)n;
  if constexpr (P) {
    for (int t = threadIdx.x; t < (L / 2) * n; t += T) {
      const int pp = div_small(t, inv_n);
      const int k1 = t - pp * n;
      const int q = 2 * pp;
      double zr = 0.0, zi = 0.0, wr = 0.0, wi = 0.0;
      if (q < lines) {
        const int r = r0 + q;
        const U4 bk = stream_block(seed, (uint32_t)(r / 2) * (uint32_t)n + (uint32_t)k1, sample,
                                   level, tag);
        box_muller(to_uniform(bk.x), to_uniform(bk.y), zr, zi);
        const double a = sq[(long long)r * n + k1];
        zr *= a;
        zi *= a;
        if (q + 1 < lines) {
          box_muller(to_uniform(bk.z), to_uniform(bk.w), wr, wi);
          const double a1 = sq[(long long)(r + 1) * n + k1];
          wr *= a1;
          wi *= a1;
        }
      }
      sre[q * n + k1] = zr;
      sim[q * n + k1] = zi;
      sre[(q + 1) * n + k1] = wr;
      sim[(q + 1) * n + k1] = wi;
    }
  } else {
    for (int t = threadIdx.x; t < L * n; t += T) {
      const int q = div_small(t, inv_n);
      const int k1 = t - q * n;
      if (q >= lines) {
        sre[t] = 0.0;
        sim[t] = 0.0;
        continue;
      }
      const int r = r0 + q;
      const U4 bk = stream_block(seed, (uint32_t)(r / 2) * (uint32_t)n + (uint32_t)k1, sample,
                                 level, tag);
      double zr, zi;
      if ((r & 1) == 0) box_muller(to_uniform(bk.x), to_uniform(bk.y), zr, zi);
      else box_muller(to_uniform(bk.z), to_uniform(bk.w), zr, zi);
      const double a = sq[(long long)r * n + k1];
      sre[t] = a * zr;
      sim[t] = a * zi;
    }
  }
  __syncthreads();
  if constexpr (C == 0) {
    static_assert(T == kBlock, "fft_line runs on kBlock threads");
    fft_line(sre, sim, tw, pl);
  } else {
    fft_lines<C, T>(sre, sim, tw, pl, L);
  }
  double2* out = u1 + ((long long)s * rows + r0) * m;
  const float inv_m = 1.0f / (float)m;
  for (int t = threadIdx.x; t < lines * m; t += T) {
    const int q = div_small(t, inv_m);
    const int j1 = t - q * m;
    out[t] = make_double2(sre[q * n + j1], sim[q * n + j1]);
  }
}

// Pass B: lines along x2 for fixed (k3, j1), L consecutive j1 of one sample:
// u1[s][k3 n + k2][j1] -> FFT over k2 -> u2[s][k3][j2][j1], j2 < m.  The L
// lines of a workgroup are adjacent in memory, so its reads are runs of
// 16 L bytes.
template <int C, int T>
__global__ void __launch_bounds__(T)
k_ce3_pass_b(int m, const double2* __restrict__ u1, const double2* __restrict__ tw, FftPlan pl,
             int L, int groups, double2* __restrict__ u2) {
  extern __shared__ double lds[];
  const int n = pl.n;
  double* sre = lds;
  double* sim = lds + L * n;
  const int per_k3 = (m + L - 1) / L;
  // the workgroups of adjacent j1 read adjacent pieces of the same lines: one
  // XCD (and its L2) takes a contiguous range of them
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const long long s = bid / groups;
  const int rem = bid - (int)(s * groups);
  const int k3 = rem / per_k3;
  const int j1_0 = (rem - k3 * per_k3) * L;
  const int lines = min(L, m - j1_0);
  const double2* in = u1 + ((long long)s * n * n + (long long)k3 * n) * m + j1_0;
  // loads in groups of kU issued before their stores
  constexpr int kU = 8;
  for (int t0 = threadIdx.x; t0 < L * n; t0 += kU * T) {
    double2 v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + u * T;
      const int k2 = t / L, q = t - k2 * L;  // L adjacent j1 of row k2 are contiguous
      v[u] = t < L * n && q < lines ? in[(long long)k2 * m + q] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + u * T;
      const int k2 = t / L, q = t - k2 * L;
      if (t < L * n) {
        sre[q * n + k2] = v[u].x;
        sim[q * n + k2] = v[u].y;
      }
    }
  }
  __syncthreads();
  if constexpr (C == 0) {
    static_assert(T == kBlock, "fft_line runs on kBlock threads");
    fft_line(sre, sim, tw, pl);
  } else {
    fft_lines<C, T>(sre, sim, tw, pl, L);
  }
  double2* out = u2 + ((long long)s * n + k3) * m * m + j1_0;
  for (int t = threadIdx.x; t < lines * m; t += T) {
    const int j2 = t / lines, q = t - j2 * lines;
    out[(long long)j2 * m + q] = make_double2(sre[q * n + j2], sim[q * n + j2]);
  }
}

// Pass C: lines along x3 for fixed (j2, j1), L consecutive j1 of one sample:
// u2[s][k3][j2][j1] -> FFT over k3 -> g at j3 < m (Re: layer 0, Im: layer 1),
// k = exp(mu_l + g_l) with l the layer of the centre, and the plain coarse
// companion (layers re-evaluated at the coarse centres, Gaussian values of the
// fine cell (2I, 2J, 2L)).
template <int C, int T>
__global__ void __launch_bounds__(T)
k_ce3_pass_c(int kind, int n_nodes, int n_layers, CePair pr, int m,
             const double2* __restrict__ u2, const double2* __restrict__ tw, FftPlan pl, int L,
             int groups, const double* __restrict__ params, double* __restrict__ k,
             double* __restrict__ kc) {
  extern __shared__ double lds[];
  const int n = pl.n;
  double* sre = lds;
  double* sim = lds + L * n;
  const int per_j2 = (m + L - 1) / L;
  // adjacent workgroups read adjacent pieces of the same lines: one XCD takes a
  // contiguous range of them
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const long long s = bid / groups;
  const int rem = bid - (int)(s * groups);
  const int j2 = rem / per_j2;
  const int j1_0 = (rem - j2 * per_j2) * L;
  const int lines = min(L, m - j1_0);
  const long long mm = (long long)m * m;
  const double2* in = u2 + (long long)s * n * mm + (long long)j2 * m + j1_0;
  // loads in groups of kU issued before their stores
  constexpr int kU = 8;
  for (int t0 = threadIdx.x; t0 < L * n; t0 += kU * T) {
    double2 v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + u * T;
      const int k3 = t / L, q = t - k3 * L;
      v[u] = t < L * n && q < lines ? in[(long long)k3 * mm + q] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + u * T;
      const int k3 = t / L, q = t - k3 * L;
      if (t < L * n) {
        sre[q * n + k3] = v[u].x;
        sim[q * n + k3] = v[u].y;
      }
    }
  }
  __syncthreads();
  if constexpr (C == 0) {
    static_assert(T == kBlock, "fft_line runs on kBlock threads");
    fft_line(sre, sim, tw, pl);
  } else {
    fft_lines<C, T>(sre, sim, tw, pl, L);
  }
  const double* prm = params + s * kParamStride;
  const int mc = m / 2;
  for (int t = threadIdx.x; t < lines * m; t += T) {
    const int j3 = t / lines, q = t - j3 * lines;
    const int j1 = j1_0 + q;
    const double g0 = sre[q * n + j3], g1 = sim[q * n + j3];
    const int ly = n_layers > 1 ? layer_of3(kind, n_nodes, prm, centre(j1, m), centre(j2, m),
                                            centre(j3, m))
                                : 0;
    if (ly == pr.l_re || ly == pr.l_im)
      k[s * mm * m + ((long long)j3 * m + j2) * m + j1] =
          exp(ly == pr.l_re ? pr.mu_re + g0 : pr.mu_im + g1);
    if (kc != nullptr && ((j1 | j2 | j3) & 1) == 0) {
      const int lc = n_layers > 1 ? layer_of3(kind, n_nodes, prm, centre(j1 / 2, mc),
                                              centre(j2 / 2, mc), centre(j3 / 2, mc))
                                  : 0;
      if (lc == pr.l_re || lc == pr.l_im)
        kc[s * (long long)mc * mc * mc + ((long long)(j3 / 2) * mc + j2 / 2) * mc + j1 / 2] =
            exp(lc == pr.l_re ? pr.mu_re + g0 : pr.mu_im + g1);
    }
  }
}

// Launch shapes of the three passes, w = the widest stage's butterflies per
// line.  Pass A's lines (along x1) are contiguous; a workgroup takes an even
// number of them, so that row pairs share their Philox blocks.  Passes B and C
// read lines across rows, a run of L adjacent values per row for L lines.
// Short lines (w <= 32): 8 lines on 256 threads, one butterfly per thread and
// stage.  Otherwise 2 lines on 192 threads with C = ceil(2 w / 192) <= 3
// butterfly slots per thread.  Measured at n = 225 and 540 (the 64^3 and 128^3
// grids, 16 and 4 samples per call): the smallest workgroups were fastest.
// Pass A on 2 lines / 192 threads: 3.8 and 10.6 ms per sampler call, against
// 4.9 and 12.6 ms on 2 lines / 384 threads and 6.0 and 17.2 ms on 4 lines /
// 384; passes B and C on 2 lines / 192 threads: 3.3 and 10.4 ms, against 3.4
// and 10.7 ms on 8 (225) or 4 (540) lines / 256 threads and 4.0 and 11.2 ms on
// one line / 192.  Wider stages take one line per 256-thread workgroup
// (fft_line) in pass A and the multi-line shape of fft_lines_per_group, or
// fft_line, in passes B and C.
static int widest_stage(const FftPlan& pl) {
  int w = 1;
  for (int st = 0; st < pl.nstages; ++st) w = std::max(w, pl.n / pl.radix[st]);
  return w;
}

template <int C, int T>
static void ce3_pass_bc(hipStream_t st, const mlmc_model& mdl, const CePair& pr, int batch, int m,
                        const double2* tw, const FftPlan& pl, int L, const double* params,
                        double2* u1, double2* u2, double* k, double* k_coarse) {
  const int n = pl.n;
  const size_t lds = 2 * (size_t)L * n * sizeof(double);
  const int gb = n * ((m + L - 1) / L);
  const int gc = m * ((m + L - 1) / L);
  hipLaunchKernelGGL((k_ce3_pass_b<C, T>), dim3(batch * gb), dim3(T), lds, st, m, u1, tw, pl, L,
                     gb, u2);
  hipLaunchKernelGGL((k_ce3_pass_c<C, T>), dim3(batch * gc), dim3(T), lds, st,
                     mdl.interface_kind, mdl.n_nodes, mdl.n_layers, pr, m, u2, tw, pl, L, gc,
                     params, k, k_coarse);
}

void launch_ce3(hipStream_t st, const mlmc_model& mdl, const CePair& pr, int level, uint64_t first,
                const uint32_t* ids, int batch, int m, const double* sq, const double2* tw,
                const FftPlan& pl, const double* params, double2* u1, double2* u2, double* k,
                double* k_coarse) {
  const int n = pl.n;
  const int L = fft_lines_per_group(pl);
  const int wide = widest_stage(pl);
  auto pass_a = [&](auto kern, int la, int ta) {
    const int ga = (n * n + la - 1) / la;
    hipLaunchKernelGGL(kern, dim3(batch * ga), dim3(ta), 2 * (size_t)la * n * sizeof(double), st,
                       mdl.seed, pr.tag, (uint32_t)level, first, ids, m, sq, tw, pl, la, ga, u1);
  };
  const int ca = (2 * wide + 191) / 192;
  if (8 * wide <= kBlock) pass_a(k_ce3_pass_a<1, kBlock, true>, 8, kBlock);
  else if (ca == 1) pass_a(k_ce3_pass_a<1, 192, true>, 2, 192);
  else if (ca == 2) pass_a(k_ce3_pass_a<2, 192, true>, 2, 192);
  else if (ca == 3) pass_a(k_ce3_pass_a<3, 192, true>, 2, 192);
  else pass_a(k_ce3_pass_a<0, kBlock, false>, 1, kBlock);
  if (8 * wide <= kBlock) {
    ce3_pass_bc<1, kBlock>(st, mdl, pr, batch, m, tw, pl, 8, params, u1, u2, k, k_coarse);
    return;
  }
  switch (ca) {
    case 1: ce3_pass_bc<1, 192>(st, mdl, pr, batch, m, tw, pl, 2, params, u1, u2, k, k_coarse); return;
    case 2: ce3_pass_bc<2, 192>(st, mdl, pr, batch, m, tw, pl, 2, params, u1, u2, k, k_coarse); return;
    case 3: ce3_pass_bc<3, 192>(st, mdl, pr, batch, m, tw, pl, 2, params, u1, u2, k, k_coarse); return;
    default: break;
  }
  if (L > 1) ce3_pass_bc<1, kBlock>(st, mdl, pr, batch, m, tw, pl, L, params, u1, u2, k, k_coarse);
  else ce3_pass_bc<0, kBlock>(st, mdl, pr, batch, m, tw, pl, 1, params, u1, u2, k, k_coarse);
}

// ---- plain coarse companion of a piecewise constant sample, CGV sub-lattices
__global__ void k_cgv_extract3(int m, long long total, const double* __restrict__ kf,
                               double* __restrict__ ksub) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int mc = m / 2;
  const long long nc = (long long)mc * mc * mc;
  const long long sa = g / nc;  // sample * 8 + a
  int I, J, L;
  cell_of(g - sa * nc, mc, I, J, L);
  const long long s = sa >> 3;
  const int a = (int)(sa & 7);
  const int i = 2 * I + (a & 1), j = 2 * J + ((a >> 1) & 1), l = 2 * L + (a >> 2);
  ksub[g] = kf[s * (long long)m * m * m + ((long long)l * m + j) * m + i];
}

void launch_cgv_extract3(hipStream_t st, int m, int batch, const double* kf, double* ksub) {
  const long long total = (long long)batch * 8 * (m / 2) * (m / 2) * (m / 2);
  hipLaunchKernelGGL(k_cgv_extract3, dim3(blocks_for(total)), dim3(kBlock), 0, st, m, total, kf,
                     ksub);
}

}  // namespace mlmc
