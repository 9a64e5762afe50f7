// Batched multigrid-preconditioned conjugate gradients on gfx950.
//
// Section 3.5 solves each sample's symmetric positive definite system with
// CG preconditioned by one multigrid cycle and stops when
// ||r_m|| / ||r_0|| < tol.  Here the multigrid is geometric and per sample:
//  * coarsening by 2 x 2 aggregation with piecewise-constant prolongation P
//    and restriction P^T; the Galerkin operator P^T A P of a two-point-flux
//    operator is again two-point-flux, with each coarse face carrying the sum
//    of the two fine faces it covers (boundary faces likewise);
//  * red-black Gauss-Seidel smoothing, red then black before the coarse
//    correction and black then red after it, so the V-cycle is symmetric;
//  * the coarse correction is scaled by omega (over-correction of the
//    aggregation coarse space);
//  * the coarsest grid (<= 8 x 8) is solved by a dense Cholesky factor.
// Every kernel covers the whole batch; samples that have converged are
// skipped through a per-sample active flag.  Per-sample dot products are
// reduced in a fixed order (thread -> wave -> workgroup partial -> one thread
// per sample), so a sample's iterates do not depend on the rest of the batch.
//
// Operator layout (per sample s, grid m x m, n = m*m):
//   T[s][0][j][i] face x1 = (i+1)h of cell (i,j) (i = m-1: boundary face),
//   T[s][1][j][i] face x2 = (j+1)h (j = m-1: boundary face),
//   tb[s][0][j]   face x1 = 0 of cell (0,j), tb[s][1][i] face x2 = 0 of (i,0).
//   (A x)_P = (sum of the four face T) x_P - sum over interior faces T x_nb.
#include "common.hpp"
#include "kernels.hpp"

namespace mlmc {

struct Faces {
  double te, tw, tn, ts;
};

__device__ __forceinline__ Faces load_faces(const double* __restrict__ Ts,
                                            const double* __restrict__ tbs, int m, int i, int j) {
  const int c = j * m + i;
  const int n = m * m;
  Faces f;
  f.te = Ts[c];
  f.tw = i > 0 ? Ts[c - 1] : tbs[j];
  f.tn = Ts[n + c];
  f.ts = j > 0 ? Ts[n + c - m] : tbs[m + i];
  return f;
}

__device__ __forceinline__ double neighbour_sum(const double* __restrict__ x, int m, int i, int j,
                                                const Faces& f) {
  const int c = j * m + i;
  double o = 0.0;
  if (i < m - 1) o += f.te * x[c + 1];
  if (i > 0) o += f.tw * x[c - 1];
  if (j < m - 1) o += f.tn * x[c + m];
  if (j > 0) o += f.ts * x[c - m];
  return o;
}

__device__ __forceinline__ double apply_at(const double* __restrict__ x, int m, int i, int j,
                                           const Faces& f) {
  const double d = f.te + f.tw + f.tn + f.ts;
  return d * x[j * m + i] - neighbour_sum(x, m, i, j, f);
}

// ------------------------------------------------------------------ hierarchy
__global__ void k_coarsen(int m, long long total, const double* __restrict__ T,
                          const double* __restrict__ tb, double* __restrict__ Tc,
                          double* __restrict__ tbc) {
  const long long g = (long long)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int mc = m / 2;
  const long long nc = (long long)mc * mc, n = (long long)m * m;
  const long long s = g / nc;
  const int rem = (int)(g - s * nc);
  const int J = rem / mc, I = rem - J * mc;
  const double* Ts = T + s * 2 * n;
  double* Tcs = Tc + s * 2 * nc;
  const int i = 2 * I, j = 2 * J;
  Tcs[rem] = Ts[j * m + i + 1] + Ts[(j + 1) * m + i + 1];
  Tcs[nc + rem] = Ts[n + (j + 1) * m + i] + Ts[n + (j + 1) * m + i + 1];
  const double* tbs = tb + s * 2 * m;
  double* tbcs = tbc + s * 2 * mc;
  if (I == 0) tbcs[J] = tbs[j] + tbs[j + 1];
  if (J == 0) tbcs[mc + I] = tbs[m + i] + tbs[m + i + 1];
}

void launch_coarsen(hipStream_t st, int m, int batch, const double* T, const double* tb,
                    double* Tc, double* tbc) {
  const long long total = (long long)batch * (m / 2) * (m / 2);
  hipLaunchKernelGGL(k_coarsen, dim3(blocks_for(total)), dim3(kBlock), 0, st, m, total, T, tb,
                     Tc, tbc);
}

// ------------------------------------------------------------------ smoother
// One thread per cell of the given colour ((i + j) % 2 == color).
__global__ void k_rbgs(int m, long long total, const double* __restrict__ T,
                       const double* __restrict__ tb, double* __restrict__ z,
                       const double* __restrict__ r, const int32_t* __restrict__ active,
                       int color, int zero_init) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int half = m / 2;
  const long long per = (long long)m * half;
  const long long s = g / per;
  if (!active[s]) return;
  const int rem = (int)(g - s * per);
  const int j = rem / half;
  const int i = 2 * (rem - j * half) + ((j + color) & 1);
  const long long n = (long long)m * m;
  const Faces f = load_faces(T + s * 2 * n, tb + s * 2 * m, m, i, j);
  const double d = f.te + f.tw + f.tn + f.ts;
  double* zs = z + s * n;
  const double rv = r[s * n + j * m + i];
  zs[j * m + i] = zero_init ? rv / d : (rv + neighbour_sum(zs, m, i, j, f)) / d;
}

void launch_rbgs(hipStream_t st, int m, int batch, const double* T, const double* tb, double* z,
                 const double* r, const int32_t* active, int color, int zero_init) {
  const long long total = (long long)batch * m * (m / 2);
  hipLaunchKernelGGL(k_rbgs, dim3(blocks_for(total)), dim3(kBlock), 0, st, m, total, T, tb, z, r,
                     active, color, zero_init);
}

// rc(I,J) = sum over the 2x2 fine cells of (r - A z)
__global__ void k_resid_restrict(int m, long long total, const double* __restrict__ T,
                                 const double* __restrict__ tb, const double* __restrict__ z,
                                 const double* __restrict__ r, double* __restrict__ rc,
                                 const int32_t* __restrict__ active) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int mc = m / 2;
  const long long nc = (long long)mc * mc, n = (long long)m * m;
  const long long s = g / nc;
  if (!active[s]) return;
  const int rem = (int)(g - s * nc);
  const int J = rem / mc, I = rem - J * mc;
  const double* Ts = T + s * 2 * n;
  const double* tbs = tb + s * 2 * m;
  const double* zs = z + s * n;
  const double* rs = r + s * n;
  double acc = 0.0;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int i = 2 * I + a, j = 2 * J + b;
      const Faces f = load_faces(Ts, tbs, m, i, j);
      acc += rs[j * m + i] - apply_at(zs, m, i, j, f);
    }
  rc[g] = acc;
}

void launch_resid_restrict(hipStream_t st, int m, int batch, const double* T, const double* tb,
                           const double* z, const double* r, double* rc,
                           const int32_t* active) {
  const long long total = (long long)batch * (m / 2) * (m / 2);
  hipLaunchKernelGGL(k_resid_restrict, dim3(blocks_for(total)), dim3(kBlock), 0, st, m, total, T,
                     tb, z, r, rc, active);
}

__global__ void k_prolong(int m, long long total, const double* __restrict__ zc,
                          double* __restrict__ z, double omega,
                          const int32_t* __restrict__ active) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long long n = (long long)m * m;
  const long long s = g / n;
  if (!active[s]) return;
  const int rem = (int)(g - s * n);
  const int j = rem / m, i = rem - j * m;
  const int mc = m / 2;
  z[g] += omega * zc[s * mc * mc + (j / 2) * mc + (i / 2)];
}

void launch_prolong(hipStream_t st, int m, int batch, const double* zc, double* z, double omega,
                    const int32_t* active) {
  const long long total = (long long)batch * m * m;
  hipLaunchKernelGGL(k_prolong, dim3(blocks_for(total)), dim3(kBlock), 0, st, m, total, zc, z,
                     omega, active);
}

// ------------------------------------------------------------------ coarsest grid
// Explicit inverse of each sample's coarsest matrix (n = m*m <= 64), so that
// every application on the coarsest grid is a matrix-vector product.  One
// 64-thread workgroup per sample builds A in LDS and inverts it in place by
// Gauss-Jordan elimination without pivoting (A is symmetric positive
// definite, so every pivot is positive):
//   for each k: a_kk <- 1, row k /= pivot; for i != k: row i -= a_ik row k,
//   with a_ik taken before the update and column k of row i ending at -a_ik/pivot.
__global__ void __launch_bounds__(64)
k_dense_factor(int m, int batch, const double* __restrict__ T, const double* __restrict__ tb,
               double* __restrict__ work, double* __restrict__ Ainv) {
  (void)work;
  __shared__ double A[64 * 64];
  __shared__ double col[64];
  const int s = blockIdx.x;
  if (s >= batch) return;
  const int n = m * m;
  const double* Ts = T + (long long)s * 2 * n;
  const double* tbs = tb + (long long)s * 2 * m;
  for (int q = threadIdx.x; q < n * n; q += 64) A[q] = 0.0;
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += 64) {
    const int j = c / m, i = c - j * m;
    const Faces f = load_faces(Ts, tbs, m, i, j);
    A[c * n + c] = f.te + f.tw + f.tn + f.ts;
    if (i < m - 1) A[c * n + c + 1] = A[(c + 1) * n + c] = -f.te;
    if (j < m - 1) A[c * n + c + m] = A[(c + m) * n + c] = -f.tn;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    for (int i = threadIdx.x; i < n; i += 64) col[i] = A[i * n + k];
    __syncthreads();
    const double piv = col[k];
    for (int j = threadIdx.x; j < n; j += 64) A[k * n + j] = (j == k ? 1.0 : A[k * n + j]) / piv;
    __syncthreads();
    for (int q = threadIdx.x; q < n * n; q += 64) {
      const int i = q / n, j = q - i * n;
      if (i != k) A[q] = (j == k ? 0.0 : A[q]) - col[i] * A[k * n + j];
    }
    __syncthreads();
  }
  double* X = Ainv + (long long)s * n * n;
  for (int q = threadIdx.x; q < n * n; q += 64) X[q] = A[q];
}

void launch_dense_factor(hipStream_t st, int m, int batch, const double* T, const double* tb,
                         double* work, double* Ainv) {
  hipLaunchKernelGGL(k_dense_factor, dim3(batch), dim3(64), 0, st, m, batch, T, tb, work, Ainv);
}

// z = A^-1 r, one thread per (sample, row).
__global__ void k_dense_apply(int n, long long total, const double* __restrict__ Ainv,
                              const double* __restrict__ r, double* __restrict__ z,
                              const int32_t* __restrict__ active) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long long s = g / n;
  if (!active[s]) return;
  const int q = (int)(g - s * n);
  const double* A = Ainv + s * n * n + (long long)q * n;
  const double* rs = r + s * n;
  double acc = 0.0;
  for (int p = 0; p < n; ++p) acc += A[p] * rs[p];
  z[g] = acc;
}

void launch_dense_apply_n(hipStream_t st, int n, int batch, const double* Ainv, const double* r,
                          double* z, const int32_t* active) {
  const long long total = (long long)batch * n;
  hipLaunchKernelGGL(k_dense_apply, dim3(blocks_for(total)), dim3(kBlock), 0, st, n, total, Ainv,
                     r, z, active);
}

void launch_dense_apply(hipStream_t st, int m, int batch, const double* Ainv, const double* r,
                        double* z, const int32_t* active) {
  const long long total = (long long)batch * m * m;
  hipLaunchKernelGGL(k_dense_apply, dim3(blocks_for(total)), dim3(kBlock), 0, st, m * m, total,
                     Ainv, r, z, active);
}

// ------------------------------------------------------------------ PCG vector kernels
// Block b of sample s (blockIdx.x = s * bps + b) owns cells b*1024 + t + 256 c.
// (Taken XCD by XCD instead, as the stencil kernels' blocks are, these mostly
// streaming kernels made the bench step 1% slower.)
#define PCG_PROLOGUE                                        \
  const int bps_ = bps;                                     \
  const int lbid = blockIdx.x;                              \
  const long long s = lbid / bps_;                          \
  const int blk = lbid - (int)(s * bps_);                   \
  const int cell0 = blk * kCellsPerBlock + threadIdx.x;

__global__ void __launch_bounds__(kBlock)
k_pcg_init(int n, const double* __restrict__ b, double* __restrict__ x, double* __restrict__ r,
           double* __restrict__ partial, int bps, const int32_t* __restrict__ only) {
  __shared__ double sh[kBlock / kWave];
  PCG_PROLOGUE
  if (only && !only[s]) return;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < kCellsPerThread; ++c) {
    const int cell = cell0 + c * kBlock;
    if (cell < n) {
      const long long e = s * n + cell;
      const double v = b[e];
      x[e] = 0.0;
      r[e] = v;
      acc += v * v;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[lbid] = t;
}

void launch_pcg_init(hipStream_t st, int n, int batch, const double* b, double* x, double* r,
                     double* partial, int bps, const int32_t* only) {
  hipLaunchKernelGGL(k_pcg_init, dim3(batch * bps), dim3(kBlock), 0, st, n, b, x, r, partial, bps,
                     only);
}

// Start from the initial guess held in x: r = b - A x, and the same partial
// sums of b^2 as k_pcg_init (the stopping rule is relative to ||b||, which for
// x = 0 is ||r_0||; with x = 0 the result equals k_pcg_init's bit for bit).
__global__ void __launch_bounds__(kBlock)
k_pcg_init_guess(int m, const double* __restrict__ T, const double* __restrict__ tb,
                 const double* __restrict__ b, const double* __restrict__ x,
                 double* __restrict__ r, double* __restrict__ partial, int bps) {
  __shared__ double sh[kBlock / kWave];
  PCG_PROLOGUE
  const int n = m * m;
  const double* Ts = T + s * 2 * n;
  const double* tbs = tb + s * 2 * m;
  const double* xs = x + s * n;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < kCellsPerThread; ++c) {
    const int cell = cell0 + c * kBlock;
    if (cell < n) {
      const int j = cell / m, i = cell - j * m;
      const Faces f = load_faces(Ts, tbs, m, i, j);
      const long long e = s * n + cell;
      const double v = b[e];
      r[e] = v - apply_at(xs, m, i, j, f);
      acc += v * v;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[lbid] = t;
}

void launch_pcg_init_guess(hipStream_t st, int m, int batch, const double* T, const double* tb,
                           const double* b, const double* x, double* r, double* partial,
                           int bps) {
  hipLaunchKernelGGL(k_pcg_init_guess, dim3(batch * bps), dim3(kBlock), 0, st, m, T, tb, b, x, r,
                     partial, bps);
}

// x0 of a fine grid from the solution of a coarse companion of the same
// sample (companion 0 of the sample's ncomp, stored one after another): each
// fine cell takes the value of the coarse cell that contains it.
__global__ void k_inject(int m, long long total, int ncomp, const double* __restrict__ xc,
                         double* __restrict__ x) {
  const long long g = (long long)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long long n = (long long)m * m;
  const long long s = g / n;
  const int rem = (int)(g - s * n);
  const int j = rem / m, i = rem - j * m;
  const int mc = m / 2;
  x[g] = xc[s * ncomp * (long long)mc * mc + (j / 2) * mc + i / 2];
}

void launch_inject(hipStream_t st, int m, int batch, int ncomp, const double* xc, double* x) {
  const long long total = (long long)batch * m * m;
  hipLaunchKernelGGL(k_inject, dim3(blocks_for(total)), dim3(kBlock), 0, st, m, total, ncomp, xc,
                     x);
}

__global__ void __launch_bounds__(kBlock)
k_spmv_dot(int m, const double* __restrict__ T, const double* __restrict__ tb,
           const double* __restrict__ p, double* __restrict__ q, double* __restrict__ partial,
           int bps, const int32_t* __restrict__ active) {
  __shared__ double sh[kBlock / kWave];
  PCG_PROLOGUE
  if (!active[s]) return;
  const int n = m * m;
  const double* Ts = T + s * 2 * n;
  const double* tbs = tb + s * 2 * m;
  const double* ps = p + s * n;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < kCellsPerThread; ++c) {
    const int cell = cell0 + c * kBlock;
    if (cell < n) {
      const int j = cell / m, i = cell - j * m;
      const Faces f = load_faces(Ts, tbs, m, i, j);
      const double v = apply_at(ps, m, i, j, f);
      q[s * n + cell] = v;
      acc += ps[cell] * v;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[lbid] = t;
}

void launch_spmv_dot(hipStream_t st, int m, int batch, const double* T, const double* tb,
                     const double* p, double* q, double* partial, int bps,
                     const int32_t* active) {
  hipLaunchKernelGGL(k_spmv_dot, dim3(batch * bps), dim3(kBlock), 0, st, m, T, tb, p, q, partial,
                     bps, active);
}

__global__ void __launch_bounds__(kBlock)
k_axpy_dot(int n, double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
           const double* __restrict__ q, const double* __restrict__ alpha,
           double* __restrict__ partial, int bps, const int32_t* __restrict__ active,
           const double* __restrict__ zold, double* __restrict__ partial2) {
  __shared__ double sh[kBlock / kWave];
  PCG_PROLOGUE
  if (!active[s]) return;
  const double a = alpha[s];
  double acc = 0.0, acc2 = 0.0;
#pragma unroll
  for (int c = 0; c < kCellsPerThread; ++c) {
    const int cell = cell0 + c * kBlock;
    if (cell < n) {
      const long long e = s * n + cell;
      x[e] += a * p[e];
      const double rv = r[e] - a * q[e];
      r[e] = rv;
      acc += rv * rv;
      if (zold) acc2 += rv * zold[e];
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[lbid] = t;
  if (zold) {
    __syncthreads();
    const double t2 = block_sum(acc2, sh);
    if (threadIdx.x == 0) partial2[lbid] = t2;
  }
}

void launch_axpy_dot(hipStream_t st, int n, int batch, double* x, double* r, const double* p,
                     const double* q, const double* alpha, double* partial, int bps,
                     const int32_t* active, const double* zold, double* partial2) {
  launch_k(k_axpy_dot, dim3(batch * bps), dim3(kBlock), 0, st, n, x, r, p, q, alpha,
                     partial, bps, active, zold, partial2);
}

__global__ void __launch_bounds__(kBlock)
k_dot(int n, const double* __restrict__ a, const double* __restrict__ b,
      double* __restrict__ partial, int bps, const int32_t* __restrict__ active) {
  __shared__ double sh[kBlock / kWave];
  PCG_PROLOGUE
  if (!active[s]) return;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < kCellsPerThread; ++c) {
    const int cell = cell0 + c * kBlock;
    if (cell < n) {
      const long long e = s * n + cell;
      acc += a[e] * b[e];
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[lbid] = t;
}

void launch_dot(hipStream_t st, int n, int batch, const double* a, const double* b,
                double* partial, int bps, const int32_t* active) {
  hipLaunchKernelGGL(k_dot, dim3(batch * bps), dim3(kBlock), 0, st, n, a, b, partial, bps, active);
}

__global__ void __launch_bounds__(kBlock)
k_pupdate(int n, double* __restrict__ p, const double* __restrict__ z,
          const double* __restrict__ beta, int bps, const int32_t* __restrict__ active,
          int first) {
  PCG_PROLOGUE
  if (!active[s]) return;
  const double bt = first ? 0.0 : beta[s];
#pragma unroll
  for (int c = 0; c < kCellsPerThread; ++c) {
    const int cell = cell0 + c * kBlock;
    if (cell < n) {
      const long long e = s * n + cell;
      p[e] = first ? z[e] : z[e] + bt * p[e];
    }
  }
}

void launch_pupdate(hipStream_t st, int n, int batch, double* p, const double* z,
                    const double* beta, int bps, const int32_t* active, int first) {
  hipLaunchKernelGGL(k_pupdate, dim3(batch * bps), dim3(kBlock), 0, st, n, p, z, beta, bps,
                     active, first);
}

__global__ void __launch_bounds__(kBlock)
k_true_residual(int m, const double* __restrict__ T, const double* __restrict__ tb,
                const double* __restrict__ b, const double* __restrict__ x,
                double* __restrict__ partial, int bps) {
  __shared__ double sh[kBlock / kWave];
  PCG_PROLOGUE
  const int n = m * m;
  const double* Ts = T + s * 2 * n;
  const double* tbs = tb + s * 2 * m;
  const double* xs = x + s * n;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < kCellsPerThread; ++c) {
    const int cell = cell0 + c * kBlock;
    if (cell < n) {
      const int j = cell / m, i = cell - j * m;
      const Faces f = load_faces(Ts, tbs, m, i, j);
      const double rv = b[s * n + cell] - apply_at(xs, m, i, j, f);
      acc += rv * rv;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[lbid] = t;
}

void launch_true_residual(hipStream_t st, int m, int batch, const double* T, const double* tb,
                          const double* b, const double* x, double* partial, int bps) {
  hipLaunchKernelGGL(k_true_residual, dim3(batch * bps), dim3(kBlock), 0, st, m, T, tb, b, x,
                     partial, bps);
}

// ------------------------------------------------------------------ per-sample scalars
// A sample's scalars come from its partial sums.  With few partials per sample
// (small grids, large batches) one thread per sample adds them in order; with
// many (kWideSum or more: large grids, few samples) one wave per sample does:
// lane l adds partials l, l + 64, ... in order and a fixed shuffle tree adds the
// lanes (result in lane 0).  The form depends only on the partial count, so a
// sample's scalars depend only on its own partials.  Both forms run kBlock
// threads per workgroup.
constexpr int kWideSum = 16;

template <bool WIDE>
__device__ __forceinline__ double sum_partials_t(const double* __restrict__ partial, int bps,
                                                 int s, int lane) {
  double acc = 0.0;
  if (WIDE) {
    // lane k adds entries k, k + 64, ... in that order; the loads of a group
    // of eight are issued before its adds, so a group costs one memory
    // latency (thousands of partials per sample on the large 3-D grids)
    constexpr int kU = 8;
    const double* ps = partial + (long long)s * bps;
    for (int q0 = lane; q0 < bps; q0 += kU * kWave) {
      double v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) v[u] = q0 + u * kWave < bps ? ps[q0 + u * kWave] : 0.0;
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (q0 + u * kWave < bps) acc += v[u];
    }
    return wave_sum(acc);
  }
  for (int q = 0; q < bps; ++q) acc += partial[(long long)s * bps + q];
  return acc;
}

#define SC_PROLOGUE                                                                         \
  const long long gtid = (long long)blockIdx.x * blockDim.x + threadIdx.x;                  \
  const int s = (int)(WIDE ? gtid / kWave : gtid);                                         \
  const int lane = WIDE ? (int)(threadIdx.x & (kWave - 1)) : 0;

static inline dim3 sc_grid(int batch, bool wide) {
  const long long threads = (long long)batch * (wide ? kWave : 1);
  return dim3((unsigned)((threads + kBlock - 1) / kBlock));
}

#define SC_LAUNCH(kern, batch, bps, ...)                                                   \
  do {                                                                                     \
    if ((bps) >= kWideSum)                                                                 \
      hipLaunchKernelGGL(kern<true>, sc_grid(batch, true), dim3(kBlock), 0, __VA_ARGS__);  \
    else                                                                                   \
      hipLaunchKernelGGL(kern<false>, sc_grid(batch, false), dim3(kBlock), 0, __VA_ARGS__); \
  } while (0)

template <bool WIDE>
__global__ void k_sc_init(int batch, const double* __restrict__ partial, int bps, SolverState S,
                          int32_t* __restrict__ status, int32_t* __restrict__ iters,
                          double* __restrict__ relres, int restart) {
  SC_PROLOGUE
  if (s >= batch || (restart && !S.active[s])) return;
  const double v = sum_partials_t<WIDE>(partial, bps, s, lane);
  if (lane != 0) return;
  S.r0sq[s] = v;
  iters[s] = 0;
  relres[s] = 0.0;
  status[s] = MLMC_SAMPLE_OK;
  if (!(v > 0.0) || !isfinite(v)) {
    S.active[s] = 0;
    if (!isfinite(v)) status[s] = MLMC_SAMPLE_BREAKDOWN;
  } else {
    S.active[s] = 1;
  }
}

void launch_sc_init(hipStream_t st, int batch, const double* partial, int bps, SolverState s,
                    int32_t* status, int32_t* iters, double* relres, int restart) {
  SC_LAUNCH(k_sc_init, batch, bps, st, batch, partial, bps, s, status, iters, relres, restart);
}

// Marks the samples whose iteration broke down for a second pass (active = 1),
// moves their iteration counts to `carried` and writes how many there are to
// *S.count.  One workgroup.
__global__ void k_sc_restart(int batch, SolverState S, int32_t* __restrict__ status,
                             int32_t* __restrict__ iters, int32_t* __restrict__ carried) {
  __shared__ double red[kBlock / kWave];
  double cnt = 0.0;
  for (int s = threadIdx.x; s < batch; s += kBlock) {
    const int v = status[s];
    const bool again = v == MLMC_SAMPLE_BREAKDOWN;
    S.active[s] = again ? 1 : 0;
    carried[s] = again ? iters[s] : 0;
    cnt += again ? 1.0 : 0.0;
  }
  const double t = block_sum(cnt, red);
  if (threadIdx.x == 0) *S.count = (int32_t)t;
}

void launch_sc_restart(hipStream_t st, int batch, SolverState s, int32_t* status, int32_t* iters,
                       int32_t* carried) {
  hipLaunchKernelGGL(k_sc_restart, dim3(1), dim3(kBlock), 0, st, batch, s, status, iters, carried);
}

__global__ void k_iters_add(int batch, int32_t* __restrict__ iters,
                            const int32_t* __restrict__ carried) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < batch) iters[s] += carried[s];
}

void launch_iters_add(hipStream_t st, int batch, int32_t* iters, const int32_t* carried) {
  hipLaunchKernelGGL(k_iters_add, dim3(blocks_for(batch)), dim3(kBlock), 0, st, batch, iters,
                     carried);
}

template <bool WIDE>
__global__ void k_sc_rho(int batch, const double* __restrict__ partial, int nparts,
                         SolverState S, int32_t* __restrict__ status, int first,
                         const double* __restrict__ partial2, int nparts2) {
  SC_PROLOGUE
  if (s >= batch || !S.active[s]) return;
  const double v = sum_partials_t<WIDE>(partial, nparts, s, lane);
  const double rzold =
      (!first && partial2) ? sum_partials_t<WIDE>(partial2, nparts2, s, lane) : 0.0;
  if (lane != 0) return;
  if (!(v > 0.0) || !isfinite(v)) {
    S.active[s] = 0;
    status[s] = MLMC_SAMPLE_BREAKDOWN;
    return;
  }
  S.beta[s] = first ? 0.0 : (v - rzold) / S.rho[s];
  S.rho[s] = v;
}

void launch_sc_rho(hipStream_t st, int batch, const double* partial, int nparts, SolverState s,
                   int32_t* status, int first, const double* partial2, int nparts2) {
  SC_LAUNCH(k_sc_rho, batch, std::max(nparts, partial2 ? nparts2 : 0), st, batch, partial, nparts,
            s, status, first, partial2, nparts2);
}

template <bool WIDE>
__global__ void k_sc_alpha(int batch, const double* __restrict__ partial, int bps, SolverState S,
                           int32_t* __restrict__ status) {
  SC_PROLOGUE
  if (blockIdx.x == 0 && threadIdx.x == 0) *S.count = 0;
  if (s >= batch || !S.active[s]) return;
  const double v = sum_partials_t<WIDE>(partial, bps, s, lane);
  if (lane != 0) return;
  if (!(v > 0.0) || !isfinite(v)) {
    S.active[s] = 0;
    status[s] = MLMC_SAMPLE_BREAKDOWN;
    return;
  }
  S.alpha[s] = S.rho[s] / v;
}

void launch_sc_alpha(hipStream_t st, int batch, const double* partial, int bps, SolverState s,
                     int32_t* status) {
  SC_LAUNCH(k_sc_alpha, batch, bps, st, batch, partial, bps, s, status);
}

template <bool WIDE>
__global__ void k_sc_conv(int batch, const double* __restrict__ partial, int bps, SolverState S,
                          int32_t* __restrict__ status, int32_t* __restrict__ iters,
                          double* __restrict__ relres, double tol, int maxit) {
  SC_PROLOGUE
  if (s >= batch || !S.active[s]) return;
  const double v = sum_partials_t<WIDE>(partial, bps, s, lane);
  if (lane != 0) return;
  const int it = iters[s] + 1;
  iters[s] = it;
  const double rr = sqrt(v / S.r0sq[s]);
  relres[s] = rr;
  if (!isfinite(v)) {
    S.active[s] = 0;
    status[s] = MLMC_SAMPLE_BREAKDOWN;
  } else if (rr < tol) {
    S.active[s] = 0;
    status[s] = MLMC_SAMPLE_OK;
  } else if (it >= maxit) {
    S.active[s] = 0;
    status[s] = MLMC_SAMPLE_NOCONV;
  } else {
    atomicAdd(S.count, 1);
  }
}

void launch_sc_conv(hipStream_t st, int batch, const double* partial, int bps, SolverState s,
                    int32_t* status, int32_t* iters, double* relres, double tol, int maxit) {
  SC_LAUNCH(k_sc_conv, batch, bps, st, batch, partial, bps, s, status, iters, relres, tol, maxit);
}

template <bool WIDE>
__global__ void k_sc_final(int batch, const double* __restrict__ partial, int bps, SolverState S,
                           double* __restrict__ relres) {
  SC_PROLOGUE
  if (s >= batch) return;
  const double v = sum_partials_t<WIDE>(partial, bps, s, lane);
  if (lane != 0) return;
  const double r0 = S.r0sq[s];
  relres[s] = r0 > 0.0 ? sqrt(v / r0) : 0.0;
}

void launch_sc_final(hipStream_t st, int batch, const double* partial, int bps, SolverState s,
                     double* relres) {
  SC_LAUNCH(k_sc_final, batch, bps, st, batch, partial, bps, s, relres);
}

}  // namespace mlmc
