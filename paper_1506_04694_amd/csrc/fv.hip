// Finite volume assembly, outflow QoI and per-level estimator sums on gfx950.
//
// Assembly (Section 3.1, eq. (3.3); harmonic-mean faces as in Section 3.4;
// Model Problem 2, eq. (3.11)): T = 2 k_P k_Q / (k_P + k_Q) on interior faces
// (2-D: face length / centre distance = 1), T = 2 k_P on the Dirichlet faces
// x1 = 0 and x1 = 1 (half-cell distance), T = 0 on the no-flow faces; the
// inflow data p = 1 enters the right-hand side b = T on column i = 0.
//
// Model Problem 1 (Section 3.4): f = 1 and p = 0 on the whole boundary, so
// every boundary face is a Dirichlet face (T = 2 k_P) and b = f h^2 = h^2.
//
// QoI (Section 3.4, M^(2)): outflow through x1 = 1 as the sum of the
// boundary-face fluxes 2 k p over the last column; inflow likewise at x1 = 0.
// M^(1): the mean of the cell-wise constant pressure over a box [lo, hi]^d,
// each cell weighted by its overlap with the box.
//
// Estimator sums (eq. (3.6), (3.7), (4.2)): one workgroup reduces a level's
// Y, Q_f, Q_c in a fixed order (per-thread strided sums, then a fixed tree),
// so the sums do not depend on timing.
#include "common.hpp"
#include "kernels.hpp"

namespace mlmc {

__global__ void k_assemble(int problem, int m, long long total, const double* __restrict__ k,
                           double* __restrict__ T, double* __restrict__ tb,
                           double* __restrict__ b) {
  // neighbouring rows (which read each other's k) on one XCD
  const long long g = (long long)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long long n = (long long)m * m;
  const long long s = g / n;
  const int rem = (int)(g - s * n);
  const int j = rem / m, i = rem - j * m;
  const double kp = k[g];
  double te, tn;
  if (i < m - 1) {
    const double kq = k[g + 1];
    te = 2.0 * kp * kq / (kp + kq);
  } else {
    te = 2.0 * kp;
  }
  const bool mp1 = problem == MLMC_PROBLEM_MEAN_PRESSURE;
  if (j < m - 1) {
    const double kq = k[g + m];
    tn = 2.0 * kp * kq / (kp + kq);
  } else {
    tn = mp1 ? 2.0 * kp : 0.0;
  }
  double* Ts = T + s * 2 * n;
  Ts[rem] = te;
  Ts[n + rem] = tn;
  const double h = 1.0 / (double)m;
  b[g] = mp1 ? h * h : ((i == 0) ? 2.0 * kp : 0.0);
  double* tbs = tb + s * 2 * m;
  if (i == 0) tbs[j] = 2.0 * kp;
  if (j == 0) tbs[m + i] = mp1 ? 2.0 * kp : 0.0;
}

void launch_assemble(hipStream_t st, int problem, int m, int batch, const double* k, double* T,
                     double* tb, double* b) {
  const long long total = (long long)batch * m * m;
  hipLaunchKernelGGL(k_assemble, dim3(blocks_for(total)), dim3(kBlock), 0, st, problem, m, total,
                     k, T, tb, b);
}

// One wave per sample.
__global__ void k_qoi(int m, int batch, const double* __restrict__ k, const double* __restrict__ p,
                      double* __restrict__ qout, double* __restrict__ qin) {
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (wave >= batch) return;
  const long long base = wave * (long long)m * m;
  double so = 0.0, si = 0.0;
  for (int j = lane; j < m; j += kWave) {
    const long long e = base + (long long)j * m + (m - 1);
    const long long w = base + (long long)j * m;
    so += 2.0 * k[e] * p[e];
    si += 2.0 * k[w] * (1.0 - p[w]);
  }
  so = wave_sum(so);
  si = wave_sum(si);
  if (lane == 0) {
    qout[wave] = so;
    if (qin) qin[wave] = si;
  }
}

void launch_qoi(hipStream_t st, int m, int batch, const double* k, const double* p, double* qout,
                double* qin) {
  const long long threads = (long long)batch * kWave;
  hipLaunchKernelGGL(k_qoi, dim3(blocks_for(threads)), dim3(kBlock), 0, st, m, batch, k, p, qout,
                     qin);
}

// Overlap of cell i's interval [i/m, (i+1)/m] with [lo, hi].
__device__ __forceinline__ double cell_overlap(int i, int m, double lo, double hi) {
  const double a = (double)i / (double)m, b = (double)(i + 1) / (double)m;
  return fmax(fmin(b, hi) - fmax(a, lo), 0.0);
}

// M^(1) over [lo, hi]^d, one wave per sample: the lanes take the cells of the
// box's index range in turn (the cells with nonzero overlap lie in [i0, i1) on
// every axis), then a fixed shuffle tree.
__global__ void k_qoi_box(int dim, int m, int batch, int i0, int i1, double lo, double hi,
                          const double* __restrict__ p, double* __restrict__ q) {
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (wave >= batch) return;
  const int w = i1 - i0;
  const long long per = dim == 3 ? (long long)m * m * m : (long long)m * m;
  const double* ps = p + wave * per;
  const int cells = dim == 3 ? w * w * w : w * w;
  double acc = 0.0;
  for (int t = lane; t < cells; t += kWave) {
    const int a = t % w, r = t / w;
    const int i = i0 + a, j = i0 + r % w, l = dim == 3 ? i0 + r / w : 0;
    double wt = cell_overlap(i, m, lo, hi) * cell_overlap(j, m, lo, hi);
    if (dim == 3) wt *= cell_overlap(l, m, lo, hi);
    acc += wt * ps[((long long)l * m + j) * m + i];
  }
  acc = wave_sum(acc);
  if (lane == 0) {
    const double side = hi - lo;
    q[wave] = acc / (dim == 3 ? side * side * side : side * side);
  }
}

void launch_qoi_box(hipStream_t st, int dim, int m, int batch, double lo, double hi,
                    const double* p, double* q) {
  // index range of the cells that meet the box (clamped to the grid)
  int i0 = (int)floor(lo * m) - 1, i1 = (int)ceil(hi * m) + 1;
  i0 = i0 < 0 ? 0 : i0;
  i1 = i1 > m ? m : i1;
  const long long threads = (long long)batch * kWave;
  hipLaunchKernelGGL(k_qoi_box, dim3(blocks_for(threads)), dim3(kBlock), 0, st, dim, m, batch, i0,
                     i1, lo, hi, p, q);
}

// Q^cgv = 2^-d sum_j Q(k^(j))  (eq. (4.1)); companions of sample s at s*ncomp + j.
__global__ void k_cgv_average(int batch, int ncomp, const double* __restrict__ qcomp,
                              double* __restrict__ qc) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= batch) return;
  double acc = 0.0;
  for (int j = 0; j < ncomp; ++j) acc += qcomp[(long long)s * ncomp + j];
  qc[s] = acc / (double)ncomp;
}

void launch_cgv_average(hipStream_t st, int batch, int ncomp, const double* qcomp, double* qc) {
  hipLaunchKernelGGL(k_cgv_average, dim3(blocks_for(batch)), dim3(kBlock), 0, st, batch, ncomp,
                     qcomp, qc);
}

// Y = Q_f - Q_c; failed = fine or any companion solve not converged.
__global__ void k_y_and_fail(int n, const double* __restrict__ qf, const double* __restrict__ qc,
                             const int32_t* __restrict__ st_f, const int32_t* __restrict__ st_c,
                             int ncomp, double* __restrict__ y, int32_t* __restrict__ failed) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  int f = st_f[s] != MLMC_SAMPLE_OK;
  for (int j = 0; j < ncomp; ++j) f |= st_c[(long long)s * ncomp + j] != MLMC_SAMPLE_OK;
  y[s] = qc ? qf[s] - qc[s] : qf[s];
  failed[s] = f;
}

void launch_y_and_fail(hipStream_t st, int n, const double* qf, const double* qc,
                       const int32_t* st_f, const int32_t* st_c, int ncomp, double* y,
                       int32_t* failed) {
  hipLaunchKernelGGL(k_y_and_fail, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, qf, qc, st_f,
                     st_c, ncomp, y, failed);
}

// out6 = {sum y, sum y^2, sum qf, sum qc, n_failed, iters_fine, iters_coarse} (7 doubles)
__global__ void __launch_bounds__(kBlock)
k_level_reduce(int n, const double* __restrict__ y, const double* __restrict__ qf,
               const double* __restrict__ qc, const int32_t* __restrict__ failed,
               const int32_t* __restrict__ it_f, const int32_t* __restrict__ it_c, int ncomp,
               double* __restrict__ out) {
  __shared__ double sh[kBlock / kWave];
  double a[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int s = threadIdx.x; s < n; s += kBlock) {
    a[0] += y[s];
    a[1] += y[s] * y[s];
    a[2] += qf[s];
    a[3] += qc ? qc[s] : 0.0;
    a[4] += (double)failed[s];
    a[5] += (double)it_f[s];
    if (it_c)
      for (int j = 0; j < ncomp; ++j) a[6] += (double)it_c[(long long)s * ncomp + j];
  }
  for (int q = 0; q < 7; ++q) {
    const double v = block_sum(a[q], sh);
    if (threadIdx.x == 0) out[q] = v;
    __syncthreads();
  }
}

void launch_level_reduce(hipStream_t st, int n, const double* y, const double* qf,
                         const double* qc, const int32_t* failed, const int32_t* it_f,
                         const int32_t* it_c, int ncomp, double* out6) {
  hipLaunchKernelGGL(k_level_reduce, dim3(1), dim3(kBlock), 0, st, n, y, qf, qc, failed, it_f,
                     it_c, ncomp, out6);
}

}  // namespace mlmc
