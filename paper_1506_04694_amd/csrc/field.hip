// Layered permeability sampling on gfx950.
//
// Section 2 (Examples 1 and 2) and Section 3.4 of Park & Teckentrup: a random
// partition into layers, independent of the layer laws; on each layer either
// a log-normal constant (Example 1) or a log-normal stationary field with the
// exponential covariance eq. (2.3), sampled by circulant embedding.
//
// Circulant embedding of an m x m grid into an n x n torus (n = n_ce):
//   setup (once per m, n, sigma2, lambda, r): first covariance row c -> 2-D FFT
//     -> eigenvalues Lambda (real); check min >= -1e-12 max; store
//     sqrt(max(Lambda, 0) / n^2), transposed, for pass A;
//   pass A, one workgroup per (sample, noise column k1): Philox normals
//     xi(k2, k1) for all k2 (rows 2p and 2p+1 take the two normal pairs of
//     block p n + k1), scaled by sqrt(Lambda / n^2), FFT along k2 in LDS,
//     keep rows j2 < m -> uT[sample][j2][k1];
//   pass B, one workgroup per (sample, row j2 < m): FFT of uT[sample][j2][:]
//     along k1 in LDS, keep j1 < m; Re -> the pair's first layer, Im -> its
//     second; the layer of each centre decides k = exp(mu_l + g_l) on the
//     cells of the pair's layers; the plain coarse companion is written from
//     the even (j1, j2) cells in the same pass.
// Layers with different covariances use separate embedding samples (pairs,
// each with its own eigenvalues and noise stream tag 2 + pair); passes A and B
// run once per pair and each pass B writes the cells of its own layers.
// Pass A's stores are strided by n; its block order is remapped so that the
// columns k1 that share cache lines run on the same XCD (and its L2).
#include <float.h>

#include "common.hpp"
#include "fft.hpp"
#include "kernels.hpp"

namespace mlmc {

// ------------------------------------------------------------ per-sample parameters
__global__ void k_sample_params(mlmc_model mdl, uint32_t level, uint64_t first,
                                const uint32_t* __restrict__ ids, int batch,
                                double* __restrict__ params) {
#pragma clang fp contract(off)
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= batch) return;
  const uint32_t sample = ids ? ids[s] : (uint32_t)(first + (uint64_t)s);
  double prm[kParamStride];
#pragma unroll
  for (int q = 0; q < kParamStride; ++q) prm[q] = 0.0;
  if (mdl.interface_kind == MLMC_IFACE_HORIZONTAL) {
    const U4 b = stream_block(mdl.seed, 0, sample, level, kTagGeometry);
    prm[0] = mdl.y_lo + (mdl.y_hi - mdl.y_lo) * to_uniform(b.x);
  } else if (mdl.interface_kind == MLMC_IFACE_PIECEWISE_LINEAR) {
    for (int q0 = 0; q0 < mdl.n_nodes; q0 += 4) {
      const U4 b = stream_block(mdl.seed, (uint32_t)(q0 / 4), sample, level, kTagGeometry);
      const uint32_t w[4] = {b.x, b.y, b.z, b.w};
      for (int t = 0; t < 4 && q0 + t < mdl.n_nodes; ++t)
        prm[q0 + t] = mdl.y_lo + (mdl.y_hi - mdl.y_lo) * to_uniform(w[t]);
    }
  } else if (mdl.interface_kind == MLMC_IFACE_PAPER_TWO_LINES) {
    const U4 b = stream_block(mdl.seed, 0, sample, level, kTagGeometry);
    const uint32_t w[4] = {b.x, b.y, b.z, b.w};
    const double lo[4] = {0.8, 0.6, 0.2, 0.4};
    for (int t = 0; t < 4; ++t) prm[t] = lo[t] + 0.1 * to_uniform(w[t]);
  } else if (mdl.interface_kind == MLMC_IFACE_TILTED_PLANE) {
    const U4 b = stream_block(mdl.seed, 0, sample, level, kTagGeometry);
    prm[0] = mdl.y_lo + (mdl.y_hi - mdl.y_lo) * to_uniform(b.x);
    prm[1] = mdl.y_lo + (mdl.y_hi - mdl.y_lo) * to_uniform(b.y);
    prm[2] = -0.1 + 0.2 * to_uniform(b.z);
  }
  {
    const U4 b = stream_block(mdl.seed, 0, sample, level, kTagLayerConst);
    double z[4];
    box_muller(to_uniform(b.x), to_uniform(b.y), z[0], z[1]);
    box_muller(to_uniform(b.z), to_uniform(b.w), z[2], z[3]);
    for (int l = 0; l < 4; ++l) prm[8 + l] = mdl.mu[l] + sqrt(mdl.sigma2[l]) * z[l];
  }
#pragma unroll
  for (int q = 0; q < kParamStride; ++q) params[(size_t)s * kParamStride + q] = prm[q];
}

void launch_sample_params(hipStream_t st, const mlmc_model& mdl, int level, uint64_t first,
                          const uint32_t* ids, int batch, double* params) {
  hipLaunchKernelGGL(k_sample_params, dim3(blocks_for(batch)), dim3(kBlock), 0, st, mdl,
                     (uint32_t)level, first, ids, batch, params);
}

// ------------------------------------------------------------ Example 1 field
__global__ void k_field_pc(int kind, int n_nodes, int m, long long total,
                           const double* __restrict__ params, double* __restrict__ k) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const long long n = (long long)m * m;
  const long long s = g / n;
  const int rem = (int)(g - s * n);
  const int j = rem / m, i = rem - j * m;
  const double* prm = params + s * kParamStride;
  const int l = layer_of(kind, n_nodes, prm, centre(i, m), centre(j, m));
  k[g] = exp(prm[8 + l]);
}

void launch_field_pc(hipStream_t st, const mlmc_model& mdl, int m, int batch,
                     const double* params, double* k) {
  const long long total = (long long)batch * m * m;
  hipLaunchKernelGGL(k_field_pc, dim3(blocks_for(total)), dim3(kBlock), 0, st,
                     mdl.interface_kind, mdl.n_nodes, m, total, params, k);
}

// ------------------------------------------------------------ circulant embedding setup
__global__ void k_twiddles(int n, double2* __restrict__ tw) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double s, c;
  sincospi(-2.0 * (double)q / (double)n, &s, &c);
  tw[q] = make_double2(c, s);
}

void launch_ce_twiddles(hipStream_t st, int n, double2* tw) {
  hipLaunchKernelGGL(k_twiddles, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, tw);
}

// c[a2][a1] = sigma2 exp(-||(d1, d2)||_r / lambda), d = min(a, n - a) h  (eq. (2.3))
__global__ void k_ce_first_row(int n, int m, double sigma2, double lambda, int norm_r,
                               double2* __restrict__ c) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long long)n * n) return;
  const int a2 = (int)(g / n), a1 = (int)(g - (long long)a2 * n);
  const double h = 1.0 / (double)m;
  const double d1 = (double)min(a1, n - a1) * h;
  const double d2 = (double)min(a2, n - a2) * h;
  const double dist = norm_r == 1 ? d1 + d2 : sqrt(d1 * d1 + d2 * d2);
  c[g] = make_double2(sigma2 * exp(-dist / lambda), 0.0);
}

void launch_ce_first_row(hipStream_t st, int n, int m, double sigma2, double lambda, int norm_r,
                         double2* c) {
  const long long total = (long long)n * n;
  hipLaunchKernelGGL(k_ce_first_row, dim3(blocks_for(total)), dim3(kBlock), 0, st, n, m,
                     sigma2, lambda, norm_r, c);
}

// In-place FFT of nlines lines of a complex array (setup only), one line per
// workgroup.
__global__ void __launch_bounds__(kBlock)
k_fft_lines(double2* __restrict__ data, long long line_stride, long long elem_stride,
            const double2* __restrict__ tw, FftPlan pl) {
  extern __shared__ double lds[];
  double* sre = lds;
  double* sim = lds + pl.n;
  double2* line = data + (long long)blockIdx.x * line_stride;
  for (int q = threadIdx.x; q < pl.n; q += kBlock) {
    const double2 v = line[q * elem_stride];
    sre[q] = v.x;
    sim[q] = v.y;
  }
  __syncthreads();
  fft_line(sre, sim, tw, pl);
  for (int q = threadIdx.x; q < pl.n; q += kBlock) line[q * elem_stride] = make_double2(sre[q], sim[q]);
}

void launch_fft_lines(hipStream_t st, double2* data, int n, int nlines, long long line_stride,
                      long long elem_stride, const double2* tw, const FftPlan& pl) {
  hipLaunchKernelGGL(k_fft_lines, dim3(nlines), dim3(kBlock), 2 * n * sizeof(double), st, data,
                     line_stride, elem_stride, tw, pl);
}

__global__ void k_minmax(const double2* __restrict__ lam, long long count,
                         double* __restrict__ partial) {
  __shared__ double smin[kBlock], smax[kBlock];
  double lo = DBL_MAX, hi = -DBL_MAX;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < count;
       q += (long long)gridDim.x * blockDim.x) {
    const double v = lam[q].x;
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = smin[0];
    partial[2 * blockIdx.x + 1] = smax[0];
  }
}

void launch_ce_minmax(hipStream_t st, const double2* lam, long long count, double* partial,
                      int nblocks) {
  hipLaunchKernelGGL(k_minmax, dim3(nblocks), dim3(kBlock), 0, st, lam, count, partial);
}

// sqT[k1][k2] = sqrt(max(Lambda[k2][k1], 0) / n^2)
__global__ void k_sqrt_transpose(const double2* __restrict__ lam, int n, double* __restrict__ sqT) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long long)n * n) return;
  const int k1 = (int)(g / n), k2 = (int)(g - (long long)k1 * n);
  const double v = lam[(long long)k2 * n + k1].x;
  sqT[g] = sqrt(fmax(v, 0.0) / ((double)n * (double)n));
}

void launch_ce_sqrt_transpose(hipStream_t st, const double2* lam, int n, double* sqT) {
  const long long total = (long long)n * n;
  hipLaunchKernelGGL(k_sqrt_transpose, dim3(blocks_for(total)), dim3(kBlock), 0, st, lam, n, sqT);
}

// ------------------------------------------------------------ pass A
// Workgroup = L consecutive columns k1 of one sample (C = 0: one column and
// the single-line FFT): noise of the columns
// scaled by sqrt(Lambda), FFT along k2, the first m outputs of each column to
// uT[s][j2][k1] (the L columns give L adjacent entries of every row j2).
// At least 4 waves per SIMD (at most 128 VGPRs): the long-line form otherwise
// takes 132 and runs 3 waves per SIMD; measured on the 256^2 x 256 and 512^2 x
// 64 fields, passes A and B together 10% and 8% faster (5 waves would spill).
template <int C, int T>
__global__ void __launch_bounds__(T, 4)
k_ce_pass_a(uint64_t seed, uint32_t tag, uint32_t level, uint64_t first,
            const uint32_t* __restrict__ ids, int m, const double* __restrict__ sqT,
            const double2* __restrict__ tw, FftPlan pl, int L, int groups,
            double2* __restrict__ uT) {
  extern __shared__ double lds[];
  const int n = pl.n;
  double* sre = lds;
  double* sim = lds + L * n;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int s = blk / groups;
  const int k1_0 = (blk - s * groups) * L;
  const int lines = min(L, n - k1_0);
  const uint32_t sample = ids ? ids[s] : (uint32_t)(first + (uint64_t)s);
  // rows 2p and 2p+1 of column k1 share Philox block p n + k1
  const int npairs = (n + 1) / 2;
  const float inv_pairs = 1.0f / (float)npairs;
  for (int t = threadIdx.x; t < L * npairs; t += T) {
    const int q = div_small(t, inv_pairs);
    const int pr = t - q * npairs;
    const int k2 = 2 * pr;
    double* xr = sre + q * n;
    double* xi = sim + q * n;
    if (q >= lines) {
      xr[k2] = 0.0;
      xi[k2] = 0.0;
      if (k2 + 1 < n) {
        xr[k2 + 1] = 0.0;
        xi[k2 + 1] = 0.0;
      }
      continue;
    }
    const int k1 = k1_0 + q;
    const double* sq = sqT + (long long)k1 * n;
    const U4 bk = stream_block(seed, (uint32_t)pr * (uint32_t)n + (uint32_t)k1, sample, level, tag);
    double zr, zi;
    box_muller(to_uniform(bk.x), to_uniform(bk.y), zr, zi);
    const double a = sq[k2];
    xr[k2] = a * zr;
    xi[k2] = a * zi;
    if (k2 + 1 < n) {
      box_muller(to_uniform(bk.z), to_uniform(bk.w), zr, zi);
      const double a1 = sq[k2 + 1];
      xr[k2 + 1] = a1 * zr;
      xi[k2 + 1] = a1 * zi;
    }
  }
  __syncthreads();
  if constexpr (C == 0) fft_line(sre, sim, tw, pl);
  else fft_lines<C, T>(sre, sim, tw, pl, L);
  double2* out = uT + (long long)s * m * n + k1_0;
  const float inv_lines = 1.0f / (float)lines;
  for (int t = threadIdx.x; t < lines * m; t += T) {
    const int j2 = div_small(t, inv_lines);
    const int q = t - j2 * lines;
    out[(long long)j2 * n + q] = make_double2(sre[q * n + j2], sim[q * n + j2]);
  }
}

template <int C, int T>
static void pass_a_c(hipStream_t st, const mlmc_model& mdl, uint32_t tag, int level,
                     uint64_t first, const uint32_t* ids, int batch, int m, const double* sqT,
                     const double2* tw, const FftPlan& pl, int L, double2* uT) {
  const int groups = (pl.n + L - 1) / L;
  hipLaunchKernelGGL((k_ce_pass_a<C, T>), dim3(batch * groups), dim3(T),
                     2 * (size_t)L * pl.n * sizeof(double), st, mdl.seed, tag, (uint32_t)level,
                     first, ids, m, sqT, tw, pl, L, groups, uT);
}

void launch_ce_pass_a(hipStream_t st, const mlmc_model& mdl, const CePair& pr, int level,
                      uint64_t first, const uint32_t* ids, int batch, int m, const double* sqT,
                      const double2* tw, const FftPlan& pl, double2* uT) {
  const int L = fft_lines_per_group(pl);
  if (L > 1)
    pass_a_c<1, kBlock>(st, mdl, pr.tag, level, first, ids, batch, m, sqT, tw, pl, L, uT);
  else pass_a_c<0, kBlock>(st, mdl, pr.tag, level, first, ids, batch, m, sqT, tw, pl, 1, uT);
}

// ------------------------------------------------------------ pass B
// Workgroup = L consecutive rows j2 of one sample (C = 0: one row and the
// single-line FFT): FFT along k1 of uT[s][j2][.],
// the first m outputs give the two Gaussian layers (real / imaginary part), then
// k = exp(mean + g) of each cell's layer, and the plain coarse companion's
// cells from the even rows and columns.
template <int C, int T>
__global__ void __launch_bounds__(T, 4)
k_ce_pass_b(int kind, int n_nodes, int n_layers, CePair pr, int m,
            const double2* __restrict__ uT, const double2* __restrict__ tw, FftPlan pl, int L,
            int groups, const double* __restrict__ params, double* __restrict__ k,
            double* __restrict__ kc) {
  extern __shared__ double lds[];
  const int n = pl.n;
  double* sre = lds;
  double* sim = lds + L * n;
  const int s = blockIdx.x / groups;
  const int j2_0 = (blockIdx.x - s * groups) * L;
  const int lines = min(L, m - j2_0);
  const double2* in = uT + ((long long)s * m + j2_0) * n;
  // loads in groups of kU issued before their stores
  constexpr int kU = 8;
  for (int q0 = threadIdx.x; q0 < L * n; q0 += kU * T) {
    double2 v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = q0 + u * T;
      v[u] = q < lines * n ? in[q] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = q0 + u * T;
      if (q < L * n) {
        sre[q] = v[u].x;
        sim[q] = v[u].y;
      }
    }
  }
  __syncthreads();
  if constexpr (C == 0) fft_line(sre, sim, tw, pl);
  else fft_lines<C, T>(sre, sim, tw, pl, L);
  const double* prm = params + (long long)s * kParamStride;
  const int mc = m / 2;
  const float inv_m = 1.0f / (float)m;
  for (int t = threadIdx.x; t < lines * m; t += T) {
    const int q = div_small(t, inv_m);
    const int j1 = t - q * m;
    const int j2 = j2_0 + q;
    const double g0 = sre[q * n + j1], g1 = sim[q * n + j1];
    const double y = centre(j2, m);
    const int l = n_layers > 1 ? layer_of(kind, n_nodes, prm, centre(j1, m), y) : 0;
    if (l == pr.l_re || l == pr.l_im)
      k[((long long)s * m + j2) * m + j1] = exp(l == pr.l_re ? pr.mu_re + g0 : pr.mu_im + g1);
    if (kc != nullptr && ((j2 & 1) == 0) && ((j1 & 1) == 0)) {
      const double yc = centre(j2 / 2, mc);
      const int lc = n_layers > 1 ? layer_of(kind, n_nodes, prm, centre(j1 / 2, mc), yc) : 0;
      if (lc == pr.l_re || lc == pr.l_im)
        kc[((long long)s * mc + j2 / 2) * mc + j1 / 2] =
            exp(lc == pr.l_re ? pr.mu_re + g0 : pr.mu_im + g1);
    }
  }
}

template <int C, int T>
static void pass_b_c(hipStream_t st, const mlmc_model& mdl, const CePair& pr, int batch, int m,
                     const double2* uT, const double2* tw, const FftPlan& pl, int L,
                     const double* params, double* k, double* k_coarse) {
  const int groups = (m + L - 1) / L;
  hipLaunchKernelGGL((k_ce_pass_b<C, T>), dim3(batch * groups), dim3(T),
                     2 * (size_t)L * pl.n * sizeof(double), st, mdl.interface_kind, mdl.n_nodes,
                     mdl.n_layers, pr, m, uT, tw, pl, L, groups, params, k, k_coarse);
}

void launch_ce_pass_b(hipStream_t st, const mlmc_model& mdl, const CePair& pr, int batch, int m,
                      const double2* uT, const double2* tw, const FftPlan& pl,
                      const double* params, double* k, double* k_coarse) {
  const int L = fft_lines_per_group(pl);
  if (L > 1) pass_b_c<1, kBlock>(st, mdl, pr, batch, m, uT, tw, pl, L, params, k, k_coarse);
  else pass_b_c<0, kBlock>(st, mdl, pr, batch, m, uT, tw, pl, 1, params, k, k_coarse);
}

// ------------------------------------------------------------ CGV sub-lattices
__global__ void k_cgv_extract(int m, long long total, const double* __restrict__ kf,
                              double* __restrict__ ksub) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int mc = m / 2;
  const long long nc = (long long)mc * mc;
  const long long sa = g / nc;              // sample * 4 + a
  const int rem = (int)(g - sa * nc);
  const int J = rem / mc, I = rem - J * mc;
  const long long s = sa >> 2;
  const int a = (int)(sa & 3);
  const int i = 2 * I + (a & 1), j = 2 * J + (a >> 1);
  ksub[g] = kf[(s * m + j) * m + i];
}

void launch_cgv_extract(hipStream_t st, int m, int batch, const double* kf, double* ksub) {
  const long long total = (long long)batch * 4 * (m / 2) * (m / 2);
  hipLaunchKernelGGL(k_cgv_extract, dim3(blocks_for(total)), dim3(kBlock), 0, st, m, total, kf,
                     ksub);
}

}  // namespace mlmc
