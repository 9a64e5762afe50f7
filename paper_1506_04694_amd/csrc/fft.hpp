// LDS-resident mixed-radix (2, 3, 4, 5) complex FP64 FFT for lines of length
// n <= kFftMax, one or several lines per workgroup.
//
// Stockham autosort formulation (natural-order input and output): at a stage
// of radix R with span Ns (product of the radices already applied), butterfly
// j (0 <= j < n/R) reads x[j + r n/R], r = 0..R-1, multiplies input r by
// exp(-2 pi i r (j mod Ns) / (Ns R)), applies the R-point DFT and writes output
// r to x[(j / Ns) Ns R + (j mod Ns) + r Ns].  Each stage loads all of its
// inputs into registers, waits at a barrier and then stores, so one LDS
// buffer (separate real and imaginary arrays) suffices.  Forward transform:
// X_k = sum_j x_j exp(-2 pi i jk / n).  Twiddles come from a table
// tw[q] = exp(-2 pi i q / n), q < n, in device memory.
#pragma once

#include <algorithm>

#include "common.hpp"

namespace mlmc {

constexpr int kFftMax = 4096;
constexpr int kFftMax3 = 1024;  // 3-D embeddings: n^3 complex values per transform
constexpr int kFftMaxStages = 16;

struct FftPlan {
  int n;
  int nstages;
  int radix[kFftMaxStages];
  // per stage: 1 / (butterflies per line) and 1 / (span before the stage),
  // rounded once to FP32 on the host (the divisors of div_small)
  float inv_nb[kFftMaxStages];
  float inv_ns[kFftMaxStages];
};

template <int R>
__device__ __forceinline__ void dft_small(double* xr, double* xi) {
  if constexpr (R == 2) {
    const double ar = xr[0], ai = xi[0], br = xr[1], bi = xi[1];
    xr[0] = ar + br; xi[0] = ai + bi;
    xr[1] = ar - br; xi[1] = ai - bi;
  } else if constexpr (R == 4) {
    const double t0r = xr[0] + xr[2], t0i = xi[0] + xi[2];
    const double t1r = xr[0] - xr[2], t1i = xi[0] - xi[2];
    const double t2r = xr[1] + xr[3], t2i = xi[1] + xi[3];
    // (x1 - x3) * (-i)
    const double t3r = xi[1] - xi[3], t3i = -(xr[1] - xr[3]);
    xr[0] = t0r + t2r; xi[0] = t0i + t2i;
    xr[2] = t0r - t2r; xi[2] = t0i - t2i;
    xr[1] = t1r + t3r; xi[1] = t1i + t3i;
    xr[3] = t1r - t3r; xi[3] = t1i - t3i;
  } else if constexpr (R == 3) {
    constexpr double c = -0.5;
    constexpr double s = -0.86602540378443864676;  // -sin(2 pi / 3)
    const double ar = xr[1] + xr[2], ai = xi[1] + xi[2];
    const double dr = xr[1] - xr[2], di = xi[1] - xi[2];
    const double tr = xr[0] + c * ar, ti = xi[0] + c * ai;
    // i s (x1 - x2)
    const double ur = -s * di, ui = s * dr;
    xr[0] = xr[0] + ar; xi[0] = xi[0] + ai;
    xr[1] = tr + ur; xi[1] = ti + ui;
    xr[2] = tr - ur; xi[2] = ti - ui;
  } else if constexpr (R == 5) {
    constexpr double c1 = 0.30901699437494742410;   // cos(2 pi / 5)
    constexpr double c2 = -0.80901699437494742410;  // cos(4 pi / 5)
    constexpr double s1 = 0.95105651629515357212;   // sin(2 pi / 5)
    constexpr double s2 = 0.58778525229247312917;   // sin(4 pi / 5)
    const double a1r = xr[1] + xr[4], a1i = xi[1] + xi[4];
    const double b1r = xr[1] - xr[4], b1i = xi[1] - xi[4];
    const double a2r = xr[2] + xr[3], a2i = xi[2] + xi[3];
    const double b2r = xr[2] - xr[3], b2i = xi[2] - xi[3];
    const double p1r = xr[0] + c1 * a1r + c2 * a2r, p1i = xi[0] + c1 * a1i + c2 * a2i;
    const double p2r = xr[0] + c2 * a1r + c1 * a2r, p2i = xi[0] + c2 * a1i + c1 * a2i;
    // q1 = s1 b1 + s2 b2 ; q2 = s2 b1 - s1 b2 ; X1 = p1 - i q1, X4 = p1 + i q1,
    // X2 = p2 - i q2, X3 = p2 + i q2   (-i (a + ib) = b - ia)
    const double q1r = s1 * b1r + s2 * b2r, q1i = s1 * b1i + s2 * b2i;
    const double q2r = s2 * b1r - s1 * b2r, q2i = s2 * b1i - s1 * b2i;
    xr[0] = xr[0] + a1r + a2r; xi[0] = xi[0] + a1i + a2i;
    xr[1] = p1r + q1i; xi[1] = p1i - q1r;
    xr[4] = p1r - q1i; xi[4] = p1i + q1r;
    xr[2] = p2r + q2i; xi[2] = p2i - q2r;
    xr[3] = p2r - q2i; xi[3] = p2i + q2r;
  }
}

// q = floor(a / d) for 0 <= a < 2^22, 1 <= d <= 2^13, through one FP32
// multiply: (a + 1/2) / d stays at least 1/(2d) away from an integer, more than
// the two roundings (relative 2^-24 each) can move it.
__device__ __forceinline__ int div_small(int a, float inv_d) {
  return (int)(((float)a + 0.5f) * inv_d);
}

template <int R>
__device__ __forceinline__ void fft_stage_one(double* __restrict__ sre, double* __restrict__ sim,
                                          const double2* __restrict__ tw, int n, int ns,
                                          float inv_ns) {
  constexpr int kMaxC = (kFftMax / R + kBlock - 1) / kBlock;
  const int nb = n / R;
  const int step = n / (ns * R);
  // butterfly j splits as j = jq ns + kk (one FP32 multiply by the plan's
  // 1 / ns instead of an integer division per butterfly)
  double vr[kMaxC][R], vi[kMaxC][R];
#pragma unroll
  for (int c = 0; c < kMaxC; ++c) {
    const int j = threadIdx.x + c * kBlock;
    if (j < nb) {
      const int kk = j - div_small(j, inv_ns) * ns;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        vr[c][r] = sre[j + r * nb];
        vi[c][r] = sim[j + r * nb];
      }
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const double2 w = tw[r * kk * step];
        const double a = vr[c][r], b = vi[c][r];
        vr[c][r] = a * w.x - b * w.y;
        vi[c][r] = a * w.y + b * w.x;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kMaxC; ++c) {
    const int j = threadIdx.x + c * kBlock;
    if (j < nb) {
      const int jq = div_small(j, inv_ns);
      const int kk = j - jq * ns;
      dft_small<R>(vr[c], vi[c]);
      const int base = jq * ns * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        sre[base + r * ns] = vr[c][r];
        sim[base + r * ns] = vi[c][r];
      }
    }
  }
  __syncthreads();
}

// In-place forward FFT of one line held in LDS (sre, sim) by kBlock threads,
// butterfly slots sized per radix for the longest line; for lines whose widest
// stage needs more than one pass of the workgroup this form keeps fewer values
// live than fft_lines.  All threads call it; the caller synchronises before.
__device__ __forceinline__ void fft_line(double* sre, double* sim, const double2* tw,
                                         const FftPlan& pl) {
  int ns = 1;
  for (int st = 0; st < pl.nstages; ++st) {
    const int R = pl.radix[st];
    const float ins = pl.inv_ns[st];
    if (R == 4) fft_stage_one<4>(sre, sim, tw, pl.n, ns, ins);
    else if (R == 2) fft_stage_one<2>(sre, sim, tw, pl.n, ns, ins);
    else if (R == 3) fft_stage_one<3>(sre, sim, tw, pl.n, ns, ins);
    else fft_stage_one<5>(sre, sim, tw, pl.n, ns, ins);
    ns *= R;
  }
}

// One Stockham stage of radix R over L lines (line q at sre + q n) by a
// workgroup of T threads; C is the largest number of butterflies (L n / R over
// T threads) a thread takes.
template <int R, int C, int T>
__device__ __forceinline__ void fft_stage(double* __restrict__ sre, double* __restrict__ sim,
                                          const double2* __restrict__ tw, int n, int ns, int L,
                                          float inv_nb, float inv_ns) {
  const int nb = n / R;
  const int step = n / (ns * R);
  const int total = L * nb;
  double vr[C][R], vi[C][R];
  int base[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int b = threadIdx.x + c * T;
    if (b < total) {
      const int q = div_small(b, inv_nb);
      const int j = b - q * nb;
      const int jq = div_small(j, inv_ns);
      const int kk = j - jq * ns;
      const double* xr = sre + q * n;
      const double* xi = sim + q * n;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        vr[c][r] = xr[j + r * nb];
        vi[c][r] = xi[j + r * nb];
      }
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const double2 w = tw[r * kk * step];
        const double a = vr[c][r], bb = vi[c][r];
        vr[c][r] = a * w.x - bb * w.y;
        vi[c][r] = a * w.y + bb * w.x;
      }
      base[c] = q * n + jq * ns * R + kk;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int b = threadIdx.x + c * T;
    if (b < total) {
      dft_small<R>(vr[c], vi[c]);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        sre[base[c] + r * ns] = vr[c][r];
        sim[base[c] + r * ns] = vi[c][r];
      }
    }
  }
  __syncthreads();
}

// In-place forward FFT of L lines held in LDS (line q at sre + q n, sim + q n)
// by a workgroup of T threads.  All threads call it; the caller synchronises
// before.
template <int C, int T>
__device__ __forceinline__ void fft_lines(double* sre, double* sim, const double2* tw,
                                          const FftPlan& pl, int L) {
  int ns = 1;
  for (int st = 0; st < pl.nstages; ++st) {
    const int R = pl.radix[st];
    const float inb = pl.inv_nb[st], ins = pl.inv_ns[st];
    if (R == 4) fft_stage<4, C, T>(sre, sim, tw, pl.n, ns, L, inb, ins);
    else if (R == 2) fft_stage<2, C, T>(sre, sim, tw, pl.n, ns, L, inb, ins);
    else if (R == 3) fft_stage<3, C, T>(sre, sim, tw, pl.n, ns, L, inb, ins);
    else fft_stage<5, C, T>(sre, sim, tw, pl.n, ns, L, inb, ins);
    ns *= R;
  }
}

// Launch shape for lines of the plan's length on 256-thread workgroups: when
// the widest stage has at most 128 butterflies, L >= 2 lines per workgroup (as
// many as keep it within 256, at most 8) with one butterfly per thread and
// stage (fft_lines<1, 256>); otherwise one line per workgroup (fft_line).
// Measured on MI355X for the embedding lengths 135 and 375: 2.9x and 1.4x
// faster than one line per workgroup; for 960 and 1875 the single-line form
// is faster than multi-slot fft_lines (fewer live registers).
inline int fft_lines_per_group(const FftPlan& pl) {
  int widest = 1;
  for (int st = 0; st < pl.nstages; ++st) widest = std::max(widest, pl.n / pl.radix[st]);
  const int L = 256 / widest;
  return L < 2 ? 1 : (L > 8 ? 8 : L);
}

}  // namespace mlmc
