// Shared device helpers for the gfx950 kernels: counter-based random numbers,
// layer geometry, wave64 reductions and launch-shape constants.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mlmc_darcy.h"
#include "unitmath.hpp"

namespace mlmc {

constexpr int kBlock = 256;          // threads per workgroup for streaming kernels
constexpr int kCellsPerThread = 4;   // cells per thread in per-sample vector kernels
constexpr int kCellsPerBlock = kBlock * kCellsPerThread;
constexpr int kWave = 64;

// XCD-aware block order: hardware dispatches consecutive workgroup ids round
// robin over the 8 XCDs; give XCD x a contiguous range of logical ids (a
// bijection of [0, nblocks)), so that neighbouring blocks share its L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int x = bid & 7, q = bid >> 3;
  const int per = nblocks >> 3, rem = nblocks & 7;
  return x * per + (x < rem ? x : rem) + q;
}

// bfloat16 storage (the upper half of an FP32 value); arithmetic is done in FP32.
struct bf16_t {
  uint16_t bits;
};

// Per-sample random parameters: [0..7] interface data, [8..11] log-k layer
// constants (piecewise constant layers), [12..15] unused.
constexpr int kParamStride = 16;

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw (SC'11): ten rounds of
//   (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2,
//   c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0),
// with the key bumped by the Weyl constants between rounds.
struct U4 {
  uint32_t x, y, z, w;
};

// Each 32 x 32 -> 64-bit product is taken whole (one v_mad_u64_u32 instead of
// separate low and high multiplies).
__device__ __forceinline__ U4 philox(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = M0 * (uint64_t)c.x, p1 = M1 * (uint64_t)c.z;
    c = U4{(uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
           (uint32_t)p0};
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// Stream tags (counter word c3).
constexpr uint32_t kTagGeometry = 0, kTagLayerConst = 1, kTagNoise = 2;

__device__ __forceinline__ U4 stream_block(uint64_t seed, uint32_t block, uint32_t sample,
                                           uint32_t level, uint32_t tag) {
  return philox(U4{block, sample, level, tag}, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// (x + 1/2) 2^-32: strictly inside (0, 1), exact in FP64.
__device__ __forceinline__ double to_uniform(uint32_t x) {
  return ((double)x + 0.5) * (1.0 / 4294967296.0);
}

// Box-Muller: two standard normals from two uniforms.  cos and sin of 2 pi u1
// come from sin/cos of pi (2 u1), whose argument is exact (no rounding of
// 2 pi u1); the logarithm and the sine/cosine are the short forms for these
// argument ranges (unitmath.hpp), a few ulps from the exact values.
__device__ __forceinline__ void box_muller(double u0, double u1, double& z0, double& z1) {
  const double r = sqrt(-2.0 * log_unit(u0));
  double s, c;
  sincospi_unit(2.0 * u1, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// ---------------------------------------------------------------- geometry
// Layer index of the point (x, y) for one sample's interface parameters.
// Contraction is disabled so that the comparisons that decide a layer are
// taken on the same rounded values as a plain FP64 evaluation.
__device__ __forceinline__ int layer_of(int kind, int n_nodes, const double* prm, double x,
                                        double y) {
#pragma clang fp contract(off)
  if (kind == MLMC_IFACE_HORIZONTAL) {
    return y < prm[0] ? 0 : 1;
  } else if (kind == MLMC_IFACE_PIECEWISE_LINEAR) {
    const double fx = (double)(n_nodes - 1) * x;
    int s = (int)floor(fx);
    if (s > n_nodes - 2) s = n_nodes - 2;
    const double t = fx - (double)s;
    const double yi = prm[s] + t * (prm[s + 1] - prm[s]);
    return y < yi ? 0 : 1;
  } else if (kind == MLMC_IFACE_PAPER_TWO_LINES) {
    const double upper = prm[0] + x * (prm[1] - prm[0]);
    const double lower = prm[2] + x * (prm[3] - prm[2]);
    return y < lower ? 0 : (y < upper ? 1 : 2);
  } else if (kind == MLMC_IFACE_TILTED_PLANE) {
    return y < prm[0] + (prm[1] - prm[0]) * x ? 0 : 1;  // the plane's trace at x3 = 1/2
  }
  return 0;
}

// 3-D: the tilted plane x2 = a + (b - a) x1 + c (x3 - 1/2); the 2-D interfaces
// are extruded along x3.
__device__ __forceinline__ int layer_of3(int kind, int n_nodes, const double* prm, double x,
                                         double y, double z) {
#pragma clang fp contract(off)
  if (kind == MLMC_IFACE_TILTED_PLANE)
    return y < prm[0] + (prm[1] - prm[0]) * x + prm[2] * (z - 0.5) ? 0 : 1;
  return layer_of(kind, n_nodes, prm, x, y);
}

__device__ __forceinline__ double centre(int i, int m) {
#pragma clang fp contract(off)
  return ((double)i + 0.5) / (double)m;
}

// ---------------------------------------------------------------- reductions
// Fixed-order wave64 tree sum (result in lane 0).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
  return v;
}

// Fixed-order block sum for kBlock threads; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) s += sh[i];
  }
  return s;
}

// Blocks of 256 threads needed to cover n items.
inline int blocks_for(long long n, int per_block = kBlock) {
  return (int)((n + per_block - 1) / per_block);
}

}  // namespace mlmc
