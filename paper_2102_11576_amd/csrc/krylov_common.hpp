// Device helpers shared by the streaming Krylov kernels: wavefront and block
// sums and the deterministic "last block finishes" grid reduction.
#pragma once

#include <math.h>

#include <array>
#include <utility>

#include "internal.hpp"

namespace rsfde {

// Largest number of basis vectors one streaming launch handles; longer
// restarts are processed in chunks of this size.
constexpr int kChunk = 32;

// ------------------------------ helpers -----------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum NV per-thread values over the block; results valid in thread 0..NV-1's
// out[] (out[v] for v < nv, broadcast through LDS to all threads).
template <int NV>
__device__ __forceinline__ void block_sum(double (&acc)[NV], int nv, double* sh /* [16][NV] */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (v < nv) {
      const double s = wave_sum(acc[v]);
      if (lane == 0) sh[wid * NV + v] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (v < nv) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += sh[w * NV + v];
      acc[v] = s;
    }
  }
  __syncthreads();
}

// Publish the block's NV sums as partials[v][blockIdx.x] (plain stores; the
// finishing kernel that reads them runs after this kernel, so the kernel
// boundary orders them and no device-scope fence is needed).
template <int NV>
__device__ __forceinline__ void publish_partials(double (&acc)[NV], int nv, RedWork rw,
                                                 double* sh /* [16*NV] */) {
  block_sum<NV>(acc, nv, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (v < nv) rw.partial[(size_t)v * kMaxRedBlocks + blockIdx.x] = acc[v];
  }
}

// In a finishing kernel: the calling wavefront adds partials[v][0..nb) in a
// fixed order (lane-strided, then a butterfly) and returns the total in every lane.
__device__ __forceinline__ double wave_total(const RedWork& rw, int v, int nb) {
  const int lane = threadIdx.x & 63;
  const double* p = rw.partial + (size_t)v * kMaxRedBlocks;
  // all loads first (independent addresses), then the fixed-order sum
  double x[kMaxRedBlocks / 64];
#pragma unroll
  for (int q = 0; q < kMaxRedBlocks / 64; ++q) {
    const int k = lane + 64 * q;
    x[q] = k < nb ? p[k] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kMaxRedBlocks / 64; ++q) s += x[q];
  return wave_sum(s);
}

constexpr int kFinishThreads = 1024;  // 16 wavefronts: one value per wavefront

}  // namespace rsfde
