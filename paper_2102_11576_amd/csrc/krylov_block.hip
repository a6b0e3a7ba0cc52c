// Block kernels of the s-step form of the restarted GMRES (Section 5 of the
// paper runs GMRES; its orthogonalisation scheme is not fixed there).  One
// block of s Krylov directions U = [u_1 .. u_s] (u_{i+1} = (M P^{-1} - theta) u_i)
// is orthogonalised against the m+1 orthonormal basis vectors Q in two passes
// over the basis instead of 2s:
//   gram:   G = [Q U]^T U   (projections C = Q^T U and U^T U in one pass: a
//           tall-skinny FP64 contraction on the matrix cores)
//   update: U <- (U - Q C) R^{-1}, R = chol(U^T U - C^T C)  (R from the host)
// Q and U are adjacent slots of the basis array V, so [Q U] is one strided
// matrix.  Partial sums are per block and added in a fixed order: results are
// deterministic.
#include "krylov_common.hpp"

namespace rsfde {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kGramThreads = 256;  // 4 wavefronts

// Partial Gram block: gpart[(r * 16 + c) * kGramBlocks + block] = sum over this
// block's elements of A[r][e] * U[c][e], r < nr, c < s, with A row r = V + r*ld
// and U column c = V + (m1 + c)*ld.  NT = number of 16-row tiles (nr <= 16 NT).
// v_mfma_f64_16x16x4: lane l supplies A[l%16][k] and B[k][l%16] with k = l/16,
// and holds D[l/16 + 4i][l%16], i < 4.  The K index runs over elements: lane
// group k takes elements base + 2k and base + 2k + 1 of each 8-element step
// (one 16-byte load per row), the same mapping for A and B.
// K chunks (c0, c0 + stride, ...) of 32 elements per row: lane group k4 loads
// elements base + 8 q + 2 k4 and + 1, so that one load instruction reads 64
// contiguous bytes of each of the wavefront's 16 rows (a mapping with 64-byte
// strides between the lane groups measured 3.5-4.0 TB/s, a third below the
// streaming kernels).  All K chunks' loads are issued before their MFMAs;
// MFMA step (q, x|y) takes the same element of A and B.
template <int NT, int K>
__device__ __forceinline__ void gram_chunks(size_t c0, size_t stride, int k4, const double* brow,
                                            bool bvalid, const double* const* arow,
                                            const bool* avalid, v4d* acc) {
  // acc[0]: the U tile (U^T U), whose A operand is the B operand itself (the
  // same row of U in the same lane), so U is read once; acc[1 + t]: Q tile t.
  double2 b[K][4], a[K][NT][4];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const size_t e = (c0 + u * stride) * 32 + 2 * k4;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      b[u][q] = bvalid ? reinterpret_cast<const double2*>(brow + e)[4 * q] : double2{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        a[u][t][q] =
            avalid[t] ? reinterpret_cast<const double2*>(arow[t] + e)[4 * q] : double2{0.0, 0.0};
  }
#pragma unroll
  for (int u = 0; u < K; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[u][q].x, b[u][q].x, acc[0], 0, 0, 0);
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[u][q].y, b[u][q].y, acc[0], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        acc[1 + t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][t][q].x, b[u][q].x, acc[1 + t], 0, 0, 0);
        acc[1 + t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][t][q].y, b[u][q].y, acc[1 + t], 0, 0, 0);
      }
    }
}

// NT Q tiles (m1 <= 16 NT) plus the U tile; U2 chunks per loop iteration (2
// where the registers allow).
template <int NT, int U2>
__global__ __launch_bounds__(kGramThreads) void k_bgram(const double* __restrict__ V, size_t ld,
                                                        int nr, int m1, int s, size_t N,
                                                        double* __restrict__ gpart) {
  __shared__ double red[4][NT + 1][64][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int i16 = lane & 15, k4 = lane >> 4;
  const bool bvalid = i16 < s;
  const double* brow = V + (size_t)(m1 + (bvalid ? i16 : 0)) * ld;
  const double* arow[NT];
  bool avalid[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int r = 16 * t + i16;
    avalid[t] = r < m1;
    arow[t] = V + (size_t)(avalid[t] ? r : 0) * ld;
  }
  v4d acc[NT + 1];
#pragma unroll
  for (int t = 0; t <= NT; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};

  // Chunks of 32 elements, wave by wave over the grid (gram_chunks).
  const size_t nchunks = N / 32;
  const size_t gw = (size_t)gridDim.x * 4;
  size_t ch = (size_t)blockIdx.x * 4 + wid;
  for (; ch + (U2 - 1) * gw < nchunks; ch += U2 * gw)
    gram_chunks<NT, U2>(ch, gw, k4, brow, bvalid, arow, avalid, acc);
  for (; ch < nchunks; ch += gw) gram_chunks<NT, 1>(ch, gw, k4, brow, bvalid, arow, avalid, acc);
  // tail (N % 32 elements): block 0, wave 0 only
  if (blockIdx.x == 0 && wid == 0) {
    const size_t e0 = nchunks * 32 + 8 * k4;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const size_t e = e0 + j;
      const double bv = (bvalid && e < N) ? brow[e] : 0.0;
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv, bv, acc[0], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const double av = (avalid[t] && e < N) ? arow[t][e] : 0.0;
        acc[1 + t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[1 + t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t <= NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) red[wid][t][lane][q] = acc[t][q];
  __syncthreads();
  if (wid == 0) {
#pragma unroll
    for (int t = 0; t <= NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double v = red[0][t][lane][q] + red[1][t][lane][q] + red[2][t][lane][q] +
                         red[3][t][lane][q];
        const int rt = k4 + 4 * q, c = i16;  // row within the tile
        // rows of G in [Q U] order: the U tile holds rows m1 + rt, Q tile t - 1 rows 16 (t - 1) + rt
        const int r = t == 0 ? m1 + rt : 16 * (t - 1) + rt;
        const bool ok = t == 0 ? rt < s : r < m1;
        if (ok && c < s) gpart[(size_t)(r * 16 + c) * kGramBlocks + blockIdx.x] = v;
      }
  }
}

// G[r * 16 + c] = sum of the partials (fixed order), written where the host
// reads it (pinned, device-visible memory); one wavefront per entry, spread
// over a grid.  Every block fences its entries at system scope and counts
// itself on *done; the last block resets the count and publishes seq.
__global__ __launch_bounds__(kFinishThreads) void k_bgram_finish(const double* __restrict__ gpart,
                                                                 int nr, int s, int nb,
                                                                 double* G, int32_t* seq_flag,
                                                                 int32_t seq, int32_t* done) {
  const int lane = threadIdx.x & 63;
  constexpr int kWaves = kFinishThreads / 64;
  for (int p = blockIdx.x * kWaves + (threadIdx.x >> 6); p < nr * s; p += gridDim.x * kWaves) {
    const int r = p / s, c = p % s;
    const double* src = gpart + (size_t)(r * 16 + c) * kGramBlocks;
    // all loads first (independent addresses), then the fixed-order sum
    double v[kGramBlocks / 64];
#pragma unroll
    for (int q = 0; q < kGramBlocks / 64; ++q) {
      const int k = lane + 64 * q;
      v[q] = k < nb ? src[k] : 0.0;
    }
    double x = 0.0;
#pragma unroll
    for (int q = 0; q < kGramBlocks / 64; ++q) x += v[q];
    x = wave_sum(x);
    if (lane == 0) G[r * 16 + c] = x;
  }
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int prior = atomicAdd(done, 1);
    if (prior == (int)gridDim.x - 1) {  // every block's entries are written and fenced
      atomicExch(done, 0);
      __threadfence_system();
      *reinterpret_cast<volatile int32_t*>(seq_flag) = seq;
    }
  }
}

// U <- (U - Q C) R^{-1} in place, U = V + m1*ld (S vectors), Q = V (nq vectors).
// coef: C row-major [nq][S] followed by R^{-1} row-major [S][S] (upper
// triangular); uniform reads, so they come through the scalar cache.
template <int S, bool ARGS>
__global__ __launch_bounds__(kRedThreads) void k_bupd(double* __restrict__ V, size_t ld, int nq,
                                                      int m1, size_t N,
                                                      const double* __restrict__ coef_dev,
                                                      const CoefArgs args) {
  const double* __restrict__ coef = ARGS ? args.v : coef_dev;
  const double* __restrict__ Rinv = coef + (size_t)nq * S;
  double* U = V + (size_t)m1 * ld;
  const size_t N2 = N / 2;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N2;
       i += (size_t)gridDim.x * blockDim.x) {
    double2 y[S];
#pragma unroll
    for (int k = 0; k < S; ++k) y[k] = reinterpret_cast<const double2*>(U + (size_t)k * ld)[i];
    int q = 0;
    for (; q + 4 <= nq; q += 4) {
      double2 x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = reinterpret_cast<const double2*>(V + (size_t)(q + u) * ld)[i];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < S; ++k) {
          const double c = coef[(q + u) * S + k];
          y[k].x -= c * x[u].x;
          y[k].y -= c * x[u].y;
        }
    }
    for (; q < nq; ++q) {
      const double2 x = reinterpret_cast<const double2*>(V + (size_t)q * ld)[i];
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const double c = coef[q * S + k];
        y[k].x -= c * x.x;
        y[k].y -= c * x.y;
      }
    }
#pragma unroll
    for (int k = S - 1; k >= 0; --k) {  // out_k = sum_{l<=k} y_l Rinv[l][k] (descending: in place)
      double2 o = {0.0, 0.0};
#pragma unroll
      for (int l = 0; l <= k; ++l) {
        const double r = Rinv[l * S + k];
        o.x += y[l].x * r;
        o.y += y[l].y * r;
      }
      reinterpret_cast<double2*>(U + (size_t)k * ld)[i] = o;
    }
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const size_t e = N - 1;
    double y[S];
#pragma unroll
    for (int k = 0; k < S; ++k) y[k] = U[(size_t)k * ld + e];
    for (int q = 0; q < nq; ++q) {
      const double x = V[(size_t)q * ld + e];
#pragma unroll
      for (int k = 0; k < S; ++k) y[k] -= coef[q * S + k] * x;
    }
#pragma unroll
    for (int k = S - 1; k >= 0; --k) {
      double o = 0.0;
#pragma unroll
      for (int l = 0; l <= k; ++l) o += y[l] * Rinv[l * S + k];
      U[(size_t)k * ld + e] = o;
    }
  }
}

// ------------------------------- launchers --------------------------------

hipError_t launch_bgram(const double* V, size_t ld, int nr, int m1, int s, size_t N,
                        double* gpart, double* G_host_dev, int32_t* seq_flag, int32_t seq,
                        int32_t* done_count, hipStream_t st) {
  // rows: the m1 rows of Q followed by the s rows of U (nr = m1 + s)
  if (nr < 1 || s < 1 || s > 16 || m1 < 1 || nr != m1 + s || nr > 16 * kGramMaxTiles)
    return hipErrorInvalidValue;
  int nb = (int)((N / 32 + 4 * 4 - 1) / (4 * 4));  // >= 4 chunks per wave
  if (nb < 1) nb = 1;
  if (nb > kGramBlocks) nb = kGramBlocks;
  const int nt = (m1 + 15) / 16;  // Q tiles; the U tile reuses the B operand's loads
  // One Q tile (two tiles of MFMAs) with two chunks per iteration runs at
  // occupancy 3: half the blocks measured faster there.
  if (nt == 1 && nb > kGramBlocks / 2) nb = kGramBlocks / 2;
  const dim3 g(nb), b(kGramThreads);
  switch (nt) {
    case 1: hipLaunchKernelGGL((k_bgram<1, 2>), g, b, 0, st, V, ld, nr, m1, s, N, gpart); break;
    case 2: hipLaunchKernelGGL((k_bgram<2, 1>), g, b, 0, st, V, ld, nr, m1, s, N, gpart); break;
    case 3: hipLaunchKernelGGL((k_bgram<3, 1>), g, b, 0, st, V, ld, nr, m1, s, N, gpart); break;
    case 4: hipLaunchKernelGGL((k_bgram<4, 1>), g, b, 0, st, V, ld, nr, m1, s, N, gpart); break;
    case 5: hipLaunchKernelGGL((k_bgram<5, 1>), g, b, 0, st, V, ld, nr, m1, s, N, gpart); break;
    default: return hipErrorInvalidValue;
  }
  const int fb = (nr * s + kFinishThreads / 64 - 1) / (kFinishThreads / 64);
  hipLaunchKernelGGL(k_bgram_finish, dim3(fb), dim3(kFinishThreads), 0, st, gpart, nr, s, nb,
                     G_host_dev, seq_flag, seq, done_count);
  return hipGetLastError();
}

hipError_t launch_bupd(double* V, size_t ld, int nq, int m1, int s, size_t N, const double* coef,
                       const double* coef_dev, hipStream_t st) {
  const dim3 g(stream_blocks(N)), b(kRedThreads);
  const size_t nc = (size_t)nq * s + (size_t)s * s;
  const bool by_args = nc <= (size_t)kCoefArgMax;
  CoefArgs a;
  if (by_args) {
    for (size_t i = 0; i < nc; ++i) a.v[i] = coef[i];
  } else if (!coef_dev) {
    return hipErrorInvalidValue;
  }
  switch (s) {
#define X(SS)                                                                                \
  case SS:                                                                                   \
    if (by_args)                                                                             \
      hipLaunchKernelGGL((k_bupd<SS, true>), g, b, 0, st, V, ld, nq, m1, N, nullptr, a);     \
    else                                                                                     \
      hipLaunchKernelGGL((k_bupd<SS, false>), g, b, 0, st, V, ld, nq, m1, N, coef_dev, a);   \
    break;
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rsfde
