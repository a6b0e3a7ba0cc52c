// The sine-transform preconditioner (Section 4.1 of the paper) as dense GEMMs
// on the gfx950 matrix cores, BF16 operands with FP32 accumulation:
//   W = S_y V S_x,  R1 = W / E1,  R2 = W / E2,  Y_k = S_y R_k S_x,
//   z = mask * Y1 + (1 - mask) * Y2,
// with S the orthonormal DST-I matrix sqrt(2/(n+1)) sin(pi i j/(n+1)) (symmetric,
// so every product below takes a sine matrix as its right operand, read by rows)
// and E1 = 1 - kx lx_i - ky ly_j, E2 = E1 + dt/eta.  Four kinds of launches:
//   mode 0: C = (sig V) S_x,   stored transposed           -> A1T [n1p][n2p]
//   mode 1: C = A1T S_y (= W^T), epilogue R1T = C/E1^T, R2T = C/E2^T
//   mode 2: C = [R1T; R2T] S_y, stored transposed          -> G [2][n2p][n1p]
//   mode 3: C = G_w S_x (= Y_w), written to z where mask == (w == 0)   (w = 0, 1)
// All dimensions are padded to multiples of 128; the padded parts of the sine
// tables are zero, so padding never leaks into the result.  Rounding: sine
// matrices in BF16 (nearest even), FP32 accumulation, the eigenvalue scaling
// in FP32.  In the two forward products (modes 0 and 1) both operands are
// carried as BF16 pairs hi + lo (about 16 significant bits; three MFMAs
// hi*hi + hi*lo + lo*hi per fragment): the scaling 1/E spans up to ~1e5 at
// stiff parameters, so plain BF16 rounding (2^-9) of either the data or the
// sine matrix leaks into the low frequencies, is amplified by the scaling and
// ruins the apply on Krylov vectors dominated by high frequencies.  After the
// scaling (modes 2 and 3) single BF16 operands suffice.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace rsfde {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

constexpr int kBM = 128, kBN = 128, kBK = 32;
constexpr int kLdsStride = kBK + 8;  // bf16 per LDS row (80 bytes: 16-byte aligned, skewed banks)
constexpr int kGemmThreads = 256;

struct GemmArgs {
  int mode;
  int M, N, K;            // padded sizes of this product (multiples of 128)
  const __bf16* A;        // row-major [M][K] (modes 1-3)
  const __bf16* A_lo;     // mode 1: low part of the split operand
  const double* V;        // mode 0: FP64 input [n2][n1] (unpadded)
  const double* sig;      // mode 0: optional scale of V
  const __bf16* S;        // right operand: symmetric [K][N] == [N][K]
  const __bf16* S_lo;     // modes 0-1: low part of the sine matrix
  __bf16* out;            // modes 0-2
  __bf16* out_lo;         // mode 0: low part of the split output
  int ld_out;             // leading dimension of the output
  __bf16* out2;           // mode 1: R2T
  const float* lamx;      // mode 1: unit-k eigenvalues, natural order, padded with 0
  const float* lamy;
  float kx, ky, dpen;
  int n1, n2;             // true sizes
  int n1p, n2p;           // padded sizes
  const uint8_t* mask;    // mode 3
  double* z;              // mode 3
  int which;              // mode 3: 0 -> write Y1 where mask == 1, 1 -> Y2 where mask == 0
};

__device__ __forceinline__ void load_tile_bf16(const __bf16* src, int ld, int r0, int c0, int t,
                                               bf16x8 (&reg)[2]) {
  const int row = t >> 1, col = (t & 1) * 16;
  const bf16x8* p = reinterpret_cast<const bf16x8*>(src + (size_t)(r0 + row) * ld + c0 + col);
  reg[0] = p[0];
  reg[1] = p[1];
}

// Mode 0: the A operand is the FP64 input (times sig), guarded to n2 x n1,
// split into BF16 hi + lo parts.
__device__ __forceinline__ void load_tile_fp64(const GemmArgs& g, int r0, int c0, int t, double s,
                                               bf16x8 (&hi)[2], bf16x8 (&lo)[2]) {
  const int row = r0 + (t >> 1), col = c0 + (t & 1) * 16;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = col + 8 * h + e;
      const double v = (row < g.n2 && c < g.n1) ? s * g.V[(size_t)row * g.n1 + c] : 0.0;
      const __bf16 a = (__bf16)(float)v;
      hi[h][e] = a;
      lo[h][e] = (__bf16)(float)(v - (double)(float)a);
    }
  }
}

__device__ __forceinline__ void store_tile(__bf16* lds, int t, const bf16x8 (&reg)[2]) {
  const int row = t >> 1, col = (t & 1) * 16;
  bf16x8* p = reinterpret_cast<bf16x8*>(lds + row * kLdsStride + col);
  p[0] = reg[0];
  p[1] = reg[1];
}

__global__ __launch_bounds__(kGemmThreads) void k_gemm_bf16(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[2][kBM * kLdsStride];
  __shared__ __attribute__((aligned(16))) __bf16 Al[2][kBM * kLdsStride];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][kBN * kLdsStride];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][kBN * kLdsStride];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
  const double sgm = (g.mode == 0 && g.sig) ? *g.sig : 1.0;
  const bool split = g.mode <= 1;

  floatx16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

  bf16x8 ra[2], rl[2], rb[2], rbl[2];
  const int KT = g.K / kBK;
  auto load = [&](int k0) {
    if (g.mode == 0) {
      load_tile_fp64(g, m0, k0, t, sgm, ra, rl);
    } else {
      load_tile_bf16(g.A, g.K, m0, k0, t, ra);
      if (split) load_tile_bf16(g.A_lo, g.K, m0, k0, t, rl);
    }
    load_tile_bf16(g.S, g.K, n0, k0, t, rb);  // rows n0.. of the symmetric S = columns of S
    if (split) load_tile_bf16(g.S_lo, g.K, n0, k0, t, rbl);
  };
  auto stash = [&](int buf) {
    store_tile(As[buf], t, ra);
    if (split) store_tile(Al[buf], t, rl);
    store_tile(Bs[buf], t, rb);
    if (split) store_tile(Bl[buf], t, rbl);
  };
  load(0);
  stash(0);
  __syncthreads();

  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) load((kt + 1) * kBK);
#pragma unroll
    for (int ks = 0; ks < kBK / 16; ++ks) {
      const int kk = ks * 16 + 8 * (lane >> 5);
      bf16x8 fa[2], fb[2];
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) {
        const int col = wn * 64 + nj * 32 + (lane & 31);
        fb[nj] = *reinterpret_cast<const bf16x8*>(&Bs[cur][col * kLdsStride + kk]);
      }
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) {
        const int row = wm * 64 + mi * 32 + (lane & 31);
        fa[mi] = *reinterpret_cast<const bf16x8*>(&As[cur][row * kLdsStride + kk]);
      }
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
          acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[mi], fb[nj], acc[mi][nj], 0, 0, 0);
      if (split) {
        bf16x8 fl[2];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
          const int row = wm * 64 + mi * 32 + (lane & 31);
          fl[mi] = *reinterpret_cast<const bf16x8*>(&Al[cur][row * kLdsStride + kk]);
        }
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)  // lo(A) * hi(S)
#pragma unroll
          for (int nj = 0; nj < 2; ++nj)
            acc[mi][nj] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(fl[mi], fb[nj], acc[mi][nj], 0, 0, 0);
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
          const int col = wn * 64 + nj * 32 + (lane & 31);
          fb[nj] = *reinterpret_cast<const bf16x8*>(&Bl[cur][col * kLdsStride + kk]);
        }
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)  // hi(A) * lo(S)
#pragma unroll
          for (int nj = 0; nj < 2; ++nj)
            acc[mi][nj] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[mi], fb[nj], acc[mi][nj], 0, 0, 0);
      }
    }
    if (kt + 1 < KT) stash(cur ^ 1);
    __syncthreads();
  }

  // Epilogue.  Accumulator layout of the 32x32 MFMA tile: lane l, register r
  // holds row 8*(r/4) + 4*(l/32) + r%4, column l%32.
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = m0 + wm * 64 + mi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int j = n0 + wn * 64 + nj * 32 + (lane & 31);
        const float c = acc[mi][nj][r];
        if (g.mode == 0) {
          const __bf16 h = (__bf16)c;  // A1T[x][y] as hi + lo
          g.out[(size_t)j * g.ld_out + i] = h;
          g.out_lo[(size_t)j * g.ld_out + i] = (__bf16)(c - (float)h);
        } else if (g.mode == 1) {
          // C[a][b] = W[b][a]: a = x frequency (row), b = y frequency (column)
          const float e1 = 1.0f - g.kx * g.lamx[i] - g.ky * g.lamy[j];
          const float e2 = e1 + g.dpen;
          g.out[(size_t)i * g.ld_out + j] = (__bf16)(c / e1);
          g.out2[(size_t)i * g.ld_out + j] = (__bf16)(c / e2);
        } else if (g.mode == 2) {
          // rows [0, n1p) are (S_y R1)^T, rows [n1p, 2 n1p) are (S_y R2)^T
          const int w = i >= g.n1p ? 1 : 0;
          const int x = i - w * g.n1p;
          g.out[(size_t)w * g.n2p * g.n1p + (size_t)j * g.ld_out + x] = (__bf16)c;
        } else {
          if (i < g.n2 && j < g.n1) {
            const size_t idx = (size_t)i * g.n1 + j;
            const bool inside = g.mask[idx] != 0;
            if (inside == (g.which == 0)) g.z[idx] = (double)c;
          }
        }
      }
}

hipError_t launch_pc_gemm_bf16(const double* v, const double* sig, double* z, const uint8_t* mask,
                               const __bf16* Sx, const __bf16* Sy, const __bf16* Sx_lo,
                               const __bf16* Sy_lo, const float* lamx,
                               const float* lamy, __bf16* A1T, __bf16* R12T, __bf16* G,
                               int n1, int n2, int n1p, int n2p, double kx, double ky,
                               double dpen, hipStream_t s) {
  __bf16* A1T_lo = A1T + (size_t)n1p * n2p;
  GemmArgs g{};
  g.n1 = n1;
  g.n2 = n2;
  g.n1p = n1p;
  g.n2p = n2p;
  g.kx = (float)kx;
  g.ky = (float)ky;
  g.dpen = (float)dpen;
  const dim3 blk(kGemmThreads);
  // mode 0: (sig V)[n2p x n1p] . S_x -> A1T [n1p][n2p]
  g.mode = 0;
  g.M = n2p; g.N = n1p; g.K = n1p;
  g.V = v; g.sig = sig; g.S = Sx; g.S_lo = Sx_lo; g.out = A1T; g.out_lo = A1T_lo; g.ld_out = n2p;
  hipLaunchKernelGGL(k_gemm_bf16, dim3(g.N / kBN, g.M / kBM), blk, 0, s, g);
  // mode 1: A1T [n1p x n2p] . S_y -> R1T, R2T [n1p][n2p]
  g.mode = 1;
  g.M = n1p; g.N = n2p; g.K = n2p;
  g.A = A1T; g.A_lo = A1T_lo; g.S = Sy; g.S_lo = Sy_lo; g.out = R12T;
  g.out2 = R12T + (size_t)n1p * n2p;
  g.ld_out = n2p;
  g.lamx = lamx; g.lamy = lamy;
  hipLaunchKernelGGL(k_gemm_bf16, dim3(g.N / kBN, g.M / kBM), blk, 0, s, g);
  // mode 2: [R1T; R2T] [2 n1p x n2p] . S_y -> G [2][n2p][n1p]
  g.mode = 2;
  g.M = 2 * n1p; g.N = n2p; g.K = n2p;
  g.A = R12T; g.S = Sy; g.out = G; g.ld_out = n1p;
  hipLaunchKernelGGL(k_gemm_bf16, dim3(g.N / kBN, g.M / kBM), blk, 0, s, g);
  // mode 3: G_w [n2p x n1p] . S_x -> z (mask select)
  g.mode = 3;
  g.M = n2p; g.N = n1p; g.K = n1p;
  g.S = Sx; g.mask = mask; g.z = z;
  for (int w = 0; w < 2; ++w) {
    g.A = G + (size_t)w * n2p * n1p;
    g.which = w;
    hipLaunchKernelGGL(k_gemm_bf16, dim3(g.N / kBN, g.M / kBM), blk, 0, s, g);
  }
  return hipGetLastError();
}

}  // namespace rsfde
