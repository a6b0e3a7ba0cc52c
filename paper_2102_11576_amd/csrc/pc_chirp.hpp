// The sine-transform preconditioner of Section 4.1 for grids whose n + 1 is not
// a power of two.  P_hat^{-1} is the same operator as in pc_kernels.hpp:
//   z = mask * S_y (W / E1) S_x + (1 - mask) * S_y (W / E2) S_x,  W = S_y V S_x,
// E1 = 1 - kx lx_i - ky ly_j, E2 = E1 + dt/eta, S the orthonormal DST-I
// sqrt(2/(n+1)) sin(pi j k / (n+1)) (Section 4.1).  Only the way a length-n
// DST-I is computed differs.
//
// Chirp form of the DST-I (Bluestein's identity jk = (j^2 + k^2 - (k-j)^2)/2):
//   sum_j x_j sin(pi j k / M) = Im( c_k sum_j (c_j x_j) conj(c_{k-j}) ),
//   c_j = exp(i pi j^2 / (2M)),  M = n + 1,
// i.e. a chirp premultiply, a Toeplitz convolution with the even kernel
// exp(-i pi m^2 / (2M)), |m| < n, and a chirp postmultiply.  The convolution
// is circular of power-of-two length L >= 2n - 1 (no wrap-around reaches
// outputs 0..n-1), done with the register-resident FFT of fft_engine.hpp; the
// kernel's spectrum `khat` (times sqrt(2/M) / L) is a set-up table in
// register-position order, so the pointwise product needs no reordering.
// Every line is one complex FFT pair (real lines cannot share one: the chirp
// mixes real and imaginary parts), about four times the work of the
// odd-extension form, which the library uses whenever n + 1 is a power of two.
//
// Passes (T = double or float internals; v and z are FP64):
//   rows:    W1 = rows of (sig * v) transformed along x           [n2][n1] T
//   columns: W  = W1 transformed along y; Y1 = S_y(W / E1), Y2 = S_y(W / E2)
//   rows:    z  = S_x of Y1 rows where mask = 1, of Y2 rows where mask = 0
#pragma once
#include "fft_common.hpp"

namespace rsfde {

template <int L>
struct CdCfg {
  using F = Fft<L, fft_pts(L)>;
  static constexpr int TPF = F::TPF;
  static constexpr int BR = (256 / TPF) > 0 ? (256 / TPF) : 1;  // lines per row block
  static constexpr int BC = (256 / TPF) > 16 ? 16 : ((256 / TPF) > 0 ? (256 / TPF) : 1);
  static constexpr int THR_R = BR * TPF;
  static constexpr int THR_C = BC * TPF;
};

// In: reg[e].re = x at sequence position pos(0, tau, e) (zero at positions >= n).
// Out: reg[e].re = (S x) at the same position (unspecified at positions >= n).
template <typename T, class F, int ST = 1>
__device__ __forceinline__ void chirp_dst(cpx<T>* reg, int tau, const cpx<T>* __restrict__ chn,
                                          const cpx<T>* __restrict__ khat,
                                          const cpx<T>* __restrict__ tw, T* lds, int n) {
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    const cpx<T> c = p < n ? chn[p] : cpx<T>{T(0), T(0)};
    const T x = reg[e].re;
    reg[e].re = x * c.re;
    reg[e].im = x * c.im;
  });
  fft_forward<T, F, true, ST>(reg, tau, tw, lds);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    reg[e] = cmul(reg[e], khat[F::pos(F::NS - 1, tau, e)]);
  });
  fft_inverse<T, F, true, ST>(reg, tau, tw, lds);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    const cpx<T> c = p < n ? chn[p] : cpx<T>{T(0), T(0)};
    reg[e].re = c.re * reg[e].im + c.im * reg[e].re;  // Im(c * y)
  });
}

// Rows: W1[r] = S_x (sig * v[r]).
template <typename T, int L>
__global__ __launch_bounds__(CdCfg<L>::THR_R) void k_cd_rows_fwd(
    const double* __restrict__ v, const double* __restrict__ sig, T* __restrict__ out,
    const cpx<T>* __restrict__ chn, const cpx<T>* __restrict__ khat,
    const cpx<T>* __restrict__ tw, int n1, int n2) {
  using C = CdCfg<L>;
  using F = typename C::F;
  __shared__ T lds[C::BR * lds_len(L)];
  const int b = threadIdx.x / F::TPF, tau = threadIdx.x % F::TPF;
  const int r = blockIdx.x * C::BR + b;
  const bool vr = r < n2;
  const double sc = sig ? *sig : 1.0;
  cpx<T> reg[F::PP];
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    reg[e].re = (vr && p < n1) ? (T)(sc * v[(size_t)r * n1 + p]) : T(0);
    reg[e].im = T(0);
  });
  chirp_dst<T, F>(reg, tau, chn, khat, tw, lds + b * lds_len(L), n1);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    if (vr && p < n1) out[(size_t)r * n1 + p] = reg[e].re;
  });
}

// Columns: W = S_y W1 column, then Y1 = S_y(W / E1) and Y2 = S_y(W / E2).
// Thread layout (tau, b) with b fastest: a wavefront touches BC adjacent
// columns of each row it reads.
template <typename T, int L>
__global__ __launch_bounds__(CdCfg<L>::THR_C) void k_cd_cols(
    const T* __restrict__ in, T* __restrict__ Y1, T* __restrict__ Y2,
    const double* __restrict__ lamx, const double* __restrict__ lamy,
    const cpx<T>* __restrict__ chn, const cpx<T>* __restrict__ khat,
    const cpx<T>* __restrict__ tw, int n1, int n2, double kx, double ky, double dpen) {
  using C = CdCfg<L>;
  using F = typename C::F;
  __shared__ T lds[C::BC * lds_len(L)];
  const int b = threadIdx.x % C::BC, tau = threadIdx.x / C::BC;
  const int c = xcd_remap(blockIdx.x, gridDim.x) * C::BC + b;
  const bool vc = c < n1;
  T* my = lds + b;  // regions interleaved (stride BC)
  cpx<T> reg[F::PP];
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    reg[e].re = (vc && p < n2) ? in[(size_t)p * n1 + c] : T(0);
    reg[e].im = T(0);
  });
  chirp_dst<T, F, C::BC>(reg, tau, chn, khat, tw, my, n2);
  const double ax = 1.0 - kx * (vc ? lamx[c] : 0.0);
  T w[F::PP];
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    const T e1 = (T)(ax - ky * (p < n2 ? lamy[p] : 0.0));
    w[e] = p < n2 ? reg[e].re : T(0);
    reg[e].re = w[e] / e1;
  });
  chirp_dst<T, F, C::BC>(reg, tau, chn, khat, tw, my, n2);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    if (vc && p < n2) Y1[(size_t)p * n1 + c] = reg[e].re;
    const T e2 = (T)(ax + dpen - ky * (p < n2 ? lamy[p] : 0.0));
    reg[e].re = w[e] / e2;
  });
  chirp_dst<T, F, C::BC>(reg, tau, chn, khat, tw, my, n2);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    if (vc && p < n2) Y2[(size_t)p * n1 + c] = reg[e].re;
  });
}

// Rows: line u = 2r + k transforms row r of Y1 (k = 0) or Y2 (k = 1) along x
// and writes z where the mask selects that branch; the two lines of a row
// write disjoint points, so no combine step is needed.
template <typename T, int L>
__global__ __launch_bounds__(CdCfg<L>::THR_R) void k_cd_rows_inv(
    const T* __restrict__ Y1, const T* __restrict__ Y2, const uint8_t* __restrict__ mask,
    double* __restrict__ z, const cpx<T>* __restrict__ chn, const cpx<T>* __restrict__ khat,
    const cpx<T>* __restrict__ tw, int n1, int n2) {
  using C = CdCfg<L>;
  using F = typename C::F;
  __shared__ T lds[C::BR * lds_len(L)];
  const int b = threadIdx.x / F::TPF, tau = threadIdx.x % F::TPF;
  const int u = blockIdx.x * C::BR + b;
  const int r = u >> 1, k = u & 1;
  const bool vr = r < n2;
  const T* src = k ? Y2 : Y1;
  cpx<T> reg[F::PP];
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    reg[e].re = (vr && p < n1) ? src[(size_t)r * n1 + p] : T(0);
    reg[e].im = T(0);
  });
  chirp_dst<T, F>(reg, tau, chn, khat, tw, lds + b * lds_len(L), n1);
  const uint8_t want = k ? 0 : 1;
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    if (vr && p < n1) {
      const size_t i = (size_t)r * n1 + p;
      if ((mask[i] != 0) == (want != 0)) z[i] = (double)reg[e].re;
    }
  });
}

// Columns without scaling (the three-dimensional plans' y transforms): out =
// S_y in for the columns c < ncol of `batch` slices [rows][ncol], slice b at
// offset b * bstride; with inB given, grid dimension z = 1 transforms inB into
// outB in the same launch.  in and out must not overlap.
template <typename T, int L>
__global__ __launch_bounds__(CdCfg<L>::THR_C) void k_cd_dst_cols(
    const T* __restrict__ inA, T* __restrict__ outA, const T* __restrict__ inB,
    T* __restrict__ outB, const cpx<T>* __restrict__ chn, const cpx<T>* __restrict__ khat,
    const cpx<T>* __restrict__ tw, int ncol, int rows, size_t bstride) {
  using C = CdCfg<L>;
  using F = typename C::F;
  __shared__ T lds[C::BC * lds_len(L)];
  const size_t off = (size_t)blockIdx.y * bstride;
  const T* in = (blockIdx.z ? inB : inA) + off;
  T* out = (blockIdx.z ? outB : outA) + off;
  const int b = threadIdx.x % C::BC, tau = threadIdx.x / C::BC;
  const int c = xcd_remap(blockIdx.x, gridDim.x) * C::BC + b;
  const bool vc = c < ncol;
  T* my = lds + b;  // regions interleaved (stride BC)
  cpx<T> reg[F::PP];
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    reg[e].re = (vc && p < rows) ? in[(size_t)p * ncol + c] : T(0);
    reg[e].im = T(0);
  });
  chirp_dst<T, F, C::BC>(reg, tau, chn, khat, tw, my, rows);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    if (vc && p < rows) out[(size_t)p * ncol + c] = reg[e].re;
  });
}

#define RSFDE_CD_CASES(X) \
  X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192)

template <typename T>
hipError_t launch_cd_rows_fwd(int L, const double* v, const double* sig, T* out, const void* chn,
                              const void* khat, const void* tw, int n1, int n2, hipStream_t s) {
  switch (L) {
#define X(LL)                                                                             \
  case LL: {                                                                              \
    using C = CdCfg<LL>;                                                                  \
    const int blocks = (n2 + C::BR - 1) / C::BR;                                          \
    hipLaunchKernelGGL((k_cd_rows_fwd<T, LL>), dim3(blocks), dim3(C::THR_R), 0, s, v, sig, \
                       out, (const cpx<T>*)chn, (const cpx<T>*)khat, (const cpx<T>*)tw, n1, n2); \
    return hipGetLastError();                                                             \
  }
    RSFDE_CD_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_cd_cols(int L, const T* in, T* Y1, T* Y2, const double* lamx,
                          const double* lamy, const void* chn, const void* khat, const void* tw,
                          int n1, int n2, double kx, double ky, double dpen, hipStream_t s) {
  switch (L) {
#define X(LL)                                                                                  \
  case LL: {                                                                                   \
    using C = CdCfg<LL>;                                                                       \
    const int blocks = (n1 + C::BC - 1) / C::BC;                                               \
    hipLaunchKernelGGL((k_cd_cols<T, LL>), dim3(blocks), dim3(C::THR_C), 0, s, in, Y1, Y2, lamx, \
                       lamy, (const cpx<T>*)chn, (const cpx<T>*)khat, (const cpx<T>*)tw, n1, n2, \
                       kx, ky, dpen);                                                          \
    return hipGetLastError();                                                                  \
  }
    RSFDE_CD_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_cd_dst_cols(int L, const T* inA, T* outA, const T* inB, T* outB, const void* chn,
                              const void* khat, const void* tw, int ncol, int rows, int batch,
                              size_t bstride, hipStream_t s) {
  if (batch < 1 || batch > 65535 || ncol < 1 || rows < 1 || !inA || !outA || (!inB) != (!outB))
    return hipErrorInvalidValue;
  switch (L) {
#define X(LL)                                                                                  \
  case LL: {                                                                                   \
    using C = CdCfg<LL>;                                                                       \
    const dim3 grid((ncol + C::BC - 1) / C::BC, batch, inB ? 2 : 1);                           \
    hipLaunchKernelGGL((k_cd_dst_cols<T, LL>), grid, dim3(C::THR_C), 0, s, inA, outA, inB,     \
                       outB, (const cpx<T>*)chn, (const cpx<T>*)khat, (const cpx<T>*)tw, ncol, \
                       rows, bstride);                                                         \
    return hipGetLastError();                                                                  \
  }
    RSFDE_CD_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_cd_rows_inv(int L, const T* Y1, const T* Y2, const uint8_t* mask, double* z,
                              const void* chn, const void* khat, const void* tw, int n1, int n2,
                              hipStream_t s) {
  switch (L) {
#define X(LL)                                                                                 \
  case LL: {                                                                                  \
    using C = CdCfg<LL>;                                                                      \
    const int blocks = (2 * n2 + C::BR - 1) / C::BR;                                          \
    hipLaunchKernelGGL((k_cd_rows_inv<T, LL>), dim3(blocks), dim3(C::THR_R), 0, s, Y1, Y2, mask, \
                       z, (const cpx<T>*)chn, (const cpx<T>*)khat, (const cpx<T>*)tw, n1, n2);  \
    return hipGetLastError();                                                                 \
  }
    RSFDE_CD_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace rsfde
