// Device-side helpers shared by the FFT-based kernels: the LDS exchange between
// FFT stages, whole forward / inverse sweeps and the XCD-aware block remap.
#pragma once

#include "internal.hpp"

namespace rsfde {

// LDS slot of sequence position p: one pad word every 16 positions breaks the
// power-of-two strides of the last stage across banks.
__device__ __forceinline__ int lds_pad(int p) { return p + (p >> 4); }
constexpr int lds_len(int L) { return L + (L >> 4) + 1; }

// Exchange registers between stage layouts through this FFT's LDS region.
// Real and imaginary parts go through the same region one after the other so
// that the region holds only L scalars.
template <typename T, class F, int TF, int TT>
__device__ __forceinline__ void lds_exchange(cpx<T>* reg, int tau, T* lds) {
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    lds[lds_pad(F::pos(TF, tau, e))] = reg[e].re;
  });
  __syncthreads();
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    reg[e].re = lds[lds_pad(F::pos(TT, tau, e))];
  });
  __syncthreads();
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    lds[lds_pad(F::pos(TF, tau, e))] = reg[e].im;
  });
  __syncthreads();
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    reg[e].im = lds[lds_pad(F::pos(TT, tau, e))];
  });
  __syncthreads();
}

// Forward DIF sweep: natural order (stage-0 positions) in, digit-reversed
// spectrum (last-stage positions) out.
template <typename T, class F>
__device__ __forceinline__ void fft_forward(cpx<T>* reg, int tau, const cpx<T>* __restrict__ tw,
                                            T* lds) {
  static_for<F::NS>([&](auto tt) {
    constexpr int t = decltype(tt)::value;
    F::template dif_stage<T, t>(reg, tau, tw);
    if constexpr (t < F::NS - 1) lds_exchange<T, F, t, t + 1>(reg, tau, lds);
  });
}

// Inverse DIT sweep: digit-reversed spectrum in, L * signal in natural order out.
template <typename T, class F>
__device__ __forceinline__ void fft_inverse(cpx<T>* reg, int tau, const cpx<T>* __restrict__ tw,
                                            T* lds) {
  static_for<F::NS>([&](auto tt) {
    constexpr int t = F::NS - 1 - decltype(tt)::value;
    F::template dit_stage<T, t>(reg, tau, tw);
    if constexpr (t > 0) lds_exchange<T, F, t, t - 1>(reg, tau, lds);
  });
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Remap the block
// index so that consecutive logical tiles (adjacent column strips) run on the
// same XCD and share its L2 lines.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = bid & 7, l = bid >> 3;
  return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

}  // namespace rsfde
