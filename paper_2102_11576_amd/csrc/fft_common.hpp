// Device-side helpers shared by the FFT-based kernels: the LDS exchange between
// FFT stages, whole forward / inverse sweeps and the XCD-aware block remap.
#pragma once

#include "internal.hpp"

namespace rsfde {

// LDS slot of sequence position p: one pad word every 16 positions breaks the
// power-of-two strides of the last stage across banks.
__device__ __forceinline__ int lds_pad(int p) { return p + (p >> 4); }
constexpr int lds_len(int L) { return L + (L >> 4) + 1; }

// LDS slots of a stage layout.  For most stages the slot of register e is
// slot(tau, 0) + delta(e) with delta independent of the thread (checked here
// at compile time over all threads): the exchange then addresses LDS through
// one base register and immediate offsets instead of one address register per
// point, which keeps the FFT kernels' register footprint low.
template <class F, int t>
struct LdsLayout {
  static constexpr int pad(int p) { return p + (p >> 4); }
  static constexpr int delta(int e) { return pad(F::pos(t, 0, e)) - pad(F::pos(t, 0, 0)); }
  static constexpr bool check() {
    for (int tau = 0; tau < F::TPF; ++tau)
      for (int e = 0; e < F::PP; ++e)
        if (pad(F::pos(t, tau, e)) - pad(F::pos(t, tau, 0)) != delta(e)) return false;
    return true;
  }
  static constexpr bool linear = check();
};

// ST: LDS stride between consecutive slots of one FFT.  A block that runs BC
// FFTs with the FFT index fastest in the thread layout (the column kernels)
// interleaves their regions (slot * BC + b): the lanes of a wavefront then
// touch consecutive words, free of bank conflicts.
template <typename T, class F, int t, int ST>
__device__ __forceinline__ void lds_put(const cpx<T>* reg, int tau, T* lds, bool im) {
  using LL = LdsLayout<F, t>;
  if constexpr (LL::linear) {
    T* b = lds + lds_pad(F::pos(t, tau, 0)) * ST;
    static_for<F::PP>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      b[LL::delta(e) * ST] = im ? reg[e].im : reg[e].re;
    });
  } else {
    static_for<F::PP>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      lds[lds_pad(F::pos(t, tau, e)) * ST] = im ? reg[e].im : reg[e].re;
    });
  }
}

template <typename T, class F, int t, int ST>
__device__ __forceinline__ void lds_get(cpx<T>* reg, int tau, const T* lds, bool im) {
  using LL = LdsLayout<F, t>;
  if constexpr (LL::linear) {
    const T* b = lds + lds_pad(F::pos(t, tau, 0)) * ST;
    static_for<F::PP>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      (im ? reg[e].im : reg[e].re) = b[LL::delta(e) * ST];
    });
  } else {
    static_for<F::PP>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      (im ? reg[e].im : reg[e].re) = lds[lds_pad(F::pos(t, tau, e)) * ST];
    });
  }
}

// Thread that holds sequence position p in the layout of stage t (inverse of
// F::pos: p = (beta / s) bl + beta % s + m s, beta = tau + u TPF).
template <class F>
constexpr int owner_of(int t, int p) {
  const int s = F::stride(t), bl = F::blocklen(t);
  const int beta = (p / bl) * s + (p % s);
  return beta % F::TPF;
}

// True when the exchange from layout TF to layout TT only moves data among
// the threads of one wavefront: every position's owners in both layouts fall
// in the same group of TW consecutive threads (TW = threads of one FFT in a
// wavefront: 64, or 64 / BC with BC FFTs interleaved per wavefront).
template <class F, int TF, int TT, int TW>
constexpr bool exchange_in_wave() {
  if (F::TPF < TW || TW < 1) return false;
  for (int p = 0; p < F::TPF * F::PP; ++p)
    if (owner_of<F>(TF, p) / TW != owner_of<F>(TT, p) / TW) return false;
  return true;
}

// Exchange registers between stage layouts through this FFT's LDS region.
// Real and imaginary parts go through the same region one after the other so
// that the region holds only L scalars.  When the exchange stays inside each
// wavefront (TW > 0 and exchange_in_wave), no block barrier is needed: a
// wavefront's LDS operations complete in order, and every wavefront only
// rewrites the positions it reads (the fences keep the compiler from
// reordering the LDS accesses).
template <typename T, class F, int TF, int TT, int ST = 1, int TW = 0>
__device__ __forceinline__ void lds_exchange(cpx<T>* reg, int tau, T* lds, bool act = true) {
  constexpr bool wave_local = TW > 0 && exchange_in_wave<F, TF, TT, TW>();
  auto sync = [] {
    if constexpr (wave_local) {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    } else {
      __syncthreads();
    }
  };
  // act = false: a thread with no transform of its own still takes part in
  // every block barrier (the block's other transforms need them).
  if (act) lds_put<T, F, TF, ST>(reg, tau, lds, false);
  sync();
  if (act) lds_get<T, F, TT, ST>(reg, tau, lds, false);
  sync();
  if (act) lds_put<T, F, TF, ST>(reg, tau, lds, true);
  sync();
  if (act) lds_get<T, F, TT, ST>(reg, tau, lds, true);
  sync();
}

// Forces the values of all registers to be computed here.  Without it the
// compiler sinks the last butterfly of a sweep into the (conditional) stores
// or pointwise products that follow, which keeps the whole butterfly tree
// live and costs a wave of occupancy.
template <typename T, int N>
__device__ __forceinline__ void materialize(cpx<T>* r) {
#pragma unroll
  for (int e = 0; e < N; ++e) asm volatile("" : "+v"(r[e].re), "+v"(r[e].im));
}

// The twiddle roots of every stage of one sweep (one per stage but the last),
// loaded up front so that their latency overlaps other work instead of
// following each exchange.
template <typename T, class F>
struct Roots {
  cpx<T> w[F::NS > 1 ? F::NS - 1 : 1] = {};
  __device__ __forceinline__ void load_fwd(int tau, const cpx<T>* __restrict__ tw) {
    static_for<F::NS - 1>([&](auto tt) {
      constexpr int t = decltype(tt)::value;
      w[t] = F::template dif_root<T, t>(tau, tw);
    });
  }
  __device__ __forceinline__ void load_inv(int tau, const cpx<T>* __restrict__ tw) {
    static_for<F::NS - 1>([&](auto tt) {
      constexpr int t = decltype(tt)::value;
      w[t] = F::template dit_root<T, t>(tau, tw);
    });
  }
  __device__ __forceinline__ cpx<T> at(int t) const { return w[t < F::NS - 1 ? t : 0]; }
};

// Forward DIF sweep: natural order (stage-0 positions) in, digit-reversed
// spectrum (last-stage positions) out.  rt: the roots (Roots::load_fwd).
template <typename T, class F, bool MAT = true, int ST = 1, int TW = 64 / ST>
__device__ __forceinline__ void fft_forward_r(cpx<T>* reg, int tau, const Roots<T, F>& rt,
                                              T* lds, bool act = true) {
  static_for<F::NS>([&](auto tt) {
    constexpr int t = decltype(tt)::value;
    if (act) F::template dif_stage_w<T, t>(reg, rt.at(t));
    if constexpr (t < F::NS - 1) lds_exchange<T, F, t, t + 1, ST, TW>(reg, tau, lds, act);
  });
  if constexpr (MAT) materialize<T, F::PP>(reg);
}
template <typename T, class F, bool MAT = true, int ST = 1, int TW = 64 / ST>
__device__ __forceinline__ void fft_forward(cpx<T>* reg, int tau, const cpx<T>* __restrict__ tw,
                                            T* lds, bool act = true) {
  Roots<T, F> rt;
  rt.load_fwd(tau, tw);
  fft_forward_r<T, F, MAT, ST, TW>(reg, tau, rt, lds, act);
}

// Inverse DIT sweep: digit-reversed spectrum in, L * signal in natural order
// out.  rt: the roots (Roots::load_inv).
template <typename T, class F, bool MAT = true, int ST = 1, int TW = 64 / ST>
__device__ __forceinline__ void fft_inverse_r(cpx<T>* reg, int tau, const Roots<T, F>& rt,
                                              T* lds, bool act = true) {
  static_for<F::NS>([&](auto tt) {
    constexpr int t = F::NS - 1 - decltype(tt)::value;
    if (act) F::template dit_stage_w<T, t>(reg, rt.at(t));
    if constexpr (t > 0) lds_exchange<T, F, t, t - 1, ST, TW>(reg, tau, lds, act);
  });
  if constexpr (MAT) materialize<T, F::PP>(reg);
}
template <typename T, class F, bool MAT = true, int ST = 1, int TW = 64 / ST>
__device__ __forceinline__ void fft_inverse(cpx<T>* reg, int tau, const cpx<T>* __restrict__ tw,
                                            T* lds, bool act = true) {
  Roots<T, F> rt;
  rt.load_inv(tau, tw);
  fft_inverse_r<T, F, MAT, ST, TW>(reg, tau, rt, lds, act);
}

// Strip-tiled layout of a [rows][cols] array of intermediates: tiles of
// [2 rows][4 columns], the tiles of one 4-column strip stored row pair after
// row pair, the strips one after another.  A column pass that owns a strip
// then reads and writes it contiguously; a row pass that owns a row pair moves
// 64-byte pieces (FP64).  hp = row pairs per strip (ceil(rows / 2)); the
// array holds 8 ceil(cols / 4) hp values.
__device__ __forceinline__ size_t tile_index(int r, int c, int hp) {
  return ((size_t)(c >> 2) * hp + (r >> 1)) * 8 + (r & 1) * 4 + (c & 3);
}
template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
};
template <>
struct Vec2<float> {
  using type = float2;
};

// Workgroups are dispatched round-robin over the 8 XCDs.  Remap the block
// index so that consecutive logical tiles (adjacent column strips) run on the
// same XCD and share its L2 lines.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = bid & 7, l = bid >> 3;
  return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

}  // namespace rsfde
