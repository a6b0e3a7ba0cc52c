// Register-resident power-of-two FFT building blocks for gfx950.
//
// An FFT of length L (a power of two) is spread over TPF = L / P threads, each
// holding P complex points in registers.  The forward transform is an in-place
// decimation-in-frequency (DIF) Cooley-Tukey sweep with radix P stages (the
// last stage takes the remaining radix); between stages the points are
// exchanged through LDS.  After the sweep, register e of thread tau holds the
// spectrum at frequency freq(pos(last, tau, e)) (mixed-radix digit reversal).
// The inverse is the exact reverse sweep (decimation in time, conjugate
// twiddles), so a pointwise operation on the digit-reversed spectrum can sit
// between forward and inverse with no reordering at all: this is what the
// Toeplitz convolutions and the sine-transform preconditioner use.  The
// inverse returns L times the input (no 1/L scaling).
//
// The index arithmetic is __host__ __device__ so that the same functions
// generate the host-side tables (symbol in position order, eigenvalue tables)
// and can be exercised by a CPU self-test.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define RS_HD __host__ __device__ __forceinline__
#else
#define RS_HD inline
#endif

#include <type_traits>
#include <utility>

namespace rsfde {

template <typename T>
struct cpx {
  T re, im;
};

template <typename T>
RS_HD cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
RS_HD cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
RS_HD cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
RS_HD cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// ---------------------------------------------------------------------------
// Compile-time loop.
// ---------------------------------------------------------------------------
template <class F, int... I>
RS_HD void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
RS_HD void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------------------
// Multiplication by the constant root of unity exp(SIGN * 2 pi i K / R),
// R <= 16, with exact special cases for multiples of pi/4.
// ---------------------------------------------------------------------------
template <typename T, int K, int R, int SIGN>
RS_HD cpx<T> mul_root(cpx<T> x) {
  constexpr int K16 = (K * 16) / R;  // angle in units of 2 pi / 16
  static_assert((K * 16) % R == 0, "R must divide 16*K");
  constexpr int k = K16 & 15;
  // cos / sin of 2 pi k / 16 for k = 0..15
  constexpr double C1 = 0.92387953251128675613;  // cos(pi/8)
  constexpr double C2 = 0.70710678118654752440;  // cos(pi/4)
  constexpr double C3 = 0.38268343236508977173;  // cos(3pi/8)
  constexpr double cs[16] = {1, C1, C2, C3, 0, -C3, -C2, -C1, -1, -C1, -C2, -C3, 0, C3, C2, C1};
  constexpr double sn[16] = {0, C3, C2, C1, 1, C1, C2, C3, 0, -C3, -C2, -C1, -1, -C1, -C2, -C3};
  if constexpr (k == 0) {
    return x;
  } else if constexpr (k == 8) {
    return {-x.re, -x.im};
  } else if constexpr (k == 4) {  // multiply by SIGN * i
    if constexpr (SIGN > 0) return {-x.im, x.re};
    else return {x.im, -x.re};
  } else if constexpr (k == 12) {  // multiply by -SIGN * i
    if constexpr (SIGN > 0) return {x.im, -x.re};
    else return {-x.im, x.re};
  } else if constexpr (k == 2 || k == 6 || k == 10 || k == 14) {
    // (+-1 +- i)/sqrt(2): c and s have equal magnitude
    constexpr T c = (T)cs[k];
    constexpr T s = (T)(SIGN > 0 ? sn[k] : -sn[k]);
    if constexpr ((c > 0) == (s > 0)) {
      // c (re - im, re + im) with s = c
      return {c * (x.re - x.im), c * (x.re + x.im)};
    } else {
      // s = -c:  (re c + im c, im c - re c)
      return {c * (x.re + x.im), c * (x.im - x.re)};
    }
  } else {
    constexpr T c = (T)cs[k];
    constexpr T s = (T)(SIGN > 0 ? sn[k] : -sn[k]);
    return {x.re * c - x.im * s, x.re * s + x.im * c};
  }
}

// In-register DFT of size R (1, 2, 4, 8 or 16), natural order in and out:
// y_q = sum_m x_m exp(SIGN 2 pi i m q / R).  Radix-2 recursion, fully unrolled.
template <typename T, int R, int SIGN>
struct Dft {
  static RS_HD void run(cpx<T>* x) {
    cpx<T> e[R / 2], o[R / 2];
    static_for<R / 2>([&](auto i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    });
    Dft<T, R / 2, SIGN>::run(e);
    Dft<T, R / 2, SIGN>::run(o);
    static_for<R / 2>([&](auto q) {
      constexpr int Q = decltype(q)::value;
      cpx<T> t = mul_root<T, Q, R, SIGN>(o[Q]);
      x[Q] = cadd(e[Q], t);
      x[Q + R / 2] = csub(e[Q], t);
    });
  }
};
template <typename T, int SIGN>
struct Dft<T, 1, SIGN> {
  static RS_HD void run(cpx<T>*) {}
};

// ---------------------------------------------------------------------------
// Shape of an FFT of length L with P points per thread (runtime forms; the
// templates below call them with constants so that they fold).
// ---------------------------------------------------------------------------
RS_HD int fft_points(int L, int P) { return P < L ? P : L; }
RS_HD int fft_tpf(int L, int P) { return L / fft_points(L, P); }
RS_HD int fft_nstages(int L, int P) {
  const int lp = ilog2(fft_points(L, P));
  const int ll = ilog2(L);
  return lp == 0 ? 0 : (ll + lp - 1) / lp;
}
RS_HD int fft_radix(int L, int P, int t) {
  const int PP = fft_points(L, P), NS = fft_nstages(L, P);
  return t < NS - 1 ? PP : (L >> ((NS - 1) * ilog2(PP)));
}
RS_HD int fft_blocklen(int L, int P, int t) { return L >> (t * ilog2(fft_points(L, P))); }
RS_HD int fft_stride(int L, int P, int t) { return fft_blocklen(L, P, t) / fft_radix(L, P, t); }

// Position (index into the length-L sequence) of register e of thread tau at stage t.
RS_HD int fft_pos(int L, int P, int t, int tau, int e) {
  const int R = fft_radix(L, P, t);
  const int u = e / R, m = e % R;
  const int beta = tau + u * fft_tpf(L, P);
  const int s = fft_stride(L, P, t);
  return (beta / s) * fft_blocklen(L, P, t) + (beta % s) + m * s;
}

// Frequency held at position p after the complete DIF sweep.
RS_HD int fft_freq(int L, int P, int p) {
  const int NS = fft_nstages(L, P);
  int f = 0, mult = 1;
  for (int t = 0; t < NS; ++t) {
    const int r = fft_radix(L, P, t);
    const int s = fft_stride(L, P, t);
    const int q = (p / s) % r;
    f += q * mult;
    mult *= r;
  }
  return f;
}

// Lower-half slot numbering of the last-stage registers: register e of thread
// tau with digit m < R/2 (i.e. frequency < L/2) owns slot beta*(R/2)+m.
RS_HD bool fft_lower_half(int L, int P, int e) {
  const int NS = fft_nstages(L, P);
  const int R = fft_radix(L, P, NS - 1);
  return (e % R) < R / 2;
}
RS_HD int fft_slot(int L, int P, int tau, int e) {
  const int NS = fft_nstages(L, P);
  const int R = fft_radix(L, P, NS - 1);
  const int u = e / R, m = e % R;
  const int beta = tau + u * fft_tpf(L, P);
  return beta * (R / 2) + m;
}
// Position of slot c (inverse of fft_slot for lower-half registers).
RS_HD int fft_slot_pos(int L, int P, int c) {
  const int NS = fft_nstages(L, P);
  const int R = fft_radix(L, P, NS - 1);
  const int h = R / 2;
  return (c / h) * R + (c % h);
}

// Slot holding frequency L - freq(p), for a position p of the upper half of
// the spectrum (freq(p) >= L/2); -1 where that frequency is L/2.  Inverts the
// digit reversal of fft_freq and then fft_slot_pos.
RS_HD int fft_mirror_slot(int L, int P, int p) {
  const int g = L - fft_freq(L, P, p);
  if (g >= L / 2) return -1;
  const int NS = fft_nstages(L, P);
  int q = 0, mult = 1;
  for (int t = 0; t < NS; ++t) {
    const int r = fft_radix(L, P, t);
    q += ((g / mult) % r) * fft_stride(L, P, t);
    mult *= r;
  }
  const int R = fft_radix(L, P, NS - 1);
  return (q / R) * (R / 2) + q % R;
}

// x[q] *= w^q for q = 1..R-1, with w^q built from the one loaded root w by
// squarings and products (at most five roundings deep for R = 16) instead of
// R-1 table loads: fewer live registers and one memory latency per butterfly.
template <typename T, int R>
RS_HD void apply_twiddles(cpx<T>* x, cpx<T> w1) {
  if constexpr (R >= 2) x[1] = cmul(x[1], w1);
  if constexpr (R >= 4) {
    const cpx<T> w2 = cmul(w1, w1);
    const cpx<T> w3 = cmul(w2, w1);
    x[2] = cmul(x[2], w2);
    x[3] = cmul(x[3], w3);
    if constexpr (R >= 8) {
      const cpx<T> w4 = cmul(w2, w2);
      x[4] = cmul(x[4], w4);
      x[5] = cmul(x[5], cmul(w4, w1));
      x[6] = cmul(x[6], cmul(w4, w2));
      x[7] = cmul(x[7], cmul(w4, w3));
      if constexpr (R >= 16) {
        const cpx<T> w8 = cmul(w4, w4);
        x[8] = cmul(x[8], w8);
        x[9] = cmul(x[9], cmul(w8, w1));
        x[10] = cmul(x[10], cmul(w8, w2));
        x[11] = cmul(x[11], cmul(w8, w3));
        const cpx<T> w12 = cmul(w8, w4);
        x[12] = cmul(x[12], w12);
        x[13] = cmul(x[13], cmul(w12, w1));
        x[14] = cmul(x[14], cmul(w12, w2));
        x[15] = cmul(x[15], cmul(w12, w3));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Per-thread stage kernels.  `tw` is the table exp(-2 pi i j / L), j < L.
// ---------------------------------------------------------------------------
template <int L, int P>
struct Fft {
  static constexpr int PP = (P < L) ? P : L;
  static constexpr int TPF = L / PP;
  static constexpr int LOGL = ilog2(L);
  static constexpr int LOGP = ilog2(PP);
  static constexpr int NS = (LOGL + LOGP - 1) / LOGP;
  static_assert((1 << LOGL) == L, "L must be a power of two");
  static_assert(L >= 2, "L >= 2");

  static constexpr int radix(int t) { return t < NS - 1 ? PP : (L >> ((NS - 1) * LOGP)); }
  static constexpr int blocklen(int t) { return L >> (t * LOGP); }
  static constexpr int stride(int t) { return blocklen(t) / radix(t); }

  static constexpr RS_HD int pos(int t, int tau, int e) {
    const int R = radix(t);
    const int u = e / R, m = e % R;
    const int beta = tau + u * TPF;
    const int s = stride(t);
    return (beta / s) * blocklen(t) + (beta % s) + m * s;
  }

  // Twiddle root of stage t for thread tau: stages before the last have radix
  // PP, one butterfly per thread and one root (exp(-2 pi i k / L_t) forward;
  // the inverse indexes the mirrored entry instead of conjugating, which keeps
  // the compiler from holding the forward roots in registers until the
  // inverse sweep).  The sweeps load every root up front, so the loads'
  // latency overlaps the first stage instead of following each exchange.
  template <typename T, int t>
  static RS_HD cpx<T> dif_root(int tau, const cpx<T>* __restrict__ tw) {
    static_assert(t < NS - 1, "the last stage has no twiddles");
    constexpr int twsh = LOGL - ilog2(blocklen(t));
    return tw[(tau % stride(t)) << twsh];
  }
  template <typename T, int t>
  static RS_HD cpx<T> dit_root(int tau, const cpx<T>* __restrict__ tw) {
    static_assert(t < NS - 1, "the last stage has no twiddles");
    constexpr int twsh = LOGL - ilog2(blocklen(t));
    return tw[(L - ((tau % stride(t)) << twsh)) & (L - 1)];
  }

  // Stage t with its root w (ignored for the last stage).
  template <typename T, int t>
  static RS_HD void dif_stage_w(cpx<T>* reg, cpx<T> w) {
    constexpr int R = radix(t);
    static_for<PP / R>([&](auto uu) {
      constexpr int u = decltype(uu)::value;
      Dft<T, R, -1>::run(reg + u * R);
      if constexpr (t < NS - 1) apply_twiddles<T, R>(reg + u * R, w);
    });
  }
  template <typename T, int t>
  static RS_HD void dit_stage_w(cpx<T>* reg, cpx<T> w) {
    constexpr int R = radix(t);
    static_for<PP / R>([&](auto uu) {
      constexpr int u = decltype(uu)::value;
      if constexpr (t < NS - 1) apply_twiddles<T, R>(reg + u * R, w);
      Dft<T, R, +1>::run(reg + u * R);
    });
  }

  template <typename T, int t>
  static RS_HD void dif_stage(cpx<T>* reg, int tau, const cpx<T>* __restrict__ tw) {
    if constexpr (t < NS - 1) dif_stage_w<T, t>(reg, dif_root<T, t>(tau, tw));
    else dif_stage_w<T, t>(reg, cpx<T>{(T)1, (T)0});
  }
  template <typename T, int t>
  static RS_HD void dit_stage(cpx<T>* reg, int tau, const cpx<T>* __restrict__ tw) {
    if constexpr (t < NS - 1) dit_stage_w<T, t>(reg, dit_root<T, t>(tau, tw));
    else dit_stage_w<T, t>(reg, cpx<T>{(T)1, (T)0});
  }
};

}  // namespace rsfde
