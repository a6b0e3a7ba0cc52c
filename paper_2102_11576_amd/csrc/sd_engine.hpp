// Symmetric form of the length-n DST-I (n + 1 = L/2 a power of two) for the
// preconditioner passes (Section 4.1: the tau matrices are diagonalised by the
// sine transform, which the paper applies with FFTs).
//
// The plain route is one complex FFT of length L over the odd extension z of
// the data (z_j = x_j, z_{L-j} = -x_j, z_0 = z_{L/2} = 0); its spectrum Z is
// odd as well (Z_{L-k} = -Z_k) and -2i times the sine sums.  Half of that FFT's
// inputs and half of its outputs are therefore redundant.  Split the transform
// as one radix-16 decimation-in-frequency stage over the groups
// p = 0..LS-1 (LS = L/16; group p holds z_{p + LS m}, m = 0..15) followed by 16
// sub-FFTs of length LS (block r holds frequencies r + 16 k).  Two symmetries
// follow from the oddness of z:
//   * group LS-p is the reversed, negated group p, so its stage outputs are
//     those of group p at index -r times -W_L^{-pr} ... : only the groups
//     p = 0..LS/2 are computed, each also supplying the inputs of the block
//     positions LS-p;
//   * block 16-r holds the reversed, negated spectrum of block r, so only the
//     blocks r = 0..8 are transformed.
// This takes 9/16 of the sub-FFT work and about half of the first stage.  The
// inverse is the exact mirror (decimation in time: block sub-FFTs first, then
// the group stage over q = 0..LS/2, whose outputs also fill positions LS-q).
//
// Spectral layout ("slots"): the n + 1 = L/2 values a pass keeps per line are
// all LS positions of blocks 1..7 and the lower halves (sub-frequency < LS/2)
// of blocks 0 and 8; a slot holds the odd spectrum at its own frequency, which
// lies above L/2 for the upper halves of blocks 1..7 (Z there is minus the
// value at L - f).  The upper halves of blocks 0 and 8 are rebuilt by odd
// symmetry from their mirror slots.  Slot numbering makes consecutive threads
// of a sub-FFT own consecutive slots for every register, so slot loads and
// stores are contiguous across a wavefront.
#pragma once

#include "fft_engine.hpp"

namespace rsfde {

// Smallest L handled by the symmetric form (sub-FFTs of at least 32 points).
constexpr int kSdMinL = 512;

template <int L>
struct Sd {
  static constexpr int LS = L / 16;  // block (sub-FFT) length
  static_assert(LS >= 32 && (LS & (LS - 1)) == 0, "symmetric DST needs L >= 512, a power of two");
  using Fs = Fft<LS, 16>;                    // sub-FFT engine, 16 points per thread
  static constexpr int TS = Fs::TPF;         // threads of one sub-FFT
  static constexpr int TPD = 9 * TS;         // block-stage threads of one transform
  static constexpr int NG = LS / 2 + 1;      // group-stage threads of one transform
  static constexpr int NPOS = 9 * LS;        // positions of the kept blocks
  static constexpr int LEN = NPOS + NPOS / 16 + 1;  // LDS scalars of one region (padded)
  static constexpr int RL = Fs::radix(Fs::NS - 1);  // radix of the sub-FFT's last stage
  static_assert(NG <= TPD, "group stage must fit the block-stage threads");

  // Natural index of register m of group p in the odd extension, as an index
  // into x (1..n valid); neg: the value enters negated (m >= 8 mirrors the
  // position L - (p + LS m) = (LS - p) + LS (15 - m)).
  static RS_HD int nat(int p, int m, bool& neg) {
    if (m < 8) {
      neg = false;
      return p + LS * m;
    }
    neg = true;
    return (LS - p) + LS * (15 - m);
  }
  // Rank of register e among the lower-half registers of the sub-FFT's last
  // stage (-1 for the upper half): sub-frequency < LS/2 iff the last digit is.
  static constexpr RS_HD int lower_rank(int e) {
    const int m = e % RL;
    return m < RL / 2 ? (e / RL) * (RL / 2) + m : -1;
  }
  // Slot of register e of thread tau of block r after the forward sweep, or -1
  // (upper half of blocks 0 and 8).
  static constexpr RS_HD int slot(int r, int tau, int e) {
    if (r >= 1 && r <= 7) return r * LS + e * TS + tau;
    const int lr = lower_rank(e);
    if (lr < 0) return -1;
    return (r == 8 ? LS / 2 : 0) + lr * TS + tau;
  }
  // Frequency (0..L-1) held at block position P = r * LS + q after the forward sweep.
  static RS_HD int freq(int P) { return P / LS + 16 * fft_freq(LS, 16, P % LS); }
  // DST index (0..L/2) of a frequency of the odd spectrum.
  static constexpr RS_HD int fold(int f) { return f <= L / 2 ? f : L - f; }
};

// Forward group stage of group p: in a[m] = z_{p + LS m}; out a[r] for r = 0..8
// is the input of block r at position p, a[16 - r] (r = 1..7) that of block r
// at position LS - p, and m8 that of block 8 at position LS - p (block 0 takes
// -a[0] there).  The roots W_L^{p r} come from w1 = W_L^p (the caller loads it
// early, with its data) by products, each applied as soon as it is formed.
template <typename T, int L>
RS_HD void sd_group_fwd(cpx<T>* a, cpx<T> w1, cpx<T>& m8) {
  Dft<T, 16, -1>::run(a);
  auto apply = [&](int r, const cpx<T>& w) {
    const cpx<T> u = cmulc(a[16 - r], w);
    a[16 - r] = {-u.re, -u.im};
    a[r] = cmul(a[r], w);
  };
  apply(1, w1);
  const cpx<T> w2 = cmul(w1, w1);
  apply(2, w2);
  const cpx<T> w3 = cmul(w2, w1);
  apply(3, w3);
  const cpx<T> w4 = cmul(w2, w2);
  apply(4, w4);
  apply(5, cmul(w4, w1));
  apply(6, cmul(w4, w2));
  apply(7, cmul(w4, w3));
  const cpx<T> w8 = cmul(w4, w4);
  const cpx<T> m = cmulc(a[8], w8);
  m8 = {-m.re, -m.im};
  a[8] = cmul(a[8], w8);
}

// Inverse group stage of group q: in c[r] = T_r[q] (r = 0..8) and
// c[16 - r] = T_r[LS - q] (r = 1..7), T_r the inverse sub-FFT of block r; out
// c[m] = L x (odd extension) at position q + LS m.  w1 = W_L^q.
template <typename T, int L>
RS_HD void sd_group_inv(cpx<T>* c, cpx<T> w1) {
  auto apply = [&](int r, const cpx<T>& w) {
    const cpx<T> u = cmul(c[16 - r], w);
    c[16 - r] = {-u.re, -u.im};
    c[r] = cmulc(c[r], w);
  };
  apply(1, w1);
  const cpx<T> w2 = cmul(w1, w1);
  apply(2, w2);
  const cpx<T> w3 = cmul(w2, w1);
  apply(3, w3);
  const cpx<T> w4 = cmul(w2, w2);
  apply(4, w4);
  apply(5, cmul(w4, w1));
  apply(6, cmul(w4, w2));
  apply(7, cmul(w4, w3));
  c[8] = cmulc(c[8], cmul(w4, w4));
  Dft<T, 16, +1>::run(c);
}

}  // namespace rsfde
