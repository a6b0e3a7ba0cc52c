// CPU self-test of the FFT engine's index arithmetic and butterflies.
// Every "thread" of one FFT is simulated in turn; the LDS exchange between
// stages is a plain array.  Checks the forward sweep against the DFT
// definition (summed in long double) and that the inverse sweep returns L x.
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "fft_engine.hpp"
#include "sd_engine.hpp"

using namespace rsfde;

template <typename T>
static std::vector<cpx<T>> twiddles(int L) {
  std::vector<cpx<T>> tw(L);
  for (int j = 0; j < L; ++j) {
    long double a = -2.0L * 3.14159265358979323846264338327950288L * j / L;
    tw[j] = {(T)std::cos(a), (T)std::sin(a)};
  }
  return tw;
}

template <int L, int P, typename T>
static double run_case(unsigned seed) {
  using F = Fft<L, P>;
  std::vector<cpx<T>> tw = twiddles<T>(L);
  std::vector<cpx<T>> x(L);
  srand(seed);
  for (auto& v : x) v = {(T)(rand() / (double)RAND_MAX - 0.5), (T)(rand() / (double)RAND_MAX - 0.5)};
  std::vector<std::array<cpx<T>, F::PP>> regs(F::TPF);
  for (int tau = 0; tau < F::TPF; ++tau)
    for (int e = 0; e < F::PP; ++e) regs[tau][e] = x[F::pos(0, tau, e)];
  std::vector<cpx<T>> buf(L);
  static_for<F::NS>([&](auto tt) {
    constexpr int t = decltype(tt)::value;
    for (int tau = 0; tau < F::TPF; ++tau) F::template dif_stage<T, t>(regs[tau].data(), tau, tw.data());
    if constexpr (t < F::NS - 1) {
      for (int tau = 0; tau < F::TPF; ++tau)
        for (int e = 0; e < F::PP; ++e) buf[F::pos(t, tau, e)] = regs[tau][e];
      for (int tau = 0; tau < F::TPF; ++tau)
        for (int e = 0; e < F::PP; ++e) regs[tau][e] = buf[F::pos(t + 1, tau, e)];
    }
  });
  // compare with the DFT definition
  double err = 0, scale = 0;
  std::vector<int> seen(L, 0);
  for (int tau = 0; tau < F::TPF; ++tau)
    for (int e = 0; e < F::PP; ++e) {
      int p = F::pos(F::NS - 1, tau, e);
      int f = fft_freq(L, P, p);
      seen[f]++;
      long double sr = 0, si = 0;
      for (int j = 0; j < L; ++j) {
        long double a = -2.0L * 3.14159265358979323846264338327950288L * (((long long)j * f) % L) / L;
        sr += x[j].re * std::cos(a) - x[j].im * std::sin(a);
        si += x[j].re * std::sin(a) + x[j].im * std::cos(a);
      }
      err = std::fmax(err, std::fabs((double)(regs[tau][e].re - sr)));
      err = std::fmax(err, std::fabs((double)(regs[tau][e].im - si)));
      scale = std::fmax(scale, std::fabs((double)sr) + std::fabs((double)si));
    }
  for (int f = 0; f < L; ++f)
    if (seen[f] != 1) { printf("freq map not a permutation at L=%d P=%d\n", L, P); return 1e9; }
  // lower-half slots: bijection onto [0, L/2) with frequency < L/2
  std::vector<int> sseen(L / 2, 0);
  for (int tau = 0; tau < F::TPF; ++tau)
    for (int e = 0; e < F::PP; ++e) {
      int p = F::pos(F::NS - 1, tau, e);
      bool lo = fft_lower_half(L, P, e);
      if (lo != (fft_freq(L, P, p) < L / 2)) { printf("lower-half test wrong L=%d\n", L); return 1e9; }
      if (lo) {
        int c = fft_slot(L, P, tau, e);
        if (c < 0 || c >= L / 2 || fft_slot_pos(L, P, c) != p) { printf("slot map wrong L=%d\n", L); return 1e9; }
        sseen[c]++;
      }
    }
  for (int c = 0; c < L / 2; ++c)
    if (L >= 2 && sseen[c] != 1) { printf("slots not a bijection L=%d\n", L); return 1e9; }
  // mirrored slots of the upper half against a search over all slots
  for (int p = 0; p < L; ++p) {
    const int f = fft_freq(L, P, p);
    if (f < L / 2) continue;
    int want = -1;
    for (int c = 0; c < L / 2; ++c)
      if (L - f != L / 2 && fft_freq(L, P, fft_slot_pos(L, P, c)) == L - f) want = c;
    if (fft_mirror_slot(L, P, p) != want) { printf("mirror slot wrong L=%d p=%d\n", L, p); return 1e9; }
  }
  // inverse sweep
  for (int t = F::NS - 1; t >= 0; --t) { (void)t; }
  static_for<F::NS>([&](auto tt) {
    constexpr int t = F::NS - 1 - decltype(tt)::value;
    for (int tau = 0; tau < F::TPF; ++tau) F::template dit_stage<T, t>(regs[tau].data(), tau, tw.data());
    if constexpr (t > 0) {
      for (int tau = 0; tau < F::TPF; ++tau)
        for (int e = 0; e < F::PP; ++e) buf[F::pos(t, tau, e)] = regs[tau][e];
      for (int tau = 0; tau < F::TPF; ++tau)
        for (int e = 0; e < F::PP; ++e) regs[tau][e] = buf[F::pos(t - 1, tau, e)];
    }
  });
  double err2 = 0;
  for (int tau = 0; tau < F::TPF; ++tau)
    for (int e = 0; e < F::PP; ++e) {
      int p = F::pos(0, tau, e);
      err2 = std::fmax(err2, std::fabs((double)(regs[tau][e].re / L - x[p].re)));
      err2 = std::fmax(err2, std::fabs((double)(regs[tau][e].im / L - x[p].im)));
    }
  double rel = err / scale;
  printf("L=%5d P=%2d %s  fwd rel err %.2e  inv err %.2e\n", L, P, sizeof(T) == 8 ? "f64" : "f32", rel, err2);
  double tol = sizeof(T) == 8 ? 1e-14 : 1e-5;
  return (rel > tol || err2 > tol) ? 1e9 : rel;
}

// Symmetric DST-I (sd_engine.hpp): forward against the sine sums, slot and
// mirror maps, and the inverse returning L x.  Every thread of one transform
// is simulated in turn with the LDS exchange as a plain array.
template <int L, typename T>
static double run_sd_case(unsigned seed) {
  using S = Sd<L>;
  using Fs = typename S::Fs;
  constexpr int LS = S::LS, n = L / 2 - 1;
  std::vector<cpx<T>> twL = twiddles<T>(L), twS = twiddles<T>(LS);
  std::vector<cpx<T>> x(n + 1);  // x[1..n]
  srand(seed);
  for (int j = 1; j <= n; ++j) x[j] = {(T)(rand() / (double)RAND_MAX - 0.5), (T)(rand() / (double)RAND_MAX - 0.5)};
  std::vector<cpx<T>> buf(S::NPOS, cpx<T>{(T)1e30, (T)1e30});
  // forward group stage
  for (int p = 0; p < S::NG; ++p) {
    cpx<T> a[16];
    for (int m = 0; m < 16; ++m) {
      bool neg;
      const int j = S::nat(p, m, neg);
      cpx<T> v = (j >= 1 && j <= n) ? x[j] : cpx<T>{(T)0, (T)0};
      a[m] = neg ? cpx<T>{-v.re, -v.im} : v;
    }
    cpx<T> m8;
    sd_group_fwd<T, L>(a, twL[p], m8);
    for (int r = 0; r <= 8; ++r) buf[r * LS + p] = a[r];
    if (p != 0 && p != LS / 2) {
      buf[LS - p] = {-a[0].re, -a[0].im};
      for (int r = 1; r <= 7; ++r) buf[r * LS + LS - p] = a[16 - r];
      buf[8 * LS + LS - p] = m8;
    }
  }
  for (int P = 0; P < S::NPOS; ++P)
    if (buf[P].re == (T)1e30) { printf("sd L=%d: block position %d not written\n", L, P); return 1e9; }
  // block stages: sub-FFT sweeps of blocks 0..8
  std::vector<std::array<cpx<T>, 16>> regs(S::TPD);
  for (int r = 0; r < 9; ++r) {
    for (int tau = 0; tau < S::TS; ++tau)
      for (int e = 0; e < 16; ++e) regs[r * S::TS + tau][e] = buf[r * LS + Fs::pos(0, tau, e)];
    std::vector<cpx<T>> sb(LS);
    static_for<Fs::NS>([&](auto tt) {
      constexpr int t = decltype(tt)::value;
      for (int tau = 0; tau < S::TS; ++tau) Fs::template dif_stage<T, t>(regs[r * S::TS + tau].data(), tau, twS.data());
      if constexpr (t < Fs::NS - 1) {
        for (int tau = 0; tau < S::TS; ++tau)
          for (int e = 0; e < 16; ++e) sb[Fs::pos(t, tau, e)] = regs[r * S::TS + tau][e];
        for (int tau = 0; tau < S::TS; ++tau)
          for (int e = 0; e < 16; ++e) regs[r * S::TS + tau][e] = sb[Fs::pos(t + 1, tau, e)];
      }
    });
  }
  // compare with the odd spectrum Z_f = 2 sigma_b(f) - 2i sigma_a(f) (sigma: sine sums)
  double err = 0, scale = 0;
  std::vector<int> sseen(L / 2, 0);
  std::vector<cpx<T>> slotv(L / 2);
  for (int r = 0; r < 9; ++r)
    for (int tau = 0; tau < S::TS; ++tau)
      for (int e = 0; e < 16; ++e) {
        const int P = r * LS + Fs::pos(Fs::NS - 1, tau, e);
        const int f = S::freq(P), k = S::fold(f);
        const double sg = f <= L / 2 ? 1.0 : -1.0;
        long double sa = 0, sb2 = 0;
        for (int j = 1; j <= n; ++j) {
          const long double sn = std::sin(3.14159265358979323846264338327950288L * (((long long)j * k) % L) / (L / 2));
          sa += x[j].re * sn;
          sb2 += x[j].im * sn;
        }
        const double zr = sg * 2.0 * (double)sb2, zi = -sg * 2.0 * (double)sa;
        const cpx<T> v = regs[r * S::TS + tau][e];
        err = std::fmax(err, std::fabs((double)v.re - zr));
        err = std::fmax(err, std::fabs((double)v.im - zi));
        scale = std::fmax(scale, std::fabs(zr) + std::fabs(zi));
        const int c = S::slot(r, tau, e);
        const bool lower = fft_freq(LS, 16, P % LS) < LS / 2;
        if ((c < 0) != ((r == 0 || r == 8) && !lower)) { printf("sd L=%d: slot set wrong\n", L); return 1e9; }
        if (c >= 0) {
          if (c >= L / 2) { printf("sd L=%d: slot out of range\n", L); return 1e9; }
          sseen[c]++;
          slotv[c] = v;
        }
      }
  for (int c = 0; c < L / 2; ++c)
    if (sseen[c] != 1) { printf("sd L=%d: slots not a bijection\n", L); return 1e9; }
  // inverse: rebuild the spectrum from the slots (mirrors for blocks 0, 8 upper halves)
  std::vector<int> by_freq(L, -1);
  for (int r = 0; r < 9; ++r)
    for (int tau = 0; tau < S::TS; ++tau)
      for (int e = 0; e < 16; ++e) {
        const int c = S::slot(r, tau, e);
        if (c >= 0) by_freq[S::freq(r * LS + Fs::pos(Fs::NS - 1, tau, e))] = c;
      }
  for (int r = 0; r < 9; ++r) {
    for (int tau = 0; tau < S::TS; ++tau)
      for (int e = 0; e < 16; ++e) {
        const int c = S::slot(r, tau, e);
        const int f = S::freq(r * LS + Fs::pos(Fs::NS - 1, tau, e));
        cpx<T> v{(T)0, (T)0};
        if (c >= 0) v = slotv[c];
        else if (f != L / 2 && f != 0) {
          const int mc = by_freq[L - f];
          if (mc < 0) { printf("sd L=%d: mirror of %d missing\n", L, f); return 1e9; }
          v = {-slotv[mc].re, -slotv[mc].im};
        }
        regs[r * S::TS + tau][e] = v;
      }
    std::vector<cpx<T>> sb(LS);
    static_for<Fs::NS>([&](auto tt) {
      constexpr int t = Fs::NS - 1 - decltype(tt)::value;
      for (int tau = 0; tau < S::TS; ++tau) Fs::template dit_stage<T, t>(regs[r * S::TS + tau].data(), tau, twS.data());
      if constexpr (t > 0) {
        for (int tau = 0; tau < S::TS; ++tau)
          for (int e = 0; e < 16; ++e) sb[Fs::pos(t, tau, e)] = regs[r * S::TS + tau][e];
        for (int tau = 0; tau < S::TS; ++tau)
          for (int e = 0; e < 16; ++e) regs[r * S::TS + tau][e] = sb[Fs::pos(t - 1, tau, e)];
      }
    });
    for (int tau = 0; tau < S::TS; ++tau)
      for (int e = 0; e < 16; ++e) buf[r * LS + Fs::pos(0, tau, e)] = regs[r * S::TS + tau][e];
  }
  std::vector<cpx<T>> y(n + 1, cpx<T>{(T)1e30, (T)1e30});
  for (int q = 0; q < S::NG; ++q) {
    cpx<T> c[16];
    for (int r = 0; r <= 8; ++r) c[r] = buf[r * LS + q];
    for (int r = 1; r <= 7; ++r) c[16 - r] = buf[r * LS + ((LS - q) & (LS - 1))];
    sd_group_inv<T, L>(c, twL[q]);
    for (int m = 0; m < 16; ++m) {
      if (m >= 8 && (q == 0 || q == LS / 2)) continue;
      bool neg;
      const int j = S::nat(q, m, neg);
      if (j < 1 || j > n) continue;
      if (y[j].re != (T)1e30) { printf("sd L=%d: output %d written twice\n", L, j); return 1e9; }
      y[j] = neg ? cpx<T>{-c[m].re, -c[m].im} : c[m];
    }
  }
  double err2 = 0;
  for (int j = 1; j <= n; ++j) {
    if (y[j].re == (T)1e30) { printf("sd L=%d: output %d missing\n", L, j); return 1e9; }
    err2 = std::fmax(err2, std::fabs((double)(y[j].re / L - x[j].re)));
    err2 = std::fmax(err2, std::fabs((double)(y[j].im / L - x[j].im)));
  }
  const double rel = err / scale;
  printf("sd L=%5d %s  fwd rel err %.2e  inv err %.2e\n", L, sizeof(T) == 8 ? "f64" : "f32", rel, err2);
  const double tol = sizeof(T) == 8 ? 1e-14 : 1e-5;
  return (rel > tol || err2 > tol) ? 1e9 : rel;
}

int main() {
  double worst = 0;
  worst = std::fmax(worst, run_case<2, 16, double>(1));
  worst = std::fmax(worst, run_case<4, 16, double>(2));
  worst = std::fmax(worst, run_case<8, 16, double>(3));
  worst = std::fmax(worst, run_case<16, 16, double>(4));
  worst = std::fmax(worst, run_case<32, 16, double>(5));
  worst = std::fmax(worst, run_case<64, 16, double>(6));
  worst = std::fmax(worst, run_case<128, 16, double>(7));
  worst = std::fmax(worst, run_case<256, 16, double>(8));
  worst = std::fmax(worst, run_case<512, 8, double>(9));
  worst = std::fmax(worst, run_case<1024, 16, double>(10));
  worst = std::fmax(worst, run_case<2048, 16, double>(11));
  worst = std::fmax(worst, run_case<4096, 16, double>(12));
  worst = std::fmax(worst, run_case<8192, 16, double>(16));
  worst = std::fmax(worst, run_case<1024, 8, double>(17));
  worst = std::fmax(worst, run_case<128, 4, double>(13));
  worst = std::fmax(worst, run_case<256, 8, float>(14));
  worst = std::fmax(worst, run_case<4096, 16, float>(15));
  worst = std::fmax(worst, run_sd_case<512, double>(21));
  worst = std::fmax(worst, run_sd_case<1024, double>(22));
  worst = std::fmax(worst, run_sd_case<2048, double>(23));
  worst = std::fmax(worst, run_sd_case<4096, double>(24));
  worst = std::fmax(worst, run_sd_case<8192, double>(25));
  worst = std::fmax(worst, run_sd_case<4096, float>(26));
  if (worst >= 1e9) { printf("FAIL\n"); return 1; }
  printf("OK\n");
  return 0;
}
