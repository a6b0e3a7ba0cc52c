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
  worst = std::fmax(worst, run_case<128, 4, double>(13));
  worst = std::fmax(worst, run_case<256, 8, float>(14));
  worst = std::fmax(worst, run_case<4096, 16, float>(15));
  if (worst >= 1e9) { printf("FAIL\n"); return 1; }
  printf("OK\n");
  return 0;
}
