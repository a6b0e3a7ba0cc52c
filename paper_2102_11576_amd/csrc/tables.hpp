// Host-side tables shared by the plan set-up and the allocation-free matrix-
// vector product: Grunwald-Letnikov first columns (Section 2, (g_form), (G)),
// circulant-embedding symbols of the Toeplitz factors and FFT twiddles.  All
// in FP64 with exact integer argument reduction of the angles.
#pragma once

#include <cmath>
#include <vector>

#include "fft_engine.hpp"

namespace rsfde {
namespace tables {

constexpr double kPi = 3.14159265358979323846264338327950288;

inline bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }
inline int next_pow2(long v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// cos(2 pi k / L) for k < L, with exact integer argument reduction by the caller.
inline std::vector<double> cos_table(int L) {
  std::vector<double> c(L);
  for (int k = 0; k < L; ++k) {
    // reduce to the first octant-free form: angle = 2 pi k / L in [0, 2 pi)
    c[k] = std::cos(2.0 * kPi * (double)k / (double)L);
  }
  // make the symmetric values exactly symmetric
  for (int k = 1; k < L; ++k) c[L - k] = c[k] = (k <= L - k) ? c[k] : c[L - k];
  return c;
}

// First column of the unit-coefficient Toeplitz matrix c * G_n^(alpha) (G).
inline std::vector<double> toeplitz_col(double alpha, int n, double c) {
  std::vector<double> g(n + 2);
  g[0] = 1.0;
  for (int l = 1; l < n + 2; ++l) g[l] = (1.0 - (alpha + 1.0) / l) * g[l - 1];
  std::vector<double> t(n);
  t[0] = 2.0 * g[1];
  if (n > 1) t[1] = g[0] + g[2];
  for (int k = 2; k < n; ++k) t[k] = g[k + 1];
  for (auto& v : t) v *= c;
  return t;
}

// Symbol of the circulant embedding of length L (L >= 2n - 1) of the symmetric
// Toeplitz matrix with first column t, divided by L, in the register-position
// order of the FFT of length L with fft_pts(L) points per thread.
inline std::vector<double> conv_symbol_pos(const std::vector<double>& t, int L) {
  const int n = (int)t.size();
  std::vector<double> ct = cos_table(L), chat(L);
  for (int f = 0; f < L; ++f) {
    double s = t[0];
    for (int j = 1; j < n; ++j) s += 2.0 * t[j] * ct[(int)(((long long)j * f) % L)];
    chat[f] = s;
  }
  const int P = fft_pts(L);
  std::vector<double> out(L);
  for (int p = 0; p < L; ++p) out[p] = chat[fft_freq(L, P, p)] / (double)L;
  return out;
}

template <typename T>
std::vector<T> twiddles(int L) {
  std::vector<T> tw(2 * (size_t)L);
  for (int j = 0; j < L; ++j) {
    // exp(-2 pi i j / L) with exact symmetry in j
    const int jj = j <= L / 2 ? j : L - j;
    const double a = 2.0 * kPi * (double)jj / (double)L;
    double c = std::cos(a), s = std::sin(a);
    if (4 * jj == L) c = 0.0;
    if (2 * jj == L) s = 0.0;
    tw[2 * (size_t)j] = (T)c;
    tw[2 * (size_t)j + 1] = (T)(j <= L / 2 ? -s : s);
  }
  return tw;
}

}  // namespace tables
}  // namespace rsfde
