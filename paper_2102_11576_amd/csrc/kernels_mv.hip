// Matrix-vector product with M = I - A + D (Section 2 of the paper: A is the
// Kronecker sum I (x) A_x + A_y (x) I of symmetric Toeplitz matrices, D the
// penalty diagonal dt/eta outside the domain), in two HBM passes:
//   row pass:    t = (1 + dpen*phi) z - kx * (Ahat_x applied along x)
//   column pass: w = t - ky * (Ahat_y applied along y)
// A third dimension adds one more column pass (z lines are the columns of the
// [n3][n1*n2] view) and runs the y pass once per z slice (grid dimension y).
// Each Toeplitz product is a circular convolution of length L >= 2n-1 with the
// real, even symbol of the circulant embedding [t_0..t_{n-1}, 0.., t_{n-1}..t_1]
// (O(N log N) per product, the fast matrix-vector product the paper relies on).
// Two real rows (or columns) are packed into one complex FFT: the symbol is
// real, so real and imaginary parts never mix.  On two-dimensional plans the
// intermediate t is kept in the strip-tiled layout (tile_index), which the
// column pass reads in whole strips.
#include "fft_common.hpp"

namespace rsfde {

template <int L>
struct MvCfg {
  using F = Fft<L, fft_pts(L)>;
  // Register e of the first (and, inverse, last) stage sits at a position at or
  // above L/2 >= n for every thread: zero on input, unused on output.
  static constexpr bool upper(int e) {
    for (int tau = 0; tau < F::TPF; ++tau)
      if (F::pos(0, tau, e) < L / 2) return false;
    return true;
  }
  static constexpr int TPF = F::TPF;
  static constexpr int BR = (256 / TPF) > 0 ? (256 / TPF) : 1;             // FFTs per row block
  // column pairs per column block: two at L = 1024 and 2048 (two-dimensional
  // grids of 511 or 1023 columns: more, smaller blocks spread them over more
  // CUs; the 3-D plans' many-column views keep the larger blocks), 512 / TPF
  // otherwise
  static constexpr int BC = (L >= 1024 && L <= 2048)
                                ? 2
                                : ((512 / TPF) > 16 ? 16 : ((512 / TPF) > 0 ? (512 / TPF) : 1));
  static constexpr int THR_R = BR * TPF;
  static constexpr int THR_C = BC * TPF;
};

// --------------------------------------------------------------------------
// Row pass.  Block = BR FFTs, FFT b handles rows 2*pair and 2*pair+1.
// TO: out in the strip-tiled layout.
// --------------------------------------------------------------------------
template <int L, bool TO>
__global__ __launch_bounds__(MvCfg<L>::THR_R) __attribute__((amdgpu_waves_per_eu(4))) void k_mv_rows(
    const double* __restrict__ z, const uint8_t* __restrict__ mask, double* __restrict__ out,
    const double* __restrict__ sym, const cpx<double>* __restrict__ tw, int n1, int n2,
    double coef, double dpen, int mode, const double* __restrict__ sub, double theta,
    const Members mb, const double* __restrict__ mk) {
  using C = MvCfg<L>;
  using F = typename C::F;
  __shared__ double lds[C::BR * lds_len(L)];
  {  // member of a batched launch (grid dimension z)
    const size_t mo = mb.off(blockIdx.z);
    z += mo;
    out += mo;
    if (sub) sub += mo;
    if (mk) coef = -mk[mo];
  }
  const int tid = threadIdx.x;
  const int b = tid / F::TPF, tau = tid % F::TPF;
  const int pair = blockIdx.x * C::BR + b;
  const int ra = 2 * pair, rb = 2 * pair + 1;
  const bool va = ra < n2, vb = rb < n2;
  const size_t ia0 = (size_t)(va ? ra : 0) * n1, ib0 = (size_t)(vb ? rb : 0) * n1;
  cpx<double> reg[F::PP];
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    if constexpr (C::upper(e)) {
      reg[e] = {0.0, 0.0};
    } else {
      const int p = F::pos(0, tau, e);
      const bool in = p < n1;
      reg[e].re = (va && in) ? z[ia0 + p] : 0.0;
      reg[e].im = (vb && in) ? z[ib0 + p] : 0.0;
    }
  });
  double* my = lds + b * lds_len(L);
  fft_forward<double, F>(reg, tau, tw, my);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const double s = sym[F::pos(F::NS - 1, tau, e)] * coef;
    reg[e].re *= s;
    reg[e].im *= s;
  });
  fft_inverse<double, F>(reg, tau, tw, my);
  const int hp = (n2 + 1) >> 1;
  // epilogue in groups of G registers: the group's loads (clamped addresses)
  // all in flight at once, then its stores
  constexpr int G = F::PP >= 2 ? 2 : F::PP;
  static_for<F::PP / G>([&](auto gg) {
    constexpr int g0 = decltype(gg)::value * G;
    if constexpr (!C::upper(g0) || !C::upper(g0 + G - 1)) {
      double za[G], zb[G], sa[G], sb[G];
      uint8_t ma[G], mb2[G];
      static_for<G>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        const int p = F::pos(0, tau, g0 + k);
        const int pp = p < n1 ? p : 0;
        za[k] = zb[k] = sa[k] = sb[k] = 0.0;
        ma[k] = mb2[k] = 1;
        if (mode == 0) {
          ma[k] = mask[ia0 + pp];
          mb2[k] = mask[ib0 + pp];
          za[k] = z[ia0 + pp];
          zb[k] = z[ib0 + pp];
        }
        if (sub) {
          sa[k] = sub[ia0 + pp];
          sb[k] = sub[ib0 + pp];
        }
      });
      static_for<G>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        const int p = F::pos(0, tau, g0 + k);
        if (p < n1) {
          if (va) {
            double v = reg[g0 + k].re;
            if (mode == 0) v += (1.0 + dpen * (double)(1 - ma[k])) * za[k];
            if (sub) v -= theta * sa[k];
            out[TO ? tile_index(ra, p, hp) : (size_t)ra * n1 + p] = v;
          }
          if (vb) {
            double v = reg[g0 + k].im;
            if (mode == 0) v += (1.0 + dpen * (double)(1 - mb2[k])) * zb[k];
            if (sub) v -= theta * sb[k];
            out[TO ? tile_index(rb, p, hp) : (size_t)rb * n1 + p] = v;
          }
        }
      });
    }
  });
}

// --------------------------------------------------------------------------
// Column pass.  Block = BC FFTs over 2*BC adjacent columns; thread layout is
// (tau, b) with b fastest so that a wavefront reads 2*BC contiguous doubles of
// several rows at once.  blockIdx.y selects a [n2][n1] slice at offset
// blockIdx.y * bstride (one slice in two dimensions).  MODE is the mode of
// the launcher (0: add t, read in the strip-tiled layout when TT); a
// compile-time mode keeps the epilogue's loads free of per-element branches,
// which measured 10 % faster at n = 2047.
// --------------------------------------------------------------------------
template <int L, int MODE, bool TT, typename ZT = double>
__global__ __launch_bounds__(MvCfg<L>::THR_C) __attribute__((amdgpu_waves_per_eu(4))) void k_mv_cols(
    const ZT* __restrict__ z, const double* __restrict__ t, double* __restrict__ out,
    const double* __restrict__ sym, const cpx<double>* __restrict__ tw, int n1, int n2,
    double coef, size_t bstride, const Members mb, const double* __restrict__ mk) {
  using C = MvCfg<L>;
  using F = typename C::F;
  __shared__ double lds[C::BC * lds_len(L)];
  {  // slice (grid dimension y) and member of a batched launch (dimension z)
    const size_t mo = mb.off(blockIdx.z);
    if (mk) coef = -mk[mo];
    const size_t off = (size_t)blockIdx.y * bstride + mo;
    z += off;
    out += off;
    if constexpr (MODE == 0) t += off;
  }
  const int tid = threadIdx.x;
  const int b = tid % C::BC, tau = tid / C::BC;
  const int strip = xcd_remap(blockIdx.x, gridDim.x);
  const int cp = strip * C::BC + b;
  const int ca = 2 * cp, cb = 2 * cp + 1;
  const bool va = ca < n1, vb = cb < n1;
  cpx<double> reg[F::PP];
  {  // loads from clamped addresses, all in flight at once
    const int cca = va ? ca : 0, ccb = vb ? cb : 0;
    static_for<F::PP>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      if constexpr (C::upper(e)) {
        reg[e] = {0.0, 0.0};
      } else {
        const int p = F::pos(0, tau, e);
        const bool in = p < n2;
        const size_t rp = (size_t)(in ? p : 0) * n1;
        const double a = (double)z[rp + cca], bb = (double)z[rp + ccb];
        reg[e].re = (va && in) ? a : 0.0;
        reg[e].im = (vb && in) ? bb : 0.0;
      }
    });
  }
  double* my = lds + b;  // regions interleaved (stride BC)
  fft_forward<double, F, true, C::BC>(reg, tau, tw, my);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const double s = sym[F::pos(F::NS - 1, tau, e)] * coef;
    reg[e].re *= s;
    reg[e].im *= s;
  });
  fft_inverse<double, F, true, C::BC>(reg, tau, tw, my);
  const int hp = (n2 + 1) >> 1;
  const int cca = va ? ca : 0;
  if constexpr (MODE == 0 && TT) {
    // epilogue in groups of 4 registers: the group's loads of t (clamped
    // addresses) all in flight at once, then its stores
    constexpr int G = F::PP >= 4 ? 4 : F::PP;
    static_for<F::PP / G>([&](auto gg) {
      constexpr int g0 = decltype(gg)::value * G;
      if constexpr (!C::upper(g0) || !C::upper(g0 + G - 1)) {
        double2 q[G];
        static_for<G>([&](auto kk) {
          constexpr int k = decltype(kk)::value;
          const int p = F::pos(0, tau, g0 + k);
          // ca is even: (ca, cb) are adjacent in one tile row (cb = n1 is the
          // strip's padding column, read but not used)
          q[k] = *(const double2*)(t + tile_index(p < n2 ? p : 0, cca, hp));
        });
        static_for<G>([&](auto kk) {
          constexpr int k = decltype(kk)::value;
          const int p = F::pos(0, tau, g0 + k);
          if (p < n2) {
            const size_t i = (size_t)p * n1 + ca;
            if (va) out[i] = reg[g0 + k].re + q[k].x;
            if (vb) out[i + 1] = reg[g0 + k].im + q[k].y;
          }
        });
      }
    });
  } else {
    static_for<F::PP>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      const int p = F::pos(0, tau, e);
      if (p < n2) {
        const size_t i = (size_t)p * n1 + ca;
        double ta = 0.0, tb = 0.0;
        if constexpr (MODE == 0) {
          ta = va ? t[i] : 0.0;
          tb = vb ? t[i + 1] : 0.0;
        }
        if (va) out[i] = reg[e].re + ta;
        if (vb) out[i + 1] = reg[e].im + tb;
      }
    });
  }
}

template <int L>
static hipError_t mv_rows_impl(const double* z, const uint8_t* mask, double* out, const double* sym,
                               const void* tw, int n1, int n2, double coef, double dpen, int mode,
                               hipStream_t s, const double* sub, double theta, bool tiled,
                               const Members& mb, const double* mk) {
  using C = MvCfg<L>;
  const int pairs = (n2 + 1) / 2;
  const int blocks = (pairs + C::BR - 1) / C::BR;
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  const dim3 grid(blocks, 1, mb.n);
  if (tiled)
    hipLaunchKernelGGL((k_mv_rows<L, true>), grid, dim3(C::THR_R), 0, s, z, mask, out, sym,
                       (const cpx<double>*)tw, n1, n2, coef, dpen, mode, sub, theta, mb, mk);
  else
    hipLaunchKernelGGL((k_mv_rows<L, false>), grid, dim3(C::THR_R), 0, s, z, mask, out,
                       sym, (const cpx<double>*)tw, n1, n2, coef, dpen, mode, sub, theta, mb, mk);
  return hipGetLastError();
}

template <int L>
static hipError_t mv_cols_impl(const void* zv, const double* t, double* out, const double* sym,
                               const void* tw, int n1, int n2, double coef, int mode, hipStream_t s,
                               int batch, size_t bstride, bool tiled, const Members& mb,
                               const double* mk, bool z32) {
  const double* z = (const double*)zv;
  using C = MvCfg<L>;
  const int pairs = (n1 + 1) / 2;
  const int blocks = (pairs + C::BC - 1) / C::BC;
  if (batch < 1 || batch > 65535) return hipErrorInvalidValue;
  if (tiled && (mode != 0 || batch != 1)) return hipErrorInvalidValue;
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  const dim3 grid(blocks, batch, mb.n), thr(C::THR_C);
  const cpx<double>* twc = (const cpx<double>*)tw;
  if (z32) {
    if (mode != 0 || !tiled) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_mv_cols<L, 0, true, float>), grid, thr, 0, s, (const float*)zv, t, out,
                       sym, twc, n1, n2, coef, bstride, mb, mk);
    return hipGetLastError();
  }
  if (mode != 0)
    hipLaunchKernelGGL((k_mv_cols<L, 1, false>), grid, thr, 0, s, z, t, out, sym, twc, n1, n2,
                       coef, bstride, mb, mk);
  else if (tiled)
    hipLaunchKernelGGL((k_mv_cols<L, 0, true>), grid, thr, 0, s, z, t, out, sym, twc, n1, n2, coef,
                       bstride, mb, mk);
  else
    hipLaunchKernelGGL((k_mv_cols<L, 0, false>), grid, thr, 0, s, z, t, out, sym, twc, n1, n2,
                       coef, bstride, mb, mk);
  return hipGetLastError();
}

#define RSFDE_L_CASES(X) \
  X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192)

hipError_t launch_mv_rows(int L, const double* z, const uint8_t* mask, double* out,
                          const double* sym, const void* tw, int n1, int n2, double coef,
                          double dpen, int mode, hipStream_t s, const double* sub, double theta,
                          bool tiled, const Members& mb, const double* mk) {
  switch (L) {
#define X(LL)                                                                                    \
  case LL:                                                                                       \
    return mv_rows_impl<LL>(z, mask, out, sym, tw, n1, n2, coef, dpen, mode, s, sub, theta, tiled, \
                            mb, mk);
    RSFDE_L_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_mv_cols(int L, const void* z, const double* t, double* out,
                          const double* sym, const void* tw, int n1, int n2, double coef,
                          int mode, hipStream_t s, int batch, size_t bstride, bool tiled,
                          const Members& mb, const double* mk, bool z32) {
  switch (L) {
#define X(LL)                                                                                   \
  case LL:                                                                                      \
    return mv_cols_impl<LL>(z, t, out, sym, tw, n1, n2, coef, mode, s, batch, bstride, tiled, mb, \
                            mk, z32);
    RSFDE_L_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace rsfde
