// The sine-transform preconditioner of Section 4.1 of the paper:
//   P_hat^{-1} = (I - Phi)(I - tau_1(A))^{-1} + Phi((1 + dt/eta) I - tau_1(A))^{-1},
// with I - tau_1(A) = (S (x) S)(I - I (x) L_x - L_y (x) I)(S (x) S) (Lemma 4.2),
// applied as three HBM passes over [n2][n1] data:
//   A (rows):    Q  = raw sine sums of each row of sig*v              (x transform)
//   B (columns): P1 = S_y( K*rho / E1 ),  P2 = S_y( K*rho / E2 )        (y transform,
//                rho = raw 2-D sine coefficients, E1 = 1 - kx lx - ky ly, E2 = E1 + dt/eta)
//   C (rows):    z  = mask * (P1 S_x) + (1 - mask) * (P2 S_x)          (x transform + combine)
// with K = 4 / ((n1+1)(n2+1)) the product of the orthonormal DST-I factors.
//
// A length-n DST-I is one length-L = 2(n+1) complex FFT of the odd extension
// (x at positions 1..n, -x mirrored, zeros at 0 and n+1): its spectrum is
// -2i * (raw sine sums).  Two real sequences share one complex FFT (a + i b):
// the spectrum is 2 sigma_b - 2i sigma_a, both parts odd in frequency.  Pass A
// stores only the lower half of the digit-reversed spectrum ("slots", n+1 per
// row: frequencies 0..n, frequency 0 being identically zero); pass B works on
// slot columns; pass C rebuilds the upper half by odd symmetry (fft_mirror_slot)
// and runs the inverse sweep, which yields the DST directly in natural order.
// T = double or float sets the arithmetic of all three passes (the input and
// output vectors are always FP64).
//
// Layout of the intermediates.  Natural (TL = false): Q, P1, P2 are
// [rows][n+1] arrays.  Two-dimensional plans (TL = true): Q is strip-tiled
// (tile_index: [2 rows][4 slots] tiles, strip after strip), and the P1/P2
// pairs are interleaved in one array of row segments (pair_index).  Pass B
// then reads Q in whole strips and writes whole 32-byte sectors, where the
// natural layout gives it 32-byte pieces of rows 8 (n+1) bytes apart; pass A
// writes 64-byte pieces of Q and pass C reads whole 128-byte lines of pairs.
#pragma once
#include "fft_common.hpp"

namespace rsfde {

// Row-segment layout of the interleaved (P1, P2) pairs: segments of
// W = 64 / sizeof(T) slots per row (one 128-byte line of pairs), the
// segments of one W-slot strip stored row after row, strip after strip.
// Within a segment the even slots fill the first half of the line and the odd
// slots the second: pass B finishes the even slot of each column pair in its
// first inverse sweep and the odd one in its second, so the blocks of one
// strip complete a whole 64-byte half-line per sweep (a line written in two
// halves at two times then leaves the L2 as two full halves).  Returns the
// element of P1 (P2 follows it); the array holds 2 W ceil(slots / W) rows values.
template <typename T>
__device__ __forceinline__ size_t pair_index(int r, int c, int rows) {
  constexpr int W = 64 / (int)sizeof(T);
  const int q = c % W;
  const int pos = (q & 1) * (W / 2) + (q >> 1);
  return (((size_t)(c / W) * rows + r) * W + pos) * 2;
}


template <int L>
struct PcCfg {
  using F = Fft<L, fft_pts(L)>;
  static constexpr int TPF = F::TPF;
  static constexpr int BR = (256 / TPF) > 0 ? (256 / TPF) : 1;
  static constexpr int THR_R = BR * TPF;
};
template <int L>
struct PcColCfg {
  using F = Fft<L, pc_cols_pts(L)>;
  static constexpr int TPF = F::TPF;
  static constexpr int BC = (512 / TPF) > 16 ? 16 : ((512 / TPF) > 0 ? (512 / TPF) : 1);
  static constexpr int THR_C = BC * TPF;
};

// --------------------------------------------------------------------------
// Pass A: row pairs (ra, rb) -> Q rows (n1+1 slots each).
// --------------------------------------------------------------------------
template <typename T, int L, bool TL>
__global__ __launch_bounds__(PcCfg<L>::THR_R) void k_pc_rows_fwd(
    const double* __restrict__ v, const double* __restrict__ sig, T* __restrict__ Q,
    const cpx<T>* __restrict__ tw, int n1, int n2, const Members mb) {
  using C = PcCfg<L>;
  using F = typename C::F;
  __shared__ T lds[C::BR * lds_len(L)];
  {  // member of a batched launch (grid dimension z); offsets in doubles
    const size_t mo = mb.off(blockIdx.z);
    v += mo;
    if (sig) sig += mo;
    Q += mo * (sizeof(double) / sizeof(T));
  }
  const int tid = threadIdx.x;
  const int b = tid / F::TPF, tau = tid % F::TPF;
  const int pair = blockIdx.x * C::BR + b;
  const int ra = 2 * pair, rb = 2 * pair + 1;
  const bool va = ra < n2, vb = rb < n2;
  const double* xa = v + (size_t)ra * n1;
  const double* xb = v + (size_t)rb * n1;
  T* my = lds + b * lds_len(L);
  // Stage both rows in this FFT's LDS region (row a at 0, row b at L/2) with
  // contiguous loads: each value is fetched once, although the odd extension
  // uses it twice.  n1 = L/2 - 1 < TPF * PP/2.
  static_for<F::PP / 2>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    const int j = tau + k * F::TPF;
    if (j < n1) {
      my[j] = va ? (T)xa[j] : (T)0;
      my[L / 2 + j] = vb ? (T)xb[j] : (T)0;
    }
  });
  __syncthreads();
  cpx<T> reg[F::PP];
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    // odd extension: x_{p-1} at p in [1, n1], -x_{L-p-1} at p in [n1+2, L-1]
    int idx = -1;
    T sgn = (T)1;
    if (p >= 1 && p <= n1) {
      idx = p - 1;
    } else if (p >= n1 + 2) {
      idx = L - p - 1;
      sgn = (T)-1;
    }
    reg[e].re = idx >= 0 ? sgn * my[idx] : (T)0;
    reg[e].im = idx >= 0 ? sgn * my[L / 2 + idx] : (T)0;
  });
  __syncthreads();  // the forward sweep reuses the region
  fft_forward<T, F>(reg, tau, tw, my);
  const T s = (T)(0.5 * (sig ? *sig : 1.0));
  const int ld = n1 + 1;
  // Slots go through the LDS region (row a at 0, row b at ld = L/2) so that
  // the global stores are contiguous across the wavefront.
  __syncthreads();
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    constexpr int R = F::radix(F::NS - 1);
    if constexpr ((e % R) < R / 2) {
      const int slot = (tau + (e / R) * F::TPF) * (R / 2) + (e % R);
      my[slot] = -reg[e].im * s;    // sigma_a
      my[ld + slot] = reg[e].re * s;  // sigma_b
    }
  });
  __syncthreads();
  if constexpr (TL) {
    // Element j of this row pair's tiles: strip j / 8, row w / 4, slot 4 (j / 8) + w % 4
    // (w = j % 8); a missing row b (odd n2) is stored as the zeros staged for it.
    constexpr int NT = (8 * ((L / 2 + 3) / 4) + F::TPF - 1) / F::TPF;
    const int hp = (n2 + 1) >> 1;
    if (va) {
      T* qp = Q + (size_t)pair * 8;
      static_for<NT>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        const int j = tau + k * F::TPF;
        const int g = j >> 3, w = j & 7, c = 4 * g + (w & 3);
        if (c < ld) qp[(size_t)g * hp * 8 + w] = my[(w >> 2) * ld + c];
      });
    }
  } else {
    static_for<F::PP / 2>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      const int j = tau + k * F::TPF;  // < L/2 = ld
      if (va) Q[(size_t)ra * ld + j] = my[j];
      if (vb) Q[(size_t)rb * ld + j] = my[ld + j];
    });
  }
}

// --------------------------------------------------------------------------
// Pass B: slot-column pairs (ca, cb) of Q -> P1, P2 columns.
// --------------------------------------------------------------------------
template <typename T, int L, bool TL>
__global__ __launch_bounds__(PcColCfg<L>::THR_C) void k_pc_cols(
    const T* __restrict__ Q, T* __restrict__ P1, T* __restrict__ P2,
    const T* __restrict__ lamx_slot, const T* __restrict__ lamy_pos,
    const cpx<T>* __restrict__ tw, int n1, int n2, T kx, T ky, T dpen, T halfK, const Members mb,
    const double* __restrict__ mk) {
  using C = PcColCfg<L>;
  using F = typename C::F;
  __shared__ T lds[C::BC * lds_len(L)];
  {  // member of a batched launch (grid dimension z)
    const size_t mo = mb.off(blockIdx.z);
    const size_t mt = mo * (sizeof(double) / sizeof(T));
    Q += mt;
    P1 += mt;
    if (P2) P2 += mt;
    if (mk) {
      kx = (T)mk[mo];
      ky = (T)mk[mo + 1];
    }
  }
  const int tid = threadIdx.x;
  const int b = tid % C::BC, tau = tid / C::BC;
  const int strip = xcd_remap(blockIdx.x, gridDim.x);
  // Column pair of FFT b.  Tiled: (2c, 2c+1), adjacent in one tile row.
  // Natural: (base + b, base + b + BC) of the block's 2 BC columns, so that
  // each inverse sweep writes BC adjacent columns of a row (with (2c, 2c+1)
  // every sweep wrote every other column and half-written lines doubled the
  // write traffic).
  const int ca = TL ? 2 * (strip * C::BC + b) : 2 * C::BC * strip + b;
  const int cb = TL ? ca + 1 : ca + C::BC;
  const int ld = n1 + 1, hp = (n2 + 1) >> 1;
  const bool va = ca < ld, vb = cb < ld;  // tiled: ld and ca even, both or neither
  using V2 = typename Vec2<T>::type;
  cpx<T> reg[F::PP];
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    int row = -1;
    T sgn = (T)1;
    if (p >= 1 && p <= n2) {
      row = p - 1;
    } else if (p >= n2 + 2) {
      row = L - p - 1;
      sgn = (T)-1;
    }
    if constexpr (TL) {
      // ca is even: (ca, cb) are adjacent elements of one tile row
      const bool ok = vb && row >= 0;
      const V2 q = ok ? *(const V2*)(Q + tile_index(row, ca, hp)) : V2{(T)0, (T)0};
      reg[e].re = sgn * q.x;
      reg[e].im = sgn * q.y;
    } else {
      reg[e].re = (va && row >= 0) ? sgn * Q[(size_t)row * ld + ca] : (T)0;
      reg[e].im = (vb && row >= 0) ? sgn * Q[(size_t)row * ld + cb] : (T)0;
    }
  });
  T* my = lds + b;  // regions interleaved (stride BC)
  // (no register materialisation between the sweeps here: it measured slower)
  fft_forward<T, F, false, C::BC>(reg, tau, tw, my);
  // spectrum = 2 rho_b - 2i rho_a; keep rho_b for the second column
  const T lxa = va ? kx * lamx_slot[ca] : (T)0;
  const T lxb = vb ? kx * lamx_slot[cb] : (T)0;
  T rho_b[F::PP];
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const T ly = ky * lamy_pos[F::pos(F::NS - 1, tau, e)];
    const T rho_a = (T)-0.5 * reg[e].im;
    rho_b[e] = (T)0.5 * reg[e].re;
    const T e1 = (T)1 - lxa - ly;
    const T e2 = e1 + dpen;
    const T r = halfK * rho_a / (e1 * e2);
    // (K rho / 2) (1/E2 - i/E1)
    reg[e].re = r * e1;
    reg[e].im = -r * e2;
  });
  fft_inverse<T, F, false, C::BC>(reg, tau, tw, my);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    if (va && p >= 1 && p <= n2) {
      if constexpr (TL) {
        *(V2*)(P1 + pair_index<T>(p - 1, ca, n2)) = V2{reg[e].re, reg[e].im};
      } else {
        const size_t i = (size_t)(p - 1) * ld + ca;
        P1[i] = reg[e].re;
        P2[i] = reg[e].im;
      }
    }
  });
  // Hide the table pointer from the optimiser so that the second sweep reloads
  // its twiddles instead of keeping the first sweep's in registers.
  // (an opaque zero offset, not opaque pointers: those lose their global
  // address space and their loads become flat loads)
  int z0 = 0;
  asm volatile("" : "+s"(z0));
  const cpx<T>* tw2 = tw + z0;
  const T* lamy2 = lamy_pos + z0;
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const T ly = ky * lamy2[F::pos(F::NS - 1, tau, e)];
    const T e1 = (T)1 - lxb - ly;
    const T e2 = e1 + dpen;
    const T r = halfK * rho_b[e] / (e1 * e2);
    reg[e].re = r * e1;
    reg[e].im = -r * e2;
  });
  fft_inverse<T, F, false, C::BC>(reg, tau, tw2, my);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    if (vb && p >= 1 && p <= n2) {
      if constexpr (TL) {
        *(V2*)(P1 + pair_index<T>(p - 1, cb, n2)) = V2{reg[e].re, reg[e].im};
      } else {
        const size_t i = (size_t)(p - 1) * ld + cb;
        P1[i] = reg[e].re;
        P2[i] = reg[e].im;
      }
    }
  });
}

// --------------------------------------------------------------------------
// Raw sine transform along columns (used between the x and z transforms of
// the three-dimensional preconditioner, where the y transform stands alone).
// One FFT of length L = 2(rows+1) per column pair: column ca of inA in the
// real part, column cb of inB in the imaginary part, both odd-extended; the
// spectrum is 2 sigma_b - 2i sigma_a, read at frequencies 1..rows.
// --------------------------------------------------------------------------
template <typename T, int L>
__global__ __launch_bounds__(PcColCfg<L>::THR_C) void k_dst_cols(
    const T* __restrict__ inA, const T* __restrict__ inB, T* __restrict__ outA,
    T* __restrict__ outB, const cpx<T>* __restrict__ tw, int ncol, int cstride, int coff,
    int rows, int ld, size_t bstride) {
  using C = PcColCfg<L>;
  using F = typename C::F;
  __shared__ T lds[C::BC * lds_len(L)];
  {
    const size_t off = (size_t)blockIdx.y * bstride;
    inA += off;
    inB += off;
    outA += off;
    outB += off;
  }
  const int tid = threadIdx.x;
  const int b = tid % C::BC, tau = tid / C::BC;
  const int c = xcd_remap(blockIdx.x, gridDim.x) * C::BC + b;
  const bool valid = c < ncol;
  const int ca = c * cstride, cb = ca + coff;
  cpx<T> reg[F::PP];
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    int row = -1;
    T sgn = (T)1;
    if (p >= 1 && p <= rows) {
      row = p - 1;
    } else if (p >= rows + 2) {
      row = L - p - 1;
      sgn = (T)-1;
    }
    const bool ok = valid && row >= 0;
    reg[e].re = ok ? sgn * inA[(size_t)row * ld + ca] : (T)0;
    reg[e].im = ok ? sgn * inB[(size_t)row * ld + cb] : (T)0;
  });
  T* my = lds + b;  // regions interleaved (stride BC)
  fft_forward<T, F, false, C::BC>(reg, tau, tw, my);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int f = fft_freq(L, pc_cols_pts(L), F::pos(F::NS - 1, tau, e));
    if (valid && f >= 1 && f <= rows) {
      const size_t i = (size_t)(f - 1) * ld;
      outA[i + ca] = (T)-0.5 * reg[e].im;
      outB[i + cb] = (T)0.5 * reg[e].re;
    }
  });
}

// Pass C's loads: one row of P1 and of P2 (ld = L/2 slots each) staged in an
// FFT's LDS region with contiguous loads (P1 at 0, P2 at ld), then barrier.
template <typename T, class F>
__device__ __forceinline__ void stage_slots(const T* p1, const T* p2, bool vr, int ld, int tau,
                                            T* my) {
  static_for<F::PP / 2>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    const int j = tau + k * F::TPF;  // < L/2 = ld
    my[j] = vr ? p1[j] : (T)0;
    my[ld + j] = vr ? p2[j] : (T)0;
  });
  __syncthreads();
}

// The same from the row-segment layout of the pairs (pair_index): one
// 2-vector load per slot, a wavefront reading whole lines.
template <typename T, class F>
__device__ __forceinline__ void stage_slots_tiled(const T* pp, int r, bool vr, int ld, int rows,
                                                  int tau, T* my) {
  using V2 = typename Vec2<T>::type;
  static_for<F::PP / 2>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    const int j = tau + k * F::TPF;  // < L/2 = ld
    const V2 q = vr ? *(const V2*)(pp + pair_index<T>(r, j, rows)) : V2{(T)0, (T)0};
    my[j] = q.x;
    my[ld + j] = q.y;
  });
  __syncthreads();
}

// The inverse sweep's input from the staged slots: P2/2 - i P1/2 on the lower
// half of the spectrum, the odd mirror (slot computed by fft_mirror_slot) on
// the upper half; a barrier follows, since the sweep reuses the region.
template <typename T, class F>
__device__ __forceinline__ void load_staged_spectrum(cpx<T>* reg, int tau, int ld, T* my) {
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    constexpr int R = F::radix(F::NS - 1);
    if constexpr ((e % R) < R / 2) {
      const int slot = (tau + (e / R) * F::TPF) * (R / 2) + (e % R);
      reg[e].re = (T)0.5 * my[ld + slot];
      reg[e].im = (T)-0.5 * my[slot];
    } else {
      const int ms = fft_mirror_slot(1 << F::LOGL, F::PP, F::pos(F::NS - 1, tau, e));
      reg[e].re = ms >= 0 ? (T)-0.5 * my[ld + ms] : (T)0;
      reg[e].im = ms >= 0 ? (T)0.5 * my[ms] : (T)0;
    }
  });
  __syncthreads();
}

// --------------------------------------------------------------------------
// Pass C: one row r per FFT; spectrum P2/2 - i P1/2 on the lower half, odd
// mirror on the upper half; the inverse sweep gives (P1 S_x) + i (P2 S_x).
// --------------------------------------------------------------------------
template <typename T, int L, bool TL>
__global__ __launch_bounds__(PcCfg<L>::THR_R) void k_pc_rows_inv(
    const T* __restrict__ P1, const T* __restrict__ P2,
    const uint8_t* __restrict__ mask, double* __restrict__ z, const cpx<T>* __restrict__ tw,
    int n1, int n2, const Members mb) {
  using C = PcCfg<L>;
  using F = typename C::F;
  __shared__ T lds[C::BR * lds_len(L)];
  {  // member of a batched launch (grid dimension z)
    const size_t mo = mb.off(blockIdx.z);
    P1 += mo * (sizeof(double) / sizeof(T));
    if (P2) P2 += mo * (sizeof(double) / sizeof(T));
    z += mo;
  }
  const int tid = threadIdx.x;
  const int b = tid / F::TPF, tau = tid % F::TPF;
  const int r = blockIdx.x * C::BR + b;
  const bool vr = r < n2;
  const int ld = n1 + 1;
  T* my = lds + b * lds_len(L);
  if constexpr (TL)
    stage_slots_tiled<T, F>(P1, r, vr, ld, n2, tau, my);
  else
    stage_slots<T, F>(P1 + (size_t)r * ld, P2 + (size_t)r * ld, vr, ld, tau, my);
  cpx<T> reg[F::PP];
  load_staged_spectrum<T, F>(reg, tau, ld, my);
  fft_inverse<T, F>(reg, tau, tw, my);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    if (vr && p >= 1 && p <= n1) {
      const size_t i = (size_t)r * n1 + (p - 1);
      z[i] = mask[i] ? (double)reg[e].re : (double)reg[e].im;
    }
  });
}

// --------------------------------------------------------------------------
// Pass C fused with the row pass of the matrix-vector product that follows it
// in every Arnoldi step (w = M P_hat^{-1} v).  With n1 + 1 a power of two both
// are row passes of one FFT length (2(n1+1) = next_pow2(2 n1)), so one block
// takes a row pair through both: two inverse sweeps of pass C give z for rows
// ra and rb (stored: the Krylov method keeps z, and the column pass reads it),
// then one convolution on z_a + i z_b gives
//   t = (1 + dpen (1 - mask)) z + coef (C_x z) - theta sub
// (t strip-tiled over n1 columns when TL, as the column pass reads it).
// z is placed at positions 1..n1 of the convolution (where pass C leaves it),
// a circular shift that the convolution carries to its output.
// --------------------------------------------------------------------------
// ZT: the storage type of z.  With ZT = float (the preconditioned basis kept
// in FP32) z is rounded when stored and the product uses the rounded values,
// so that w = M z holds for the z that is kept.
template <typename T, int L, bool TL, typename ZT = double>
__global__ __launch_bounds__(PcCfg<L>::THR_R) __attribute__((amdgpu_waves_per_eu(4)))
void k_pc_rows_inv_mv(const T* __restrict__ P1, const T* __restrict__ P2,
                      const uint8_t* __restrict__ mask,
                      ZT* __restrict__ z, double* __restrict__ t,
                      const cpx<T>* __restrict__ twT, const cpx<double>* __restrict__ tw64,
                      const double* __restrict__ sym, double coef, double dpen,
                      const double* __restrict__ sub, double theta, int n1, int n2,
                      const Members mb, const double* __restrict__ mk) {
  using C = PcCfg<L>;
  using F = typename C::F;
  __shared__ double lds[C::BR * lds_len(L)];
  {  // member of a batched launch (grid dimension z)
    const size_t mo = mb.off(blockIdx.z);
    P1 += mo * (sizeof(double) / sizeof(T));
    if (P2) P2 += mo * (sizeof(double) / sizeof(T));
    z += mo;
    t += mo;
    if (sub) sub += mo;
    if (mk) coef = -mk[mo];
  }
  const int tid = threadIdx.x;
  const int b = tid / F::TPF, tau = tid % F::TPF;
  const int pair = blockIdx.x * C::BR + b;
  const int ra = 2 * pair, rb = 2 * pair + 1;
  const bool va = ra < n2, vb = rb < n2;
  const int ld = n1 + 1;
  double* my = lds + b * lds_len(L);
  double zb[F::PP];  // row b's z at this thread's positions, kept for the convolution
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    // opaque offsets: no per-point address is hoisted out of the loop (the
    // pointers keep their global address space: opaque pointers would not)
    int z0 = 0, th = tau;
    asm volatile("" : "+s"(z0), "+v"(th));
    const T* P1h = P1 + z0;
    const T* P2h = P2 ? P2 + z0 : nullptr;
    const cpx<T>* twh = twT + z0;
    ZT* zh = z + z0;
    const uint8_t* mh = mask + z0;
    const int r = ra + h;
    const bool vr = r < n2;
    T* myT = reinterpret_cast<T*>(my);
    __syncthreads();  // the previous row's sweep may still read the region
    if constexpr (TL)
      stage_slots_tiled<T, F>(P1h, r, vr, ld, n2, th, myT);
    else
      stage_slots<T, F>(P1h + (size_t)r * ld, P2h + (size_t)r * ld, vr, ld, th, myT);
    cpx<T> reg[F::PP];
    load_staged_spectrum<T, F>(reg, th, ld, myT);
    fft_inverse<T, F>(reg, th, twh, myT);
    static_for<F::PP>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      const int p = F::pos(0, th, e);
      double zv = 0.0;
      if (vr && p >= 1 && p <= n1) {
        const size_t i = (size_t)r * n1 + (p - 1);
        zv = (double)(ZT)(mh[i] ? (double)reg[e].re : (double)reg[e].im);
        zh[i] = (ZT)zv;
      }
      if (h == 1) zb[e] = zv;
    });
  }
  // Convolution input z_a + i z_b at the sweep's own positions: row b from
  // registers, row a read back where this same thread stored it (no other
  // thread's write is involved, so no barrier is needed).
  cpx<double> reg[F::PP];
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    const bool in = p >= 1 && p <= n1;
    reg[e].re = (va && in) ? (double)z[(size_t)ra * n1 + (p - 1)] : 0.0;
    reg[e].im = zb[e];
  });
  fft_forward<double, F>(reg, tau, tw64, my);
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const double sc = sym[F::pos(F::NS - 1, tau, e)] * coef;
    reg[e].re *= sc;
    reg[e].im *= sc;
  });
  fft_inverse<double, F>(reg, tau, tw64, my);
  const int hp = (n2 + 1) >> 1;
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int p = F::pos(0, tau, e);
    if (p >= 1 && p <= n1) {
      if (va) {
        const size_t i = (size_t)ra * n1 + (p - 1);
        double v = reg[e].re + (1.0 + dpen * (double)(1 - mask[i])) * (double)z[i];
        if (sub) v -= theta * sub[i];
        t[TL ? tile_index(ra, p - 1, hp) : i] = v;
      }
      if (vb) {
        const size_t i = (size_t)rb * n1 + (p - 1);
        double v = reg[e].im + (1.0 + dpen * (double)(1 - mask[i])) * (double)z[i];
        if (sub) v -= theta * sub[i];
        t[TL ? tile_index(rb, p - 1, hp) : i] = v;
      }
    }
  });
}

}  // namespace rsfde

#include "sd_kernels.hpp"

namespace rsfde {

// ------------------------------- launchers --------------------------------
template <typename T, int L, bool TL>
static hipError_t pc_rows_fwd_impl(const double* v, const double* sig, T* Q, const void* tw,
                                   int n1, int n2, hipStream_t s, const Members& mb) {
  using C = PcCfg<L>;
  const int pairs = (n2 + 1) / 2;
  const int blocks = (pairs + C::BR - 1) / C::BR;
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_pc_rows_fwd<T, L, TL>), dim3(blocks, 1, mb.n), dim3(C::THR_R), 0, s, v,
                     sig, Q, (const cpx<T>*)tw, n1, n2, mb);
  return hipGetLastError();
}

template <typename T, int L, bool TL>
static hipError_t pc_cols_impl(const T* Q, T* P1, T* P2, const T* lamx, const T* lamy,
                               const void* tw, int n1, int n2, double kx, double ky, double dpen,
                               double Kfac, hipStream_t s, const Members& mb, const double* mk) {
  using C = PcColCfg<L>;
  const int pairs = (n1 + 1) / 2;
  const int blocks = (pairs + C::BC - 1) / C::BC;
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_pc_cols<T, L, TL>), dim3(blocks, 1, mb.n), dim3(C::THR_C), 0, s, Q, P1, P2,
                     lamx, lamy, (const cpx<T>*)tw, n1, n2, (T)kx, (T)ky, (T)dpen,
                     (T)(0.5 * Kfac), mb, mk);
  return hipGetLastError();
}

template <typename T, int L, bool TL>
static hipError_t pc_rows_inv_impl(const T* P1, const T* P2,
                                   const uint8_t* mask, double* z, const void* tw, int n1, int n2,
                                   hipStream_t s, const Members& mb) {
  using C = PcCfg<L>;
  const int blocks = (n2 + C::BR - 1) / C::BR;
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_pc_rows_inv<T, L, TL>), dim3(blocks, 1, mb.n), dim3(C::THR_R), 0, s, P1,
                     P2, mask, z, (const cpx<T>*)tw, n1, n2, mb);
  return hipGetLastError();
}

template <typename T, int L, bool TL>
static hipError_t pc_rows_inv_mv_impl(const T* P1, const T* P2,
                                      const uint8_t* mask, void* z, bool z32, double* t, const void* twT,
                                      const void* tw64, const double* sym, double coef,
                                      double dpen, const double* sub, double theta, int n1,
                                      int n2, hipStream_t s, const Members& mb, const double* mk) {
  using C = PcCfg<L>;
  const int pairs = (n2 + 1) / 2;
  const int blocks = (pairs + C::BR - 1) / C::BR;
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  if (z32) {
    if constexpr (TL)
      hipLaunchKernelGGL((k_pc_rows_inv_mv<T, L, TL, float>), dim3(blocks, 1, mb.n), dim3(C::THR_R),
                         0, s, P1, P2, mask, (float*)z, t, (const cpx<T>*)twT,
                         (const cpx<double>*)tw64, sym, coef, dpen, sub, theta, n1, n2, mb, mk);
    else
      return hipErrorInvalidValue;  // FP32 storage of z: two-dimensional (tiled) plans only
  } else {
    hipLaunchKernelGGL((k_pc_rows_inv_mv<T, L, TL>), dim3(blocks, 1, mb.n), dim3(C::THR_R), 0, s, P1,
                       P2, mask, (double*)z, t, (const cpx<T>*)twT, (const cpx<double>*)tw64, sym,
                       coef, dpen, sub, theta, n1, n2, mb, mk);
  }
  return hipGetLastError();
}

template <typename T, int L>
static hipError_t dst_cols_impl(const T* inA, const T* inB, T* outA, T* outB, const void* tw,
                                int ncol, int cstride, int coff, int rows, int ld, int batch,
                                size_t bstride, hipStream_t s) {
  using C = PcColCfg<L>;
  if (L != 2 * (rows + 1) || batch < 1 || batch > 65535 || ncol < 1) return hipErrorInvalidValue;
  const int blocks = (ncol + C::BC - 1) / C::BC;
  hipLaunchKernelGGL((k_dst_cols<T, L>), dim3(blocks, batch), dim3(C::THR_C), 0, s, inA, inB, outA,
                     outB, (const cpx<T>*)tw, ncol, cstride, coff, rows, ld, bstride);
  return hipGetLastError();
}

template <typename T, int L>
static hipError_t sd_rows_fwd_impl(const double* v, const double* sig, T* Q, const void* twL,
                                   const void* twS, int n1, int n2, hipStream_t s,
                                   const Members& mb) {
  using C = SdRows<L>;
  const int pairs = (n2 + 1) / 2;
  const int blocks = (pairs + C::ND - 1) / C::ND;
  hipLaunchKernelGGL((k_sd_rows_fwd<T, L>), dim3(blocks, 1, mb.n), dim3(C::THR), 0, s, v, sig, Q,
                     (const cpx<T>*)twL, (const cpx<T>*)twS, n1, n2, mb);
  return hipGetLastError();
}

template <typename T, int L>
static hipError_t sd_cols_impl(const T* Q, T* P, const T* lamx, const T* lamy, const void* twL,
                               const void* twS, int n1, int n2, double kx, double ky,
                               double dpen, double Kfac, hipStream_t s, const Members& mb,
                               const double* mk) {
  using C = SdCols<L>;
  constexpr int BC = C::BC;
  const int pairs = (n1 + 1) / 2;
  const int blocks = (pairs + BC - 1) / BC;
  hipLaunchKernelGGL((k_sd_cols<T, L>), dim3(blocks, 1, mb.n), dim3(C::THR), 0, s, Q, P, lamx,
                     lamy, (const cpx<T>*)twL, (const cpx<T>*)twS, n1, n2, (T)kx, (T)ky, (T)dpen,
                     (T)(0.5 * Kfac), mb, mk);
  return hipGetLastError();
}

template <typename T, int L>
static hipError_t sd_rows_inv_impl(const T* P, const uint8_t* mask, double* z, const void* twL,
                                   const void* twS, const int32_t* msl, int n1, int n2,
                                   hipStream_t s, const Members& mb) {
  using C = SdRows<L>;
  const int blocks = (n2 + C::ND - 1) / C::ND;
  hipLaunchKernelGGL((k_sd_rows_inv<T, L>), dim3(blocks, 1, mb.n), dim3(C::THR), 0, s, P, mask, z,
                     (const cpx<T>*)twL, (const cpx<T>*)twS, msl, n1, n2, mb);
  return hipGetLastError();
}

template <typename T, int L>
static hipError_t sd_rows_inv_mv_impl(const T* P, const uint8_t* mask, void* z, bool z32,
                                      double* t, const void* twL, const void* twS,
                                      const int32_t* msl, const void* tw64, const double* sym,
                                      double coef, double dpen, const double* sub, double theta,
                                      int n1, int n2, hipStream_t s, const Members& mb,
                                      const double* mk) {
  using M = SdMvCfg<L>;
  const int blocks = (n2 + 1) / 2;
  if (z32)
    hipLaunchKernelGGL((k_sd_rows_inv_mv<T, L, float>), dim3(blocks, 1, mb.n), dim3(M::THR), 0, s,
                       P, mask, (float*)z, t, (const cpx<T>*)twL, (const cpx<T>*)twS, msl,
                       (const cpx<double>*)tw64, sym, coef, dpen, sub, theta, n1, n2, mb, mk);
  else
    hipLaunchKernelGGL((k_sd_rows_inv_mv<T, L>), dim3(blocks, 1, mb.n), dim3(M::THR), 0, s, P,
                       mask, (double*)z, t, (const cpx<T>*)twL, (const cpx<T>*)twS, msl,
                       (const cpx<double>*)tw64, sym, coef, dpen, sub, theta, n1, n2, mb, mk);
  return hipGetLastError();
}

// Pass selection: the symmetric form for the tiled layouts when its tables are
// given and L >= kSdMinL, the plain FFT form otherwise.
template <typename T, int L>
static hipError_t rows_fwd_any(const double* v, const double* sig, T* Q, const void* tw, int n1,
                               int n2, bool tiled, hipStream_t s, const Members& mb,
                               const SdTabs& sd) {
  if constexpr (L >= kSdMinL) {
    if (tiled && sd.twS) return sd_rows_fwd_impl<T, L>(v, sig, Q, tw, sd.twS, n1, n2, s, mb);
  }
  return tiled ? pc_rows_fwd_impl<T, L, true>(v, sig, Q, tw, n1, n2, s, mb)
               : pc_rows_fwd_impl<T, L, false>(v, sig, Q, tw, n1, n2, s, mb);
}

template <typename T, int L>
static hipError_t cols_any(const T* Q, T* P1, T* P2, const T* lamx, const T* lamy, const void* tw,
                           int n1, int n2, double kx, double ky, double dpen, double Kfac,
                           bool tiled, hipStream_t s, const Members& mb, const double* mk,
                           const SdTabs& sd) {
  if constexpr (L >= kSdMinL) {
    if (tiled && sd.twS)
      return sd_cols_impl<T, L>(Q, P1, lamx, lamy, tw, sd.twS, n1, n2, kx, ky, dpen, Kfac, s, mb,
                                mk);
  }
  return tiled ? pc_cols_impl<T, L, true>(Q, P1, P2, lamx, lamy, tw, n1, n2, kx, ky, dpen, Kfac,
                                          s, mb, mk)
               : pc_cols_impl<T, L, false>(Q, P1, P2, lamx, lamy, tw, n1, n2, kx, ky, dpen, Kfac,
                                           s, mb, mk);
}

template <typename T, int L>
static hipError_t rows_inv_any(const T* P1, const T* P2, const uint8_t* mask, double* z,
                               const void* tw, int n1, int n2, bool tiled, hipStream_t s,
                               const Members& mb, const SdTabs& sd) {
  if constexpr (L >= kSdMinL) {
    if (tiled && sd.twS)
      return sd_rows_inv_impl<T, L>(P1, mask, z, tw, sd.twS, sd.msl, n1, n2, s, mb);
  }
  return tiled ? pc_rows_inv_impl<T, L, true>(P1, P2, mask, z, tw, n1, n2, s, mb)
               : pc_rows_inv_impl<T, L, false>(P1, P2, mask, z, tw, n1, n2, s, mb);
}

template <typename T, int L>
static hipError_t rows_inv_mv_any(const T* P1, const T* P2, const uint8_t* mask, void* z,
                                  bool z32, double* t, const void* twT, const void* tw64,
                                  const double* sym, double coef, double dpen, const double* sub,
                                  double theta, int n1, int n2, bool tiled, hipStream_t s,
                                  const Members& mb, const double* mk, const SdTabs& sd) {
  if constexpr (L >= kSdMinL) {
    if (tiled && sd.twS)
      return sd_rows_inv_mv_impl<T, L>(P1, mask, z, z32, t, twT, sd.twS, sd.msl, tw64,
                                       sym, coef, dpen, sub, theta, n1, n2,
                                       s, mb, mk);
  }
  return tiled ? pc_rows_inv_mv_impl<T, L, true>(P1, P2, mask, z, z32, t, twT, tw64, sym, coef,
                                                 dpen, sub, theta, n1, n2, s, mb, mk)
               : pc_rows_inv_mv_impl<T, L, false>(P1, P2, mask, z, z32, t, twT, tw64, sym, coef,
                                                  dpen, sub, theta, n1, n2, s, mb, mk);
}

#define RSFDE_LD_CASES(X) \
  X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192)

template <typename T>
hipError_t launch_pc_rows_fwd(int Lx, const double* v, const double* sig, T* Q, const void* tw,
                              int n1, int n2, bool tiled, hipStream_t s, const Members& mb,
                              const SdTabs& sd) {
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  switch (Lx) {
#define X(LL) \
  case LL:    \
    return rows_fwd_any<T, LL>(v, sig, Q, tw, n1, n2, tiled, s, mb, sd);
    RSFDE_LD_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_pc_cols(int Ly, const T* Q, T* P1, T* P2, const T* lamx_slot,
                          const T* lamy_pos, const void* tw, int n1, int n2, double kx, double ky,
                          double dpen, double Kfac, bool tiled, hipStream_t s, const Members& mb,
                          const double* mk, const SdTabs& sd) {
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  switch (Ly) {
#define X(LL)                                                                                 \
  case LL:                                                                                    \
    return cols_any<T, LL>(Q, P1, P2, lamx_slot, lamy_pos, tw, n1, n2, kx, ky, dpen, Kfac, tiled, \
                           s, mb, mk, sd);
    RSFDE_LD_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_dst_cols(int L, const T* inA, const T* inB, T* outA, T* outB, const void* tw,
                           int ncol, int cstride, int coff, int rows, int ld, int batch,
                           size_t bstride, hipStream_t s) {
  switch (L) {
#define X(LL) \
  case LL:    \
    return dst_cols_impl<T, LL>(inA, inB, outA, outB, tw, ncol, cstride, coff, rows, ld, batch, \
                                bstride, s);
    RSFDE_LD_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_pc_rows_inv(int Lx, const T* P1, const T* P2,
                              const uint8_t* mask, double* z, const void* tw, int n1, int n2,
                              bool tiled, hipStream_t s, const Members& mb, const SdTabs& sd) {
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  switch (Lx) {
#define X(LL) \
  case LL:    \
    return rows_inv_any<T, LL>(P1, P2, mask, z, tw, n1, n2, tiled, s, mb, sd);
    RSFDE_LD_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_pc_rows_inv_mv(int L, const T* P1, const T* P2,
                                 const uint8_t* mask, void* z, double* t, const void* twT,
                                 const void* tw64, const double* sym, double coef, double dpen,
                                 const double* sub, double theta, int n1, int n2, bool tiled,
                                 hipStream_t s, const Members& mb, const double* mk, bool z32,
                                 const SdTabs& sd) {
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  switch (L) {
#define X(LL)                                                                                  \
  case LL:                                                                                     \
    return rows_inv_mv_any<T, LL>(P1, P2, mask, z, z32, t, twT, tw64, sym, coef, dpen, sub,    \
                                  theta, n1, n2, tiled, s, mb, mk, sd);
    RSFDE_LD_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace rsfde
