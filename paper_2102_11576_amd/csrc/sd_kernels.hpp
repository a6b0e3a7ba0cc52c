// Passes A, B and C of the power-of-two preconditioner (Section 4.1, Lemma
// 4.2) on the symmetric sine transform of sd_engine.hpp, for the
// two-dimensional (strip-tiled) layouts and L >= kSdMinL.  Same intermediates
// as the plain passes (Q strip-tiled, the (P1, P2) pairs in pair_index order),
// but the x slots follow Sd<L>::slot, and pass B's y eigenvalues are indexed
// by block position.  One transform takes 9 sub-FFTs of TS threads (TPD
// threads); the row passes run ND transforms per block and pass B BC column
// pairs, interleaved (SdRows, SdCols).
#pragma once

#include "sd_engine.hpp"

namespace rsfde {

// Transforms per block of the row passes and column pairs per block of pass B
// (one transform = 9 sub-FFTs of TS threads each): one from L = 4096 on and
// up to L = 1024 (grids of at most 511 rows or columns: more, smaller blocks
// spread them over more CUs), 16 / TS = 2 at L = 2048.  Small blocks keep
// more of them resident per CU (pass B's pair takes 38 KB of LDS with its
// stash at L = 4096), which hides more latency.
template <int L>
struct SdRows {
  static constexpr int ND = (L <= 1024 || Sd<L>::TS >= 16) ? 1 : 16 / Sd<L>::TS;
  static constexpr int THR = ND * Sd<L>::TPD;
};
template <int L>
struct SdCols {
  static constexpr int BC = (L <= 1024 || Sd<L>::TS >= 16) ? 1 : 16 / Sd<L>::TS;
  // Up to L = 2048 the two inverse sweeps of a column pair run at once, on a
  // second set of BC TPD threads (too few column pairs to fill the GPU there).
  static constexpr bool CONC = L <= 2048;
  static constexpr int THR = (CONC ? 2 : 1) * BC * Sd<L>::TPD;
};
// Threads of one sub-FFT inside one wavefront (ST: LDS interleave of the
// transforms of a block): its exchanges then need no block barrier.
template <int L, int ST>
constexpr int sd_tw() {
  static_assert(Sd<L>::TS * ST <= 64 || (Sd<L>::TS * ST) % 64 == 0, "sub-FFT thread groups");
  return (Sd<L>::TS * ST <= 64) ? Sd<L>::TS : 64 / ST;
}

// Forward symmetric sweep of one transform.  Group-stage threads (g, group p)
// hold the odd extension's values at positions p + LS m in v[]; w1 = W_L^p and
// rs, the sub-FFT roots, come loaded with the values (their latency overlaps
// that of the data); after the
// sweep, block-stage threads (block r, sub-FFT thread tau; all threads of the
// transform) hold the spectrum of block r in v[] (sub-FFT DIF order).  The
// group stage's 18 outputs go through the transform's LDS region one part at
// a time (real, then imaginary), so v[] serves both roles.
template <typename T, int L, int ST, int TWs, bool MAT>
__device__ __forceinline__ void sd_forward(cpx<T>* v, bool g, int p, int r, int tau, cpx<T> w1,
                                           const Roots<T, typename Sd<L>::Fs>& rs, T* region,
                                           bool act = true) {
  using S = Sd<L>;
  using Fs = typename S::Fs;
  constexpr int LS = S::LS;
  cpx<T> m8{(T)0, (T)0};
  if (g) sd_group_fwd<T, L>(v, w1, m8);
  const bool mir = g && p != 0 && p != LS / 2;
  const int pd = lds_pad(p), pm = lds_pad(LS - p);
  constexpr int BL = LS + LS / 16;  // padded length of one block
  T* base = region + lds_pad(r * LS) * ST;
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    const bool im = part == 1;
    if (g) {
      static_for<9>([&](auto rr) {
        constexpr int q = decltype(rr)::value;
        region[(q * BL + pd) * ST] = im ? v[q].im : v[q].re;
      });
    }
    if (mir) {
      region[pm * ST] = im ? -v[0].im : -v[0].re;
      static_for<7>([&](auto rr) {
        constexpr int q = decltype(rr)::value + 1;
        region[(q * BL + pm) * ST] = im ? v[16 - q].im : v[16 - q].re;
      });
      region[(8 * BL + pm) * ST] = im ? m8.im : m8.re;
    }
    __syncthreads();
    if (act) lds_get<T, Fs, 0, ST>(v, tau, base, im);
    __syncthreads();
  }
  fft_forward_r<T, Fs, MAT, ST, TWs>(v, tau, rs, base, act);
}

// Inverse symmetric sweep: block-stage threads hold the odd spectrum of block
// r in v[] (sub-FFT DIF order); afterwards group-stage threads (g, group q)
// hold L times the odd extension at positions q + LS m in v[].  w1 = W_L^q and
// rs (the sub-FFT roots, Roots::load_inv) are loaded by the caller up front.
template <typename T, int L, int ST, int TWs, bool MAT>
__device__ __forceinline__ void sd_inverse(cpx<T>* v, bool g, int q, int r, int tau, cpx<T> w1,
                                           const Roots<T, typename Sd<L>::Fs>& rs, T* region,
                                           bool act = true) {
  using S = Sd<L>;
  using Fs = typename S::Fs;
  constexpr int LS = S::LS;
  constexpr int BL = LS + LS / 16;
  T* base = region + lds_pad(r * LS) * ST;
  fft_inverse_r<T, Fs, MAT, ST, TWs>(v, tau, rs, base, act);
  const int qd = lds_pad(q), qm = lds_pad((LS - q) & (LS - 1));
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    const bool im = part == 1;
    if (act) lds_put<T, Fs, 0, ST>(v, tau, base, im);
    __syncthreads();
    if (g) {
      static_for<9>([&](auto rr) {
        constexpr int k = decltype(rr)::value;
        (im ? v[k].im : v[k].re) = region[(k * BL + qd) * ST];
      });
      static_for<7>([&](auto rr) {
        constexpr int k = decltype(rr)::value + 1;
        (im ? v[16 - k].im : v[16 - k].re) = region[(k * BL + qm) * ST];
      });
    }
    __syncthreads();
  }
  if (g) sd_group_inv<T, L>(v, w1);
}

// Spectrum of one row from the pairs of pass B (pair_index layout): P2/2 - i P1/2
// at every slot; the upper halves of blocks 0 and 8 from their mirror slots
// (msl, -1 where the frequency is L/2) with the sign of odd symmetry.  Every
// load is unconditional (clamped to a valid address, the value then selected
// or scaled by 0), so that all of them are in flight at once.
template <typename T, int L>
__device__ __forceinline__ void sd_load_spectrum(cpx<T>* v, const T* __restrict__ P, int row,
                                                 bool vr, int r, int tau, int rows,
                                                 const int32_t* __restrict__ msl) {
  using S = Sd<L>;
  using Fs = typename S::Fs;
  using V2 = typename Vec2<T>::type;
  constexpr int LS = S::LS, TS = S::TS;
  const bool edge = r == 0 || r == 8;
  const int mid0 = r * LS + tau;                     // blocks 1..7: every register
  const int edge0 = (r == 8 ? LS / 2 : 0) + tau;     // blocks 0, 8: lower half
  const int mbase = r == 8 ? LS : 0;
  const int rr = vr ? row : 0;
  const T half = vr ? (T)0.5 : (T)0;
  int c[16];
  int sgn[16];  // odd-symmetry sign of the upper registers (0: frequency L/2)
  static_for<16>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    constexpr int lr = S::lower_rank(e);
    if constexpr (lr >= 0) {
      c[e] = edge ? edge0 + lr * TS : mid0 + e * TS;
    } else {
      const int m = msl[edge ? mbase + Fs::pos(Fs::NS - 1, tau, e) : 0];
      c[e] = edge ? (m >= 0 ? m : 0) : mid0 + e * TS;
      sgn[e] = edge ? (m >= 0 ? -1 : 0) : 1;
    }
  });
  static_for<16>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const V2 q = *(const V2*)(P + pair_index<T>(rr, c[e], rows));
    T h = half;
    if constexpr (S::lower_rank(e) < 0) h = (T)sgn[e] * half;
    v[e].re = h * q.y;
    v[e].im = -h * q.x;
  });
}

// z = mask ? re : im at the natural positions of group q's outputs (skipping
// the duplicates of the self-mirrored groups 0 and LS/2), stored as ZT; with
// st given, the stored values are also staged there (index j - 1).  The mask
// bytes are loaded first, all at once.
template <typename T, int L, typename ZT>
__device__ __forceinline__ void sd_store_z(const cpx<T>* v, int q, int row, bool vr, int n1,
                                           const uint8_t* __restrict__ mask, ZT* __restrict__ z,
                                           double* st) {
  using S = Sd<L>;
  const size_t rb = (size_t)(vr ? row : 0) * n1;
  static_for<2>([&](auto hh) {  // two halves of 8 registers
    constexpr int m0 = decltype(hh)::value * 8;
    bool ok[8];
    uint8_t mk[8];
    static_for<8>([&](auto mm) {
      constexpr int m = m0 + decltype(mm)::value;
      bool neg;
      const int j = S::nat(q, m, neg);
      ok[m - m0] = vr && (m < 8 || (q != 0 && q != S::LS / 2)) && j >= 1 && j <= n1;
      mk[m - m0] = mask[rb + (ok[m - m0] ? j - 1 : 0)];
    });
    static_for<8>([&](auto mm) {
      constexpr int m = m0 + decltype(mm)::value;
      bool neg;
      const int j = S::nat(q, m, neg);
      if (ok[m - m0]) {
        const T val = mk[m - m0] ? v[m].re : v[m].im;
        const ZT zv = (ZT)(neg ? -(double)val : (double)val);
        z[rb + (j - 1)] = zv;
        if (st) st[j - 1] = (double)zv;
      }
    });
  });
}

// --------------------------------------------------------------------------
// Pass A: row pairs (ra, rb) -> Q (strip-tiled), ND row pairs per block.
// --------------------------------------------------------------------------
template <typename T, int L>
__global__ __launch_bounds__(SdRows<L>::THR) void k_sd_rows_fwd(
    const double* __restrict__ v, const double* __restrict__ sig, T* __restrict__ Q,
    const cpx<T>* __restrict__ twL, const cpx<T>* __restrict__ twS, int n1, int n2,
    const Members mb) {
  using S = Sd<L>;
  using C = SdRows<L>;
  __shared__ T lds[C::ND * S::LEN];
  {  // member of a batched launch (grid dimension z); offsets in doubles
    const size_t mo = mb.off(blockIdx.z);
    v += mo;
    if (sig) sig += mo;
    Q += mo * (sizeof(double) / sizeof(T));
  }
  const int tid = threadIdx.x;
  const int d = tid / S::TPD, tg = tid % S::TPD;
  const int pair = blockIdx.x * C::ND + d;
  const int ra = 2 * pair, rb = ra + 1;
  const bool va = ra < n2, vb = rb < n2;
  const bool g = tg < S::NG;
  const int r = tg / S::TS, tau = tg % S::TS;
  // loads from clamped addresses, all in flight at once; out-of-range values select 0
  const double* xa = v + (size_t)(va ? ra : 0) * n1;
  const double* xb = v + (size_t)(vb ? rb : 0) * n1;
  cpx<T> reg[16];
  const cpx<T> w1 = twL[g ? tg : 0];
  Roots<T, typename S::Fs> rs;
  rs.load_fwd(tau, twS);
  if (g) {
    static_for<16>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      bool neg;
      const int j = S::nat(tg, m, neg);
      const bool in = j >= 1 && j <= n1;
      const int jj = in ? j - 1 : 0;
      const T a = (T)xa[jj], b = (T)xb[jj];
      const T sa = (va && in) ? (neg ? (T)-1 : (T)1) : (T)0;
      const T sb = (vb && in) ? (neg ? (T)-1 : (T)1) : (T)0;
      reg[m].re = sa * a;
      reg[m].im = sb * b;
    });
  }
  sd_forward<T, L, 1, sd_tw<L, 1>(), true>(reg, g, tg, r, tau, w1, rs, lds + d * S::LEN);
  if (!va) return;
  const T s = (T)(0.5 * (sig ? *sig : 1.0));
  const int hp = (n2 + 1) >> 1;
  // spectrum = 2 sigma_b - 2i sigma_a; row b of an odd n2 holds the zeros loaded for it
  static_for<16>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const int c = S::slot(r, tau, e);
    if (c >= 0) {
      const size_t i = tile_index(ra, c, hp);
      Q[i] = -reg[e].im * s;
      Q[i + 4] = reg[e].re * s;
    }
  });
}

// --------------------------------------------------------------------------
// Pass B: slot-column pairs (2c, 2c+1) of Q -> (P1, P2) pairs, ND column pairs
// per block, interleaved (column pair fastest in the thread index).
// --------------------------------------------------------------------------
template <typename T, int L>
__global__ __launch_bounds__(SdCols<L>::THR) __attribute__((amdgpu_waves_per_eu(3))) void k_sd_cols(
    const T* __restrict__ Q, T* __restrict__ P, const T* __restrict__ lamx_slot,
    const T* __restrict__ lamy_blk, const cpx<T>* __restrict__ twL,
    const cpx<T>* __restrict__ twS, int n1, int n2, T kx, T ky, T dpen, T halfK,
    const Members mb, const double* __restrict__ mk) {
  using S = Sd<L>;
  constexpr int BC = SdCols<L>::BC;
  constexpr int TWs = sd_tw<L, BC>();
  using Fs = typename S::Fs;
  using V2 = typename Vec2<T>::type;
  __shared__ T lds[(SdCols<L>::CONC ? 2 : 1) * BC * S::LEN];
  __shared__ T stash[BC * 16 * S::TPD];  // rho_b between the two inverse sweeps
  {  // member of a batched launch (grid dimension z)
    const size_t mo = mb.off(blockIdx.z);
    const size_t mt = mo * (sizeof(double) / sizeof(T));
    Q += mt;
    P += mt;
    if (mk) {
      kx = (T)mk[mo];
      ky = (T)mk[mo + 1];
    }
  }
  constexpr bool CONC = SdCols<L>::CONC;
  const int tid = threadIdx.x;
  // set h = 1 (CONC only) takes the second inverse sweep
  const int h = CONC ? tid / (BC * S::TPD) : 0;
  const int tl = tid - h * (BC * S::TPD);
  const int b = tl % BC, tg = tl / BC;
  const int strip = xcd_remap(blockIdx.x, gridDim.x);
  const int ca = 2 * (strip * BC + b), cb = ca + 1;
  const int ld = n1 + 1, hp = (n2 + 1) >> 1;
  const bool va = ca < ld;  // ld even: both columns or neither
  const bool f0 = h == 0;   // threads of the forward sweep
  const bool g = tg < S::NG;
  const int r = tg / S::TS, tau = tg % S::TS;
  cpx<T> reg[16];
  // the loads of the tables (clamped addresses) go out with the data's
  const cpx<T> w1 = twL[g ? tg : 0];  // the group root of all three sweeps (W_L^p)
  const T lxa = kx * lamx_slot[va ? ca : 0], lxb = kx * lamx_slot[va ? cb : 0];
  if (g && f0) {  // clamped loads, all in flight at once
    const int cc = va ? ca : 0;
    static_for<16>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      bool neg;
      const int j = S::nat(tg, m, neg);
      const bool ok = va && j >= 1 && j <= n2;
      const V2 q = *(const V2*)(Q + tile_index(ok ? j - 1 : 0, cc, hp));
      const T sgn = ok ? (neg ? (T)-1 : (T)1) : (T)0;
      reg[m].re = sgn * q.x;
      reg[m].im = sgn * q.y;
    });
  }
  T* my = lds + h * (BC * S::LEN) + b;  // regions interleaved (stride BC); one per set
  {
    Roots<T, Fs> rs;  // (loaded per sweep: held across the kernel they cost occupancy)
    rs.load_fwd(tau, twS);
    sd_forward<T, L, BC, TWs, false>(reg, g && f0, tg, r, tau, w1, rs, my, f0);
  }
  // spectrum = 2 rho_b - 2i rho_a; rho_b waits in LDS for the second column
  // (in registers it would cost a wavefront of occupancy)
  // The y eigenvalues stay in registers for the second column (a block of
  // 2.25 wavefronts is held to 3 per SIMD by its LDS anyway).
  const T* lamy = lamy_blk + r * S::LS;
  T* rb = stash + tg * BC + b;
  T ly[16];
  static_for<16>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    ly[e] = ky * lamy[Fs::pos(Fs::NS - 1, tau, e)];
  });
  if (f0) {
    static_for<16>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      const T rho_a = (T)-0.5 * reg[e].im;
      rb[e * S::TPD * BC] = (T)0.5 * reg[e].re;
      const T e1 = (T)1 - lxa - ly[e];
      const T e2 = e1 + dpen;
      const T q = halfK * rho_a / (e1 * e2);
      // (K rho / 2) (1/E2 - i/E1)
      reg[e].re = q * e1;
      reg[e].im = -q * e2;
    });
  }
  if constexpr (CONC) {
    // the second set takes rho_b from the stash and runs its sweep beside the first
    __syncthreads();
    if (!f0) {
      static_for<16>([&](auto ee) {
        constexpr int e = decltype(ee)::value;
        const T e1 = (T)1 - lxb - ly[e];
        const T e2 = e1 + dpen;
        const T q = halfK * rb[e * S::TPD * BC] / (e1 * e2);
        reg[e].re = q * e1;
        reg[e].im = -q * e2;
      });
    }
    {
      Roots<T, Fs> rs;
      rs.load_inv(tau, twS);
      sd_inverse<T, L, BC, TWs, false>(reg, g, tg, r, tau, w1, rs, my);
    }
    if (g && va) {
      const int cw = f0 ? ca : cb;
      static_for<16>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        bool neg;
        const int j = S::nat(tg, m, neg);
        if ((m < 8 || (tg != 0 && tg != S::LS / 2)) && j >= 1 && j <= n2)
          *(V2*)(P + pair_index<T>(j - 1, cw, n2)) =
              neg ? V2{-reg[m].re, -reg[m].im} : V2{reg[m].re, reg[m].im};
      });
    }
    return;
  }
  {
    Roots<T, Fs> rs;
    rs.load_inv(tau, twS);
    sd_inverse<T, L, BC, TWs, false>(reg, g, tg, r, tau, w1, rs, my);
  }
  if (g && va) {
    static_for<16>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      bool neg;
      const int j = S::nat(tg, m, neg);
      if ((m < 8 || (tg != 0 && tg != S::LS / 2)) && j >= 1 && j <= n2)
        *(V2*)(P + pair_index<T>(j - 1, ca, n2)) =
            neg ? V2{-reg[m].re, -reg[m].im} : V2{reg[m].re, reg[m].im};
    });
  }
  static_for<16>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    const T e1 = (T)1 - lxb - ly[e];
    const T e2 = e1 + dpen;
    const T q = halfK * rb[e * S::TPD * BC] / (e1 * e2);
    reg[e].re = q * e1;
    reg[e].im = -q * e2;
  });
  {
    Roots<T, Fs> rs;
    rs.load_inv(tau, twS);
    sd_inverse<T, L, BC, TWs, false>(reg, g, tg, r, tau, w1, rs, my);
  }
  if (g && va) {
    static_for<16>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      bool neg;
      const int j = S::nat(tg, m, neg);
      if ((m < 8 || (tg != 0 && tg != S::LS / 2)) && j >= 1 && j <= n2)
        *(V2*)(P + pair_index<T>(j - 1, cb, n2)) =
            neg ? V2{-reg[m].re, -reg[m].im} : V2{reg[m].re, reg[m].im};
    });
  }
}

// --------------------------------------------------------------------------
// Pass C: one row per transform, ND rows per block; the inverse sweep of
// P2/2 - i P1/2 gives (P1 S_x) + i (P2 S_x), combined by the mask into z.
// --------------------------------------------------------------------------
template <typename T, int L>
__global__ __launch_bounds__(SdRows<L>::THR) void k_sd_rows_inv(
    const T* __restrict__ P, const uint8_t* __restrict__ mask, double* __restrict__ z,
    const cpx<T>* __restrict__ twL, const cpx<T>* __restrict__ twS,
    const int32_t* __restrict__ msl, int n1, int n2, const Members mb) {
  using S = Sd<L>;
  using C = SdRows<L>;
  __shared__ T lds[C::ND * S::LEN];
  {  // member of a batched launch (grid dimension z)
    const size_t mo = mb.off(blockIdx.z);
    P += mo * (sizeof(double) / sizeof(T));
    z += mo;
  }
  const int tid = threadIdx.x;
  const int d = tid / S::TPD, tg = tid % S::TPD;
  const int row = blockIdx.x * C::ND + d;
  const bool vr = row < n2;
  const bool g = tg < S::NG;
  const int r = tg / S::TS, tau = tg % S::TS;
  cpx<T> reg[16];
  const cpx<T> w1 = twL[g ? tg : 0];
  Roots<T, typename S::Fs> rs;
  rs.load_inv(tau, twS);
  sd_load_spectrum<T, L>(reg, P, row, vr, r, tau, n2, msl);
  sd_inverse<T, L, 1, sd_tw<L, 1>(), true>(reg, g, tg, r, tau, w1, rs, lds + d * S::LEN);
  if (g) sd_store_z<T, L, double>(reg, tg, row, vr, n1, mask, z, nullptr);
}

// --------------------------------------------------------------------------
// Pass C fused with the row pass of the matrix-vector product (w = M P^{-1} v
// in every Arnoldi step; the convolution length of the x Toeplitz factor is L
// as well).  NP row pairs per block: first the 2 NP inverse sine transforms
// (rows 2 pair, 2 pair + 1), which store z and stage it in LDS in natural
// order; then one convolution per pair on z_a + i z_b,
//   t = (1 + dpen (1 - mask)) z + coef (C_x z) - theta sub
// (strip-tiled), with z at positions 1..n1 of the convolution.  Positions at
// and above L/2 are zero on input and unused on output, known at compile time.
// ZT: storage type of z (FP32 storage rounds z before the product uses it).
// --------------------------------------------------------------------------
template <int L>
struct SdMvCfg {
  using S = Sd<L>;
  using F = Fft<L, fft_pts(L)>;  // convolution engine
  // Up to L = 2048 (grids of at most 1023 rows, too few row pairs to fill the
  // GPU) the two sine transforms of a row pair run at once, on 2 TPD
  // threads.  From L = 4096 on they run one after the other on the first TPD
  // threads (a block is then the convolution's TPF threads, and a block per
  // row pair keeps the whole grid resident at once on 256 CUs).
  // (At L = 2048 the two transform regions and the staged z hold the
  // concurrent form to three waves per SIMD by their LDS, so its occupancy
  // hint asks for three; the smaller lengths compile the same either way.)
  static constexpr bool CONC = L <= 2048;
  static constexpr int TD = CONC ? 2 * S::TPD : S::TPD;
  static constexpr int THR = TD > F::TPF ? TD : F::TPF;
  // LDS in doubles.  Sequential: row a's staged z [0, L/2), then the transform
  // region (type T), which row b's staged z [L/2, L) replaces.  Concurrent:
  // the staged z of both rows [0, L), then the two regions.  The convolution
  // overlays all.
  template <typename T>
  static constexpr int lds_doubles() {
    constexpr int a = CONC ? L + (2 * S::LEN * (int)sizeof(T) + 7) / 8
                           : L / 2 + (S::LEN * (int)sizeof(T) + 7) / 8;
    constexpr int b = lds_len(L);
    return a > b ? a : b;
  }
  // register e of the convolution's first (last) stage is at or above L/2 for every thread
  static constexpr bool upper(int e) {
    for (int tau = 0; tau < F::TPF; ++tau)
      if (F::pos(0, tau, e) < L / 2) return false;
    return true;
  }
};

template <typename T, int L, typename ZT = double>
__global__ __launch_bounds__(SdMvCfg<L>::THR) __attribute__((amdgpu_waves_per_eu(SdMvCfg<L>::CONC ? 3 : 4)))
void k_sd_rows_inv_mv(
    const T* __restrict__ P, const uint8_t* __restrict__ mask, ZT* __restrict__ z,
    double* __restrict__ t, const cpx<T>* __restrict__ twL, const cpx<T>* __restrict__ twS,
    const int32_t* __restrict__ msl, const cpx<double>* __restrict__ tw64,
    const double* __restrict__ sym, double coef, double dpen, const double* __restrict__ sub,
    double theta, int n1, int n2, const Members mb, const double* __restrict__ mk) {
  using S = Sd<L>;
  using M = SdMvCfg<L>;
  using F = typename M::F;
  constexpr int TWs = sd_tw<L, 1>();
  __shared__ double lds[M::template lds_doubles<T>()];
  {  // member of a batched launch (grid dimension z)
    const size_t mo = mb.off(blockIdx.z);
    P += mo * (sizeof(double) / sizeof(T));
    z += mo;
    t += mo;
    if (sub) sub += mo;
    if (mk) coef = -mk[mo];
  }
  const int tid = threadIdx.x;
  const int pair = blockIdx.x;
  const int ra = 2 * pair, rb = ra + 1;
  const bool va = ra < n2, vb = rb < n2;
  // ---- the inverse sine transforms of rows ra and rb
  if constexpr (M::CONC) {  // both at once: row ra + h on threads [h TPD, (h + 1) TPD)
    const int h = tid >= S::TPD ? 1 : 0;
    const int th = tid - h * S::TPD;
    const bool act = tid < 2 * S::TPD;
    const bool g = act && th < S::NG;
    const int r = act ? th / S::TS : 0, tau = th % S::TS;
    const int row = ra + h;
    const bool vr = row < n2;
    T* region = reinterpret_cast<T*>(lds + L) + h * S::LEN;
    cpx<T> reg[16];
    const cpx<T> w1 = twL[g ? th : 0];
    Roots<T, typename S::Fs> rs;
    rs.load_inv(tau, twS);
    if (act) sd_load_spectrum<T, L>(reg, P, row, vr, r, tau, n2, msl);
    sd_inverse<T, L, 1, TWs, true>(reg, g, th, r, tau, w1, rs, region, act);
    if (g) sd_store_z<T, L, ZT>(reg, th, row, vr, n1, mask, z, lds + h * (L / 2));
    __syncthreads();
  } else {
    const bool act = tid < S::TPD;
    T* region = reinterpret_cast<T*>(lds + L / 2);
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      // opaque copy of the thread index: nothing per point (slots, addresses) is
      // hoisted out of the loop, where it would stay live across the whole
      // transform (the pointers stay plain: an opaque pointer loses its global
      // address space, and flat loads wait on LDS traffic too)
      int th = tid;
      asm volatile("" : "+v"(th));
      const bool g = th < S::NG;
      const int r = act ? th / S::TS : 0, tau = th % S::TS;
      const int row = ra + h;
      const bool vr = row < n2;
      cpx<T> reg[16];
      const cpx<T> w1 = twL[g ? th : 0];
      Roots<T, typename S::Fs> rs;
      rs.load_inv(tau, twS);
      if (act) sd_load_spectrum<T, L>(reg, P, row, vr, r, tau, n2, msl);
      sd_inverse<T, L, 1, TWs, true>(reg, g, th, r, tau, w1, rs, region, act);
      // (sd_inverse ends with a barrier: row b's staged z may replace the region)
      if (g) sd_store_z<T, L, ZT>(reg, th, row, vr, n1, mask, z, lds + h * (L / 2));
    }
    __syncthreads();
  }
  // ---- the convolution of z_a + i z_b
  const bool act = tid < F::TPF;
  const int tc = act ? tid : 0;
  Roots<double, F> rcf, rci;  // both sweeps' roots, loaded up front
  rcf.load_fwd(tc, tw64);
  rci.load_inv(tc, tw64);
  cpx<double> reg[F::PP];
  static_for<F::PP>([&](auto ee) {
    constexpr int e = decltype(ee)::value;
    if constexpr (M::upper(e)) {
      reg[e] = {0.0, 0.0};
    } else {
      const int p = F::pos(0, tc, e);
      const bool in = act && p >= 1 && p <= n1;
      reg[e].re = (va && in) ? lds[p - 1] : 0.0;
      reg[e].im = (vb && in) ? lds[L / 2 + p - 1] : 0.0;
    }
  });
  __syncthreads();  // the convolution's region overlays the staged z
  fft_forward_r<double, F>(reg, tc, rcf, lds, act);
  if (act) {
    static_for<F::PP>([&](auto ee) {
      constexpr int e = decltype(ee)::value;
      const double sc = sym[F::pos(F::NS - 1, tc, e)] * coef;
      reg[e].re *= sc;
      reg[e].im *= sc;
    });
  }
  fft_inverse_r<double, F>(reg, tc, rci, lds, act);
  if (!act) return;
  // Epilogue in groups of G registers: the group's loads (clamped addresses)
  // all in flight at once, then its stores.
  const int hp = (n2 + 1) >> 1;
  const size_t ia0 = (size_t)(va ? ra : 0) * n1, ib0 = (size_t)(vb ? rb : 0) * n1;
  constexpr int G = 4;
  static_for<F::PP / G>([&](auto gg) {
    constexpr int g0 = decltype(gg)::value * G;
    static_assert(M::upper(g0) == M::upper(g0 + G - 1), "register group straddles L/2");
    if constexpr (!M::upper(g0)) {
      double za[G], zb[G], sa[G], sb[G];
      uint8_t ma[G], mb2[G];
      static_for<G>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        const int p = F::pos(0, tc, g0 + k);
        const int pp = (p >= 1 && p <= n1) ? p - 1 : 0;
        ma[k] = mask[ia0 + pp];
        mb2[k] = mask[ib0 + pp];
        za[k] = (double)z[ia0 + pp];
        zb[k] = (double)z[ib0 + pp];
        sa[k] = sub ? sub[ia0 + pp] : 0.0;
        sb[k] = sub ? sub[ib0 + pp] : 0.0;
      });
      static_for<G>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        const int p = F::pos(0, tc, g0 + k);
        if (p >= 1 && p <= n1) {
          if (va)
            t[tile_index(ra, p - 1, hp)] = reg[g0 + k].re +
                (1.0 + dpen * (double)(1 - ma[k])) * za[k] - theta * sa[k];
          if (vb)
            t[tile_index(rb, p - 1, hp)] = reg[g0 + k].im +
                (1.0 + dpen * (double)(1 - mb2[k])) * zb[k] - theta * sb[k];
        }
      });
    }
  });
}

}  // namespace rsfde
