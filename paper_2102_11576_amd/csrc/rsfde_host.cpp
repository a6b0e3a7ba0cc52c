// Host side of librsfde: plan construction (coefficients, symbols, eigenvalue
// tables), the restarted flexible GMRES driver and the C ABI of rsfde.h.
//
// Set-up follows Section 2 (grid, Grunwald-Letnikov weights (g_form), the
// Toeplitz first column of (G), c_x = dt kx c_alpha / h_x^alpha) and Section 4.1
// (tau-matrix eigenvalues from the first column).  Everything is computed once
// in FP64 on the host, with exact argument reduction of the cosines, and
// uploaded as O(n) tables; kx and ky enter only as scalars at apply time.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <new>
#include <thread>
#include <vector>

#include "../../include/rsfde.h"
#include "internal.hpp"
#include "tables.hpp"
#include "sd_engine.hpp"

namespace rsfde {

namespace {

using namespace tables;


struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

#define CK(expr)                                   \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return RSFDE_EHIP;       \
  } while (0)


}  // namespace

struct Plan {
  int dev = 0;
  hipStream_t s0 = nullptr;
  int n1 = 0, n2 = 0;
  size_t N = 0, ldv = 0;
  double alpha1 = 0, alpha2 = 0, kx = 0, ky = 0, eta = 0, dt = 0, dpen = 0;
  int Lcx = 0, Lcy = 0, Ldx = 0, Ldy = 0;
  int Lgx = 0, Lgy = 0;  // chirp-DST convolution lengths (0: power-of-two path)
  int max_restart = 0;
  // three-dimensional plans (rsfde_setup3), arrays [n3][n2][n1]; n3 may be 1
  // (A_z is then the 1 x 1 matrix c_z 2 g_1, not absent)
  bool is3d = false;
  int n3 = 1;
  double alpha3 = 0, kz = 0;
  int Lcz = 0, Ldz = 0;
  int Lgz = 0;               // chirp form (some n + 1 not a power of two): z length
  void* chz[2] = {nullptr, nullptr};
  void* khz[2] = {nullptr, nullptr};
  double* symz = nullptr;
  double* lamz64 = nullptr;  // z eigenvalues (unit kz), register-position order of Ldz
  float* lamz32 = nullptr;
  double* lamc64 = nullptr;  // kx lx(slot) + ky ly(j) for the column j * (n1+1) + slot
  float* lamc32 = nullptr;
  std::vector<double> lx3, ly3;  // unit-k x (slot order; natural in the chirp form) and y
                                 // eigenvalues, for new kx, ky
  void* R3 = nullptr;        // preconditioner intermediate (y-transformed)
  double* t3 = nullptr;      // matrix-vector intermediate (after the y pass)

  uint8_t* mask = nullptr;
  double* V = nullptr;
  double* Z = nullptr;
  double* b = nullptr;
  double* w = nullptr;
  double* t = nullptr;
  double* mu = nullptr;
  double* pb = nullptr;  // P_hat^{-1} b (left preconditioning)
  void* Q = nullptr;
  void* P1 = nullptr;
  void* P2 = nullptr;
  double* symx = nullptr;
  double* symy = nullptr;
  double* lamx64 = nullptr;
  double* lamy64 = nullptr;
  float* lamx32 = nullptr;
  float* lamy32 = nullptr;
  // symmetric sine transform (two-dimensional passes, L >= kSdMinL): used along
  // x / y, and the mirror slots of the x transform
  bool sdx = false, sdy = false;
  int32_t* msl = nullptr;
  // chirp-form preconditioner (n + 1 not a power of two)
  double* lamx_n = nullptr;  // tau eigenvalues, natural order, unit k
  double* lamy_n = nullptr;
  void* chx[2] = {nullptr, nullptr};  // [0] FP64, [1] FP32 tables
  void* khx[2] = {nullptr, nullptr};
  void* chy[2] = {nullptr, nullptr};
  void* khy[2] = {nullptr, nullptr};
  std::map<int, void*> tw64, tw32;
  // BF16 / MFMA preconditioner
  int n1p = 0, n2p = 0;
  __bf16* Sx16 = nullptr;
  __bf16* Sy16 = nullptr;
  __bf16* Sx16lo = nullptr;  // S - bf16(S), for the split forward products
  __bf16* Sy16lo = nullptr;
  float* lamx_nat = nullptr;
  float* lamy_nat = nullptr;
  __bf16* A1T = nullptr;
  __bf16* R12T = nullptr;
  __bf16* G = nullptr;
  KrylovState* ks = nullptr;
  RedWork rw{nullptr};
  // s-step blocks: Gram partials, Gram result (pinned, device-visible), update
  // coefficients (device) and their pinned staging copy
  double* gpart = nullptr;
  double* gram_h = nullptr;
  double* gram_d = nullptr;
  double* coef_d = nullptr;
  double* coef_h = nullptr;
  int32_t gram_seq = 0;  // last sequence number handed to a Gram block
  HostStatus* hs = nullptr;      // pinned host memory
  HostStatus* hs_dev = nullptr;  // its device-visible address
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::vector<void*> allocs;

  // kernel timing (rsfde_profile)
  struct ProfRec {
    int cat;
    hipEvent_t a, b;
    double bytes;
  };
  bool prof_on = false;
  bool trace = false;  // RSFDE_TRACE=1: s-step block diagnostics on stderr
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> ev_pool;
  hipEvent_t take_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }

  ~Plan() {
    for (void* p : allocs) (void)hipFree(p);
    if (hs) (void)hipHostFree(hs);
    if (gram_h) (void)hipHostFree(gram_h);
    if (coef_h) (void)hipHostFree(coef_h);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& r : prof_recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
  }

  template <typename T>
  hipError_t dalloc(T** p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, count * sizeof(T) > 0 ? count * sizeof(T) : 16);
    if (e != hipSuccess) return e;
    allocs.push_back(q);
    *p = (T*)q;
    return hipSuccess;
  }
};

namespace {

hipStream_t pick(Plan* P, void* s) { return s ? (hipStream_t)s : P->s0; }

enum ProfCat {
  kCatMvRows, kCatMvCols, kCatPcRows, kCatPcCols, kCatPcRowsInv, kCatMultidot, kCatAxpy,
  kCatUpdate, kCatResidual, kCatRhs, kCatOther, kCatPcGemm, kCatCdRows, kCatCdCols,
  kCatCdRowsInv, kCatGram, kCatBupd, kCatPcInvMv, kCatDstCols, kNumCats
};
const char* const kCatNames[kNumCats] = {"mv_rows", "mv_cols", "pc_rows_fwd", "pc_cols",
                                         "pc_rows_inv", "multidot", "axpy_givens", "update",
                                         "residual", "rhs", "other", "pc_gemm_bf16",
                                         "cd_rows_fwd", "cd_cols", "cd_rows_inv", "block_gram",
                                         "block_update", "pc_inv_mv_rows", "dst_cols"};

// Brackets one kernel launch with timing events when profiling is on.
struct ProfScope {
  Plan* P;
  hipStream_t s;
  int cat;
  double bytes;
  hipEvent_t a = nullptr;
  ProfScope(Plan* P_, hipStream_t s_, int cat_, double bytes_) : P(P_), s(s_), cat(cat_), bytes(bytes_) {
    if (P->prof_on) {
      a = P->take_event();
      if (a && hipEventRecord(a, s) != hipSuccess) a = nullptr;
    }
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = P->take_event();
    if (b && hipEventRecord(b, s) == hipSuccess) P->prof_recs.push_back({cat, a, b, bytes});
  }
};



// Eigenvalues of tau(T_n) for k = 1..n (index k-1): t_0 + 2 sum_j t_j cos(j k pi/(n+1)).
std::vector<double> tau_eigs(const std::vector<double>& t) {
  const int n = (int)t.size();
  const int L = 2 * (n + 1);
  std::vector<double> ct = cos_table(L), lam(n);
  for (int k = 1; k <= n; ++k) {
    double s = t[0];
    for (int j = 1; j < n; ++j) s += 2.0 * t[j] * ct[(int)(((long long)j * k) % L)];
    lam[k - 1] = s;
  }
  return lam;
}


// In-place forward DFT X_f = sum_p a_p exp(-2 pi i p f / L), L a power of two
// (iterative radix-2 with the symmetric twiddle table).
void fft_host(std::vector<std::complex<double>>& a) {
  const int L = (int)a.size();
  for (int i = 1, j = 0; i < L; ++i) {
    int bit = L >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  const std::vector<double> tw = twiddles<double>(L);
  for (int len = 2; len <= L; len <<= 1) {
    const int step = L / len;
    for (int i = 0; i < L; i += len)
      for (int k = 0; k < len / 2; ++k) {
        const std::complex<double> w(tw[2 * (size_t)(k * step)], tw[2 * (size_t)(k * step) + 1]);
        const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
  }
}

// Tables of the chirp form of the length-n orthonormal DST-I (M = n + 1):
//   chn[p]  = exp(i pi (p+1)^2 / (2M)), p < n (interleaved re, im);
//   khat[p] = sqrt(2/M) / L * K_f at f = freq(p), K = DFT_L of the even kernel
//             k[m mod L] = exp(-i pi m^2 / (2M)), |m| < n.
// Phases are reduced exactly: m^2 mod 4M in integers.
void chirp_tables(int n, int L, std::vector<double>& chn, std::vector<double>& khat) {
  const long long M4 = 4LL * (n + 1);
  auto ang = [&](long long j) {
    return kPi * (double)((j * j) % M4) / (2.0 * (double)(n + 1));
  };
  chn.assign(2 * (size_t)n, 0.0);
  for (int p = 0; p < n; ++p) {
    const double a = ang(p + 1);
    chn[2 * (size_t)p] = std::cos(a);
    chn[2 * (size_t)p + 1] = std::sin(a);
  }
  std::vector<std::complex<double>> k(L, {0.0, 0.0});
  for (int m = 0; m < n; ++m) {
    const double a = ang(m);
    const std::complex<double> c(std::cos(a), -std::sin(a));
    k[m] = c;
    if (m) k[L - m] = c;
  }
  fft_host(k);
  const double sc = std::sqrt(2.0 / (n + 1)) / (double)L;
  const int P = fft_pts(L);
  khat.assign(2 * (size_t)L, 0.0);
  for (int p = 0; p < L; ++p) {
    const std::complex<double> v = k[fft_freq(L, P, p)] * sc;
    khat[2 * (size_t)p] = v.real();
    khat[2 * (size_t)p + 1] = v.imag();
  }
}

// float -> bf16, round to nearest even (finite inputs).
uint16_t to_bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

float from_bf16_bits(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Orthonormal DST-I matrix sqrt(2/(n+1)) sin(pi (i+1)(j+1)/(n+1)) (Section 4.1),
// zero-padded to np x np, as BF16 bit patterns: hi = bf16(S), lo = bf16(S - hi).
void sine_matrix_bf16(int n, int np, std::vector<uint16_t>& hi, std::vector<uint16_t>& lo) {
  const int L = 2 * (n + 1);
  std::vector<double> sn(L);
  for (int m = 0; m < L; ++m) sn[m] = std::sin(kPi * (double)m / (double)(n + 1));
  const double c = std::sqrt(2.0 / (n + 1));
  hi.assign((size_t)np * np, 0);
  lo.assign((size_t)np * np, 0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double v = c * sn[(int)(((long long)(i + 1) * (j + 1)) % L)];
      const uint16_t h = to_bf16_bits((float)v);
      hi[(size_t)i * np + j] = h;
      lo[(size_t)i * np + j] = to_bf16_bits((float)(v - (double)from_bf16_bits(h)));
    }
}

template <typename T>
hipError_t upload(Plan* P, T** dst, const std::vector<T>& src, hipStream_t s) {
  hipError_t e = P->dalloc(dst, src.size());
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

hipError_t ensure_twiddles(Plan* P, int L, hipStream_t s) {
  if (L <= 0 || P->tw64.count(L)) return hipSuccess;
  double* d = nullptr;
  float* f = nullptr;
  hipError_t e = upload(P, &d, twiddles<double>(L), s);
  if (e != hipSuccess) return e;
  e = upload(P, &f, twiddles<float>(L), s);
  if (e != hipSuccess) return e;
  P->tw64[L] = d;
  P->tw32[L] = f;
  return hipSuccess;
}

// Section 4.1's x and y eigenvalues of a 3-D plan folded into one value per
// column of the [n3][ld n2] view: kx lx(slot) + ky ly(j), column j ld + slot,
// ld = n1 + 1 slots (odd-extension form) or n1 natural positions (chirp form).
std::vector<double> fold_xy3(const Plan* P) {
  const size_t ld = (size_t)P->n1 + (P->Lgx ? 0 : 1);
  std::vector<double> lamc(ld * (size_t)P->n2);
  for (int j = 0; j < P->n2; ++j)
    for (size_t c = 0; c < ld; ++c) lamc[(size_t)j * ld + c] = P->kx * P->lx3[c] + P->ky * P->ly3[j];
  return lamc;
}

// The y and z passes of the three-dimensional product: t3 = t - ky (A_y along
// y) x slice by slice, then y = t3 - kz (A_z along z) x on the [n3][n1*n2] view.
int matvec_cols3(Plan* P, const double* x, double* y, hipStream_t s) {
  const double N = (double)P->N;
  const int plane = P->n1 * P->n2;
  {
    ProfScope ps(P, s, kCatMvCols, 24.0 * N);
    CK(launch_mv_cols(P->Lcy, x, P->t, P->t3, P->symy, P->tw64[P->Lcy], P->n1, P->n2, -P->ky, 0, s,
                      P->n3, (size_t)plane));
  }
  {
    ProfScope ps(P, s, kCatMvCols, 24.0 * N);
    CK(launch_mv_cols(P->Lcz, x, P->t3, y, P->symz, P->tw64[P->Lcz], plane, P->n3, -P->kz, 0, s));
  }
  return RSFDE_OK;
}

// y = M x - theta * sub (sub = NULL: y = M x).
int matvec_impl(Plan* P, const double* x, double* y, hipStream_t s, const double* sub = nullptr,
                double theta = 0.0) {
  const double N = (double)P->N;
  if (P->is3d) {
    const int rows = P->n2 * P->n3;
    {
      ProfScope ps(P, s, kCatMvRows, (sub ? 25.0 : 17.0) * N);
      CK(launch_mv_rows(P->Lcx, x, P->mask, P->t, P->symx, P->tw64[P->Lcx], P->n1, rows, -P->kx,
                        P->dpen, 0, s, sub, theta));
    }
    return matvec_cols3(P, x, y, s);
  }
  {  // t strip-tiled (two-dimensional plans)
    ProfScope ps(P, s, kCatMvRows, (sub ? 25.0 : 17.0) * N);
    CK(launch_mv_rows(P->Lcx, x, P->mask, P->t, P->symx, P->tw64[P->Lcx], P->n1, P->n2, -P->kx,
                      P->dpen, 0, s, sub, theta, true));
  }
  {
    ProfScope ps(P, s, kCatMvCols, 24.0 * N);
    CK(launch_mv_cols(P->Lcy, x, P->t, y, P->symy, P->tw64[P->Lcy], P->n1, P->n2, -P->ky, 0, s, 1,
                      0, true));
  }
  return RSFDE_OK;
}

// Chirp-form P_hat^{-1} (any n): three passes with T internals.
template <typename T>
int precond_chirp(Plan* P, const double* r, const double* sig, double* z, int t,
                  std::map<int, void*>& tw, hipStream_t s) {
  const double N = (double)P->N, ts = (double)sizeof(T);
  T *W = (T*)P->Q, *Y1 = (T*)P->P1, *Y2 = (T*)P->P2;
  {
    ProfScope ps(P, s, kCatCdRows, 8.0 * N + ts * N);
    CK(launch_cd_rows_fwd<T>(P->Lgx, r, sig, W, P->chx[t], P->khx[t], tw[P->Lgx], P->n1, P->n2,
                             s));
  }
  {
    ProfScope ps(P, s, kCatCdCols, 3.0 * ts * N);
    CK(launch_cd_cols<T>(P->Lgy, W, Y1, Y2, P->lamx_n, P->lamy_n, P->chy[t], P->khy[t],
                         tw[P->Lgy], P->n1, P->n2, P->kx, P->ky, P->dpen, s));
  }
  {
    ProfScope ps(P, s, kCatCdRowsInv, 2.0 * ts * N + 9.0 * N);
    CK(launch_cd_rows_inv<T>(P->Lgx, Y1, Y2, P->mask, z, P->chx[t], P->khx[t], tw[P->Lgx], P->n1,
                             P->n2, s));
  }
  return RSFDE_OK;
}

// Three-dimensional P_hat^{-1} in the chirp form (some n + 1 not a power of
// two), T internals; S is the orthonormal DST-I along an axis, S S = I:
//   A:  W1 = S_x (sig v)                                 (all n2 n3 rows)
//   B1: W2 = S_y W1                                      (columns of each z slice)
//   B2: Y1 = S_z (S_z W2 / E1), Y2 = S_z (S_z W2 / E2)   (columns of the [n3][n1 n2]
//       view; E1 = 1 - (kx lx + ky ly) - kz lz, E2 = E1 + dt/eta)
//   B3: W1 = S_y Y1, W2 = S_y Y2                         (per z slice)
//   C:  z  = S_x W1 where mask = 1, S_x W2 where mask = 0  (all rows)
template <typename T>
int precond3_chirp(Plan* P, const double* r, const double* sig, double* z, int t,
                   std::map<int, void*>& tw, hipStream_t s) {
  const int n1 = P->n1, n2 = P->n2, n3 = P->n3, rows = n2 * n3, plane = n1 * n2;
  const double N = (double)P->N, ts = (double)sizeof(T);
  T *W1 = (T*)P->Q, *W2 = (T*)P->R3, *Y1 = (T*)P->P1, *Y2 = (T*)P->P2;
  {
    ProfScope ps(P, s, kCatCdRows, 8.0 * N + ts * N);
    CK(launch_cd_rows_fwd<T>(P->Lgx, r, sig, W1, P->chx[t], P->khx[t], tw[P->Lgx], n1, rows, s));
  }
  {
    ProfScope ps(P, s, kCatCdCols, 2.0 * ts * N);
    CK(launch_cd_dst_cols<T>(P->Lgy, W1, W2, nullptr, nullptr, P->chy[t], P->khy[t], tw[P->Lgy], n1,
                             n2, n3, (size_t)plane, s));
  }
  {
    ProfScope ps(P, s, kCatCdCols, 3.0 * ts * N);
    CK(launch_cd_cols<T>(P->Lgz, W2, Y1, Y2, P->lamc64, P->lamz64, P->chz[t], P->khz[t],
                         tw[P->Lgz], plane, n3, 1.0, P->kz, P->dpen, s));
  }
  {
    ProfScope ps(P, s, kCatCdCols, 4.0 * ts * N);
    CK(launch_cd_dst_cols<T>(P->Lgy, Y1, W1, Y2, W2, P->chy[t], P->khy[t], tw[P->Lgy], n1, n2, n3,
                             (size_t)plane, s));
  }
  {
    ProfScope ps(P, s, kCatCdRowsInv, 2.0 * ts * N + 9.0 * N);
    CK(launch_cd_rows_inv<T>(P->Lgx, W1, W2, P->mask, z, P->chx[t], P->khx[t], tw[P->Lgx], n1,
                             rows, s));
  }
  return RSFDE_OK;
}

// Three-dimensional P_hat^{-1} (n + 1 a power of two on every axis), T internals:
//   A:  Q  = raw x-sine sums of the rows of sig*v            (all n2*n3 rows)
//   B1: R  = raw y-sine sums of Q's columns                   (per z slice)
//   B2: P1, P2 = raw z-sine sums of K R / E1 and K R / E2     (columns of the
//       [n3][(n1+1) n2] view; E1 = 1 - kx lx - ky ly - kz lz, E2 = E1 + dt/eta)
//   B3: Q, R = raw y-sine sums of P1, P2                      (per z slice)
//   C:  z  = mask (Q S_x) + (1 - mask) (R S_x), fused with the matrix-vector row
//       pass when w is given (then followed by the y and z passes into w).
// K = 8 / ((n1+1)(n2+1)(n3+1)) collects the orthonormal sine factors.
template <typename T>
int precond3(Plan* P, const double* r, const double* sig, double* z, std::map<int, void*>& tw,
             const T* lamc, const T* lamz, hipStream_t s, double* w, const double* sub,
             double theta) {
  if (P->Lgx) {  // chirp form, then the product unfused
    const int rc = precond3_chirp<T>(P, r, sig, z, sizeof(T) == 8 ? 0 : 1, tw, s);
    if (rc != RSFDE_OK || !w) return rc;
    return matvec_impl(P, z, w, s, sub, theta);
  }
  const int n1 = P->n1, n2 = P->n2, n3 = P->n3, ld = n1 + 1, rows = n2 * n3;
  const size_t plane = (size_t)ld * n2;
  const double Kfac = 8.0 / ((double)(n1 + 1) * (double)(n2 + 1) * (double)(n3 + 1));
  const double N = (double)P->N, S = (double)plane * n3, ts = (double)sizeof(T);
  T *Q = (T*)P->Q, *R = (T*)P->R3, *P1 = (T*)P->P1, *P2 = (T*)P->P2;
  {
    ProfScope ps(P, s, kCatPcRows, 8.0 * N + ts * S);
    CK(launch_pc_rows_fwd<T>(P->Ldx, r, sig, Q, tw[P->Ldx], n1, rows, false, s));
  }
  {
    ProfScope ps(P, s, kCatDstCols, 2.0 * ts * S);
    CK(launch_dst_cols<T>(P->Ldy, Q, Q, R, R, tw[P->Ldy], ld / 2, 2, 1, n2, ld, n3, plane, s));
  }
  {
    ProfScope ps(P, s, kCatPcCols, 3.0 * ts * S);
    CK(launch_pc_cols<T>(P->Ldz, R, P1, P2, lamc, lamz, tw[P->Ldz], (int)plane - 1, n3, 1.0, P->kz,
                         P->dpen, Kfac, false, s));
  }
  {
    ProfScope ps(P, s, kCatDstCols, 4.0 * ts * S);
    CK(launch_dst_cols<T>(P->Ldy, P1, P2, Q, R, tw[P->Ldy], ld, 1, 0, n2, ld, n3, plane, s));
  }
  if (!w || P->Ldx != P->Lcx) {  // unfused (n1 = 1: convolution and sine lengths differ)
    {
      ProfScope ps(P, s, kCatPcRowsInv, 2.0 * ts * S + 9.0 * N);
      CK(launch_pc_rows_inv<T>(P->Ldx, Q, R, P->mask, z, tw[P->Ldx], n1, rows, false, s));
    }
    return w ? matvec_impl(P, z, w, s, sub, theta) : RSFDE_OK;
  }
  {
    ProfScope ps(P, s, kCatPcInvMv, 2.0 * ts * S + 17.0 * N + (sub ? 8.0 * N : 0.0));
    CK(launch_pc_rows_inv_mv<T>(P->Ldx, Q, R, P->mask, z, P->t, tw[P->Ldx],
                                P->tw64[P->Ldx], P->symx, -P->kx, P->dpen, sub, theta, n1, rows,
                                false, s));
  }
  return matvec_cols3(P, z, w, s);
}

// Symmetric-transform tables of the x (rows) and y (columns) passes in the
// precision of T (empty where the plain FFT form is used).
template <typename T>
SdTabs sd_x(Plan* P) {
  SdTabs t;
  if (P->sdx) {
    t.twS = (sizeof(T) == 8 ? P->tw64 : P->tw32)[P->Ldx / 16];
    t.msl = P->msl;
  }
  return t;
}
template <typename T>
SdTabs sd_y(Plan* P) {
  SdTabs t;
  if (P->sdy) t.twS = (sizeof(T) == 8 ? P->tw64 : P->tw32)[P->Ldy / 16];
  return t;
}

int precond_impl(Plan* P, const double* r, const double* sig, double* z, int precision,
                 hipStream_t s) {
  if (P->is3d) {
    if (precision == RSFDE_FP64)
      return precond3<double>(P, r, sig, z, P->tw64, P->lamc64, P->lamz64, s, nullptr, nullptr, 0.0);
    if (precision == RSFDE_FP32)
      return precond3<float>(P, r, sig, z, P->tw32, P->lamc32, P->lamz32, s, nullptr, nullptr, 0.0);
    return RSFDE_EUNSUPPORTED;
  }
  if (precision == RSFDE_BF16) {
    ProfScope ps(P, s, kCatPcGemm, 17.0 * (double)P->N);
    CK(launch_pc_gemm_bf16(r, sig, z, P->mask, P->Sx16, P->Sy16, P->Sx16lo, P->Sy16lo, P->lamx_nat,
                           P->lamy_nat, P->A1T,
                           P->R12T, P->G, P->n1, P->n2, P->n1p, P->n2p, P->kx, P->ky, P->dpen, s));
    return RSFDE_OK;
  }
  if (P->Lgx) {
    if (precision == RSFDE_FP64) return precond_chirp<double>(P, r, sig, z, 0, P->tw64, s);
    if (precision == RSFDE_FP32) return precond_chirp<float>(P, r, sig, z, 1, P->tw32, s);
    return RSFDE_EUNSUPPORTED;
  }
  const double Kfac = 4.0 / ((double)(P->n1 + 1) * (double)(P->n2 + 1));
  const double N = (double)P->N, S = (double)(P->n1 + 1) * (double)P->n2;
  if (precision == RSFDE_FP64) {
    double *Q = (double*)P->Q, *P1 = (double*)P->P1, *P2 = (double*)P->P2;
    {
      ProfScope ps(P, s, kCatPcRows, 8.0 * N + 8.0 * S);
      CK(launch_pc_rows_fwd<double>(P->Ldx, r, sig, Q, P->tw64[P->Ldx], P->n1, P->n2, true, s,
                                    Members::one(), sd_x<double>(P)));
    }
    {
      ProfScope ps(P, s, kCatPcCols, 24.0 * S);
      CK(launch_pc_cols<double>(P->Ldy, Q, P1, P2, P->lamx64, P->lamy64, P->tw64[P->Ldy], P->n1,
                                P->n2, P->kx, P->ky, P->dpen, Kfac, true, s, Members::one(),
                                nullptr, sd_y<double>(P)));
    }
    {
      ProfScope ps(P, s, kCatPcRowsInv, 16.0 * S + 9.0 * N);
      CK(launch_pc_rows_inv<double>(P->Ldx, P1, P2, P->mask, z, P->tw64[P->Ldx],
                                    P->n1, P->n2, true, s, Members::one(), sd_x<double>(P)));
    }
    return RSFDE_OK;
  }
  if (precision == RSFDE_FP32) {
    float *Q = (float*)P->Q, *P1 = (float*)P->P1, *P2 = (float*)P->P2;
    {
      ProfScope ps(P, s, kCatPcRows, 8.0 * N + 4.0 * S);
      CK(launch_pc_rows_fwd<float>(P->Ldx, r, sig, Q, P->tw32[P->Ldx], P->n1, P->n2, true, s,
                                   Members::one(), sd_x<float>(P)));
    }
    {
      ProfScope ps(P, s, kCatPcCols, 12.0 * S);
      CK(launch_pc_cols<float>(P->Ldy, Q, P1, P2, P->lamx32, P->lamy32, P->tw32[P->Ldy], P->n1,
                               P->n2, P->kx, P->ky, P->dpen, Kfac, true, s, Members::one(),
                               nullptr, sd_y<float>(P)));
    }
    {
      ProfScope ps(P, s, kCatPcRowsInv, 8.0 * S + 9.0 * N);
      CK(launch_pc_rows_inv<float>(P->Ldx, P1, P2, P->mask, z, P->tw32[P->Ldx],
                                   P->n1, P->n2, true, s, Members::one(), sd_x<float>(P)));
    }
    return RSFDE_OK;
  }
  return RSFDE_EUNSUPPORTED;
}

// w = M P_hat^{-1} (sig v) - theta sub, z = P_hat^{-1} (sig v) (stored): the
// preconditioner's last pass and the matrix-vector row pass run as one kernel
// when n1 + 1 and n2 + 1 are powers of two (FP64 / FP32 internals); otherwise
// the two operators run one after the other.
int precond_matvec_impl(Plan* P, const double* v, const double* sig, void* zv, double* w,
                        int precision, hipStream_t s, const double* sub = nullptr,
                        double theta = 0.0, bool z32 = false) {
  double* z = (double*)zv;  // a float array when z32 (fused two-dimensional path only)
  if (P->is3d) {
    if (precision == RSFDE_FP64)
      return precond3<double>(P, v, sig, z, P->tw64, P->lamc64, P->lamz64, s, w, sub, theta);
    if (precision == RSFDE_FP32)
      return precond3<float>(P, v, sig, z, P->tw32, P->lamc32, P->lamz32, s, w, sub, theta);
    return RSFDE_EUNSUPPORTED;
  }
  const bool fused = P->Ldx && P->Ldy && P->Ldx == P->Lcx &&
                     (precision == RSFDE_FP64 || precision == RSFDE_FP32);
  if (z32 && !fused) return RSFDE_EUNSUPPORTED;
  if (!fused) {
    int rc = precond_impl(P, v, sig, z, precision, s);
    if (rc) return rc;
    return matvec_impl(P, z, w, s, sub, theta);
  }
  const double Kfac = 4.0 / ((double)(P->n1 + 1) * (double)(P->n2 + 1));
  const double N = (double)P->N, S = (double)(P->n1 + 1) * (double)P->n2;
  const double extra = (sub ? 8.0 * N : 0.0) - (z32 ? 4.0 * N : 0.0);
  if (precision == RSFDE_FP64) {
    double *Q = (double*)P->Q, *P1 = (double*)P->P1, *P2 = (double*)P->P2;
    {
      ProfScope ps(P, s, kCatPcRows, 8.0 * N + 8.0 * S);
      CK(launch_pc_rows_fwd<double>(P->Ldx, v, sig, Q, P->tw64[P->Ldx], P->n1, P->n2, true, s,
                                    Members::one(), sd_x<double>(P)));
    }
    {
      ProfScope ps(P, s, kCatPcCols, 24.0 * S);
      CK(launch_pc_cols<double>(P->Ldy, Q, P1, P2, P->lamx64, P->lamy64, P->tw64[P->Ldy], P->n1,
                                P->n2, P->kx, P->ky, P->dpen, Kfac, true, s, Members::one(),
                                nullptr, sd_y<double>(P)));
    }
    {
      ProfScope ps(P, s, kCatPcInvMv, 16.0 * S + 17.0 * N + extra);
      CK(launch_pc_rows_inv_mv<double>(P->Ldx, P1, P2, P->mask, z, P->t,
                                       P->tw64[P->Ldx], P->tw64[P->Ldx], P->symx, -P->kx, P->dpen,
                                       sub, theta, P->n1, P->n2, true, s, Members::one(), nullptr,
                                       z32, sd_x<double>(P)));
    }
  } else {
    float *Q = (float*)P->Q, *P1 = (float*)P->P1, *P2 = (float*)P->P2;
    {
      ProfScope ps(P, s, kCatPcRows, 8.0 * N + 4.0 * S);
      CK(launch_pc_rows_fwd<float>(P->Ldx, v, sig, Q, P->tw32[P->Ldx], P->n1, P->n2, true, s,
                                   Members::one(), sd_x<float>(P)));
    }
    {
      ProfScope ps(P, s, kCatPcCols, 12.0 * S);
      CK(launch_pc_cols<float>(P->Ldy, Q, P1, P2, P->lamx32, P->lamy32, P->tw32[P->Ldy], P->n1,
                               P->n2, P->kx, P->ky, P->dpen, Kfac, true, s, Members::one(),
                               nullptr, sd_y<float>(P)));
    }
    {
      ProfScope ps(P, s, kCatPcInvMv, 8.0 * S + 17.0 * N + extra);
      CK(launch_pc_rows_inv_mv<float>(P->Ldx, P1, P2, P->mask, z, P->t,
                                      P->tw32[P->Ldx], P->tw64[P->Ldx], P->symx, -P->kx, P->dpen,
                                      sub, theta, P->n1, P->n2, true, s, Members::one(), nullptr,
                                      z32, sd_x<float>(P)));
    }
  }
  {
    ProfScope ps(P, s, kCatMvCols, (z32 ? 20.0 : 24.0) * N);
    CK(launch_mv_cols(P->Lcy, z, P->t, w, P->symy, P->tw64[P->Lcy], P->n1, P->n2, -P->ky, 0, s, 1,
                      0, true, Members::one(), nullptr, z32));
  }
  return RSFDE_OK;
}

int validate_opts(Plan* P, const rsfde_solver_opts* o) {
  if (!o) return RSFDE_EINVAL;
  if (P->is3d && o->precision == RSFDE_BF16) return RSFDE_EUNSUPPORTED;
  if (o->restart < 1 || o->restart > P->max_restart) return RSFDE_EINVAL;
  if (o->max_iters < 1) return RSFDE_EINVAL;
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return RSFDE_EINVAL;
  if (o->precond != RSFDE_PRECOND_TAU && o->precond != RSFDE_PRECOND_NONE) return RSFDE_EINVAL;
  if (o->precision < RSFDE_FP64 || o->precision > RSFDE_BF16) return RSFDE_EINVAL;
  if (o->reorth < -1 || o->reorth > 1) return RSFDE_EINVAL;
  if (o->side != RSFDE_RIGHT && o->side != RSFDE_LEFT) return RSFDE_EINVAL;
  if (o->sstep < 0 || o->sstep > 16) return RSFDE_EINVAL;
  if (o->zstore != RSFDE_ZSTORE_FP64 && o->zstore != RSFDE_ZSTORE_FP32) return RSFDE_EINVAL;
  if (o->zstore == RSFDE_ZSTORE_FP32) {
    // the preconditioned basis in FP32: the fused two-dimensional path only
    const bool fused = !P->is3d && P->Ldx && P->Ldy && P->Ldx == P->Lcx;
    if (!fused || o->precond != RSFDE_PRECOND_TAU || o->side != RSFDE_RIGHT ||
        o->precision == RSFDE_BF16)
      return RSFDE_EUNSUPPORTED;
  }
  if (o->sstep >= 2) {
    if (o->precond != RSFDE_PRECOND_TAU || o->side != RSFDE_RIGHT) return RSFDE_EUNSUPPORTED;
    if (o->restart + 1 + o->sstep > 16 * kGramMaxTiles) return RSFDE_EUNSUPPORTED;
  }
  (void)P;
  return RSFDE_OK;
}

double vread(const volatile double* p) { return *p; }
int vread(const volatile int32_t* p) { return *p; }

int finish(rsfde_stats* st, int code, int iters, int restarts, double beta, double bnorm) {
  if (st) {
    st->iters = iters;
    st->restarts = restarts;
    st->status = code;
    st->reserved = 0;
    st->relres = bnorm > 0.0 ? beta / bnorm : 0.0;
    st->bnorm = bnorm;
  }
  return code;
}

// Restarted GMRES on M x = P->b (||b|| already in hs->bnorm); x holds the
// initial guess and receives the solution.
//  right (default): flexible GMRES, z_j = P_hat^{-1} v_j stored per step,
//    x += Z y; every cycle restarts from the true residual b - M x and the
//    solve stops when ||b - M x|| <= tol ||b||.
//  left (the convention of the experiments of Section 5): Arnoldi on
//    P_hat^{-1} M, x += V y; stops when the residual estimate of
//    ||P_hat^{-1}(b - M x)|| is <= tol ||P_hat^{-1} b||.
int solve_core_sstep(Plan* P, double* x, const rsfde_solver_opts* o, rsfde_stats* st,
                     hipStream_t s);

int solve_core(Plan* P, double* x, const rsfde_solver_opts* o, rsfde_stats* st, hipStream_t s) {
  if (o->sstep >= 2 && P->N >= 4096) return solve_core_sstep(P, x, o, st, s);
  const size_t N = P->N, ld = P->ldv;
  volatile HostStatus* hs = P->hs;
  const bool tau = o->precond == RSFDE_PRECOND_TAU;
  const bool left = tau && o->side == RSFDE_LEFT;
  int rc = RSFDE_OK;
  CK(hipStreamSynchronize(s));
  if (vread(&hs->flags) & kFlagNonFinite) return finish(st, RSFDE_ENONFINITE, 0, 0, 0, 0);
  double bnorm = vread(&hs->bnorm);
  if (bnorm == 0.0) {
    CK(hipMemsetAsync(x, 0, N * sizeof(double), s));
    CK(hipStreamSynchronize(s));
    return finish(st, RSFDE_OK, 0, 0, 0.0, 0.0);
  }
  if (left) {  // reference norm ||P_hat^{-1} b||
    rc = precond_impl(P, P->b, nullptr, P->pb, o->precision, s);
    if (rc) return finish(st, rc, 0, 0, 0, bnorm);
    CK(launch_norm(P->pb, N, P->rw, P->hs_dev, s));
    CK(hipStreamSynchronize(s));
    if (vread(&hs->flags) & kFlagNonFinite) return finish(st, RSFDE_ENONFINITE, 0, 0, 0, 0);
    bnorm = vread(&hs->bnorm);
  }
  const double thresh = o->tol * bnorm;
  // Two Gram-Schmidt passes (CGS2) unless one is requested (reorth = -1):
  // single-pass classical Gram-Schmidt loses orthogonality on long cycles at
  // high stiffness (139 against 116 iterations per step at 2047^2, alpha = 1.9)
  // and with the BF16 preconditioner's rounding.
  const bool reorth = o->reorth >= 0;
  int total = 0, cycles = 0;
  double beta = 0.0;
  for (;;) {
    rc = matvec_impl(P, x, P->w, s);
    if (rc) return finish(st, rc, total, cycles, beta, bnorm);
    if (left) {
      rc = precond_impl(P, P->w, nullptr, P->Z, o->precision, s);
      if (rc) return finish(st, rc, total, cycles, beta, bnorm);
      ProfScope ps(P, s, kCatResidual, 24.0 * N);
      CK(launch_residual(P->pb, P->Z, P->V, N, P->rw, P->ks, P->hs_dev, s));
    } else {
      ProfScope ps(P, s, kCatResidual, 24.0 * N);
      CK(launch_residual(P->b, P->w, P->V, N, P->rw, P->ks, P->hs_dev, s));
    }
    CK(hipStreamSynchronize(s));
    if (vread(&hs->flags) & kFlagNonFinite) return finish(st, RSFDE_ENONFINITE, total, cycles, beta, bnorm);
    beta = vread(&hs->beta);
    if (beta <= thresh) return finish(st, RSFDE_OK, total, cycles, beta, bnorm);
    if (total >= o->max_iters) return finish(st, RSFDE_ENOTCONV, total, cycles, beta, bnorm);
    ++cycles;
    const int jmax = std::min(o->restart, o->max_iters - total);
    int jc = -1;
    for (int j = 0; j < jmax; ++j) {
      double* vj = P->V + (size_t)j * ld;
      double* zj = P->Z + (size_t)j * ld;
      const double* sig = &P->ks->vscale[j];
      const double* wv = P->w;  // the vector Arnoldi orthogonalises
      if (left) {  // w = P_hat^{-1} M v_j
        rc = matvec_impl(P, vj, P->w, s);
        if (rc) return finish(st, rc, total, cycles, beta, bnorm);
        rc = precond_impl(P, P->w, sig, zj, o->precision, s);
        if (rc) return finish(st, rc, total, cycles, beta, bnorm);
        wv = zj;
      } else {  // z_j = P_hat^{-1} v_j, w = M z_j
        if (tau) {
          void* zs = o->zstore == RSFDE_ZSTORE_FP32 ? (void*)((float*)P->Z + (size_t)j * ld)
                                                    : (void*)zj;
          rc = precond_matvec_impl(P, vj, sig, zs, P->w, o->precision, s, nullptr, 0.0,
                                   o->zstore == RSFDE_ZSTORE_FP32);
          if (rc) return finish(st, rc, total, cycles, beta, bnorm);
        } else {
          {
            ProfScope ps(P, s, kCatOther, 16.0 * N);
            CK(launch_scale_copy(vj, sig, zj, N, s));
          }
          rc = matvec_impl(P, zj, P->w, s);
          if (rc) return finish(st, rc, total, cycles, beta, bnorm);
        }
      }
      double* vnext = P->V + (size_t)(j + 1) * ld;
      {
        ProfScope ps(P, s, kCatMultidot, 8.0 * (j + 2) * (double)N);
        CK(launch_multidot(P->V, ld, j + 1, wv, N, P->rw, P->ks, j, false, s));
      }
      {
        ProfScope ps(P, s, kCatAxpy, 8.0 * (j + 3) * (double)N);
        CK(launch_axpy_givens(P->V, ld, j + 1, wv, vnext, N, P->rw, P->ks, j, false, !reorth,
                              P->hs_dev, s));
      }
      if (reorth) {  // classical Gram-Schmidt, second pass
        {
          ProfScope ps(P, s, kCatMultidot, 8.0 * (j + 2) * (double)N);
          CK(launch_multidot(P->V, ld, j + 1, vnext, N, P->rw, P->ks, j, true, s));
        }
        {
          ProfScope ps(P, s, kCatAxpy, 8.0 * (j + 3) * (double)N);
          CK(launch_axpy_givens(P->V, ld, j + 1, vnext, vnext, N, P->rw, P->ks, j, true, true,
                                P->hs_dev, s));
        }
      }
      CK(hipEventRecord(P->ev[j & 1], s));
      // Look one iteration behind: the device runs step j while the host
      // checks step j-1.  A converged j-1 leaves step j's work unused
      // (it writes only column j and vectors j, j+1).
      if (j > 0) {
        CK(hipEventSynchronize(P->ev[(j - 1) & 1]));
        if (vread(&hs->flags) & kFlagNonFinite)
          return finish(st, RSFDE_ENONFINITE, total + j, cycles, beta, bnorm);
        if (vread(&hs->est[j - 1]) <= thresh) {
          jc = j;
          break;
        }
      }
    }
    if (jc < 0) {
      CK(hipEventSynchronize(P->ev[(jmax - 1) & 1]));
      if (vread(&hs->flags) & kFlagNonFinite)
        return finish(st, RSFDE_ENONFINITE, total + jmax, cycles, beta, bnorm);
      jc = jmax;
    }
    const double est = vread(&hs->est[jc - 1]);
    {
      ProfScope ps(P, s, kCatUpdate, 8.0 * (jc + 2) * (double)N);
      CK(launch_update(left ? P->V : P->Z, ld, jc, x, N, P->ks, left, s, Members::one(), nullptr,
                       !left && o->zstore == RSFDE_ZSTORE_FP32));
    }
    total += jc;
    if (left && est <= thresh) {  // stop on the preconditioned estimate
      CK(hipStreamSynchronize(s));
      return finish(st, RSFDE_OK, total, cycles, est, bnorm);
    }
  }
}

// ---------------------------------------------------------------------------
// s-step form of the right-preconditioned restarted GMRES.  Per block of s
// steps: s preconditioner + matrix-vector applications build the directions
// u_{i+1} = (M P^{-1} - theta) u_i from u_0 = q_m (theta = 1, the centre of
// the preconditioned spectrum); one Gram pass G = [Q U]^T U on the matrix
// cores; on the host C = Q^T U, R = chol(U^T U - C^T C) (a second block pass
// when that loses too many digits); one update pass U <- (U - Q C) R^{-1}.
// The Hessenberg columns of the block follow from
//   (M P^{-1}) Q S_l = Q (S_r) with S the block's coordinates,
// the Givens rotations and residual estimates are the usual ones (host), and
// the solution update uses the stored P^{-1} u vectors with coefficients
// W y, W the triangular map from basis vectors to directions.
// ---------------------------------------------------------------------------

// Upper-triangular R with R^T R = A (s x s, row-major), column by column.
// Returns the number of leading pivots accepted: a pivot fails when it is not
// positive or below rel * A_kk (the direction is numerically dependent on the
// ones before it, or A = U^T U - C^T C lost it to cancellation).
int cholesky_upper(const std::vector<double>& A, int n, std::vector<double>& R, double rel) {
  R.assign((size_t)n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    double d = A[k * n + k];
    for (int i = 0; i < k; ++i) d -= R[i * n + k] * R[i * n + k];
    if (!(d > rel * std::fabs(A[k * n + k])) || !std::isfinite(d)) return k;
    const double rk = std::sqrt(d);
    R[k * n + k] = rk;
    for (int j = k + 1; j < n; ++j) {
      double v = A[k * n + j];
      for (int i = 0; i < k; ++i) v -= R[i * n + k] * R[i * n + j];
      R[k * n + j] = v / rk;
    }
  }
  return n;
}

// Inverse of an upper-triangular n x n matrix (row-major).
std::vector<double> upper_inverse(const std::vector<double>& R, int n) {
  std::vector<double> X((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    X[j * n + j] = 1.0 / R[j * n + j];
    for (int i = j - 1; i >= 0; --i) {
      double v = 0.0;
      for (int k = i + 1; k <= j; ++k) v += R[i * n + k] * X[k * n + j];
      X[i * n + j] = -v / R[i * n + i];
    }
  }
  return X;
}

// One block projection / Cholesky-QR step on the host from the Gram result:
// C [nq][ss] (row-major) and R [ss][ss]; returns the number of directions
// whose pivots were accepted (the leading part of R is valid).
int block_factor(const double* G, int nq, int ss, std::vector<double>& C, std::vector<double>& R) {
  C.assign((size_t)nq * ss, 0.0);
  for (int i = 0; i < nq; ++i)
    for (int k = 0; k < ss; ++k) C[i * ss + k] = G[i * 16 + k];
  std::vector<double> A((size_t)ss * ss);
  for (int a = 0; a < ss; ++a)
    for (int b = 0; b < ss; ++b) {
      double v = G[(nq + a) * 16 + b];
      for (int i = 0; i < nq; ++i) v -= C[i * ss + a] * C[i * ss + b];
      A[a * ss + b] = v;
    }
  for (int a = 0; a < ss; ++a)  // symmetrise
    for (int b = a + 1; b < ss; ++b) A[a * ss + b] = A[b * ss + a] = 0.5 * (A[a * ss + b] + A[b * ss + a]);
  return cholesky_upper(A, ss, R, 1e-13);
}

// Leading k x k part of a row-major n x n matrix, and the first k columns of
// a row-major [rows][n] matrix.
std::vector<double> lead_square(const std::vector<double>& A, int n, int k) {
  std::vector<double> B((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) B[(size_t)i * k + j] = A[(size_t)i * n + j];
  return B;
}
std::vector<double> lead_cols(const std::vector<double>& A, int rows, int n, int k) {
  std::vector<double> B((size_t)rows * k);
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < k; ++j) B[(size_t)i * k + j] = A[(size_t)i * n + j];
  return B;
}

int solve_core(Plan* P, double* x, const rsfde_solver_opts* o, rsfde_stats* st, hipStream_t s);

// Enqueues the Gram block of the s-step form and waits for it by polling the
// sequence word its finishing kernel publishes in pinned memory (this wakes
// sooner than a stream synchronisation); stops early if the stream drains or
// fails without publishing.
int gram_block(Plan* P, int nr, int nq, int ss, hipStream_t s) {
  const int32_t seq = ++P->gram_seq;
  {
    ProfScope ps(P, s, kCatGram, 8.0 * (double)nr * (double)P->N);  // [Q U] read once
    CK(launch_bgram(P->V, P->ldv, nr, nq, ss, P->N, P->gpart, P->gram_d, &P->hs_dev->gram_seq,
                    seq, &P->ks->gram_done, s));
  }
  for (unsigned it = 1;; ++it) {
    if (vread(&P->hs->gram_seq) == seq) return RSFDE_OK;
    if ((it & 255) == 0) {
      const hipError_t q = hipStreamQuery(s);
      if (q == hipSuccess) return vread(&P->hs->gram_seq) == seq ? RSFDE_OK : RSFDE_EHIP;
      if (q != hipErrorNotReady) return RSFDE_EHIP;
    }
    __builtin_ia32_pause();
  }
}

// Enqueues U <- (U - Q C) R^{-1} with coef = C [nq][ss] then R^{-1} [ss][ss]
// (host).  Small tables travel as kernel arguments; larger ones go through
// the pinned staging buffer, which no earlier copy can still be reading: every
// earlier copy precedes a Gram block the host has already waited for.
int block_update(Plan* P, int nq, int ss, const double* coef, hipStream_t s) {
  const size_t nc = (size_t)nq * ss + (size_t)ss * ss;
  if (nc > (size_t)kCoefArgMax) {
    std::copy(coef, coef + nc, P->coef_h);
    CK(hipMemcpyAsync(P->coef_d, P->coef_h, nc * sizeof(double), hipMemcpyHostToDevice, s));
  }
  ProfScope ps(P, s, kCatBupd, 8.0 * (double)(nq + 2 * ss) * (double)P->N);
  CK(launch_bupd(P->V, P->ldv, nq, nq, ss, P->N, coef, P->coef_d, s));
  return RSFDE_OK;
}

// finish() that also reports the count of reorthogonalised / truncated blocks
int finish_ev(rsfde_stats* st, int events, int code, int iters, int restarts, double beta,
              double bnorm) {
  const int rc = finish(st, code, iters, restarts, beta, bnorm);
  if (st) st->reserved = events;
  return rc;
}

int solve_core_sstep(Plan* P, double* x, const rsfde_solver_opts* o, rsfde_stats* st,
                     hipStream_t s) {
  const size_t N = P->N, ld = P->ldv;
  volatile HostStatus* hs = P->hs;
  const int S = o->sstep, RS = o->restart;
  const double theta = 1.0;
  CK(hipStreamSynchronize(s));
  if (vread(&hs->flags) & kFlagNonFinite) return finish_ev(st, 0, RSFDE_ENONFINITE, 0, 0, 0, 0);
  const double bnorm = vread(&hs->bnorm);
  if (bnorm == 0.0) {
    CK(hipMemsetAsync(x, 0, N * sizeof(double), s));
    CK(hipStreamSynchronize(s));
    return finish_ev(st, 0, RSFDE_OK, 0, 0, 0.0, 0.0);
  }
  const double thresh = o->tol * bnorm;
  const int LH = RS + 1;                        // leading dimension of H (row-major [row][col])
  std::vector<double> Hraw((size_t)LH * RS), Hrot((size_t)LH * RS), W((size_t)RS * RS);
  std::vector<double> cs(RS), sn(RS), g(RS + 1), C, R, C2, R2;
  int total = 0, cycles = 0, events = 0;
  double beta = 0.0;
  for (;;) {
    int rc = matvec_impl(P, x, P->w, s);
    if (rc) return finish_ev(st, events, rc, total, cycles, beta, bnorm);
    {
      ProfScope ps(P, s, kCatResidual, 24.0 * N);
      CK(launch_residual(P->b, P->w, P->V, N, P->rw, P->ks, P->hs_dev, s));
    }
    CK(hipStreamSynchronize(s));
    if (vread(&hs->flags) & kFlagNonFinite) return finish_ev(st, events, RSFDE_ENONFINITE, total, cycles, beta, bnorm);
    beta = vread(&hs->beta);
    if (beta <= thresh) return finish_ev(st, events, RSFDE_OK, total, cycles, beta, bnorm);
    if (total >= o->max_iters) return finish_ev(st, events, RSFDE_ENOTCONV, total, cycles, beta, bnorm);
    ++cycles;
    {  // q_0 = r / beta, stored normalised
      ProfScope ps(P, s, kCatOther, 16.0 * N);
      CK(launch_scale_copy(P->V, &P->ks->vscale[0], P->V, N, s));
    }
    const int jmax = std::min(RS, o->max_iters - total);
    std::fill(Hraw.begin(), Hraw.end(), 0.0);
    std::fill(Hrot.begin(), Hrot.end(), 0.0);
    std::fill(W.begin(), W.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int m = 0, jc = -1;
    while (m < jmax) {
      int ss = std::min(S, jmax - m);
      W[(size_t)m * RS + m] = 1.0;  // q_m is itself the first direction of the block
      for (int i = 0; i < ss; ++i) {
        double* ui = P->V + (size_t)(m + i) * ld;
        void* zi = o->zstore == RSFDE_ZSTORE_FP32 ? (void*)((float*)P->Z + (size_t)(m + i) * ld)
                                                  : (void*)(P->Z + (size_t)(m + i) * ld);
        rc = precond_matvec_impl(P, ui, nullptr, zi, P->V + (size_t)(m + i + 1) * ld, o->precision,
                                 s, ui, theta, o->zstore == RSFDE_ZSTORE_FP32);
        if (rc) return finish_ev(st, events, rc, total, cycles, beta, bnorm);
      }
      const int nq = m + 1;
      int nr = m + 1 + ss;
      rc = gram_block(P, nr, nq, ss, s);
      if (rc) return finish_ev(st, events, rc, total, cycles, beta, bnorm);
      const double* G = P->gram_h;
      for (int i = 0; i < nr * 16; ++i)
        if (!std::isfinite(G[i])) return finish_ev(st, events, RSFDE_ENONFINITE, total, cycles, beta, bnorm);
      int kp = block_factor(G, nq, ss, C, R);
      if (P->trace) {
        std::fprintf(stderr, "[rsfde s-step] cycle %d m %d ss %d pivots %d  diag(U^T U)", cycles, m,
                     ss, kp);
        for (int k = 0; k < ss; ++k) std::fprintf(stderr, " %.3e", G[(nq + k) * 16 + k]);
        std::fprintf(stderr, "  R_kk");
        for (int k = 0; k < kp; ++k) std::fprintf(stderr, " %.3e", R[(size_t)k * ss + k]);
        std::fprintf(stderr, "\n");
      }
      std::vector<double> Capply;  // projections still to subtract from the stored block
      bool second = false;
      if (kp < ss) {
        // second block pass: U <- U - Q C, then project and factor again
        ++events;
        std::vector<double> coef((size_t)nq * ss + (size_t)ss * ss, 0.0);
        std::copy(C.begin(), C.end(), coef.begin());
        for (int k = 0; k < ss; ++k) coef[(size_t)nq * ss + k * ss + k] = 1.0;
        rc = block_update(P, nq, ss, coef.data(), s);
        if (rc) return finish_ev(st, events, rc, total, cycles, beta, bnorm);
        rc = gram_block(P, nr, nq, ss, s);
        if (rc) return finish_ev(st, events, rc, total, cycles, beta, bnorm);
        kp = block_factor(P->gram_h, nq, ss, C2, R2);
        if (P->trace) {
          std::fprintf(stderr, "[rsfde s-step]   second pass pivots %d  diag(U'^T U')", kp);
          for (int k = 0; k < ss; ++k) std::fprintf(stderr, " %.3e", P->gram_h[(nq + k) * 16 + k]);
          std::fprintf(stderr, "\n");
        }
        if (kp == 0 && m > 0) {
          // even the first direction of the block is numerically in the span of
          // the basis (which has lost orthogonality): end the cycle with the m
          // columns built so far and restart from the true residual
          ++events;
          jc = m;
          break;
        }
        if (kp == 0) {
          // at the start of a cycle: finish this solve with the one-vector form
          rsfde_solver_opts o1 = *o;
          o1.sstep = 0;
          o1.max_iters = std::max(1, o->max_iters - total);
          const int rc1 = solve_core(P, x, &o1, st, s);
          if (st) {
            st->iters += total;
            st->reserved = events + 1;
          }
          return rc1;
        }
        for (size_t i = 0; i < C.size(); ++i) C[i] += C2[i];  // total projections
        R = R2;
        second = true;
      }
      Capply = second ? C2 : C;
      if (kp < ss) {  // keep the leading kp directions of the block
        ++events;
        C = lead_cols(C, nq, ss, kp);
        Capply = lead_cols(Capply, nq, ss, kp);
        R = lead_square(R, ss, kp);
        ss = kp;
        nr = nq + ss;
      }
      // Hessenberg columns m..m+ss-1:  H_blk = (S_r - H_old Top) T^{-1}
      {
        std::vector<double> Sl((size_t)nr * ss, 0.0), Sr((size_t)nr * ss, 0.0);
        // S column 0 = e_m; column k>=1: rows < nq = C[:, k-1], rows nq.. = R[:, k-1]
        auto Scol = [&](int row, int k) -> double {
          if (k == 0) return row == m ? 1.0 : 0.0;
          if (row < nq) return C[(size_t)row * ss + (k - 1)];
          return R[(size_t)(row - nq) * ss + (k - 1)];
        };
        for (int r = 0; r < nr; ++r)
          for (int k = 0; k < ss; ++k) {
            Sl[(size_t)r * ss + k] = Scol(r, k);
            Sr[(size_t)r * ss + k] = Scol(r, k + 1) + theta * Scol(r, k);
          }
        // T = rows m..m+ss-1 of S_l (upper triangular), Top = rows < m
        std::vector<double> T((size_t)ss * ss);
        for (int a = 0; a < ss; ++a)
          for (int k = 0; k < ss; ++k) T[(size_t)a * ss + k] = Sl[(size_t)(m + a) * ss + k];
        const std::vector<double> Ti = upper_inverse(T, ss);
        std::vector<double> X((size_t)nr * ss);
        for (int r = 0; r < nr; ++r)
          for (int k = 0; k < ss; ++k) {
            double v = Sr[(size_t)r * ss + k];
            for (int c = 0; c < m; ++c) v -= Hraw[(size_t)r * RS + c] * Sl[(size_t)c * ss + k];
            X[(size_t)r * ss + k] = v;
          }
        for (int r = 0; r < nr; ++r)
          for (int k = 0; k < ss; ++k) {
            double v = 0.0;
            for (int a = 0; a <= k; ++a) v += X[(size_t)r * ss + a] * Ti[(size_t)a * ss + k];
            // Hessenberg: entries below the subdiagonal are rounding noise
            Hraw[(size_t)r * RS + (m + k)] = (r <= m + k + 1) ? v : 0.0;
          }
      }
      // direction map W for q_{m+1..m+ss-1} (q_{m+ss} is the next block's first direction)
      for (int k = 0; k + 1 < ss; ++k) {
        const int col = m + 1 + k;
        for (int i = 0; i <= col; ++i) {
          double v = (i == col) ? 1.0 : 0.0;
          for (int c = 0; c < nq; ++c) v -= W[(size_t)i * RS + c] * C[(size_t)c * ss + k];
          for (int l = 0; l < k; ++l) v -= W[(size_t)i * RS + (m + 1 + l)] * R[(size_t)l * ss + k];
          W[(size_t)i * RS + col] = v / R[(size_t)k * ss + k];
        }
      }
      // Givens rotations and residual estimates, column by column
      for (int k = 0; k < ss && jc < 0; ++k) {
        const int c = m + k;
        for (int r = 0; r <= c + 1; ++r) Hrot[(size_t)r * RS + c] = Hraw[(size_t)r * RS + c];
        for (int i = 0; i < c; ++i) {
          const double a = Hrot[(size_t)i * RS + c], b2 = Hrot[(size_t)(i + 1) * RS + c];
          Hrot[(size_t)i * RS + c] = cs[i] * a + sn[i] * b2;
          Hrot[(size_t)(i + 1) * RS + c] = -sn[i] * a + cs[i] * b2;
        }
        const double a = Hrot[(size_t)c * RS + c], b2 = Hrot[(size_t)(c + 1) * RS + c];
        const double den = std::hypot(a, b2);
        cs[c] = den > 0.0 ? a / den : 1.0;
        sn[c] = den > 0.0 ? b2 / den : 0.0;
        Hrot[(size_t)c * RS + c] = den;
        Hrot[(size_t)(c + 1) * RS + c] = 0.0;
        g[c + 1] = -sn[c] * g[c];
        g[c] = cs[c] * g[c];
        if (!std::isfinite(den) || !std::isfinite(g[c + 1]))
          return finish_ev(st, events, RSFDE_ENONFINITE, total + c, cycles, beta, bnorm);
        if (std::fabs(g[c + 1]) <= thresh) jc = c + 1;
      }
      if (jc > 0) break;
      if (m + ss < jmax) {  // the block becomes orthonormal basis vectors
        const std::vector<double> Ri = upper_inverse(R, ss);
        std::vector<double> coef(Capply);
        coef.insert(coef.end(), Ri.begin(), Ri.end());
        rc = block_update(P, nq, ss, coef.data(), s);
        if (rc) return finish_ev(st, events, rc, total, cycles, beta, bnorm);
      }
      m += ss;
    }
    if (jc < 0) jc = m;
    // y = R^{-1} g (rotated Hessenberg), coefficients of the stored P^{-1} u: W y
    std::vector<double> y(jc);
    for (int i = jc - 1; i >= 0; --i) {
      double v = g[i];
      for (int k = i + 1; k < jc; ++k) v -= Hrot[(size_t)i * RS + k] * y[k];
      const double d = Hrot[(size_t)i * RS + i];
      y[i] = d != 0.0 ? v / d : 0.0;
    }
    std::vector<double> cz(jc);
    for (int i = 0; i < jc; ++i) {
      double v = 0.0;
      for (int l = i; l < jc; ++l) v += W[(size_t)i * RS + l] * y[l];
      cz[i] = v;
    }
    {
      ProfScope ps(P, s, kCatUpdate, 8.0 * (jc + 2) * (double)N);
      CK(launch_update_coef(P->Z, ld, jc, x, N, cz.data(), s, o->zstore == RSFDE_ZSTORE_FP32));
    }
    total += jc;
  }
}

}  // namespace
}  // namespace rsfde

using rsfde::Plan;

namespace rsfde {
namespace {

// Workspaces every plan needs: the mask copy, Krylov basis V (restart + 1
// vectors) and Z (restart), five work vectors, three (four in 3-D)
// preconditioner intermediates of `slots` values (sized for FP64; P1 of
// p1_slots when that is larger), the 3-D
// matrix-vector intermediate, reduction and s-step buffers, pinned status
// words and events.  Enqueued on s.
int alloc_common(Plan* P, const uint8_t* mask_dev, size_t slots, hipStream_t s,
                 size_t p1_slots = 0) {
  const size_t N = P->N, ld = P->ldv;
  const int max_restart = P->max_restart;
#define AL(ptr, cnt)                                              \
  do {                                                            \
    if (P->dalloc(&(ptr), (cnt)) != hipSuccess) return RSFDE_ENOMEM; \
  } while (0)
  AL(P->mask, N);
  AL(P->V, (size_t)(max_restart + 1) * ld);
  AL(P->Z, (size_t)max_restart * ld);
  AL(P->b, ld);
  AL(P->w, ld);
  // t: the matrix-vector intermediate, strip-tiled on two-dimensional plans
  AL(P->t, P->is3d ? ld
                   : std::max(ld, (size_t)8 * (size_t)((P->n1 + 3) / 4) *
                                      (size_t)((P->n2 + 1) / 2)));
  AL(P->mu, ld);
  AL(P->pb, ld);
  double* q = nullptr;
  AL(q, slots);
  P->Q = q;
  AL(q, std::max(slots, p1_slots));
  P->P1 = q;
  AL(q, slots);
  P->P2 = q;
  if (P->is3d) {
    AL(q, slots);
    P->R3 = q;
    AL(P->t3, ld);
  }
  AL(P->ks, 1);
  AL(P->rw.partial, (size_t)(kMaxRestart + 2) * kMaxRedBlocks);
  AL(P->gpart, (size_t)16 * 16 * kGramMaxTiles * kGramBlocks);
  AL(P->coef_d, (size_t)16 * 16 * kGramMaxTiles + 256);
#undef AL
  if (hipHostMalloc((void**)&P->hs, sizeof(HostStatus), hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess)
    return RSFDE_ENOMEM;
  std::memset((void*)P->hs, 0, sizeof(HostStatus));
  if (hipHostGetDevicePointer((void**)&P->hs_dev, P->hs, 0) != hipSuccess) return RSFDE_EHIP;
  if (hipHostMalloc((void**)&P->gram_h, sizeof(double) * 16 * 16 * kGramMaxTiles,
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostMalloc((void**)&P->coef_h, sizeof(double) * (16 * 16 * kGramMaxTiles + 256),
                    hipHostMallocDefault) != hipSuccess)
    return RSFDE_ENOMEM;
  if (hipHostGetDevicePointer((void**)&P->gram_d, P->gram_h, 0) != hipSuccess) return RSFDE_EHIP;
  for (auto& e : P->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return RSFDE_EHIP;

  if (hipMemcpyAsync(P->mask, mask_dev, N, hipMemcpyDeviceToDevice, s) != hipSuccess) return RSFDE_EHIP;
  if (hipMemsetAsync(P->ks, 0, sizeof(KrylovState), s) != hipSuccess) return RSFDE_EHIP;
  return RSFDE_OK;
}

// Pass A/B table of the power-of-two sine transform along x: eigenvalues in
// slot order (0 at frequency 0).
std::vector<double> slot_eigs(const std::vector<double>& lx, int Lx) {
  const int n1 = (int)lx.size(), Px = fft_pts(Lx);
  std::vector<double> lam(n1 + 1, 0.0);
  for (int c = 0; c < n1 + 1; ++c) {
    const int f = fft_freq(Lx, Px, fft_slot_pos(Lx, Px, c));
    lam[c] = (f >= 1 && f <= n1) ? lx[f - 1] : 0.0;
  }
  return lam;
}

// Column-pass eigenvalues in register-position order of the length-L FFT
// (even in frequency; 0 at frequencies 0 and L/2).
std::vector<double> pos_eigs(const std::vector<double>& ly, int L) {
  const int n = (int)ly.size(), Py = pc_cols_pts(L);
  std::vector<double> lam(L);
  for (int p = 0; p < L; ++p) {
    const int f = fft_freq(L, Py, p);
    const int g = std::min(f, L - f);
    lam[p] = (g >= 1 && g <= n) ? ly[g - 1] : 0.0;
  }
  return lam;
}

// Tables of the symmetric sine transform of length L (sd_engine.hpp) for the
// eigenvalues lam (natural order, lam[k-1] at DST index k): in slot order
// (x direction), in block-position order (y direction, 9 L/16 entries), and
// the mirror slots of the upper halves of blocks 0 and 8 (-1 at frequency L/2).
template <int L>
void sd_tables_L(const std::vector<double>& lam, std::vector<double>* by_slot,
                 std::vector<double>* by_pos, std::vector<int32_t>* msl) {
  using S = Sd<L>;
  using Fs = typename S::Fs;
  const int n = (int)lam.size();
  auto lam_of = [&](int f) {
    const int k = S::fold(f);
    return (k >= 1 && k <= n) ? lam[k - 1] : 0.0;
  };
  std::vector<int> slot_at(S::NPOS, -1), slot_of_freq(L, -1);
  for (int r = 0; r < 9; ++r)
    for (int tau = 0; tau < S::TS; ++tau)
      for (int e = 0; e < 16; ++e) {
        const int P = r * S::LS + Fs::pos(Fs::NS - 1, tau, e);
        const int c = S::slot(r, tau, e);
        slot_at[P] = c;
        if (c >= 0) slot_of_freq[S::freq(P)] = c;
      }
  if (by_slot) {
    by_slot->assign(L / 2, 0.0);
    for (int P = 0; P < S::NPOS; ++P)
      if (slot_at[P] >= 0) (*by_slot)[slot_at[P]] = lam_of(S::freq(P));
  }
  if (by_pos) {
    by_pos->assign(S::NPOS, 0.0);
    for (int P = 0; P < S::NPOS; ++P) (*by_pos)[P] = lam_of(S::freq(P));
  }
  if (msl) {
    msl->assign(2 * S::LS, -1);
    for (int h = 0; h < 2; ++h)
      for (int q = 0; q < S::LS; ++q) {
        const int P = (h ? 8 : 0) * S::LS + q;
        if (slot_at[P] >= 0) continue;
        const int g = L - S::freq(P);
        (*msl)[h * S::LS + q] = (g == L / 2) ? -1 : slot_of_freq[g];
      }
  }
}

bool sd_tables(int L, const std::vector<double>& lam, std::vector<double>* by_slot,
               std::vector<double>* by_pos, std::vector<int32_t>* msl) {
  switch (L) {
    case 512: sd_tables_L<512>(lam, by_slot, by_pos, msl); return true;
    case 1024: sd_tables_L<1024>(lam, by_slot, by_pos, msl); return true;
    case 2048: sd_tables_L<2048>(lam, by_slot, by_pos, msl); return true;
    case 4096: sd_tables_L<4096>(lam, by_slot, by_pos, msl); return true;
    case 8192: sd_tables_L<8192>(lam, by_slot, by_pos, msl); return true;
    default: return false;
  }
}

}  // namespace
}  // namespace rsfde

struct rsfde_plan_s {
  Plan p;
};

extern "C" {

const char* rsfde_strerror(int code) {
  switch (code) {
    case RSFDE_OK: return "ok";
    case RSFDE_EINVAL: return "invalid argument";
    case RSFDE_ENOMEM: return "out of memory";
    case RSFDE_EHIP: return "HIP runtime error";
    case RSFDE_ENOTCONV: return "iteration cap reached before convergence";
    case RSFDE_EBREAKDOWN: return "Krylov breakdown";
    case RSFDE_ENONFINITE: return "non-finite value";
    case RSFDE_EUNSUPPORTED: return "unsupported shape or option";
    default: return "unknown error";
  }
}

int rsfde_setup(rsfde_plan* out, const rsfde_grid* grid, double alpha1, double alpha2,
                double kx, double ky, const uint8_t* mask_dev, double eta, double dt,
                int32_t max_restart, void* stream) {
  using namespace rsfde;
  if (!out) return RSFDE_EINVAL;
  *out = nullptr;
  if (!grid || !mask_dev) return RSFDE_EINVAL;
  const int n1 = grid->n1, n2 = grid->n2;
  if (n1 < 1 || n2 < 1) return RSFDE_EINVAL;
  if (!(grid->x_hi > grid->x_lo) || !(grid->y_hi > grid->y_lo)) return RSFDE_EINVAL;
  if (!std::isfinite(grid->x_lo) || !std::isfinite(grid->x_hi) || !std::isfinite(grid->y_lo) ||
      !std::isfinite(grid->y_hi))
    return RSFDE_EINVAL;
  if (!(alpha1 > 1.0 && alpha1 < 2.0) || !(alpha2 > 1.0 && alpha2 < 2.0)) return RSFDE_EINVAL;
  if (!(kx >= 0.0) || !(ky >= 0.0) || !std::isfinite(kx) || !std::isfinite(ky)) return RSFDE_EINVAL;
  if (!(eta > 0.0) || !(dt > 0.0) || !std::isfinite(eta) || !std::isfinite(dt)) return RSFDE_EINVAL;
  if (max_restart <= 0) max_restart = 30;
  if (max_restart > kMaxRestart) return RSFDE_EINVAL;
  if (n1 > kMaxN || n2 > kMaxN) return RSFDE_EUNSUPPORTED;

  rsfde_plan_s* h = new (std::nothrow) rsfde_plan_s();
  if (!h) return RSFDE_ENOMEM;
  Plan* P = &h->p;
  int rc = RSFDE_OK;
  // RSFDE_TRACE=1: a failed setup names its line and the last HIP error.
  const char* trace_env = std::getenv("RSFDE_TRACE");
  const bool tr_on = trace_env && trace_env[0] == '1';
  auto failx = [&](int line, int code) {
    if (tr_on)
      std::fprintf(stderr, "[rsfde] setup failed at line %d (%d): last HIP error %s\n", line, code,
                   hipGetErrorString(hipGetLastError()));
    delete h;
    return code;
  };
  if (hipGetDevice(&P->dev) != hipSuccess) return failx(__LINE__, RSFDE_EHIP);
  hipStream_t s = (hipStream_t)stream;
  P->s0 = s;
  P->n1 = n1;
  P->n2 = n2;
  P->N = (size_t)n1 * (size_t)n2;
  P->ldv = (P->N + 63) / 64 * 64;
  P->alpha1 = alpha1;
  P->alpha2 = alpha2;
  P->kx = kx;
  P->ky = ky;
  P->eta = eta;
  P->dt = dt;
  P->dpen = dt / eta;
  P->max_restart = max_restart;
  {
    const char* tr = std::getenv("RSFDE_TRACE");
    P->trace = tr && tr[0] == '1';
  }

  // Section 2: mesh widths and unit-k coefficients c = dt c_alpha / h^alpha.
  const double hx = (grid->x_hi - grid->x_lo) / (n1 + 1);
  const double hy = (grid->y_hi - grid->y_lo) / (n2 + 1);
  const double ca1 = -1.0 / (2.0 * std::cos(alpha1 * kPi / 2.0));
  const double ca2 = -1.0 / (2.0 * std::cos(alpha2 * kPi / 2.0));
  const double cx1 = dt * ca1 / std::pow(hx, alpha1);
  const double cy1 = dt * ca2 / std::pow(hy, alpha2);
  const std::vector<double> tx = toeplitz_col(alpha1, n1, cx1);
  const std::vector<double> ty = toeplitz_col(alpha2, n2, cy1);

  P->Lcx = std::max(2, next_pow2(2L * n1));
  P->Lcy = std::max(2, next_pow2(2L * n2));
  P->Ldx = is_pow2(n1 + 1) ? 2 * (n1 + 1) : 0;
  P->Ldy = is_pow2(n2 + 1) ? 2 * (n2 + 1) : 0;
  if (P->Ldx == 0 || P->Ldy == 0) {  // chirp form in both directions
    P->Ldx = P->Ldy = 0;
    P->Lgx = std::max(2, next_pow2(2L * n1 - 1));
    P->Lgy = std::max(2, next_pow2(2L * n2 - 1));
  }

  // Pass A/B/C intermediates: Q strip-tiled, 8 values per tile of 2 rows x 4
  // slots (at least the (n1 + 1) n2 of the natural layout).  P1 holds the
  // interleaved P1/P2 pairs in row segments of 8 (FP64) or 16 (FP32) slots.
  const size_t slots = (size_t)8 * (size_t)((n1 + 4) / 4) * (size_t)((n2 + 1) / 2);
  const size_t pair_slots = (size_t)2 * (size_t)((n1 + 16) / 16 * 16) * (size_t)n2;
  if ((rc = alloc_common(P, mask_dev, slots, s, std::max(2 * slots, pair_slots))) != RSFDE_OK)
    return failx(__LINE__, rc);

  // Matrix-vector symbols (unit kx, ky).
  if (upload(P, &P->symx, conv_symbol_pos(tx, P->Lcx), s) != hipSuccess) return failx(__LINE__, RSFDE_ENOMEM);
  if (upload(P, &P->symy, conv_symbol_pos(ty, P->Lcy), s) != hipSuccess) return failx(__LINE__, RSFDE_ENOMEM);
  for (int L : {P->Lcx, P->Lcy, P->Ldx, P->Ldy, P->Lgx, P->Lgy})
    if (ensure_twiddles(P, L, s) != hipSuccess) return failx(__LINE__, RSFDE_ENOMEM);

  // Preconditioner tables (Section 4.1), in the layouts of the three passes.
  if (P->Ldx && P->Ldy) {
    P->sdx = P->Ldx >= kSdMinL;
    P->sdy = P->Ldy >= kSdMinL;
    std::vector<double> lamx, lamy;
    std::vector<int32_t> msl;
    if (P->sdx) {
      if (!sd_tables(P->Ldx, tau_eigs(tx), &lamx, nullptr, &msl)) return failx(__LINE__, RSFDE_EUNSUPPORTED);
      if (upload(P, &P->msl, msl, s) != hipSuccess || ensure_twiddles(P, P->Ldx / 16, s) != hipSuccess)
        return failx(__LINE__, RSFDE_ENOMEM);
    } else {
      lamx = slot_eigs(tau_eigs(tx), P->Ldx);
    }
    if (P->sdy) {
      if (!sd_tables(P->Ldy, tau_eigs(ty), nullptr, &lamy, nullptr)) return failx(__LINE__, RSFDE_EUNSUPPORTED);
      if (ensure_twiddles(P, P->Ldy / 16, s) != hipSuccess) return failx(__LINE__, RSFDE_ENOMEM);
    } else {
      lamy = pos_eigs(tau_eigs(ty), P->Ldy);
    }
    std::vector<float> lamx_f(lamx.begin(), lamx.end()), lamy_f(lamy.begin(), lamy.end());
    if (upload(P, &P->lamx64, lamx, s) != hipSuccess || upload(P, &P->lamy64, lamy, s) != hipSuccess ||
        upload(P, &P->lamx32, lamx_f, s) != hipSuccess || upload(P, &P->lamy32, lamy_f, s) != hipSuccess)
      return failx(__LINE__, RSFDE_ENOMEM);
  }
  if (P->Lgx) {  // chirp-form tables
    const std::vector<double> lx = tau_eigs(tx), ly = tau_eigs(ty);
    if (upload(P, &P->lamx_n, lx, s) != hipSuccess || upload(P, &P->lamy_n, ly, s) != hipSuccess)
      return failx(__LINE__, RSFDE_ENOMEM);
    struct Dir { int n, L; void **ch, **kh; };
    for (Dir d : {Dir{n1, P->Lgx, P->chx, P->khx}, Dir{n2, P->Lgy, P->chy, P->khy}}) {
      std::vector<double> ch, kh;
      chirp_tables(d.n, d.L, ch, kh);
      const std::vector<float> chf(ch.begin(), ch.end()), khf(kh.begin(), kh.end());
      double *a = nullptr, *b = nullptr;
      float *c = nullptr, *e = nullptr;
      if (upload(P, &a, ch, s) != hipSuccess || upload(P, &b, kh, s) != hipSuccess ||
          upload(P, &c, chf, s) != hipSuccess || upload(P, &e, khf, s) != hipSuccess)
        return failx(__LINE__, RSFDE_ENOMEM);
      d.ch[0] = a;
      d.kh[0] = b;
      d.ch[1] = c;
      d.kh[1] = e;
    }
  }
  // BF16 / MFMA preconditioner: padded sine matrices, natural-order eigenvalues
  {
    P->n1p = (n1 + 127) / 128 * 128;
    P->n2p = (n2 + 127) / 128 * 128;
    const std::vector<double> lx = tau_eigs(tx), ly = tau_eigs(ty);
    std::vector<float> lxn(P->n1p, 0.f), lyn(P->n2p, 0.f);
    for (int i = 0; i < n1; ++i) lxn[i] = (float)lx[i];
    for (int j = 0; j < n2; ++j) lyn[j] = (float)ly[j];
    std::vector<uint16_t> sx, sxl, sy, syl;
    sine_matrix_bf16(n1, P->n1p, sx, sxl);
    sine_matrix_bf16(n2, P->n2p, sy, syl);
    uint16_t *sxd = nullptr, *syd = nullptr, *sxld = nullptr, *syld = nullptr;
    if (upload(P, &sxd, sx, s) != hipSuccess || upload(P, &syd, sy, s) != hipSuccess ||
        upload(P, &sxld, sxl, s) != hipSuccess || upload(P, &syld, syl, s) != hipSuccess ||
        upload(P, &P->lamx_nat, lxn, s) != hipSuccess || upload(P, &P->lamy_nat, lyn, s) != hipSuccess)
      return failx(__LINE__, RSFDE_ENOMEM);
    P->Sx16 = (__bf16*)sxd;
    P->Sy16 = (__bf16*)syd;
    P->Sx16lo = (__bf16*)sxld;
    P->Sy16lo = (__bf16*)syld;
    const size_t pp = (size_t)P->n1p * (size_t)P->n2p;
    if (P->dalloc(&P->A1T, 2 * pp) != hipSuccess || P->dalloc(&P->R12T, 2 * pp) != hipSuccess ||
        P->dalloc(&P->G, 2 * pp) != hipSuccess)
      return failx(__LINE__, RSFDE_ENOMEM);
  }
  if (hipStreamSynchronize(s) != hipSuccess) return failx(__LINE__, RSFDE_EHIP);
  (void)rc;
  *out = h;
  return RSFDE_OK;
}

int rsfde_setup3(rsfde_plan* out, const rsfde_grid3* grid, double alpha1, double alpha2,
                 double alpha3, double kx, double ky, double kz, const uint8_t* mask_dev,
                 double eta, double dt, int32_t max_restart, void* stream) {
  using namespace rsfde;
  if (!out) return RSFDE_EINVAL;
  *out = nullptr;
  if (!grid || !mask_dev) return RSFDE_EINVAL;
  const int n[3] = {grid->n1, grid->n2, grid->n3};
  const double lo[3] = {grid->x_lo, grid->y_lo, grid->z_lo};
  const double hi[3] = {grid->x_hi, grid->y_hi, grid->z_hi};
  const double al[3] = {alpha1, alpha2, alpha3};
  const double ks[3] = {kx, ky, kz};
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1) return RSFDE_EINVAL;
    if (!std::isfinite(lo[a]) || !std::isfinite(hi[a]) || !(hi[a] > lo[a])) return RSFDE_EINVAL;
    if (!(al[a] > 1.0 && al[a] < 2.0)) return RSFDE_EINVAL;
    if (!(ks[a] >= 0.0) || !std::isfinite(ks[a])) return RSFDE_EINVAL;
  }
  if (!(eta > 0.0) || !(dt > 0.0) || !std::isfinite(eta) || !std::isfinite(dt)) return RSFDE_EINVAL;
  if (max_restart <= 0) max_restart = 30;
  if (max_restart > kMaxRestart) return RSFDE_EINVAL;
  bool pow2 = true;
  for (int a = 0; a < 3; ++a) {
    if (n[a] > kMaxN) return RSFDE_EUNSUPPORTED;
    pow2 = pow2 && is_pow2(n[a] + 1);
  }
  const size_t N = (size_t)n[0] * (size_t)n[1] * (size_t)n[2];
  const size_t slots = (size_t)(n[0] + 1) * (size_t)n[1] * (size_t)n[2];
  if (slots > (size_t)INT32_MAX) return RSFDE_EUNSUPPORTED;

  rsfde_plan_s* h = new (std::nothrow) rsfde_plan_s();
  if (!h) return RSFDE_ENOMEM;
  Plan* P = &h->p;
  auto fail = [&](int code) {
    delete h;
    return code;
  };
  if (hipGetDevice(&P->dev) != hipSuccess) return fail(RSFDE_EHIP);
  hipStream_t s = (hipStream_t)stream;
  P->s0 = s;
  P->n1 = n[0];
  P->n2 = n[1];
  P->n3 = n[2];
  P->is3d = true;
  P->N = N;
  P->ldv = (N + 63) / 64 * 64;
  P->alpha1 = alpha1;
  P->alpha2 = alpha2;
  P->alpha3 = alpha3;
  P->kx = kx;
  P->ky = ky;
  P->kz = kz;
  P->eta = eta;
  P->dt = dt;
  P->dpen = dt / eta;
  P->max_restart = max_restart;
  {
    const char* tr = std::getenv("RSFDE_TRACE");
    P->trace = tr && tr[0] == '1';
  }
  // Section 2 on each axis: unit-k Toeplitz columns c = dt c_alpha / h^alpha.
  std::vector<double> t[3];
  for (int a = 0; a < 3; ++a) {
    const double hstep = (hi[a] - lo[a]) / (n[a] + 1);
    const double ca = -1.0 / (2.0 * std::cos(al[a] * kPi / 2.0));
    t[a] = toeplitz_col(al[a], n[a], dt * ca / std::pow(hstep, al[a]));
  }
  P->Lcx = std::max(2, next_pow2(2L * n[0]));
  P->Lcy = std::max(2, next_pow2(2L * n[1]));
  P->Lcz = std::max(2, next_pow2(2L * n[2]));
  if (pow2) {  // odd-extension sine transforms
    P->Ldx = 2 * (n[0] + 1);
    P->Ldy = 2 * (n[1] + 1);
    P->Ldz = 2 * (n[2] + 1);
  } else {  // chirp form on every axis
    P->Lgx = std::max(2, next_pow2(2L * n[0] - 1));
    P->Lgy = std::max(2, next_pow2(2L * n[1] - 1));
    P->Lgz = std::max(2, next_pow2(2L * n[2] - 1));
  }
  int rc = alloc_common(P, mask_dev, slots, s);
  if (rc != RSFDE_OK) return fail(rc);
  if (upload(P, &P->symx, conv_symbol_pos(t[0], P->Lcx), s) != hipSuccess ||
      upload(P, &P->symy, conv_symbol_pos(t[1], P->Lcy), s) != hipSuccess ||
      upload(P, &P->symz, conv_symbol_pos(t[2], P->Lcz), s) != hipSuccess)
    return fail(RSFDE_ENOMEM);
  for (int L : {P->Lcx, P->Lcy, P->Lcz, P->Ldx, P->Ldy, P->Ldz, P->Lgx, P->Lgy, P->Lgz})
    if (ensure_twiddles(P, L, s) != hipSuccess) return fail(RSFDE_ENOMEM);
  if (!pow2) {  // chirp tables per axis (FP64 and FP32)
    struct Dir { int n, L; void **ch, **kh; };
    for (Dir d : {Dir{n[0], P->Lgx, P->chx, P->khx}, Dir{n[1], P->Lgy, P->chy, P->khy},
                  Dir{n[2], P->Lgz, P->chz, P->khz}}) {
      std::vector<double> ch, kh;
      chirp_tables(d.n, d.L, ch, kh);
      const std::vector<float> chf(ch.begin(), ch.end()), khf(kh.begin(), kh.end());
      double *a = nullptr, *b = nullptr;
      float *c = nullptr, *e = nullptr;
      if (upload(P, &a, ch, s) != hipSuccess || upload(P, &b, kh, s) != hipSuccess ||
          upload(P, &c, chf, s) != hipSuccess || upload(P, &e, khf, s) != hipSuccess)
        return fail(RSFDE_ENOMEM);
      d.ch[0] = a;
      d.kh[0] = b;
      d.ch[1] = c;
      d.kh[1] = e;
    }
  }
  // Section 4.1's eigenvalues: x in slot order folded with y into one value per
  // column of the [n3][(n1+1) n2] view (k included), z in position order (unit kz).
  // (chirp form: natural order on every axis)
  P->lx3 = pow2 ? slot_eigs(tau_eigs(t[0]), P->Ldx) : tau_eigs(t[0]);
  P->ly3 = tau_eigs(t[1]);
  const std::vector<double> lamc = fold_xy3(P);
  const std::vector<double> lamz = pow2 ? pos_eigs(tau_eigs(t[2]), P->Ldz) : tau_eigs(t[2]);
  const std::vector<float> lamc_f(lamc.begin(), lamc.end()), lamz_f(lamz.begin(), lamz.end());
  if (upload(P, &P->lamc64, lamc, s) != hipSuccess || upload(P, &P->lamc32, lamc_f, s) != hipSuccess ||
      upload(P, &P->lamz64, lamz, s) != hipSuccess || upload(P, &P->lamz32, lamz_f, s) != hipSuccess)
    return fail(RSFDE_ENOMEM);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(RSFDE_EHIP);
  *out = h;
  return RSFDE_OK;
}

int rsfde_set_coeffs(rsfde_plan plan, double kx, double ky) {
  if (!plan) return RSFDE_EINVAL;
  return rsfde_set_coeffs3(plan, kx, ky, plan->p.is3d ? plan->p.kz : 0.0);
}

int rsfde_set_coeffs3(rsfde_plan plan, double kx, double ky, double kz) {
  using namespace rsfde;
  if (!plan) return RSFDE_EINVAL;
  if (!(kx >= 0.0) || !(ky >= 0.0) || !(kz >= 0.0) || !std::isfinite(kx) || !std::isfinite(ky) ||
      !std::isfinite(kz))
    return RSFDE_EINVAL;
  Plan* P = &plan->p;
  if (!P->is3d) {
    if (kz != 0.0) return RSFDE_EINVAL;  // a two-dimensional plan has no z factor
    P->kx = kx;
    P->ky = ky;
    return RSFDE_OK;
  }
  P->kz = kz;  // applied at launch
  if (kx == P->kx && ky == P->ky) return RSFDE_OK;
  // the folded x/y eigenvalue table carries kx and ky: rebuild it once the
  // device has finished the work that may read it
  DeviceGuard g(P->dev);
  if (!g.ok) return RSFDE_EHIP;
  const double kx0 = P->kx, ky0 = P->ky;
  P->kx = kx;
  P->ky = ky;
  const std::vector<double> lamc = fold_xy3(P);
  const std::vector<float> lamc_f(lamc.begin(), lamc.end());
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(P->lamc64, lamc.data(), lamc.size() * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(P->lamc32, lamc_f.data(), lamc_f.size() * sizeof(float), hipMemcpyHostToDevice) !=
          hipSuccess) {
    P->kx = kx0;  // the table may be half written: the plan keeps its old k
    P->ky = ky0;
    return RSFDE_EHIP;
  }
  return RSFDE_OK;
}

int rsfde_matvec(rsfde_plan plan, const double* x, double* y, void* stream) {
  if (!plan || !x || !y || x == y) return RSFDE_EINVAL;
  Plan* P = &plan->p;
  rsfde::DeviceGuard g(P->dev);
  if (!g.ok) return RSFDE_EHIP;
  return rsfde::matvec_impl(P, x, y, rsfde::pick(P, stream));
}

int rsfde_precond_apply(rsfde_plan plan, const double* r, double* z, int32_t precision,
                        void* stream) {
  if (!plan || !r || !z || r == z) return RSFDE_EINVAL;
  if (precision < RSFDE_FP64 || precision > RSFDE_BF16) return RSFDE_EINVAL;
  Plan* P = &plan->p;
  rsfde::DeviceGuard g(P->dev);
  if (!g.ok) return RSFDE_EHIP;
  return rsfde::precond_impl(P, r, nullptr, z, precision, rsfde::pick(P, stream));
}

int rsfde_step(rsfde_plan plan, const double* u_prev, const double* u_prev2, int32_t f_kind,
               const rsfde_solver_opts* opts, double* u_next, rsfde_stats* stats, void* stream) {
  return rsfde_step_src(plan, u_prev, u_prev2, f_kind, nullptr, 0.0, opts, u_next, stats, stream);
}

int rsfde_step_src(rsfde_plan plan, const double* u_prev, const double* u_prev2, int32_t f_kind,
                   const double* src, double src_scale, const rsfde_solver_opts* opts,
                   double* u_next, rsfde_stats* stats, void* stream) {
  using namespace rsfde;
  if (!plan || !u_prev || !u_next || u_next == u_prev) return finish(stats, RSFDE_EINVAL, 0, 0, 0, 0);
  if (src && (src == u_next || !std::isfinite(src_scale))) return finish(stats, RSFDE_EINVAL, 0, 0, 0, 0);
  if (f_kind < RSFDE_F_NONE || f_kind > RSFDE_F_DECAY) return finish(stats, RSFDE_EINVAL, 0, 0, 0, 0);
  Plan* P = &plan->p;
  int rc = validate_opts(P, opts);
  if (rc) return finish(stats, rc, 0, 0, 0, 0);
  DeviceGuard g(P->dev);
  if (!g.ok) return finish(stats, RSFDE_EHIP, 0, 0, 0, 0);
  hipStream_t s = pick(P, stream);
  P->hs->flags = 0;
  {
    ProfScope ps(P, s, kCatRhs, (u_prev2 ? 33.0 : 25.0) * (double)P->N + (src ? 8.0 : 0.0) * (double)P->N);
    if (launch_rhs(u_prev, u_prev2, P->mask, P->dt, f_kind, src, src_scale, P->b, u_next, P->N,
                   P->rw, P->hs_dev, s) != hipSuccess)
      return finish(stats, RSFDE_EHIP, 0, 0, 0, 0);
  }
  return solve_core(P, u_next, opts, stats, s);
}

int rsfde_solve(rsfde_plan plan, const double* b, double* x, const rsfde_solver_opts* opts,
                rsfde_stats* stats, void* stream) {
  using namespace rsfde;
  if (!plan || !b || !x || b == x) return finish(stats, RSFDE_EINVAL, 0, 0, 0, 0);
  Plan* P = &plan->p;
  int rc = validate_opts(P, opts);
  if (rc) return finish(stats, rc, 0, 0, 0, 0);
  DeviceGuard g(P->dev);
  if (!g.ok) return finish(stats, RSFDE_EHIP, 0, 0, 0, 0);
  hipStream_t s = pick(P, stream);
  P->hs->flags = 0;
  // copy b into the plan and take its norm (f = 0, dt = 0: b = u, x0 -> scratch)
  if (launch_rhs(b, nullptr, P->mask, 0.0, RSFDE_F_NONE, nullptr, 0.0, P->b, P->t, P->N, P->rw,
                 P->hs_dev, s) != hipSuccess)
    return finish(stats, RSFDE_EHIP, 0, 0, 0, 0);
  return solve_core(P, x, opts, stats, s);
}

int rsfde_adjoint_step(rsfde_plan plan, const double* u_prev, const double* u_cur,
                       const double* lam_cur, int32_t f_kind, const rsfde_solver_opts* opts,
                       double* lam_prev, double* mu_guess, double* dk_dev, rsfde_stats* stats,
                       void* stream) {
  using namespace rsfde;
  if (!plan || !u_prev || !u_cur || !lam_cur || !lam_prev || !dk_dev || lam_prev == lam_cur)
    return finish(stats, RSFDE_EINVAL, 0, 0, 0, 0);
  if (f_kind < RSFDE_F_NONE || f_kind > RSFDE_F_DECAY) return finish(stats, RSFDE_EINVAL, 0, 0, 0, 0);
  Plan* P = &plan->p;
  int rc = validate_opts(P, opts);
  if (rc) return finish(stats, rc, 0, 0, 0, 0);
  DeviceGuard g(P->dev);
  if (!g.ok) return finish(stats, RSFDE_EHIP, 0, 0, 0, 0);
  hipStream_t s = pick(P, stream);
  double* mu = mu_guess ? mu_guess : P->mu;
  if (!mu_guess && hipMemsetAsync(mu, 0, P->N * sizeof(double), s) != hipSuccess)
    return finish(stats, RSFDE_EHIP, 0, 0, 0, 0);
  P->hs->flags = 0;
  if (launch_rhs(lam_cur, nullptr, P->mask, 0.0, RSFDE_F_NONE, nullptr, 0.0, P->b, P->t, P->N,
                 P->rw, P->hs_dev, s) != hipSuccess)
    return finish(stats, RSFDE_EHIP, 0, 0, 0, 0);
  rc = solve_core(P, mu, opts, stats, s);
  if (rc != RSFDE_OK) return rc;
  // directional derivatives of M with respect to kx, ky (and kz), dotted with
  // mu: the unit-k factors applied along each axis (3-D: y slice by slice on
  // [n3][n2][n1], z on the [n3][n1 n2] view)
  const int rows = P->n2 * P->n3, plane = P->n1 * P->n2;
  if (launch_mv_rows(P->Lcx, u_cur, P->mask, P->t, P->symx, P->tw64[P->Lcx], P->n1, rows, 1.0, 0.0,
                     1, s) != hipSuccess ||
      launch_dot_accum(mu, P->t, P->N, P->rw, 4, dk_dev, s) != hipSuccess ||
      launch_mv_cols(P->Lcy, u_cur, nullptr, P->t, P->symy, P->tw64[P->Lcy], P->n1, P->n2, 1.0, 1,
                     s, P->n3, (size_t)plane) != hipSuccess ||
      launch_dot_accum(mu, P->t, P->N, P->rw, 5, dk_dev + 1, s) != hipSuccess ||
      (P->is3d &&
       (launch_mv_cols(P->Lcz, u_cur, nullptr, P->t, P->symz, P->tw64[P->Lcz], plane, P->n3, 1.0, 1,
                       s) != hipSuccess ||
        launch_dot_accum(mu, P->t, P->N, P->rw, 6, dk_dev + 2, s) != hipSuccess)) ||
      launch_adj_lambda(mu, u_prev, P->mask, P->dt, f_kind, lam_prev, P->N, s) != hipSuccess)
    return finish(stats, RSFDE_EHIP, stats ? stats->iters : 0, 0, 0, 0);
  if (hipStreamSynchronize(s) != hipSuccess) return finish(stats, RSFDE_EHIP, 0, 0, 0, 0);
  return RSFDE_OK;
}

int rsfde_march_ensemble(int32_t count, const rsfde_plan* plans, const double* const* u0,
                         int32_t m, int32_t f_kind, const rsfde_solver_opts* opts,
                         double* const* u_out, double* const* work, rsfde_stats* stats,
                         void* const* streams) {
  if (count < 1 || !plans || !u0 || !u_out || !work || !opts || m < 0) return RSFDE_EINVAL;
  if (f_kind < RSFDE_F_NONE || f_kind > RSFDE_F_DECAY) return RSFDE_EINVAL;
  for (int i = 0; i < count; ++i) {
    if (!plans[i] || !u0[i] || !u_out[i] || !work[2 * i] || !work[2 * i + 1]) return RSFDE_EINVAL;
    const double* bufs[4] = {u0[i], u_out[i], work[2 * i], work[2 * i + 1]};
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b)
        if (bufs[a] == bufs[b]) return RSFDE_EINVAL;
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return RSFDE_EINVAL;
    const int rc = rsfde::validate_opts(&plans[i]->p, opts);
    if (rc) return rc;
  }
  std::vector<int> rcs(count, RSFDE_OK);
  auto member = [&](int i) {
    Plan* P = &plans[i]->p;
    void* st = streams ? streams[i] : nullptr;
    double* slot[3] = {u_out[i], work[2 * i], work[2 * i + 1]};
    const double* prev2 = nullptr;
    const double* prev = u0[i];
    int64_t iters = 0;
    rsfde_stats s1{};
    int last = -1;  // slot index of prev
    for (int k = 1; k <= m; ++k) {
      // a slot that holds neither u^{k-1} nor u^{k-2}; the last step writes u_out
      int nx = 0;
      if (k == m) {
        nx = 0;
      } else {
        for (nx = 0; nx < 3; ++nx)
          if (slot[nx] != prev && slot[nx] != prev2) break;
      }
      if (slot[nx] == prev || slot[nx] == prev2) {  // u_out busy: use a free work slot
        for (nx = 1; nx < 3; ++nx)
          if (slot[nx] != prev && slot[nx] != prev2) break;
      }
      const int rc = rsfde_step(plans[i], prev, prev2, f_kind, opts, slot[nx], &s1, st);
      iters += s1.iters;
      if (rc != RSFDE_OK) {
        rcs[i] = rc;
        break;
      }
      prev2 = prev;
      prev = slot[nx];
      last = nx;
    }
    if (rcs[i] == RSFDE_OK) {
      rsfde::DeviceGuard g(P->dev);
      hipStream_t s = rsfde::pick(P, st);
      if (m == 0) {
        if (hipMemcpyAsync(u_out[i], u0[i], P->N * sizeof(double), hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
          rcs[i] = RSFDE_EHIP;
      } else if (last != 0) {
        if (hipMemcpyAsync(u_out[i], slot[last], P->N * sizeof(double), hipMemcpyDeviceToDevice,
                           s) != hipSuccess)
          rcs[i] = RSFDE_EHIP;
      }
      if (rcs[i] == RSFDE_OK && hipStreamSynchronize(s) != hipSuccess) rcs[i] = RSFDE_EHIP;
    }
    if (stats) {
      stats[i] = s1;
      stats[i].iters = (int32_t)std::min<int64_t>(iters, INT32_MAX);
      stats[i].status = rcs[i];
    }
  };
  std::vector<std::thread> th;
  th.reserve(count);
  for (int i = 0; i < count; ++i) th.emplace_back(member, i);
  for (auto& t : th) t.join();
  for (int i = 0; i < count; ++i)
    if (rcs[i] != RSFDE_OK) return rcs[i];
  return RSFDE_OK;
}

int rsfde_profile(rsfde_plan plan, int32_t enable) {
  if (!plan) return RSFDE_EINVAL;
  plan->p.prof_on = enable != 0;
  return RSFDE_OK;
}

int rsfde_profile_read(rsfde_plan plan, rsfde_kernel_profile* out, int32_t max, int32_t* count) {
  using namespace rsfde;
  if (!plan || !count || (max > 0 && !out) || max < 0) return RSFDE_EINVAL;
  Plan* P = &plan->p;
  DeviceGuard g(P->dev);
  if (!g.ok) return RSFDE_EHIP;
  int64_t launches[kNumCats] = {0};
  double ms[kNumCats] = {0}, bytes[kNumCats] = {0};
  int rc = RSFDE_OK;
  for (auto& r : P->prof_recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
      rc = RSFDE_EHIP;
    launches[r.cat] += 1;
    ms[r.cat] += t;
    bytes[r.cat] += r.bytes;
    P->ev_pool.push_back(r.a);
    P->ev_pool.push_back(r.b);
  }
  P->prof_recs.clear();
  int n = 0;
  for (int c = 0; c < kNumCats; ++c) {
    if (!launches[c]) continue;
    if (n < max) {
      std::memset(&out[n], 0, sizeof(rsfde_kernel_profile));
      std::strncpy(out[n].name, kCatNames[c], sizeof(out[n].name) - 1);
      out[n].launches = launches[c];
      out[n].total_ms = ms[c];
      out[n].bytes = bytes[c];
    }
    ++n;
  }
  *count = n < max ? n : max;
  return rc;
}

int rsfde_destroy(rsfde_plan plan) {
  if (!plan) return RSFDE_OK;
  int dev = plan->p.dev;
  {
    rsfde::DeviceGuard g(dev);
    (void)hipDeviceSynchronize();
  }
  delete plan;
  return RSFDE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched independent solves (rsfde_batch_*): B members share the grid, the
// orders, the mask, eta and dt, and each has its own kx, ky, right-hand side
// and Krylov state.  Every operator and Krylov kernel runs once per step for
// all members still iterating (the members are a grid dimension of each
// launch), and the host takes one decision per inner step for the whole
// batch.  Each member owns one region of the batch allocation, the same
// layout at a fixed stride: KrylovState, reduction partials, its (kx, ky),
// the bases V and Z, b, w, t, x and the preconditioner intermediates.
// ---------------------------------------------------------------------------

struct rsfde_batch_s {
  rsfde_plan plan = nullptr;  // tables (symbols, eigenvalues, twiddles) and the mask
  int B = 0;
  size_t MS = 0;              // member stride (doubles)
  double* region = nullptr;   // B * MS doubles
  size_t o_ks = 0, o_part = 0, o_k = 0, o_V = 0, o_Z = 0, o_b = 0, o_w = 0, o_t = 0, o_x = 0,
         o_Q = 0, o_P1 = 0;
  rsfde::HostStatus* hs = nullptr;      // pinned [B]
  rsfde::HostStatus* hs_dev = nullptr;
  hipEvent_t ev = nullptr;
  std::vector<double> kx, ky;
  ~rsfde_batch_s() {
    if (region) (void)hipFree(region);
    if (hs) (void)hipHostFree(hs);
    if (ev) (void)hipEventDestroy(ev);
    if (plan) rsfde_destroy(plan);
  }
};

namespace rsfde {
namespace {

size_t r64(size_t v) { return (v + 63) / 64 * 64; }

Members members_of(const rsfde_batch_s* Bt, const std::vector<int>& ids) {
  Members mb{};
  mb.n = (int)ids.size();
  for (int k = 0; k < mb.n; ++k) mb.m[k] = ids[k];
  mb.stride = Bt->MS;
  return mb;
}

// w = M x for the members of mb (vectors at member-0 addresses of the region).
int batch_matvec(rsfde_batch_s* Bt, const double* x, double* w, const Members& mb, hipStream_t s) {
  Plan* P = &Bt->plan->p;
  const double* mk = Bt->region + Bt->o_k;
  double* t = Bt->region + Bt->o_t;
  CK(launch_mv_rows(P->Lcx, x, P->mask, t, P->symx, P->tw64[P->Lcx], P->n1, P->n2, 0.0, P->dpen, 0,
                    s, nullptr, 0.0, true, mb, mk));
  CK(launch_mv_cols(P->Lcy, x, t, w, P->symy, P->tw64[P->Lcy], P->n1, P->n2, 0.0, 0, s, 1, 0, true,
                    mb, mk + 1));
  return RSFDE_OK;
}

// The three preconditioner passes (power-of-two path) for the members of mb:
// Q, P1 from the region; with w given, the last pass is fused with the
// matrix-vector row pass and the column pass completes w = M z.
template <typename T>
int batch_precond(rsfde_batch_s* Bt, const double* v, const double* sig, double* z, double* w,
                  const Members& mb, hipStream_t s) {
  Plan* P = &Bt->plan->p;
  const double* mk = Bt->region + Bt->o_k;
  T* Q = (T*)(Bt->region + Bt->o_Q);
  T* P1 = (T*)(Bt->region + Bt->o_P1);
  auto& tw = sizeof(T) == 8 ? P->tw64 : P->tw32;
  const T* lamx = sizeof(T) == 8 ? (const T*)P->lamx64 : (const T*)P->lamx32;
  const T* lamy = sizeof(T) == 8 ? (const T*)P->lamy64 : (const T*)P->lamy32;
  const double Kfac = 4.0 / ((double)(P->n1 + 1) * (double)(P->n2 + 1));
  CK(launch_pc_rows_fwd<T>(P->Ldx, v, sig, Q, tw[P->Ldx], P->n1, P->n2, true, s, mb, sd_x<T>(P)));
  CK(launch_pc_cols<T>(P->Ldy, Q, P1, nullptr, lamx, lamy, tw[P->Ldy], P->n1, P->n2, 0.0, 0.0,
                       P->dpen, Kfac, true, s, mb, mk, sd_y<T>(P)));
  if (!w) {
    CK(launch_pc_rows_inv<T>(P->Ldx, P1, nullptr, P->mask, z, tw[P->Ldx], P->n1, P->n2, true, s,
                             mb, sd_x<T>(P)));
    return RSFDE_OK;
  }
  double* t = Bt->region + Bt->o_t;
  CK(launch_pc_rows_inv_mv<T>(P->Ldx, P1, nullptr, P->mask, z, t, tw[P->Ldx], P->tw64[P->Ldx],
                              P->symx, 0.0, P->dpen, nullptr, 0.0, P->n1, P->n2, true, s, mb, mk,
                              false, sd_x<T>(P)));
  CK(launch_mv_cols(P->Lcy, z, t, w, P->symy, P->tw64[P->Lcy], P->n1, P->n2, 0.0, 0, s, 1, 0, true,
                    mb, mk + 1));
  return RSFDE_OK;
}

int batch_precond_any(rsfde_batch_s* Bt, int precision, const double* v, const double* sig,
                      double* z, double* w, const Members& mb, hipStream_t s) {
  return precision == RSFDE_FP32 ? batch_precond<float>(Bt, v, sig, z, w, mb, s)
                                 : batch_precond<double>(Bt, v, sig, z, w, mb, s);
}

// Flexible GMRES(restart), one Arnoldi vector per step (two Gram-Schmidt
// passes unless reorth = -1), right preconditioning, for every member at once:
// the same algorithm and stopping rule as the single-plan one-vector form
// (true residual ||b - M x|| <= tol ||b|| at the start of every cycle, the
// residual estimate ending a cycle early).  b and x0 are in the region;
// hs[m].bnorm holds ||b_m||.
int batch_solve(rsfde_batch_s* Bt, const rsfde_solver_opts* o, rsfde_stats* st, hipStream_t s) {
  Plan* P = &Bt->plan->p;
  const int B = Bt->B;
  const size_t N = P->N, ld = P->ldv;
  volatile HostStatus* hs = Bt->hs;
  const bool reorth = o->reorth >= 0;
  double* R = Bt->region;
  KrylovState* ks = (KrylovState*)(R + Bt->o_ks);
  RedWork rw{R + Bt->o_part};
  double *V = R + Bt->o_V, *Zb = R + Bt->o_Z, *b = R + Bt->o_b, *w = R + Bt->o_w, *x = R + Bt->o_x;
  CK(hipStreamSynchronize(s));
  std::vector<int> total(B, 0), cycles(B, 0), status(B, RSFDE_OK);
  std::vector<double> bnorm(B), thresh(B), beta(B, 0.0);
  std::vector<int> active;
  for (int m = 0; m < B; ++m) {
    bnorm[m] = hs[m].bnorm;
    thresh[m] = o->tol * bnorm[m];
    if (hs[m].flags & kFlagNonFinite) {
      status[m] = RSFDE_ENONFINITE;
    } else if (bnorm[m] == 0.0) {
      CK(hipMemsetAsync(x + (size_t)m * Bt->MS, 0, N * sizeof(double), s));
    } else {
      active.push_back(m);
    }
  }
  while (!active.empty()) {
    const Members ma = members_of(Bt, active);
    if (int rc = batch_matvec(Bt, x, w, ma, s)) return rc;
    CK(launch_residual(b, w, V, N, rw, ks, Bt->hs_dev, s, ma));
    CK(hipStreamSynchronize(s));
    std::vector<int> iterating;
    for (int m : active) {
      beta[m] = hs[m].beta;
      if (hs[m].flags & kFlagNonFinite) status[m] = RSFDE_ENONFINITE;
      else if (beta[m] <= thresh[m]) status[m] = RSFDE_OK;
      else if (total[m] >= o->max_iters) status[m] = RSFDE_ENOTCONV;
      else {
        iterating.push_back(m);
        ++cycles[m];
      }
    }
    active = iterating;
    if (active.empty()) break;
    std::vector<int> jc(B, 0);
    for (int j = 0; j < o->restart && !iterating.empty(); ++j) {
      const Members mi = members_of(Bt, iterating);
      double* vj = V + (size_t)j * ld;
      double* zj = Zb + (size_t)j * ld;
      double* vnext = V + (size_t)(j + 1) * ld;
      if (int rc = batch_precond_any(Bt, o->precision, vj, &ks->vscale[j], zj, w, mi, s)) return rc;
      CK(launch_multidot(V, ld, j + 1, w, N, rw, ks, j, false, s, mi));
      CK(launch_axpy_givens(V, ld, j + 1, w, vnext, N, rw, ks, j, false, !reorth, Bt->hs_dev, s, mi));
      if (reorth) {
        CK(launch_multidot(V, ld, j + 1, vnext, N, rw, ks, j, true, s, mi));
        CK(launch_axpy_givens(V, ld, j + 1, vnext, vnext, N, rw, ks, j, true, true, Bt->hs_dev, s,
                              mi));
      }
      CK(hipEventRecord(Bt->ev, s));
      CK(hipEventSynchronize(Bt->ev));
      std::vector<int> still;
      for (int m : iterating) {
        ++total[m];
        const bool bad = (hs[m].flags & kFlagNonFinite) != 0;
        if (bad || hs[m].est[j] <= thresh[m] || j + 1 == o->restart || total[m] >= o->max_iters)
          jc[m] = j + 1;
        else
          still.push_back(m);
      }
      iterating = still;
    }
    std::vector<int32_t> jcs;
    int jmax = 0;
    for (int m : active) {
      jcs.push_back(jc[m]);
      jmax = std::max(jmax, jc[m]);
    }
    CK(launch_update(Zb, ld, jmax, x, N, ks, false, s, members_of(Bt, active), jcs.data()));
  }
  CK(hipStreamSynchronize(s));
  int rc_all = RSFDE_OK;
  for (int m = 0; m < B; ++m) {
    finish(st ? &st[m] : nullptr, status[m], total[m], cycles[m], beta[m], bnorm[m]);
    if (status[m] != RSFDE_OK && rc_all == RSFDE_OK) rc_all = status[m];
  }
  return rc_all;
}

// Copy B vectors between a caller array [B][N] and region slot `off`.
hipError_t batch_copy(rsfde_batch_s* Bt, double* dst, size_t dpitch, const double* src,
                      size_t spitch, hipStream_t s) {
  const size_t N = Bt->plan->p.N;
  return hipMemcpy2DAsync(dst, dpitch * sizeof(double), src, spitch * sizeof(double),
                          N * sizeof(double), (size_t)Bt->B, hipMemcpyDeviceToDevice, s);
}

}  // namespace
}  // namespace rsfde

extern "C" {

int rsfde_batch_setup(rsfde_batch* out, const rsfde_grid* grid, double alpha1, double alpha2,
                      int32_t count, const double* kx, const double* ky, const uint8_t* mask_dev,
                      double eta, double dt, int32_t max_restart, void* stream) {
  using namespace rsfde;
  if (!out) return RSFDE_EINVAL;
  *out = nullptr;
  if (!grid || !kx || !ky || !mask_dev || count < 1) return RSFDE_EINVAL;
  if (count > kMaxBatch) return RSFDE_EUNSUPPORTED;
  for (int m = 0; m < count; ++m)
    if (!(kx[m] >= 0.0) || !(ky[m] >= 0.0) || !std::isfinite(kx[m]) || !std::isfinite(ky[m]))
      return RSFDE_EINVAL;
  if (max_restart <= 0) max_restart = 30;
  if (max_restart > kMaxRestart) return RSFDE_EINVAL;
  if (grid->n1 >= 1 && grid->n2 >= 1 && (!is_pow2(grid->n1 + 1) || !is_pow2(grid->n2 + 1)))
    return RSFDE_EUNSUPPORTED;  // the batched passes are the power-of-two (odd-extension) ones
  auto* Bt = new (std::nothrow) rsfde_batch_s();
  if (!Bt) return RSFDE_ENOMEM;
  int rc = rsfde_setup(&Bt->plan, grid, alpha1, alpha2, kx[0], ky[0], mask_dev, eta, dt, 1, stream);
  if (rc) {
    delete Bt;
    return rc;
  }
  Plan* P = &Bt->plan->p;
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard g(P->dev);
  if (!g.ok) {
    delete Bt;
    return RSFDE_EHIP;
  }
  Bt->B = count;
  Bt->kx.assign(kx, kx + count);
  Bt->ky.assign(ky, ky + count);
  const size_t ld = P->ldv, n1 = P->n1, n2 = P->n2;
  const size_t slots = 8 * ((n1 + 4) / 4) * ((n2 + 1) / 2);
  const size_t pair_slots = 2 * ((n1 + 16) / 16 * 16) * n2;
  const size_t t_len = std::max(ld, 8 * ((n1 + 3) / 4) * ((n2 + 1) / 2));
  size_t o = 0;
  auto take = [&](size_t& off, size_t count_d) {
    off = o;
    o += r64(count_d);
  };
  take(Bt->o_ks, (sizeof(KrylovState) + 7) / 8);
  take(Bt->o_part, (size_t)(kMaxRestart + 2) * kMaxRedBlocks);
  take(Bt->o_k, 2);
  take(Bt->o_V, (size_t)(max_restart + 1) * ld);
  take(Bt->o_Z, (size_t)max_restart * ld);
  take(Bt->o_b, ld);
  take(Bt->o_w, ld);
  take(Bt->o_t, t_len);
  take(Bt->o_x, ld);
  take(Bt->o_Q, slots);
  take(Bt->o_P1, std::max(2 * slots, pair_slots));
  Bt->MS = o;
  if (hipMalloc((void**)&Bt->region, (size_t)count * Bt->MS * sizeof(double)) != hipSuccess) {
    Bt->region = nullptr;
    delete Bt;
    return RSFDE_ENOMEM;
  }
  if (hipHostMalloc((void**)&Bt->hs, (size_t)count * sizeof(HostStatus),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    Bt->hs = nullptr;
    delete Bt;
    return RSFDE_ENOMEM;
  }
  std::memset((void*)Bt->hs, 0, (size_t)count * sizeof(HostStatus));
  if (hipHostGetDevicePointer((void**)&Bt->hs_dev, Bt->hs, 0) != hipSuccess ||
      hipEventCreateWithFlags(&Bt->ev, hipEventDisableTiming) != hipSuccess) {
    delete Bt;
    return RSFDE_EHIP;
  }
  for (int m = 0; m < count; ++m) {
    double* base = Bt->region + (size_t)m * Bt->MS;
    const double k2[2] = {kx[m], ky[m]};
    if (hipMemsetAsync(base + Bt->o_ks, 0, sizeof(KrylovState), s) != hipSuccess ||
        hipMemcpyAsync(base + Bt->o_k, k2, sizeof(k2), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      delete Bt;
      return RSFDE_EHIP;
    }
  }
  *out = Bt;
  return RSFDE_OK;
}

int rsfde_batch_set_coeffs(rsfde_batch batch, const double* kx, const double* ky) {
  if (!batch || !kx || !ky) return RSFDE_EINVAL;
  for (int m = 0; m < batch->B; ++m)
    if (!(kx[m] >= 0.0) || !(ky[m] >= 0.0) || !std::isfinite(kx[m]) || !std::isfinite(ky[m]))
      return RSFDE_EINVAL;
  rsfde::DeviceGuard g(batch->plan->p.dev);
  if (!g.ok) return RSFDE_EHIP;
  for (int m = 0; m < batch->B; ++m) {
    const double k2[2] = {kx[m], ky[m]};
    if (hipMemcpy(batch->region + (size_t)m * batch->MS + batch->o_k, k2, sizeof(k2),
                  hipMemcpyHostToDevice) != hipSuccess)
      return RSFDE_EHIP;
    batch->kx[m] = kx[m];
    batch->ky[m] = ky[m];
  }
  return RSFDE_OK;
}

int rsfde_batch_matvec(rsfde_batch batch, const double* x, double* y, void* stream) {
  using namespace rsfde;
  if (!batch || !x || !y || x == y) return RSFDE_EINVAL;
  Plan* P = &batch->plan->p;
  DeviceGuard g(P->dev);
  if (!g.ok) return RSFDE_EHIP;
  hipStream_t s = pick(P, stream);
  std::vector<int> all(batch->B);
  for (int m = 0; m < batch->B; ++m) all[m] = m;
  double* xr = batch->region + batch->o_x;
  double* wr = batch->region + batch->o_w;
  CK(batch_copy(batch, xr, batch->MS, x, P->N, s));
  if (int rc = batch_matvec(batch, xr, wr, members_of(batch, all), s)) return rc;
  CK(batch_copy(batch, y, P->N, wr, batch->MS, s));
  return RSFDE_OK;
}

int rsfde_batch_precond_apply(rsfde_batch batch, const double* r, double* z, int32_t precision,
                              void* stream) {
  using namespace rsfde;
  if (!batch || !r || !z || r == z) return RSFDE_EINVAL;
  if (precision != RSFDE_FP64 && precision != RSFDE_FP32) return RSFDE_EUNSUPPORTED;
  Plan* P = &batch->plan->p;
  DeviceGuard g(P->dev);
  if (!g.ok) return RSFDE_EHIP;
  hipStream_t s = pick(P, stream);
  std::vector<int> all(batch->B);
  for (int m = 0; m < batch->B; ++m) all[m] = m;
  double* xr = batch->region + batch->o_x;
  double* wr = batch->region + batch->o_w;
  CK(batch_copy(batch, xr, batch->MS, r, P->N, s));
  if (int rc = batch_precond_any(batch, precision, xr, nullptr, wr, nullptr, members_of(batch, all), s))
    return rc;
  CK(batch_copy(batch, z, P->N, wr, batch->MS, s));
  return RSFDE_OK;
}

int rsfde_batch_step(rsfde_batch batch, const double* u_prev, const double* u_prev2,
                     int32_t f_kind, const rsfde_solver_opts* opts, double* u_next,
                     rsfde_stats* stats, void* stream) {
  using namespace rsfde;
  auto fail = [&](int code) {
    if (batch && stats)
      for (int m = 0; m < batch->B; ++m) finish(&stats[m], code, 0, 0, 0, 0);
    return code;
  };
  if (!batch || !u_prev || !u_next || u_next == u_prev) return fail(RSFDE_EINVAL);
  if (f_kind < RSFDE_F_NONE || f_kind > RSFDE_F_DECAY) return fail(RSFDE_EINVAL);
  Plan* P = &batch->plan->p;
  if (!opts) return fail(RSFDE_EINVAL);
  rsfde_solver_opts o = *opts;
  if (o.restart < 1 || o.restart > (int)((batch->o_Z - batch->o_V) / P->ldv) - 1)
    return fail(RSFDE_EINVAL);
  if (o.max_iters < 1 || !(o.tol > 0.0) || !std::isfinite(o.tol) || o.reorth < -1 || o.reorth > 1)
    return fail(RSFDE_EINVAL);
  if (o.precision != RSFDE_FP64 && o.precision != RSFDE_FP32) return fail(RSFDE_EUNSUPPORTED);
  if (o.precond != RSFDE_PRECOND_TAU || o.side != RSFDE_RIGHT || o.sstep > 1 ||
      o.zstore != RSFDE_ZSTORE_FP64)
    return fail(RSFDE_EUNSUPPORTED);
  DeviceGuard g(P->dev);
  if (!g.ok) return fail(RSFDE_EHIP);
  hipStream_t s = pick(P, stream);
  for (int m = 0; m < batch->B; ++m) batch->hs[m].flags = 0;
  std::vector<int> all(batch->B);
  for (int m = 0; m < batch->B; ++m) all[m] = m;
  const Members mb = members_of(batch, all);
  double* R = batch->region;
  if (launch_rhs(u_prev, u_prev2, P->mask, P->dt, f_kind, nullptr, 0.0, R + batch->o_b,
                 R + batch->o_x, P->N, RedWork{R + batch->o_part}, batch->hs_dev, s, mb, P->N) !=
      hipSuccess)
    return fail(RSFDE_EHIP);
  const int rc = batch_solve(batch, &o, stats, s);
  if (batch_copy(batch, u_next, P->N, R + batch->o_x, batch->MS, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(RSFDE_EHIP);
  return rc;
}

int rsfde_batch_destroy(rsfde_batch batch) {
  if (!batch) return RSFDE_OK;
  {
    rsfde::DeviceGuard g(batch->plan->p.dev);
    (void)hipDeviceSynchronize();
  }
  delete batch;
  return RSFDE_OK;
}

}  // extern "C"
