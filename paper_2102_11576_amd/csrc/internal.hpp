// Internal declarations shared by the host driver and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fft_engine.hpp"

namespace rsfde {

constexpr int kMaxRestart = 64;       // largest GMRES restart length supported
constexpr int kRedThreads = 256;      // threads per block of the streaming reductions
constexpr int kMaxRedBlocks = 512;    // upper bound on blocks of a streaming reduction
constexpr int kMaxN = 4096;           // grid points per direction (FFT lengths <= 8192)

// Members of a batched launch (independent solves of one grid, rsfde_batch_*):
// slot k of the launch's member grid dimension works on member m[k], whose
// per-member arrays start m[k] * stride doubles after the pointers the launch
// is given.  A single plan launches one member with stride 0.
constexpr int kMaxBatch = 32;
struct Members {
  int32_t n;             // members in the launch (grid dimension z of the FFT
                         // kernels, y of the streaming Krylov kernels)
  int32_t m[kMaxBatch];  // their member indices
  size_t stride;         // doubles between consecutive members' arrays
  __host__ __device__ size_t off(int k) const { return (size_t)m[k] * stride; }
  static Members one() {
    Members b{};
    b.n = 1;
    return b;
  }
};

// Points per thread of the register-resident FFT of length L: 16, except 8 at
// L = 1024.  At L = 8192, 16 points make a transform 512 threads, two blocks
// per CU by their LDS, in four register stages where 8 points take five.  At
// L = 1024 (grids of at most 511 lines, too few blocks to fill the GPU) 8
// points give each block twice the threads.
constexpr int fft_pts(int L) { return L < 16 ? L : (L == 1024 ? 8 : 16); }
// Points per thread in pass B of the power-of-two preconditioner.
constexpr int pc_cols_pts(int L) { return L < 16 ? L : 16; }

// Values the device writes for the host after each Arnoldi step.  Lives in
// pinned, device-visible host memory; the host reads it after an event.
struct HostStatus {
  double est[kMaxRestart];  // |g_{j+1}|: residual-norm estimate after inner step j
  double beta;              // ||r|| of the last residual kernel
  double bnorm;             // ||b||
  int32_t flags;            // bit 0: non-finite value seen
  int32_t gram_seq;         // sequence number of the last Gram block written (s-step form)
};
constexpr int kFlagNonFinite = 1;

// Device-side Arnoldi / Givens state.
struct KrylovState {
  double H[(kMaxRestart + 1) * kMaxRestart];  // column-major, ld = kMaxRestart + 1
  double cs[kMaxRestart];
  double sn[kMaxRestart];
  double g[kMaxRestart + 1];
  double vscale[kMaxRestart + 1];             // V_i is stored unnormalised: v_i = vscale[i] * V_i
  double h2[kMaxRestart + 1];                 // second Gram-Schmidt pass (reorthogonalisation)
  int32_t gram_done;                          // blocks of a Gram finish done (0 between launches)
};
constexpr int kLdH = kMaxRestart + 1;

// Reduction workspace: per-block partial sums [value][block], read by the
// single-block finishing kernel launched after each streaming kernel.
struct RedWork {
  double* partial;     // [kMaxRestart + 2][kMaxRedBlocks]
};

// ----------------------------- FFT kernels --------------------------------
// Row pass of the matrix-vector product:
//   out = coef * (C_x z) + diag * z - theta * sub,
//   diag = (mode==0) ? 1 + dpen (1 - mask) : 0 (sub = NULL: no shift term),
// where C_x is the Toeplitz matrix whose circulant embedding of length L has
// the symbol `sym` (already divided by L, stored in register-position order).
// tiled: out in the strip-tiled layout (tile_index; 8 ceil(n1/4) ceil(n2/2)
// values), as the column pass reads t on two-dimensional plans.
// Batched (mb.n > 1 or a nonzero stride): z, out and sub advance by the
// member offset; with mk given, coef = -mk[offset] (mk: the member's k).
hipError_t launch_mv_rows(int L, const double* z, const uint8_t* mask, double* out,
                          const double* sym, const void* tw, int n1, int n2,
                          double coef, double dpen, int mode, hipStream_t s,
                          const double* sub = nullptr, double theta = 0.0, bool tiled = false,
                          const Members& mb = Members::one(), const double* mk = nullptr);
// Column pass: out = coef * (C_y z) + (mode==0 ? t : 0) on `batch` [n2][n1]
// slices, slice b at offset b * bstride of z, t and out.  tiled (mode 0, one
// slice): t in the strip-tiled layout.
// z32 (mode 0, tiled, one slice): z is a float array (the preconditioned
// basis kept in FP32).
hipError_t launch_mv_cols(int L, const void* z, const double* t, double* out,
                          const double* sym, const void* tw, int n1, int n2,
                          double coef, int mode, hipStream_t s, int batch = 1,
                          size_t bstride = 0, bool tiled = false,
                          const Members& mb = Members::one(), const double* mk = nullptr,
                          bool z32 = false);

// Tables of the symmetric sine transform along one direction (sd_kernels.hpp;
// used by the tiled passes when L >= kSdMinL and twS is given): twS, the
// twiddles exp(-2 pi i j / (L/16)) in the pass's precision; msl (x only), the
// mirror slots of the upper halves of blocks 0 and 8 (2 L/16 entries, -1 at
// frequency L/2).  With the symmetric form the x slots follow Sd<L>::slot and
// pass B's y eigenvalues are indexed by block position (9 L/16 entries).
struct SdTabs {
  const void* twS = nullptr;
  const int32_t* msl = nullptr;
};

// Sine-transform preconditioner, three passes; T = float or double internally.
// tiled = false: Q, P1, P2 are [n2][n1+1] arrays.  tiled = true: Q is
// strip-tiled (tile_index; 8 ceil((n1+1)/4) ceil(n2/2) T values) and the
// interleaved P1/P2 pairs (array P1, P2 unused) are in row segments
// (pair_index; 2 W ceil((n1+1)/W) n2 T values, W = 64 / sizeof(T)).
// Pass A: Q[r][slot] = raw x-sine sums of (sig * v) rows.
// Batched: v, sig (when given), Q advance by the member offset (in doubles).
template <typename T>
hipError_t launch_pc_rows_fwd(int Lx, const double* v, const double* sig, T* Q,
                              const void* tw, int n1, int n2, bool tiled, hipStream_t s,
                              const Members& mb = Members::one(), const SdTabs& sd = SdTabs{});
// Pass B: column sine transforms of Q, the two eigenvalue scalings, two inverse
// column transforms -> P1, P2 (slot layout in x, natural rows in y).
// Batched: Q, P1, P2 advance by the member offset; with mk given, the
// member's (kx, ky) are mk[offset], mk[offset + 1].
template <typename T>
hipError_t launch_pc_cols(int Ly, const T* Q, T* P1, T* P2, const T* lamx_slot,
                          const T* lamy_pos, const void* tw, int n1, int n2,
                          double kx, double ky, double dpen, double Kfac, bool tiled,
                          hipStream_t s, const Members& mb = Members::one(),
                          const double* mk = nullptr, const SdTabs& sd = SdTabs{});
// Raw sine transform (DST-I without normalisation) along the columns of
// `batch` slices of [rows][ld] values (slice b at offset b * bstride):
//   outA[k-1][ca] = sum_{p=1..rows} inA[p-1][ca] sin(pi k p / (rows + 1)), k = 1..rows,
// and likewise inB column cb -> outB, with ca = c * cstride, cb = ca + coff for
// c = 0..ncol-1 (cstride 2, coff 1: adjacent column pairs of one array;
// cstride 1, coff 0: the same column of two arrays).  L = 2 (rows + 1).
template <typename T>
hipError_t launch_dst_cols(int L, const T* inA, const T* inB, T* outA, T* outB, const void* tw,
                           int ncol, int cstride, int coff, int rows, int ld, int batch,
                           size_t bstride, hipStream_t s);
// Pass C: inverse row transforms of P1, P2 and the mask combine -> z (FP64).
template <typename T>
hipError_t launch_pc_rows_inv(int Lx, const T* P1, const T* P2,
                              const uint8_t* mask, double* z, const void* tw,
                              int n1, int n2, bool tiled, hipStream_t s,
                              const Members& mb = Members::one(), const SdTabs& sd = SdTabs{});

// Pass C fused with the matrix-vector row pass (n1 + 1 a power of two, so
// L = 2(n1+1) is also the convolution length): z = pass C output (stored),
// t = (1 + dpen (1 - mask)) z + coef (C_x z) - theta sub (sub may be NULL);
// tiled: P1/P2 pairs in row segments, t strip-tiled over n1 columns.
// Batched: P1, P2, z, t, sub advance by the member offset; with mk given,
// coef = -mk[offset].  z32: z is stored in FP32 (a float array; tiled only),
// and the product uses the stored (rounded) values.
template <typename T>
hipError_t launch_pc_rows_inv_mv(int L, const T* P1, const T* P2,
                                 const uint8_t* mask, void* z, double* t, const void* twT,
                                 const void* tw64, const double* sym, double coef, double dpen,
                                 const double* sub, double theta, int n1, int n2, bool tiled,
                                 hipStream_t s, const Members& mb = Members::one(),
                                 const double* mk = nullptr, bool z32 = false,
                                 const SdTabs& sd = SdTabs{});

// Chirp (Bluestein) form of the same preconditioner for any n (n + 1 not a
// power of two): T internals, tables chn (n entries) and khat (L entries, in
// register-position order) per direction; W1 holds n1*n2 T values, Y1 and Y2
// likewise.  L >= 2n - 1 is the convolution length of that direction.
template <typename T>
hipError_t launch_cd_rows_fwd(int L, const double* v, const double* sig, T* W1, const void* chn,
                              const void* khat, const void* tw, int n1, int n2, hipStream_t s);
template <typename T>
hipError_t launch_cd_cols(int L, const T* W1, T* Y1, T* Y2, const double* lamx,
                          const double* lamy, const void* chn, const void* khat, const void* tw,
                          int n1, int n2, double kx, double ky, double dpen, hipStream_t s);
template <typename T>
hipError_t launch_cd_rows_inv(int L, const T* Y1, const T* Y2, const uint8_t* mask, double* z,
                              const void* chn, const void* khat, const void* tw, int n1, int n2,
                              hipStream_t s);
// Three-dimensional plans: out = S in along the rows of `batch` slices of
// [rows][ncol] T values (slice b at offset b * bstride, the columns c < ncol);
// inB / outB (both or neither): a second array in the same launch.
template <typename T>
hipError_t launch_cd_dst_cols(int L, const T* inA, T* outA, const T* inB, T* outB, const void* chn,
                              const void* khat, const void* tw, int ncol, int rows, int batch,
                              size_t bstride, hipStream_t s);

// BF16 / MFMA form of the same preconditioner (dense sine-transform GEMMs,
// any n; dimensions padded to multiples of 128).  A1T holds 2 n1p n2p values
// (hi and lo parts of the split intermediate).
hipError_t launch_pc_gemm_bf16(const double* v, const double* sig, double* z, const uint8_t* mask,
                               const __bf16* Sx, const __bf16* Sy, const __bf16* Sx_lo,
                               const __bf16* Sy_lo, const float* lamx,
                               const float* lamy, __bf16* A1T, __bf16* R12T, __bf16* G,
                               int n1, int n2, int n1p, int n2p, double kx, double ky,
                               double dpen, hipStream_t s);

// ---------------------------- Krylov kernels ------------------------------
// b = u + dt * mask * (f(u) + src_scale * src)  (src may be NULL), x0 = 2u - u2
// (or u), ||b|| -> hs->bnorm.
// Batched (Krylov kernels): every per-member pointer (vectors, bases, the
// KrylovState, the reduction partials) advances by the member offset, and hs
// is an array indexed by member; u and u2 advance by ustride per member.
hipError_t launch_rhs(const double* u, const double* u2, const uint8_t* mask, double dt,
                      int f_kind, const double* src, double src_scale, double* b, double* x0,
                      size_t N, RedWork rw, HostStatus* hs, hipStream_t s,
                      const Members& mb = Members::one(), size_t ustride = 0);
// ||v|| -> hs->bnorm.
hipError_t launch_norm(const double* v, size_t N, RedWork rw, HostStatus* hs, hipStream_t s);
hipError_t launch_residual(const double* b, const double* w, double* r, size_t N,
                           RedWork rw, KrylovState* ks, HostStatus* hs, hipStream_t s,
                           const Members& mb = Members::one());
// h_i = <v_i, w>, i < nv, into column j of H (second = false) or into ks->h2
// (second = true: the reorthogonalisation pass).
hipError_t launch_multidot(const double* V, size_t ldv, int nv, const double* w, size_t N,
                           RedWork rw, KrylovState* ks, int j, bool second, hipStream_t s,
                           const Members& mb = Members::one());
// vout = w - sum_i c_i v_i with c = column j of H (second = false) or ks->h2;
// finish = true also takes ||vout|| and does the Givens step (adding h2 into
// column j first when second = true).
hipError_t launch_axpy_givens(const double* V, size_t ldv, int nv, const double* w,
                              double* vout, size_t N, RedWork rw, KrylovState* ks, int j,
                              bool second, bool finish, HostStatus* hs, hipStream_t s,
                              const Members& mb = Members::one());
// x += sum_{i<jc} y_i Z_i with R y = g; scaled = true multiplies y_i by
// vscale[i] (Z = the unnormalised basis V: left preconditioning).
// Batched: member slot k uses jc[k] vectors (jcs given; jc = their maximum).
// z32: Z is a float array (vector i at Z + i * ldz floats).
hipError_t launch_update(const void* Z, size_t ldz, int jc, double* x, size_t N,
                         KrylovState* ks, bool scaled, hipStream_t s,
                         const Members& mb = Members::one(), const int32_t* jcs = nullptr,
                         bool z32 = false);
// x += sum_{i<jc} c_i Z_i with the coefficients c given (device array).
// As launch_update with the coefficients y given on the host (jc doubles,
// passed to the kernels as arguments).
hipError_t launch_update_coef(const void* Z, size_t ldz, int jc, double* x, size_t N,
                              const double* c_host, hipStream_t s, bool z32 = false);

// s-step blocks (krylov_block.hip).  G (pinned, device-visible, [nr][16]) =
// [V_0 .. V_{nr-1}]^T [V_{m1} .. V_{m1+s-1}]; gpart holds
// 16 * 16 * kGramMaxTiles * kGramBlocks partial sums.
constexpr int kGramBlocks = 1024;
constexpr int kGramMaxTiles = 5;  // up to 80 Gram rows
// After G is written and fenced, the finishing kernel stores seq to *seq_flag
// (pinned host memory), so that the host can wait for G by polling that word.
// done_count: a device word that is 0 between launches (the finishing
// kernel's blocks count themselves on it and the last one resets it).
hipError_t launch_bgram(const double* V, size_t ld, int nr, int m1, int s, size_t N,
                        double* gpart, double* G_host_dev, int32_t* seq_flag, int32_t seq,
                        int32_t* done_count, hipStream_t st);
// V_{m1..m1+s-1} <- (V_{m1..} - V_{0..nq-1} C) R^{-1}; coef = C [nq][s] then R^{-1} [s][s]
// (nq*s + s*s doubles).  Up to kCoefArgMax coefficients travel as kernel
// arguments (coef is then a host pointer); more are read from coef_dev, which
// the caller has filled on the stream.
constexpr int kCoefArgMax = 448;
struct CoefArgs {
  double v[kCoefArgMax];
};
hipError_t launch_bupd(double* V, size_t ld, int nq, int m1, int s, size_t N, const double* coef,
                       const double* coef_dev, hipStream_t st);
hipError_t launch_scale_copy(const double* v, const double* sig, double* z, size_t N,
                             hipStream_t s);
hipError_t launch_adj_lambda(const double* mu, const double* u_prev, const uint8_t* mask,
                             double dt, int f_kind, double* lam_prev, size_t N, hipStream_t s);
hipError_t launch_dot_accum(const double* a, const double* b, size_t N, RedWork rw,
                            int counter_slot, double* acc, hipStream_t s);

int red_blocks(size_t N);
// Grid of a streaming kernel without a cross-block reduction (grid-stride
// loops over double2 pairs): up to 4096 blocks, for memory-level parallelism.
int stream_blocks(size_t N);

}  // namespace rsfde
