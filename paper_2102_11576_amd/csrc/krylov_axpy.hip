// Fused update of the Arnoldi step: V_{j+1} = w - sum_i h_i v_i (stored
// unnormalised) and ||V_{j+1}||^2 in the same pass; the last block then sets
// H[j+1][j] = beta, vscale[j+1] = 1/beta, applies the previous Givens rotations
// to column j, forms rotation j (Section 5: GMRES) and publishes the residual
// estimate |g_{j+1}| for the host.  nv > kChunk runs in chunks; only the last
// chunk finishes.
#include "krylov_common.hpp"

namespace rsfde {

template <int NV, bool FINAL>
__global__ __launch_bounds__(kRedThreads) void k_axpy_givens(const double* __restrict__ V,
                                                             size_t ldv, const double* win,
                                                             double* vout, size_t N, RedWork rw,
                                                             const double* coef, int v0,
                                                             const double* vscale,
                                                             const Members mb) {
  __shared__ double sh[16 * 1];
  {  // member of a batched launch (grid dimension y)
    const size_t mo = mb.off(blockIdx.y);
    V += mo;
    win += mo;
    vout += mo;
    rw.partial += mo;
    coef += mo;
    vscale += mo;
  }
  double c[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) c[v] = coef[v0 + v] * vscale[v0 + v];
  double acc[1] = {0.0};
  const size_t N2 = N / 2;
  const double2* w2 = reinterpret_cast<const double2*>(win);
  double2* o2 = reinterpret_cast<double2*>(vout);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N2;
       i += (size_t)gridDim.x * blockDim.x) {
    double2 x[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = reinterpret_cast<const double2*>(V + (size_t)v * ldv)[i];
    double2 u = w2[i];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      u.x -= c[v] * x[v].x;
      u.y -= c[v] * x[v].y;
    }
    o2[i] = u;
    if (FINAL) acc[0] += u.x * u.x + u.y * u.y;
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double u = win[N - 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) u -= c[v] * V[(size_t)v * ldv + N - 1];
    vout[N - 1] = u;
    if (FINAL) acc[0] += u * u;
  }
  if constexpr (FINAL) publish_partials<1>(acc, 1, rw, sh);
}

// beta = ||V_{j+1}||, H[j+1][j] = beta, vscale[j+1] = 1/beta, the previous
// Givens rotations applied to column j, rotation j, and |g_{j+1}| for the host.
__global__ __launch_bounds__(kFinishThreads) void k_givens(RedWork rw, int nb, KrylovState* ks,
                                                           int j, int add_h2, HostStatus* hs,
                                                           const Members mb) {
  if ((threadIdx.x >> 6) > 0) return;
  rw.partial += mb.off(blockIdx.y);
  ks = (KrylovState*)((double*)ks + mb.off(blockIdx.y));
  hs += mb.m[blockIdx.y];
  const double uu = wave_total(rw, 0, nb);
  if (threadIdx.x != 0) return;
  double* Hj = ks->H + (size_t)j * kLdH;
  if (add_h2)
    for (int i = 0; i <= j; ++i) Hj[i] += ks->h2[i];
  const double beta = sqrt(uu);
  Hj[j + 1] = beta;
  ks->vscale[j + 1] = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int i = 0; i < j; ++i) {
    const double a = Hj[i], bb = Hj[i + 1];
    Hj[i] = ks->cs[i] * a + ks->sn[i] * bb;
    Hj[i + 1] = -ks->sn[i] * a + ks->cs[i] * bb;
  }
  const double a = Hj[j], bb = Hj[j + 1];
  const double den = hypot(a, bb);
  const double cs = den > 0.0 ? a / den : 1.0;
  const double sn = den > 0.0 ? bb / den : 0.0;
  ks->cs[j] = cs;
  ks->sn[j] = sn;
  Hj[j] = den;
  Hj[j + 1] = 0.0;
  const double gj = ks->g[j];
  ks->g[j] = cs * gj;
  ks->g[j + 1] = -sn * gj;
  hs->est[j] = fabs(ks->g[j + 1]);
  if (!isfinite(beta) || !isfinite(den) || !isfinite(gj)) hs->flags |= kFlagNonFinite;
  __threadfence_system();
}

using AxpyFn = void (*)(const double*, size_t, const double*, double*, size_t, RedWork,
                        const double*, int, const double*, const Members&, dim3, hipStream_t);

template <int NV, bool FINAL>
static void run_axpy(const double* V, size_t ldv, const double* win, double* vout, size_t N,
                     RedWork rw, const double* coef, int v0, const double* vscale,
                     const Members& mb, dim3 g, hipStream_t s) {
  hipLaunchKernelGGL((k_axpy_givens<NV, FINAL>), g, dim3(kRedThreads), 0, s, V, ldv, win, vout, N,
                     rw, coef, v0, vscale, mb);
}
template <bool FINAL, int... I>
static constexpr std::array<AxpyFn, sizeof...(I)> axpy_table(std::integer_sequence<int, I...>) {
  return {&run_axpy<I + 1, FINAL>...};
}
static const auto kAxpyFinal = axpy_table<true>(std::make_integer_sequence<int, kChunk>{});
static const auto kAxpyPart = axpy_table<false>(std::make_integer_sequence<int, kChunk>{});

hipError_t launch_axpy_givens(const double* V, size_t ldv, int nv, const double* w, double* vout,
                              size_t N, RedWork rw, KrylovState* ks, int j, bool second,
                              bool finish, HostStatus* hs, hipStream_t s, const Members& mb) {
  if (nv < 1 || nv > kMaxRestart) return hipErrorInvalidValue;
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  const double* coef = second ? ks->h2 : ks->H + (size_t)j * kLdH;
  for (int v0 = 0; v0 < nv; v0 += kChunk) {
    const int n = nv - v0 < kChunk ? nv - v0 : kChunk;
    const bool last = finish && v0 + n == nv;
    const double* win = v0 == 0 ? w : vout;
    const int nb = red_blocks(N);
    (last ? kAxpyFinal : kAxpyPart)[n - 1](V + (size_t)v0 * ldv, ldv, win, vout, N, rw, coef, v0,
                                           ks->vscale, mb, dim3(nb, mb.n), s);
    if (last)
      hipLaunchKernelGGL(k_givens, dim3(1, mb.n), dim3(kFinishThreads), 0, s, rw, nb, ks, j,
                         second ? 1 : 0, hs, mb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rsfde
