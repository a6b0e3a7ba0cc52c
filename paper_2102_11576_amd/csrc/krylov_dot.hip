// Fused multi-dot of the Arnoldi step (classical Gram-Schmidt projections):
// h_i = vscale[i] * <V_i, w> for i < nv in one pass over the basis, written to
// column j of the Hessenberg matrix.  The vector count is a template
// parameter, so every basis load is unconditional and the loop unrolls: all
// NV + 1 streams are in flight at once.  nv > kChunk runs in chunks.
#include "krylov_common.hpp"

namespace rsfde {

template <int NV>
__global__ __launch_bounds__(kRedThreads) void k_multidot(const double* __restrict__ V, size_t ldv,
                                                          const double* __restrict__ w, size_t N,
                                                          RedWork rw, KrylovState* ks, int j,
                                                          int v0, const Members mb) {
  __shared__ double sh[16 * NV];
  {  // member of a batched launch (grid dimension y)
    const size_t mo = mb.off(blockIdx.y);
    V += mo;
    w += mo;
    rw.partial += mo;
  }
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  const size_t N2 = N / 2;
  const double2* w2 = reinterpret_cast<const double2*>(w);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N2;
       i += (size_t)gridDim.x * blockDim.x) {
    const double2 wv = w2[i];
    double2 x[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = reinterpret_cast<const double2*>(V + (size_t)v * ldv)[i];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += x[v].x * wv.x + x[v].y * wv.y;
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const double wl = w[N - 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += V[(size_t)v * ldv + N - 1] * wl;
  }
  publish_partials<NV>(acc, NV, rw, sh);
}

// dst[v0 + v] = vscale[v0 + v] * (sum of the partials of value v), v < nv;
// dst is column j of H or the reorthogonalisation vector h2.
__global__ __launch_bounds__(kFinishThreads) void k_multidot_finish(RedWork rw, int nb, int nv,
                                                                    KrylovState* ks, double* dst,
                                                                    int v0, const Members mb) {
  {
    const size_t mo = mb.off(blockIdx.y);
    rw.partial += mo;
    ks = (KrylovState*)((double*)ks + mo);
    dst += mo;
  }
  const int lane = threadIdx.x & 63;
  for (int v = threadIdx.x >> 6; v < nv; v += kFinishThreads / 64) {
    const double t = wave_total(rw, v, nb);
    if (lane == 0) dst[v0 + v] = ks->vscale[v0 + v] * t;
  }
}

using MultidotFn = void (*)(const double*, size_t, const double*, size_t, RedWork, KrylovState*,
                            int, int, const Members&, dim3, hipStream_t);

template <int NV>
static void run_multidot(const double* V, size_t ldv, const double* w, size_t N, RedWork rw,
                         KrylovState* ks, int j, int v0, const Members& mb, dim3 g, hipStream_t s) {
  hipLaunchKernelGGL(k_multidot<NV>, g, dim3(kRedThreads), 0, s, V, ldv, w, N, rw, ks, j, v0, mb);
}
template <int... I>
static constexpr std::array<MultidotFn, sizeof...(I)> multidot_table(std::integer_sequence<int, I...>) {
  return {&run_multidot<I + 1>...};
}
static const auto kMultidot = multidot_table(std::make_integer_sequence<int, kChunk>{});

hipError_t launch_multidot(const double* V, size_t ldv, int nv, const double* w, size_t N,
                           RedWork rw, KrylovState* ks, int j, bool second, hipStream_t s,
                           const Members& mb) {
  if (nv < 1 || nv > kMaxRestart) return hipErrorInvalidValue;
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  double* dst = second ? ks->h2 : ks->H + (size_t)j * kLdH;
  for (int v0 = 0; v0 < nv; v0 += kChunk) {
    const int n = nv - v0 < kChunk ? nv - v0 : kChunk;
    const int nb = red_blocks(N);
    kMultidot[n - 1](V + (size_t)v0 * ldv, ldv, w, N, rw, ks, j, v0, mb, dim3(nb, mb.n), s);
    hipLaunchKernelGGL(k_multidot_finish, dim3(1, mb.n), dim3(kFinishThreads), 0, s, rw, nb, n, ks,
                       dst, v0, mb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rsfde
