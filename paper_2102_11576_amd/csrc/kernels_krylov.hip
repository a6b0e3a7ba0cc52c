// Streaming kernels of the restarted flexible GMRES (Section 5 of the paper:
// GMRES with the sine-transform preconditioner, restart length m_r) and of the
// implicit time step (right-hand side of the linear system of Section 2).
//
// Reductions are deterministic: every block reduces its share in a fixed order
// and publishes one partial per value; a one-block finishing kernel launched
// next adds the partials in block order and finishes the step (norms,
// Hessenberg entries, Givens rotation, residual estimate).  The Krylov basis is stored
// unnormalised, v_i = vscale[i] * V_i, which removes a separate normalisation
// pass: readers apply vscale[i] on the fly.
#include "krylov_common.hpp"

namespace rsfde {

int stream_blocks(size_t N) {
  size_t b = (N / 2 + (size_t)kRedThreads - 1) / (size_t)kRedThreads;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

int red_blocks(size_t N) {
  size_t b = (N + (size_t)kRedThreads * 16 - 1) / ((size_t)kRedThreads * 16);
  if (b < 16) {  // small vectors: one element pair per thread, up to 16 blocks
    const size_t m = (N + (size_t)kRedThreads * 2 - 1) / ((size_t)kRedThreads * 2);
    b = m < 16 ? m : 16;
  }
  if (b < 1) b = 1;
  if (b > (size_t)kMaxRedBlocks) b = kMaxRedBlocks;
  return (int)b;
}

__device__ __forceinline__ double f_eval(int kind, double u) {
  switch (kind) {
    case 1: return u * (1.0 - u);
    case 2: return sin(u);
    case 3: return u - u * u * u;
    case 4: return -u;
    default: return 0.0;
  }
}
__device__ __forceinline__ double fprime_eval(int kind, double u) {
  switch (kind) {
    case 1: return 1.0 - 2.0 * u;
    case 2: return cos(u);
    case 3: return 1.0 - 3.0 * u * u;
    case 4: return -1.0;
    default: return 0.0;
  }
}

// ------------------------------- kernels ----------------------------------

// b = u + dt * mask * (f(u) + src_scale * src)  (zero extension of the source
// outside the domain; src = NULL means no field term); x0 = 2u - u2 (u2 given)
// or u (first step); partials of ||b||^2 and of the count of non-finite values.
__global__ __launch_bounds__(kRedThreads) void k_rhs(const double* __restrict__ u,
                                                     const double* __restrict__ u2,
                                                     const uint8_t* __restrict__ mask, double dt,
                                                     int f_kind, const double* __restrict__ src,
                                                     double src_scale, double* __restrict__ b,
                                                     double* x0, size_t N, RedWork rw,
                                                     const Members mb, size_t ustride) {
  __shared__ double sh[16 * 2];
  {  // member of a batched launch (grid dimension y)
    const size_t mo = mb.off(blockIdx.y), uo = (size_t)mb.m[blockIdx.y] * ustride;
    u += uo;
    if (u2) u2 += uo;
    if (src) src += uo;
    b += mo;
    x0 += mo;
    rw.partial += mo;
  }
  double acc[2] = {0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    const double ui = u[i];
    double fi = f_eval(f_kind, ui);
    if (src) fi += src_scale * src[i];
    const double bi = ui + dt * (double)mask[i] * fi;
    const double xi = u2 ? 2.0 * ui - u2[i] : ui;
    b[i] = bi;
    x0[i] = xi;
    acc[0] += bi * bi;
    acc[1] += (isfinite(bi) && isfinite(xi)) ? 0.0 : 1.0;
  }
  publish_partials<2>(acc, 2, rw, sh);
}

__global__ __launch_bounds__(kFinishThreads) void k_rhs_finish(RedWork rw, int nb, HostStatus* hs,
                                                               const Members mb) {
  rw.partial += mb.off(blockIdx.y);
  hs += mb.m[blockIdx.y];
  const int wv = threadIdx.x >> 6;
  if (wv > 0) return;
  const double bb = wave_total(rw, 0, nb);
  const double bad = wave_total(rw, 1, nb);
  if (threadIdx.x == 0) {
    hs->bnorm = sqrt(bb);
    if (bad != 0.0 || !isfinite(bb)) hs->flags |= kFlagNonFinite;
    __threadfence_system();
  }
}

// r = b - w and partials of ||r||^2.
__global__ __launch_bounds__(kRedThreads) void k_residual(const double* __restrict__ b,
                                                          const double* __restrict__ w,
                                                          double* __restrict__ r, size_t N,
                                                          RedWork rw, const Members mb) {
  __shared__ double sh[16 * 1];
  {
    const size_t mo = mb.off(blockIdx.y);
    b += mo;
    w += mo;
    r += mo;
    rw.partial += mo;
  }
  double acc[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    const double ri = b[i] - w[i];
    r[i] = ri;
    acc[0] += ri * ri;
  }
  publish_partials<1>(acc, 1, rw, sh);
}

// Start of a restart cycle: beta = ||r||, g = (beta, 0, ...), vscale[0] = 1/beta.
__global__ __launch_bounds__(kFinishThreads) void k_residual_finish(RedWork rw, int nb,
                                                                    KrylovState* ks,
                                                                    HostStatus* hs,
                                                                    const Members mb) {
  if ((threadIdx.x >> 6) > 0) return;
  rw.partial += mb.off(blockIdx.y);
  ks = (KrylovState*)((double*)ks + mb.off(blockIdx.y));
  hs += mb.m[blockIdx.y];
  const double rr = wave_total(rw, 0, nb);
  if (threadIdx.x == 0) {
    const double beta = sqrt(rr);
    ks->g[0] = beta;
    ks->vscale[0] = beta > 0.0 ? 1.0 / beta : 0.0;
    hs->beta = beta;
    if (!isfinite(beta)) hs->flags |= kFlagNonFinite;
    __threadfence_system();
  }
}

__global__ void k_scale_copy(const double* __restrict__ v, const double* __restrict__ sig,
                             double* __restrict__ z, size_t N) {
  const double s = sig ? *sig : 1.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x)
    z[i] = s * v[i];
}

// lambda^{k-1} = mu + dt * mask * f'(u^{k-1}) * mu
__global__ void k_adj_lambda(const double* __restrict__ mu, const double* __restrict__ u_prev,
                             const uint8_t* __restrict__ mask, double dt, int f_kind,
                             double* __restrict__ lam, size_t N) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    const double m = mu[i];
    lam[i] = m + dt * (double)mask[i] * fprime_eval(f_kind, u_prev[i]) * m;
  }
}

// partials of <a, b>
__global__ __launch_bounds__(kRedThreads) void k_dot(const double* __restrict__ a,
                                                     const double* __restrict__ b, size_t N,
                                                     RedWork rw) {
  __shared__ double sh[16 * 1];
  double acc[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x)
    acc[0] += a[i] * b[i];
  publish_partials<1>(acc, 1, rw, sh);
}

// hs->bnorm = sqrt(<a, a>) from k_dot partials
__global__ __launch_bounds__(kFinishThreads) void k_norm_finish(RedWork rw, int nb, HostStatus* hs) {
  if ((threadIdx.x >> 6) > 0) return;
  const double d = wave_total(rw, 0, nb);
  if (threadIdx.x == 0) {
    hs->bnorm = sqrt(d);
    if (!isfinite(d)) hs->flags |= kFlagNonFinite;
    __threadfence_system();
  }
}

// *acc_out += <a, b>
__global__ __launch_bounds__(kFinishThreads) void k_dot_finish(RedWork rw, int nb, double* acc_out) {
  if ((threadIdx.x >> 6) > 0) return;
  const double d = wave_total(rw, 0, nb);
  if (threadIdx.x == 0) *acc_out += d;
}

// ------------------------------- launchers --------------------------------

hipError_t launch_rhs(const double* u, const double* u2, const uint8_t* mask, double dt,
                      int f_kind, const double* src, double src_scale, double* b, double* x0,
                      size_t N, RedWork rw, HostStatus* hs, hipStream_t s, const Members& mb,
                      size_t ustride) {
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  const int nb = red_blocks(N);
  hipLaunchKernelGGL(k_rhs, dim3(nb, mb.n), dim3(kRedThreads), 0, s, u, u2, mask, dt, f_kind, src,
                     src_scale, b, x0, N, rw, mb, ustride);
  hipLaunchKernelGGL(k_rhs_finish, dim3(1, mb.n), dim3(kFinishThreads), 0, s, rw, nb, hs, mb);
  return hipGetLastError();
}

hipError_t launch_residual(const double* b, const double* w, double* r, size_t N, RedWork rw,
                           KrylovState* ks, HostStatus* hs, hipStream_t s, const Members& mb) {
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  const int nb = red_blocks(N);
  hipLaunchKernelGGL(k_residual, dim3(nb, mb.n), dim3(kRedThreads), 0, s, b, w, r, N, rw, mb);
  hipLaunchKernelGGL(k_residual_finish, dim3(1, mb.n), dim3(kFinishThreads), 0, s, rw, nb, ks, hs,
                     mb);
  return hipGetLastError();
}

hipError_t launch_scale_copy(const double* v, const double* sig, double* z, size_t N,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(red_blocks(N)), dim3(kRedThreads), 0, s, v, sig, z, N);
  return hipGetLastError();
}

hipError_t launch_adj_lambda(const double* mu, const double* u_prev, const uint8_t* mask,
                             double dt, int f_kind, double* lam_prev, size_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_lambda, dim3(red_blocks(N)), dim3(kRedThreads), 0, s, mu, u_prev, mask,
                     dt, f_kind, lam_prev, N);
  return hipGetLastError();
}

hipError_t launch_norm(const double* v, size_t N, RedWork rw, HostStatus* hs, hipStream_t s) {
  const int nb = red_blocks(N);
  hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kRedThreads), 0, s, v, v, N, rw);
  hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(kFinishThreads), 0, s, rw, nb, hs);
  return hipGetLastError();
}

hipError_t launch_dot_accum(const double* a, const double* b, size_t N, RedWork rw,
                            int /*counter_slot*/, double* acc, hipStream_t s) {
  const int nb = red_blocks(N);
  hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kRedThreads), 0, s, a, b, N, rw);
  hipLaunchKernelGGL(k_dot_finish, dim3(1), dim3(kFinishThreads), 0, s, rw, nb, acc);
  return hipGetLastError();
}

}  // namespace rsfde
