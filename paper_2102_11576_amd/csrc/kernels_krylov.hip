// Streaming kernels of the restarted flexible GMRES (Section 5 of the paper:
// GMRES with the sine-transform preconditioner, restart length m_r) and of the
// implicit time step (right-hand side of the linear system of Section 2).
//
// Reductions are deterministic: every block reduces its share in a fixed order
// and publishes one partial per value; the last block to finish (ticket
// counter) adds the partials in block order and finishes the step (Hessenberg
// entries, Givens rotation, residual estimate).  The Krylov basis is stored
// unnormalised, v_i = vscale[i] * V_i, which removes a separate normalisation
// pass: readers apply vscale[i] on the fly.
#include <math.h>

#include "internal.hpp"

namespace rsfde {

// ------------------------------ helpers -----------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum NV per-thread values over the block; results valid in thread 0..NV-1's
// out[] (out[v] for v < nv, broadcast through LDS to all threads).
template <int NV>
__device__ __forceinline__ void block_sum(double (&acc)[NV], int nv, double* sh /* [16][NV] */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (v < nv) {
      const double s = wave_sum(acc[v]);
      if (lane == 0) sh[wid * NV + v] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (v < nv) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += sh[w * NV + v];
      acc[v] = s;
    }
  }
  __syncthreads();
}

// Publish the block's NV sums; return true in the last block, whose acc[] then
// holds the grand totals (added in block order).
template <int NV>
__device__ bool publish_and_finish(double (&acc)[NV], int nv, RedWork rw, int slot,
                                   double* sh /* [16*NV] */) {
  block_sum<NV>(acc, nv, sh);
  const int nb = gridDim.x;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (v < nv) rw.partial[(size_t)v * kMaxRedBlocks + blockIdx.x] = acc[v];
  }
  __threadfence();
  __shared__ unsigned ticket;
  if (threadIdx.x == 0) ticket = atomicAdd(&rw.counters[slot], 1u);
  __syncthreads();
  if (ticket != (unsigned)(nb - 1)) return false;
  __threadfence();
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double s = 0.0;
    if (v < nv)
      for (int k = threadIdx.x; k < nb; k += blockDim.x)
        s += rw.partial[(size_t)v * kMaxRedBlocks + k];
    acc[v] = s;
  }
  block_sum<NV>(acc, nv, sh);
  if (threadIdx.x == 0) rw.counters[slot] = 0u;  // ready for the next launch
  return true;
}

int red_blocks(size_t N) {
  size_t b = (N + (size_t)kRedThreads * 8 - 1) / ((size_t)kRedThreads * 8);
  if (b < 1) b = 1;
  if (b > (size_t)kMaxRedBlocks) b = kMaxRedBlocks;
  return (int)b;
}

__device__ __forceinline__ double f_eval(int kind, double u) {
  switch (kind) {
    case 1: return u * (1.0 - u);
    case 2: return sin(u);
    case 3: return u - u * u * u;
    default: return 0.0;
  }
}
__device__ __forceinline__ double fprime_eval(int kind, double u) {
  switch (kind) {
    case 1: return 1.0 - 2.0 * u;
    case 2: return cos(u);
    case 3: return 1.0 - 3.0 * u * u;
    default: return 0.0;
  }
}

// ------------------------------- kernels ----------------------------------

// b = u + dt * mask * f(u)  (zero extension of f outside the domain);
// x0 = 2u - u2 (u2 given) or u (first step);  ||b||^2 -> hs->bnorm.
__global__ __launch_bounds__(kRedThreads) void k_rhs(const double* __restrict__ u,
                                                     const double* __restrict__ u2,
                                                     const uint8_t* __restrict__ mask, double dt,
                                                     int f_kind, double* __restrict__ b,
                                                     double* x0, size_t N, RedWork rw,
                                                     HostStatus* hs) {
  __shared__ double sh[16 * 2];
  double acc[2] = {0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    const double ui = u[i];
    const double bi = ui + dt * (double)mask[i] * f_eval(f_kind, ui);
    const double xi = u2 ? 2.0 * ui - u2[i] : ui;
    b[i] = bi;
    x0[i] = xi;
    acc[0] += bi * bi;
    acc[1] += (isfinite(bi) && isfinite(xi)) ? 0.0 : 1.0;
  }
  if (publish_and_finish<2>(acc, 2, rw, 0, sh) && threadIdx.x == 0) {
    hs->bnorm = sqrt(acc[0]);
    if (acc[1] != 0.0 || !isfinite(acc[0])) hs->flags |= kFlagNonFinite;
    __threadfence_system();
  }
}

// r = b - w, ||r|| -> start of a restart cycle: g = (beta, 0, ...), vscale[0] = 1/beta.
__global__ __launch_bounds__(kRedThreads) void k_residual(const double* __restrict__ b,
                                                          const double* __restrict__ w,
                                                          double* __restrict__ r, size_t N,
                                                          RedWork rw, KrylovState* ks,
                                                          HostStatus* hs) {
  __shared__ double sh[16 * 1];
  double acc[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    const double ri = b[i] - w[i];
    r[i] = ri;
    acc[0] += ri * ri;
  }
  if (publish_and_finish<1>(acc, 1, rw, 1, sh) && threadIdx.x == 0) {
    const double beta = sqrt(acc[0]);
    ks->g[0] = beta;
    ks->vscale[0] = beta > 0.0 ? 1.0 / beta : 0.0;
    hs->beta = beta;
    if (!isfinite(beta)) hs->flags |= kFlagNonFinite;
    __threadfence_system();
  }
}

// h_i = vscale[i] * <V_i, w>, i < nv  ->  H[0..nv-1][j].
template <int NVMAX>
__global__ __launch_bounds__(kRedThreads) void k_multidot(const double* __restrict__ V, size_t ldv,
                                                          int nv, const double* __restrict__ w,
                                                          size_t N, RedWork rw, KrylovState* ks,
                                                          int j) {
  __shared__ double sh[16 * NVMAX];
  double acc[NVMAX];
#pragma unroll
  for (int v = 0; v < NVMAX; ++v) acc[v] = 0.0;
  const size_t N2 = N / 2;
  const double2* w2 = reinterpret_cast<const double2*>(w);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N2;
       i += (size_t)gridDim.x * blockDim.x) {
    const double2 wv = w2[i];
#pragma unroll
    for (int v = 0; v < NVMAX; ++v) {
      if (v < nv) {
        const double2 x = reinterpret_cast<const double2*>(V + (size_t)v * ldv)[i];
        acc[v] += x.x * wv.x + x.y * wv.y;
      }
    }
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const double wl = w[N - 1];
#pragma unroll
    for (int v = 0; v < NVMAX; ++v)
      if (v < nv) acc[v] += V[(size_t)v * ldv + N - 1] * wl;
  }
  if (publish_and_finish<NVMAX>(acc, nv, rw, 2, sh) && threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NVMAX; ++v)
      if (v < nv) ks->H[(size_t)j * kLdH + v] = ks->vscale[v] * acc[v];
  }
}

// V_{j+1} = w - sum_i h_i v_i (stored unnormalised), then in the last block:
// beta = ||V_{j+1}||, vscale[j+1] = 1/beta, the Givens rotations of column j,
// and the residual estimate |g_{j+1}| for the host.
template <int NVMAX>
__global__ __launch_bounds__(kRedThreads) void k_axpy_givens(const double* __restrict__ V,
                                                             size_t ldv, int nv,
                                                             const double* __restrict__ w,
                                                             double* __restrict__ vout, size_t N,
                                                             RedWork rw, KrylovState* ks, int j,
                                                             HostStatus* hs) {
  __shared__ double sh[16 * 1];
  double c[NVMAX];
#pragma unroll
  for (int v = 0; v < NVMAX; ++v)
    c[v] = (v < nv) ? ks->H[(size_t)j * kLdH + v] * ks->vscale[v] : 0.0;
  double acc[1] = {0.0};
  const size_t N2 = N / 2;
  const double2* w2 = reinterpret_cast<const double2*>(w);
  double2* o2 = reinterpret_cast<double2*>(vout);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N2;
       i += (size_t)gridDim.x * blockDim.x) {
    double2 u = w2[i];
#pragma unroll
    for (int v = 0; v < NVMAX; ++v) {
      if (v < nv) {
        const double2 x = reinterpret_cast<const double2*>(V + (size_t)v * ldv)[i];
        u.x -= c[v] * x.x;
        u.y -= c[v] * x.y;
      }
    }
    o2[i] = u;
    acc[0] += u.x * u.x + u.y * u.y;
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double u = w[N - 1];
#pragma unroll
    for (int v = 0; v < NVMAX; ++v)
      if (v < nv) u -= c[v] * V[(size_t)v * ldv + N - 1];
    vout[N - 1] = u;
    acc[0] += u * u;
  }
  // every block has read H[.][j] above, before any block can finish
  if (publish_and_finish<1>(acc, 1, rw, 3, sh) && threadIdx.x == 0) {
    double* Hj = ks->H + (size_t)j * kLdH;
    const double beta = sqrt(acc[0]);
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
}

// x += sum_{i<jc} y_i Z_i with R y = g (R = rotated Hessenberg, upper triangular).
template <int NVMAX>
__global__ __launch_bounds__(kRedThreads) void k_update(const double* __restrict__ Z, size_t ldz,
                                                        int jc, double* __restrict__ x, size_t N,
                                                        const KrylovState* __restrict__ ks) {
  __shared__ double y[kMaxRestart];
  if (threadIdx.x == 0) {
    for (int i = jc - 1; i >= 0; --i) {
      double s = ks->g[i];
      for (int k = i + 1; k < jc; ++k) s -= ks->H[(size_t)k * kLdH + i] * y[k];
      const double d = ks->H[(size_t)i * kLdH + i];
      y[i] = d != 0.0 ? s / d : 0.0;
    }
  }
  __syncthreads();
  double c[NVMAX];
#pragma unroll
  for (int v = 0; v < NVMAX; ++v) c[v] = v < jc ? y[v] : 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x) {
    double s = x[i];
#pragma unroll
    for (int v = 0; v < NVMAX; ++v)
      if (v < jc) s += c[v] * Z[(size_t)v * ldz + i];
    x[i] = s;
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

// *acc += <a, b>
__global__ __launch_bounds__(kRedThreads) void k_dot_accum(const double* __restrict__ a,
                                                           const double* __restrict__ b, size_t N,
                                                           RedWork rw, int slot, double* acc_out) {
  __shared__ double sh[16 * 1];
  double acc[1] = {0.0};
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (size_t)gridDim.x * blockDim.x)
    acc[0] += a[i] * b[i];
  if (publish_and_finish<1>(acc, 1, rw, slot, sh) && threadIdx.x == 0) *acc_out += acc[0];
}

// ------------------------------- launchers --------------------------------

hipError_t launch_rhs(const double* u, const double* u2, const uint8_t* mask, double dt,
                      int f_kind, double* b, double* x0, size_t N, RedWork rw, HostStatus* hs,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_rhs, dim3(red_blocks(N)), dim3(kRedThreads), 0, s, u, u2, mask, dt, f_kind,
                     b, x0, N, rw, hs);
  return hipGetLastError();
}

hipError_t launch_residual(const double* b, const double* w, double* r, size_t N, RedWork rw,
                           KrylovState* ks, HostStatus* hs, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(red_blocks(N)), dim3(kRedThreads), 0, s, b, w, r, N, rw, ks,
                     hs);
  return hipGetLastError();
}

hipError_t launch_multidot(const double* V, size_t ldv, int nv, const double* w, size_t N,
                           RedWork rw, KrylovState* ks, int j, hipStream_t s) {
  const dim3 g(red_blocks(N)), t(kRedThreads);
  if (nv <= 8) hipLaunchKernelGGL(k_multidot<8>, g, t, 0, s, V, ldv, nv, w, N, rw, ks, j);
  else if (nv <= 16) hipLaunchKernelGGL(k_multidot<16>, g, t, 0, s, V, ldv, nv, w, N, rw, ks, j);
  else if (nv <= 32) hipLaunchKernelGGL(k_multidot<32>, g, t, 0, s, V, ldv, nv, w, N, rw, ks, j);
  else if (nv <= 64) hipLaunchKernelGGL(k_multidot<64>, g, t, 0, s, V, ldv, nv, w, N, rw, ks, j);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_axpy_givens(const double* V, size_t ldv, int nv, const double* w, double* vout,
                              size_t N, RedWork rw, KrylovState* ks, int j, HostStatus* hs,
                              hipStream_t s) {
  const dim3 g(red_blocks(N)), t(kRedThreads);
  if (nv <= 8)
    hipLaunchKernelGGL(k_axpy_givens<8>, g, t, 0, s, V, ldv, nv, w, vout, N, rw, ks, j, hs);
  else if (nv <= 16)
    hipLaunchKernelGGL(k_axpy_givens<16>, g, t, 0, s, V, ldv, nv, w, vout, N, rw, ks, j, hs);
  else if (nv <= 32)
    hipLaunchKernelGGL(k_axpy_givens<32>, g, t, 0, s, V, ldv, nv, w, vout, N, rw, ks, j, hs);
  else if (nv <= 64)
    hipLaunchKernelGGL(k_axpy_givens<64>, g, t, 0, s, V, ldv, nv, w, vout, N, rw, ks, j, hs);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_update(const double* Z, size_t ldz, int jc, double* x, size_t N,
                         KrylovState* ks, hipStream_t s) {
  const dim3 g(red_blocks(N)), t(kRedThreads);
  if (jc <= 0) return hipSuccess;
  if (jc <= 8) hipLaunchKernelGGL(k_update<8>, g, t, 0, s, Z, ldz, jc, x, N, ks);
  else if (jc <= 16) hipLaunchKernelGGL(k_update<16>, g, t, 0, s, Z, ldz, jc, x, N, ks);
  else if (jc <= 32) hipLaunchKernelGGL(k_update<32>, g, t, 0, s, Z, ldz, jc, x, N, ks);
  else if (jc <= 64) hipLaunchKernelGGL(k_update<64>, g, t, 0, s, Z, ldz, jc, x, N, ks);
  else return hipErrorInvalidValue;
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

hipError_t launch_dot_accum(const double* a, const double* b, size_t N, RedWork rw,
                            int counter_slot, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_accum, dim3(red_blocks(N)), dim3(kRedThreads), 0, s, a, b, N, rw,
                     counter_slot, acc);
  return hipGetLastError();
}

}  // namespace rsfde
