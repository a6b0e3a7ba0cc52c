// Solution update at the end of a restart cycle:
// x += sum_{i<jc} y_i Z_i with R y = g (R = the rotated, upper-triangular
// Hessenberg matrix).  Z is the preconditioned basis of the flexible GMRES, or
// (scaled = true) the unnormalised Arnoldi basis V of left preconditioning,
// whose vectors carry the factors vscale[i].  Every block solves the small
// triangular system itself.
#include "krylov_common.hpp"

namespace rsfde {

// Coefficients given by the host, passed as a kernel argument.
struct UpdateCoef {
  double v[kMaxRestart];
};

template <int NV>
__global__ __launch_bounds__(kRedThreads) void k_update(const double* __restrict__ Z, size_t ldz,
                                                        double* __restrict__ x, size_t N,
                                                        const KrylovState* __restrict__ ks,
                                                        int v0, int jc, bool scaled, bool given,
                                                        const UpdateCoef cgiven) {
  __shared__ double y[kMaxRestart];
  if (given) {
    if (threadIdx.x < NV) y[v0 + threadIdx.x] = cgiven.v[v0 + threadIdx.x];
  } else if (threadIdx.x == 0) {
    for (int i = jc - 1; i >= 0; --i) {
      double s = ks->g[i];
      for (int k = i + 1; k < jc; ++k) s -= ks->H[(size_t)k * kLdH + i] * y[k];
      const double d = ks->H[(size_t)i * kLdH + i];
      y[i] = d != 0.0 ? s / d : 0.0;
    }
  }
  __syncthreads();
  double c[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) c[v] = y[v0 + v] * (scaled && !given ? ks->vscale[v0 + v] : 1.0);
  const size_t N2 = N / 2;
  double2* x2 = reinterpret_cast<double2*>(x);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N2;
       i += (size_t)gridDim.x * blockDim.x) {
    double2 z[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) z[v] = reinterpret_cast<const double2*>(Z + (size_t)v * ldz)[i];
    double2 s = x2[i];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      s.x += c[v] * z[v].x;
      s.y += c[v] * z[v].y;
    }
    x2[i] = s;
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double s = x[N - 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) s += c[v] * Z[(size_t)v * ldz + N - 1];
    x[N - 1] = s;
  }
}

using UpdateFn = void (*)(const double*, size_t, double*, size_t, const KrylovState*, int, int,
                          bool, bool, const UpdateCoef&, dim3, hipStream_t);
template <int NV>
static void run_update(const double* Z, size_t ldz, double* x, size_t N, const KrylovState* ks,
                       int v0, int jc, bool scaled, bool given, const UpdateCoef& cg, dim3 g,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_update<NV>, g, dim3(kRedThreads), 0, s, Z, ldz, x, N, ks, v0, jc, scaled,
                     given, cg);
}
template <int... I>
static constexpr std::array<UpdateFn, sizeof...(I)> update_table(std::integer_sequence<int, I...>) {
  return {&run_update<I + 1>...};
}
static const auto kUpdate = update_table(std::make_integer_sequence<int, kChunk>{});

hipError_t launch_update(const double* Z, size_t ldz, int jc, double* x, size_t N,
                         KrylovState* ks, bool scaled, hipStream_t s) {
  if (jc <= 0) return hipSuccess;
  if (jc > kMaxRestart) return hipErrorInvalidValue;
  const UpdateCoef none{};
  for (int v0 = 0; v0 < jc; v0 += kChunk) {
    const int n = jc - v0 < kChunk ? jc - v0 : kChunk;
    kUpdate[n - 1](Z + (size_t)v0 * ldz, ldz, x, N, ks, v0, jc, scaled, false, none,
                   dim3(stream_blocks(N)), s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_update_coef(const double* Z, size_t ldz, int jc, double* x, size_t N,
                              const double* c_host, hipStream_t s) {
  if (jc <= 0) return hipSuccess;
  if (jc > kMaxRestart) return hipErrorInvalidValue;
  UpdateCoef cg{};
  for (int i = 0; i < jc; ++i) cg.v[i] = c_host[i];
  for (int v0 = 0; v0 < jc; v0 += kChunk) {
    const int n = jc - v0 < kChunk ? jc - v0 : kChunk;
    kUpdate[n - 1](Z + (size_t)v0 * ldz, ldz, x, N, nullptr, v0, jc, false, true, cg,
                   dim3(stream_blocks(N)), s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rsfde
