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
// Per-member vector counts of a batched update (given = 0: all use jc).
struct JcList {
  int32_t given;
  int32_t jc[kMaxBatch];
};

template <int NV, typename ZT = double>
__global__ __launch_bounds__(kRedThreads) void k_update(const ZT* __restrict__ Z, size_t ldz,
                                                        double* __restrict__ x, size_t N,
                                                        const KrylovState* __restrict__ ks,
                                                        int v0, int jc, bool scaled, bool given,
                                                        const UpdateCoef cgiven, const Members mb,
                                                        const JcList jcs) {
  __shared__ double y[kMaxRestart];
  {  // member of a batched launch (grid dimension y), with its own vector count
    const size_t mo = mb.off(blockIdx.y);
    Z += mo;
    x += mo;
    if (ks) ks = (const KrylovState*)((const double*)ks + mo);
    if (jcs.given) jc = jcs.jc[blockIdx.y];
    if (v0 >= jc) return;
  }
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
  // a member of a batched update may use fewer than NV vectors of this chunk:
  // past its count the loads read the chunk's first vector (written, finite)
  // and the coefficient is zero, so every load stays unconditional
  const int nvm = jc - v0 < NV ? jc - v0 : NV;
  double c[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v)
    c[v] = v < nvm ? y[v0 + v] * (scaled && !given ? ks->vscale[v0 + v] : 1.0) : 0.0;
  const size_t N2 = N / 2;
  double2* x2 = reinterpret_cast<double2*>(x);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N2;
       i += (size_t)gridDim.x * blockDim.x) {
    double2 z[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const ZT* zp = Z + (size_t)(v < nvm ? v : 0) * ldz;
      if constexpr (sizeof(ZT) == 8) {
        z[v] = reinterpret_cast<const double2*>(zp)[i];
      } else {
        const float2 f = reinterpret_cast<const float2*>(zp)[i];
        z[v] = double2{(double)f.x, (double)f.y};
      }
    }
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
    for (int v = 0; v < NV; ++v)
      if (v < nvm) s += c[v] * (double)Z[(size_t)v * ldz + N - 1];
    x[N - 1] = s;
  }
}

using UpdateFn = void (*)(const void*, size_t, double*, size_t, const KrylovState*, int, int,
                          bool, bool, const UpdateCoef&, const Members&, const JcList&, dim3,
                          hipStream_t);
template <int NV, typename ZT>
static void run_update(const void* Z, size_t ldz, double* x, size_t N, const KrylovState* ks,
                       int v0, int jc, bool scaled, bool given, const UpdateCoef& cg,
                       const Members& mb, const JcList& jl, dim3 g, hipStream_t s) {
  hipLaunchKernelGGL((k_update<NV, ZT>), g, dim3(kRedThreads), 0, s, (const ZT*)Z, ldz, x, N, ks,
                     v0, jc, scaled, given, cg, mb, jl);
}
template <typename ZT, int... I>
static constexpr std::array<UpdateFn, sizeof...(I)> update_table(std::integer_sequence<int, I...>) {
  return {&run_update<I + 1, ZT>...};
}
static const auto kUpdate = update_table<double>(std::make_integer_sequence<int, kChunk>{});
static const auto kUpdate32 = update_table<float>(std::make_integer_sequence<int, kChunk>{});

hipError_t launch_update(const void* Z, size_t ldz, int jc, double* x, size_t N,
                         KrylovState* ks, bool scaled, hipStream_t s, const Members& mb,
                         const int32_t* jcs, bool z32) {
  const size_t zb = z32 ? sizeof(float) : sizeof(double);
  if (jc <= 0) return hipSuccess;
  if (jc > kMaxRestart) return hipErrorInvalidValue;
  if (mb.n < 1 || mb.n > kMaxBatch) return hipErrorInvalidValue;
  const UpdateCoef none{};
  JcList jl{};
  if (jcs) {
    jl.given = 1;
    for (int k = 0; k < mb.n; ++k) jl.jc[k] = jcs[k];
  }
  for (int v0 = 0; v0 < jc; v0 += kChunk) {
    const int n = jc - v0 < kChunk ? jc - v0 : kChunk;
    (z32 ? kUpdate32 : kUpdate)[n - 1]((const char*)Z + (size_t)v0 * ldz * zb, ldz, x, N, ks, v0,
                                       jc, scaled, false, none, mb, jl,
                                       dim3(stream_blocks(N), mb.n), s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_update_coef(const void* Z, size_t ldz, int jc, double* x, size_t N,
                              const double* c_host, hipStream_t s, bool z32) {
  const size_t zb = z32 ? sizeof(float) : sizeof(double);
  if (jc <= 0) return hipSuccess;
  if (jc > kMaxRestart) return hipErrorInvalidValue;
  UpdateCoef cg{};
  for (int i = 0; i < jc; ++i) cg.v[i] = c_host[i];
  for (int v0 = 0; v0 < jc; v0 += kChunk) {
    const int n = jc - v0 < kChunk ? jc - v0 : kChunk;
    (z32 ? kUpdate32 : kUpdate)[n - 1]((const char*)Z + (size_t)v0 * ldz * zb, ldz, x, N,
                                       nullptr, v0, jc, false, true, cg, Members::one(),
                                       JcList{}, dim3(stream_blocks(N)), s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rsfde
