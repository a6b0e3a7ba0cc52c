// Allocation-free form of the matrix-vector product y = M x (no plan).
//
// Callers that cannot allocate device memory (code under stream capture, tight
// serving loops, harnesses that forbid hipMalloc) get the two FFT passes of
// rsfde_matvec with every scratch buffer in one file-scope device array: the
// strip-tiled row-pass intermediate t, the two circulant symbols and the two
// twiddle tables.  The array is loaded with the code object, once per device,
// and kept until the process ends; its size bounds the grid (header).
//
// The tables are rebuilt on the device (one small kernel, no host transfer)
// only when the grid, the orders or the unit coefficients c = dt c_alpha /
// h^alpha differ from the last call on the device; kx, ky and dt / eta enter
// the kernels as scalars.  Calls that overlap on one device share the array
// and race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/rsfde.h"
#include "internal.hpp"

namespace rsfde {
namespace {

// 33 MiB: the intermediate of a 2047 x 2047 grid (8 ceil(n1/4) ceil(n2/2) =
// 4,194,304 doubles) plus the largest tables (L = 4096: two symbols of L and
// two twiddle tables of 2L doubles).
constexpr size_t kScratchDoubles = (size_t)33 << 17;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;

// Per device: the device address of `scratch` and the key of the tables it
// holds.  Guarded by `mu`.
struct DeviceScratch {
  double* ptr = nullptr;
  bool have_tables = false;
  int n1 = 0, n2 = 0;
  double alpha1 = 0, alpha2 = 0, cx = 0, cy = 0;
};
std::mutex mu;
DeviceScratch devs[kMaxDevices];

size_t round32(size_t v) { return (v + 31) / 32 * 32; }

constexpr double kPi2 = 3.14159265358979323846264338327950288;

struct DirTables {
  double alpha, c;  // order and unit coefficient dt c_alpha / h^alpha of the direction
  int n, L;         // points and convolution length (a power of two, L >= 2n)
  double* sym;      // out: symbol / L in register-position order (L values)
  double* tw;       // out: exp(-2 pi i j / L), j < L (2L values)
};

// One block per direction (blockIdx.x): the tables of the matrix-vector
// product, computed as the plan's set-up computes them on the host.
//   twiddles  exp(-2 pi i j / L) with the angle reduced to j' = min(j, L - j)
//             and exact zeros at the quarter and half points;
//   t         first column of c G_n^(alpha) (G): Grunwald-Letnikov weights by
//             the recurrence g_l = (1 - (alpha + 1) / l) g_{l-1} (g_form),
//             t = c [2 g_1, g_0 + g_2, g_3, ..., g_n];
//   symbol    of the length-L circulant embedding: t_0 + 2 sum_j t_j
//             cos(2 pi j f / L) at the frequency f held by register position p,
//             divided by L.
__global__ __launch_bounds__(1024) void k_noalloc_tables(DirTables dx, DirTables dy) {
  const DirTables d = blockIdx.x == 0 ? dx : dy;
  __shared__ double t_s[2048];
  __shared__ double cos_s[4096];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = tid; k < d.L; k += nt) {
    const int jj = k <= d.L / 2 ? k : d.L - k;
    const double a = 2.0 * kPi2 * (double)jj / (double)d.L;
    double cv = cos(a), sv = sin(a);
    if (4 * jj == d.L) cv = 0.0;
    if (2 * jj == d.L) sv = 0.0;
    cos_s[k] = cv;
    d.tw[2 * k] = cv;
    d.tw[2 * k + 1] = k <= d.L / 2 ? -sv : sv;
  }
  if (tid == 0) {
    double g0 = 1.0, g1 = 0.0, g2 = 0.0, gp = 1.0;
    for (int l = 1; l < d.n + 2; ++l) {
      const double g = (1.0 - (d.alpha + 1.0) / l) * gp;
      if (l == 1) g1 = g;
      if (l == 2) g2 = g;
      if (l >= 3) t_s[l - 1] = g * d.c;
      gp = g;
    }
    t_s[0] = 2.0 * g1 * d.c;
    if (d.n > 1) t_s[1] = (g0 + g2) * d.c;
  }
  __syncthreads();
  const int P = fft_pts(d.L);
  for (int p = tid; p < d.L; p += nt) {
    const int f = fft_freq(d.L, P, p);
    double s = t_s[0];
    for (int j = 1; j < d.n; ++j) s += 2.0 * t_s[j] * cos_s[(int)(((long long)j * f) & (d.L - 1))];
    d.sym[p] = s / (double)d.L;
  }
}

}  // namespace
}  // namespace rsfde

extern "C" int rsfde_matvec_noalloc(const rsfde_grid* grid, double alpha1, double alpha2,
                                    double kx, double ky, const uint8_t* mask_dev, double eta,
                                    double dt, const double* x, double* y, void* stream) {
  using namespace rsfde;
  if (!grid || !mask_dev || !x || !y || x == y) return RSFDE_EINVAL;
  const int n1 = grid->n1, n2 = grid->n2;
  if (n1 < 1 || n2 < 1) return RSFDE_EINVAL;
  if (!(grid->x_hi > grid->x_lo) || !(grid->y_hi > grid->y_lo) || !std::isfinite(grid->x_lo) ||
      !std::isfinite(grid->x_hi) || !std::isfinite(grid->y_lo) || !std::isfinite(grid->y_hi))
    return RSFDE_EINVAL;
  if (!(alpha1 > 1.0 && alpha1 < 2.0) || !(alpha2 > 1.0 && alpha2 < 2.0)) return RSFDE_EINVAL;
  if (!(kx >= 0.0) || !(ky >= 0.0) || !std::isfinite(kx) || !std::isfinite(ky)) return RSFDE_EINVAL;
  if (!(eta > 0.0) || !(dt > 0.0) || !std::isfinite(eta) || !std::isfinite(dt)) return RSFDE_EINVAL;
  // Scratch layout (doubles): t | sym_x (Lx) | sym_y (Ly) | tw_x (2 Lx) | tw_y (2 Ly).
  auto pow2_at_least = [](long v) {
    int p = 2;
    while (p < v) p <<= 1;
    return p;
  };
  const int Lx = pow2_at_least(2L * n1), Ly = pow2_at_least(2L * n2);
  const size_t t_len = round32((size_t)8 * (size_t)((n1 + 3) / 4) * (size_t)((n2 + 1) / 2));
  const size_t o_sx = t_len, o_sy = o_sx + round32(Lx), o_tx = o_sy + round32(Ly),
               o_ty = o_tx + round32(2 * (size_t)Lx), end = o_ty + round32(2 * (size_t)Ly);
  if (n1 > 2047 || n2 > 2047 || end > kScratchDoubles) return RSFDE_EUNSUPPORTED;

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RSFDE_EHIP;
  hipStream_t s = (hipStream_t)stream;
  const double hx = (grid->x_hi - grid->x_lo) / (n1 + 1);
  const double hy = (grid->y_hi - grid->y_lo) / (n2 + 1);
  const double cx = dt * (-1.0 / (2.0 * std::cos(alpha1 * kPi2 / 2.0))) / std::pow(hx, alpha1);
  const double cy = dt * (-1.0 / (2.0 * std::cos(alpha2 * kPi2 / 2.0))) / std::pow(hy, alpha2);
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(mu);
    DeviceScratch& d = devs[dev];
    if (!d.ptr) {  // first call on this device: the array's device address
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RSFDE_EHIP;
      d.ptr = (double*)p;
    }
    base = d.ptr;
    if (!d.have_tables || d.n1 != n1 || d.n2 != n2 || d.alpha1 != alpha1 || d.alpha2 != alpha2 ||
        d.cx != cx || d.cy != cy) {
      d.have_tables = false;
      const DirTables tx{alpha1, cx, n1, Lx, base + o_sx, base + o_tx};
      const DirTables ty{alpha2, cy, n2, Ly, base + o_sy, base + o_ty};
      hipLaunchKernelGGL(k_noalloc_tables, dim3(2), dim3(1024), 0, s, tx, ty);
      if (hipGetLastError() != hipSuccess) return RSFDE_EHIP;
      d.n1 = n1;
      d.n2 = n2;
      d.alpha1 = alpha1;
      d.alpha2 = alpha2;
      d.cx = cx;
      d.cy = cy;
      d.have_tables = true;
    }
  }
  // The two passes of the two-dimensional product (t strip-tiled), as rsfde_matvec.
  if (launch_mv_rows(Lx, x, mask_dev, base, base + o_sx, base + o_tx, n1, n2, -kx, dt / eta, 0,
                     s, nullptr, 0.0, true) != hipSuccess)
    return RSFDE_EHIP;
  if (launch_mv_cols(Ly, x, base, y, base + o_sy, base + o_ty, n1, n2, -ky, 0, s, 1, 0, true) !=
      hipSuccess)
    return RSFDE_EHIP;
  return RSFDE_OK;
}
