// Chirp-form sine-transform preconditioner with double internal arithmetic
// (explicit instantiations).
#include "pc_chirp.hpp"

namespace rsfde {
template hipError_t launch_cd_rows_fwd<double>(int, const double*, const double*, double*, const void*,
                                            const void*, const void*, int, int, hipStream_t);
template hipError_t launch_cd_cols<double>(int, const double*, double*, double*, const double*, const double*,
                                        const void*, const void*, const void*, int, int, double,
                                        double, double, hipStream_t);
template hipError_t launch_cd_rows_inv<double>(int, const double*, const double*, const uint8_t*, double*,
                                            const void*, const void*, const void*, int, int,
                                            hipStream_t);
template hipError_t launch_cd_dst_cols<double>(int, const double*, double*, const double*, double*, const void*,
                                            const void*, const void*, int, int, int, size_t,
                                            hipStream_t);
}  // namespace rsfde
