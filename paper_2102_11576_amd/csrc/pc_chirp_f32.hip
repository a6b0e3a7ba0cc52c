// Chirp-form sine-transform preconditioner with float internal arithmetic
// (explicit instantiations).
#include "pc_chirp.hpp"

namespace rsfde {
template hipError_t launch_cd_rows_fwd<float>(int, const double*, const double*, float*, const void*,
                                            const void*, const void*, int, int, hipStream_t);
template hipError_t launch_cd_cols<float>(int, const float*, float*, float*, const double*, const double*,
                                        const void*, const void*, const void*, int, int, double,
                                        double, double, hipStream_t);
template hipError_t launch_cd_rows_inv<float>(int, const float*, const float*, const uint8_t*, double*,
                                            const void*, const void*, const void*, int, int,
                                            hipStream_t);
template hipError_t launch_cd_dst_cols<float>(int, const float*, float*, const float*, float*, const void*,
                                            const void*, const void*, int, int, int, size_t,
                                            hipStream_t);
}  // namespace rsfde
