// Preconditioner passes with float internal arithmetic (explicit instantiations).
#include "pc_kernels.hpp"

namespace rsfde {
template hipError_t launch_pc_rows_fwd<float>(int, const double*, const double*, float*, const void*,
                                            int, int, bool, hipStream_t, const Members&, const SdTabs&);
template hipError_t launch_pc_cols<float>(int, const float*, float*, float*, const float*, const float*,
                                        const void*, int, int, double, double, double, double,
                                        bool, hipStream_t, const Members&, const double*, const SdTabs&);
template hipError_t launch_pc_rows_inv<float>(int, const float*, const float*,
                                            const uint8_t*, double*, const void*, int, int,
                                            bool, hipStream_t, const Members&, const SdTabs&);
template hipError_t launch_pc_rows_inv_mv<float>(int, const float*, const float*,
                                             const uint8_t*, void*, double*, const void*,
                                             const void*, const double*, double, double,
                                             const double*, double, int, int, bool, hipStream_t,
                                             const Members&, const double*, bool, const SdTabs&);
template hipError_t launch_dst_cols<float>(int, const float*, const float*, float*, float*, const void*, int,
                                          int, int, int, int, int, size_t, hipStream_t);
}  // namespace rsfde
