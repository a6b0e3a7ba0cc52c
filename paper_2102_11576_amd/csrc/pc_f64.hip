// Preconditioner passes with double internal arithmetic (explicit instantiations).
#include "pc_kernels.hpp"

namespace rsfde {
template hipError_t launch_pc_rows_fwd<double>(int, const double*, const double*, double*, const void*,
                                            int, int, bool, hipStream_t, const Members&, const SdTabs&);
template hipError_t launch_pc_cols<double>(int, const double*, double*, double*, const double*, const double*,
                                        const void*, int, int, double, double, double, double,
                                        bool, hipStream_t, const Members&, const double*, const SdTabs&);
template hipError_t launch_pc_rows_inv<double>(int, const double*, const double*,
                                            const uint8_t*, double*, const void*, int, int,
                                            bool, hipStream_t, const Members&, const SdTabs&);
template hipError_t launch_pc_rows_inv_mv<double>(int, const double*, const double*,
                                             const uint8_t*, void*, double*, const void*,
                                             const void*, const double*, double, double,
                                             const double*, double, int, int, bool, hipStream_t,
                                             const Members&, const double*, bool, const SdTabs&);
template hipError_t launch_dst_cols<double>(int, const double*, const double*, double*, double*, const void*, int,
                                          int, int, int, int, int, size_t, hipStream_t);
}  // namespace rsfde
