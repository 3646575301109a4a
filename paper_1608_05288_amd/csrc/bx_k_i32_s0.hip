// Tiled UTIL kernel, int32 costs, without LDS staging of lane tables:
// its two store variants (plain / non-temporal blocked rows).
#include "bx_util_kernels.h"

namespace bx {

void launch_tiles_i32_s0(const Descs &d, int32_t t0, int32_t n, bool nt, hipStream_t st) {
    if (n <= 0) return;
    if (nt)
        hipLaunchKernelGGL((util_tiles_kernel<CostI, false, true>), dim3(n + d.pf_extra), dim3(kUtilThreads), 0, st, d, t0);
    else
        hipLaunchKernelGGL((util_tiles_kernel<CostI, false, false>), dim3(n + d.pf_extra), dim3(kUtilThreads), 0, st, d, t0);
}

}  // namespace bx
