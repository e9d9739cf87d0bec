// NTT / INTT of limbs at N = 2^16: a streaming first stage, then two
// workgroups of the 2^15 engine per limb (see ckks_device.h). Only plain
// transforms are provided at this ring degree.
#include "ckks_device.h"

namespace ckks {
hipError_t launch_fwd_16(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s) {
    (void)seed;
    if (op != F_COPY || tb.log_n != 16) return hipErrorInvalidValue;
    const int per = (1 << 15) / (kPairThreads * kPairsPerThread);
    if (tb.ntt_fp) {
        hipLaunchKernelGGL((k_first_stage<true, false>), dim3(n * per), dim3(kPairThreads), 0, s, tb, items, n);
        hipLaunchKernelGGL((k_fwd_halves<16, 5, true>), dim3(xcd_grid(2 * n)), dim3(1024), 0, s, tb, items, n);
    } else {
        hipLaunchKernelGGL((k_first_stage<false, false>), dim3(n * per), dim3(kPairThreads), 0, s, tb, items, n);
        hipLaunchKernelGGL((k_fwd_halves<16, 5, false>), dim3(xcd_grid(2 * n)), dim3(1024), 0, s, tb, items, n);
    }
    return hipGetLastError();
}
hipError_t launch_inv_16(const DevTables &tb, int op, const Item *items, int n, hipStream_t s) {
    if (op != I_COPY || tb.log_n != 16) return hipErrorInvalidValue;
    const int per = (1 << 15) / (kPairThreads * kPairsPerThread);
    if (tb.ntt_fp) {
        hipLaunchKernelGGL((k_first_stage<true, true>), dim3(n * per), dim3(kPairThreads), 0, s, tb, items, n);
        hipLaunchKernelGGL((k_inv_classes<16, 5, true>), dim3(xcd_grid(2 * n)), dim3(1024), 0, s, tb, items, n);
    } else {
        hipLaunchKernelGGL((k_first_stage<false, true>), dim3(n * per), dim3(kPairThreads), 0, s, tb, items, n);
        hipLaunchKernelGGL((k_inv_classes<16, 5, false>), dim3(xcd_grid(2 * n)), dim3(1024), 0, s, tb, items, n);
    }
    return hipGetLastError();
}
}  // namespace ckks
