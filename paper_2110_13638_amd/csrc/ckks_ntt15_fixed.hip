// N = 2^15 forward kernels whose conversion size is fixed at compile time
// (ModUp digit size 1..4, special-prime count 1..2), see ckks_device.h.
#include "ckks_device.h"

namespace ckks {
hipError_t launch_fwd_15_fixed(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s) {
    CKKS_FWD_FIXED(15, 5)
    return hipErrorInvalidValue;
}
}  // namespace ckks
