// inverse NTT kernels for N = 2^15 (see ckks_device.h).
#include "ckks_device.h"

namespace ckks {
hipError_t launch_inv_15(const DevTables &tb, int op, const Item *items, int n, hipStream_t s) {
    switch (tb.log_n) { CKKS_INV_CASE(15, 5) }
    return hipErrorInvalidValue;
}
}  // namespace ckks
