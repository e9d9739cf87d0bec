// forward NTT kernels for N = 2^15 (see ckks_device.h).
#include "ckks_device.h"

namespace ckks {
hipError_t launch_fwd_15(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s) {
    if (modup_s(op) || relin_np(op) || moddown_np(op)) return launch_fwd_15_fixed(tb, op, items, n, seed, s);
    if (is_modup(op)) op = F_MODUP;
    if (is_moddown(op)) op = F_MODDOWN;
    if (is_relin(op)) op = is_relin_rs(op) ? F_RELIN_RS : F_RELIN;
    switch (tb.log_n) { CKKS_FWD_CASE(15, 5) }
    return hipErrorInvalidValue;
}
}  // namespace ckks
