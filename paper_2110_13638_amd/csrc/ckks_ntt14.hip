// NTT kernels for N = 2^14 (see ckks_device.h).
#include "ckks_device.h"

namespace ckks {
hipError_t launch_fwd_14(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s) {
    // one-prime digits and 1-2 special primes: conversions of a fixed size
    if (tb.ntt_wide) CKKS_FWD_FIXED_SMALL(14, 5)
    else CKKS_FWD_FIXED_SMALL(14, 4)
    if (is_modup(op)) op = F_MODUP;
    if (is_moddown(op)) op = F_MODDOWN;
    if (is_relin(op)) op = is_relin_rs(op) ? F_RELIN_RS : F_RELIN;
    if (tb.ntt_wide) {
        switch (tb.log_n) {
            CKKS_FWD_CASE(14, 5)
        }
    }
    switch (tb.log_n) {
        CKKS_FWD_CASE(14, 4)
    }
    return hipErrorInvalidValue;
}
hipError_t launch_inv_14(const DevTables &tb, int op, const Item *items, int n, hipStream_t s) {
    if (tb.ntt_wide) {
        switch (tb.log_n) {
            CKKS_INV_CASE(14, 5)
        }
    }
    switch (tb.log_n) {
        CKKS_INV_CASE(14, 4)
    }
    return hipErrorInvalidValue;
}
}  // namespace ckks
