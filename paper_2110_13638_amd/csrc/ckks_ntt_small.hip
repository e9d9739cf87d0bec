// NTT kernels for N = 2^10 .. 2^12 (see ckks_device.h).
#include "ckks_device.h"

namespace ckks {
hipError_t launch_fwd_small(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s) {
    if (is_modup(op)) op = F_MODUP;
    if (is_moddown(op)) op = F_MODDOWN;
    if (is_relin(op)) op = is_relin_rs(op) ? F_RELIN_RS : F_RELIN;
    if (tb.ntt_wide) {
        switch (tb.log_n) {
            CKKS_FWD_CASE(11, 5)
            CKKS_FWD_CASE(12, 5)
        }
    }
    switch (tb.log_n) {
        CKKS_FWD_CASE(10, 4)
        CKKS_FWD_CASE(11, 4)
        CKKS_FWD_CASE(12, 4)
    }
    return hipErrorInvalidValue;
}
hipError_t launch_inv_small(const DevTables &tb, int op, const Item *items, int n, hipStream_t s) {
    if (tb.ntt_wide) {
        switch (tb.log_n) {
            CKKS_INV_CASE(11, 5)
            CKKS_INV_CASE(12, 5)
        }
    }
    switch (tb.log_n) {
        CKKS_INV_CASE(10, 4)
        CKKS_INV_CASE(11, 4)
        CKKS_INV_CASE(12, 4)
    }
    return hipErrorInvalidValue;
}
}  // namespace ckks
