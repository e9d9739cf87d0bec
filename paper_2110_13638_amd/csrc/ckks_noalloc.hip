// Allocation-free variant of the batched HMult + relinearise + rescale call
// for callers that cannot allocate device memory (code under stream
// capture, tight serving loops, hosts that forbid hipMalloc). Its scratch
// limbs and work-item tables live in one fixed device array of this
// translation unit instead of a caller workspace.
#include <stdio.h>

#include <memory>
#include <mutex>

#include "../../include/ckks.h"
#include "ckks_internal.h"

namespace ckks {
int set_error(int code, const char *msg);
void set_no_alloc(bool on);
}  // namespace ckks

using namespace ckks;

// One copy per GPU the library runs on, held until the process ends.
static __device__ __align__(256) uint8_t scratch[CKKS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch` on each device (null: not looked up yet)

// The array's device address on the current device, looked up once per
// device with that device current. Host code never uses the array's name
// as an address: on the host it only stands for the symbol.
int scratch_ptr(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return set_error(CKKS_EDEVICE, "hmult_noalloc: no current device");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_error(CKKS_EDEVICE, "hmult_noalloc: hipGetSymbolAddress of the scratch array failed");
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return CKKS_OK;
}

// clears the thread's no-allocation mode on every return path
struct NoAllocScope {
    NoAllocScope() { set_no_alloc(true); }
    ~NoAllocScope() { set_no_alloc(false); }
};
}  // namespace

extern "C" int ckks_hmult_relin_rescale_noalloc(const ckks_ctx *ctx, const uint64_t *const *rk, const ckks_ct *a,
                                                const ckks_ct *b, ckks_ct *out, uint32_t B, void *stream) {
    if (!ctx || (B && (!a || !b || !out || !rk))) return set_error(CKKS_EINVAL, "hmult_noalloc: null argument");
    if (B == 0) return CKKS_OK;
    // size check first (host planning only): the call's scratch limbs and
    // descriptor tables must fit the fixed array
    uint32_t levels_small[64];
    uint32_t *levels = levels_small;
    std::unique_ptr<uint32_t[]> levels_big;
    if (B > 64) {
        levels_big.reset(new uint32_t[B]);
        levels = levels_big.get();
    }
    for (uint32_t x = 0; x < B; x++) levels[x] = a[x].level;
    const size_t need = ckks_workspace_bytes(ctx, CKKS_OP_HMULT, B, levels);
    if (need == 0 || need > (size_t)CKKS_NOALLOC_SCRATCH_BYTES) {
        char msg[200];
        snprintf(msg, sizeof msg,
                 "hmult_noalloc: this batch needs %zu bytes of scratch; the fixed scratch holds %zu "
                 "(use ckks_hmult_relin_rescale with a caller workspace)",
                 need, (size_t)CKKS_NOALLOC_SCRATCH_BYTES);
        return set_error(CKKS_ENOMEM, msg);
    }
    void *ws = nullptr;
    const int rc = scratch_ptr(&ws);
    if (rc != CKKS_OK) return rc;
    NoAllocScope scope;
    return ckks_hmult_relin_rescale(ctx, rk, a, b, out, B, ws, (size_t)CKKS_NOALLOC_SCRATCH_BYTES, stream);
}
