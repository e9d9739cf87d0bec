// Internal declarations shared by the host runtime's sources
// (ckks_host.cpp: contexts, encoding, planning, recording, serialisation and
// the client-side calls; ckks_eval.cpp: the server-side ciphertext
// operations; ckks_linear.cpp: the linear layers). Not part of the public ABI.
#pragma once
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <deque>
#include <type_traits>
#include <string>
#include <functional>
#include <mutex>
#include <vector>

#include "../../include/ckks.h"
#include "ckks_internal.h"

namespace ckks {
hipError_t launch_fwd(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s);
hipError_t launch_inv(const DevTables &tb, int op, const Item *items, int n, hipStream_t s);
hipError_t launch_ew(const DevTables &tb, const EwItem *items, int n, u64 seed, hipStream_t s);
hipError_t launch_ip(const DevTables &tb, const IpItem *items, int n, hipStream_t s);
hipError_t launch_hoist(const DevTables &tb, int staged_rows, const HoItem *items, int n, hipStream_t s);
hipError_t launch_ip_seq(const DevTables &tb, const IpSeqItem *items, int n, hipStream_t s);
hipError_t launch_linear(const DevTables &tb, const u64 *const *in_ptrs, const u64 *wt,
                         u64 *const *out_ptrs, u32 n_in, u32 n_out, u32 limbs, u32 in_stride,
                         u32 out_stride, hipStream_t s);
hipError_t launch_reduce_weights(const DevTables &tb, const i64 *W, u64 *wt, u32 count, u32 limbs,
                                 hipStream_t s);
hipError_t launch_linear_mfma(const DevTables &tb, const int8_t *wd, u32 rows_pad, u32 k_pad, const u32 *cols,
                              u32 n_in, u32 n_out, const u64 *const *in_ptrs, u64 *const *out_ptrs, u32 t_lo,
                              u32 t_cnt, bool small, u32 in_stride, u32 out_stride, hipStream_t s);
hipError_t launch_weight_digits(const i64 *W, u32 n_out, u32 n_in, u32 rows_pad, u32 k_pad, int8_t *wd,
                                hipStream_t s);
hipError_t launch_linear_grouped(const DevTables &tb, const LinGroup *groups, u32 n_groups, const u32 *cols,
                                 const u64 *wt, const double2 *wf, u32 wt_stride, const u64 *const *in_ptrs, u64 *const *out_ptrs,
                                 u32 limbs, u32 in_stride, u32 out_stride, u32 max_rows, hipStream_t s);

// kernel op codes (mirrors of the enums in the kernel file)
enum {
    F_COPY = 0, F_MODUP = 1, F_RESCALE = 2, F_MODDOWN = 3, F_RELIN = 4, F_SAMPLE = 5, F_INT = 6, F_RELIN_RS = 7,
    F_MODUP_S1 = 8, F_RELIN_P1 = 12, F_RELIN_RS_P1 = 14, F_MODDOWN_P1 = 16
};
enum { I_COPY = 0, I_MUL = 1, I_SCALE = 2, I_DECRYPT = 3 };
enum {
    EW_ADD = 0, EW_SUB = 1, EW_MUL = 2, EW_MUL_CONST = 3, EW_ADD_CONST = 4, EW_TENSOR = 5,
    EW_COPY = 6, EW_AUTOMORPH = 7, EW_NEG = 8, EW_KEYGEN = 9, EW_ENCRYPT = 10, EW_SQUARE_S = 11,
    EW_HMULT_FIN = 12, EW_HMULT_T = 14
};
enum { TAG_SK = 1, TAG_PK_A = 2, TAG_PK_E = 3, TAG_SWK_A = 4, TAG_SWK_E = 5, TAG_ENC_V = 6,
       TAG_ENC_E0 = 7, TAG_ENC_E1 = 8 };
enum { S_TERNARY = 0, S_CBD = 1 };

typedef unsigned __int128 u128;

// ---------------------------------------------------------------------
// errors (message kept per host thread, see ckks_last_error)
// ---------------------------------------------------------------------
int set_error(int code, const char *msg);
int fail(int code, const char *fmt, ...);
#define HIP_TRY(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) return fail(CKKS_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
#define CK(x)                  \
    do {                       \
        int r_ = (x);          \
        if (r_ != CKKS_OK) return r_; \
    } while (0)

// ---------------------------------------------------------------------
// integer helpers
// ---------------------------------------------------------------------
inline u64 mulmod(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }
inline u64 powmod(u64 a, u64 e, u64 q) {
    u64 r = 1 % q;
    a %= q;
    for (; e; e >>= 1) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
    }
    return r;
}
inline u64 invmod(u64 a, u64 q) { return powmod(a, q - 2, q); }
inline u64 shoup_companion(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }
inline bool is_prime(u64 n) {
    static const u64 bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (u64 b : bases) {
        if (n == b) return true;
        if (n % b == 0) return false;
    }
    u64 d = n - 1;
    int r = 0;
    while (!(d & 1)) d >>= 1, r++;
    for (u64 b : bases) {
        u64 x = powmod(b, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int k = 1; k < r && comp; k++) {
            x = mulmod(x, x, n);
            if (x == n - 1) comp = false;
        }
        if (comp) return false;
    }
    return true;
}
inline u32 bitrev(u32 x, u32 bits) {
    u32 r = 0;
    for (u32 i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}
// smallest primitive 2N-th root of unity mod q
inline u64 smallest_psi(u64 q, u32 log_n) {
    const u64 n = 1ull << log_n, two_n = n << 1;
    u64 g = 0;
    for (u64 x = 2; x < q && !g; x++) {
        u64 c = powmod(x, (q - 1) / two_n, q);
        if (powmod(c, n, q) == q - 1) g = c;
    }
    if (!g) return 0;
    u64 best = g, g2 = mulmod(g, g, q), cur = g;
    for (u64 k = 1; k < n; k++) {
        cur = mulmod(cur, g2, q);
        best = std::min(best, cur);
    }
    return best;
}

// little multiword unsigned integers for the CRT lift
typedef std::vector<u64> Big;
inline void big_mul_small(Big &a, u64 m) {
    u64 carry = 0;
    for (auto &w : a) {
        u128 t = (u128)w * m + carry;
        w = (u64)t;
        carry = (u64)(t >> 64);
    }
    if (carry) a.push_back(carry);
}
inline int big_cmp(const Big &a, const Big &b) {
    size_t n = std::max(a.size(), b.size());
    for (size_t i = n; i-- > 0;) {
        u64 x = i < a.size() ? a[i] : 0, y = i < b.size() ? b[i] : 0;
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}
inline void big_sub(Big &a, const Big &b) {  // a -= b, a >= b
    u64 borrow = 0;
    for (size_t i = 0; i < a.size(); i++) {
        u64 y = i < b.size() ? b[i] : 0;
        u128 t = (u128)a[i] - y - borrow;
        a[i] = (u64)t;
        borrow = (u64)(t >> 64) ? 1 : 0;
    }
}
inline void big_addmul(Big &acc, const Big &b, u64 m) {  // acc += b * m
    if (acc.size() < b.size() + 2) acc.resize(b.size() + 2, 0);
    u64 carry = 0;
    size_t i = 0;
    for (; i < b.size(); i++) {
        u128 t = (u128)b[i] * m + acc[i] + carry;
        acc[i] = (u64)t;
        carry = (u64)(t >> 64);
    }
    for (; carry && i < acc.size(); i++) {
        u128 t = (u128)acc[i] + carry;
        acc[i] = (u64)t;
        carry = (u64)(t >> 64);
    }
}
inline double big_to_double(const Big &a) {
    double d = 0;
    for (size_t i = a.size(); i-- > 0;) d = d * 18446744073709551616.0 + (double)a[i];
    return d;
}

}  // namespace ckks

using namespace ckks;


// ---------------------------------------------------------------------
// context
// ---------------------------------------------------------------------
// Launch recording (see ckks_record_begin): the arena receives every
// host-to-device upload of launch data made while recording, and each
// kernel launch is kept as a closure over its (device-resident) arguments.
typedef std::function<hipError_t(hipStream_t)> LaunchFn;
struct Recorder {
    uint8_t *arena = nullptr;
    size_t cap = 0, used = 0;
    std::vector<LaunchFn> launches;
};

// Pinned host ring for launch-data uploads: a copy from pinned memory is
// asynchronous, so the host keeps planning the next call while the device
// works. Each region stays reserved until the event recorded after its copy
// has completed.
struct Staging {
    uint8_t *buf = nullptr;
    size_t cap = 0, head = 0;
    struct Region {
        size_t lo, hi;
        hipEvent_t done;
    };
    std::deque<Region> inflight;
    ~Staging() {  // teardown: errors cannot be reported from here
        for (auto &r : inflight) {
            (void)hipEventSynchronize(r.done);
            (void)hipEventDestroy(r.done);
        }
        if (buf) (void)hipHostFree(buf);
    }
};
constexpr size_t kStagingBytes = (size_t)64 << 20;

struct ckks_ctx {
    u32 log_n, N, n_q, n_p, n_prim, dnum, alpha, digits_top;
    Recorder *rec = nullptr;  // non-null while recording
    Staging *stage = nullptr;  // created on the first upload
    std::mutex stage_mu;       // host threads sharing the context take turns on the ring
    ~ckks_ctx() { delete stage; }
    std::vector<u64> primes;
    std::vector<u64> image;  // device table image (u64 words)
    size_t off_pc, off_tw, off_itw, off_twf, off_itwf, off_modup, off_moddown, off_rescale;
    DevTables tb{};
    bool uploaded = false;
    // encoder
    std::vector<std::complex<double>> fft_roots;  // e^{2 pi i k / M}, k < M
    std::vector<std::complex<double>> twist;      // zeta^i, i < M
    std::vector<u32> slot_index;                  // k_j = (5^j mod 2N - 1) / 4
    // CRT per level
    std::vector<std::vector<Big>> qhat;    // [level][i]
    std::vector<std::vector<u64>> qhat_inv;
    std::vector<Big> Q, Qhalf;
};

inline size_t align_words(size_t w) { return (w + 31) & ~(size_t)31; }  // 256 bytes

struct ckks_plan {
    const ckks_ctx *c;
    std::vector<LaunchFn> launches;
};

namespace ckks {
// ---------------------------------------------------------------------
// optional per-launch timing with HIP events on the launch stream
// ---------------------------------------------------------------------
struct ProfRec {
    std::string name;
    u32 items;
    hipEvent_t e0, e1;
};
extern bool g_prof_on;
extern std::vector<ProfRec> g_prof;
std::string launch_name(int kind, int op, u32 log_n);

// ---------------------------------------------------------------------
// planning: scratch carving + work-item tables
// ---------------------------------------------------------------------
struct Launch {
    int kind;  // 0 fwd, 1 inv, 2 ew, 3 ip, 5 hoisted rotations, 6 ip (sequential ciphertexts)
    int op;
    size_t off;
    int n;
    u64 seed;
    int fp = 0;  // NTT launches: every item's prime is below 2^50 and takes the FP64 engine
};
inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
// set while a call must not allocate (ckks_hmult_relin_rescale_noalloc)
extern thread_local bool g_no_alloc;
// Host-to-device copy of launch data (descriptors, pointer tables, weight
// images); while recording, the bytes go to the recording arena and *where
// receives that address instead of dst.
int upload(const ckks_ctx *c, uint8_t *dst, const void *src, size_t bytes, hipStream_t s, uint8_t **where);
// Run a launch now and, while recording, keep it for replays.
hipError_t issue(const ckks_ctx *c, hipStream_t s, LaunchFn f);
// descriptor buffer recycled per host thread
std::vector<uint8_t> &desc_pool();
struct Plan {
    const ckks_ctx *c;
    uint8_t *ws;          // device base (may be null when sizing)
    size_t scratch = 0;   // bytes of scratch carved so far
    std::vector<uint8_t> desc;
    std::vector<Launch> launches;
    explicit Plan(const ckks_ctx *cc, void *w) : c(cc), ws((uint8_t *)w) {
        desc.swap(desc_pool());
        desc.clear();
    }
    ~Plan() {
        if (desc.capacity() > desc_pool().capacity()) desc_pool().swap(desc);
    }
    Plan(const Plan &) = delete;
    Plan &operator=(const Plan &) = delete;
    u64 *limbs(size_t count) {
        const size_t bytes = count * c->N * 8;
        u64 *p = ws ? (u64 *)(ws + scratch) : (u64 *)(uintptr_t)(0x1000 + scratch);
        scratch += (bytes + 255) & ~(size_t)255;
        return p;
    }
    template <class T>
    void add(int kind, int op, const std::vector<T> &v, u64 seed = 0) {
        if (v.empty()) return;
        if constexpr (std::is_same<T, Item>::value) {
            // NTT launches: with the FP64 engine enabled, items whose prime
            // is below 2^50 go to one launch and the rest to another (each
            // kernel carries one engine); relative order is kept
            if ((kind == 0 || kind == 1) && c->tb.ntt_fp) {
                // a ModUp item converts in FP64 too: its digit's primes must also be below 2^50;
                // a ModDown + rescale item needs the dropped prime q_l below 2^50
                const bool modup = kind == 0 && (op == F_MODUP || (op >= F_MODUP_S1 && op < F_MODUP_S1 + 4));
                const bool relin = kind == 0 && (op == F_RELIN || op == F_RELIN_RS || (op >= F_RELIN_P1 && op <= F_RELIN_RS_P1 + 1));
                auto fp_ok = [&](const Item &it) {
                    if (c->primes[it.prime] >= kFpPrimeBound) return false;
                    if (relin && c->primes[it.a] >= kFpPrimeBound) return false;
                    // sources of 2^50 or more are converted in FP64 below 2^15 by
                    // the generic and one-prime-digit kernels; the fixed
                    // multi-prime kernels (2^13 .. 2^15) and every 2^15 kernel
                    // need every source below 2^50
                    if (modup && (c->log_n >= 15 || (c->log_n >= 13 && op > F_MODUP_S1 && op < F_MODUP_S1 + 4))) {
                        const u32 sz = op == F_MODUP ? it.b : (u32)(op - F_MODUP_S1 + 1);
                        for (u32 i = 0; i < sz; i++)
                            if (c->primes[it.c * c->alpha + i] >= kFpPrimeBound) return false;
                    }
                    return true;
                };
                // written straight into the descriptor buffer: FP64 items, then the rest
                std::vector<uint8_t> cls(v.size());
                size_t n_fp = 0;
                for (size_t i = 0; i < v.size(); i++) n_fp += (cls[i] = fp_ok(v[i]) ? 1 : 0);
                for (int want = 1; want >= 0; want--) {
                    const size_t n = want ? n_fp : v.size() - n_fp;
                    if (!n) continue;
                    Item *dst = (Item *)reserve(n * sizeof(Item), kind, op, (int)n, seed, want);
                    for (size_t i = 0; i < v.size(); i++)
                        if (cls[i] == want) *dst++ = v[i];
                }
                return;
            }
        }
        if constexpr (std::is_same<T, IpItem>::value || std::is_same<T, HoItem>::value) {
            // key-switch inner product and hoisted rotations: items of primes
            // below 2^50 take the FP64 kernel
            if ((kind == 3 || kind == 5) && c->tb.ntt_fp) {
                std::vector<uint8_t> cls(v.size());
                size_t n_fp = 0;
                for (size_t i = 0; i < v.size(); i++) n_fp += (cls[i] = c->primes[v[i].prime] < kFpPrimeBound ? 1 : 0);
                for (int want = 1; want >= 0; want--) {
                    const size_t n = want ? n_fp : v.size() - n_fp;
                    if (!n) continue;
                    T *dst = (T *)reserve(n * sizeof(T), kind, op, (int)n, seed, want);
                    for (size_t i = 0; i < v.size(); i++)
                        if (cls[i] == want) *dst++ = v[i];
                }
                return;
            }
        }
        if constexpr (std::is_same<T, EwItem>::value) op = (int)v[0].op;  // for the launch name
        memcpy(reserve(v.size() * sizeof(T), kind, op, (int)v.size(), seed, 0), v.data(), v.size() * sizeof(T));
    }
    // space for one launch's descriptors (256-byte aligned) and its record
    void *reserve(size_t bytes, int kind, int op, int n, u64 seed, int fp) {
        const size_t off = (desc.size() + 255) & ~(size_t)255;
        desc.resize(off + bytes);
        launches.push_back({kind, op, off, n, seed, fp});
        return desc.data() + off;
    }
    size_t total() const { return ((scratch + 255) & ~(size_t)255) + desc.size(); }
    int run(size_t ws_bytes, hipStream_t s) {
        if (total() > ws_bytes)
            return fail(CKKS_ENOMEM, "workspace too small: need %zu bytes, got %zu", total(), ws_bytes);
        if (!ws && total()) return fail(CKKS_EINVAL, "null workspace");
        if (((uintptr_t)ws) & 255) return fail(CKKS_EINVAL, "workspace not 256-byte aligned");
        if (c->log_n > kMaxFusedLogN)
            for (const Launch &L : launches)
                if (!((L.kind == 0 && L.op == F_COPY) || (L.kind == 1 && L.op == I_COPY) || L.kind == 2))
                    return fail(CKKS_EPARAMS, "N = 2^%u supports plain transforms (ckks_ntt, ckks_intt) and "
                                "element-wise operations only", c->log_n);
        const size_t doff = (scratch + 255) & ~(size_t)255;
        uint8_t *dbase = ws + doff;
        const int urc = upload(c, ws + doff, desc.data(), desc.size(), s, &dbase);
        if (urc != CKKS_OK) return urc;
        for (const Launch &L : launches) {
            const uint8_t *p = dbase + L.off;
            hipError_t e = hipSuccess;
            ProfRec rec;
            const bool prof = g_prof_on && !g_no_alloc;
            if (prof) {
                rec.name = launch_name(L.kind, L.op, c->log_n);
                rec.items = (u32)L.n;
                HIP_TRY(hipEventCreate(&rec.e0));
                HIP_TRY(hipEventCreate(&rec.e1));
                HIP_TRY(hipEventRecord(rec.e0, s));
            }
            DevTables tl = c->tb;
            tl.ntt_fp = (u32)L.fp;
            e = issue(c, s, [tb = tl, L, p](hipStream_t st) {
                switch (L.kind) {
                    case 0: return launch_fwd(tb, L.op, (const Item *)p, L.n, L.seed, st);
                    case 1: return launch_inv(tb, L.op, (const Item *)p, L.n, st);
                    case 2: return launch_ew(tb, (const EwItem *)p, L.n, L.seed, st);
                    case 3: return launch_ip(tb, (const IpItem *)p, L.n, st);
                    case 5: return launch_hoist(tb, L.op, (const HoItem *)p, L.n, st);
                    case 6: return launch_ip_seq(tb, (const IpSeqItem *)p, L.n, st);
                }
                return hipErrorInvalidValue;
            });
            if (e != hipSuccess) return fail(CKKS_EDEVICE, "kernel launch: %s", hipGetErrorString(e));
            if (prof) {
                HIP_TRY(hipEventRecord(rec.e1, s));
                g_prof.push_back(rec);
            }
        }
        return CKKS_OK;
    }
};

// ModUp items, one launch per digit size (ckks_host.cpp)
void add_modup(Plan &P, const std::vector<Item> &v);
// ModDown + rescale kernel for the context's special-prime count
int relin_op(const ckks_ctx *c, bool rescale);
int moddown_op(const ckks_ctx *c);
// one ciphertext's share of the key-switch inner product
struct IpCt {
    u32 level;
    const u64 *key;  // switching key of this ciphertext (per item: one client's key each)
    const u64 *ext;
    u64 *acc;
    std::vector<const u64 *> own0, own1;  // per data limb t <= level
    std::vector<const u64 *> own2, own3;  // a0, b0 of a product (P d folded into the sums)
};
// items of the inner product: ciphertexts of one level and one switching
// key are grouped by kIpCts so that each key residue is loaded once per
// group (requests of different clients, i.e. different keys, share the
// launch but not an item). Items are
// emitted prime by prime (every group's item for prime 0, then prime 1, ...)
// so that the blocks in flight at any time share one prime's key limbs
// (2 beta limbs), which then stay in L2 instead of every group re-reading
// all primes' keys.
inline bool ip_before(const IpCt &x, const IpCt &y) {
    return x.level != y.level ? x.level < y.level : (uintptr_t)x.key < (uintptr_t)y.key;
}
inline bool ip_same(const IpCt &x, const IpCt &y) { return x.level == y.level && x.key == y.key; }
void add_ip_items(const ckks_ctx *c, std::vector<IpItem> &v, const std::vector<IpCt> &cts);
void add_ip(Plan &P, const std::vector<IpCt> &cts);
// transform items launched prime by prime (twiddle tables shared in L2)
void order_by_prime(std::vector<Item> &v);

inline u64 *limb(const ckks_ctx *c, const ckks_ct &ct, u32 poly, u32 i) {
    return ct.data + ((size_t)poly * ct.limb_stride + i) * c->N;
}
inline Item item0() {
    Item it;
    memset(&it, 0, sizeof it);
    return it;
}
inline EwItem ew0() {
    EwItem it;
    memset(&it, 0, sizeof it);
    return it;
}

inline int check_ctx(const ckks_ctx *c) {
    if (!c) return fail(CKKS_EINVAL, "null context");
    if (!c->uploaded) return fail(CKKS_EINVAL, "context tables not uploaded (ckks_ctx_upload)");
    return CKKS_OK;
}
// device buffers of ciphertexts and plaintexts: the kernels move residues
// in 16-byte pairs
inline bool bad_ptr(const void *p) { return !p || (((uintptr_t)p) & 15); }
inline int check_ct(const ckks_ctx *c, const ckks_ct &ct, const char *what) {
    if (bad_ptr(ct.data)) return fail(CKKS_EINVAL, "%s: null or not 16-byte aligned data", what);
    if (ct.level >= c->n_q) return fail(CKKS_ELEVEL, "%s: level %u beyond top %u", what, ct.level, c->n_q - 1);
    if (ct.limb_stride < ct.level + 1) return fail(CKKS_EINVAL, "%s: limb_stride < level + 1", what);
    if (ct.n_poly < 2 || ct.n_poly > 3) return fail(CKKS_EINVAL, "%s: n_poly must be 2 or 3", what);
    return CKKS_OK;
}
#define CK(x)                  \
    do {                       \
        int r_ = (x);          \
        if (r_ != CKKS_OK) return r_; \
    } while (0)

// ---------------------------------------------------------------------
// key switching core (ckks_eval.cpp): for each b, d_b (NTT form, L_b
// limbs) -> out_c = addend_c + ModDown(acc_c) for c = 0, 1.
// ---------------------------------------------------------------------
// ---------------------------------------------------------------------
// key switching core: for each b, d_b (NTT form, L_b limbs) ->
// out_c = addend_c + ModDown(acc_c) for c = 0, 1.
// ---------------------------------------------------------------------
struct KsJob {
    u32 level;
    const u64 *key;               // switching key (device)
    std::vector<const u64 *> dl;  // limbs of the polynomial to switch (NTT form)
    const u64 *addend[2];         // limb 0 of the poly added to each output, or null
    u64 *out[2];                  // limb 0 of each output poly (limbs contiguous)
};
void plan_keyswitch(Plan &P, const std::vector<KsJob> &jobs);
// the fused HMult's launches (ckks_eval.cpp; also sized by ckks_workspace_bytes)
int plan_hmult(Plan &P, const u64 *const *rk, const ckks_ct *a, const ckks_ct *b, ckks_ct *out, u32 B);
// element-wise binary operations (ckks_eval.cpp)
int ew_binary(const ckks_ctx *c, u32 op, const ckks_ct *a, const ckks_ct *b, const ckks_pt *p, const int64_t *v,
              const double *vs, ckks_ct *out, u32 B, void *ws, size_t ws_bytes, void *stream, const char *name);
}  // namespace ckks
