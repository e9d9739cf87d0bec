// Host runtime behind the C ABI of libckks_hip.so: parameter checks, prime
// and root search, device table image, FP64 canonical-embedding encoder,
// exact CRT decoder, and the per-op planners that turn ciphertext
// descriptors into flat work-item tables for the gfx950 kernels.
//
// The library never allocates device memory: every call receives a caller
// workspace, carves scratch limbs from its front and places the work-item
// tables at its end, uploads the tables with one asynchronous copy and
// launches the kernels on the caller's stream.
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
hipError_t launch_hoist(const DevTables &tb, const HoItem *items, int n, hipStream_t s);
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
    F_MODUP_S1 = 8, F_RELIN_P1 = 12, F_RELIN_RS_P1 = 14
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
// errors
// ---------------------------------------------------------------------
static thread_local std::string g_err;
int set_error(int code, const char *msg) {
    g_err = msg;
    return code;
}
static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
#define HIP_TRY(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) return fail(CKKS_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------
// integer helpers
// ---------------------------------------------------------------------
static u64 mulmod(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }
static u64 powmod(u64 a, u64 e, u64 q) {
    u64 r = 1 % q;
    a %= q;
    for (; e; e >>= 1) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
    }
    return r;
}
static u64 invmod(u64 a, u64 q) { return powmod(a, q - 2, q); }
static u64 shoup_companion(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }
static bool is_prime(u64 n) {
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
static u32 bitrev(u32 x, u32 bits) {
    u32 r = 0;
    for (u32 i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}
// smallest primitive 2N-th root of unity mod q
static u64 smallest_psi(u64 q, u32 log_n) {
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
static void big_mul_small(Big &a, u64 m) {
    u64 carry = 0;
    for (auto &w : a) {
        u128 t = (u128)w * m + carry;
        w = (u64)t;
        carry = (u64)(t >> 64);
    }
    if (carry) a.push_back(carry);
}
static int big_cmp(const Big &a, const Big &b) {
    size_t n = std::max(a.size(), b.size());
    for (size_t i = n; i-- > 0;) {
        u64 x = i < a.size() ? a[i] : 0, y = i < b.size() ? b[i] : 0;
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}
static void big_sub(Big &a, const Big &b) {  // a -= b, a >= b
    u64 borrow = 0;
    for (size_t i = 0; i < a.size(); i++) {
        u64 y = i < b.size() ? b[i] : 0;
        u128 t = (u128)a[i] - y - borrow;
        a[i] = (u64)t;
        borrow = (u64)(t >> 64) ? 1 : 0;
    }
}
static void big_addmul(Big &acc, const Big &b, u64 m) {  // acc += b * m
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
static double big_to_double(const Big &a) {
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
    ~Staging() {
        for (auto &r : inflight) {
            hipEventSynchronize(r.done);
            hipEventDestroy(r.done);
        }
        if (buf) hipHostFree(buf);
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

static size_t align_words(size_t w) { return (w + 31) & ~(size_t)31; }  // 256 bytes

extern "C" const char *ckks_last_error(void) { return g_err.c_str(); }

extern "C" int ckks_find_primes(uint32_t log_n, const uint32_t *bits, uint32_t n, uint64_t *out) {
    if (!bits || !out || log_n < 1 || log_n > 20) return fail(CKKS_EINVAL, "find_primes: bad args");
    const u64 two_n = 2ull << log_n;
    for (u32 i = 0; i < n; i++) {
        if (bits[i] < 2 || bits[i] > 62) return fail(CKKS_EINVAL, "find_primes: bits out of range");
        u64 top = (bits[i] == 64) ? ~0ull : ((1ull << bits[i]) - 1);
        u64 c = (top / two_n) * two_n + 1;
        if (c > top) c -= two_n;
        for (;;) {
            if (c < two_n) return fail(CKKS_EPARAMS, "find_primes: exhausted");
            bool used = false;
            for (u32 k = 0; k < i; k++) used |= out[k] == c;
            if (!used && is_prime(c)) break;
            c -= two_n;
        }
        out[i] = c;
    }
    return CKKS_OK;
}

extern "C" int ckks_parameterise(uint32_t cost, uint32_t scale_bits, double special_mult,
                                 uint32_t *bits_out, uint32_t bits_cap, uint32_t *n_bits, uint32_t *log_n) {
    if (!bits_out || !n_bits || !log_n || bits_cap < cost + 2) return fail(CKKS_EINVAL, "parameterise: bad args");
    u32 count = cost + 2, sum = 0;
    for (u32 i = 0; i < count; i++) bits_out[i] = scale_bits;
    bits_out[0] = (u32)(bits_out[0] * special_mult);
    bits_out[count - 1] = (u32)(bits_out[count - 1] * special_mult);
    for (u32 i = 0; i < count; i++) sum += bits_out[i];
    u64 b = 27;
    while (b < sum) b *= 2;
    u64 n = 1024 * (b / 27);
    u32 ln = 0;
    while ((1ull << ln) < n) ln++;
    *n_bits = count;
    *log_n = ln;
    return CKKS_OK;
}

extern "C" int ckks_ctx_create(const ckks_params *p, ckks_ctx **out) {
    if (!p || !out || !p->q || (p->n_p && !p->p)) return fail(CKKS_EINVAL, "ctx_create: null argument");
    if (p->log_n < kMinLogN || p->log_n > kMaxLogN)
        return fail(CKKS_EPARAMS, "ctx_create: log_n %u outside [%d, %d]", p->log_n, kMinLogN, kMaxLogN);
    if (p->n_q < 1 || p->n_p < 1 || p->n_q + p->n_p > (u32)kMaxPrimes || p->dnum < 1 || p->dnum > p->n_q)
        return fail(CKKS_EPARAMS, "ctx_create: bad prime counts / dnum");
    ckks_ctx *c = new ckks_ctx();
    c->tb.ntt_wide = 0;
    c->tb.ew_log = 2;
    c->tb.xcd_remap = 1;
    c->tb.fuse_tail = 0;
    c->tb.ip_cts = kIpCts;
    c->tb.lin_mfma = 1;
    c->tb.ntt_fp = 1;
    c->log_n = p->log_n;
    c->N = 1u << p->log_n;
    c->n_q = p->n_q;
    c->n_p = p->n_p;
    c->n_prim = p->n_q + p->n_p;
    c->dnum = p->dnum;
    c->alpha = (p->n_q + p->dnum - 1) / p->dnum;
    c->digits_top = (p->n_q + c->alpha - 1) / c->alpha;
    for (u32 i = 0; i < p->n_q; i++) c->primes.push_back(p->q[i]);
    for (u32 i = 0; i < p->n_p; i++) c->primes.push_back(p->p[i]);
    const u64 two_n = 2ull * c->N;
    for (u32 i = 0; i < c->n_prim; i++) {
        u64 q = c->primes[i];
        if (q >= (1ull << 61) || q % two_n != 1 || !is_prime(q)) {
            delete c;
            return fail(CKKS_EPARAMS, "ctx_create: prime %u (%llu) must be a prime < 2^61, 1 mod 2N", i,
                        (unsigned long long)q);
        }
        for (u32 k = 0; k < i; k++)
            if (c->primes[k] == q) {
                delete c;
                return fail(CKKS_EPARAMS, "ctx_create: duplicate prime");
            }
    }
    const u32 N = c->N, np = c->n_prim, nq = c->n_q, npp = c->n_p, A = c->alpha;
    // ---- device image layout
    size_t w = 0;
    c->off_pc = w;
    w = align_words(w + np * (sizeof(PrimeConst) / 8));
    c->off_tw = w;
    w = align_words(w + (size_t)np * N * 2);
    c->off_itw = w;
    w = align_words(w + (size_t)np * N * 2);
    c->off_twf = w;
    w = align_words(w + (size_t)np * N * 2);
    c->off_itwf = w;
    w = align_words(w + (size_t)np * N * 2);
    c->off_modup = w;
    const u32 blockw = modup_block_words(A, np);
    w = align_words(w + (size_t)c->digits_top * A * blockw);
    c->off_moddown = w;
    w = align_words(w + 2 * npp + (size_t)npp * nq);
    c->off_rescale = w;
    w = align_words(w + (size_t)nq * nq * 2);
    c->image.assign(w, 0);
    u64 *img = c->image.data();
    // ---- per prime
    u64 Pmod[kMaxPrimes];
    for (u32 i = 0; i < np; i++) {
        const u64 q = c->primes[i];
        PrimeConst pc{};
        pc.q = q;
        pc.two_q = 2 * q;
        u128 r = (~(u128)0) / q;  // floor((2^128 - 1) / q) == floor(2^128 / q) for odd q
        pc.br_hi = (u64)(r >> 64);
        pc.br_lo = (u64)r;
        pc.mu = (u64)((~(u64)0) / q);
        const u64 psi = smallest_psi(q, c->log_n);
        if (!psi) {
            delete c;
            return fail(CKKS_EPARAMS, "ctx_create: no 2N-th root for prime %u", i);
        }
        // forward twiddle table tw[k] = psi^brv(k), inverse itw[k] = tw[k]^-1
        ulonglong2 *tw = reinterpret_cast<ulonglong2 *>(img + c->off_tw) + (size_t)i * N;
        ulonglong2 *itw = reinterpret_cast<ulonglong2 *>(img + c->off_itw) + (size_t)i * N;
        std::vector<u64> pw(N);
        u64 x = 1;
        for (u32 k = 0; k < N; k++) pw[k] = x, x = mulmod(x, psi, q);
        for (u32 k = 0; k < N; k++) {
            const u64 v = pw[bitrev(k, c->log_n)];
            const u64 iv = invmod(v, q);
            tw[k].x = v;
            tw[k].y = shoup_companion(v, q);
            itw[k].x = iv;
            itw[k].y = shoup_companion(iv, q);
        }
        pc.ninv = invmod(N % q, q);
        pc.ninv_sh = shoup_companion(pc.ninv, q);
        pc.last_w = mulmod(itw[1].x, pc.ninv, q);
        pc.last_w_sh = shoup_companion(pc.last_w, q);
        // FP64 copies (exact for q < 2^50; w / q and 1 / q correctly rounded).
        // Transform multipliers are stored centred, |w| <= (q - 1) / 2, so
        // that |w / q| <= 1/2: a product with any |y| < 2^52 then has
        // |y w / q| < 2^51, where the rounding constant of fp_mulmod gives
        // the nearest integer quotient
        const double qd = (double)q;
        auto centred = [q, qd](u64 v) { return v > q / 2 ? (double)v - qd : (double)v; };
        double *twf = reinterpret_cast<double *>(img + c->off_twf) + (size_t)i * N * 2;
        double *itwf = reinterpret_cast<double *>(img + c->off_itwf) + (size_t)i * N * 2;
        for (u32 k = 0; k < N; k++) {
            twf[2 * k] = centred(tw[k].x);
            twf[2 * k + 1] = twf[2 * k] / qd;
            itwf[2 * k] = centred(itw[k].x);
            itwf[2 * k + 1] = itwf[2 * k] / qd;
        }
        pc.qf = qd;
        pc.qinvf = 1.0 / qd;
        pc.qmf = 4503599627370496.0 + qd;
        pc.ninvf = centred(pc.ninv);
        pc.ninvqf = pc.ninvf / qd;
        pc.last_wf = centred(pc.last_w);
        pc.last_wqf = pc.last_wf / qd;
        u64 P = 1;
        for (u32 m = 0; m < npp; m++) P = mulmod(P, c->primes[nq + m] % q, q);
        Pmod[i] = P;
        pc.pmod = P;
        pc.pmod_sh = shoup_companion(P, q);
        if (i < nq) {
            pc.pinv = invmod(P, q);
            pc.pinv_sh = shoup_companion(pc.pinv, q);
        }
        memcpy(img + c->off_pc + i * (sizeof(PrimeConst) / 8), &pc, sizeof pc);
    }
    (void)Pmod;
    // ---- ModUp blocks: digit j truncated to s primes
    for (u32 j = 0; j < c->digits_top; j++)
        for (u32 s = 1; s <= A; s++) {
            u64 *blk = img + c->off_modup + (size_t)(j * A + s - 1) * blockw;
            const u32 lo = j * A;
            if (lo + s > nq) continue;
            for (u32 i = 0; i < s; i++) {
                const u64 qi = c->primes[lo + i];
                u64 hat = 1;
                for (u32 m = 0; m < s; m++)
                    if (m != i) hat = mulmod(hat, c->primes[lo + m] % qi, qi);
                const u64 inv = invmod(hat, qi);
                blk[2 * i] = inv;
                blk[2 * i + 1] = shoup_companion(inv, qi);
                for (u32 t = 0; t < np; t++) {
                    const u64 qt = c->primes[t];
                    u64 h = 1;
                    for (u32 m = 0; m < s; m++)
                        if (m != i) h = mulmod(h, c->primes[lo + m] % qt, qt);
                    blk[2 * A + (size_t)i * np + t] = h;
                }
            }
        }
    // ---- ModDown block
    {
        u64 *blk = img + c->off_moddown;
        for (u32 m = 0; m < npp; m++) {
            const u64 pm = c->primes[nq + m];
            u64 hat = 1;
            for (u32 k = 0; k < npp; k++)
                if (k != m) hat = mulmod(hat, c->primes[nq + k] % pm, pm);
            const u64 inv = invmod(hat, pm);
            blk[2 * m] = inv;
            blk[2 * m + 1] = shoup_companion(inv, pm);
            for (u32 t = 0; t < nq; t++) {
                const u64 qt = c->primes[t];
                u64 h = 1;
                for (u32 k = 0; k < npp; k++)
                    if (k != m) h = mulmod(h, c->primes[nq + k] % qt, qt);
                blk[2 * npp + (size_t)m * nq + t] = h;
            }
        }
    }
    // ---- rescale: q_l^-1 mod q_i
    for (u32 l = 1; l < nq; l++)
        for (u32 i = 0; i < l; i++) {
            const u64 qi = c->primes[i];
            const u64 inv = invmod(c->primes[l] % qi, qi);
            u64 *e = img + c->off_rescale + ((size_t)l * nq + i) * 2;
            e[0] = inv;
            e[1] = shoup_companion(inv, qi);
        }
    // ---- encoder tables
    const u32 M = N / 2;
    c->fft_roots.resize(M);
    for (u32 k = 0; k < M; k++) c->fft_roots[k] = std::polar(1.0, 2.0 * M_PI * (double)k / (double)M);
    c->twist.resize(M);
    for (u32 i = 0; i < M; i++) c->twist[i] = std::polar(1.0, M_PI * (double)i / (double)N);
    c->slot_index.resize(M);
    u64 e = 1;
    for (u32 j = 0; j < M; j++) {
        c->slot_index[j] = (u32)((e - 1) / 4);
        e = e * 5 % two_n;
    }
    // ---- CRT tables per level
    c->qhat.resize(nq);
    c->qhat_inv.resize(nq);
    c->Q.resize(nq);
    c->Qhalf.resize(nq);
    for (u32 l = 0; l < nq; l++) {
        Big Q{1};
        for (u32 i = 0; i <= l; i++) big_mul_small(Q, c->primes[i]);
        c->Q[l] = Q;
        Big h = Q;  // Q >> 1
        for (size_t k = 0; k < h.size(); k++) h[k] = (h[k] >> 1) | (k + 1 < h.size() ? (h[k + 1] << 63) : 0);
        c->Qhalf[l] = h;
        for (u32 i = 0; i <= l; i++) {
            Big qh{1};
            u64 hm = 1;
            for (u32 m = 0; m <= l; m++)
                if (m != i) big_mul_small(qh, c->primes[m]), hm = mulmod(hm, c->primes[m] % c->primes[i], c->primes[i]);
            c->qhat[l].push_back(qh);
            c->qhat_inv[l].push_back(invmod(hm, c->primes[i]));
        }
    }
    *out = c;
    return CKKS_OK;
}

extern "C" void ckks_ctx_destroy(ckks_ctx *ctx) { delete ctx; }
extern "C" size_t ckks_ctx_device_bytes(const ckks_ctx *c) { return c ? c->image.size() * 8 : 0; }
extern "C" uint32_t ckks_ctx_log_n(const ckks_ctx *c) { return c ? c->log_n : 0; }
extern "C" uint32_t ckks_ctx_max_level(const ckks_ctx *c) { return c ? c->n_q - 1 : 0; }
extern "C" uint32_t ckks_ctx_digits(const ckks_ctx *c, uint32_t level) {
    return c ? (level + 1 + c->alpha - 1) / c->alpha : 0;
}
extern "C" uint64_t ckks_ctx_prime(const ckks_ctx *c, uint32_t i) {
    return (c && i < c->n_prim) ? c->primes[i] : 0;
}

extern "C" int ckks_ctx_upload(ckks_ctx *c, void *dev, void *stream) {
    if (!c || !dev) return fail(CKKS_EINVAL, "ctx_upload: null argument");
    if (((uintptr_t)dev) & 255) return fail(CKKS_EINVAL, "ctx_upload: device buffer not 256-byte aligned");
    HIP_TRY(hipMemcpyAsync(dev, c->image.data(), c->image.size() * 8, hipMemcpyHostToDevice, (hipStream_t)stream));
    const u64 *base = (const u64 *)dev;
    DevTables &t = c->tb;
    t.pc = reinterpret_cast<const PrimeConst *>(base + c->off_pc);
    t.tw = reinterpret_cast<const ulonglong2 *>(base + c->off_tw);
    t.itw = reinterpret_cast<const ulonglong2 *>(base + c->off_itw);
    t.twf = reinterpret_cast<const double2 *>(base + c->off_twf);
    t.itwf = reinterpret_cast<const double2 *>(base + c->off_itwf);
    t.modup = base + c->off_modup;
    t.moddown = base + c->off_moddown;
    t.rescale = reinterpret_cast<const ulonglong2 *>(base + c->off_rescale);
    t.log_n = c->log_n;
    t.n_q = c->n_q;
    t.n_p = c->n_p;
    t.n_prim = c->n_prim;
    t.alpha = c->alpha;
    t.n_digits_top = c->digits_top;
    c->uploaded = true;
    return CKKS_OK;
}

extern "C" int ckks_ctx_set_tuning(ckks_ctx *c, int knob, int value) {
    if (!c) return fail(CKKS_EINVAL, "set_tuning: null context");
    switch (knob) {
        case CKKS_TUNE_NTT_WIDE:
            if (value != 0 && value != 1) return fail(CKKS_EINVAL, "set_tuning: NTT_WIDE takes 0 or 1");
            if (value && (c->log_n < 11 || c->log_n > 14)) return fail(CKKS_EINVAL, "set_tuning: NTT_WIDE needs N in 2^11..2^14");
            c->tb.ntt_wide = (u32)value;
            return CKKS_OK;
        case CKKS_TUNE_EW_LOG:
            if (value < 1 || value > 3) return fail(CKKS_EINVAL, "set_tuning: EW_LOG takes 1..3");
            c->tb.ew_log = (u32)value;
            return CKKS_OK;
        case CKKS_TUNE_XCD_REMAP:
            if (value != 0 && value != 1) return fail(CKKS_EINVAL, "set_tuning: XCD_REMAP takes 0 or 1");
            c->tb.xcd_remap = (u32)value;
            return CKKS_OK;
        case CKKS_TUNE_FUSE_TAIL:
            if (value != 0 && value != 1) return fail(CKKS_EINVAL, "set_tuning: FUSE_TAIL takes 0 or 1");
            c->tb.fuse_tail = (u32)value;
            return CKKS_OK;
        case CKKS_TUNE_LIN_MFMA:
            if (value != 0 && value != 1) return fail(CKKS_EINVAL, "set_tuning: LIN_MFMA takes 0 or 1");
            c->tb.lin_mfma = (u32)value;
            return CKKS_OK;
        case CKKS_TUNE_NTT_FP:
            if (value != 0 && value != 1) return fail(CKKS_EINVAL, "set_tuning: NTT_FP takes 0 or 1");
            c->tb.ntt_fp = (u32)value;
            return CKKS_OK;
        case CKKS_TUNE_IP_CTS:
            if (value != 2 && value != kIpCts && value != kIpSeqCts)
                return fail(CKKS_EINVAL, "set_tuning: IP_CTS takes 2, %d or %d", kIpCts, kIpSeqCts);
            c->tb.ip_cts = (u32)value;
            return CKKS_OK;
    }
    return fail(CKKS_EINVAL, "set_tuning: unknown knob");
}
extern "C" int ckks_ctx_get_tuning(const ckks_ctx *c, int knob) {
    if (!c) return -1;
    switch (knob) {
        case CKKS_TUNE_NTT_WIDE: return (int)c->tb.ntt_wide;
        case CKKS_TUNE_EW_LOG: return (int)c->tb.ew_log;
        case CKKS_TUNE_XCD_REMAP: return (int)c->tb.xcd_remap;
        case CKKS_TUNE_FUSE_TAIL: return (int)c->tb.fuse_tail;
        case CKKS_TUNE_IP_CTS: return (int)c->tb.ip_cts;
        case CKKS_TUNE_LIN_MFMA: return (int)c->tb.lin_mfma;
        case CKKS_TUNE_NTT_FP: return (int)c->tb.ntt_fp;
    }
    return -1;
}

extern "C" size_t ckks_ct_bytes(const ckks_ctx *c, uint32_t n_poly, uint32_t level) {
    return c ? (size_t)n_poly * (level + 1) * c->N * 8 : 0;
}
extern "C" size_t ckks_pt_bytes(const ckks_ctx *c, uint32_t level) { return c ? (size_t)(level + 1) * c->N * 8 : 0; }
extern "C" size_t ckks_key_bytes(const ckks_ctx *c, int kind) {
    if (!c) return 0;
    const size_t limb = (size_t)c->N * 8;
    switch (kind) {
        case CKKS_KEY_SECRET: return c->n_prim * limb;
        case CKKS_KEY_PUBLIC: return 2 * c->n_q * limb;
        case CKKS_KEY_SWITCH: return (size_t)c->digits_top * 2 * c->n_prim * limb;
    }
    return 0;
}
extern "C" uint32_t ckks_galois_elt(const ckks_ctx *c, int32_t step) {
    if (!c) return 0;
    const i64 half = c->N / 2;
    i64 r = ((i64)step % half + half) % half;
    return (u32)powmod(5, (u64)r, 2ull * c->N);
}

// ---------------------------------------------------------------------
// encoder / decoder (host FP64)
// ---------------------------------------------------------------------
// in-place iterative radix-2 DFT of size M: X_k = sum_i x_i e^{sign 2 pi i k i / M}
static void host_fft(const ckks_ctx *c, std::vector<std::complex<double>> &x, int sign) {
    const u32 M = (u32)x.size();
    u32 lg = 0;
    while ((1u << lg) < M) lg++;
    for (u32 i = 0; i < M; i++) {
        u32 r = bitrev(i, lg);
        if (r > i) std::swap(x[i], x[r]);
    }
    for (u32 len = 2; len <= M; len <<= 1) {
        const u32 half = len >> 1, step = M / len;
        for (u32 s = 0; s < M; s += len)
            for (u32 j = 0; j < half; j++) {
                std::complex<double> w = c->fft_roots[(size_t)j * step];
                if (sign < 0) w = std::conj(w);
                const std::complex<double> u = x[s + j], v = x[s + j + half] * w;
                x[s + j] = u + v;
                x[s + j + half] = u - v;
            }
    }
}

extern "C" int ckks_encode(const ckks_ctx *c, const double *re, const double *im, size_t n, double scale,
                           int64_t *coeffs) {
    if (!c || (!re && n) || !coeffs) return fail(CKKS_EINVAL, "encode: null argument");
    const u32 M = c->N / 2;
    if (n > M) return fail(CKKS_EINVAL, "encode: %zu values exceed %u slots", n, M);
    std::vector<std::complex<double>> Z(M, 0.0);
    for (size_t j = 0; j < n; j++) Z[c->slot_index[j]] = std::complex<double>(re[j], im ? im[j] : 0.0) * scale;
    host_fft(c, Z, -1);  // sum_k Z_k e^{-2 pi i k i / M}
    for (u32 i = 0; i < M; i++) {
        const std::complex<double> wv = Z[i] / (double)M * std::conj(c->twist[i]);
        const double a = wv.real(), b = wv.imag();
        const double ra = a < 0 ? -floor(-a + 0.5) : floor(a + 0.5);
        const double rb = b < 0 ? -floor(-b + 0.5) : floor(b + 0.5);
        if (fabs(ra) >= 4611686018427387904.0 || fabs(rb) >= 4611686018427387904.0)
            return fail(CKKS_EINVAL, "encode: coefficient reaches 2^62 (scale too large)");
        coeffs[i] = (int64_t)ra;
        coeffs[i + M] = (int64_t)rb;
    }
    return CKKS_OK;
}

// a constant c at scale s is the constant polynomial round_half_away(c s)
static int scalar_int(double c, double scale, int64_t *out) {
    const double v = c * scale;
    if (!std::isfinite(v)) return fail(CKKS_EINVAL, "encode_scalar: constant or scale not finite");
    const double r = v < 0 ? -floor(-v + 0.5) : floor(v + 0.5);
    if (fabs(r) >= 4611686018427387904.0) return fail(CKKS_EINVAL, "encode_scalar: |c * scale| reaches 2^62");
    *out = (int64_t)r;
    return CKKS_OK;
}

extern "C" int ckks_encode_scalars(const ckks_ctx *c, const double *vals, size_t n, double scale, int64_t *out) {
    if (!c || (n && (!vals || !out))) return fail(CKKS_EINVAL, "encode_scalars: null argument");
    for (size_t k = 0; k < n; k++) {
        const int r = scalar_int(vals[k], scale, out + k);
        if (r != CKKS_OK) return r;
    }
    return CKKS_OK;
}

extern "C" int ckks_encode_scalar(const ckks_ctx *c, double val, double scale, uint32_t level, uint64_t *per_limb) {
    if (!c || !per_limb) return fail(CKKS_EINVAL, "encode_scalar: null argument");
    if (level >= c->n_q) return fail(CKKS_ELEVEL, "encode_scalar: level %u beyond top %u", level, c->n_q - 1);
    int64_t v;
    const int r = scalar_int(val, scale, &v);
    if (r != CKKS_OK) return r;
    for (u32 i = 0; i <= level; i++) {
        const u64 q = c->primes[i];
        const u64 m = (u64)(v < 0 ? -(v + 1) : v) % q;  // |v| - 1 for negative v, no overflow
        per_limb[i] = v >= 0 ? m : (q - 1 - m);
    }
    return CKKS_OK;
}

extern "C" int ckks_decode(const ckks_ctx *c, const uint64_t *res, uint32_t level, double scale, double *re,
                           double *im, size_t n) {
    if (!c || !res || (!re && n)) return fail(CKKS_EINVAL, "decode: null argument");
    if (level >= c->n_q) return fail(CKKS_ELEVEL, "decode: level %u out of range", level);
    const u32 N = c->N, M = N / 2;
    if (n > M) return fail(CKKS_EINVAL, "decode: too many slots");
    std::vector<double> m(N);
    const Big &Q = c->Q[level], &Qh = c->Qhalf[level];
    for (u32 j = 0; j < N; j++) {
        Big acc(Q.size() + 2, 0);
        for (u32 i = 0; i <= level; i++) {
            const u64 qi = c->primes[i];
            const u64 y = mulmod(res[(size_t)i * N + j] % qi, c->qhat_inv[level][i], qi);
            big_addmul(acc, c->qhat[level][i], y);
        }
        while (big_cmp(acc, Q) >= 0) big_sub(acc, Q);
        if (big_cmp(acc, Qh) > 0) {
            Big neg = Q;
            neg.resize(acc.size(), 0);
            big_sub(neg, acc);
            m[j] = -big_to_double(neg);
        } else {
            m[j] = big_to_double(acc);
        }
    }
    std::vector<std::complex<double>> w(M);
    for (u32 i = 0; i < M; i++) w[i] = std::complex<double>(m[i], m[i + M]) * c->twist[i];
    host_fft(c, w, +1);
    for (size_t j = 0; j < n; j++) {
        const std::complex<double> z = w[c->slot_index[j]] / scale;
        re[j] = z.real();
        if (im) im[j] = z.imag();
    }
    return CKKS_OK;
}

// ---------------------------------------------------------------------
// optional per-launch timing with HIP events on the launch stream
// ---------------------------------------------------------------------
namespace {
struct ProfRec {
    std::string name;
    u32 items;
    hipEvent_t e0, e1;
};
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
const char *fwd_names[] = {"ntt_fwd", "ntt_fwd_modup", "ntt_fwd_rescale", "ntt_fwd_moddown",
                           "ntt_fwd_moddown_z", "ntt_fwd_sample", "ntt_fwd_int", "ntt_fwd_relin_rescale",
                           "ntt_fwd_modup", "ntt_fwd_modup", "ntt_fwd_modup", "ntt_fwd_modup",
                           "ntt_fwd_moddown_z", "ntt_fwd_moddown_z", "ntt_fwd_relin_rescale", "ntt_fwd_relin_rescale"};
const char *inv_names[] = {"ntt_inv", "ntt_inv_mul", "ntt_inv_scale", "ntt_inv_decrypt"};
const char *ew_names[] = {"ew_add", "ew_sub", "ew_mul", "ew_mul_const", "ew_add_const", "ew_tensor", "ew_copy",
                          "ew_automorph", "ew_neg", "ew_keygen", "ew_encrypt", "ew_square_s", "ew_hmult_fin",
                          "ew_unused", "ew_hmult_t"};
std::string launch_name(int kind, int op, u32 log_n) {
    char b[64];
    switch (kind) {
        case 0: snprintf(b, sizeof b, "%s/N=2^%u", fwd_names[op], log_n); break;
        case 1: snprintf(b, sizeof b, "%s/N=2^%u", inv_names[op], log_n); break;
        case 2: snprintf(b, sizeof b, "%s/N=2^%u", op >= 0 && op < 15 ? ew_names[op] : "elementwise", log_n); break;
        case 3:
        case 6: snprintf(b, sizeof b, "keyswitch_inner_product/N=2^%u", log_n); break;
        case 5: snprintf(b, sizeof b, "hoisted_rotations/N=2^%u", log_n); break;
        case 7: snprintf(b, sizeof b, "linear_mfma/N=2^%u", log_n); break;
        case 8: snprintf(b, sizeof b, "linear_grouped/N=2^%u", log_n); break;
        default: snprintf(b, sizeof b, "linear/N=2^%u", log_n); break;
    }
    return b;
}
}  // namespace

extern "C" int ckks_profile_enable(int on) {
    g_prof_on = on != 0;
    return CKKS_OK;
}

extern "C" int ckks_profile_collect(ckks_launch_record *out, uint32_t cap, uint32_t *n) {
    if (!n) return fail(CKKS_EINVAL, "profile_collect: null count");
    u32 k = 0;
    for (auto &r : g_prof) {
        if (hipEventSynchronize(r.e1) != hipSuccess) return fail(CKKS_EDEVICE, "profile_collect: event sync");
        float ms = 0;
        hipEventElapsedTime(&ms, r.e0, r.e1);
        if (out && k < cap) {
            memset(&out[k], 0, sizeof out[k]);
            snprintf(out[k].name, sizeof out[k].name, "%s", r.name.c_str());
            out[k].items = r.items;
            out[k].ms = ms;
        }
        k++;
        hipEventDestroy(r.e0);
        hipEventDestroy(r.e1);
    }
    g_prof.clear();
    *n = k;
    return CKKS_OK;
}

// ---------------------------------------------------------------------
// planning: scratch carving + work-item tables
// ---------------------------------------------------------------------
namespace {
struct Launch {
    int kind;  // 0 fwd, 1 inv, 2 ew, 3 ip, 5 hoisted rotations, 6 ip (sequential ciphertexts)
    int op;
    size_t off;
    int n;
    u64 seed;
    int fp = 0;  // NTT launches: every item's prime is below 2^50 and takes the FP64 engine
};
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Host-to-device copy of launch data (descriptors, pointer tables, weight
// images). While recording, the bytes go to the recording arena, where they
// stay for replays, and *where receives that address instead of dst.
// Calls that must not allocate (ckks_hmult_relin_rescale_noalloc) set this
// flag for their duration on the calling thread: uploads then skip the
// pinned staging ring (created on first use) and its events and copy
// straight from the host descriptor buffer, and no profiling events are made.
static thread_local bool g_no_alloc = false;
}  // namespace
namespace ckks {
void set_no_alloc(bool on) { g_no_alloc = on; }
}  // namespace ckks
namespace {

int upload(const ckks_ctx *c, uint8_t *dst, const void *src, size_t bytes, hipStream_t s, uint8_t **where) {
    if (c->rec) {
        Recorder &r = *c->rec;
        const size_t off = al256(r.used);
        if (off + bytes > r.cap) return fail(CKKS_ENOMEM, "record: arena of %zu bytes is too small", r.cap);
        dst = r.arena + off;
        r.used = off + bytes;
    }
    *where = dst;
    if (!bytes) return CKKS_OK;
    if (g_no_alloc) {
        // pageable copy (synchronous with respect to the host)
        HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
        return CKKS_OK;
    }
    // The staging ring is mutable state of a context that is otherwise
    // read-only after upload: calls from several host threads on one
    // context serialise here (the copies stay asynchronous).
    ckks_ctx *cm = const_cast<ckks_ctx *>(c);
    std::lock_guard<std::mutex> lock(cm->stage_mu);
    if (!cm->stage) {
        Staging *st = new Staging();
        if (hipHostMalloc((void **)&st->buf, kStagingBytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            st->buf = nullptr;
        } else {
            st->cap = kStagingBytes;
        }
        cm->stage = st;
    }
    Staging &st = *cm->stage;
    if (!st.buf || bytes > st.cap / 2) {
        // pageable copy (synchronous with respect to the host)
        HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
        return CKKS_OK;
    }
    size_t lo = al256(st.head);
    if (lo + bytes > st.cap) lo = 0;
    const size_t hi = lo + bytes;
    // wait for the in-flight regions this one overlaps (oldest first)
    while (!st.inflight.empty()) {
        const Staging::Region &r = st.inflight.front();
        const bool overlap = r.lo < hi && lo < r.hi;
        if (!overlap && hipEventQuery(r.done) != hipSuccess) break;
        HIP_TRY(hipEventSynchronize(r.done));
        HIP_TRY(hipEventDestroy(r.done));
        st.inflight.pop_front();
    }
    for (const Staging::Region &r : st.inflight)
        if (r.lo < hi && lo < r.hi) {  // an older region further back still overlaps
            HIP_TRY(hipEventSynchronize(r.done));
        }
    memcpy(st.buf + lo, src, bytes);
    HIP_TRY(hipMemcpyAsync(dst, st.buf + lo, bytes, hipMemcpyHostToDevice, s));
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ev, s));
    st.inflight.push_back({lo, hi, ev});
    st.head = hi;
    return CKKS_OK;
}
// Run a launch now and, while recording, keep it for replays.
hipError_t issue(const ckks_ctx *c, hipStream_t s, LaunchFn f) {
    const hipError_t e = f(s);
    if (e == hipSuccess && c->rec) c->rec->launches.push_back(std::move(f));
    return e;
}

// Descriptor buffers are recycled per host thread: a large batch's tables
// (megabytes) are then written into memory that is already mapped instead
// of freshly faulted-in pages on every call.
static std::vector<uint8_t> &desc_pool() {
    thread_local std::vector<uint8_t> pool;
    return pool;
}
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
                    // below 2^15 (the generic ModUp kernel) sources of 2^50 or more
                    // are converted too; at 2^15 every source must be below 2^50
                    if (modup && c->log_n >= 15) {
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
                    case 5: return launch_hoist(tb, (const HoItem *)p, L.n, st);
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

// ModUp items (sources pre-multiplied by hat_i^-1), one launch per digit
// size: sizes 1..4 use the kernels with the size fixed at compile time
void add_modup(Plan &P, const std::vector<Item> &v) {
    std::vector<Item> by[5];
    size_t cnt[5] = {0, 0, 0, 0, 0};
    for (const Item &it : v) cnt[it.b <= 4 ? it.b : 0]++;
    for (int i = 0; i < 5; i++) by[i].reserve(cnt[i]);
    for (const Item &it : v) by[it.b <= 4 ? it.b : 0].push_back(it);
    for (u32 sz = 1; sz <= 4; sz++) P.add(0, F_MODUP_S1 + (int)sz - 1, by[sz]);
    P.add(0, F_MODUP, by[0]);
}
// ModDown + rescale kernel for the context's special-prime count
int relin_op(const ckks_ctx *c, bool rescale) {
    const int base = rescale ? F_RELIN_RS_P1 : F_RELIN_P1;
    if (c->n_p <= 2) return base + (int)c->n_p - 1;
    return rescale ? F_RELIN_RS : F_RELIN;
}

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
static bool ip_before(const IpCt &x, const IpCt &y) {
    return x.level != y.level ? x.level < y.level : (uintptr_t)x.key < (uintptr_t)y.key;
}
static bool ip_same(const IpCt &x, const IpCt &y) { return x.level == y.level && x.key == y.key; }
void add_ip_items(const ckks_ctx *c, std::vector<IpItem> &v, const std::vector<IpCt> &cts) {
    std::vector<size_t> order(cts.size());
    for (size_t i = 0; i < order.size(); i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return ip_before(cts[x], cts[y]); });
    struct Grp {
        size_t g, h;
        u32 L, E, beta;
        const u64 *key;
    };
    std::vector<Grp> groups;
    const size_t group = c->tb.ip_cts == 2 ? 2 : (size_t)kIpCts;  // 16 -> 4 for the deep-digit rest
    for (size_t g = 0; g < order.size();) {
        size_t h = g;
        while (h < order.size() && ip_same(cts[order[h]], cts[order[g]]) && h - g < group) h++;
        const u32 L = cts[order[g]].level + 1;
        groups.push_back({g, h, L, L + c->n_p, (L + c->alpha - 1) / c->alpha, cts[order[g]].key});
        g = h;
    }
    for (u32 p = 0; p < c->n_prim; p++) {
        for (const Grp &G : groups) {
            if (p < c->n_q && p >= G.L) continue;  // data prime above this group's level
            const u32 t = p < c->n_q ? p : G.L + (p - c->n_q);
            IpItem it;
            memset(&it, 0, sizeof it);
            it.n_ct = (u32)(G.h - G.g);
            it.prime = p;
            it.beta = G.beta;
            it.own_digit = t < G.L ? t / c->alpha : 0xFFFFFFFFu;
            it.E = G.E;
            it.pos = t;
            it.key = G.key;
            for (size_t k = G.g; k < G.h; k++) {
                const IpCt &x = cts[order[k]];
                it.ext[k - G.g] = x.ext;
                it.acc[k - G.g] = x.acc;
                it.own0[k - G.g] = t < G.L ? x.own0[t] : nullptr;
                it.own1[k - G.g] = (t < G.L && !x.own1.empty()) ? x.own1[t] : nullptr;
                it.own2[k - G.g] = (t < G.L && !x.own2.empty()) ? x.own2[t] : nullptr;
                it.own3[k - G.g] = (t < G.L && !x.own3.empty()) ? x.own3[t] : nullptr;
            }
            v.push_back(it);
        }
    }
}

// the inner product of a batch: with IP_CTS = 16 and at most kIpSeqBeta
// digits, ciphertexts of one level go 16 at a time through k_ip_seq;
// otherwise groups of 2 or 4 through k_ip
void add_ip(Plan &P, const std::vector<IpCt> &cts) {
    const ckks_ctx *c = P.c;
    std::vector<IpItem> ip;
    std::vector<IpSeqItem> seq;
    if (c->tb.ip_cts == (u32)kIpSeqCts) {
        std::vector<IpCt> rest;
        std::vector<size_t> order(cts.size());
        for (size_t i = 0; i < order.size(); i++) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return ip_before(cts[x], cts[y]); });
        for (size_t g = 0; g < order.size();) {
            size_t h = g;
            while (h < order.size() && ip_same(cts[order[h]], cts[order[g]]) && h - g < (size_t)kIpSeqCts) h++;
            const u32 L = cts[order[g]].level + 1, E = L + c->n_p, beta = (L + c->alpha - 1) / c->alpha;
            if (beta > (u32)kIpSeqBeta) {
                for (size_t k = g; k < h; k++) rest.push_back(cts[order[k]]);
                g = h;
                continue;
            }
            for (u32 t = 0; t < E; t++) {
                IpSeqItem it;
                memset(&it, 0, sizeof it);
                it.n_ct = (u32)(h - g);
                it.prime = t < L ? t : c->n_q + (t - L);
                it.beta = beta;
                it.own_digit = t < L ? t / c->alpha : 0xFFFFFFFFu;
                it.E = E;
                it.pos = t;
                it.key = cts[order[g]].key;
                for (size_t k = g; k < h; k++) {
                    const IpCt &x = cts[order[k]];
                    it.ext[k - g] = x.ext;
                    it.acc[k - g] = x.acc;
                    it.own0[k - g] = t < L ? x.own0[t] : nullptr;
                    it.own1[k - g] = (t < L && !x.own1.empty()) ? x.own1[t] : nullptr;
                    it.own2[k - g] = (t < L && !x.own2.empty()) ? x.own2[t] : nullptr;
                    it.own3[k - g] = (t < L && !x.own3.empty()) ? x.own3[t] : nullptr;
                }
                seq.push_back(it);
            }
            g = h;
        }
        add_ip_items(c, ip, rest);
    } else {
        add_ip_items(c, ip, cts);
    }
    P.add(6, 0, seq);
    P.add(3, 0, ip);
}

// Transform items whose inputs are their own limbs only: launched prime by
// prime, so that the workgroups in flight on one XCD (consecutive items)
// read one prime's twiddle tables from that XCD's L2 (stable: within a
// prime the caller's order is kept).
void order_by_prime(std::vector<Item> &v) {
    std::stable_sort(v.begin(), v.end(), [](const Item &x, const Item &y) { return x.prime < y.prime; });
}

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

int check_ctx(const ckks_ctx *c) {
    if (!c) return fail(CKKS_EINVAL, "null context");
    if (!c->uploaded) return fail(CKKS_EINVAL, "context tables not uploaded (ckks_ctx_upload)");
    return CKKS_OK;
}
// device buffers of ciphertexts and plaintexts: the kernels move residues
// in 16-byte pairs
inline bool bad_ptr(const void *p) { return !p || (((uintptr_t)p) & 15); }
int check_ct(const ckks_ctx *c, const ckks_ct &ct, const char *what) {
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

void plan_keyswitch(Plan &P, const std::vector<KsJob> &jobs) {
    const ckks_ctx *c = P.c;
    const u32 N = c->N, k = c->n_p, A = c->alpha;
    std::vector<Item> icopy, modup, ipP, mdown;
    std::vector<IpCt> ipc;
    for (const KsJob &J : jobs) {
        const u32 L = J.level + 1, E = L + k, beta = (L + A - 1) / A;
        u64 *dcoef = P.limbs(L);
        u64 *ext = P.limbs((size_t)beta * E);
        u64 *acc = P.limbs((size_t)2 * E);
        for (u32 i = 0; i < L; i++) {
            const u32 j = i / A, lo = j * A, sz = std::min(A, L - lo);
            Item it = item0();
            it.in[0] = J.dl[i];
            it.out = dcoef + (size_t)i * N;
            it.prime = i;
            it.b = 2;  // times hat_i^-1 of its digit: the ModUp source
            it.c = j * A + sz - 1;
            it.a = i - lo;
            icopy.push_back(it);
        }
        for (u32 j = 0; j < beta; j++) {
            const u32 lo = j * A, s = std::min(A, L - lo);
            for (u32 t = 0; t < E; t++) {
                if (t >= lo && t < lo + s) continue;
                Item it = item0();
                it.in[0] = dcoef + (size_t)lo * N;
                it.a = lo;
                it.b = s;
                it.c = j;
                it.prime = t < L ? t : c->n_q + (t - L);
                it.out = ext + ((size_t)j * E + t) * N;
                modup.push_back(it);
            }
        }
        {
            IpCt x;
            x.level = J.level;
            x.key = J.key;
            x.ext = ext;
            x.acc = acc;
            x.own0 = J.dl;
            ipc.push_back(x);
        }
        for (u32 cc = 0; cc < 2; cc++)
            for (u32 m = 0; m < k; m++) {
                Item it = item0();
                it.in[0] = acc + ((size_t)cc * E + L + m) * N;
                it.out = (u64 *)it.in[0];
                it.prime = c->n_q + m;
                ipP.push_back(it);
            }
        for (u32 cc = 0; cc < 2; cc++)
            for (u32 i = 0; i < L; i++) {
                Item it = item0();
                it.in[0] = acc + ((size_t)cc * E + L) * N;
                it.a = c->n_q;
                it.b = k;
                it.in[1] = acc + ((size_t)cc * E + i) * N;
                it.in[2] = J.addend[cc] ? J.addend[cc] + (size_t)i * N : nullptr;
                it.prime = i;
                it.out = J.out[cc] + (size_t)i * N;
                mdown.push_back(it);
            }
    }
    P.add(1, I_SCALE, icopy);
    add_modup(P, modup);
    add_ip(P, ipc);
    P.add(1, I_COPY, ipP);
    P.add(0, F_MODDOWN, mdown);
}
}  // namespace

struct ckks_plan {
    const ckks_ctx *c;
    std::vector<LaunchFn> launches;
};

extern "C" int ckks_record_begin(ckks_ctx *c, void *arena, size_t arena_bytes) {
    if (!c || (!arena && arena_bytes)) return fail(CKKS_EINVAL, "record_begin: null argument");
    if (((uintptr_t)arena) & 255) return fail(CKKS_EINVAL, "record_begin: arena not 256-byte aligned");
    if (c->rec) return fail(CKKS_EINVAL, "record_begin: already recording");
    c->rec = new Recorder();
    c->rec->arena = (uint8_t *)arena;
    c->rec->cap = arena_bytes;
    return CKKS_OK;
}
extern "C" int ckks_record_end(ckks_ctx *c, ckks_plan **plan, size_t *arena_used) {
    if (!c || !plan) return fail(CKKS_EINVAL, "record_end: null argument");
    if (!c->rec) return fail(CKKS_EINVAL, "record_end: not recording");
    ckks_plan *p = new ckks_plan();
    p->c = c;
    p->launches = std::move(c->rec->launches);
    if (arena_used) *arena_used = c->rec->used;
    delete c->rec;
    c->rec = nullptr;
    *plan = p;
    return CKKS_OK;
}
extern "C" int ckks_plan_launch(const ckks_plan *p, void *stream) {
    if (!p) return fail(CKKS_EINVAL, "plan_launch: null plan");
    for (const LaunchFn &f : p->launches) {
        const hipError_t e = f((hipStream_t)stream);
        if (e != hipSuccess) return fail(CKKS_EDEVICE, "plan_launch: %s", hipGetErrorString(e));
    }
    return CKKS_OK;
}
extern "C" uint32_t ckks_plan_launch_count(const ckks_plan *p) { return p ? (uint32_t)p->launches.size() : 0; }
extern "C" void ckks_plan_destroy(ckks_plan *p) { delete p; }

namespace ckks {
// upload for the graph runtime (same recording rules as the entry points)
int ctx_upload_bytes(const ckks_ctx *c, void *dst, const void *src, size_t bytes, void *stream, void **where) {
    uint8_t *w = nullptr;
    CK(upload(c, (uint8_t *)dst, src, bytes, (hipStream_t)stream, &w));
    *where = w;
    return CKKS_OK;
}
}  // namespace ckks

// ---------------------------------------------------------------------
// serialisation
// ---------------------------------------------------------------------
namespace {
struct SerHeader {
    uint32_t magic, version, kind, log_n, n_q, n_p, dnum, n_poly, level, key_kind;
    double scale;
    uint64_t chain, payload;
};
static_assert(sizeof(SerHeader) == 64, "serial header is 64 bytes");
constexpr uint32_t kSerMagic = 0x534B4B43u;  // "CKKS"

uint64_t chain_hash(const ckks_ctx *c) {
    uint64_t h = 1469598103934665603ull;
    for (u64 q : c->primes)
        for (int b = 0; b < 8; b++) h = (h ^ ((q >> (8 * b)) & 0xFF)) * 1099511628211ull;
    return h;
}
// shape of a serialisable object: base pointer, polys, limbs per poly, limb stride
int ser_shape(const ckks_ctx *c, int obj_kind, const void *obj, int key_kind, SerHeader &h, u64 **base,
              u32 *stride) {
    memset(&h, 0, sizeof h);
    h.magic = kSerMagic;
    h.version = 1;
    h.kind = (u32)obj_kind;
    h.log_n = c->log_n;
    h.n_q = c->n_q;
    h.n_p = c->n_p;
    h.dnum = c->dnum;
    h.chain = chain_hash(c);
    h.key_kind = (u32)key_kind;
    if (!obj) return fail(CKKS_EINVAL, "serialize: null object");
    switch (obj_kind) {
        case CKKS_OBJ_CT: {
            const ckks_ct *x = (const ckks_ct *)obj;
            CK(check_ct(c, *x, "serialize"));
            h.n_poly = x->n_poly;
            h.level = x->level;
            h.scale = x->scale;
            *base = x->data;
            *stride = x->limb_stride;
            break;
        }
        case CKKS_OBJ_PT: {
            const ckks_pt *x = (const ckks_pt *)obj;
            if (!x->data || x->level >= c->n_q) return fail(CKKS_EINVAL, "serialize: bad plaintext");
            h.n_poly = 1;
            h.level = x->level;
            h.scale = x->scale;
            *base = x->data;
            *stride = x->level + 1;
            break;
        }
        case CKKS_OBJ_KEY: {
            *base = (u64 *)obj;
            switch (key_kind) {
                case CKKS_KEY_SECRET: h.n_poly = 1, h.level = c->n_prim - 1; break;
                case CKKS_KEY_PUBLIC: h.n_poly = 2, h.level = c->n_q - 1; break;
                case CKKS_KEY_SWITCH: h.n_poly = 2 * c->digits_top, h.level = c->n_prim - 1; break;
                default: return fail(CKKS_EINVAL, "serialize: unknown key kind %d", key_kind);
            }
            *stride = h.level + 1;
            break;
        }
        default: return fail(CKKS_EINVAL, "serialize: unknown object kind %d", obj_kind);
    }
    h.payload = (u64)h.n_poly * (h.level + 1) * c->N * 8;
    return CKKS_OK;
}
}  // namespace

extern "C" int ckks_serialize(const ckks_ctx *c, int obj_kind, const void *obj, int key_kind, void *host_bytes,
                              size_t *n, void *stream) {
    if (!c || !n) return fail(CKKS_EINVAL, "serialize: null argument");
    SerHeader h;
    u64 *base = nullptr;
    u32 stride = 0;
    CK(ser_shape(c, obj_kind, obj, key_kind, h, &base, &stride));
    const size_t need = sizeof h + h.payload;
    if (!host_bytes) {
        *n = need;
        return CKKS_OK;
    }
    if (*n < need) {
        *n = need;
        return fail(CKKS_ENOMEM, "serialize: buffer of %zu bytes, need %zu", *n, need);
    }
    if (c->rec) return fail(CKKS_EINVAL, "serialize: not allowed while recording");
    uint8_t *out = (uint8_t *)host_bytes;
    memcpy(out, &h, sizeof h);
    const size_t poly = (size_t)(h.level + 1) * c->N * 8;
    hipStream_t s = (hipStream_t)stream;
    for (u32 t = 0; t < h.n_poly; t++)
        HIP_TRY(hipMemcpyAsync(out + sizeof h + t * poly, base + (size_t)t * stride * c->N, poly,
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n = need;
    return CKKS_OK;
}

extern "C" int ckks_deserialize(const ckks_ctx *c, int obj_kind, const void *host_bytes, size_t n, void *obj,
                                int key_kind, void *stream) {
    if (!c || !host_bytes || !obj) return fail(CKKS_EINVAL, "deserialize: null argument");
    if (c->rec) return fail(CKKS_EINVAL, "deserialize: not allowed while recording");
    if (n < sizeof(SerHeader)) return fail(CKKS_EINVAL, "deserialize: %zu bytes is shorter than the header", n);
    SerHeader h;
    memcpy(&h, host_bytes, sizeof h);
    if (h.magic != kSerMagic || h.version != 1) return fail(CKKS_EINVAL, "deserialize: not a serialised object");
    if (h.kind != (u32)obj_kind) return fail(CKKS_EINVAL, "deserialize: object kind %u, expected %d", h.kind, obj_kind);
    if (h.log_n != c->log_n || h.n_q != c->n_q || h.n_p != c->n_p || h.dnum != c->dnum || h.chain != chain_hash(c))
        return fail(CKKS_EPARAMS, "deserialize: parameters differ from the context");
    if (h.level >= c->n_prim || h.n_poly == 0 || h.payload != (u64)h.n_poly * (h.level + 1) * c->N * 8 ||
        n < sizeof h + h.payload)
        return fail(CKKS_EINVAL, "deserialize: inconsistent header or truncated bytes");
    u64 *base = nullptr;
    u32 stride = h.level + 1;
    switch (obj_kind) {
        case CKKS_OBJ_CT: {
            ckks_ct *x = (ckks_ct *)obj;
            if (!x->data || h.level >= c->n_q || h.n_poly < 2 || h.n_poly > 3)
                return fail(CKKS_EINVAL, "deserialize: bad ciphertext");
            if (x->limb_stride < h.level + 1) return fail(CKKS_EINVAL, "deserialize: limb_stride too small");
            base = x->data;
            stride = x->limb_stride;
            x->n_poly = h.n_poly;
            x->level = h.level;
            x->scale = h.scale;
            break;
        }
        case CKKS_OBJ_PT: {
            ckks_pt *x = (ckks_pt *)obj;
            if (!x->data || h.level >= c->n_q || h.n_poly != 1) return fail(CKKS_EINVAL, "deserialize: bad plaintext");
            base = x->data;
            x->level = h.level;
            x->scale = h.scale;
            break;
        }
        case CKKS_OBJ_KEY: {
            SerHeader want;
            u64 *dummy = nullptr;
            u32 st = 0;
            CK(ser_shape(c, CKKS_OBJ_KEY, obj, key_kind, want, &dummy, &st));
            if (h.key_kind != (u32)key_kind || h.n_poly != want.n_poly || h.level != want.level)
                return fail(CKKS_EINVAL, "deserialize: key kind or shape differs");
            base = (u64 *)obj;
            break;
        }
        default: return fail(CKKS_EINVAL, "deserialize: unknown object kind %d", obj_kind);
    }
    const uint8_t *in = (const uint8_t *)host_bytes + sizeof h;
    const size_t poly = (size_t)(h.level + 1) * c->N * 8;
    hipStream_t s = (hipStream_t)stream;
    for (u32 t = 0; t < h.n_poly; t++)
        HIP_TRY(hipMemcpyAsync(base + (size_t)t * stride * c->N, in + t * poly, poly, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return CKKS_OK;
}



// ---------------------------------------------------------------------
// workspace sizing: run the planner on placeholder objects
// ---------------------------------------------------------------------
static int plan_hmult(Plan &P, const u64 *const *rk, const ckks_ct *a, const ckks_ct *b, ckks_ct *out, u32 B);

extern "C" size_t ckks_workspace_bytes(const ckks_ctx *c, int op, uint32_t B, const uint32_t *levels) {
    if (!c) return 0;
    const size_t limb = (size_t)c->N * 8;
    const size_t desc_pad = 4096;
    auto lev = [&](u32 b) { return levels ? levels[b] : c->n_q - 1; };
    size_t items = 0, scratch = 0;
    switch (op) {
        case CKKS_OP_NTT: return (size_t)B * sizeof(Item) + desc_pad;
        case CKKS_OP_ELEMENTWISE: {
            for (u32 b = 0; b < B; b++) items += 3 * (lev(b) + 1);
            return items * sizeof(EwItem) + desc_pad;
        }
        case CKKS_OP_RESCALE: {
            for (u32 b = 0; b < B; b++) items += 3 * (lev(b) + 1), scratch += 3 * limb + 768;
            return scratch + items * sizeof(Item) + 2 * desc_pad;
        }
        case CKKS_OP_KEYSWITCH:
        case CKKS_OP_HMULT: {
            std::vector<ckks_ct> x(B);
            for (u32 b = 0; b < B; b++) {
                x[b] = ckks_ct{(u64 *)(uintptr_t)0x100000, 2, lev(b), lev(b) + 1, 0, 1.0};
            }
            Plan P(c, nullptr);
            // every item with its own key: the most inner-product items
            std::vector<const u64 *> keys(B);
            for (u32 b = 0; b < B; b++) keys[b] = (const u64 *)(uintptr_t)(0x100000 + 256 * (size_t)b);
            if (op == CKKS_OP_HMULT) {
                std::vector<ckks_ct> o = x;
                plan_hmult(P, keys.data(), x.data(), x.data(), o.data(), B);
            } else {
                std::vector<KsJob> jobs(B);
                for (u32 b = 0; b < B; b++) {
                    jobs[b].level = lev(b);
                    jobs[b].key = keys[b];
                    jobs[b].dl.assign(lev(b) + 1, (const u64 *)(uintptr_t)0x100000);
                    jobs[b].addend[0] = jobs[b].addend[1] = nullptr;
                    jobs[b].out[0] = jobs[b].out[1] = (u64 *)(uintptr_t)0x100000;
                    P.limbs(2 * (lev(b) + 1));  // rotate: automorphism staging
                }
                plan_keyswitch(P, jobs);
                std::vector<EwItem> ew(B * 2 * (c->n_q));
                P.add(2, 0, ew);
            }
            return P.total() + 2 * desc_pad;
        }
        case CKKS_OP_KEYGEN: {
            // switching key: digits x n_prim error limbs + n_prim staging for s'
            scratch = ((size_t)c->digits_top * c->n_prim + c->n_prim) * (limb + 256);
            items = (size_t)c->digits_top * c->n_prim * 2 + c->n_prim;
            return scratch + items * (sizeof(Item) + sizeof(EwItem)) + 2 * desc_pad;
        }
        case CKKS_OP_ENCRYPT: {
            u32 L = lev(0) + 1;
            return 3 * (size_t)L * (limb + 256) + 4 * L * (sizeof(Item) + sizeof(EwItem)) + 2 * desc_pad;
        }
        case CKKS_OP_LINEAR: {
            const u32 n_out = B, L = levels ? levels[0] + 1 : c->n_q, n_in = levels ? levels[1] : 1;
            return (size_t)L * n_out * n_in * 8 + (size_t)(n_in + n_out) * 8 + 3 * desc_pad;
        }
    }
    return 0;
}

// ---------------------------------------------------------------------
// NTT primitives
// ---------------------------------------------------------------------
static int ntt_common(const ckks_ctx *c, uint64_t *const *limbs, const uint32_t *pidx, uint32_t n, void *ws,
                      size_t ws_bytes, void *stream, bool inverse) {
    CK(check_ctx(c));
    if ((!limbs || !pidx) && n) return fail(CKKS_EINVAL, "ntt: null argument");
    Plan P(c, ws);
    std::vector<Item> v;
    for (u32 i = 0; i < n; i++) {
        if (pidx[i] >= c->n_prim) return fail(CKKS_EINVAL, "ntt: prime index %u out of range", pidx[i]);
        if (!limbs[i]) return fail(CKKS_EINVAL, "ntt: null limb");
        Item it = item0();
        it.in[0] = limbs[i];
        it.out = limbs[i];
        it.prime = pidx[i];
        v.push_back(it);
    }
    order_by_prime(v);
    if (inverse)
        P.add(1, I_COPY, v);
    else
        P.add(0, F_COPY, v);
    return P.run(ws_bytes, (hipStream_t)stream);
}
extern "C" int ckks_ntt(const ckks_ctx *c, uint64_t *const *limbs, const uint32_t *pidx, uint32_t n, void *ws,
                        size_t ws_bytes, void *stream) {
    return ntt_common(c, limbs, pidx, n, ws, ws_bytes, stream, false);
}
extern "C" int ckks_intt(const ckks_ctx *c, uint64_t *const *limbs, const uint32_t *pidx, uint32_t n, void *ws,
                         size_t ws_bytes, void *stream) {
    return ntt_common(c, limbs, pidx, n, ws, ws_bytes, stream, true);
}

// ---------------------------------------------------------------------
// client side
// ---------------------------------------------------------------------
static void add_sample(std::vector<Item> &v, u64 *out, u32 prime, u32 kind, u32 obj, u32 tag) {
    Item it = item0();
    it.out = out;
    it.prime = prime;
    it.a = kind;
    it.b = obj;
    it.c = tag;
    v.push_back(it);
}

extern "C" int ckks_keygen_secret(const ckks_ctx *c, uint64_t seed, uint64_t *sk, void *ws, size_t ws_bytes,
                                  void *stream) {
    CK(check_ctx(c));
    if (!sk) return fail(CKKS_EINVAL, "keygen_secret: null key");
    Plan P(c, ws);
    std::vector<Item> v;
    for (u32 i = 0; i < c->n_prim; i++) add_sample(v, sk + (size_t)i * c->N, i, S_TERNARY, 0, TAG_SK);
    P.add(0, F_SAMPLE, v, seed);
    return P.run(ws_bytes, (hipStream_t)stream);
}

extern "C" int ckks_keygen_public(const ckks_ctx *c, const uint64_t *sk, uint64_t seed, uint64_t *pk, void *ws,
                                  size_t ws_bytes, void *stream) {
    CK(check_ctx(c));
    if (!sk || !pk) return fail(CKKS_EINVAL, "keygen_public: null argument");
    Plan P(c, ws);
    const u32 N = c->N;
    u64 *eh = P.limbs(c->n_q);
    std::vector<Item> smp;
    std::vector<EwItem> ew;
    for (u32 i = 0; i < c->n_q; i++) {
        add_sample(smp, eh + (size_t)i * N, i, S_CBD, 0, TAG_PK_E);
        EwItem e = ew0();
        e.op = EW_KEYGEN;
        e.prime = i;
        e.x[0] = eh + (size_t)i * N;
        e.x[1] = sk + (size_t)i * N;
        e.x[2] = nullptr;
        e.y[0] = pk + (size_t)i * N;
        e.y[1] = pk + ((size_t)c->n_q + i) * N;
        e.v = (i64)(((u64)TAG_PK_A << 32) | 0u);
        ew.push_back(e);
    }
    P.add(0, F_SAMPLE, smp, seed);
    P.add(2, 0, ew, seed);
    return P.run(ws_bytes, (hipStream_t)stream);
}

// switching key from s' (NTT form over all primes, device) to s
static int keygen_switch(const ckks_ctx *c, Plan &P, const u64 *sk, const u64 *sprime, u64 seed, u32 key_id,
                         u64 *key) {
    const u32 N = c->N, np = c->n_prim, A = c->alpha;
    u64 *eh = P.limbs((size_t)c->digits_top * np);
    std::vector<Item> smp;
    std::vector<EwItem> ew;
    for (u32 j = 0; j < c->digits_top; j++) {
        const u32 obj = (key_id << 8) | j, lo = j * A, hi = std::min(lo + A, c->n_q);
        for (u32 i = 0; i < np; i++) {
            u64 *e = eh + ((size_t)j * np + i) * N;
            add_sample(smp, e, i, S_CBD, obj, TAG_SWK_E);
            EwItem w = ew0();
            w.op = EW_KEYGEN;
            w.prime = i;
            w.x[0] = e;
            w.x[1] = sk + (size_t)i * N;
            w.x[2] = (i >= lo && i < hi) ? sprime + (size_t)i * N : nullptr;
            w.y[0] = key + (((size_t)j * 2 + 0) * np + i) * N;
            w.y[1] = key + (((size_t)j * 2 + 1) * np + i) * N;
            w.v = (i64)(((u64)TAG_SWK_A << 32) | obj);
            ew.push_back(w);
        }
    }
    P.add(0, F_SAMPLE, smp, seed);
    P.add(2, 0, ew, seed);
    return CKKS_OK;
}

extern "C" int ckks_keygen_relin(const ckks_ctx *c, const uint64_t *sk, uint64_t seed, uint64_t *rk, void *ws,
                                 size_t ws_bytes, void *stream) {
    CK(check_ctx(c));
    if (!sk || !rk) return fail(CKKS_EINVAL, "keygen_relin: null argument");
    Plan P(c, ws);
    u64 *s2 = P.limbs(c->n_prim);
    std::vector<EwItem> sq;
    for (u32 i = 0; i < c->n_prim; i++) {
        EwItem w = ew0();
        w.op = EW_SQUARE_S;
        w.prime = i;
        w.x[0] = sk + (size_t)i * c->N;
        w.y[0] = s2 + (size_t)i * c->N;
        sq.push_back(w);
    }
    P.add(2, 0, sq);
    CK(keygen_switch(c, P, sk, s2, seed, 0, rk));
    return P.run(ws_bytes, (hipStream_t)stream);
}

extern "C" int ckks_keygen_galois(const ckks_ctx *c, const uint64_t *sk, uint32_t g, uint64_t seed, uint64_t *gk,
                                  void *ws, size_t ws_bytes, void *stream) {
    CK(check_ctx(c));
    if (!sk || !gk) return fail(CKKS_EINVAL, "keygen_galois: null argument");
    if (!(g & 1) || g >= 2 * c->N) return fail(CKKS_EINVAL, "keygen_galois: element %u not odd / < 2N", g);
    if (g >= (1u << 24)) return fail(CKKS_EINVAL, "keygen_galois: element too large for the object id");
    Plan P(c, ws);
    u64 *sg = P.limbs(c->n_prim);
    std::vector<EwItem> am;
    for (u32 i = 0; i < c->n_prim; i++) {
        EwItem w = ew0();
        w.op = EW_AUTOMORPH;
        w.prime = i;
        w.v = g;
        w.x[0] = sk + (size_t)i * c->N;
        w.y[0] = sg + (size_t)i * c->N;
        am.push_back(w);
    }
    P.add(2, 0, am);
    CK(keygen_switch(c, P, sk, sg, seed, g, gk));
    return P.run(ws_bytes, (hipStream_t)stream);
}

extern "C" int ckks_pt_load(const ckks_ctx *c, const int64_t *coeffs, ckks_pt *out, void *ws, size_t ws_bytes,
                            void *stream) {
    CK(check_ctx(c));
    if (!coeffs || !out || !out->data) return fail(CKKS_EINVAL, "pt_load: null argument");
    if (out->level >= c->n_q) return fail(CKKS_ELEVEL, "pt_load: level out of range");
    Plan P(c, ws);
    std::vector<Item> v;
    for (u32 i = 0; i <= out->level; i++) {
        Item it = item0();
        it.in[0] = (const u64 *)coeffs;
        it.out = out->data + (size_t)i * c->N;
        it.prime = i;
        v.push_back(it);
    }
    P.add(0, F_INT, v);
    return P.run(ws_bytes, (hipStream_t)stream);
}

extern "C" int ckks_encrypt(const ckks_ctx *c, const uint64_t *pk, const ckks_pt *pt, uint64_t seed, uint32_t obj,
                            ckks_ct *out, void *ws, size_t ws_bytes, void *stream) {
    CK(check_ctx(c));
    if (!pk || !pt || !pt->data || !out || !out->data) return fail(CKKS_EINVAL, "encrypt: null argument");
    if (pt->level >= c->n_q) return fail(CKKS_ELEVEL, "encrypt: level out of range");
    const u32 L = pt->level + 1, N = c->N;
    if (out->limb_stride < L) out->limb_stride = L;
    Plan P(c, ws);
    u64 *vh = P.limbs(L), *e0 = P.limbs(L), *e1 = P.limbs(L);
    std::vector<Item> smp;
    std::vector<EwItem> ew;
    for (u32 i = 0; i < L; i++) {
        add_sample(smp, vh + (size_t)i * N, i, S_TERNARY, obj, TAG_ENC_V);
        add_sample(smp, e0 + (size_t)i * N, i, S_CBD, obj, TAG_ENC_E0);
        add_sample(smp, e1 + (size_t)i * N, i, S_CBD, obj, TAG_ENC_E1);
        EwItem w = ew0();
        w.op = EW_ENCRYPT;
        w.prime = i;
        w.x[0] = vh + (size_t)i * N;
        w.x[1] = e0 + (size_t)i * N;
        w.x[2] = e1 + (size_t)i * N;
        w.x[3] = pk + (size_t)i * N;
        w.x[4] = pk + ((size_t)c->n_q + i) * N;
        w.x[5] = pt->data + (size_t)i * N;
        w.y[0] = out->data + (size_t)i * N;
        w.y[1] = out->data + ((size_t)out->limb_stride + i) * N;
        ew.push_back(w);
    }
    P.add(0, F_SAMPLE, smp, seed);
    P.add(2, 0, ew, seed);
    CK(P.run(ws_bytes, (hipStream_t)stream));
    out->n_poly = 2;
    out->level = pt->level;
    out->scale = pt->scale;
    return CKKS_OK;
}

extern "C" int ckks_decrypt(const ckks_ctx *c, const uint64_t *sk, const ckks_ct *ct, uint64_t *m, void *ws,
                            size_t ws_bytes, void *stream) {
    CK(check_ctx(c));
    if (!sk || !ct || !m) return fail(CKKS_EINVAL, "decrypt: null argument");
    CK(check_ct(c, *ct, "decrypt"));
    Plan P(c, ws);
    std::vector<Item> v;
    for (u32 i = 0; i <= ct->level; i++) {
        Item it = item0();
        it.in[0] = limb(c, *ct, 0, i);
        it.in[1] = limb(c, *ct, 1, i);
        it.in[2] = ct->n_poly == 3 ? limb(c, *ct, 2, i) : nullptr;
        it.in[3] = sk + (size_t)i * c->N;
        it.a = ct->n_poly;
        it.prime = i;
        it.out = m + (size_t)i * c->N;
        v.push_back(it);
    }
    P.add(1, I_DECRYPT, v);
    return P.run(ws_bytes, (hipStream_t)stream);
}

// ---------------------------------------------------------------------
// server side: elementwise ops
// ---------------------------------------------------------------------
static int ew_binary(const ckks_ctx *c, u32 op, const ckks_ct *a, const ckks_ct *b, const ckks_pt *p,
                     const int64_t *v, const double *vs, ckks_ct *out, u32 B, void *ws, size_t ws_bytes,
                     void *stream, const char *name) {
    CK(check_ctx(c));
    if (!a || !out || (B && !out)) return fail(CKKS_EINVAL, "%s: null argument", name);
    Plan P(c, ws);
    std::vector<EwItem> items;
    for (u32 k = 0; k < B; k++) {
        CK(check_ct(c, a[k], name));
        if (bad_ptr(out[k].data)) return fail(CKKS_EINVAL, "%s: null or unaligned output", name);
        const u32 L = a[k].level + 1;
        u32 n_poly_out = a[k].n_poly;
        double scale = a[k].scale;
        if (b) {
            CK(check_ct(c, b[k], name));
            if (b[k].level != a[k].level)
                return fail(CKKS_ELEVEL, "%s: level %u vs %u (mod-switch the higher one first)", name, a[k].level,
                            b[k].level);
            if (op == EW_TENSOR) {
                if (a[k].n_poly != 2 || b[k].n_poly != 2) return fail(CKKS_EINVAL, "%s: inputs must have 2 polys", name);
                n_poly_out = 3;
                scale = a[k].scale * b[k].scale;
            } else {
                if (a[k].scale != b[k].scale)
                    return fail(CKKS_ESCALE, "%s: scales %.17g vs %.17g differ", name, a[k].scale, b[k].scale);
                if (a[k].n_poly != b[k].n_poly) return fail(CKKS_EINVAL, "%s: poly counts differ", name);
            }
        }
        if (p) {
            if (bad_ptr(p[k].data)) return fail(CKKS_EINVAL, "%s: null or unaligned plaintext", name);
            if (p[k].level < a[k].level) return fail(CKKS_ELEVEL, "%s: plaintext level below ciphertext", name);
            if (op == EW_ADD && a[k].scale != p[k].scale)
                return fail(CKKS_ESCALE, "%s: scales %.17g vs %.17g differ", name, a[k].scale, p[k].scale);
            if (op == EW_MUL) scale = a[k].scale * p[k].scale;
        }
        if (op == EW_MUL_CONST) scale = a[k].scale * vs[k];
        ckks_ct o = out[k];
        if (o.limb_stride < L) o.limb_stride = L;
        for (u32 i = 0; i < L; i++) {
            if (op == EW_TENSOR) {
                EwItem w = ew0();
                w.op = EW_TENSOR;
                w.prime = i;
                w.x[0] = limb(c, a[k], 0, i);
                w.x[1] = limb(c, a[k], 1, i);
                w.x[2] = limb(c, b[k], 0, i);
                w.x[3] = limb(c, b[k], 1, i);
                w.y[0] = limb(c, o, 0, i);
                w.y[1] = limb(c, o, 1, i);
                w.y[2] = limb(c, o, 2, i);
                items.push_back(w);
                continue;
            }
            for (u32 t = 0; t < a[k].n_poly; t++) {
                EwItem w = ew0();
                w.prime = i;
                w.x[0] = limb(c, a[k], t, i);
                w.y[0] = limb(c, o, t, i);
                if (b) {
                    w.op = op;
                    w.x[1] = limb(c, b[k], t, i);
                } else if (p) {
                    if (op == EW_ADD && t > 0) {
                        w.op = EW_COPY;
                    } else {
                        w.op = op;
                        w.x[1] = p[k].data + (size_t)i * c->N;
                    }
                } else {
                    if (op == EW_ADD_CONST && t > 0)
                        w.op = EW_COPY;
                    else
                        w.op = op, w.v = v[k];
                }
                if (w.op == EW_COPY && w.x[0] == w.y[0]) continue;
                items.push_back(w);
            }
        }
        out[k].n_poly = n_poly_out;
        out[k].level = a[k].level;
        out[k].limb_stride = o.limb_stride;
        out[k].scale = scale;
    }
    P.add(2, 0, items);
    return P.run(ws_bytes, (hipStream_t)stream);
}

extern "C" int ckks_add(const ckks_ctx *c, const ckks_ct *a, const ckks_ct *b, ckks_ct *out, uint32_t B, void *ws,
                        size_t ws_bytes, void *stream) {
    if (!b) return fail(CKKS_EINVAL, "add: null argument");
    return ew_binary(c, EW_ADD, a, b, nullptr, nullptr, nullptr, out, B, ws, ws_bytes, stream, "add");
}
extern "C" int ckks_sub(const ckks_ctx *c, const ckks_ct *a, const ckks_ct *b, ckks_ct *out, uint32_t B, void *ws,
                        size_t ws_bytes, void *stream) {
    if (!b) return fail(CKKS_EINVAL, "sub: null argument");
    return ew_binary(c, EW_SUB, a, b, nullptr, nullptr, nullptr, out, B, ws, ws_bytes, stream, "sub");
}
extern "C" int ckks_add_plain(const ckks_ctx *c, const ckks_ct *a, const ckks_pt *p, ckks_ct *out, uint32_t B,
                              void *ws, size_t ws_bytes, void *stream) {
    if (!p) return fail(CKKS_EINVAL, "add_plain: null argument");
    return ew_binary(c, EW_ADD, a, nullptr, p, nullptr, nullptr, out, B, ws, ws_bytes, stream, "add_plain");
}
extern "C" int ckks_multiply_plain(const ckks_ctx *c, const ckks_ct *a, const ckks_pt *p, ckks_ct *out,
                                   uint32_t B, void *ws, size_t ws_bytes, void *stream) {
    if (!p) return fail(CKKS_EINVAL, "multiply_plain: null argument");
    return ew_binary(c, EW_MUL, a, nullptr, p, nullptr, nullptr, out, B, ws, ws_bytes, stream, "multiply_plain");
}
extern "C" int ckks_multiply_scalar(const ckks_ctx *c, const ckks_ct *a, const int64_t *v, const double *vs,
                                    ckks_ct *out, uint32_t B, void *ws, size_t ws_bytes, void *stream) {
    if (!v || !vs) return fail(CKKS_EINVAL, "multiply_scalar: null argument");
    return ew_binary(c, EW_MUL_CONST, a, nullptr, nullptr, v, vs, out, B, ws, ws_bytes, stream, "multiply_scalar");
}
extern "C" int ckks_add_scalar(const ckks_ctx *c, const ckks_ct *a, const int64_t *v, ckks_ct *out, uint32_t B,
                               void *ws, size_t ws_bytes, void *stream) {
    if (!v) return fail(CKKS_EINVAL, "add_scalar: null argument");
    return ew_binary(c, EW_ADD_CONST, a, nullptr, nullptr, v, nullptr, out, B, ws, ws_bytes, stream, "add_scalar");
}
extern "C" int ckks_multiply(const ckks_ctx *c, const ckks_ct *a, const ckks_ct *b, ckks_ct *out3, uint32_t B,
                             void *ws, size_t ws_bytes, void *stream) {
    if (!b) return fail(CKKS_EINVAL, "multiply: null argument");
    return ew_binary(c, EW_TENSOR, a, b, nullptr, nullptr, nullptr, out3, B, ws, ws_bytes, stream, "multiply");
}

extern "C" int ckks_mod_switch_to(const ckks_ctx *c, ckks_ct *ct, uint32_t level) {
    if (!c || !ct) return fail(CKKS_EINVAL, "mod_switch_to: null argument");
    if (level > ct->level) return fail(CKKS_ELEVEL, "mod_switch_to: cannot raise level %u to %u", ct->level, level);
    ct->level = level;
    return CKKS_OK;
}

// ---------------------------------------------------------------------
// server side: key switching, rescale, rotation, fused HMult
// ---------------------------------------------------------------------
extern "C" int ckks_relinearize(const ckks_ctx *c, const uint64_t *const *rk, const ckks_ct *in3, ckks_ct *out,
                                uint32_t B, void *ws, size_t ws_bytes, void *stream) {
    CK(check_ctx(c));
    if (!rk || !in3 || !out) return fail(CKKS_EINVAL, "relinearize: null argument");
    Plan P(c, ws);
    std::vector<KsJob> jobs(B);
    for (u32 k = 0; k < B; k++) {
        if (!rk[k]) return fail(CKKS_ENOKEY, "relinearize: null key for item %u", k);
        if (bad_ptr(rk[k])) return fail(CKKS_EINVAL, "relinearize: key of item %u not 16-byte aligned", k);
        CK(check_ct(c, in3[k], "relinearize"));
        if (in3[k].n_poly != 3) return fail(CKKS_EINVAL, "relinearize: input must have 3 polys");
        if (bad_ptr(out[k].data)) return fail(CKKS_EINVAL, "relinearize: null or unaligned output");
        if (out[k].data == in3[k].data) return fail(CKKS_EINVAL, "relinearize: out must not alias in");
        const u32 L = in3[k].level + 1;
        if (out[k].limb_stride < L) out[k].limb_stride = L;
        KsJob &J = jobs[k];
        J.level = in3[k].level;
        J.key = rk[k];
        for (u32 i = 0; i < L; i++) J.dl.push_back(limb(c, in3[k], 2, i));
        for (u32 cc = 0; cc < 2; cc++) {
            J.addend[cc] = limb(c, in3[k], cc, 0);
            J.out[cc] = limb(c, out[k], cc, 0);
        }
    }
    plan_keyswitch(P, jobs);
    CK(P.run(ws_bytes, (hipStream_t)stream));
    for (u32 k = 0; k < B; k++) {
        out[k].n_poly = 2;
        out[k].level = in3[k].level;
        out[k].scale = in3[k].scale;
    }
    return CKKS_OK;
}

extern "C" int ckks_rotate(const ckks_ctx *c, const uint64_t *const *gk, const uint32_t *galois_elts,
                           const ckks_ct *in, ckks_ct *out, uint32_t B, void *ws, size_t ws_bytes, void *stream) {
    CK(check_ctx(c));
    if (!gk || !galois_elts || !in || !out) return fail(CKKS_EINVAL, "rotate: null argument");
    Plan P(c, ws);
    std::vector<EwItem> am;
    std::vector<KsJob> jobs(B);
    for (u32 k = 0; k < B; k++) {
        const u32 g = galois_elts[k];
        if (!(g & 1) || g >= 2 * c->N) return fail(CKKS_EINVAL, "rotate: Galois element %u not odd / < 2N", g);
        if (!gk[k]) return fail(CKKS_ENOKEY, "rotate: null Galois key for item %u", k);
        if (bad_ptr(gk[k])) return fail(CKKS_EINVAL, "rotate: key of item %u not 16-byte aligned", k);
        CK(check_ct(c, in[k], "rotate"));
        if (in[k].n_poly != 2) return fail(CKKS_EINVAL, "rotate: input must have 2 polys");
        if (bad_ptr(out[k].data) || out[k].data == in[k].data)
            return fail(CKKS_EINVAL, "rotate: out null, unaligned or aliasing in");
        const u32 L = in[k].level + 1, N = c->N;
        if (out[k].limb_stride < L) out[k].limb_stride = L;
        u64 *rot = P.limbs(2 * L);
        for (u32 t = 0; t < 2; t++)
            for (u32 i = 0; i < L; i++) {
                EwItem w = ew0();
                w.op = EW_AUTOMORPH;
                w.prime = i;
                w.v = g;
                w.x[0] = limb(c, in[k], t, i);
                w.y[0] = rot + ((size_t)t * L + i) * N;
                am.push_back(w);
            }
        KsJob &J = jobs[k];
        J.level = in[k].level;
        J.key = gk[k];
        for (u32 i = 0; i < L; i++) J.dl.push_back(rot + ((size_t)L + i) * N);
        J.addend[0] = rot;
        J.addend[1] = nullptr;
        J.out[0] = limb(c, out[k], 0, 0);
        J.out[1] = limb(c, out[k], 1, 0);
    }
    P.add(2, 0, am);
    plan_keyswitch(P, jobs);
    CK(P.run(ws_bytes, (hipStream_t)stream));
    for (u32 k = 0; k < B; k++) {
        out[k].n_poly = 2;
        out[k].level = in[k].level;
        out[k].scale = in[k].scale;
    }
    return CKKS_OK;
}

// rescale of a batch; v (or null): per item, a signed constant added to
// every slot of the first polynomial after the division
static int rescale_impl(const ckks_ctx *c, const ckks_ct *in, const int64_t *v, ckks_ct *out, uint32_t B, void *ws,
                        size_t ws_bytes, void *stream) {
    CK(check_ctx(c));
    if (!in || !out) return fail(CKKS_EINVAL, "rescale: null argument");
    Plan P(c, ws);
    std::vector<Item> top, res;
    for (u32 k = 0; k < B; k++) {
        CK(check_ct(c, in[k], "rescale"));
        if (in[k].level == 0) return fail(CKKS_EDEPTH, "rescale: no prime left (level 0)");
        if (bad_ptr(out[k].data)) return fail(CKKS_EINVAL, "rescale: null or unaligned output");
        const u32 l = in[k].level;
        ckks_ct o = out[k];
        if (o.data == in[k].data) o.limb_stride = in[k].limb_stride;
        else if (o.limb_stride < l) o.limb_stride = l;
        u64 *tp = P.limbs(in[k].n_poly);
        for (u32 t = 0; t < in[k].n_poly; t++) {
            Item it = item0();
            it.in[0] = limb(c, in[k], t, l);
            it.out = tp + (size_t)t * c->N;
            it.prime = l;
            top.push_back(it);
            for (u32 i = 0; i < l; i++) {
                Item r = item0();
                r.in[0] = tp + (size_t)t * c->N;
                r.in[1] = limb(c, in[k], t, i);
                r.a = l;
                r.prime = i;
                r.out = limb(c, o, t, i);
                r.v = (v && t == 0) ? v[k] : 0;
                res.push_back(r);
            }
        }
        out[k].limb_stride = o.limb_stride;
    }
    P.add(1, I_COPY, top);
    P.add(0, F_RESCALE, res);
    CK(P.run(ws_bytes, (hipStream_t)stream));
    for (u32 k = 0; k < B; k++) {
        // read everything from in[k] first: out may be the same array
        const u32 n_poly = in[k].n_poly, l = in[k].level;
        const double scale = in[k].scale / (double)c->primes[l];
        out[k].n_poly = n_poly;
        out[k].level = l - 1;
        out[k].scale = scale;
    }
    return CKKS_OK;
}
extern "C" int ckks_rescale(const ckks_ctx *c, const ckks_ct *in, ckks_ct *out, uint32_t B, void *ws,
                            size_t ws_bytes, void *stream) {
    return rescale_impl(c, in, nullptr, out, B, ws, ws_bytes, stream);
}
extern "C" int ckks_rescale_add_scalar(const ckks_ctx *c, const ckks_ct *in, const int64_t *v, ckks_ct *out,
                                       uint32_t B, void *ws, size_t ws_bytes, void *stream) {
    if (!v) return fail(CKKS_EINVAL, "rescale_add_scalar: null constants");
    return rescale_impl(c, in, v, out, B, ws, ws_bytes, stream);
}

// Fused HMult + relinearise + rescale over a ragged batch:
//   1. INTT(a1 b1) per limb, stored pre-multiplied by its digit's hat^-1;
//   2. ModUp of every digit to every other prime, NTT;
//   3. key-switch inner product (the digit's own limbs use a1 b1 directly);
//   4. INTT of the special-prime part of both accumulators;
//   5. top limb: u = acc_l P^-1 + d_c (elementwise), INTT(u);
//   6. per limb i < l: z = conv_i(acc_P) P^-1 + rescale correction of the
//      relinearised top limb u - conv_l(acc_P) P^-1 (elementwise), NTT(z);
//   7. elementwise: out_c = (acc_c P^-1 + d_c - z_c) q_l^-1 for both polys.
// The corrections run in streaming elementwise kernels so that every NTT of
// the pipeline stays a plain register-resident transform.
// By linearity this equals relinearise (ModDown) followed by rescale.
static int plan_hmult(Plan &P, const u64 *const *rk, const ckks_ct *a, const ckks_ct *b, ckks_ct *out, u32 B) {
    const ckks_ctx *c = P.c;
    const u32 N = c->N, k = c->n_p, A = c->alpha;
    const bool fuse = c->tb.fuse_tail != 0;
    std::vector<Item> mul, modup, scale, fin;
    std::vector<EwItem> tt, tail;
    std::vector<IpCt> ipc;
    {
        size_t n_mul = 0, n_modup = 0, n_fin = 0;
        for (u32 x = 0; x < B; x++) {
            const u32 L = a[x].level + 1, E = L + k, beta = (L + A - 1) / A;
            n_mul += L;
            n_modup += (size_t)beta * E - L;
            n_fin += 2 * (size_t)(L - 1);
        }
        mul.reserve(n_mul);
        modup.reserve(n_modup);
        fin.reserve(n_fin);
        scale.reserve((size_t)B * 2 * (k + 1));
        tt.reserve((size_t)B * 2);
        ipc.reserve(B);
        if (!fuse) tail.reserve(n_fin / 2);
    }
    for (u32 x = 0; x < B; x++) {
        const u32 l = a[x].level, L = l + 1, E = L + k, beta = (L + A - 1) / A;
        u64 *dcoef = P.limbs(L);
        u64 *ext = P.limbs((size_t)beta * E);
        u64 *acc = P.limbs((size_t)2 * E);
        u64 *top = P.limbs(2);
        u64 *zh = fuse ? nullptr : P.limbs((size_t)2 * l);
        // d2 = a1 b1 -> INTT -> times hat_i^-1 (the ModUp input of its digit)
        for (u32 i = 0; i < L; i++) {
            const u32 j = i / A, lo = j * A, s = std::min(A, L - lo);
            Item it = item0();
            it.in[0] = limb(c, a[x], 1, i);
            it.in[1] = limb(c, b[x], 1, i);
            it.out = dcoef + (size_t)i * N;
            it.prime = i;
            it.v = 1;
            it.c = j * A + s - 1;
            it.a = i - lo;
            mul.push_back(it);
        }
        // ModUp of every digit to the primes outside it, then NTT
        for (u32 j = 0; j < beta; j++) {
            const u32 lo = j * A, s = std::min(A, L - lo);
            for (u32 t = 0; t < E; t++) {
                if (t >= lo && t < lo + s) continue;
                Item it = item0();
                it.in[0] = dcoef + (size_t)lo * N;
                it.a = lo;
                it.b = s;
                it.c = j;
                it.v = 1;
                it.prime = t < L ? t : c->n_q + (t - L);
                it.out = ext + ((size_t)j * E + t) * N;
                modup.push_back(it);
            }
        }
        // key-switch inner product; data limbs also take P d_0, P d_1
        {
            IpCt y;
            y.level = l;
            y.key = rk[x];
            y.ext = ext;
            y.acc = acc;
            for (u32 t = 0; t < L; t++) {
                y.own0.push_back(limb(c, a[x], 1, t));
                y.own1.push_back(limb(c, b[x], 1, t));
                y.own2.push_back(limb(c, a[x], 0, t));
                y.own3.push_back(limb(c, b[x], 0, t));
            }
            ipc.push_back(y);
        }
        for (u32 cc = 0; cc < 2; cc++) {
            // special-prime part: INTT, times hat_m^-1 (in place)
            for (u32 m = 0; m < k; m++) {
                Item it = item0();
                it.in[0] = acc + ((size_t)cc * E + L + m) * N;
                it.out = (u64 *)it.in[0];
                it.prime = c->n_q + m;
                it.a = m;
                scale.push_back(it);
            }
            // top limb: INTT, times P^-1; then minus conv_l(y) P^-1
            Item it = item0();
            it.in[0] = acc + ((size_t)cc * E + l) * N;
            it.out = top + (size_t)cc * N;
            it.prime = l;
            it.b = 1;
            scale.push_back(it);
            EwItem v = ew0();
            v.op = EW_HMULT_T;
            v.prime = l;
            v.x[0] = top + (size_t)cc * N;
            v.x[1] = acc + ((size_t)cc * E + L) * N;
            v.y[0] = top + (size_t)cc * N;
            tt.push_back(v);
        }
        // remaining limbs: ModDown correction, NTT, rescale
        for (u32 cc = 0; cc < 2; cc++)
            for (u32 i = 0; i < l; i++) {
                Item it = item0();
                it.in[0] = acc + ((size_t)cc * E + L) * N;
                it.in[1] = top + (size_t)cc * N;
                it.in[2] = acc + ((size_t)cc * E + i) * N;
                it.out = fuse ? limb(c, out[x], cc, i) : zh + ((size_t)cc * l + i) * N;
                it.prime = i;
                it.a = l;
                fin.push_back(it);
            }
        if (!fuse)
            for (u32 i = 0; i < l; i++) {
                EwItem w = ew0();
                w.op = EW_HMULT_FIN;
                w.prime = i;
                w.v = l;
                w.x[0] = zh + (size_t)i * N;
                w.x[1] = zh + ((size_t)l + i) * N;
                w.x[2] = acc + (size_t)i * N;
                w.x[3] = acc + ((size_t)E + i) * N;
                w.y[0] = limb(c, out[x], 0, i);
                w.y[1] = limb(c, out[x], 1, i);
                tail.push_back(w);
            }
    }
    order_by_prime(mul);
    P.add(1, I_MUL, mul);
    add_modup(P, modup);
    add_ip(P, ipc);
    P.add(1, I_SCALE, scale);
    P.add(2, 0, tt);
    P.add(0, relin_op(c, fuse), fin);
    if (!fuse) P.add(2, 0, tail);
    return CKKS_OK;
}

extern "C" int ckks_hmult_relin_rescale(const ckks_ctx *c, const uint64_t *const *rk, const ckks_ct *a,
                                        const ckks_ct *b, ckks_ct *out, uint32_t B, void *ws, size_t ws_bytes,
                                        void *stream) {
    CK(check_ctx(c));
    if (!rk || !a || !b || !out) return fail(CKKS_EINVAL, "hmult: null argument");
    for (u32 x = 0; x < B; x++) {
        if (!rk[x]) return fail(CKKS_ENOKEY, "hmult: null relinearisation key for item %u", x);
        if (bad_ptr(rk[x])) return fail(CKKS_EINVAL, "hmult: key of item %u not 16-byte aligned", x);
        CK(check_ct(c, a[x], "hmult a"));
        CK(check_ct(c, b[x], "hmult b"));
        if (a[x].n_poly != 2 || b[x].n_poly != 2) return fail(CKKS_EINVAL, "hmult: inputs must have 2 polys");
        if (a[x].level != b[x].level) return fail(CKKS_ELEVEL, "hmult: levels %u vs %u", a[x].level, b[x].level);
        if (a[x].level == 0) return fail(CKKS_EDEPTH, "hmult: no prime left to rescale");
        if (bad_ptr(out[x].data)) return fail(CKKS_EINVAL, "hmult: null or unaligned output");
        if (out[x].data == a[x].data || out[x].data == b[x].data)
            return fail(CKKS_EINVAL, "hmult: out must not alias an input");
        if (out[x].limb_stride < a[x].level) out[x].limb_stride = a[x].level;
    }
    Plan P(c, ws);
    CK(plan_hmult(P, rk, a, b, out, B));
    CK(P.run(ws_bytes, (hipStream_t)stream));
    for (u32 x = 0; x < B; x++) {
        out[x].n_poly = 2;
        out[x].level = a[x].level - 1;
        out[x].scale = a[x].scale * b[x].scale / (double)c->primes[a[x].level];
    }
    return CKKS_OK;
}

// ---------------------------------------------------------------------
// hoisted rotations with plaintext weights
// ---------------------------------------------------------------------
extern "C" size_t ckks_hoisted_linear_workspace_bytes(const ckks_ctx *c, uint32_t B, uint32_t level,
                                                      uint32_t n_rot) {
    if (!c) return 0;
    const size_t L = level + 1, E = L + c->n_p, beta = (L + c->alpha - 1) / c->alpha;
    const size_t limb = ((size_t)c->N * 8 + 255) & ~(size_t)255;
    const size_t per_ct = (L + beta * E + 2 * E) * limb;
    const size_t items = B * (L + beta * E + 2 * (c->n_p + L)) * sizeof(Item) +
                         E * ((B + kHoCts - 1) / kHoCts) * sizeof(HoItem) + (size_t)n_rot * E * sizeof(Item);
    return B * per_ct + ((size_t)n_rot * E + 1) * limb + items + 16 * 4096;
}

extern "C" int ckks_hoisted_linear(const ckks_ctx *c, const ckks_ct *in, ckks_ct *out, uint32_t B, uint32_t n_rot,
                                   const uint32_t *galois_elts, const uint64_t *const *galois_keys,
                                   const int64_t *pt_coeffs, double pt_scale, void *ws, size_t ws_bytes,
                                   void *stream) {
    CK(check_ctx(c));
    if (!in || !out || !galois_elts || !pt_coeffs || !B || !n_rot) return fail(CKKS_EINVAL, "hoisted: bad argument");
    const u32 l = in[0].level, L = l + 1, N = c->N, k = c->n_p, A = c->alpha, E = L + k, beta = (L + A - 1) / A;
    for (u32 x = 0; x < B; x++) {
        CK(check_ct(c, in[x], "hoisted"));
        if (in[x].n_poly != 2) return fail(CKKS_EINVAL, "hoisted: inputs must have 2 polys");
        if (in[x].level != l) return fail(CKKS_ELEVEL, "hoisted: input levels differ");
        if (bad_ptr(out[x].data)) return fail(CKKS_EINVAL, "hoisted: null or unaligned output");
        if (out[x].data == in[x].data) return fail(CKKS_EINVAL, "hoisted: out must not alias the input");
        if (out[x].limb_stride < L) out[x].limb_stride = L;
    }
    for (u32 i = 0; i < n_rot; i++) {
        const u32 g = galois_elts[i];
        if (!(g & 1) || g >= 2 * N) return fail(CKKS_EINVAL, "hoisted: bad Galois element %u", g);
        if (g != 1 && (!galois_keys || !galois_keys[i])) return fail(CKKS_ENOKEY, "hoisted: no key for element %u", g);
        if (g != 1 && bad_ptr(galois_keys[i])) return fail(CKKS_EINVAL, "hoisted: key for element %u not 16-byte aligned", g);
    }
    if ((size_t)n_rot * 12 > (size_t)N * 8) return fail(CKKS_EINVAL, "hoisted: too many rotations");
    const size_t need = ckks_hoisted_linear_workspace_bytes(c, B, l, n_rot);
    if (!ws || ws_bytes < need) return fail(CKKS_ENOMEM, "hoisted: workspace too small: need %zu", need);
    hipStream_t s = (hipStream_t)stream;
    Plan P(c, ws);
    // rotation tables: key bases and Galois elements
    uint8_t *tab_ws = (uint8_t *)P.limbs(1);
    std::vector<uint8_t> tab((size_t)n_rot * 12, 0);
    for (u32 i = 0; i < n_rot; i++) {
        const u64 *kp = galois_elts[i] == 1 ? nullptr : galois_keys[i];
        memcpy(tab.data() + (size_t)i * 8, &kp, 8);
        memcpy(tab.data() + (size_t)n_rot * 8 + (size_t)i * 4, &galois_elts[i], 4);
    }
    uint8_t *tab_dev = nullptr;
    CK(upload(c, tab_ws, tab.data(), tab.size(), s, &tab_dev));
    // plaintexts over Q_l U P in NTT form
    u64 *pts = P.limbs((size_t)n_rot * E);
    std::vector<Item> ptl, isc, modup, scl, mdown;
    for (u32 i = 0; i < n_rot; i++)
        for (u32 t = 0; t < E; t++) {
            Item it = item0();
            it.in[0] = (const u64 *)(pt_coeffs + (size_t)i * N);
            it.out = pts + ((size_t)i * E + t) * N;
            it.prime = t < L ? t : c->n_q + (t - L);
            ptl.push_back(it);
        }
    std::vector<HoItem> ho;
    std::vector<u64 *> accs(B);
    std::vector<u64 *> exts(B);
    for (u32 x = 0; x < B; x++) {
        u64 *dcoef = P.limbs(L);
        u64 *ext = P.limbs((size_t)beta * E);
        u64 *acc = P.limbs((size_t)2 * E);
        accs[x] = acc;
        exts[x] = ext;
        for (u32 i = 0; i < L; i++) {
            const u32 j = i / A, lo = j * A, sz = std::min(A, L - lo);
            Item it = item0();
            it.in[0] = limb(c, in[x], 1, i);
            it.out = dcoef + (size_t)i * N;
            it.prime = i;
            it.b = 2;
            it.c = j * A + sz - 1;
            it.a = i - lo;
            isc.push_back(it);
        }
        for (u32 j = 0; j < beta; j++) {
            const u32 lo = j * A, sz = std::min(A, L - lo);
            for (u32 t = 0; t < E; t++) {
                if (t >= lo && t < lo + sz) continue;
                Item it = item0();
                it.in[0] = dcoef + (size_t)lo * N;
                it.a = lo;
                it.b = sz;
                it.c = j;
                it.v = 1;
                it.prime = t < L ? t : c->n_q + (t - L);
                it.out = ext + ((size_t)j * E + t) * N;
                modup.push_back(it);
            }
        }
        for (u32 cc = 0; cc < 2; cc++)
            for (u32 m = 0; m < k; m++) {
                Item it = item0();
                it.in[0] = acc + ((size_t)cc * E + L + m) * N;
                it.out = (u64 *)it.in[0];
                it.prime = c->n_q + m;
                scl.push_back(it);
            }
        for (u32 cc = 0; cc < 2; cc++)
            for (u32 i = 0; i < L; i++) {
                Item it = item0();
                it.in[0] = acc + ((size_t)cc * E + L) * N;
                it.a = c->n_q;
                it.b = k;
                it.in[1] = acc + ((size_t)cc * E + i) * N;
                it.prime = i;
                it.out = limb(c, out[x], cc, i);
                mdown.push_back(it);
            }
    }
    for (u32 g0 = 0; g0 < B; g0 += kHoCts) {
        const u32 n = std::min<u32>(kHoCts, B - g0);
        for (u32 t = 0; t < E; t++) {
            HoItem h;
            memset(&h, 0, sizeof h);
            h.n_ct = n;
            h.prime = t < L ? t : c->n_q + (t - L);
            h.pos = t;
            h.E = E;
            h.L = L;
            h.beta = beta;
            h.alpha = A;
            h.n_rot = n_rot;
            h.keys = (const u64 *const *)tab_dev;
            h.galois = (const u32 *)(tab_dev + (size_t)n_rot * 8);
            h.pts = pts;
            for (u32 q = 0; q < n; q++) {
                h.ext[q] = exts[g0 + q];
                h.c0[q] = t < L ? limb(c, in[g0 + q], 0, t) : nullptr;
                h.c1[q] = limb(c, in[g0 + q], 1, 0);
                h.acc[q] = accs[g0 + q];
            }
            ho.push_back(h);
        }
    }
    P.add(0, F_INT, ptl);
    P.add(1, I_SCALE, isc);
    add_modup(P, modup);
    P.add(5, 0, ho);
    P.add(1, I_COPY, scl);
    P.add(0, F_MODDOWN, mdown);
    CK(P.run(ws_bytes, s));
    for (u32 x = 0; x < B; x++) {
        out[x].n_poly = 2;
        out[x].level = l;
        out[x].scale = in[x].scale * pt_scale;
    }
    return CKKS_OK;
}

// ---------------------------------------------------------------------
// encrypted linear layer
// ---------------------------------------------------------------------
extern "C" int ckks_linear(const ckks_ctx *c, const ckks_ct *in, uint32_t n_in, const int64_t *W, double w_scale,
                           ckks_ct *out, uint32_t n_out, void *ws, size_t ws_bytes, void *stream) {
    CK(check_ctx(c));
    if (!in || !W || !out || !n_in || !n_out) return fail(CKKS_EINVAL, "linear: bad argument");
    const u32 l = in[0].level, L = l + 1, stride = in[0].limb_stride;
    for (u32 i = 0; i < n_in; i++) {
        CK(check_ct(c, in[i], "linear"));
        if (in[i].n_poly != 2) return fail(CKKS_EINVAL, "linear: inputs must have 2 polys");
        if (in[i].level != l) return fail(CKKS_ELEVEL, "linear: input levels differ");
        if (in[i].scale != in[0].scale) return fail(CKKS_ESCALE, "linear: input scales differ");
        if (in[i].limb_stride != stride) return fail(CKKS_EINVAL, "linear: input limb strides differ");
    }
    const u32 ostride = std::max(out[0].limb_stride, L);
    for (u32 j = 0; j < n_out; j++)
        if (!out[j].data || std::max(out[j].limb_stride, L) != ostride)
            return fail(CKKS_EINVAL, "linear: outputs need data and one limb stride");
    const size_t wt_bytes = (size_t)L * n_out * n_in * 8;
    const size_t ptr_off = (wt_bytes + 255) & ~(size_t)255;
    const size_t need = ptr_off + (size_t)(n_in + n_out) * 8;
    if (need > ws_bytes) return fail(CKKS_ENOMEM, "linear: workspace too small: need %zu", need);
    if (!ws || (((uintptr_t)ws) & 255)) return fail(CKKS_EINVAL, "linear: null or unaligned workspace");
    uint8_t *w8 = (uint8_t *)ws;
    u64 *wt = (u64 *)w8;
    std::vector<const u64 *> ptrs(n_in + n_out);
    for (u32 i = 0; i < n_in; i++) ptrs[i] = in[i].data;
    for (u32 j = 0; j < n_out; j++) ptrs[n_in + j] = out[j].data;
    hipStream_t s = (hipStream_t)stream;
    uint8_t *pt8 = nullptr;
    CK(upload(c, w8 + ptr_off, ptrs.data(), ptrs.size() * 8, s, &pt8));
    const u32 cnt = n_out * n_in;
    HIP_TRY(issue(c, s, [tb = c->tb, W, wt, cnt, L](hipStream_t st) {
        return launch_reduce_weights(tb, W, wt, cnt, L, st);
    }));
    ProfRec rec;
    if (g_prof_on) {
        rec.name = launch_name(4, 0, c->log_n);
        rec.items = n_out;
        HIP_TRY(hipEventCreate(&rec.e0));
        HIP_TRY(hipEventCreate(&rec.e1));
        HIP_TRY(hipEventRecord(rec.e0, s));
    }
    HIP_TRY(issue(c, s, [tb = c->tb, pt8, wt, n_in, n_out, L, stride, ostride](hipStream_t st) {
        return launch_linear(tb, (const u64 *const *)pt8, wt, (u64 *const *)(pt8 + (size_t)n_in * 8), n_in, n_out, L,
                             stride, ostride, st);
    }));
    if (g_prof_on) {
        HIP_TRY(hipEventRecord(rec.e1, s));
        g_prof.push_back(rec);
    }
    for (u32 j = 0; j < n_out; j++) {
        out[j].n_poly = 2;
        out[j].level = l;
        out[j].limb_stride = ostride;
        out[j].scale = in[0].scale * w_scale;
    }
    return CKKS_OK;
}

// ---------------------------------------------------------------------
// encrypted linear layer, sparse rows (CSR)
// ---------------------------------------------------------------------

extern "C" size_t ckks_linear_csr_workspace_bytes(const ckks_ctx *c, uint32_t n_in, uint32_t n_out, size_t nnz,
                                                  uint32_t level) {
    if (!c) return 0;
    const size_t L = level + 1;
    const size_t grouped = al256(n_out * sizeof(LinGroup)) + al256(nnz * 4) + al256(L * nnz * 8) + al256(L * nnz * 16);
    // matrix-core path (every row has the same column list, of nnz / n_out
    // entries, which may repeat an input): column list, weights as int64,
    // pointer table and the weights' digit planes
    const size_t ncols = std::max((size_t)n_in, n_out ? (nnz + n_out - 1) / n_out : 0);
    const size_t rows_pad = ((size_t)n_out + 31) / 32 * 32, k_pad = (ncols + 63) / 64 * 64;
    const size_t mfma = al256(ncols * 4) + al256(nnz * 8) + al256((size_t)(n_in + n_out) * 8) +
                        al256((size_t)kWDig * rows_pad * k_pad);
    return std::max(grouped, mfma) + al256((size_t)(n_in + n_out) * 8) + 1024;
}

namespace {
// the matrix-core path for a layer whose rows all use one column list
int linear_mfma(const ckks_ctx *c, const ckks_ct *in, u32 n_in, u32 n_out, const u32 *cols, u32 ncols,
                const int64_t *w, u32 L, u32 stride, u32 ostride, ckks_ct *out, void *ws, size_t ws_bytes,
                hipStream_t s) {
    const size_t rows_pad = ((size_t)n_out + 31) / 32 * 32, k_pad = ((size_t)ncols + 63) / 64 * 64;
    const size_t o_cols = 0, o_w = al256((size_t)ncols * 4), o_ptr = o_w + al256((size_t)n_out * ncols * 8),
                 o_wd = o_ptr + al256((size_t)(n_in + n_out) * 8),
                 need = o_wd + al256((size_t)kWDig * rows_pad * k_pad);
    if (need > ws_bytes) return fail(CKKS_ENOMEM, "linear_csr: workspace too small: need %zu", need);
    std::vector<uint8_t> img(o_wd, 0);
    memcpy(img.data() + o_cols, cols, (size_t)ncols * 4);
    memcpy(img.data() + o_w, w, (size_t)n_out * ncols * 8);
    std::vector<const u64 *> ptrs(n_in + n_out);
    for (u32 i = 0; i < n_in; i++) ptrs[i] = in[i].data;
    for (u32 j = 0; j < n_out; j++) ptrs[n_in + j] = out[j].data;
    memcpy(img.data() + o_ptr, ptrs.data(), ptrs.size() * 8);
    uint8_t *w8 = nullptr;
    CK(upload(c, (uint8_t *)ws, img.data(), img.size(), s, &w8));
    // the digit planes live in the workspace, at o_wd, in every case: while
    // recording the image above goes to the arena, but the planes are still
    // written into the workspace by the recorded kernel on every replay
    int8_t *wd = (int8_t *)((uint8_t *)ws + o_wd);
    const u32 rp = (u32)rows_pad, kp = (u32)k_pad;
    ProfRec rec;
    if (g_prof_on) {
        rec.name = launch_name(7, 0, c->log_n);
        rec.items = n_out;
        HIP_TRY(hipEventCreate(&rec.e0));
        HIP_TRY(hipEventCreate(&rec.e1));
        HIP_TRY(hipEventRecord(rec.e0, s));
    }
    HIP_TRY(issue(c, s, [w8, o_w, n_out, ncols, rp, kp, wd](hipStream_t st) {
        return launch_weight_digits((const i64 *)(w8 + o_w), n_out, ncols, rp, kp, wd, st);
    }));
    // one launch per run of consecutive limbs of one digit count: primes
    // below 2^42 take six residue digits, larger ones nine
    for (u32 t0 = 0; t0 < L;) {
        const bool small = c->primes[t0] < (1ull << 42);
        u32 t1 = t0 + 1;
        while (t1 < L && (c->primes[t1] < (1ull << 42)) == small) t1++;
        const u32 tc = t1 - t0;
        HIP_TRY(issue(c, s, [tb = c->tb, wd, rp, kp, w8, o_cols, o_ptr, ncols, n_in, n_out, t0, tc, small, stride,
                             ostride](hipStream_t st) {
            return launch_linear_mfma(tb, wd, rp, kp, (const u32 *)(w8 + o_cols), ncols, n_out,
                                      (const u64 *const *)(w8 + o_ptr), (u64 *const *)(w8 + o_ptr + (size_t)n_in * 8),
                                      t0, tc, small, stride, ostride, st);
        }));
        t0 = t1;
    }
    if (g_prof_on) {
        HIP_TRY(hipEventRecord(rec.e1, s));
        g_prof.push_back(rec);
    }
    return CKKS_OK;
}
}  // namespace

extern "C" int ckks_linear_csr(const ckks_ctx *c, const ckks_ct *in, uint32_t n_in, uint32_t n_out,
                               const uint32_t *row_ptr, const uint32_t *col, const int64_t *w, double w_scale,
                               ckks_ct *out, void *ws, size_t ws_bytes, void *stream) {
    CK(check_ctx(c));
    if (!in || !out || !row_ptr || !col || !w || !n_in || !n_out) return fail(CKKS_EINVAL, "linear_csr: bad argument");
    const u32 l = in[0].level, L = l + 1, stride = in[0].limb_stride;
    for (u32 i = 0; i < n_in; i++) {
        CK(check_ct(c, in[i], "linear_csr"));
        if (in[i].n_poly != 2) return fail(CKKS_EINVAL, "linear_csr: inputs must have 2 polys");
        if (in[i].level != l) return fail(CKKS_ELEVEL, "linear_csr: input levels differ");
        if (in[i].scale != in[0].scale) return fail(CKKS_ESCALE, "linear_csr: input scales differ");
        if (in[i].limb_stride != stride) return fail(CKKS_EINVAL, "linear_csr: input limb strides differ");
    }
    const u32 ostride = std::max(out[0].limb_stride, L);
    for (u32 j = 0; j < n_out; j++)
        if (!out[j].data || std::max(out[j].limb_stride, L) != ostride)
            return fail(CKKS_EINVAL, "linear_csr: outputs need data and one limb stride");
    const size_t nnz = row_ptr[n_out];
    for (u32 j = 0; j < n_out; j++)
        if (row_ptr[j + 1] < row_ptr[j]) return fail(CKKS_EINVAL, "linear_csr: row_ptr not monotone");
    for (size_t e = 0; e < nnz; e++)
        if (col[e] >= n_in) return fail(CKKS_EINVAL, "linear_csr: column %u out of range", col[e]);
    if (!ws || (((uintptr_t)ws) & 255)) return fail(CKKS_EINVAL, "linear_csr: null or unaligned workspace");
    if (c->tb.lin_mfma) {
        // one column list for every row and small weights: the matrix cores
        const u32 nc = row_ptr[1] - row_ptr[0];
        bool same = nc > 0 && nc <= kMfmaMaxIn && (size_t)nc * n_out == nnz;
        for (u32 j = 1; same && j < n_out; j++) same = memcmp(col, col + (size_t)j * nc, (size_t)nc * 4) == 0;
        for (size_t e = 0; same && e < nnz; e++) same = w[e] <= kWMax && w[e] >= -kWMax;
        if (same) {
            CK(linear_mfma(c, in, n_in, n_out, col, nc, w, L, stride, ostride, out, ws, ws_bytes,
                           (hipStream_t)stream));
            for (u32 j = 0; j < n_out; j++) {
                out[j].n_poly = 2;
                out[j].level = l;
                out[j].limb_stride = ostride;
                out[j].scale = in[0].scale * w_scale;
            }
            return CKKS_OK;
        }
    }
    // groups of consecutive rows with identical column lists
    std::vector<LinGroup> groups;
    std::vector<u32> cols;
    std::vector<i64> wv;
    for (u32 j = 0; j < n_out;) {
        const u32 b = row_ptr[j], n = row_ptr[j + 1] - b;
        u32 r = 1;
        while (j + r < n_out && r < (u32)kLinRows) {
            const u32 b2 = row_ptr[j + r], n2 = row_ptr[j + r + 1] - b2;
            if (n2 != n || memcmp(col + b, col + b2, n * 4) != 0) break;
            r++;
        }
        LinGroup g{j, r, (u32)cols.size(), n, (u32)wv.size(), 0};
        cols.insert(cols.end(), col + b, col + b + n);
        for (u32 k = 0; k < r; k++) wv.insert(wv.end(), w + row_ptr[j + k], w + row_ptr[j + k] + n);
        groups.push_back(g);
        j += r;
    }
    const size_t W = wv.size();
    std::vector<u64> wt((size_t)L * W);
    for (u32 t = 0; t < L; t++) {
        const u64 q = c->primes[t];
        for (size_t e = 0; e < W; e++) {
            const i64 v = wv[e];
            u64 m = v >= 0 ? (u64)v % q : (q - ((u64)(-(v + 1)) + 1) % q) % q;
            wt[(size_t)t * W + e] = m;
        }
    }
    // FP64 copies (w, w / q) for the limbs whose prime is below 2^50
    std::vector<double> wf((size_t)L * W * 2, 0.0);
    for (u32 t = 0; t < L; t++) {
        const u64 q = c->primes[t];
        if (q >= kFpPrimeBound) continue;
        for (size_t e = 0; e < W; e++) {
            const double v = (double)wt[(size_t)t * W + e];
            wf[2 * ((size_t)t * W + e)] = v;
            wf[2 * ((size_t)t * W + e) + 1] = v / (double)q;
        }
    }
    const size_t o_groups = 0, o_cols = al256(groups.size() * sizeof(LinGroup)), o_wt = o_cols + al256(cols.size() * 4),
                 o_wf = o_wt + al256(wt.size() * 8), o_ptr = o_wf + al256(wf.size() * 8),
                 need = o_ptr + al256((size_t)(n_in + n_out) * 8);
    if (need > ws_bytes) return fail(CKKS_ENOMEM, "linear_csr: workspace too small: need %zu", need);
    std::vector<uint8_t> img(need, 0);
    memcpy(img.data() + o_groups, groups.data(), groups.size() * sizeof(LinGroup));
    memcpy(img.data() + o_cols, cols.data(), cols.size() * 4);
    memcpy(img.data() + o_wt, wt.data(), wt.size() * 8);
    memcpy(img.data() + o_wf, wf.data(), wf.size() * 8);
    std::vector<const u64 *> ptrs(n_in + n_out);
    for (u32 i = 0; i < n_in; i++) ptrs[i] = in[i].data;
    for (u32 j = 0; j < n_out; j++) ptrs[n_in + j] = out[j].data;
    memcpy(img.data() + o_ptr, ptrs.data(), ptrs.size() * 8);
    hipStream_t s = (hipStream_t)stream;
    uint8_t *w8 = nullptr;
    CK(upload(c, (uint8_t *)ws, img.data(), need, s, &w8));
    ProfRec rec;
    if (g_prof_on) {
        rec.name = launch_name(8, 0, c->log_n);
        rec.items = (u32)groups.size();
        HIP_TRY(hipEventCreate(&rec.e0));
        HIP_TRY(hipEventCreate(&rec.e1));
        HIP_TRY(hipEventRecord(rec.e0, s));
    }
    const u32 n_groups = (u32)groups.size();
    u32 max_rows = 1;
    for (const LinGroup &g : groups) max_rows = std::max(max_rows, g.nrows);
    HIP_TRY(issue(c, s, [tb = c->tb, w8, n_groups, o_groups, o_cols, o_wt, o_wf, o_ptr, W, n_in, L, stride,
                         ostride, max_rows](hipStream_t st) {
        return launch_linear_grouped(tb, (const LinGroup *)(w8 + o_groups), n_groups, (const u32 *)(w8 + o_cols),
                                     (const u64 *)(w8 + o_wt), (const double2 *)(w8 + o_wf), (u32)W,
                                     (const u64 *const *)(w8 + o_ptr),
                                     (u64 *const *)(w8 + o_ptr + (size_t)n_in * 8), L, stride, ostride, max_rows,
                                     st);
    }));
    if (g_prof_on) {
        HIP_TRY(hipEventRecord(rec.e1, s));
        g_prof.push_back(rec);
    }
    for (u32 j = 0; j < n_out; j++) {
        out[j].n_poly = 2;
        out[j].level = l;
        out[j].limb_stride = ostride;
        out[j].scale = in[0].scale * w_scale;
    }
    return CKKS_OK;
}
