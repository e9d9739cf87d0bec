// Host runtime behind the C ABI of libckks_hip.so: parameter checks, prime
// and root search, device table image, FP64 canonical-embedding encoder,
// exact CRT decoder, and the per-op planners that turn ciphertext
// descriptors into flat work-item tables for the gfx950 kernels.
//
// The library never allocates device memory: every call receives a caller
// workspace, carves scratch limbs from its front and places the work-item
// tables at its end, uploads the tables with one asynchronous copy and
// launches the kernels on the caller's stream.
#include "ckks_runtime.h"

namespace ckks {
static thread_local std::string g_err;
int set_error(int code, const char *msg) {
    g_err = msg;
    return code;
}
int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
}  // namespace ckks

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
namespace ckks {
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
namespace {
const char *fwd_names[] = {"ntt_fwd", "ntt_fwd_modup", "ntt_fwd_rescale", "ntt_fwd_moddown",
                           "ntt_fwd_moddown_z", "ntt_fwd_sample", "ntt_fwd_int", "ntt_fwd_relin_rescale",
                           "ntt_fwd_modup", "ntt_fwd_modup", "ntt_fwd_modup", "ntt_fwd_modup",
                           "ntt_fwd_moddown_z", "ntt_fwd_moddown_z", "ntt_fwd_relin_rescale", "ntt_fwd_relin_rescale",
                           "ntt_fwd_moddown", "ntt_fwd_moddown"};
const char *inv_names[] = {"ntt_inv", "ntt_inv_mul", "ntt_inv_scale", "ntt_inv_decrypt"};
const char *ew_names[] = {"ew_add", "ew_sub", "ew_mul", "ew_mul_const", "ew_add_const", "ew_tensor", "ew_copy",
                          "ew_automorph", "ew_neg", "ew_keygen", "ew_encrypt", "ew_square_s", "ew_hmult_fin",
                          "ew_unused", "ew_hmult_t"};
}  // namespace
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
}  // namespace ckks

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
        if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) ms = 0;  // reported as 0 ms
        if (out && k < cap) {
            memset(&out[k], 0, sizeof out[k]);
            snprintf(out[k].name, sizeof out[k].name, "%s", r.name.c_str());
            out[k].items = r.items;
            out[k].ms = ms;
        }
        k++;
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    g_prof.clear();
    *n = k;
    return CKKS_OK;
}

// ---------------------------------------------------------------------
// planning: scratch carving + work-item tables

// ---------------------------------------------------------------------
// planning: scratch carving + work-item tables
// ---------------------------------------------------------------------
namespace ckks {
// Calls that must not allocate (ckks_hmult_relin_rescale_noalloc) set this
// flag for their duration on the calling thread: uploads then skip the
// pinned staging ring (created on first use) and its events and copy
// straight from the host descriptor buffer, and no profiling events are made.
thread_local bool g_no_alloc = false;
void set_no_alloc(bool on) { g_no_alloc = on; }

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
std::vector<uint8_t> &desc_pool() {
    thread_local std::vector<uint8_t> pool;
    return pool;
}

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
// ModDown kernel for the context's special-prime count
int moddown_op(const ckks_ctx *c) { return c->n_p <= 2 ? F_MODDOWN_P1 + (int)c->n_p - 1 : F_MODDOWN; }

// items of the inner product: ciphertexts of one level and one switching
// key are grouped by kIpCts so that each key residue is loaded once per
// group (requests of different clients, i.e. different keys, share the
// launch but not an item). Items are
// emitted prime by prime (every group's item for prime 0, then prime 1, ...)
// so that the blocks in flight at any time share one prime's key limbs
// (2 beta limbs), which then stay in L2 instead of every group re-reading
// all primes' keys.
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
}  // namespace ckks


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
