// Server-side ciphertext operations of the host runtime: element-wise
// operations, the key-switching planner (relinearisation, rotation,
// hoisted rotations), rescale and the fused batched HMult. Each call checks
// its descriptors, builds the work-item tables and runs them through a Plan.
#include "ckks_runtime.h"

namespace ckks {
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
    P.add(0, moddown_op(c), mdown);
}
}  // namespace ckks

// server side: elementwise ops
// ---------------------------------------------------------------------
int ckks::ew_binary(const ckks_ctx *c, u32 op, const ckks_ct *a, const ckks_ct *b, const ckks_pt *p,
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
int ckks::plan_hmult(Plan &P, const u64 *const *rk, const ckks_ct *a, const ckks_ct *b, ckks_ct *out, u32 B) {
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
        // ModUp of every digit to the primes outside it, then NTT; limb-major,
        // so that consecutive items (one XCD's) share a prime's twiddle table
        for (u32 t = 0; t < E; t++) {
            for (u32 j = 0; j < beta; j++) {
                const u32 lo = j * A, s = std::min(A, L - lo);
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
        // remaining limbs: ModDown correction, NTT, rescale; limb-major, so
        // that the two polynomials' items of one prime share its twiddles
        for (u32 i = 0; i < l; i++)
            for (u32 cc = 0; cc < 2; cc++) {
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
    const size_t items = B * (L + beta * E + 2 * (c->n_p + L)) * sizeof(Item) + E * B * sizeof(HoItem) +
                         (size_t)n_rot * E * sizeof(Item);
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
    // Staged form (see kHoChunk): every Galois element is 1 mod 2N / kHoChunk,
    // so each aligned block of kHoChunk slots is mapped onto itself; then up
    // to kHoStageRows rows (ciphertexts x digits) of a block sit in LDS.
    u32 per = kHoCts;
    bool staged = N >= kHoChunk && beta <= kHoStageRows;
    for (u32 i = 0; i < n_rot && staged; i++) staged = galois_elts[i] % (2 * N / kHoChunk) == 1;
    if (staged) per = std::min<u32>(kHoCts, kHoStageRows / beta);
    // items ordered by limb, so the workgroups that read one limb of a key run together
    for (u32 t = 0; t < E; t++) {
        for (u32 g0 = 0; g0 < B; g0 += per) {
            const u32 n = std::min<u32>(per, B - g0);
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
    P.add(5, staged ? (int)(per * beta) : 0, ho);
    P.add(1, I_COPY, scl);
    P.add(0, moddown_op(c), mdown);
    CK(P.run(ws_bytes, s));
    for (u32 x = 0; x < B; x++) {
        out[x].n_poly = 2;
        out[x].level = l;
        out[x].scale = in[x].scale * pt_scale;
    }
    return CKKS_OK;
}

// ---------------------------------------------------------------------
