// Encrypted linear layers of the host runtime: dense rows (ckks_linear),
// sparse rows in CSR form (ckks_linear_csr) with its row groups for the
// grouped VALU kernel, and the matrix-core path for rows that share one
// column list.
#include "ckks_runtime.h"

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
