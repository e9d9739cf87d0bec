// Graph runtime: forward neuronal firing over a multi-directed graph of
// encrypted layers (the paper's Algorithms 1-5 and the graph rules of
// Section 4: a node fires once every in-edge carries a signal, multiple
// inputs are stacked in edge order, the result is broadcast to every
// out-edge, parallel edges are independent edges).
//
// A signal is a list of ciphertexts. Node receptors are batched calls of
// the C ABI (linear layer, rescale, bias, rotations, square). Planning runs
// the same traversal without device work to fix every node's output count,
// level and scale, and to lay out all outputs and scratch in the caller's
// workspace.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/ckks.h"

namespace ckks {
int set_error(int code, const char *msg);
int ctx_upload_bytes(const ckks_ctx *c, void *dst, const void *src, size_t bytes, void *stream, void **where);
}

namespace {
typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;

int gfail(int code, const char *msg) { return ckks::set_error(code, msg); }

i64 round_half_away(double x) { return (i64)(x < 0 ? -floor(-x + 0.5) : floor(x + 0.5)); }
size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

std::vector<std::pair<int, int>> naf(i64 n) {  // (position, +-1), least significant first
    std::vector<std::pair<int, int>> out;
    int k = 0;
    while (n != 0) {
        if (n & 1) {
            int d = 2 - (int)(n & 3);
            out.push_back({k, d});
            n -= d;
        }
        n >>= 1;  // arithmetic shift: n is even here
        k++;
    }
    return out;
}

struct Node {
    int kind = 0;
    // input
    u32 in_count = 0, in_level = 0;
    double in_scale = 1.0;
    // linear
    u32 n_out = 0;
    std::vector<u32> row_ptr, col;
    std::vector<i64> w;
    double w_scale = 1.0;
    std::vector<double> bias;
    // diagonal dense
    std::vector<int32_t> in_steps, post_steps;
    std::vector<i64> diag;  // [n_diag][N]
    double pt_scale = 1.0;
    std::vector<double> bias_slots;
    std::vector<i64> bias_coeffs;  // [N], at the output scale
    bool hoisted = false;
    // polynomial activation
    std::vector<double> coeffs;  // c_0 .. c_d
    // wiring
    std::vector<u32> in_edges, out_edges;
    // plan
    u32 out_count = 0, out_level = 0, in_lvl_used = 0;
    double out_scale = 0;
    size_t out_off = 0, pt_off = 0;
    std::vector<ckks_ct> out;
    bool fired = false;
};
struct Edge {
    u32 from, to;
    bool has = false;
    std::vector<ckks_ct> sig;
};
}  // namespace

struct ckks_graph {
    const ckks_ctx *c;
    u32 N;
    std::vector<Node> nodes;
    std::vector<Edge> edges;
    bool planned = false;
    size_t ws_total = 0, scratch_off = 0, scratch_bytes = 0;
    // run state
    bool dry = true;
    uint8_t *ws = nullptr;
    void *stream = nullptr;
    const u64 *rk = nullptr;
    std::map<u32, const u64 *> gk;
    int err = CKKS_OK;
};

namespace {
// ------------------------------------------------------------------
// receptors
// ------------------------------------------------------------------
struct Sig {
    std::vector<ckks_ct> v;
};

// level match (Section 4.1): switch every ciphertext down to the lowest level
int match_levels(std::vector<ckks_ct> &v) {
    if (v.empty()) return CKKS_OK;
    u32 lo = v[0].level;
    for (auto &x : v) lo = std::min(lo, x.level);
    for (auto &x : v) x.level = lo;
    for (auto &x : v)
        if (x.scale != v[0].scale) return gfail(CKKS_ESCALE, "graph: inputs of a node have different scales");
    return CKKS_OK;
}

size_t ct_bytes(const ckks_graph *g, u32 level) { return (size_t)2 * (level + 1) * g->N * 8; }

void need(ckks_graph *g, size_t bytes) { g->scratch_bytes = std::max(g->scratch_bytes, bytes); }

uint8_t *scratch(ckks_graph *g) { return g->ws + g->scratch_off; }
size_t scratch_avail(ckks_graph *g) { return g->ws_total - g->scratch_off; }

#define GK(x)                            \
    do {                                 \
        int r_ = (x);                    \
        if (r_ != CKKS_OK) return r_;    \
    } while (0)

std::vector<ckks_ct> make_cts(ckks_graph *g, size_t off, u32 count, u32 level, u32 stride, double scale) {
    std::vector<ckks_ct> v(count);
    for (u32 i = 0; i < count; i++) {
        v[i].data = g->dry ? nullptr : (u64 *)(g->ws + off + (size_t)i * 2 * stride * g->N * 8);
        v[i].n_poly = 2;
        v[i].level = level;
        v[i].limb_stride = stride;
        v[i].reserved = 0;
        v[i].scale = scale;
    }
    return v;
}

// rotate every ciphertext of `in` by `step` slots into `out`, composing the
// step from power-of-two keys (non-adjacent form) when it has no key
int rotate_all(ckks_graph *g, const std::vector<ckks_ct> &in, std::vector<ckks_ct> &out, std::vector<ckks_ct> &tmp,
               i64 step) {
    const i64 half = g->N / 2;
    step = ((step % half) + half) % half;
    const u32 B = (u32)in.size();
    if (step == 0) return gfail(CKKS_EINVAL, "graph: zero rotation requested");
    std::vector<std::pair<u32, int>> seq;  // galois element per hop
    u32 ge = ckks_galois_elt(g->c, (int32_t)step);
    if (g->dry || g->gk.count(ge)) {
        seq.push_back({ge, 0});
    }
    if (!g->dry && !g->gk.count(ge)) {
        const i64 s = step <= half / 2 ? step : step - half;
        for (auto &d : naf(s)) {
            u32 e = ckks_galois_elt(g->c, (int32_t)(d.second * (i64)(1ll << d.first)));
            if (!g->gk.count(e)) return gfail(CKKS_ENOKEY, "graph: missing Galois key for a rotation");
            seq.push_back({e, 0});
        }
    }
    size_t ws_need = ckks_workspace_bytes(g->c, CKKS_OP_KEYSWITCH, B, nullptr);
    need(g, ws_need);
    if (g->dry) return CKKS_OK;
    // alternate between out and tmp so that the last hop lands in out
    const bool odd = (seq.size() % 2) == 1;
    const std::vector<ckks_ct> *src = &in;
    for (size_t h = 0; h < seq.size(); h++) {
        const bool to_out = odd ? (h % 2 == 0) : (h % 2 == 1);
        std::vector<ckks_ct> &dst = to_out ? out : tmp;
        for (u32 b = 0; b < B; b++) dst[b].level = (*src)[b].level;
        const std::vector<const u64 *> keys(B, g->gk[seq[h].first]);
        const std::vector<u32> elts(B, seq[h].first);
        GK(ckks_rotate(g->c, keys.data(), elts.data(), src->data(), dst.data(), B, scratch(g), scratch_avail(g),
                       g->stream));
        src = &dst;
    }
    return CKKS_OK;
}

int fire_linear(ckks_graph *g, Node &n, std::vector<ckks_ct> in) {
    GK(match_levels(in));
    if (in.size() == 0 || n.col.empty()) return gfail(CKKS_EINVAL, "graph: empty linear node");
    for (u32 c : n.col)
        if (c >= in.size()) return gfail(CKKS_EINVAL, "graph: linear column beyond the node's input count");
    const u32 l = in[0].level;
    if (l == 0) return gfail(CKKS_EDEPTH, "graph: no level left for a linear node");
    n.out_level = l - 1;
    n.in_lvl_used = l;
    n.out_count = n.n_out;
    const double s_prod = in[0].scale * n.w_scale;
    n.out_scale = s_prod / (double)ckks_ctx_prime(g->c, l);
    n.out = make_cts(g, n.out_off, n.n_out, l, l + 1, s_prod);
    need(g, ckks_linear_csr_workspace_bytes(g->c, (u32)in.size(), n.n_out, n.w.size(), l));
    need(g, ckks_workspace_bytes(g->c, CKKS_OP_RESCALE, n.n_out, nullptr));
    need(g, ckks_workspace_bytes(g->c, CKKS_OP_ELEMENTWISE, n.n_out, nullptr));
    if (g->dry) {
        for (auto &x : n.out) x.level = l - 1, x.scale = n.out_scale;
        return CKKS_OK;
    }
    GK(ckks_linear_csr(g->c, in.data(), (u32)in.size(), n.n_out, n.row_ptr.data(), n.col.data(), n.w.data(),
                       n.w_scale, n.out.data(), scratch(g), scratch_avail(g), g->stream));
    if (n.bias.empty()) {
        GK(ckks_rescale(g->c, n.out.data(), n.out.data(), n.n_out, scratch(g), scratch_avail(g), g->stream));
    } else {
        // the bias at the scale after the rescale, added in the rescale's pass
        std::vector<i64> v(n.n_out);
        for (u32 j = 0; j < n.n_out; j++) v[j] = round_half_away(n.bias[j] * n.out_scale);
        GK(ckks_rescale_add_scalar(g->c, n.out.data(), v.data(), n.out.data(), n.n_out, scratch(g),
                                   scratch_avail(g), g->stream));
    }
    return CKKS_OK;
}

int fire_square(ckks_graph *g, Node &n, std::vector<ckks_ct> in) {
    GK(match_levels(in));
    const u32 B = (u32)in.size(), l = in[0].level;
    if (l == 0) return gfail(CKKS_EDEPTH, "graph: no level left for a square node");
    n.out_count = B;
    n.out_level = l - 1;
    n.out_scale = in[0].scale * in[0].scale / (double)ckks_ctx_prime(g->c, l);
    n.out = make_cts(g, n.out_off, B, l - 1, l, n.out_scale);
    std::vector<u32> lv(B, l);
    need(g, ckks_workspace_bytes(g->c, CKKS_OP_HMULT, B, lv.data()));
    if (g->dry) return CKKS_OK;
    const std::vector<const u64 *> keys(B, g->rk);
    return ckks_hmult_relin_rescale(g->c, keys.data(), in.data(), in.data(), n.out.data(), B, scratch(g),
                                    scratch_avail(g), g->stream);
}

// p(x) by Horner's rule: h = rescale(x c_d); h = rescale(relin(x' (x) (h + c_k)))
// for k = d-1..1 with x' switched down to h's level; h += c_0
int fire_poly(ckks_graph *g, Node &n, std::vector<ckks_ct> in) {
    GK(match_levels(in));
    const u32 B = (u32)in.size(), l = in[0].level, d = (u32)n.coeffs.size() - 1;
    if (l < d) return gfail(CKKS_EDEPTH, "graph: not enough levels for the polynomial activation");
    const size_t cb = ct_bytes(g, l);
    std::vector<ckks_ct> h = make_cts(g, n.out_off, B, l, l + 1, 1.0);
    std::vector<ckks_ct> t = make_cts(g, n.out_off + al(B * cb), B, l, l + 1, 1.0);
    const double s_x = in[0].scale;
    n.out_count = B;
    std::vector<u32> lv(B, l);
    need(g, ckks_workspace_bytes(g->c, CKKS_OP_HMULT, B, lv.data()));
    need(g, ckks_workspace_bytes(g->c, CKKS_OP_RESCALE, B, nullptr));
    need(g, ckks_workspace_bytes(g->c, CKKS_OP_ELEMENTWISE, B, nullptr));
    // h = rescale(x * c_d) + c_{d-1} (c_0 when d = 1), the constant added in
    // the rescale's pass at the scale after it
    double hs = s_x * n.w_scale;
    hs /= (double)ckks_ctx_prime(g->c, l);
    const u32 k_first = d >= 2 ? d - 1 : 0;
    if (!g->dry) {
        std::vector<i64> v(B, round_half_away(n.coeffs[d] * n.w_scale));
        std::vector<double> vs(B, n.w_scale);
        GK(ckks_multiply_scalar(g->c, in.data(), v.data(), vs.data(), h.data(), B, scratch(g), scratch_avail(g),
                                g->stream));
        std::vector<i64> c1(B, round_half_away(n.coeffs[k_first] * hs));
        GK(ckks_rescale_add_scalar(g->c, h.data(), c1.data(), h.data(), B, scratch(g), scratch_avail(g),
                                   g->stream));
    }
    u32 hl = l - 1;
    auto set = [&](std::vector<ckks_ct> &v, u32 level, double scale) {
        for (auto &x : v) x.level = level, x.scale = scale;
    };
    set(h, hl, hs);
    for (u32 k = d - 1; k >= 1; k--) {
        if (!g->dry && k != k_first) {
            std::vector<i64> v(B, round_half_away(n.coeffs[k] * hs));
            GK(ckks_add_scalar(g->c, h.data(), v.data(), h.data(), B, scratch(g), scratch_avail(g), g->stream));
        }
        std::vector<ckks_ct> xs = in;
        for (auto &x : xs) x.level = hl;  // switch down: a view
        const double ps = s_x * hs;
        if (!g->dry) {
            const std::vector<const u64 *> keys(B, g->rk);
            GK(ckks_hmult_relin_rescale(g->c, keys.data(), xs.data(), h.data(), t.data(), B, scratch(g),
                                        scratch_avail(g), g->stream));
        }
        hs = ps / (double)ckks_ctx_prime(g->c, hl);
        hl -= 1;
        std::swap(h, t);
        set(h, hl, hs);
        set(t, hl, hs);
    }
    if (!g->dry && d >= 2) {
        std::vector<i64> v(B, round_half_away(n.coeffs[0] * hs));
        GK(ckks_add_scalar(g->c, h.data(), v.data(), h.data(), B, scratch(g), scratch_avail(g), g->stream));
    }
    n.out_level = hl;
    n.out_scale = hs;
    n.in_lvl_used = l;
    n.out = h;
    return CKKS_OK;
}

// acc = sum_i diag_i (x) rot(x, in_steps[i]); rescale; acc += rot(acc, r)
// for r in post_steps; acc += bias
int fire_diag(ckks_graph *g, Node &n, std::vector<ckks_ct> in) {
    GK(match_levels(in));
    const u32 B = (u32)in.size(), l = in[0].level, L = l + 1, nd = (u32)n.in_steps.size();
    if (l == 0) return gfail(CKKS_EDEPTH, "graph: no level left for a diagonal dense node");
    n.out_count = B;
    n.out_level = l - 1;
    n.in_lvl_used = l;
    const double s_prod = in[0].scale * n.pt_scale;
    n.out_scale = s_prod / (double)ckks_ctx_prime(g->c, l);
    // node region: acc (the output), rot tmp x2, product, plaintexts
    const size_t cb = ct_bytes(g, l);
    std::vector<ckks_ct> acc = make_cts(g, n.out_off, B, l, L, s_prod);
    std::vector<ckks_ct> rot = make_cts(g, n.out_off + al(B * cb), B, l, L, in[0].scale);
    std::vector<ckks_ct> tmp = make_cts(g, n.out_off + 2 * al(B * cb), B, l, L, in[0].scale);
    std::vector<ckks_ct> prod = make_cts(g, n.out_off + 3 * al(B * cb), B, l, L, s_prod);
    const size_t limb = (size_t)g->N * 8;
    n.pt_off = n.out_off + 4 * al(B * cb);
    need(g, ckks_workspace_bytes(g->c, CKKS_OP_ELEMENTWISE, B, nullptr));
    need(g, ckks_workspace_bytes(g->c, CKKS_OP_RESCALE, B, nullptr));
    need(g, ckks_workspace_bytes(g->c, CKKS_OP_NTT, L, nullptr) + al(limb));
    if (n.hoisted) {
        // one hoisted call: every diagonal's rotation shares the decomposition of x
        need(g, al((size_t)nd * limb) + ckks_hoisted_linear_workspace_bytes(g->c, B, l, nd));
        if (!g->dry) {
            std::vector<u32> elts(nd);
            std::vector<const u64 *> keys(nd, nullptr);
            const i64 half = g->N / 2;
            for (u32 i = 0; i < nd; i++) {
                const i64 st = ((n.in_steps[i] % half) + half) % half;
                elts[i] = st == 0 ? 1u : ckks_galois_elt(g->c, (int32_t)st);
                if (st != 0) {
                    auto it = g->gk.find(elts[i]);
                    if (it == g->gk.end()) return gfail(CKKS_ENOKEY, "graph: hoisted rotation needs its own key");
                    keys[i] = it->second;
                }
            }
            void *coef = nullptr;
            GK(ckks::ctx_upload_bytes(g->c, scratch(g), n.diag.data(), (size_t)nd * limb, g->stream, &coef));
            GK(ckks_hoisted_linear(g->c, in.data(), acc.data(), B, nd, elts.data(), keys.data(),
                                   (const int64_t *)coef, n.pt_scale, scratch(g) + al((size_t)nd * limb),
                                   scratch_avail(g) - al((size_t)nd * limb), g->stream));
            GK(ckks_rescale(g->c, acc.data(), acc.data(), B, scratch(g), scratch_avail(g), g->stream));
        }
    } else if (!g->dry) {
        // plaintexts: integer coefficients -> NTT form at level l (diagonals)
        for (u32 i = 0; i < nd; i++) {
            void *coef = nullptr;
            u64 *pt = (u64 *)(g->ws + n.pt_off + (size_t)i * L * limb);
            GK(ckks::ctx_upload_bytes(g->c, scratch(g), n.diag.data() + (size_t)i * g->N, limb, g->stream, &coef));
            ckks_pt p{pt, l, 0, n.pt_scale};
            GK(ckks_pt_load(g->c, (const int64_t *)coef, &p, scratch(g) + al(limb), scratch_avail(g) - al(limb),
                            g->stream));
        }
    }
    for (u32 i = 0; i < nd && !n.hoisted; i++) {
        const std::vector<ckks_ct> *src = &in;
        if (n.in_steps[i] != 0) {
            GK(rotate_all(g, in, rot, tmp, n.in_steps[i]));
            src = &rot;
        }
        if (g->dry) continue;
        std::vector<ckks_pt> pts(B);
        for (u32 b = 0; b < B; b++)
            pts[b] = ckks_pt{(u64 *)(g->ws + n.pt_off + (size_t)i * L * limb), l, 0, n.pt_scale};
        std::vector<ckks_ct> &dst = (i == 0) ? acc : prod;
        GK(ckks_multiply_plain(g->c, src->data(), pts.data(), dst.data(), B, scratch(g), scratch_avail(g),
                               g->stream));
        if (i > 0)
            GK(ckks_add(g->c, acc.data(), prod.data(), acc.data(), B, scratch(g), scratch_avail(g), g->stream));
    }
    if (!g->dry && !n.hoisted) GK(ckks_rescale(g->c, acc.data(), acc.data(), B, scratch(g), scratch_avail(g), g->stream));
    for (auto &x : acc) x.level = l - 1, x.scale = n.out_scale;
    for (auto &x : rot) x.level = l - 1, x.scale = n.out_scale;
    for (auto &x : tmp) x.level = l - 1, x.scale = n.out_scale;
    for (int32_t r : n.post_steps) {
        GK(rotate_all(g, acc, rot, tmp, r));
        if (!g->dry)
            GK(ckks_add(g->c, acc.data(), rot.data(), acc.data(), B, scratch(g), scratch_avail(g), g->stream));
    }
    const bool has_bias = !n.bias_slots.empty() || !n.bias_coeffs.empty();
    if (has_bias && n.bias_coeffs.empty() && g->dry) {
        n.bias_coeffs.assign(g->N, 0);
        GK(ckks_encode(g->c, n.bias_slots.data(), nullptr, n.bias_slots.size(), n.out_scale, n.bias_coeffs.data()));
    }
    if (has_bias && !g->dry) {
        void *coef = nullptr;
        u64 *pt = (u64 *)(g->ws + n.pt_off + (size_t)nd * L * limb);
        GK(ckks::ctx_upload_bytes(g->c, scratch(g), n.bias_coeffs.data(), limb, g->stream, &coef));
        ckks_pt p{pt, l - 1, 0, n.out_scale};
        GK(ckks_pt_load(g->c, (const int64_t *)coef, &p, scratch(g) + al(limb), scratch_avail(g) - al(limb),
                        g->stream));
        std::vector<ckks_pt> pts(B, p);
        GK(ckks_add_plain(g->c, acc.data(), pts.data(), acc.data(), B, scratch(g), scratch_avail(g), g->stream));
    }
    n.out = acc;
    return CKKS_OK;
}

size_t node_region(ckks_graph *g, const Node &n, u32 in_count, u32 in_level) {
    switch (n.kind) {
        case CKKS_NODE_LINEAR: return al((size_t)n.n_out * ct_bytes(g, in_level));
        case CKKS_NODE_SQUARE: return al((size_t)in_count * ct_bytes(g, in_level ? in_level - 1 : 0));
        case CKKS_NODE_POLY: return 2 * al((size_t)in_count * ct_bytes(g, in_level));
        case CKKS_NODE_DIAG_DENSE:
            return 4 * al((size_t)in_count * ct_bytes(g, in_level)) +
                   al(((size_t)n.in_steps.size() + 1) * (in_level + 1) * g->N * 8);
    }
    return 0;
}

// ------------------------------------------------------------------
// Algorithms 1-5
// ------------------------------------------------------------------
// get_inbound_signal: the bootstrap signal if given, else the in-edge
// signals stacked in edge order; nothing until every in-edge carries one
bool get_inbound(ckks_graph *g, u32 id, const std::vector<ckks_ct> *boot, std::vector<ckks_ct> &s) {
    if (boot) {
        s = *boot;
        return true;
    }
    s.clear();
    for (u32 e : g->nodes[id].in_edges) {
        if (!g->edges[e].has) return false;
        s.insert(s.end(), g->edges[e].sig.begin(), g->edges[e].sig.end());
    }
    return !g->nodes[id].in_edges.empty();
}

// apply_signal: the node's forward receptor
int apply_signal(ckks_graph *g, u32 id, std::vector<ckks_ct> &s) {
    Node &n = g->nodes[id];
    if (g->dry) {
        u32 lv = s.empty() ? 0 : s[0].level;
        for (auto &x : s) lv = std::min(lv, x.level);
        n.out_off = g->scratch_off;  // provisional; fixed below
        g->scratch_off += node_region(g, n, (u32)s.size(), lv);
        n.out_off = g->scratch_off - node_region(g, n, (u32)s.size(), lv);
    }
    int rc = CKKS_OK;
    switch (n.kind) {
        case CKKS_NODE_INPUT:
        case CKKS_NODE_OUTPUT:
            n.out = s;
            n.out_count = (u32)s.size();
            break;
        case CKKS_NODE_LINEAR: rc = fire_linear(g, n, s); break;
        case CKKS_NODE_SQUARE: rc = fire_square(g, n, s); break;
        case CKKS_NODE_DIAG_DENSE: rc = fire_diag(g, n, s); break;
        case CKKS_NODE_POLY: rc = fire_poly(g, n, s); break;
        default: rc = gfail(CKKS_EINVAL, "graph: unknown node kind");
    }
    if (rc != CKKS_OK) return rc;
    s = n.out;
    return CKKS_OK;
}

// set_outbound_signals: broadcast the result to every out-edge
void set_outbound(ckks_graph *g, u32 id, const std::vector<ckks_ct> &s) {
    for (u32 e : g->nodes[id].out_edges) {
        g->edges[e].sig = s;
        g->edges[e].has = true;
    }
}

int signal_carrier(ckks_graph *g, u32 id, const std::vector<ckks_ct> *boot) {
    std::vector<ckks_ct> s;
    if (g->nodes[id].fired) return CKKS_OK;
    if (!get_inbound(g, id, boot, s)) return CKKS_OK;
    GK(apply_signal(g, id, s));
    g->nodes[id].fired = true;
    set_outbound(g, id, s);
    std::vector<u32> succ;
    for (u32 e : g->nodes[id].out_edges) {
        u32 t = g->edges[e].to;
        if (std::find(succ.begin(), succ.end(), t) == succ.end()) succ.push_back(t);
    }
    for (u32 t : succ) GK(signal_carrier(g, t, nullptr));
    return CKKS_OK;
}

// neuronal_firing: stimulate every input node with its signal
int neuronal_firing(ckks_graph *g, const std::vector<std::vector<ckks_ct>> &inputs) {
    for (auto &n : g->nodes) n.fired = false;
    for (auto &e : g->edges) e.has = false, e.sig.clear();
    u32 k = 0;
    for (u32 id = 0; id < g->nodes.size(); id++)
        if (g->nodes[id].kind == CKKS_NODE_INPUT) GK(signal_carrier(g, id, &inputs[k++]));
    return CKKS_OK;
}
}  // namespace

// ------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------
extern "C" int ckks_graph_create(const ckks_ctx *c, ckks_graph **out) {
    if (!c || !out) return gfail(CKKS_EINVAL, "graph_create: null argument");
    ckks_graph *g = new ckks_graph();
    g->c = c;
    g->N = 1u << ckks_ctx_log_n(c);
    *out = g;
    return CKKS_OK;
}

extern "C" void ckks_graph_destroy(ckks_graph *g) { delete g; }

extern "C" int ckks_graph_add_node(ckks_graph *g, int kind, const void *attrs, uint32_t *id) {
    if (!g || !id) return gfail(CKKS_EINVAL, "graph_add_node: null argument");
    Node n;
    n.kind = kind;
    switch (kind) {
        case CKKS_NODE_INPUT: {
            const ckks_input_attrs *a = (const ckks_input_attrs *)attrs;
            if (!a || !a->n_ct) return gfail(CKKS_EINVAL, "graph_add_node: input needs attrs");
            n.in_count = a->n_ct;
            n.in_level = a->level;
            n.in_scale = a->scale;
            break;
        }
        case CKKS_NODE_LINEAR: {
            const ckks_linear_attrs *a = (const ckks_linear_attrs *)attrs;
            if (!a || !a->n_out || !a->row_ptr || !a->col || !a->w) return gfail(CKKS_EINVAL, "graph: linear attrs");
            n.n_out = a->n_out;
            n.row_ptr.assign(a->row_ptr, a->row_ptr + a->n_out + 1);
            const u32 nnz = a->row_ptr[a->n_out];
            n.col.assign(a->col, a->col + nnz);
            n.w_scale = a->w_scale;
            n.w.resize(nnz);
            for (u32 e = 0; e < nnz; e++) n.w[e] = round_half_away(a->w[e] * a->w_scale);
            if (a->bias) n.bias.assign(a->bias, a->bias + a->n_out);
            break;
        }
        case CKKS_NODE_DIAG_DENSE: {
            const ckks_diag_attrs *a = (const ckks_diag_attrs *)attrs;
            if (!a || !a->n_diag || !a->in_steps || !a->diag_coeffs) return gfail(CKKS_EINVAL, "graph: diag attrs");
            n.in_steps.assign(a->in_steps, a->in_steps + a->n_diag);
            n.diag.assign(a->diag_coeffs, a->diag_coeffs + (size_t)a->n_diag * g->N);
            n.pt_scale = a->pt_scale;
            if (a->n_post) n.post_steps.assign(a->post_steps, a->post_steps + a->n_post);
            n.hoisted = a->hoisted != 0;
            if (a->bias_coeffs) n.bias_coeffs.assign(a->bias_coeffs, a->bias_coeffs + g->N);
            else if (a->bias_slots) n.bias_slots.assign(a->bias_slots, a->bias_slots + a->n_bias_slots);
            break;
        }
        case CKKS_NODE_POLY: {
            const ckks_poly_attrs *a = (const ckks_poly_attrs *)attrs;
            if (!a || a->degree < 1 || !a->coeffs || !(a->w_scale > 0)) return gfail(CKKS_EINVAL, "graph: poly attrs");
            n.coeffs.assign(a->coeffs, a->coeffs + a->degree + 1);
            n.w_scale = a->w_scale;
            break;
        }
        case CKKS_NODE_SQUARE:
        case CKKS_NODE_OUTPUT: break;
        default: return gfail(CKKS_EINVAL, "graph_add_node: unknown kind");
    }
    g->nodes.push_back(n);
    g->planned = false;
    *id = (u32)g->nodes.size() - 1;
    return CKKS_OK;
}

extern "C" int ckks_graph_add_edge(ckks_graph *g, uint32_t from, uint32_t to) {
    if (!g || from >= g->nodes.size() || to >= g->nodes.size()) return gfail(CKKS_EINVAL, "graph_add_edge: bad node");
    if (g->nodes[to].kind == CKKS_NODE_INPUT) return gfail(CKKS_EINVAL, "graph_add_edge: input nodes take no edges");
    g->edges.push_back(Edge{from, to});
    g->nodes[from].out_edges.push_back((u32)g->edges.size() - 1);
    g->nodes[to].in_edges.push_back((u32)g->edges.size() - 1);
    g->planned = false;
    return CKKS_OK;
}

static std::vector<std::vector<ckks_ct>> split_inputs(ckks_graph *g, const ckks_ct *inputs) {
    std::vector<std::vector<ckks_ct>> v;
    size_t k = 0;
    for (auto &n : g->nodes)
        if (n.kind == CKKS_NODE_INPUT) {
            std::vector<ckks_ct> s(n.in_count);
            for (u32 i = 0; i < n.in_count; i++) {
                if (inputs) {
                    s[i] = inputs[k++];
                } else {
                    s[i] = ckks_ct{nullptr, 2, n.in_level, n.in_level + 1, 0, n.in_scale};
                }
            }
            v.push_back(s);
        }
    return v;
}

extern "C" int ckks_graph_plan(ckks_graph *g, size_t *ws_bytes, uint32_t *n_outputs) {
    if (!g || !ws_bytes) return gfail(CKKS_EINVAL, "graph_plan: null argument");
    g->dry = true;
    g->scratch_off = 0;
    g->scratch_bytes = 0;
    int rc = neuronal_firing(g, split_inputs(g, nullptr));
    if (rc != CKKS_OK) return rc;
    u32 nout = 0;
    for (auto &n : g->nodes) {
        if (n.kind == CKKS_NODE_OUTPUT) {
            if (!n.fired) return gfail(CKKS_EINVAL, "graph_plan: an output node is unreachable");
            nout += n.out_count;
        }
    }
    g->scratch_off = al(g->scratch_off);
    g->ws_total = g->scratch_off + al(g->scratch_bytes) + 4096;
    g->planned = true;
    *ws_bytes = g->ws_total;
    if (n_outputs) *n_outputs = nout;
    return CKKS_OK;
}

extern "C" int ckks_graph_run(ckks_graph *g, const ckks_ct *inputs, uint32_t n_inputs, ckks_ct *outputs,
                              uint32_t n_outputs, const uint64_t *rk, const uint32_t *galois_elts,
                              const uint64_t *const *galois_keys, uint32_t n_galois, void *ws, size_t ws_bytes,
                              void *stream) {
    if (!g || !inputs || !outputs) return gfail(CKKS_EINVAL, "graph_run: null argument");
    if (!g->planned) return gfail(CKKS_EINVAL, "graph_run: call ckks_graph_plan first");
    if (ws_bytes < g->ws_total || !ws) return gfail(CKKS_ENOMEM, "graph_run: workspace smaller than planned");
    u32 expect_in = 0;
    for (auto &n : g->nodes)
        if (n.kind == CKKS_NODE_INPUT) expect_in += n.in_count;
    if (n_inputs != expect_in) return gfail(CKKS_EINVAL, "graph_run: input count differs from the input nodes");
    size_t k = 0;
    for (auto &n : g->nodes)
        if (n.kind == CKKS_NODE_INPUT)
            for (u32 i = 0; i < n.in_count; i++, k++)
                if (inputs[k].level != n.in_level || inputs[k].scale != n.in_scale)
                    return gfail(CKKS_ELEVEL, "graph_run: input level/scale differs from the plan");
    g->dry = false;
    g->ws = (uint8_t *)ws;
    g->stream = stream;
    g->rk = rk;
    g->gk.clear();
    for (u32 i = 0; i < n_galois; i++) g->gk[galois_elts[i]] = galois_keys[i];
    const size_t planned_off = g->scratch_off;
    // node regions keep the planned offsets; scratch follows them
    int rc = neuronal_firing(g, split_inputs(g, inputs));
    g->scratch_off = planned_off;
    if (rc != CKKS_OK) return rc;
    u32 o = 0;
    for (auto &n : g->nodes)
        if (n.kind == CKKS_NODE_OUTPUT)
            for (auto &x : n.out) {
                if (o >= n_outputs) return gfail(CKKS_EINVAL, "graph_run: output array too small");
                outputs[o++] = x;
            }
    return CKKS_OK;
}

// ------------------------------------------------------------------
// Algorithms 6-7: automatic parameterisation groups
// ------------------------------------------------------------------
// The cost of a node is the multiplicative depth it consumes (one for
// linear, diagonal and square nodes, none for input and output nodes); an
// edge costs what its destination costs. autoHE_discover labels every node
// with, per source, the largest cost accumulated on any path from that
// source; at a concern node (an output, where ciphertexts leave the graph)
// the traversal restarts with the node as a new source. autoHE then merges
// sources that meet at a common node into one group whose cost is the
// largest label any of its sources reached.
namespace {
u32 node_cost(const Node &n) {
    // a polynomial activation of degree d consumes d levels (Horner's rule)
    if (n.kind == CKKS_NODE_POLY) return n.coeffs.empty() ? 0u : (u32)(n.coeffs.size() - 1);
    return (n.kind == CKKS_NODE_LINEAR || n.kind == CKKS_NODE_DIAG_DENSE || n.kind == CKKS_NODE_SQUARE) ? 1u : 0u;
}

void autohe_discover(ckks_graph *g, std::vector<std::map<u32, u32>> &sources, u32 n, u32 src, u32 cost,
                     std::vector<char> &restarted) {
    if (src != n) {
        auto it = sources[n].find(src);
        if (it == sources[n].end() || it->second < cost) sources[n][src] = cost;
        else return;  // an equal or longer path from this source was already propagated
    }
    const Node &node = g->nodes[n];
    if (node.kind == CKKS_NODE_OUTPUT && src != n) {
        // concern: restart from this node as a new source (reading of the
        // printed recursion, which would otherwise call itself unchanged)
        if (!restarted[n]) {
            restarted[n] = 1;
            autohe_discover(g, sources, n, n, 0, restarted);
        }
        return;
    }
    std::vector<u32> succ;
    for (u32 e : node.out_edges) {
        u32 t = g->edges[e].to;
        if (std::find(succ.begin(), succ.end(), t) == succ.end()) succ.push_back(t);
    }
    for (u32 t : succ) autohe_discover(g, sources, t, src, cost + node_cost(g->nodes[t]), restarted);
}
}  // namespace

extern "C" int ckks_graph_autohe(ckks_graph *g, uint32_t *n_groups, uint32_t *group_of_node,
                                 uint32_t *group_cost, uint32_t cap) {
    if (!g || !n_groups) return gfail(CKKS_EINVAL, "graph_autohe: null argument");
    const u32 n = (u32)g->nodes.size();
    std::vector<std::map<u32, u32>> sources(n);
    std::vector<char> restarted(n, 0);
    std::vector<u32> inputs;
    for (u32 i = 0; i < n; i++)
        if (g->nodes[i].kind == CKKS_NODE_INPUT) inputs.push_back(i);
    for (u32 i : inputs) autohe_discover(g, sources, i, i, 0, restarted);
    // group assignment and merging (union of sources meeting at a node)
    std::vector<int> group(n, -1);
    std::vector<u32> cost;
    std::vector<u32> all_src = inputs;
    for (u32 i = 0; i < n; i++)
        if (restarted[i]) all_src.push_back(i);
    for (u32 i : all_src) {
        if (group[i] < 0) {
            group[i] = (int)cost.size();
            cost.push_back(0);
        }
        for (u32 j = 0; j < n; j++) {
            const auto &src = sources[j];
            if (!src.count(i)) continue;
            const int gi = group[i];
            for (auto &kv : src) {
                const int old = group[kv.first];
                if (old >= 0 && old != gi) {
                    // merge the old group into gi
                    for (u32 x = 0; x < n; x++)
                        if (group[x] == old) group[x] = gi;
                    cost[gi] = std::max(cost[gi], cost[old]);
                }
                group[kv.first] = gi;
                cost[gi] = std::max(cost[gi], kv.second);
            }
        }
    }
    // every other node joins the group of the sources that reach it
    for (u32 j = 0; j < n; j++)
        if (group[j] < 0 && !sources[j].empty()) group[j] = group[sources[j].begin()->first];
    // compact group ids
    std::map<int, u32> ids;
    for (u32 i : all_src) ids.emplace(group[i], 0);
    u32 k = 0;
    for (auto &kv : ids) kv.second = k++;
    *n_groups = k;
    if (group_of_node || group_cost) {
        for (u32 i = 0; i < n && i < cap; i++)
            if (group_of_node) group_of_node[i] = group[i] >= 0 ? ids[group[i]] : 0xFFFFFFFFu;
        if (group_cost)
            for (auto &kv : ids)
                if (kv.second < cap) group_cost[kv.second] = cost[kv.first];
    }
    return CKKS_OK;
}
