// Drives the host side of libckks_hip (parameter checks, prime search,
// context tables, encoder / decoder, constant encoding, workspace sizing
// of every operation, the graph planner and Algorithms 6-8, and the error
// paths of the device entry points, which return before any launch) in an
// AddressSanitizer / UndefinedBehaviorSanitizer build. Nothing here
// touches a GPU: the kernel launchers are stand-ins that are never reached.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/ckks.h"
#include "../../paper_2110_13638_amd/csrc/ckks_internal.h"

namespace ckks {
#define STUB(...) { fprintf(stderr, "a kernel launcher was reached\n"); abort(); }
hipError_t launch_fwd(const DevTables &, int, const Item *, int, u64, hipStream_t) STUB()
hipError_t launch_inv(const DevTables &, int, const Item *, int, hipStream_t) STUB()
hipError_t launch_ew(const DevTables &, const EwItem *, int, u64, hipStream_t) STUB()
hipError_t launch_ip(const DevTables &, const IpItem *, int, hipStream_t) STUB()
hipError_t launch_hoist(const DevTables &, int, const HoItem *, int, hipStream_t) STUB()
hipError_t launch_ip_seq(const DevTables &, const IpSeqItem *, int, hipStream_t) STUB()
hipError_t launch_linear(const DevTables &, const u64 *const *, const u64 *, u64 *const *, u32, u32, u32, u32, u32,
                         hipStream_t) STUB()
hipError_t launch_reduce_weights(const DevTables &, const i64 *, u64 *, u32, u32, hipStream_t) STUB()
hipError_t launch_linear_mfma(const DevTables &, const int8_t *, u32, u32, const u32 *, u32, u32, const u64 *const *,
                              u64 *const *, u32, u32, bool, u32, u32, hipStream_t) STUB()
hipError_t launch_weight_digits(const i64 *, u32, u32, u32, u32, int8_t *, hipStream_t) STUB()
hipError_t launch_linear_grouped(const DevTables &, const LinGroup *, u32, const u32 *, const u64 *, const double2 *,
                                 u32, const u64 *const *, u64 *const *, u32, u32, u32, u32, hipStream_t) STUB()
}  // namespace ckks

#define CHECK(cond)                                                             \
    do {                                                                        \
        if (!(cond)) {                                                          \
            fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #cond, ckks_last_error()); \
            exit(1);                                                            \
        }                                                                       \
    } while (0)

static void chain(uint32_t log_n, std::vector<uint32_t> bits, uint32_t n_p, uint32_t dnum) {
    std::vector<uint64_t> pr(bits.size());
    CHECK(ckks_find_primes(log_n, bits.data(), (uint32_t)bits.size(), pr.data()) == CKKS_OK);
    const uint32_t n_q = (uint32_t)bits.size() - n_p, N = 1u << log_n;
    ckks_params prm{log_n, n_q, pr.data(), n_p, pr.data() + n_q, dnum};
    ckks_ctx *c = nullptr;
    CHECK(ckks_ctx_create(&prm, &c) == CKKS_OK);
    CHECK(ckks_ctx_device_bytes(c) > 0);
    // encoder / decoder round trip on the host
    std::vector<double> re(N / 2), im(N / 2), ro(N / 2), io(N / 2);
    for (uint32_t j = 0; j < N / 2; j++) re[j] = sin(0.1 * j), im[j] = cos(0.3 * j);
    std::vector<int64_t> co(N);
    CHECK(ckks_encode(c, re.data(), im.data(), N / 2, ldexp(1.0, 30), co.data()) == CKKS_OK);
    const uint32_t L = n_q;
    std::vector<uint64_t> res((size_t)L * N);
    for (uint32_t i = 0; i < L; i++)
        for (uint32_t j = 0; j < N; j++) {
            const int64_t v = co[j];
            const uint64_t q = pr[i];
            res[(size_t)i * N + j] = v >= 0 ? (uint64_t)v % q : q - (uint64_t)(-v) % q;
        }
    CHECK(ckks_decode(c, res.data(), L - 1, ldexp(1.0, 30), ro.data(), io.data(), N / 2) == CKKS_OK);
    for (uint32_t j = 0; j < N / 2; j++) CHECK(fabs(ro[j] - re[j]) < 1e-6 && fabs(io[j] - im[j]) < 1e-6);
    // constants
    std::vector<double> vals = {0.5, -1.25, 3e-9, 0.0};
    std::vector<int64_t> iv(vals.size());
    CHECK(ckks_encode_scalars(c, vals.data(), vals.size(), ldexp(1.0, 40), iv.data()) == CKKS_OK);
    std::vector<uint64_t> per(L);
    CHECK(ckks_encode_scalar(c, -0.75, ldexp(1.0, 40), L - 1, per.data()) == CKKS_OK);
    CHECK(ckks_encode_scalar(c, -0.75, ldexp(1.0, 40), L + 3, per.data()) == CKKS_ELEVEL);
    double huge = 1e30;
    CHECK(ckks_encode_scalars(c, &huge, 1, ldexp(1.0, 40), iv.data()) == CKKS_EINVAL);
    for (int32_t st : {1, -1, 7, (int32_t)N / 2 - 1}) CHECK(ckks_galois_elt(c, st) % 2 == 1);
    // workspace sizing of every operation, ragged levels
    std::vector<uint32_t> lv;
    for (uint32_t b = 0; b < 9; b++) lv.push_back(1 + b % (L - 1));
    for (int op = CKKS_OP_NTT; op <= CKKS_OP_ENCRYPT; op++)
        CHECK(ckks_workspace_bytes(c, op, (uint32_t)lv.size(), lv.data()) > 0);
    uint32_t lin[2] = {L - 1, 40};
    CHECK(ckks_workspace_bytes(c, CKKS_OP_LINEAR, 7, lin) > 0);
    CHECK(ckks_linear_csr_workspace_bytes(c, 40, 7, 280, L - 1) > 0);
    CHECK(ckks_hoisted_linear_workspace_bytes(c, 3, L - 1, 5) > 0);
    // device entry points refuse a context whose tables were never uploaded
    ckks_ct a{nullptr, 2, L - 1, L, 0, 1.0};
    const uint64_t *rk = nullptr;
    CHECK(ckks_hmult_relin_rescale(c, &rk, &a, &a, &a, 1, nullptr, 0, nullptr) == CKKS_EINVAL);
    CHECK(ckks_hmult_relin_rescale_noalloc(nullptr, &rk, &a, &a, &a, 1, nullptr) == CKKS_EINVAL);
    // graph: input -> linear -> square -> poly -> output, planned, and Algorithms 6-7
    ckks_graph *g = nullptr;
    CHECK(ckks_graph_create(c, &g) == CKKS_OK);
    ckks_input_attrs ia{4, L - 1, ldexp(1.0, 30)};
    uint32_t n_in, n_lin, n_sq, n_poly, n_out;
    CHECK(ckks_graph_add_node(g, CKKS_NODE_INPUT, &ia, &n_in) == CKKS_OK);
    std::vector<uint32_t> rp = {0, 3, 5}, col = {0, 1, 3, 2, 2};
    std::vector<double> w = {0.1, -0.2, 0.3, 0.05, 0.7}, bias = {0.01, -0.02};
    ckks_linear_attrs la{2, rp.data(), col.data(), w.data(), ldexp(1.0, 30), bias.data()};
    CHECK(ckks_graph_add_node(g, CKKS_NODE_LINEAR, &la, &n_lin) == CKKS_OK);
    CHECK(ckks_graph_add_node(g, CKKS_NODE_SQUARE, nullptr, &n_sq) == CKKS_OK);
    std::vector<double> pc = {0.5, 0.197, 0.0, -0.004};
    ckks_poly_attrs pa{3, pc.data(), ldexp(1.0, 30)};
    CHECK(ckks_graph_add_node(g, CKKS_NODE_POLY, &pa, &n_poly) == CKKS_OK);
    CHECK(ckks_graph_add_node(g, CKKS_NODE_OUTPUT, nullptr, &n_out) == CKKS_OK);
    CHECK(ckks_graph_add_edge(g, n_in, n_lin) == CKKS_OK);
    CHECK(ckks_graph_add_edge(g, n_lin, n_sq) == CKKS_OK);
    CHECK(ckks_graph_add_edge(g, n_sq, n_poly) == CKKS_OK);
    CHECK(ckks_graph_add_edge(g, n_poly, n_out) == CKKS_OK);
    CHECK(ckks_graph_add_edge(g, n_out, 99) != CKKS_OK);
    size_t ws = 0;
    uint32_t outs = 0;
    const int plan = ckks_graph_plan(g, &ws, &outs);
    CHECK(plan == CKKS_OK || plan == CKKS_EDEPTH);
    uint32_t ng = 0, grp[8], cost[8];
    CHECK(ckks_graph_autohe(g, &ng, grp, cost, 8) == CKKS_OK);
    // the output is a concern node: its own group; the rest costs linear 1 + square 1 + poly 3
    CHECK(ng == 2 && grp[n_in] == grp[n_lin] && grp[n_lin] == grp[n_poly] && grp[n_out] != grp[n_in]);
    CHECK(cost[grp[n_in]] == 5);
    ckks_graph_destroy(g);
    ckks_ctx_destroy(c);
}

int main() {
    // Algorithm 8 for every cost up to 9
    for (uint32_t cost = 0; cost < 10; cost++) {
        uint32_t bits[16], nb = 0, ln = 0;
        CHECK(ckks_parameterise(cost, 40, 1.5, bits, 16, &nb, &ln) == CKKS_OK);
        CHECK(nb == cost + 2);
    }
    uint32_t bits[4];
    uint32_t nb, ln;
    CHECK(ckks_parameterise(5, 40, 1.5, bits, 4, &nb, &ln) != CKKS_OK);  // output too small
    ckks_params bad{16, 0, nullptr, 0, nullptr, 1};
    ckks_ctx *c = nullptr;
    CHECK(ckks_ctx_create(&bad, &c) != CKKS_OK && c == nullptr);
    chain(12, {60, 40, 40, 40, 60}, 1, 4);
    chain(11, {50, 50, 50, 50, 50, 60, 60}, 2, 2);
    chain(10, {60, 40, 60}, 1, 2);
    chain(16, {50, 50, 60}, 1, 2);
    printf("host driver ok\n");
    return 0;
}
