// gfx950 kernels for RNS-CKKS ciphertext arithmetic: element-wise ops,
// the key-switch inner product, hoisted rotations, linear layers, and the
// launch dispatch to the per-ring NTT translation units (ckks_ntt_*.hip).
// Modular arithmetic and the NTT engine are in ckks_device.h.
#include "ckks_device.h"

namespace ckks {
// ---------------------------------------------------------------------
// elementwise kernels (grid-stride over items x N/2 pairs of residues)
// ---------------------------------------------------------------------
enum EwOp : u32 {
    EW_ADD = 0,
    EW_SUB = 1,
    EW_MUL = 2,        // y0 = x0 * x1
    EW_MUL_CONST = 3,  // y0 = x0 * v
    EW_ADD_CONST = 4,  // y0 = x0 + v
    EW_TENSOR = 5,     // y0 = x0 x2, y1 = x0 x3 + x1 x2, y2 = x1 x3
    EW_COPY = 6,       // y0 = x0
    EW_AUTOMORPH = 7,  // y0[k] = x0[perm_g(k)] with g = v (NTT domain)
    EW_NEG = 8,
    EW_KEYGEN = 9,     // y0 = -a s + x0 (+ P s' when x2), y1 = a; a sampled uniform
    EW_ENCRYPT = 10,   // y0 = x0 x3 + x1 + x5, y1 = x0 x4 + x2 (v, e0, e1, b, a, m)
    EW_SQUARE_S = 11,  // y0 = x0^2
    // HMult rescale of limb i < l = v, both polys: y_c = (x_{2+c} P^-1 -
    // x_c) q_l^-1 with z_c (x0, x1) and the accumulators acc'_c (x2, x3)
    EW_HMULT_FIN = 12,
    // relinearised top limb in the coefficient domain: y0 = u - conv_l(y) P^-1
    // with u (x0) the INTT'd top limb and y (x1, n_p limbs) the INTT'd
    // special-prime accumulator times hat_m^-1
    EW_HMULT_T = 14,
};

__device__ __forceinline__ u32 brev_n(u32 x, u32 log_n) { return __brev(x) >> (32 - log_n); }

// One workgroup serves one descriptor over kEwPer * 256 consecutive residues,
// so the descriptor is read once per thread through wave-uniform loads.
template <int kEwPer>
__global__ void __launch_bounds__(256) k_ew(DevTables tb, const EwItem *__restrict__ items, int nitems,
                                            u64 seed) {
    const u32 N = 1u << tb.log_n;
    const u32 per_item = (N + 256 * kEwPer - 1) / (256 * kEwPer);
    const u32 iid = __builtin_amdgcn_readfirstlane(blockIdx.x / per_item);
    const u32 chunk = blockIdx.x - iid * per_item;
    if ((int)iid >= nitems) return;
    const EwItem it = items[iid];
    const PrimeConst pc = tb.pc[it.prime];
    const u64 q = pc.q;
#pragma unroll
    for (int e = 0; e < kEwPer; e++) {
        const u32 j = (chunk * kEwPer + e) * 256 + threadIdx.x;
        if (j >= N) break;
        switch (it.op) {
            case EW_ADD: it.y[0][j] = addm(it.x[0][j], it.x[1][j], q); break;
            case EW_SUB: it.y[0][j] = subm(it.x[0][j], it.x[1][j], q); break;
            case EW_MUL: it.y[0][j] = mulm(it.x[0][j], it.x[1][j], pc); break;
            case EW_MUL_CONST: it.y[0][j] = mulm(it.x[0][j], reduce_signed(it.v, pc), pc); break;
            case EW_ADD_CONST: it.y[0][j] = addm(it.x[0][j], reduce_signed(it.v, pc), q); break;
            case EW_TENSOR: {
                const u64 a0 = it.x[0][j], a1 = it.x[1][j], b0 = it.x[2][j], b1 = it.x[3][j];
                Acc128 t;
                t.mac(a0, b1);
                t.mac(a1, b0);
                const u64 d0 = mulm(a0, b0, pc), d1 = t.reduce(pc), d2 = mulm(a1, b1, pc);
                it.y[0][j] = d0;
                it.y[1][j] = d1;
                it.y[2][j] = d2;
                break;
            }
            case EW_COPY: it.y[0][j] = it.x[0][j]; break;
            case EW_AUTOMORPH: {
                const u32 two_n_mask = 2 * N - 1;
                const u32 e = 2 * brev_n(j, tb.log_n) + 1;
                const u32 eg = (u32)(((u64)e * (u64)it.v) & two_n_mask);
                const u32 src = brev_n((eg - 1) >> 1, tb.log_n);
                it.y[0][j] = it.x[0][src];
                break;
            }
            case EW_NEG: it.y[0][j] = subm(0, it.x[0][j], q); break;
            case EW_KEYGEN: {
                // a uniform in the NTT domain (limb = prime index), obj = v>>8 bits
                const u32 obj = (u32)(it.v & 0xFFFFFFFF), tag = (u32)(it.v >> 32);
                const u64 a = sample_uniform(j, it.prime, obj, tag, seed, pc);
                u64 b = addm(subm(0, mulm(a, it.x[1][j], pc), q), it.x[0][j], q);
                if (it.x[2]) b = addm(b, mulm(pc.pmod, it.x[2][j], pc), q);
                it.y[0][j] = b;
                it.y[1][j] = a;
                break;
            }
            case EW_ENCRYPT: {
                const u64 v = it.x[0][j];
                it.y[0][j] = addm(addm(mulm(v, it.x[3][j], pc), it.x[1][j], q), it.x[5][j], q);
                it.y[1][j] = addm(mulm(v, it.x[4][j], pc), it.x[2][j], q);
                break;
            }
            case EW_SQUARE_S: it.y[0][j] = mulm(it.x[0][j], it.x[0][j], pc); break;
            case EW_HMULT_FIN: {
                const ulonglong2 qi = tb.rescale[(size_t)it.v * tb.n_q + it.prime];
                const u64 u0 = shoup(it.x[2][j], pc.pinv, pc.pinv_sh, q);
                const u64 u1 = shoup(it.x[3][j], pc.pinv, pc.pinv_sh, q);
                it.y[0][j] = shoup(subm(u0, it.x[0][j], q), qi.x, qi.y, q);
                it.y[1][j] = shoup(subm(u1, it.x[1][j], q), qi.x, qi.y, q);
                break;
            }
            case EW_HMULT_T: {
                // x0: INTT'd top limb u; x1: y = INTT(acc_P) hat_m^-1 (n_p limbs)
                const u64 *hat = tb.moddown + 2 * tb.n_p + it.prime;
                Acc128 a;
                for (u32 m = 0; m < tb.n_p; m++) a.mac(it.x[1][(size_t)m * N + j], hat[(size_t)m * tb.n_q]);
                it.y[0][j] = subm(it.x[0][j], shoup(a.reduce(pc), pc.pinv, pc.pinv_sh, q), q);
                break;
            }
        }
    }
}

// Key-switch inner product over the extended basis: one item per target
// limb `pos` (prime `prime`) and up to kIpCts ciphertexts of one level. For
// each digit j < beta the ModUp'd limb (ext + (j E + pos) N), or for the digit
// that owns the target the input limb own0 (times own1 when given), is
// multiplied by the key limbs (b_j, a_j) of that prime; sums are 128-bit and
// reduced once. Each key residue is loaded once for all the item's
// ciphertexts. acc + pos N receives the b-sum, acc + (E + pos) N the a-sum.
// FP64 product of two residues below t < 2^50: x y - k t with k the integer
// nearest to fl(x y) (1/t), so |result| <= 0.75 t, exactly
__device__ __forceinline__ double fp_mulv(double x, double y, double t, double tinv) {
#pragma clang fp contract(off)
    const double h = x * y;
    const double l = __builtin_fma(x, y, -h);
    const double k = __builtin_fma(h, tinv, kRound) - kRound;
    return __builtin_fma(-k, t, h) + l;
}

// The inner product in FP64 for an item whose prime t is below 2^50: each
// digit term is an FP64 product (<= 0.75 t), sums are re-centred every four
// digits, the P d fold multiplies by P mod t (ratio P/t from 1/t, error
// <= 2^-52), and the final re-centred sum (|.| <= t/2 + 1) becomes a residue.
// Each thread takes kEwPer residues as pairs (16-byte loads and stores);
// the digit loop is unrolled for BETA digits (0: a runtime loop); FULL:
// the item holds NCT ciphertexts, so no per-ciphertext test separates the
// loads of one digit.
template <int kEwPer, int NCT, int BETA, bool FULL>
__device__ __forceinline__ void ip_fp_item(const DevTables &tb, const IpItem &it, u32 chunk) {
#pragma clang fp contract(off)
    const u32 N = 1u << tb.log_n;
    const PrimeConst pc = tb.pc[it.prime];
    const double t = pc.qf, tinv = pc.qinvf;
    const double pm = fp_from_u64(pc.pmod), pmq = pm * tinv;
    const size_t kstride = (size_t)tb.n_prim * N;  // one key component
    const u32 beta = BETA ? (u32)BETA : it.beta;
    auto ld2 = [](const u64 *p, u32 x, double (&v)[2]) {
        const ulonglong2 a = *reinterpret_cast<const ulonglong2 *>(p + x);
        v[0] = fp_from_u64(a.x);
        v[1] = fp_from_u64(a.y);
    };
#pragma unroll
    for (int e = 0; e < kEwPer / 2; e++) {
        const u32 x = 2 * ((chunk * (kEwPer / 2) + e) * 256 + threadIdx.x);
        if (x >= N) break;
        double s0[NCT][2], s1[NCT][2];
#pragma unroll
        for (int c = 0; c < NCT; c++) s0[c][0] = s0[c][1] = s1[c][0] = s1[c][1] = 0.0;
        auto digit = [&](u32 j) {
            const u64 *kb = it.key + (size_t)(2 * j) * kstride + (size_t)it.prime * N;
            double k0[2], k1[2];
            ld2(kb, x, k0);
            ld2(kb + kstride, x, k1);
#pragma unroll
            for (int c = 0; c < NCT; c++) {
                if (!FULL && (u32)c >= it.n_ct) break;
                double v[2];
                // the own digit's limb, else digit j's ModUp output (a select, not a branch)
                const bool own = j == it.own_digit;
                ld2(own ? it.own0[c] : it.ext[c] + ((size_t)j * it.E + it.pos) * N, x, v);
                if (own && it.own1[c]) {
                    double w[2];
                    ld2(it.own1[c], x, w);
                    v[0] = fp_mulv(v[0], w[0], t, tinv);
                    v[1] = fp_mulv(v[1], w[1], t, tinv);
                }
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    s0[c][h] = s0[c][h] + fp_mulv(v[h], k0[h], t, tinv);
                    s1[c][h] = s1[c][h] + fp_mulv(v[h], k1[h], t, tinv);
                    if ((j & 3) == 3) {
                        s0[c][h] = fp_center(s0[c][h], t, tinv);
                        s1[c][h] = fp_center(s1[c][h], t, tinv);
                    }
                }
            }
        };
        if constexpr (BETA > 0) {
#pragma unroll
            for (int j = 0; j < BETA; j++) digit((u32)j);
        } else {
            for (u32 j = 0; j < beta; j++) digit(j);
        }
#pragma unroll
        for (int c = 0; c < NCT; c++) {
            if (!FULL && (u32)c >= it.n_ct) break;
            double r0[2], r1[2];
#pragma unroll
            for (int h = 0; h < 2; h++) r0[h] = fp_center(s0[c][h], t, tinv), r1[h] = fp_center(s1[c][h], t, tinv);
            if (it.own2[c]) {
                double a0[2], b0[2], a1[2], b1[2];
                ld2(it.own2[c], x, a0);
                ld2(it.own3[c], x, b0);
                ld2(it.own0[c], x, a1);
                ld2(it.own1[c], x, b1);
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const double d0 = fp_mulv(a0[h], b0[h], t, tinv);
                    const double d1 = fp_mulv(a0[h], b1[h], t, tinv) + fp_mulv(a1[h], b0[h], t, tinv);
                    r0[h] = fp_center(r0[h] + fp_mulmod(d0, pm, pmq, t), t, tinv);
                    r1[h] = fp_center(r1[h] + fp_mulmod(d1, pm, pmq, t), t, tinv);
                }
            }
            *reinterpret_cast<ulonglong2 *>(it.acc[c] + (size_t)it.pos * N + x) =
                ulonglong2{fp_to_residue(r0[0], pc.qmf, pc.q), fp_to_residue(r0[1], pc.qmf, pc.q)};
            *reinterpret_cast<ulonglong2 *>(it.acc[c] + ((size_t)it.E + it.pos) * N + x) =
                ulonglong2{fp_to_residue(r1[0], pc.qmf, pc.q), fp_to_residue(r1[1], pc.qmf, pc.q)};
        }
    }
}
template <int kEwPer, int NCT>
__global__ void __launch_bounds__(256) k_ip_fp(DevTables tb, const IpItem *__restrict__ items, int nitems) {
    const u32 N = 1u << tb.log_n;
    const u32 per_item = (N + 256 * kEwPer - 1) / (256 * kEwPer);
    const u32 iid = __builtin_amdgcn_readfirstlane(blockIdx.x / per_item);
    const u32 chunk = blockIdx.x - iid * per_item;
    if ((int)iid >= nitems) return;
    const IpItem it = items[iid];
    if (it.n_ct == NCT) {
        switch (it.beta) {
            case 1: ip_fp_item<kEwPer, NCT, 1, true>(tb, it, chunk); break;
            case 2: ip_fp_item<kEwPer, NCT, 2, true>(tb, it, chunk); break;
            case 3: ip_fp_item<kEwPer, NCT, 3, true>(tb, it, chunk); break;
            case 4: ip_fp_item<kEwPer, NCT, 4, true>(tb, it, chunk); break;
            default: ip_fp_item<kEwPer, NCT, 0, true>(tb, it, chunk); break;
        }
        return;
    }
    switch (it.beta) {
        case 1: ip_fp_item<kEwPer, NCT, 1, false>(tb, it, chunk); break;
        case 2: ip_fp_item<kEwPer, NCT, 2, false>(tb, it, chunk); break;
        case 3: ip_fp_item<kEwPer, NCT, 3, false>(tb, it, chunk); break;
        case 4: ip_fp_item<kEwPer, NCT, 4, false>(tb, it, chunk); break;
        default: ip_fp_item<kEwPer, NCT, 0, false>(tb, it, chunk); break;
    }
}

// FULL as in ip_fp_item.
template <int kEwPer, int NCT, bool FULL>
__device__ __forceinline__ void ip_int_item(const DevTables &tb, const IpItem &it, u32 chunk) {
    const u32 N = 1u << tb.log_n;
    const PrimeConst pc = tb.pc[it.prime];
    const size_t kstride = (size_t)tb.n_prim * N;  // one key component
#pragma unroll
    for (int e = 0; e < kEwPer; e++) {
        const u32 x = (chunk * kEwPer + e) * 256 + threadIdx.x;
        if (x >= N) break;
        Acc128 s0[NCT], s1[NCT];
        for (u32 j = 0; j < it.beta; j++) {
            const u64 *kb = it.key + (size_t)(2 * j) * kstride + (size_t)it.prime * N;
            const u64 k0 = kb[x], k1 = kb[kstride + x];
#pragma unroll
            for (int c = 0; c < NCT; c++) {
                if (!FULL && (u32)c >= it.n_ct) break;
                // the own digit's limb, else digit j's ModUp output (a select, not a branch)
                const bool own = j == it.own_digit;
                u64 v = (own ? it.own0[c] : it.ext[c] + ((size_t)j * it.E + it.pos) * N)[x];
                if (own && it.own1[c]) v = mulm(v, it.own1[c][x], pc);
                s0[c].mac(v, k0);
                s1[c].mac(v, k1);
            }
        }
#pragma unroll
        for (int c = 0; c < NCT; c++) {
            if (!FULL && (u32)c >= it.n_ct) break;
            if (it.own2[c]) {
                const u64 a0 = it.own2[c][x], b0 = it.own3[c][x], a1 = it.own0[c][x], b1 = it.own1[c][x];
                Acc128 t;
                t.mac(a0, b1);
                t.mac(a1, b0);
                s0[c].add(shoup(mulm(a0, b0, pc), pc.pmod, pc.pmod_sh, pc.q));
                s1[c].add(shoup(t.reduce(pc), pc.pmod, pc.pmod_sh, pc.q));
            }
            it.acc[c][(size_t)it.pos * N + x] = s0[c].reduce(pc);
            it.acc[c][((size_t)it.E + it.pos) * N + x] = s1[c].reduce(pc);
        }
    }
}
template <int kEwPer, int NCT>
__global__ void __launch_bounds__(256) k_ip(DevTables tb, const IpItem *__restrict__ items, int nitems) {
    const u32 N = 1u << tb.log_n;
    const u32 per_item = (N + 256 * kEwPer - 1) / (256 * kEwPer);
    const u32 iid = __builtin_amdgcn_readfirstlane(blockIdx.x / per_item);
    const u32 chunk = blockIdx.x - iid * per_item;
    if ((int)iid >= nitems) return;
    const IpItem it = items[iid];
    if (it.n_ct == NCT)
        ip_int_item<kEwPer, NCT, true>(tb, it, chunk);
    else
        ip_int_item<kEwPer, NCT, false>(tb, it, chunk);
}

template <int kEwPer>
__global__ void __launch_bounds__(256) k_ip_seq(DevTables tb, const IpSeqItem *__restrict__ items, int nitems) {
    const u32 N = 1u << tb.log_n;
    const u32 per_item = (N + 256 * kEwPer - 1) / (256 * kEwPer);
    const u32 iid = __builtin_amdgcn_readfirstlane(blockIdx.x / per_item);
    const u32 chunk = blockIdx.x - iid * per_item;
    if ((int)iid >= nitems) return;
    const IpSeqItem &it = items[iid];
    const u32 n_ct = it.n_ct, beta = it.beta, own = it.own_digit, E = it.E, pos = it.pos;
    const PrimeConst pc = tb.pc[it.prime];
    const size_t kstride = (size_t)tb.n_prim * N;  // one key component
    const u64 *kb = it.key + (size_t)it.prime * N;
#pragma unroll
    for (int e = 0; e < kEwPer; e++) {
        const u32 x = (chunk * kEwPer + e) * 256 + threadIdx.x;
        if (x >= N) break;
        u64 k0[kIpSeqBeta], k1[kIpSeqBeta];
#pragma unroll
        for (int j = 0; j < kIpSeqBeta; j++) {
            if ((u32)j >= beta) break;
            k0[j] = kb[(size_t)(2 * j) * kstride + x];
            k1[j] = kb[(size_t)(2 * j + 1) * kstride + x];
        }
        for (u32 c = 0; c < n_ct; c++) {
            Acc128 s0, s1;
#pragma unroll
            for (int j = 0; j < kIpSeqBeta; j++) {
                if ((u32)j >= beta) break;
                u64 v;
                if ((u32)j == own) {
                    v = it.own1[c] ? mulm(it.own0[c][x], it.own1[c][x], pc) : it.own0[c][x];
                } else {
                    v = it.ext[c][((size_t)j * E + pos) * N + x];
                }
                s0.mac(v, k0[j]);
                s1.mac(v, k1[j]);
            }
            if (it.own2[c]) {
                const u64 a0 = it.own2[c][x], b0 = it.own3[c][x], a1 = it.own0[c][x], b1 = it.own1[c][x];
                Acc128 t;
                t.mac(a0, b1);
                t.mac(a1, b0);
                s0.add(shoup(mulm(a0, b0, pc), pc.pmod, pc.pmod_sh, pc.q));
                s1.add(shoup(t.reduce(pc), pc.pmod, pc.pmod_sh, pc.q));
            }
            it.acc[c][(size_t)pos * N + x] = s0.reduce(pc);
            it.acc[c][((size_t)E + pos) * N + x] = s1.reduce(pc);
        }
    }
}

// source index of NTT slot j under X -> X^g (slot k holds a(psi^(2 brv(k) + 1)))
__device__ __forceinline__ u32 automorph_src(u32 j, u32 g, u32 log_n) {
    const u32 two_n_mask = (2u << log_n) - 1;
    const u32 e = 2 * brev_n(j, log_n) + 1;
    const u32 eg = (u32)(((u64)e * (u64)g) & two_n_mask);
    return brev_n((eg - 1) >> 1, log_n);
}

// Hoisted rotations with plaintext weights; see HoItem. The 128-bit
// weighted sums are reduced every kHoFold rotations (each term < q^2).
//
// STAGED: every rotation of the launch maps each aligned block of
// kHoChunk NTT slots onto itself (the host checks that every Galois
// element is 1 modulo 2N / kHoChunk), so a workgroup owns one such
// block, copies its part of the digits once into LDS ([ct][digit]
// [kHoChunk]) and reads the automorphism's sources from there for every
// rotation instead of re-reading them from memory.
constexpr int kHoFold = 8;
constexpr u32 kHoKeyBatch = 8;  // digits whose key residues are in flight together
template <int kEwPer, bool STAGED, int NCT>
__device__ __forceinline__ void hoist_item(const DevTables &tb, const HoItem &it, u32 chunk) {
    extern __shared__ u64 ho_lds[];
    const u32 N = 1u << tb.log_n;
    const PrimeConst pc = tb.pc[it.prime];
    const size_t kstride = (size_t)tb.n_prim * N;  // one key component
    const bool data = it.pos < it.L;
    const u32 own = data ? it.pos / it.alpha : 0xFFFFFFFFu;
    const u32 base = chunk * kHoChunk;
    if constexpr (STAGED) {
#pragma unroll
        for (int c = 0; c < NCT; c++) {
            for (u32 j = 0; j < it.beta; j++) {
                const u32 x = base + threadIdx.x;
                ho_lds[(c * it.beta + j) * kHoChunk + threadIdx.x] =
                    (j == own) ? it.c1[c][(size_t)it.pos * N + x] : it.ext[c][((size_t)j * it.E + it.pos) * N + x];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < kEwPer; e++) {
        const u32 x = (chunk * kEwPer + e) * 256 + threadIdx.x;
        if (x >= N) break;
        Acc128 tb_[kHoCts], ta_[kHoCts];
        for (u32 i = 0; i < it.n_rot; i++) {
            const u32 g = it.galois[i];
            const u64 w = it.pts[((size_t)i * it.E + it.pos) * N + x];
            if (g == 1) {
                // identity: P (c0, c1) on data limbs, nothing on special limbs
                if (data) {
#pragma unroll
                    for (int c = 0; c < NCT; c++) {
                        const u64 p0 = shoup(it.c0[c][x], pc.pmod, pc.pmod_sh, pc.q);
                        const u64 p1 = shoup(it.c1[c][(size_t)it.pos * N + x], pc.pmod, pc.pmod_sh, pc.q);
                        tb_[c].mac(p0, w);
                        ta_[c].mac(p1, w);
                    }
                }
            } else {
                const u32 src = automorph_src(x, g, tb.log_n);
                const u64 *key = it.keys[i] + (size_t)it.prime * N + x;
                Acc128 sb[kHoCts], sa[kHoCts];
                const u32 ls = (src - base) & (kHoChunk - 1);
                for (u32 j0 = 0; j0 < it.beta; j0 += kHoKeyBatch) {
                    // the batch's key residues are loaded together, then used
                    u64 kk[2 * kHoKeyBatch];
#pragma unroll
                    for (u32 jj = 0; jj < kHoKeyBatch; jj++)
                        if (j0 + jj < it.beta) {
                            kk[2 * jj] = key[(size_t)(2 * (j0 + jj)) * kstride];
                            kk[2 * jj + 1] = key[(size_t)(2 * (j0 + jj) + 1) * kstride];
                        }
#pragma unroll
                    for (u32 jj = 0; jj < kHoKeyBatch; jj++) {
                        const u32 j = j0 + jj;
                        if (j >= it.beta) break;
#pragma unroll
                        for (int c = 0; c < NCT; c++) {
                            u64 v;
                            if constexpr (STAGED)
                                v = ho_lds[(c * it.beta + j) * kHoChunk + ls];
                            else
                                v = (j == own) ? it.c1[c][(size_t)it.pos * N + src]
                                               : it.ext[c][((size_t)j * it.E + it.pos) * N + src];
                            sb[c].mac(v, kk[2 * jj]);
                            sa[c].mac(v, kk[2 * jj + 1]);
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < NCT; c++) {
                    u64 rb = sb[c].reduce(pc);
                    if (data) rb = addm(rb, shoup(it.c0[c][src], pc.pmod, pc.pmod_sh, pc.q), pc.q);
                    tb_[c].mac(rb, w);
                    ta_[c].mac(sa[c].reduce(pc), w);
                }
            }
            if ((i & (kHoFold - 1)) == kHoFold - 1) {
#pragma unroll
                for (int c = 0; c < NCT; c++) {
                    tb_[c] = Acc128{tb_[c].reduce(pc), 0};
                    ta_[c] = Acc128{ta_[c].reduce(pc), 0};
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NCT; c++) {
            it.acc[c][(size_t)it.pos * N + x] = tb_[c].reduce(pc);
            it.acc[c][((size_t)it.E + it.pos) * N + x] = ta_[c].reduce(pc);
        }
    }
}
template <int kEwPer, bool STAGED>
__global__ void __launch_bounds__(256) k_hoist(DevTables tb, const HoItem *__restrict__ items, int nitems) {
    static_assert(!STAGED || kEwPer == 1, "a staged workgroup owns one block of kHoChunk slots");
    const u32 N = 1u << tb.log_n;
    const u32 per_item = (N + 256 * kEwPer - 1) / (256 * kEwPer);
    const u32 iid = __builtin_amdgcn_readfirstlane(blockIdx.x / per_item);
    const u32 chunk = blockIdx.x - iid * per_item;
    if ((int)iid >= nitems) return;
    const HoItem it = items[iid];
    switch (it.n_ct) {  // ciphertexts per item, unrolled
        case 1: hoist_item<kEwPer, STAGED, 1>(tb, it, chunk); break;
        case 2: hoist_item<kEwPer, STAGED, 2>(tb, it, chunk); break;
        case 3: hoist_item<kEwPer, STAGED, 3>(tb, it, chunk); break;
        default: hoist_item<kEwPer, STAGED, kHoCts>(tb, it, chunk);
    }
}

// Hoisted rotations in FP64 for an item whose prime t is below 2^50: every
// product is an FP64 product of two residues (<= 0.75 t), the digit sums
// and the per-rotation sums are re-centred every four terms, P (c0, c1)
// uses an FP64 product by P mod t (ratio from 1/t, error <= 2^-52).
// STAGED as in k_hoist; the staged digits are held as FP64 values.
template <int kEwPer, bool STAGED, int NCT>
__device__ __forceinline__ void hoist_fp_item(const DevTables &tb, const HoItem &it, u32 chunk) {
#pragma clang fp contract(off)
    extern __shared__ u64 ho_lds[];
    double *const sv = reinterpret_cast<double *>(ho_lds);
    const u32 N = 1u << tb.log_n;
    const PrimeConst pc = tb.pc[it.prime];
    const double t = pc.qf, tinv = pc.qinvf;
    const double pm = fp_from_u64(pc.pmod), pmq = pm * tinv;
    const size_t kstride = (size_t)tb.n_prim * N;  // one key component
    const bool data = it.pos < it.L;
    const u32 own = data ? it.pos / it.alpha : 0xFFFFFFFFu;
    const u32 base = chunk * kHoChunk;
    if constexpr (STAGED) {
#pragma unroll
        for (int c = 0; c < NCT; c++) {
            for (u32 j = 0; j < it.beta; j++) {
                const u32 x = base + threadIdx.x;
                sv[(c * it.beta + j) * kHoChunk + threadIdx.x] = fp_from_u64(
                    (j == own) ? it.c1[c][(size_t)it.pos * N + x] : it.ext[c][((size_t)j * it.E + it.pos) * N + x]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < kEwPer; e++) {
        const u32 x = (chunk * kEwPer + e) * 256 + threadIdx.x;
        if (x >= N) break;
        double tb_[kHoCts], ta_[kHoCts];
#pragma unroll
        for (int c = 0; c < NCT; c++) tb_[c] = ta_[c] = 0.0;
        for (u32 i = 0; i < it.n_rot; i++) {
            const u32 g = it.galois[i];
            const double w = fp_from_u64(it.pts[((size_t)i * it.E + it.pos) * N + x]);
            if (g == 1) {
                // identity: P (c0, c1) on data limbs, nothing on special limbs
                if (data) {
#pragma unroll
                    for (int c = 0; c < NCT; c++) {
                        const double p0 = fp_mulmod(fp_from_u64(it.c0[c][x]), pm, pmq, t);
                        const double p1 = fp_mulmod(fp_from_u64(it.c1[c][(size_t)it.pos * N + x]), pm, pmq, t);
                        tb_[c] = tb_[c] + fp_mulv(p0, w, t, tinv);
                        ta_[c] = ta_[c] + fp_mulv(p1, w, t, tinv);
                    }
                }
            } else {
                const u32 src = automorph_src(x, g, tb.log_n);
                const u64 *key = it.keys[i] + (size_t)it.prime * N + x;
                double sb[kHoCts], sa[kHoCts];
#pragma unroll
                for (int c = 0; c < NCT; c++) sb[c] = sa[c] = 0.0;
                const u32 ls = (src - base) & (kHoChunk - 1);
                for (u32 j0 = 0; j0 < it.beta; j0 += kHoKeyBatch) {
                    // the batch's key residues are loaded together, then used
                    u64 kk[2 * kHoKeyBatch];
#pragma unroll
                    for (u32 jj = 0; jj < kHoKeyBatch; jj++)
                        if (j0 + jj < it.beta) {
                            kk[2 * jj] = key[(size_t)(2 * (j0 + jj)) * kstride];
                            kk[2 * jj + 1] = key[(size_t)(2 * (j0 + jj) + 1) * kstride];
                        }
#pragma unroll
                    for (u32 jj = 0; jj < kHoKeyBatch; jj++) {
                        const u32 j = j0 + jj;
                        if (j >= it.beta) break;
                        const double k0 = fp_from_u64(kk[2 * jj]), k1 = fp_from_u64(kk[2 * jj + 1]);
#pragma unroll
                        for (int c = 0; c < NCT; c++) {
                            double v;
                            if constexpr (STAGED)
                                v = sv[(c * it.beta + j) * kHoChunk + ls];
                            else
                                v = fp_from_u64((j == own) ? it.c1[c][(size_t)it.pos * N + src]
                                                           : it.ext[c][((size_t)j * it.E + it.pos) * N + src]);
                            sb[c] = sb[c] + fp_mulv(v, k0, t, tinv);
                            sa[c] = sa[c] + fp_mulv(v, k1, t, tinv);
                            if ((j & 3) == 3) {
                                sb[c] = fp_center(sb[c], t, tinv);
                                sa[c] = fp_center(sa[c], t, tinv);
                            }
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < NCT; c++) {
                    double rb = fp_center(sb[c], t, tinv);
                    if (data) rb = fp_center(rb + fp_mulmod(fp_from_u64(it.c0[c][src]), pm, pmq, t), t, tinv);
                    tb_[c] = tb_[c] + fp_mulv(rb, w, t, tinv);
                    ta_[c] = ta_[c] + fp_mulv(fp_center(sa[c], t, tinv), w, t, tinv);
                }
            }
            if ((i & 3) == 3) {
#pragma unroll
                for (int c = 0; c < NCT; c++) {
                    tb_[c] = fp_center(tb_[c], t, tinv);
                    ta_[c] = fp_center(ta_[c], t, tinv);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NCT; c++) {
            it.acc[c][(size_t)it.pos * N + x] = fp_to_residue(fp_center(tb_[c], t, tinv), pc.qmf, pc.q);
            it.acc[c][((size_t)it.E + it.pos) * N + x] = fp_to_residue(fp_center(ta_[c], t, tinv), pc.qmf, pc.q);
        }
    }
}
template <int kEwPer, bool STAGED>
__global__ void __launch_bounds__(256) k_hoist_fp(DevTables tb, const HoItem *__restrict__ items, int nitems) {
#pragma clang fp contract(off)
    static_assert(!STAGED || kEwPer == 1, "a staged workgroup owns one block of kHoChunk slots");
    const u32 N = 1u << tb.log_n;
    const u32 per_item = (N + 256 * kEwPer - 1) / (256 * kEwPer);
    const u32 iid = __builtin_amdgcn_readfirstlane(blockIdx.x / per_item);
    const u32 chunk = blockIdx.x - iid * per_item;
    if ((int)iid >= nitems) return;
    const HoItem it = items[iid];
    switch (it.n_ct) {  // ciphertexts per item, unrolled
        case 1: hoist_fp_item<kEwPer, STAGED, 1>(tb, it, chunk); break;
        case 2: hoist_fp_item<kEwPer, STAGED, 2>(tb, it, chunk); break;
        case 3: hoist_fp_item<kEwPer, STAGED, 3>(tb, it, chunk); break;
        default: hoist_fp_item<kEwPer, STAGED, kHoCts>(tb, it, chunk);
    }
}

// The 128-bit sums of the linear layers are reduced every kLinFold terms:
// each product is below q^2 < 2^122, so 32 terms plus a reduced carry stay
// below 2^128 for any layer width.
constexpr u32 kLinFold = 32;

// Encrypted linear layer: out[j][p][t][k] = sum_i Wt[j][i] * in[i][p][t][k]
// with Wt the weights reduced mod q_t (done by k_reduce_weights). One
// thread owns one residue position for JT outputs; inputs are read once
// per output tile.
template <int JT>
__global__ void __launch_bounds__(256)
k_linear(DevTables tb, const u64 *const *__restrict__ in_ptrs, const u64 *__restrict__ wt,
         u64 *const *__restrict__ out_ptrs, u32 n_in, u32 n_out, u32 limbs, u32 in_stride,
         u32 out_stride) {
    const u32 N = 1u << tb.log_n;
    const u32 per_poly = limbs * N;
    const size_t pos_total = (size_t)2 * per_poly;
    const u32 tiles = (n_out + JT - 1) / JT;
    const size_t total = pos_total * tiles;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        const u32 tile = (u32)(g / pos_total);
        const size_t pos = g - (size_t)tile * pos_total;
        const u32 p = (u32)(pos / per_poly);
        const u32 rem = (u32)(pos - (size_t)p * per_poly);
        const u32 t = rem >> tb.log_n, k = rem & (N - 1);
        const PrimeConst pc = tb.pc[t];
        const size_t in_off = ((size_t)p * in_stride + t) * N + k;
        const u32 j0 = tile * JT;
        Acc128 acc[JT];
        const u64 *wrow = wt + ((size_t)t * n_out + j0) * n_in;
        for (u32 i = 0; i < n_in; i++) {
            const u64 x = in_ptrs[i][in_off];
#pragma unroll
            for (int jj = 0; jj < JT; jj++)
                if (j0 + jj < n_out) acc[jj].mac(x, wrow[(size_t)jj * n_in + i]);
            if ((i & (kLinFold - 1)) == kLinFold - 1) {
#pragma unroll
                for (int jj = 0; jj < JT; jj++) acc[jj] = Acc128{acc[jj].reduce(pc), 0};
            }
        }
        const size_t out_off = ((size_t)p * out_stride + t) * N + k;
#pragma unroll
        for (int jj = 0; jj < JT; jj++)
            if (j0 + jj < n_out) out_ptrs[j0 + jj][out_off] = acc[jj].reduce(pc);
    }
}

// Grouped sparse linear layer. One thread owns kLinRes consecutive residue
// positions (poly p, limb t, slots k .. k + kLinRes - 1) of one row group:
// it loads each of the group's input residues once (two 16-byte loads per
// column) and accumulates all of the group's rows. Weights (reduced mod
// q_t, layout [t][w]) and the group descriptor are wave-uniform and read
// through the scalar cache; the next column's input pointer is fetched
// while the current column is multiplied.
constexpr int kLinRes = 4;
// NR: rows per group of the launch at most (accumulators per thread)
template <int NR>
__global__ void __launch_bounds__(256)
k_linear_grouped(DevTables tb, const LinGroup *__restrict__ groups, u32 n_groups, const u32 *__restrict__ cols,
                 const u64 *__restrict__ wt, const double2 *__restrict__ wf, u32 wt_stride,
                 const u64 *const *__restrict__ in_ptrs, u64 *const *__restrict__ out_ptrs, u32 limbs, u32 in_stride,
                 u32 out_stride) {
    const u32 N = 1u << tb.log_n, NQ = N / kLinRes;
    const size_t per_group = (size_t)2 * limbs * NQ;
    const size_t total = per_group * n_groups;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        // NQ >= 256 and k fastest: (group, p, t) is uniform across a wave
        const u32 gi = __builtin_amdgcn_readfirstlane((u32)(g / per_group));
        const u32 rem = (u32)(g - (size_t)gi * per_group);
        const u32 pt = __builtin_amdgcn_readfirstlane(rem / NQ);
        const u32 k = (rem - pt * NQ) * kLinRes;
        const u32 p = pt / limbs, t = pt - p * limbs;
        const LinGroup G = groups[gi];
        const PrimeConst pc = tb.pc[t];
        const size_t in_off = ((size_t)p * in_stride + t) * N + k;
        const size_t out_off = ((size_t)p * out_stride + t) * N + k;
        const u32 *gc = cols + G.col_off;
        auto load4 = [&](const u64 *src, u64 (&x)[kLinRes]) {
            const ulonglong2 a = *reinterpret_cast<const ulonglong2 *>(src + in_off);
            const ulonglong2 b = *reinterpret_cast<const ulonglong2 *>(src + in_off + 2);
            x[0] = a.x, x[1] = a.y, x[2] = b.x, x[3] = b.y;
        };
        auto store4 = [&](u32 row, const u64 (&y)[kLinRes]) {
            u64 *dst = out_ptrs[row] + out_off;
            *reinterpret_cast<ulonglong2 *>(dst) = ulonglong2{y[0], y[1]};
            *reinterpret_cast<ulonglong2 *>(dst + 2) = ulonglong2{y[2], y[3]};
        };
        if (tb.ntt_fp && pc.q < kFpPrimeBound) {
            // FP64: products by (w, w/q) from the table, |term| < q, sums
            // re-centred every four columns (wave-uniform branch on the limb)
#pragma clang fp contract(off)
            const double2 *wv = wf + (size_t)t * wt_stride + G.w_off;
            const double q = pc.qf, qinv = pc.qinvf;
            double acc[NR][kLinRes];
#pragma unroll
            for (int r = 0; r < NR; r++)
#pragma unroll
                for (int e = 0; e < kLinRes; e++) acc[r][e] = 0.0;
            const u64 *next = in_ptrs[gc[0]];
            for (u32 c = 0; c < G.ncols; c++) {
                u64 xi[kLinRes];
                load4(next, xi);
                if (c + 1 < G.ncols) next = in_ptrs[gc[c + 1]];
                double x[kLinRes];
#pragma unroll
                for (int e = 0; e < kLinRes; e++) x[e] = fp_from_u64(xi[e]);
#pragma unroll
                for (int r = 0; r < NR; r++)
                    if ((u32)r < G.nrows) {
                        const double2 w2 = wv[(size_t)r * G.ncols + c];
#pragma unroll
                        for (int e = 0; e < kLinRes; e++) acc[r][e] = acc[r][e] + fp_mulmod(x[e], w2.x, w2.y, q);
                    }
                if ((c & 3) == 3) {
#pragma unroll
                    for (int r = 0; r < NR; r++)
#pragma unroll
                        for (int e = 0; e < kLinRes; e++) acc[r][e] = fp_center(acc[r][e], q, qinv);
                }
            }
#pragma unroll
            for (int r = 0; r < NR; r++)
                if ((u32)r < G.nrows) {
                    u64 y[kLinRes];
#pragma unroll
                    for (int e = 0; e < kLinRes; e++)
                        y[e] = fp_to_residue(fp_center(acc[r][e], q, qinv), pc.qmf, pc.q);
                    store4(G.row0 + r, y);
                }
            continue;
        }
        // 64-bit integer engine: 128-bit sums folded every kLinFold columns,
        // two residues at a time (the sums of all rows stay in registers)
        const u64 *w = wt + (size_t)t * wt_stride + G.w_off;
        for (int h = 0; h < kLinRes; h += 2) {
            Acc128 acc[NR][2];
            for (u32 c = 0; c < G.ncols; c++) {
                const u64 *src = in_ptrs[gc[c]] + in_off + h;
                const ulonglong2 x = *reinterpret_cast<const ulonglong2 *>(src);
#pragma unroll
                for (int r = 0; r < NR; r++)
                    if ((u32)r < G.nrows) {
                        const u64 wr = w[(size_t)r * G.ncols + c];
                        acc[r][0].mac(x.x, wr);
                        acc[r][1].mac(x.y, wr);
                    }
                if ((c & (kLinFold - 1)) == kLinFold - 1) {
#pragma unroll
                    for (int r = 0; r < NR; r++) {
                        acc[r][0] = Acc128{acc[r][0].reduce(pc), 0};
                        acc[r][1] = Acc128{acc[r][1].reduce(pc), 0};
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < NR; r++)
                if ((u32)r < G.nrows)
                    *reinterpret_cast<ulonglong2 *>(out_ptrs[G.row0 + r] + out_off + h) =
                        ulonglong2{acc[r][0].reduce(pc), acc[r][1].reduce(pc)};
        }
    }
}

// Dense linear layer on the matrix cores. One workgroup = 8 waves on one
// tile of 16 U consecutive residues (poly p, limb t, slots k0..k0+16U-1),
// U sub-tiles of 16; wave w owns output rows 16 (8 blockIdx.y + w) .. +15
// (one 16-row MFMA tile) for every sub-tile, so each weight fragment it
// loads serves 16 U residues. The waves share the tile's inputs: per chunk
// of 64 inputs each thread loads 2 U residues (inputs 2U srow .. 2U srow +
// 2U - 1 of slot tid % 16U; the inputs' pointers staged in LDS two chunks
// ahead), splits them into XD 7-bit digits (9, or 6 where every prime of
// the launch is below 2^42) and stores digit b of each four consecutive
// inputs as one word of the int8 B fragments in LDS (double-buffered: the
// next chunk's residues are loaded while the matrix cores work on the
// current one). Each wave
// multiplies its weight-digit A fragments (Wd [kWDig][rows_pad][k_pad],
// row-major, 16 bytes per lane) with the B fragments of each sub-tile by
// v_mfma_i32_16x16x64_i8, accumulating digit products of weight
// 128^(a + b) together. Lane layout of that instruction (checked on the
// device): A[l % 16][16 (l / 16) + e], B[16 (l / 16) + e][l % 16]
// D[4 (l / 16) + r][l % 16].
typedef int v4i __attribute__((ext_vector_type(4)));
constexpr int kMfmaWaves = 8;
// XD residue digits: 9 cover primes below 2^63, 6 primes below 2^42 (the
// 40-bit primes of the network chains: a third fewer digit products).
// U: sub-tiles per wave (accumulators: U x (kWDig + XD - 1) fragments)
template <int XD, int U>
__global__ void __launch_bounds__(64 * kMfmaWaves)
k_linear_mfma(DevTables tb, const int8_t *__restrict__ wd, u32 rows_pad, u32 k_pad, const u32 *__restrict__ cols,
              u32 n_in, u32 n_out, const u64 *const *__restrict__ in_ptrs, u64 *const *__restrict__ out_ptrs,
              u32 t_lo, u32 t_cnt, u32 in_stride, u32 out_stride) {
    constexpr int S = kWDig + XD - 1;  // digit weights 128^0 .. 128^(S-1)
    constexpr int kMfmaTile = 16 * U, IPT = 2 * U;  // residues per tile, inputs per staging thread
    // B fragments of two chunks: [buffer][digit][slot][lane group], 16 int8
    // each, one pad fragment per slot: a slot's row is 20 words, so the 16
    // slots of a sub-tile's fragment read fall in distinct banks
    __shared__ v4i bfrag[2][XD][kMfmaTile][5];
    // limb-0 pointers of the inputs of two chunks (staged two chunks ahead,
    // so the residue loads of the next chunk need no dependent global loads)
    __shared__ const u64 *cptr[2][64];
    const u32 N = 1u << tb.log_n;
    const u32 tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const u32 tile = blockIdx.x;  // 32 residues of one (p, t)
    const u32 pt = (tile * kMfmaTile) >> tb.log_n, k0 = (tile * kMfmaTile) & (N - 1);
    const u32 p = pt / t_cnt, t = t_lo + (pt - p * t_cnt);
    const u32 row0 = (blockIdx.y * kMfmaWaves + wave) * 16;
    const bool rows = row0 < rows_pad;  // every wave still stages inputs and meets the barriers
    const u32 col = lane & 15, grp = lane >> 4;
    const u32 scol = tid & (kMfmaTile - 1), srow = tid / kMfmaTile;  // staging: slot, inputs IPT srow .. +IPT-1
    const size_t in_off = ((size_t)p * in_stride + t) * N + k0 + scol;
    auto stage_ptrs = [&](u32 kc) {
        if (tid < 64) {
            const u32 i = kc + tid;
            cptr[(kc >> 6) & 1][tid] = i < n_in ? in_ptrs[cols[i]] : nullptr;
        }
    };
    auto load = [&](u32 kc, u64 (&x)[IPT]) {
        const u32 pb = (kc >> 6) & 1;
#pragma unroll
        for (int v = 0; v < IPT; v++) {
            const u64 *src = cptr[pb][IPT * srow + v];
            x[v] = src ? src[in_off] : 0;
        }
    };
    // digit b of the four consecutive inputs i0 + 4 h + v (i0 = IPT srow,
    // v = 0..3) is one word: bytes e = (i0 + 4 h) % 16 + v of lane group
    // g = (i0 + 4 h) / 16
    auto stage = [&](int buf, const u64 (&x)[IPT]) {
        u32 *w32 = reinterpret_cast<u32 *>(&bfrag[buf][0][0][0]);
#pragma unroll
        for (int h = 0; h < IPT / 4; h++) {
            const u32 i4 = IPT * srow + 4 * h, g = i4 >> 4, e4 = (i4 & 15) >> 2;
#pragma unroll
            for (int b = 0; b < XD; b++) {
                u32 w = 0;
#pragma unroll
                for (int v = 0; v < 4; v++) w |= (u32)((x[4 * h + v] >> (7 * b)) & 127) << (8 * v);
                w32[(b * kMfmaTile + scol) * 20 + g * 4 + e4] = w;
            }
        }
    };
    v4i acc[U][S];
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
        for (int s = 0; s < S; s++) acc[u][s] = v4i{0, 0, 0, 0};
    const size_t plane = (size_t)rows_pad * k_pad;
    const size_t arow = (size_t)(row0 + col) * k_pad + 16 * grp;
    stage_ptrs(0);
    if (64 < k_pad) stage_ptrs(64);
    __syncthreads();
    {
        u64 x[IPT];
        load(0, x);
        stage(0, x);
    }
    __syncthreads();
    int buf = 0;
    for (u32 kc = 0; kc < k_pad; kc += 64, buf ^= 1) {
        const bool more = kc + 64 < k_pad;
        u64 xn[IPT] = {};
        if (more) load(kc + 64, xn);
        // chunk kc's pointer slot is free: its residues were loaded in the
        // previous iteration, which ended at a barrier
        if (kc + 128 < k_pad) stage_ptrs(kc + 128);
        if (rows) {
            v4i ad[kWDig];
#pragma unroll
            for (int a = 0; a < kWDig; a++) ad[a] = *reinterpret_cast<const v4i *>(wd + a * plane + arow + kc);
#pragma unroll
            for (int u = 0; u < U; u++) {
                v4i bd[XD];
#pragma unroll
                for (int b = 0; b < XD; b++) bd[b] = bfrag[buf][b][16 * u + col][grp];
#pragma unroll
                for (int a = 0; a < kWDig; a++)
#pragma unroll
                    for (int b = 0; b < XD; b++)
                        acc[u][a + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ad[a], bd[b], acc[u][a + b], 0, 0, 0);
            }
        }
        if (more) stage(buf ^ 1, xn);
        __syncthreads();
    }
    if (!rows) return;
    const PrimeConst pc = tb.pc[t];
    const size_t out_off = ((size_t)p * out_stride + t) * N + k0 + col;
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const u32 j = row0 + 4 * grp + r;
            // v = sum_s acc_s 2^(7 s), signed, |v| < 2^(7 S + 32)
            __int128 v = 0;
#pragma unroll
            for (int s = S - 1; s >= 0; s--) v = v * 128 + (__int128)acc[u][s][r];
            const bool neg = v < 0;
            const unsigned __int128 m = neg ? (unsigned __int128)(-v) : (unsigned __int128)v;
            const u64 red = barrett128((u64)m, (u64)(m >> 64), pc);
            if (j < n_out) out_ptrs[j][out_off + 16 * u] = neg && red ? pc.q - red : red;
        }
}

// balanced base-128 digits of the weights: W[j][i] = sum_a d_a 128^a with
// d_a in [-64, 63]; wd [kWDig][rows_pad][k_pad] int8, zero padded
__global__ void k_weight_digits(const i64 *__restrict__ W, u32 n_out, u32 n_in, u32 rows_pad, u32 k_pad,
                                int8_t *__restrict__ wd) {
    const size_t total = (size_t)rows_pad * k_pad;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        const u32 j = (u32)(g / k_pad), i = (u32)(g - (size_t)j * k_pad);
        i64 w = (j < n_out && i < n_in) ? W[(size_t)j * n_in + i] : 0;
#pragma unroll
        for (int a = 0; a < kWDig; a++) {
            const i64 d = ((w + 64) & 127) - 64;
            wd[(size_t)a * total + g] = (int8_t)d;
            w = (w - d) >> 7;  // exact: w - d is a multiple of 128
        }
    }
}

// Wt[t][j][i] = W[j][i] mod q_t
__global__ void k_reduce_weights(DevTables tb, const i64 *__restrict__ W, u64 *__restrict__ wt, u32 count,
                                 u32 limbs) {
    const size_t total = (size_t)count * limbs;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        const u32 t = (u32)(g / count), e = (u32)(g - (size_t)t * count);
        wt[g] = reduce_signed(W[e], tb.pc[t]);
    }
}

// Residues per thread: 16 below N = 2^15 and 32 at 2^15 by default; the
// wide variant doubles that (32 for 2^11..2^14, 64 at 2^15) and is a
// tuning choice. Each ring's kernels live in their own translation unit.
hipError_t launch_fwd(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (tb.log_n) {
        case 16: return launch_fwd_16(tb, op, items, n, seed, s);
        case 15: return launch_fwd_15(tb, op, items, n, seed, s);
        case 14: return launch_fwd_14(tb, op, items, n, seed, s);
        case 13: return launch_fwd_13(tb, op, items, n, seed, s);
        case 10:
        case 11:
        case 12: return launch_fwd_small(tb, op, items, n, seed, s);
    }
    return hipErrorInvalidValue;
}
hipError_t launch_inv(const DevTables &tb, int op, const Item *items, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (tb.log_n) {
        case 16: return launch_inv_16(tb, op, items, n, s);
        case 15: return launch_inv_15(tb, op, items, n, s);
        case 14: return launch_inv_14(tb, op, items, n, s);
        case 13: return launch_inv_13(tb, op, items, n, s);
        case 10:
        case 11:
        case 12: return launch_inv_small(tb, op, items, n, s);
    }
    return hipErrorInvalidValue;
}

static int ew_grid(size_t work) {
    size_t blocks = (work + 255) / 256;
    const size_t cap = 256 * 64;  // enough resident waves on 256 CUs
    return (int)(blocks < cap ? (blocks ? blocks : 1) : cap);
}

static u32 ew_blocks(const DevTables &tb, int n, int per) {
    const u32 N = 1u << tb.log_n;
    return (u32)n * ((N + 256 * per - 1) / (256 * per));
}
hipError_t launch_ew(const DevTables &tb, const EwItem *items, int n, u64 seed, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (tb.ew_log) {
        case 1: hipLaunchKernelGGL(k_ew<2>, dim3(ew_blocks(tb, n, 2)), dim3(256), 0, s, tb, items, n, seed); break;
        case 3: hipLaunchKernelGGL(k_ew<8>, dim3(ew_blocks(tb, n, 8)), dim3(256), 0, s, tb, items, n, seed); break;
        default: hipLaunchKernelGGL(k_ew<4>, dim3(ew_blocks(tb, n, 4)), dim3(256), 0, s, tb, items, n, seed);
    }
    return hipGetLastError();
}
hipError_t launch_hoist(const DevTables &tb, int staged_rows, const HoItem *items, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (staged_rows > 0) {  // one workgroup per kHoChunk slots, rows x kHoChunk staged residues
        if (staged_rows > (int)kHoStageRows || (1u << tb.log_n) < kHoChunk) return hipErrorInvalidValue;
        const size_t lds = (size_t)staged_rows * kHoChunk * sizeof(u64);
        if (tb.ntt_fp)
            hipLaunchKernelGGL((k_hoist_fp<1, true>), dim3(ew_blocks(tb, n, 1)), dim3(256), lds, s, tb, items, n);
        else
            hipLaunchKernelGGL((k_hoist<1, true>), dim3(ew_blocks(tb, n, 1)), dim3(256), lds, s, tb, items, n);
        return hipGetLastError();
    }
    if (tb.ntt_fp)  // every item's prime is below 2^50
        hipLaunchKernelGGL((k_hoist_fp<2, false>), dim3(ew_blocks(tb, n, 2)), dim3(256), 0, s, tb, items, n);
    else
        hipLaunchKernelGGL((k_hoist<2, false>), dim3(ew_blocks(tb, n, 2)), dim3(256), 0, s, tb, items, n);
    return hipGetLastError();
}
template <int NCT>
static void launch_ip_t(const DevTables &tb, const IpItem *items, int n, hipStream_t s) {
    if (tb.ntt_fp) {  // every item's prime is below 2^50
        switch (tb.ew_log) {
            case 1: hipLaunchKernelGGL((k_ip_fp<2, NCT>), dim3(ew_blocks(tb, n, 2)), dim3(256), 0, s, tb, items, n); break;
            case 3: hipLaunchKernelGGL((k_ip_fp<8, NCT>), dim3(ew_blocks(tb, n, 8)), dim3(256), 0, s, tb, items, n); break;
            default: hipLaunchKernelGGL((k_ip_fp<4, NCT>), dim3(ew_blocks(tb, n, 4)), dim3(256), 0, s, tb, items, n);
        }
        return;
    }
    switch (tb.ew_log) {
        case 1: hipLaunchKernelGGL((k_ip<2, NCT>), dim3(ew_blocks(tb, n, 2)), dim3(256), 0, s, tb, items, n); break;
        case 3: hipLaunchKernelGGL((k_ip<8, NCT>), dim3(ew_blocks(tb, n, 8)), dim3(256), 0, s, tb, items, n); break;
        default: hipLaunchKernelGGL((k_ip<4, NCT>), dim3(ew_blocks(tb, n, 4)), dim3(256), 0, s, tb, items, n);
    }
}
hipError_t launch_ip_seq(const DevTables &tb, const IpSeqItem *items, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (tb.ew_log) {
        case 1: hipLaunchKernelGGL(k_ip_seq<2>, dim3(ew_blocks(tb, n, 2)), dim3(256), 0, s, tb, items, n); break;
        case 3: hipLaunchKernelGGL(k_ip_seq<8>, dim3(ew_blocks(tb, n, 8)), dim3(256), 0, s, tb, items, n); break;
        default: hipLaunchKernelGGL(k_ip_seq<4>, dim3(ew_blocks(tb, n, 4)), dim3(256), 0, s, tb, items, n);
    }
    return hipGetLastError();
}
hipError_t launch_ip(const DevTables &tb, const IpItem *items, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (tb.ip_cts == 2)
        launch_ip_t<2>(tb, items, n, s);
    else
        launch_ip_t<kIpCts>(tb, items, n, s);
    return hipGetLastError();
}
hipError_t launch_linear(const DevTables &tb, const u64 *const *in_ptrs, const u64 *wt,
                         u64 *const *out_ptrs, u32 n_in, u32 n_out, u32 limbs, u32 in_stride,
                         u32 out_stride, hipStream_t s) {
    constexpr int JT = 8;
    const size_t work = ((size_t)2 * limbs << tb.log_n) * ((n_out + JT - 1) / JT);
    hipLaunchKernelGGL((k_linear<JT>), dim3(ew_grid(work)), dim3(256), 0, s, tb, in_ptrs, wt, out_ptrs,
                       n_in, n_out, limbs, in_stride, out_stride);
    return hipGetLastError();
}
hipError_t launch_linear_grouped(const DevTables &tb, const LinGroup *groups, u32 n_groups, const u32 *cols,
                                 const u64 *wt, const double2 *wf, u32 wt_stride, const u64 *const *in_ptrs,
                                 u64 *const *out_ptrs, u32 limbs, u32 in_stride, u32 out_stride, u32 max_rows,
                                 hipStream_t s) {
    const size_t work = (((size_t)2 * limbs << tb.log_n) / kLinRes) * n_groups;
    // accumulators for the largest group only (a conv layer's groups are its filters)
#define CKKS_LIN_GROUPED(NR)                                                                                    \
    hipLaunchKernelGGL(k_linear_grouped<NR>, dim3(ew_grid(work)), dim3(256), 0, s, tb, groups, n_groups, cols, wt, \
                       wf, wt_stride, in_ptrs, out_ptrs, limbs, in_stride, out_stride)
    if (max_rows <= 2)
        CKKS_LIN_GROUPED(2);
    else if (max_rows <= 4)
        CKKS_LIN_GROUPED(4);
    else if (max_rows <= 5)
        CKKS_LIN_GROUPED(5);
    else
        CKKS_LIN_GROUPED(kLinRows);
#undef CKKS_LIN_GROUPED
    return hipGetLastError();
}
// limbs t_lo .. t_lo + t_cnt - 1 of both polys; `small`: all their primes
// are below 2^42 (six residue digits)
hipError_t launch_linear_mfma(const DevTables &tb, const int8_t *wd, u32 rows_pad, u32 k_pad, const u32 *cols,
                              u32 n_in, u32 n_out, const u64 *const *in_ptrs, u64 *const *out_ptrs, u32 t_lo,
                              u32 t_cnt, bool small, u32 in_stride, u32 out_stride, hipStream_t s) {
    const u32 N = 1u << tb.log_n;
    const u32 row_blocks = (rows_pad + 16 * kMfmaWaves - 1) / (16 * kMfmaWaves);
    // six residue digits leave room for four sub-tiles' accumulators, nine for two
    if (small)
        hipLaunchKernelGGL((k_linear_mfma<6, 4>), dim3((u32)(((size_t)2 * t_cnt * N) / 64), row_blocks),
                           dim3(64 * kMfmaWaves), 0, s, tb, wd, rows_pad, k_pad, cols, n_in, n_out, in_ptrs, out_ptrs,
                           t_lo, t_cnt, in_stride, out_stride);
    else
        hipLaunchKernelGGL((k_linear_mfma<kXDig, 2>), dim3((u32)(((size_t)2 * t_cnt * N) / 32), row_blocks),
                           dim3(64 * kMfmaWaves), 0, s, tb, wd, rows_pad, k_pad, cols, n_in, n_out, in_ptrs, out_ptrs,
                           t_lo, t_cnt, in_stride, out_stride);
    return hipGetLastError();
}
hipError_t launch_weight_digits(const i64 *W, u32 n_out, u32 n_in, u32 rows_pad, u32 k_pad, int8_t *wd,
                                hipStream_t s) {
    const size_t work = (size_t)rows_pad * k_pad;
    hipLaunchKernelGGL(k_weight_digits, dim3(ew_grid(work)), dim3(256), 0, s, W, n_out, n_in, rows_pad, k_pad, wd);
    return hipGetLastError();
}
hipError_t launch_reduce_weights(const DevTables &tb, const i64 *W, u64 *wt, u32 count, u32 limbs,
                                 hipStream_t s) {
    const size_t work = (size_t)count * limbs;
    hipLaunchKernelGGL(k_reduce_weights, dim3(ew_grid(work)), dim3(256), 0, s, tb, W, wt, count, limbs);
    return hipGetLastError();
}

}  // namespace ckks
