// gfx950 kernels for RNS-CKKS ciphertext arithmetic.
//
// Every kernel works on u64 residues in [0, q) (limb-major: one limb = N
// contiguous residues modulo one prime). Modular arithmetic runs on the
// VALU (no MFMA: the work is modular integer arithmetic, not a float
// contraction):
//   - fixed operands (twiddles, conversion constants) use Shoup's
//     multiplication with a precomputed companion floor(w 2^64 / q), lazy
//     in [0, 2q);
//   - variable x variable products use a 128-bit product and an exact
//     128-bit Barrett reduction with floor(2^128 / q);
//   - NTT butterflies keep Harvey's lazy ranges ([0, 4q) forward, [0, 2q)
//     inverse), so primes must stay below 2^61.
//
// NTT-shaped kernels: one workgroup per limb. N = 2^LOGN residues live in
// registers, E = 2^LOGE per thread (T = N / E threads). The log N butterfly
// stages are grouped in phases of LOGE stages; inside a phase every thread
// owns the whole butterfly closure of its E residues, so a phase runs with
// no communication. Between phases the residues are re-distributed through
// LDS (two 32-bit half-word rounds, one pad word per 32 to spread banks).
// Loads and stores use the coalesced layout "residue c of thread t is
// index c*T + t"; an element-wise prologue (what to load) and epilogue
// (what to store) fuse basis conversions, rescale and key-switch steps
// into the transform so intermediate limbs do not round-trip through HBM.
#include <type_traits>

#include "ckks_internal.h"

namespace ckks {

// ---------------------------------------------------------------------
// modular arithmetic
// ---------------------------------------------------------------------
__device__ __forceinline__ u64 shoup_lazy(u64 y, u64 w, u64 wsh, u64 q) {
    u64 qt = __umul64hi(y, wsh);
    return y * w - qt * q;  // in [0, 2q) for any y < 2^64 when w < q
}
__device__ __forceinline__ u64 csub(u64 x, u64 q) { return x >= q ? x - q : x; }
__device__ __forceinline__ u64 shoup(u64 y, u64 w, u64 wsh, u64 q) {
    return csub(shoup_lazy(y, w, wsh, q), q);
}
__device__ __forceinline__ u64 addm(u64 a, u64 b, u64 q) { return csub(a + b, q); }
__device__ __forceinline__ u64 subm(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }

// Exact floor((hi:lo) * floor(2^128/q) / 2^128) is either floor(z/q) or one
// less, so one conditional subtraction completes the reduction.
__device__ __forceinline__ u64 barrett128(u64 lo, u64 hi, const PrimeConst &pc) {
    u64 c1 = __umul64hi(lo, pc.br_lo);
    u64 t_lo = lo * pc.br_hi, t_hi = __umul64hi(lo, pc.br_hi);
    u64 s = t_lo + c1;
    u64 k1 = s < c1;
    u64 u_lo = hi * pc.br_lo, u_hi = __umul64hi(hi, pc.br_lo);
    u64 s2 = s + u_lo;
    u64 k2 = s2 < u_lo;
    u64 quot = hi * pc.br_hi + t_hi + u_hi + k1 + k2;
    u64 r = lo - quot * pc.q;
    return csub(r, pc.q);
}
__device__ __forceinline__ u64 mulm(u64 a, u64 b, const PrimeConst &pc) {
    return barrett128(a * b, __umul64hi(a, b), pc);
}
struct Acc128 {
    u64 lo = 0, hi = 0;
    __device__ __forceinline__ void mac(u64 a, u64 b) {
        u64 l = a * b, h = __umul64hi(a, b);
        lo += l;
        hi += h + (lo < l);
    }
    __device__ __forceinline__ void add(u64 a) {
        lo += a;
        hi += (lo < a);
    }
    __device__ __forceinline__ u64 reduce(const PrimeConst &pc) const { return barrett128(lo, hi, pc); }
};
// x < 2^64 reduced mod q with floor(2^64/q): quotient estimate off by at most one
__device__ __forceinline__ u64 reduce64(u64 x, const PrimeConst &pc) {
    u64 qt = __umul64hi(x, pc.mu);
    return csub(x - qt * pc.q, pc.q);
}
__device__ __forceinline__ u64 reduce_signed(i64 v, const PrimeConst &pc) {
    if (v >= 0) return reduce64((u64)v, pc);
    u64 m = reduce64((u64)(-(v + 1)) + 1, pc);
    return m == 0 ? 0 : pc.q - m;
}

// (r - h) mod q for r, h in [0, q_l): branch-free (one 64-bit reduction)
__device__ __forceinline__ u64 centered_mod(u64 r, u64 h, const PrimeConst &pc) {
    const bool ge = r >= h;
    const u64 m = reduce64(ge ? r - h : h - r, pc);
    return ge ? m : (m ? pc.q - m : 0);
}

// compile-time loop: f(std::integral_constant<int, I>) for I in [B, E)
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// ---------------------------------------------------------------------
// Buffer-resource access to limbs: one VGPR offset (the thread's residue)
// plus a scalar byte offset per residue slot, so the 32 loads of a
// workgroup-per-limb kernel share one address register. Out-of-range
// offsets read zero / drop the write instead of faulting.
// ---------------------------------------------------------------------
typedef __attribute__((ext_vector_type(2))) unsigned u32x2;
struct Buf {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ explicit Buf(const u64 *p)
        : r(__builtin_amdgcn_make_buffer_rsrc((void *)p, 0, 0x7fffffff, 0x00020000)) {}
    __device__ __forceinline__ u64 ld(u32 voff, u32 soff) const {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
        return ((u64)v.y << 32) | v.x;
    }
    __device__ __forceinline__ void st(u32 voff, u32 soff, u64 x) const {
        u32x2 v;
        v.x = (u32)x;
        v.y = (u32)(x >> 32);
        __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)voff, (int)soff, 0);
    }
};

// ---------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the samplers
// ---------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(u32 c0, u32 c1, u32 c2, u32 c3, u64 seed) {
    u32 k0 = (u32)seed, k1 = (u32)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; r++) {
        u32 hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        u32 hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        u32 n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}
constexpr u32 kNoLimb = 0xFFFFFFFFu;
enum SampleKind : u32 { kTernary = 0, kCbd = 1 };
__device__ __forceinline__ i64 sample_small(u32 kind, u32 j, u32 obj, u32 tag, u64 seed) {
    uint4 w = philox(j, kNoLimb, obj, tag, seed);
    if (kind == kTernary) return (i64)(((u64)w.x * 3u) >> 32) - 1;
    return (i64)__popc(w.x & 0x1FFFFFu) - (i64)__popc(w.y & 0x1FFFFFu);
}
__device__ __forceinline__ u64 sample_uniform(u32 j, u32 limb, u32 obj, u32 tag, u64 seed,
                                              const PrimeConst &pc) {
    uint4 w = philox(j, limb, obj, tag, seed);
    u64 lo = ((u64)w.y << 32) | w.x, hi = ((u64)w.w << 32) | w.z;
    return barrett128(lo, hi, pc);
}

// ---------------------------------------------------------------------
// NTT engine
// ---------------------------------------------------------------------
// butterflies issued between scheduling barriers: bounds how many twiddle
// pairs the scheduler keeps in flight (register pressure at 32 residues per
// thread)
constexpr int kTwiddleChunk = 8;
// residues converted per pass over the source limbs of a basis conversion
constexpr int kConvChunk = 8;
// residues whose epilogue inputs are loaded together before any is stored
constexpr int kEpiChunk = 8;

template <int LOGN, int LOGE>
struct Ntt {
    static constexpr int N = 1 << LOGN;
    static constexpr int E = 1 << LOGE;
    static constexpr int T = N >> LOGE;
    static constexpr int NPH = (LOGN + LOGE - 1) / LOGE;
    static constexpr int LDS_WORDS = N + (N >> 5);

    static __host__ __device__ __forceinline__ constexpr int width(int p) {
        return (LOGN - p * LOGE) < LOGE ? (LOGN - p * LOGE) : LOGE;
    }
    // Residue index held in register `reg` by thread `tid` during phase p:
    // index = base(p, tid) | off(p, reg), the two parts having disjoint
    // bits (thread bits vs. register bits), so index = base + off and the
    // LDS pad below also splits: pad(base | off) = pad(base) + pad(off).
    static __device__ __forceinline__ u32 base(int p, u32 tid) {
        const int s0 = p * LOGE, w = width(p), lo_bits = LOGN - s0 - w;
        const u32 gamma = (w == LOGE) ? tid : (tid << (LOGE - w));
        const u32 lo = gamma & ((1u << lo_bits) - 1);
        const u32 hi = gamma >> lo_bits;
        return (hi << (LOGN - s0)) | lo;
    }
    static __device__ __forceinline__ constexpr u32 off(int p, int reg) {
        const int s0 = p * LOGE, w = width(p), lo_bits = LOGN - s0 - w;
        const u32 g = (u32)(reg >> w), c = (u32)(reg & ((1 << w) - 1));
        // g only exists in the (last, partial) phase where lo_bits == 0
        return (g << (LOGN - s0)) | (c << lo_bits);
    }
    static __device__ __forceinline__ u32 index(int p, u32 tid, int reg) { return base(p, tid) | off(p, reg); }
    // the "hi" coordinate (butterfly group base) of group g in phase p
    static __device__ __forceinline__ u32 group_hi(int p, u32 tid, int g) {
        const int s0 = p * LOGE, w = width(p), lo_bits = LOGN - s0 - w;
        if (p == 0) return 0;
        const u32 gamma = (w == LOGE) ? tid : ((tid << (LOGE - w)) + (u32)g);
        return gamma >> lo_bits;
    }
    static __device__ __forceinline__ constexpr u32 pad(u32 j) { return j + (j >> 5); }

    // move residues from phase layout PF to phase layout PT through LDS
    template <int PF, int PT>
    static __device__ __forceinline__ void exchange(u64 (&r)[E], u32 *lds, u32 tid) {
        u32 tmp[E];
        u32 *wb = lds + pad(base(PF, tid));
        const u32 *rb = lds + pad(base(PT, tid));
#pragma unroll
        for (int k = 0; k < E; k++) wb[pad(off(PF, k))] = (u32)r[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < E; k++) tmp[k] = rb[pad(off(PT, k))];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < E; k++) wb[pad(off(PF, k))] = (u32)(r[k] >> 32);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < E; k++) r[k] = ((u64)rb[pad(off(PT, k))] << 32) | tmp[k];
        __syncthreads();
    }

    // Forward stage s = P * LOGE + D of phase P: Cooley-Tukey butterflies
    // (X, Y) -> (X + W Y, X - W Y), W = tw[2^s + group], Harvey lazy ranges.
    template <int P, int D>
    static __device__ __forceinline__ void fwd_stage(u64 (&r)[E], u32 tid, const ulonglong2 *__restrict__ tw,
                                                     u64 q) {
        constexpr int w = width(P), s0 = P * LOGE, half = 1 << (w - 1 - D);
        const u64 two_q = q << 1;
#pragma unroll
        for (int b = 0; b < E / 2; b++) {
            const int g = b >> (w - 1);
            const int bl = b & ((1 << (w - 1)) - 1);
            const int c = ((bl >> (w - 1 - D)) << (w - D)) | (bl & (half - 1));
            const u32 hi = group_hi(P, tid, g);
            const int x = g * (1 << w) + c, y = x + half;
            const u32 ti = (1u << (s0 + D)) + (hi << D) + (u32)(c >> (w - D));
            const ulonglong2 W = tw[ti];
            u64 X = r[x];
            X = X >= two_q ? X - two_q : X;
            const u64 Tm = shoup_lazy(r[y], W.x, W.y, q);
            r[x] = X + Tm;
            r[y] = X - Tm + two_q;
            if ((b & (kTwiddleChunk - 1)) == kTwiddleChunk - 1) __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (D + 1 < w) fwd_stage<P, D + 1>(r, tid, tw, q);
    }
    template <int P>
    static __device__ __forceinline__ void fwd_phase(u64 (&r)[E], u32 *lds, u32 tid,
                                                     const ulonglong2 *__restrict__ tw, u64 q) {
        if constexpr (P > 0) exchange<P - 1, P>(r, lds, tid);
        fwd_stage<P, 0>(r, tid, tw, q);
        if constexpr (P + 1 < NPH) fwd_phase<P + 1>(r, lds, tid, tw, q);
    }

    // forward: natural order in, "slot k = a(psi^(2brv(k)+1))" out, stage s
    // (2^s groups, half-size N >> (s+1)) multiplies by tw[2^s + group].
    // Inputs in [0, q) in the coalesced layout; outputs fully reduced.
    static __device__ __forceinline__ void forward(u64 (&r)[E], u32 *lds, u32 tid, const ulonglong2 *__restrict__ tw,
                                                   u64 q) {
        fwd_phase<0>(r, lds, tid, tw, q);
        exchange<NPH - 1, 0>(r, lds, tid);
        const u64 two_q = q << 1;
#pragma unroll
        for (int k = 0; k < E; k++) {
            u64 v = r[k];
            v = v >= two_q ? v - two_q : v;
            r[k] = v >= q ? v - q : v;
        }
    }

    // Inverse stage s = P * LOGE + D: Gentleman-Sande (X, Y) -> (X + Y,
    // (X - Y) W^-1) with the inverse twiddles; stage 0 folds in N^-1.
    template <int P, int D>
    static __device__ __forceinline__ void inv_stage(u64 (&r)[E], u32 tid, const ulonglong2 *__restrict__ itw,
                                                     const PrimeConst &pc) {
        constexpr int w = width(P), s0 = P * LOGE, half = 1 << (w - 1 - D);
        constexpr bool last = (s0 + D) == 0;
        const u64 q = pc.q, two_q = q << 1;
#pragma unroll
        for (int b = 0; b < E / 2; b++) {
            const int g = b >> (w - 1);
            const int bl = b & ((1 << (w - 1)) - 1);
            const int c = ((bl >> (w - 1 - D)) << (w - D)) | (bl & (half - 1));
            const u32 hi = group_hi(P, tid, g);
            const int x = g * (1 << w) + c, y = x + half;
            const u64 X = r[x], Y = r[y];
            if constexpr (last) {
                r[x] = shoup_lazy(X + Y, pc.ninv, pc.ninv_sh, q);
                r[y] = shoup_lazy(X - Y + two_q, pc.last_w, pc.last_w_sh, q);
            } else {
                const u32 ti = (1u << (s0 + D)) + (hi << D) + (u32)(c >> (w - D));
                const ulonglong2 W = itw[ti];
                const u64 U = X + Y;
                r[x] = U >= two_q ? U - two_q : U;
                r[y] = shoup_lazy(X - Y + two_q, W.x, W.y, q);
            }
            if ((b & (kTwiddleChunk - 1)) == kTwiddleChunk - 1) __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (D > 0) inv_stage<P, D - 1>(r, tid, itw, pc);
    }
    template <int P>
    static __device__ __forceinline__ void inv_phase(u64 (&r)[E], u32 *lds, u32 tid,
                                                     const ulonglong2 *__restrict__ itw, const PrimeConst &pc) {
        if constexpr (P < NPH - 1) exchange<P + 1, P>(r, lds, tid);
        inv_stage<P, width(P) - 1>(r, tid, itw, pc);
        if constexpr (P > 0) inv_phase<P - 1>(r, lds, tid, itw, pc);
    }

    // inverse: exactly the forward stages undone in reverse order. Inputs
    // in [0, q) in the coalesced layout; outputs fully reduced, coalesced.
    static __device__ __forceinline__ void inverse(u64 (&r)[E], u32 *lds, u32 tid, const ulonglong2 *__restrict__ itw,
                                                   const PrimeConst &pc) {
        exchange<0, NPH - 1>(r, lds, tid);
        inv_phase<NPH - 1>(r, lds, tid, itw, pc);
#pragma unroll
        for (int k = 0; k < E; k++) r[k] = csub(r[k], pc.q);
    }
};

// ---------------------------------------------------------------------
// fused prologues / epilogues
// ---------------------------------------------------------------------
enum FwdOp : int {
    F_COPY = 0,     // in[0] -> NTT -> out
    F_MODUP = 1,    // ModUp digit conversion -> NTT -> out
    F_RESCALE = 2,  // rescale correction -> NTT -> (in[1] - .) q_l^-1 -> out
    F_MODDOWN = 3,  // ModDown conversion -> NTT -> (in[1] - .) P^-1 (+ in[2]) -> out
    // ModDown + rescale of one limb i < l of an HMult accumulator:
    // z = conv_i(y) P^-1 + [t]_centred -> NTT, with y (in[0], n_p limbs) =
    // INTT(acc_P) hat_m^-1 and t (in[1]) the relinearised top limb in the
    // coefficient domain; l = a; out = z
    F_RELIN = 4,
    F_SAMPLE = 5,   // sampled small polynomial -> NTT -> out
    F_INT = 6,      // signed int64 coefficients -> NTT -> out
    F_RELIN_RS = 7, // F_RELIN, then out = (acc' P^-1 - z) q_l^-1, acc' (in[2]) the accumulator limb
};
enum InvOp : int {
    I_COPY = 0,     // in[0] -> INTT -> out
    I_MUL = 1,      // in[0] * in[1] -> INTT -> out
    I_SCALE = 2,    // in[0] -> INTT -> * (hat_m^-1 mod p_m, m = a | P^-1 mod q when b = 1 |
                    //   the ModUp source factor hat_i^-1 when b = 2) -> out
    I_DECRYPT = 3,  // c0 + c1 s (+ c2 s^2) -> INTT -> out
};

// XCD-aware item order: the chip dispatches workgroup b to XCD (b mod 8).
// Consecutive items (which often read the same source limbs) are mapped
// to one XCD so those limbs are reused from that XCD's L2.
__device__ __forceinline__ int xcd_item(int nitems, u32 remap) {
    const int b = blockIdx.x, nb = gridDim.x;
    if (!remap) return b < nitems ? b : -1;
    const int per = nb >> 3;  // grid is padded to a multiple of 8
    const int it = (b & 7) * per + (b >> 3);
    return it < nitems ? it : -1;
}
__host__ __device__ inline int xcd_grid(int nitems) { return (nitems + 7) & ~7; }

template <int LOGN, int LOGE, int OP>
__global__ void __launch_bounds__(1 << (LOGN - LOGE))
k_fwd(DevTables tb, const Item *__restrict__ items, int nitems, u64 seed) {
    using NT = Ntt<LOGN, LOGE>;
    constexpr int N = NT::N, E = NT::E, T = NT::T;
    __shared__ u32 lds[NT::LDS_WORDS];
    const int iid = xcd_item(nitems, tb.xcd_remap);
    if (iid < 0) return;
    const Item it = items[iid];
    const u32 tid = threadIdx.x, vo = tid * 8;
    const PrimeConst pc = tb.pc[it.prime];
    const u64 q = pc.q;
    u64 r[E];

    // ---- prologue: residues of the polynomial to transform (coefficients)
    if constexpr (OP == F_COPY) {
#pragma unroll
        for (int c = 0; c < E; c++) r[c] = Buf(it.in[0]).ld(vo, c * T * 8);
    } else if constexpr (OP == F_MODUP || OP == F_MODDOWN) {
        // sum_i [x_i * hat_i^-1]_{q_i} * (hat_i mod t), one Barrett at the end
        const u32 lo = it.a, s = it.b;  // first source prime index, count
        const u64 *blk;
        const u64 *hat;
        u32 hat_stride;
        if constexpr (OP == F_MODUP) {
            blk = tb.modup + (size_t)(it.c * tb.alpha + s - 1) * modup_block_words(tb.alpha, tb.n_prim);
            hat = blk + 2 * tb.alpha + it.prime;  // hat[i * n_prim + t]
            hat_stride = tb.n_prim;
        } else {
            blk = tb.moddown;
            hat = blk + 2 * tb.n_p + it.prime;  // hat[m * n_q + t]
            hat_stride = tb.n_q;
        }
        const Buf src(it.in[0]);
        constexpr int kCC = E >= 32 ? 4 : kConvChunk;
        static_for<0, E / kCC>([&](auto C0) {
            constexpr int c0 = decltype(C0)::value * kCC;
            Acc128 acc[kCC];
            for (u32 i = 0; i < s; i++) {
                const u64 inv = blk[2 * i], inv_sh = blk[2 * i + 1], qi = tb.pc[lo + i].q, h = hat[i * hat_stride];
#pragma unroll
                for (int c = 0; c < kCC; c++) {
                    const u64 x = src.ld(vo, (i * N + (c0 + c) * T) * 8);
                    // ModUp sources arrive pre-multiplied by hat_i^-1 (it.v == 1)
                    const u64 y = (OP == F_MODUP && it.v == 1) ? x : shoup(x, inv, inv_sh, qi);
                    acc[c].mac(y, h);
                }
            }
#pragma unroll
            for (int c = 0; c < kCC; c++) r[c0 + c] = acc[c].reduce(pc);
        });
    } else if constexpr (OP == F_RELIN || OP == F_RELIN_RS) {
        const PrimeConst pl = tb.pc[it.a];  // q_l
        const u64 hl = pl.q >> 1;
        const u64 *hat = tb.moddown + 2 * tb.n_p + it.prime;  // hat[m * n_q]: P/p_m mod q_i
        const Buf ys(it.in[0]), ts(it.in[1]);
        constexpr int kCC = E >= 32 ? 4 : kConvChunk;
        static_for<0, E / kCC>([&](auto C0) {
            constexpr int c0 = decltype(C0)::value * kCC;
            Acc128 acc[kCC];
            for (u32 m = 0; m < tb.n_p; m++) {
                const u64 h = hat[(size_t)m * tb.n_q];
#pragma unroll
                for (int c = 0; c < kCC; c++) acc[c].mac(ys.ld(vo, (m * N + (c0 + c) * T) * 8), h);
            }
#pragma unroll
            for (int c = 0; c < kCC; c++) {
                const u64 tc = centered_mod(addm(ts.ld(vo, (c0 + c) * T * 8), hl, pl.q), hl, pc);
                r[c0 + c] = addm(shoup(acc[c].reduce(pc), pc.pinv, pc.pinv_sh, q), tc, q);
            }
        });
    } else if constexpr (OP == F_RESCALE) {
        const PrimeConst pl = tb.pc[it.a];  // q_l
        const u64 hl = pl.q >> 1;
#pragma unroll
        for (int c = 0; c < E; c++) {
            r[c] = centered_mod(addm(Buf(it.in[0]).ld(vo, c * T * 8), hl, pl.q), hl, pc);
        }
    } else if constexpr (OP == F_SAMPLE) {
        // it.a = kind, it.b = object id, it.c = domain tag
#pragma unroll
        for (int c = 0; c < E; c++) r[c] = reduce_signed(sample_small(it.a, c * T + tid, it.b, it.c, seed), pc);
    } else if constexpr (OP == F_INT) {
        const i64 *src = reinterpret_cast<const i64 *>(it.in[0]);
#pragma unroll
        for (int c = 0; c < E; c++) r[c] = reduce_signed((i64)Buf((const u64 *)src).ld(vo, c * T * 8), pc);
    }

    NT::forward(r, lds, tid, tb.tw + (size_t)it.prime * N, q);

    // ---- epilogue
    if constexpr (OP == F_COPY || OP == F_MODUP || OP == F_SAMPLE || OP == F_INT || OP == F_RELIN) {
#pragma unroll
        for (int c = 0; c < E; c++) Buf(it.out).st(vo, c * T * 8, r[c]);
    } else if constexpr (OP == F_RESCALE) {
        const ulonglong2 qi = tb.rescale[(size_t)it.a * tb.n_q + it.prime];
        const Buf in1(it.in[1]), dst(it.out);
#pragma unroll
        for (int c0 = 0; c0 < E; c0 += kEpiChunk) {
            u64 x[kEpiChunk];
#pragma unroll
            for (int c = 0; c < kEpiChunk; c++) x[c] = in1.ld(vo, (c0 + c) * T * 8);
#pragma unroll
            for (int c = 0; c < kEpiChunk; c++)
                dst.st(vo, (c0 + c) * T * 8, shoup(subm(x[c], r[c0 + c], q), qi.x, qi.y, q));
        }
    } else if constexpr (OP == F_RELIN_RS) {
        // y = (acc' P^-1 - z) q_l^-1 with acc' (in[2]) the accumulator limb
        const ulonglong2 qi = tb.rescale[(size_t)it.a * tb.n_q + it.prime];
        const Buf accb(it.in[2]), dst(it.out);
        constexpr int kRC = 4;
#pragma unroll
        for (int c0 = 0; c0 < E; c0 += kRC) {
            u64 x[kRC];
#pragma unroll
            for (int c = 0; c < kRC; c++) x[c] = accb.ld(vo, (c0 + c) * T * 8);
#pragma unroll
            for (int c = 0; c < kRC; c++) {
                const u64 u = shoup(x[c], pc.pinv, pc.pinv_sh, q);
                dst.st(vo, (c0 + c) * T * 8, shoup(subm(u, r[c0 + c], q), qi.x, qi.y, q));
            }
        }
    } else if constexpr (OP == F_MODDOWN) {
        const Buf in1(it.in[1]), in2(it.in[2] ? it.in[2] : it.in[1]), dst(it.out);
        const bool add = it.in[2] != nullptr;
#pragma unroll
        for (int c0 = 0; c0 < E; c0 += kEpiChunk) {
            u64 x[kEpiChunk], a[kEpiChunk];
#pragma unroll
            for (int c = 0; c < kEpiChunk; c++) {
                x[c] = in1.ld(vo, (c0 + c) * T * 8);
                a[c] = add ? in2.ld(vo, (c0 + c) * T * 8) : 0;
            }
#pragma unroll
            for (int c = 0; c < kEpiChunk; c++) {
                u64 y = shoup(subm(x[c], r[c0 + c], q), pc.pinv, pc.pinv_sh, q);
                dst.st(vo, (c0 + c) * T * 8, add ? addm(y, a[c], q) : y);
            }
        }
    }
}

template <int LOGN, int LOGE, int OP>
__global__ void __launch_bounds__(1 << (LOGN - LOGE))
k_inv(DevTables tb, const Item *__restrict__ items, int nitems) {
    using NT = Ntt<LOGN, LOGE>;
    constexpr int N = NT::N, E = NT::E, T = NT::T;
    __shared__ u32 lds[NT::LDS_WORDS];
    const int iid = xcd_item(nitems, tb.xcd_remap);
    if (iid < 0) return;
    const Item it = items[iid];
    const u32 tid = threadIdx.x, vo = tid * 8;
    const PrimeConst pc = tb.pc[it.prime];
    const u64 q = pc.q;
    u64 r[E];

    if constexpr (OP == I_COPY || OP == I_SCALE) {
#pragma unroll
        for (int c = 0; c < E; c++) r[c] = Buf(it.in[0]).ld(vo, c * T * 8);
    } else if constexpr (OP == I_MUL) {
#pragma unroll
        for (int c = 0; c < E; c++) r[c] = mulm(Buf(it.in[0]).ld(vo, c * T * 8), Buf(it.in[1]).ld(vo, c * T * 8), pc);
    } else if constexpr (OP == I_DECRYPT) {
        const u64 *s = it.in[3];
#pragma unroll
        for (int c = 0; c < E; c++) {
            const u32 so = c * T * 8;
            const u64 sj = Buf(s).ld(vo, so);
            u64 m = addm(Buf(it.in[0]).ld(vo, so), mulm(Buf(it.in[1]).ld(vo, so), sj, pc), q);
            if (it.a == 3) m = addm(m, mulm(Buf(it.in[2]).ld(vo, so), mulm(sj, sj, pc), pc), q);
            r[c] = m;
        }
    }

    NT::inverse(r, lds, tid, tb.itw + (size_t)it.prime * N, pc);

    if constexpr (OP == I_MUL) {
        // it.v == 1: store [x * hat_i^-1]_{q_i}, the ModUp input (digit block it.c, position it.a)
        if (it.v == 1) {
            const u64 *blk = tb.modup + (size_t)it.c * modup_block_words(tb.alpha, tb.n_prim);
            const u64 inv = blk[2 * it.a], inv_sh = blk[2 * it.a + 1];
#pragma unroll
            for (int c = 0; c < E; c++) r[c] = shoup(r[c], inv, inv_sh, q);
        }
    } else if constexpr (OP == I_SCALE) {
        // b == 0: hat_m^-1 mod p_m for special prime m = a; b == 1: P^-1 mod q;
        // b == 2: hat_i^-1 of ModUp digit block c, position a (a ModUp source)
        const u64 *blk = tb.modup + (size_t)it.c * modup_block_words(tb.alpha, tb.n_prim);
        const u64 inv = it.b == 1 ? pc.pinv : it.b == 2 ? blk[2 * it.a] : tb.moddown[2 * it.a];
        const u64 inv_sh = it.b == 1 ? pc.pinv_sh : it.b == 2 ? blk[2 * it.a + 1] : tb.moddown[2 * it.a + 1];
#pragma unroll
        for (int c = 0; c < E; c++) r[c] = shoup(r[c], inv, inv_sh, q);
    }
#pragma unroll
    for (int c = 0; c < E; c++) Buf(it.out).st(vo, c * T * 8, r[c]);
}

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
template <int kEwPer>
__global__ void __launch_bounds__(256) k_ip(DevTables tb, const IpItem *__restrict__ items, int nitems) {
    const u32 N = 1u << tb.log_n;
    const u32 per_item = (N + 256 * kEwPer - 1) / (256 * kEwPer);
    const u32 iid = __builtin_amdgcn_readfirstlane(blockIdx.x / per_item);
    const u32 chunk = blockIdx.x - iid * per_item;
    if ((int)iid >= nitems) return;
    const IpItem it = items[iid];
    const PrimeConst pc = tb.pc[it.prime];
    const size_t kstride = (size_t)tb.n_prim * N;  // one key component
#pragma unroll
    for (int e = 0; e < kEwPer; e++) {
        const u32 x = (chunk * kEwPer + e) * 256 + threadIdx.x;
        if (x >= N) break;
        Acc128 s0[kIpCts], s1[kIpCts];
        for (u32 j = 0; j < it.beta; j++) {
            const u64 *kb = it.key + (size_t)(2 * j) * kstride + (size_t)it.prime * N;
            const u64 k0 = kb[x], k1 = kb[kstride + x];
#pragma unroll
            for (int c = 0; c < kIpCts; c++) {
                if ((u32)c >= it.n_ct) break;
                u64 v;
                if (j == it.own_digit) {
                    v = it.own1[c] ? mulm(it.own0[c][x], it.own1[c][x], pc) : it.own0[c][x];
                } else {
                    v = it.ext[c][((size_t)j * it.E + it.pos) * N + x];
                }
                s0[c].mac(v, k0);
                s1[c].mac(v, k1);
            }
        }
#pragma unroll
        for (int c = 0; c < kIpCts; c++) {
            if ((u32)c >= it.n_ct) break;
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

// source index of NTT slot j under X -> X^g (slot k holds a(psi^(2 brv(k) + 1)))
__device__ __forceinline__ u32 automorph_src(u32 j, u32 g, u32 log_n) {
    const u32 two_n_mask = (2u << log_n) - 1;
    const u32 e = 2 * brev_n(j, log_n) + 1;
    const u32 eg = (u32)(((u64)e * (u64)g) & two_n_mask);
    return brev_n((eg - 1) >> 1, log_n);
}

// Hoisted rotations with plaintext weights; see HoItem. The 128-bit
// weighted sums are reduced every kHoFold rotations (each term < q^2).
constexpr int kHoFold = 8;
template <int kEwPer>
__global__ void __launch_bounds__(256) k_hoist(DevTables tb, const HoItem *__restrict__ items, int nitems) {
    const u32 N = 1u << tb.log_n;
    const u32 per_item = (N + 256 * kEwPer - 1) / (256 * kEwPer);
    const u32 iid = __builtin_amdgcn_readfirstlane(blockIdx.x / per_item);
    const u32 chunk = blockIdx.x - iid * per_item;
    if ((int)iid >= nitems) return;
    const HoItem it = items[iid];
    const PrimeConst pc = tb.pc[it.prime];
    const size_t kstride = (size_t)tb.n_prim * N;  // one key component
    const bool data = it.pos < it.L;
    const u32 own = data ? it.pos / it.alpha : 0xFFFFFFFFu;
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
                    for (int c = 0; c < kHoCts; c++) {
                        if ((u32)c >= it.n_ct) break;
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
                for (u32 j = 0; j < it.beta; j++) {
                    const u64 k0 = key[(size_t)(2 * j) * kstride], k1 = key[(size_t)(2 * j + 1) * kstride];
#pragma unroll
                    for (int c = 0; c < kHoCts; c++) {
                        if ((u32)c >= it.n_ct) break;
                        const u64 v = (j == own) ? it.c1[c][(size_t)it.pos * N + src]
                                                 : it.ext[c][((size_t)j * it.E + it.pos) * N + src];
                        sb[c].mac(v, k0);
                        sa[c].mac(v, k1);
                    }
                }
#pragma unroll
                for (int c = 0; c < kHoCts; c++) {
                    if ((u32)c >= it.n_ct) break;
                    u64 rb = sb[c].reduce(pc);
                    if (data) rb = addm(rb, shoup(it.c0[c][src], pc.pmod, pc.pmod_sh, pc.q), pc.q);
                    tb_[c].mac(rb, w);
                    ta_[c].mac(sa[c].reduce(pc), w);
                }
            }
            if ((i & (kHoFold - 1)) == kHoFold - 1) {
#pragma unroll
                for (int c = 0; c < kHoCts; c++) {
                    tb_[c] = Acc128{tb_[c].reduce(pc), 0};
                    ta_[c] = Acc128{ta_[c].reduce(pc), 0};
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kHoCts; c++) {
            if ((u32)c >= it.n_ct) break;
            it.acc[c][(size_t)it.pos * N + x] = tb_[c].reduce(pc);
            it.acc[c][((size_t)it.E + it.pos) * N + x] = ta_[c].reduce(pc);
        }
    }
}

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
        }
        const size_t out_off = ((size_t)p * out_stride + t) * N + k;
#pragma unroll
        for (int jj = 0; jj < JT; jj++)
            if (j0 + jj < n_out) out_ptrs[j0 + jj][out_off] = acc[jj].reduce(pc);
    }
}

// Grouped sparse linear layer. One thread owns one residue position
// (poly p, limb t, slot k) of one row group: it loads each of the group's
// input residues once and accumulates all of the group's rows in 128-bit
// accumulators. Weights (reduced mod q_t, layout [t][w]) and the group
// descriptor are wave-uniform and read through the scalar cache.
__global__ void __launch_bounds__(256)
k_linear_grouped(DevTables tb, const LinGroup *__restrict__ groups, u32 n_groups, const u32 *__restrict__ cols,
                 const u64 *__restrict__ wt, u32 wt_stride, const u64 *const *__restrict__ in_ptrs,
                 u64 *const *__restrict__ out_ptrs, u32 limbs, u32 in_stride, u32 out_stride) {
    const u32 N = 1u << tb.log_n;
    const size_t per_group = (size_t)2 * limbs * N;
    const size_t total = per_group * n_groups;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        // N >= 64 and k fastest: (group, p, t) is uniform across a wave
        const u32 gi = __builtin_amdgcn_readfirstlane((u32)(g / per_group));
        const u32 rem = (u32)(g - (size_t)gi * per_group);
        const u32 pt = __builtin_amdgcn_readfirstlane(rem >> tb.log_n);
        const u32 k = rem & (N - 1);
        const u32 p = pt / limbs, t = pt - p * limbs;
        const LinGroup G = groups[gi];
        const PrimeConst pc = tb.pc[t];
        const u64 *w = wt + (size_t)t * wt_stride + G.w_off;
        const size_t in_off = ((size_t)p * in_stride + t) * N + k;
        Acc128 acc[kLinRows];
        for (u32 c = 0; c < G.ncols; c++) {
            const u64 x = in_ptrs[cols[G.col_off + c]][in_off];
#pragma unroll
            for (int r = 0; r < kLinRows; r++)
                if ((u32)r < G.nrows) acc[r].mac(x, w[(size_t)r * G.ncols + c]);
        }
        const size_t out_off = ((size_t)p * out_stride + t) * N + k;
#pragma unroll
        for (int r = 0; r < kLinRows; r++)
            if ((u32)r < G.nrows) out_ptrs[G.row0 + r][out_off] = acc[r].reduce(pc);
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

// ---------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------
template <int LOGN, int LOGE, int OP>
static hipError_t launch_fwd_t(const DevTables &tb, const Item *items, int n, u64 seed, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd<LOGN, LOGE, OP>), dim3(xcd_grid(n)), dim3(Ntt<LOGN, LOGE>::T), 0, s, tb,
                       items, n, seed);
    return hipGetLastError();
}
template <int LOGN, int LOGE, int OP>
static hipError_t launch_inv_t(const DevTables &tb, const Item *items, int n, hipStream_t s) {
    hipLaunchKernelGGL((k_inv<LOGN, LOGE, OP>), dim3(xcd_grid(n)), dim3(Ntt<LOGN, LOGE>::T), 0, s, tb,
                       items, n);
    return hipGetLastError();
}

// residues per thread: 32 for the large rings (one 1024-thread workgroup
// per 2^15 limb), 16 below.
#define CKKS_FWD_CASE(LN, LE)                                                        \
    case LN:                                                                         \
        switch (op) {                                                                \
            case F_COPY: return launch_fwd_t<LN, LE, F_COPY>(tb, items, n, seed, s);       \
            case F_MODUP: return launch_fwd_t<LN, LE, F_MODUP>(tb, items, n, seed, s);     \
            case F_RESCALE: return launch_fwd_t<LN, LE, F_RESCALE>(tb, items, n, seed, s); \
            case F_MODDOWN: return launch_fwd_t<LN, LE, F_MODDOWN>(tb, items, n, seed, s); \
            case F_RELIN: return launch_fwd_t<LN, LE, F_RELIN>(tb, items, n, seed, s);     \
            case F_RELIN_RS: return launch_fwd_t<LN, LE, F_RELIN_RS>(tb, items, n, seed, s); \
            case F_SAMPLE: return launch_fwd_t<LN, LE, F_SAMPLE>(tb, items, n, seed, s);   \
            case F_INT: return launch_fwd_t<LN, LE, F_INT>(tb, items, n, seed, s);         \
        }                                                                            \
        break;
#define CKKS_INV_CASE(LN, LE)                                                        \
    case LN:                                                                         \
        switch (op) {                                                                \
            case I_COPY: return launch_inv_t<LN, LE, I_COPY>(tb, items, n, s);             \
            case I_MUL: return launch_inv_t<LN, LE, I_MUL>(tb, items, n, s);               \
            case I_SCALE: return launch_inv_t<LN, LE, I_SCALE>(tb, items, n, s);           \
            case I_DECRYPT: return launch_inv_t<LN, LE, I_DECRYPT>(tb, items, n, s);       \
        }                                                                            \
        break;

// Residues per thread: 16 below N = 2^15 and 32 at 2^15 by default; the
// wide variant doubles that (32 for 2^11..2^14, 64 at 2^15) and is a
// tuning choice.
hipError_t launch_fwd(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (tb.ntt_wide) {
        switch (tb.log_n) {
            CKKS_FWD_CASE(11, 5)
            CKKS_FWD_CASE(12, 5)
            CKKS_FWD_CASE(13, 5)
            CKKS_FWD_CASE(14, 5)
            CKKS_FWD_CASE(15, 6)
        }
    }
    switch (tb.log_n) {
        CKKS_FWD_CASE(10, 4)
        CKKS_FWD_CASE(11, 4)
        CKKS_FWD_CASE(12, 4)
        CKKS_FWD_CASE(13, 4)
        CKKS_FWD_CASE(14, 4)
        CKKS_FWD_CASE(15, 5)
    }
    return hipErrorInvalidValue;
}
hipError_t launch_inv(const DevTables &tb, int op, const Item *items, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (tb.ntt_wide) {
        switch (tb.log_n) {
            CKKS_INV_CASE(11, 5)
            CKKS_INV_CASE(12, 5)
            CKKS_INV_CASE(13, 5)
            CKKS_INV_CASE(14, 5)
            CKKS_INV_CASE(15, 6)
        }
    }
    switch (tb.log_n) {
        CKKS_INV_CASE(10, 4)
        CKKS_INV_CASE(11, 4)
        CKKS_INV_CASE(12, 4)
        CKKS_INV_CASE(13, 4)
        CKKS_INV_CASE(14, 4)
        CKKS_INV_CASE(15, 5)
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
hipError_t launch_hoist(const DevTables &tb, const HoItem *items, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hoist<2>, dim3(ew_blocks(tb, n, 2)), dim3(256), 0, s, tb, items, n);
    return hipGetLastError();
}
hipError_t launch_ip(const DevTables &tb, const IpItem *items, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (tb.ew_log) {
        case 1: hipLaunchKernelGGL(k_ip<2>, dim3(ew_blocks(tb, n, 2)), dim3(256), 0, s, tb, items, n); break;
        case 3: hipLaunchKernelGGL(k_ip<8>, dim3(ew_blocks(tb, n, 8)), dim3(256), 0, s, tb, items, n); break;
        default: hipLaunchKernelGGL(k_ip<4>, dim3(ew_blocks(tb, n, 4)), dim3(256), 0, s, tb, items, n);
    }
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
                                 const u64 *wt, u32 wt_stride, const u64 *const *in_ptrs, u64 *const *out_ptrs,
                                 u32 limbs, u32 in_stride, u32 out_stride, hipStream_t s) {
    const size_t work = ((size_t)2 * limbs << tb.log_n) * n_groups;
    hipLaunchKernelGGL(k_linear_grouped, dim3(ew_grid(work)), dim3(256), 0, s, tb, groups, n_groups, cols, wt,
                       wt_stride, in_ptrs, out_ptrs, limbs, in_stride, out_stride);
    return hipGetLastError();
}
hipError_t launch_reduce_weights(const DevTables &tb, const i64 *W, u64 *wt, u32 count, u32 limbs,
                                 hipStream_t s) {
    const size_t work = (size_t)count * limbs;
    hipLaunchKernelGGL(k_reduce_weights, dim3(ew_grid(work)), dim3(256), 0, s, tb, W, wt, count, limbs);
    return hipGetLastError();
}

}  // namespace ckks
