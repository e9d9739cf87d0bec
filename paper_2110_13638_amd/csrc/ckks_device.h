// gfx950 device code for RNS-CKKS ciphertext arithmetic: modular
// arithmetic, the register-resident NTT engine and the NTT kernels with
// their fused prologues / epilogues (instantiated per ring degree by the
// ckks_ntt_*.hip translation units, which compile in parallel).
//
// Every kernel works on u64 residues in [0, q) (limb-major: one limb = N
// contiguous residues modulo one prime) at its boundaries. Modular
// arithmetic runs on the VALU in one of two engines, chosen per launch by
// the primes of its items (the host splits launches by prime class):
//   - FP64 (primes below 2^50): residues are integer-valued doubles inside
//     the kernel; products are split exactly by an FMA and reduced with a
//     rounded quotient (fp_mulmod below), at the full FP64 FMA rate;
//   - 64-bit integer (every prime): fixed operands (twiddles, conversion
//     constants) use Shoup's multiplication with a precomputed companion
//     floor(w 2^64 / q), lazy in [0, 2q); variable x variable products use
//     a 128-bit product and an exact 128-bit Barrett reduction with
//     floor(2^128 / q); NTT butterflies keep Harvey's lazy ranges ([0, 4q)
//     forward, [0, 2q) inverse), so primes must stay below 2^61.
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
#pragma once
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

// ---------------------------------------------------------------------
// FP64 modular arithmetic for primes below 2^50 (the double-precision
// scheme of van der Hoeven, Lecerf and Quintin, "Modular SIMD arithmetic in
// Mathemagix", ACM TOMS 43(1), 2016): a residue is an integer-valued double,
// an FMA returns the exact low part of a product and a rounded
// multiplication by w/q (or 1/q) the quotient. gfx950 issues one FP64 FMA
// per lane per cycle, the rate of a single 32-bit integer operation, while
// an exact 64-bit Shoup product takes about twenty of those.
//   fp_mulmod(y, w, w/q): y w - k q with k = fl(y (w/q) + 1.5 2^52) -
//   1.5 2^52. For integer-valued y, w with |y w| < 2^104 the result is
//   exactly y w - k q (h - k q and h + l are integers below 2^53), so the
//   residue is always right; its size depends on k. While |y (w/q)| < 2^51
//   the sum lands in [2^52, 2^53), where doubles are the integers, and k is
//   the integer nearest to y (w/q): |result| <= q (1/2 + |y| |w/q| 2^-53).
//   Beyond 2^51 the spacing is 2 and k can be off by one more. The
//   transform multipliers are therefore stored centred (|w/q| <= 1/2), so
//   every |y| < 2^52 takes the nearest quotient (a committed CPU emulation
//   of both transform schedules checks the bounds below exactly).
// The arithmetic is written out operation by operation: no contraction
// into FMAs beyond the explicit ones.
// ---------------------------------------------------------------------
constexpr double kRound = 6755399441055744.0;  // 1.5 * 2^52: (x + kRound) - kRound rounds |x| < 2^51 to nearest
constexpr double kTwo52 = 4503599627370496.0;
constexpr u64 kMant52 = (1ull << 52) - 1;
__device__ __forceinline__ double fp_mulmod(double y, double w, double wq, double q) {
#pragma clang fp contract(off)
    const double h = y * w;
    const double l = __builtin_fma(y, w, -h);
    const double k = __builtin_fma(y, wq, kRound) - kRound;
    return __builtin_fma(-k, q, h) + l;
}
// x - q round(x / q): |result| <= q / 2 + 1 for |x| <= 2^52
__device__ __forceinline__ double fp_center(double x, double q, double qinv) {
#pragma clang fp contract(off)
    const double k = __builtin_fma(x, qinv, kRound) - kRound;
    return __builtin_fma(-k, q, x);
}
// x < 2^52 as a double (exact): the integer placed in the mantissa of 2^52
__device__ __forceinline__ double fp_from_u64(u64 x) {
#pragma clang fp contract(off)
    return __builtin_bit_cast(double, x | 0x4330000000000000ull) - kTwo52;
}
// integer-valued v with |v| < q to its residue in [0, q); qm = 2^52 + q
__device__ __forceinline__ u64 fp_to_residue(double v, double qm, u64 q) {
#pragma clang fp contract(off)
    const u64 u = __builtin_bit_cast(u64, v + qm) & kMant52;  // v + q, in (0, 2q)
    return csub(u, q);
}

// a wave-uniform 64-bit value held in scalar registers (frees vector
// registers for the register-resident limb)
__device__ __forceinline__ u64 uniform64(u64 x) {
    const u32 lo = __builtin_amdgcn_readfirstlane((u32)x), hi = __builtin_amdgcn_readfirstlane((u32)(x >> 32));
    return ((u64)hi << 32) | lo;
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
constexpr int kTwiddleChunk = 16;
constexpr int kTwiddleChunkFp = 8;
// the inverse stages keep more constants live: fewer barriers spill less
// (integer engine); the FP64 inverse stays spill-free with half as many
constexpr int kTwiddleChunkInv = 16;
constexpr int kTwiddleChunkInvFp = 8;
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
    // tm: twiddle-table multiplier. A full transform reads stage s's
    // twiddles at tw[2^s + group] (tm = 1); half h of a transform of twice
    // the size, after its first stage, is a transform of this size whose
    // stage s reads tw[(2 + h) 2^s + group] of the larger table (tm = 2 + h).
    template <int P, int D>
    static __device__ __forceinline__ void fwd_stage(u64 (&r)[E], u32 tid, const ulonglong2 *__restrict__ tw,
                                                     u64 q, u32 tm) {
        constexpr int w = width(P), s0 = P * LOGE, half = 1 << (w - 1 - D);
        const u64 two_q = q << 1;
#pragma unroll
        for (int b = 0; b < E / 2; b++) {
            const int g = b >> (w - 1);
            const int bl = b & ((1 << (w - 1)) - 1);
            const int c = ((bl >> (w - 1 - D)) << (w - D)) | (bl & (half - 1));
            const u32 hi = group_hi(P, tid, g);
            const int x = g * (1 << w) + c, y = x + half;
            const u32 ti = (tm << (s0 + D)) + (hi << D) + (u32)(c >> (w - D));
            const ulonglong2 W = tw[ti];
            u64 X = r[x];
            X = X >= two_q ? X - two_q : X;
            const u64 Tm = shoup_lazy(r[y], W.x, W.y, q);
            r[x] = X + Tm;
            r[y] = X - Tm + two_q;
            if ((b & (kTwiddleChunk - 1)) == kTwiddleChunk - 1) __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (D + 1 < w) fwd_stage<P, D + 1>(r, tid, tw, q, tm);
    }
    template <int P>
    static __device__ __forceinline__ void fwd_phase(u64 (&r)[E], u32 *lds, u32 tid,
                                                     const ulonglong2 *__restrict__ tw, u64 q, u32 tm) {
        if constexpr (P > 0) exchange<P - 1, P>(r, lds, tid);
        fwd_stage<P, 0>(r, tid, tw, q, tm);
        if constexpr (P + 1 < NPH) fwd_phase<P + 1>(r, lds, tid, tw, q, tm);
    }

    // forward: natural order in, "slot k = a(psi^(2brv(k)+1))" out, stage s
    // (2^s groups, half-size N >> (s+1)) multiplies by tw[2^s + group].
    // Inputs in [0, q) in the coalesced layout; outputs fully reduced.
    static __device__ __forceinline__ void forward(u64 (&r)[E], u32 *lds, u32 tid, const ulonglong2 *__restrict__ tw,
                                                   u64 q, u32 tm = 1) {
        fwd_phase<0>(r, lds, tid, tw, q, tm);
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
            if ((b & (kTwiddleChunkInv - 1)) == kTwiddleChunkInv - 1) __builtin_amdgcn_sched_barrier(0);
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

    // ---- the same transforms in FP64 arithmetic (q < 2^50), same stage
    // order, twiddle indices and data movement; residues are signed
    // integer-valued doubles between the stages.
    template <int PF, int PT>
    static __device__ __forceinline__ void exchange_f(double (&d)[E], u32 *lds, u32 tid) {
        u64 t[E];
#pragma unroll
        for (int k = 0; k < E; k++) t[k] = __builtin_bit_cast(u64, d[k]);
        exchange<PF, PT>(t, lds, tid);
#pragma unroll
        for (int k = 0; k < E; k++) d[k] = __builtin_bit_cast(double, t[k]);
    }

    // Forward stage s: (X, Y) -> (X + W Y, X - W Y). With centred twiddles
    // |W Y mod q| <= q (1/2 + |Y| 2^-54), so the magnitude bound grows by at
    // most 0.63 q per stage; X is re-centred (|X| <= q/2 + 1) on stages
    // s = 2 mod 3, so with inputs below q every value stays below 2.4 q
    // < 2^52 (the multiplier's input range) and every sum is exact.
    template <int P, int D>
    static __device__ __forceinline__ void fwd_stage_f(double (&r)[E], u32 tid, const double2 *__restrict__ tw,
                                                       double q, double qinv, u32 tm) {
#pragma clang fp contract(off)
        constexpr int w = width(P), s0 = P * LOGE, half = 1 << (w - 1 - D);
        constexpr bool recentre = ((s0 + D) % 3) == 2;
#pragma unroll
        for (int b = 0; b < E / 2; b++) {
            const int g = b >> (w - 1);
            const int bl = b & ((1 << (w - 1)) - 1);
            const int c = ((bl >> (w - 1 - D)) << (w - D)) | (bl & (half - 1));
            const u32 hi = group_hi(P, tid, g);
            const int x = g * (1 << w) + c, y = x + half;
            const u32 ti = (tm << (s0 + D)) + (hi << D) + (u32)(c >> (w - D));
            const double2 W = tw[ti];
            double X = r[x];
            if constexpr (recentre) X = fp_center(X, q, qinv);
            const double Tm = fp_mulmod(r[y], W.x, W.y, q);
            r[x] = X + Tm;
            r[y] = X - Tm;
            if ((b & (kTwiddleChunkFp - 1)) == kTwiddleChunkFp - 1) __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (D + 1 < w) fwd_stage_f<P, D + 1>(r, tid, tw, q, qinv, tm);
    }
    template <int P>
    static __device__ __forceinline__ void fwd_phase_f(double (&r)[E], u32 *lds, u32 tid,
                                                       const double2 *__restrict__ tw, double q, double qinv, u32 tm) {
        if constexpr (P > 0) exchange_f<P - 1, P>(r, lds, tid);
        fwd_stage_f<P, 0>(r, tid, tw, q, qinv, tm);
        if constexpr (P + 1 < NPH) fwd_phase_f<P + 1>(r, lds, tid, tw, q, qinv, tm);
    }
    // forward() for q < 2^50: inputs in [0, q), outputs fully reduced
    static __device__ __forceinline__ void forward_fp(u64 (&r)[E], u32 *lds, u32 tid,
                                                      const double2 *__restrict__ tw, const PrimeConst &pc,
                                                      u32 tm = 1) {
        double d[E];
#pragma unroll
        for (int k = 0; k < E; k++) d[k] = fp_from_u64(r[k]);
        forward_fpd(d, r, lds, tid, tw, pc, tm);
    }
    // the same from integer-valued doubles with |d| < 2q; residues to r
    static __device__ __forceinline__ void forward_fpd(double (&d)[E], u64 (&r)[E], u32 *lds, u32 tid,
                                                       const double2 *__restrict__ tw, const PrimeConst &pc,
                                                       u32 tm = 1) {
        fwd_phase_f<0>(d, lds, tid, tw, pc.qf, pc.qinvf, tm);
        exchange_f<NPH - 1, 0>(d, lds, tid);
#pragma unroll
        for (int k = 0; k < E; k++) r[k] = fp_to_residue(fp_center(d[k], pc.qf, pc.qinvf), pc.qmf, pc.q);
    }

    // Inverse stage s: (X, Y) -> (X + Y, (X - Y) W^-1); the sum is re-centred
    // on every second stage executed, so inputs stay below 2q and
    // differences below 4q. The last stage multiplies both outputs
    // (by centred N^-1 and W^-1 N^-1), leaving |.| <= q (1/2 + 4q 2^-54) < q.
    template <int P, int D>
    static __device__ __forceinline__ void inv_stage_f(double (&r)[E], u32 tid, const double2 *__restrict__ itw,
                                                       const PrimeConst &pc) {
#pragma clang fp contract(off)
        constexpr int w = width(P), s0 = P * LOGE, half = 1 << (w - 1 - D);
        constexpr bool last = (s0 + D) == 0;
        constexpr bool recentre = ((LOGN - 1 - (s0 + D)) & 1) == 1;
        const double q = pc.qf;
#pragma unroll
        for (int b = 0; b < E / 2; b++) {
            const int g = b >> (w - 1);
            const int bl = b & ((1 << (w - 1)) - 1);
            const int c = ((bl >> (w - 1 - D)) << (w - D)) | (bl & (half - 1));
            const u32 hi = group_hi(P, tid, g);
            const int x = g * (1 << w) + c, y = x + half;
            const double X = r[x], Y = r[y];
            if constexpr (last) {
                r[x] = fp_mulmod(X + Y, pc.ninvf, pc.ninvqf, q);
                r[y] = fp_mulmod(X - Y, pc.last_wf, pc.last_wqf, q);
            } else {
                const u32 ti = (1u << (s0 + D)) + (hi << D) + (u32)(c >> (w - D));
                const double2 W = itw[ti];
                const double U = X + Y;
                r[x] = recentre ? fp_center(U, q, pc.qinvf) : U;
                r[y] = fp_mulmod(X - Y, W.x, W.y, q);
            }
            if ((b & (kTwiddleChunkInvFp - 1)) == kTwiddleChunkInvFp - 1) __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (D > 0) inv_stage_f<P, D - 1>(r, tid, itw, pc);
    }
    template <int P>
    static __device__ __forceinline__ void inv_phase_f(double (&r)[E], u32 *lds, u32 tid,
                                                       const double2 *__restrict__ itw, const PrimeConst &pc) {
        if constexpr (P < NPH - 1) exchange_f<P + 1, P>(r, lds, tid);
        inv_stage_f<P, width(P) - 1>(r, tid, itw, pc);
        if constexpr (P > 0) inv_phase_f<P - 1>(r, lds, tid, itw, pc);
    }
    // inverse() for q < 2^50: inputs in [0, q), outputs fully reduced
    static __device__ __forceinline__ void inverse_fp(u64 (&r)[E], u32 *lds, u32 tid,
                                                      const double2 *__restrict__ itw, const PrimeConst &pc) {
        double d[E];
#pragma unroll
        for (int k = 0; k < E; k++) d[k] = fp_from_u64(r[k]);
        inverse_fpd(d, r, lds, tid, itw, pc);
    }
    // the same from integer-valued doubles with |d| <= q; residues to r
    static __device__ __forceinline__ void inverse_fpd(double (&d)[E], u64 (&r)[E], u32 *lds, u32 tid,
                                                       const double2 *__restrict__ itw, const PrimeConst &pc) {
        exchange_f<0, NPH - 1>(d, lds, tid);
        inv_phase_f<NPH - 1>(d, lds, tid, itw, pc);
#pragma unroll
        for (int k = 0; k < E; k++) r[k] = fp_to_residue(d[k], pc.qmf, pc.q);
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
    // the same operations with a digit size (ModUp) or special-prime count
    // (ModDown + rescale) fixed at compile time: fully unrolled conversions
    // keep the transform register-resident (no spills)
    F_MODUP_S1 = 8, F_MODUP_S2 = 9, F_MODUP_S3 = 10, F_MODUP_S4 = 11,
    F_RELIN_P1 = 12, F_RELIN_P2 = 13, F_RELIN_RS_P1 = 14, F_RELIN_RS_P2 = 15,
    F_MODDOWN_P1 = 16, F_MODDOWN_P2 = 17,  // F_MODDOWN with 1 or 2 special primes
};
__host__ __device__ constexpr bool is_modup(int op) { return op == F_MODUP || (op >= F_MODUP_S1 && op <= F_MODUP_S4); }
__host__ __device__ constexpr int modup_s(int op) { return op >= F_MODUP_S1 && op <= F_MODUP_S4 ? op - F_MODUP_S1 + 1 : 0; }
__host__ __device__ constexpr bool is_relin_rs(int op) { return op == F_RELIN_RS || op == F_RELIN_RS_P1 || op == F_RELIN_RS_P2; }
__host__ __device__ constexpr bool is_relin(int op) { return op == F_RELIN || op == F_RELIN_P1 || op == F_RELIN_P2 || is_relin_rs(op); }
__host__ __device__ constexpr bool is_moddown(int op) { return op == F_MODDOWN || op == F_MODDOWN_P1 || op == F_MODDOWN_P2; }
__host__ __device__ constexpr int moddown_np(int op) { return op == F_MODDOWN_P1 ? 1 : op == F_MODDOWN_P2 ? 2 : 0; }
__host__ __device__ constexpr int relin_np(int op) {
    return op == F_RELIN_P1 || op == F_RELIN_RS_P1 ? 1 : op == F_RELIN_P2 || op == F_RELIN_RS_P2 ? 2 : 0;
}
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

// One work item of k_fwd; FP selects the transform's arithmetic. The whole
// item (prologue, transform, epilogue) is instantiated per engine so no
// register assignment has to be shared across the two.
template <int LOGN, int LOGE, int OP, bool FP>
__device__ __forceinline__ void fwd_item(const DevTables &tb, const Item &it, u32 *lds, u64 seed) {
    using NT = Ntt<LOGN, LOGE>;
    constexpr int N = NT::N, E = NT::E, T = NT::T;
    const u32 tid = threadIdx.x, vo = tid * 8;
    const PrimeConst pc = tb.pc[it.prime];
    const u64 q = pc.q;
    u64 r[E];

    // ---- prologue: residues of the polynomial to transform (coefficients)
    // FP64 ModUp / ModDown + rescale: the conversion sum stays in doubles
    // and feeds the transform
    constexpr bool kFpModup = FP && is_modup(OP);
    constexpr bool kFpRelin = FP && is_relin(OP);
    double d[kFpModup || kFpRelin ? E : 1];
    if constexpr (OP == F_COPY) {
#pragma unroll
        for (int c = 0; c < E; c++) r[c] = Buf(it.in[0]).ld(vo, c * T * 8);
    } else if constexpr (kFpModup) {
        // sum_i src_i (hat_i mod t) with the target t below 2^50 (and, at
        // N = 2^15 or for a fixed digit size above one, every source
        // prime): each term is an FP64
        // modular product of magnitude
        // <= 0.75 t (its quotient from hat_i * (1/t), relative error
        // <= 2^-52); partial sums are re-centred every four terms and at the
        // end, so the transform starts from |d| <= t/2 + 1
#pragma clang fp contract(off)
        constexpr int S = modup_s(OP);
        const u32 s = S ? (u32)S : it.b;
        const u64 *blk = tb.modup + (size_t)(it.c * tb.alpha + s - 1) * modup_block_words(tb.alpha, tb.n_prim);
        const u64 *hat = blk + 2 * tb.alpha + it.prime;
        const Buf src(it.in[0]);
        const double t = pc.qf, tinv = pc.qinvf;
#pragma unroll
        for (int c = 0; c < E; c++) d[c] = 0.0;
        auto term = [&](u32 i) {
            const u64 hh = hat[i * tb.n_prim];
            const double h = fp_from_u64(hh);
            const double hq = h * tinv;
            // below 2^15, generic and one-prime-digit kernels: a source
            // prime of 2^50 or more (a 60-bit base prime) enters as
            // hi 2^26 + lo, two products (<= 0.5 t each)
            if constexpr (LOGN <= 14 && S <= 1) {
                if (tb.pc[it.c * tb.alpha + i].q >= kFpPrimeBound) {
                    constexpr int kSC = kConvChunk / 2;
                    const double h26 = fp_from_u64(mulm(hh, 1ull << 26, pc)), h26q = h26 * tinv;
#pragma unroll
                    for (int c0 = 0; c0 < E; c0 += kSC) {
                        u64 y[kSC];
#pragma unroll
                        for (int c = 0; c < kSC; c++) y[c] = src.ld(vo, (i * N + (c0 + c) * T) * 8);
#pragma unroll
                        for (int c = 0; c < kSC; c++) {
                            const double hi = fp_from_u64(y[c] >> 26), lo = fp_from_u64(y[c] & ((1ull << 26) - 1));
                            d[c0 + c] = d[c0 + c] + (fp_mulmod(hi, h26, h26q, t) + fp_mulmod(lo, h, hq, t));
                            if ((i & 3) == 3) d[c0 + c] = fp_center(d[c0 + c], t, tinv);
                        }
                    }
                    return;
                }
            }
#pragma unroll
            for (int c0 = 0; c0 < E; c0 += kConvChunk) {
                double x[kConvChunk];
#pragma unroll
                for (int c = 0; c < kConvChunk; c++) x[c] = fp_from_u64(src.ld(vo, (i * N + (c0 + c) * T) * 8));
#pragma unroll
                for (int c = 0; c < kConvChunk; c++) {
                    d[c0 + c] = d[c0 + c] + fp_mulmod(x[c], h, hq, t);
                    if ((i & 3) == 3) d[c0 + c] = fp_center(d[c0 + c], t, tinv);
                }
            }
        };
        if constexpr (S > 0) {
#pragma unroll
            for (int i = 0; i < S; i++) term((u32)i);
        } else {
            for (u32 i = 0; i < s; i++) term(i);
        }
#pragma unroll
        for (int c = 0; c < E; c++) d[c] = fp_center(d[c], t, tinv);
    } else if constexpr (is_modup(OP)) {
        // sources arrive as [x_i hat_i^-1]_{q_i}: sum_i src_i (hat_i mod t), one Barrett at the end
        constexpr int S = modup_s(OP);  // 0: digit size from the item
        const u32 s = S ? (u32)S : it.b;
        const u64 *blk = tb.modup + (size_t)(it.c * tb.alpha + s - 1) * modup_block_words(tb.alpha, tb.n_prim);
        const u64 *hat = blk + 2 * tb.alpha + it.prime;  // hat[i * n_prim + t]
        const Buf src(it.in[0]);
        constexpr int kCC = E >= 32 ? 4 : kConvChunk;
        static_for<0, E / kCC>([&](auto C0) {
            constexpr int c0 = decltype(C0)::value * kCC;
            Acc128 acc[kCC];
            auto term = [&](u32 i) {
                const u64 h = hat[i * tb.n_prim];
#pragma unroll
                for (int c = 0; c < kCC; c++) acc[c].mac(src.ld(vo, (i * N + (c0 + c) * T) * 8), h);
            };
            if constexpr (S > 0) {
#pragma unroll
                for (int i = 0; i < S; i++) term((u32)i);
            } else {
                for (u32 i = 0; i < s; i++) term(i);
            }
#pragma unroll
            for (int c = 0; c < kCC; c++) r[c0 + c] = acc[c].reduce(pc);
        });
    } else if constexpr (is_moddown(OP)) {
        // sum_m [x_m * hat_m^-1]_{p_m} * (hat_m mod t), one Barrett at the end
        constexpr int NP = moddown_np(OP);  // 0: count from the item
        const u32 lo = it.a, s = NP ? (u32)NP : it.b;  // first source prime index, count
        const u64 *blk = tb.moddown;
        const u64 *hat = blk + 2 * tb.n_p + it.prime;  // hat[m * n_q + t]
        const Buf src(it.in[0]);
        constexpr int kCC = E >= 32 ? 4 : kConvChunk;
        static_for<0, E / kCC>([&](auto C0) {
            constexpr int c0 = decltype(C0)::value * kCC;
            Acc128 acc[kCC];
            for (u32 i = 0; i < s; i++) {
                const u64 inv = blk[2 * i], inv_sh = blk[2 * i + 1], qi = tb.pc[lo + i].q, h = hat[i * tb.n_q];
#pragma unroll
                for (int c = 0; c < kCC; c++) acc[c].mac(shoup(src.ld(vo, (i * N + (c0 + c) * T) * 8), inv, inv_sh, qi), h);
            }
#pragma unroll
            for (int c = 0; c < kCC; c++) r[c0 + c] = acc[c].reduce(pc);
        });
    } else if constexpr (kFpRelin) {
        // z = conv_i(y) P^-1 + [t]_centred with q_i and q_l below 2^50. A
        // special-prime residue y_m (up to 61 bits) enters as
        // hi 2^26 + lo: hi (2^26 hat_m mod q_i) + lo hat_m, two FP64 modular
        // products of magnitude <= q_i (0.5 + 2^-16); the sum is re-centred
        // every two special primes and before the P^-1 product
#pragma clang fp contract(off)
        const PrimeConst pl = tb.pc[it.a];  // q_l
        const u64 hl = pl.q >> 1;
        const double hlf = fp_from_u64(hl);
        const u64 *hat = tb.moddown + 2 * tb.n_p + it.prime;  // hat[m * n_q]: P/p_m mod q_i
        const Buf ys(it.in[0]), ts(it.in[1]);
        constexpr int NP = relin_np(OP);
        const double qf = pc.qf, qinv = pc.qinvf;
        const double pv = fp_from_u64(pc.pinv), pvq = pv * qinv;
#pragma unroll
        for (int c = 0; c < E; c++) d[c] = 0.0;
        auto term = [&](u32 m) {
            const u64 h = hat[(size_t)m * tb.n_q];
            const double hd = fp_from_u64(h), hq = hd * qinv;
            const double hd26 = fp_from_u64(mulm(h, 1ull << 26, pc)), hq26 = hd26 * qinv;
#pragma unroll
            for (int c0 = 0; c0 < E; c0 += kConvChunk) {
                u64 y[kConvChunk];
#pragma unroll
                for (int c = 0; c < kConvChunk; c++) y[c] = ys.ld(vo, (m * N + (c0 + c) * T) * 8);
#pragma unroll
                for (int c = 0; c < kConvChunk; c++) {
                    const double hi = fp_from_u64(y[c] >> 26), lo = fp_from_u64(y[c] & ((1ull << 26) - 1));
                    d[c0 + c] = d[c0 + c] + (fp_mulmod(hi, hd26, hq26, qf) + fp_mulmod(lo, hd, hq, qf));
                    if (m & 1) d[c0 + c] = fp_center(d[c0 + c], qf, qinv);
                }
            }
        };
        if constexpr (NP > 0) {
#pragma unroll
            for (int m = 0; m < NP; m++) term((u32)m);
        } else {
            for (u32 m = 0; m < tb.n_p; m++) term(m);
        }
#pragma unroll
        for (int c = 0; c < E; c++) {
            const double z = fp_mulmod(fp_center(d[c], qf, qinv), pv, pvq, qf);  // |z| < q_i
            const double tc = fp_from_u64(addm(ts.ld(vo, c * T * 8), hl, pl.q)) - hlf;  // |tc| <= q_l / 2
            d[c] = fp_center(z + tc, qf, qinv);
        }
    } else if constexpr (is_relin(OP)) {
        const PrimeConst pl = tb.pc[it.a];  // q_l
        const u64 hl = pl.q >> 1;
        const u64 *hat = tb.moddown + 2 * tb.n_p + it.prime;  // hat[m * n_q]: P/p_m mod q_i
        const Buf ys(it.in[0]), ts(it.in[1]);
        constexpr int NP = relin_np(OP);  // 0: count from the tables
        constexpr int kCC = E >= 32 ? 4 : kConvChunk;
        static_for<0, E / kCC>([&](auto C0) {
            constexpr int c0 = decltype(C0)::value * kCC;
            Acc128 acc[kCC];
            auto term = [&](u32 m) {
                const u64 h = hat[(size_t)m * tb.n_q];
#pragma unroll
                for (int c = 0; c < kCC; c++) acc[c].mac(ys.ld(vo, (m * N + (c0 + c) * T) * 8), h);
            };
            if constexpr (NP > 0) {
#pragma unroll
                for (int m = 0; m < NP; m++) term((u32)m);
            } else {
                for (u32 m = 0; m < tb.n_p; m++) term(m);
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

    if constexpr (kFpModup || kFpRelin)
        NT::forward_fpd(d, r, lds, tid, tb.twf + (size_t)it.prime * N, pc);
    else if constexpr (FP)
        NT::forward_fp(r, lds, tid, tb.twf + (size_t)it.prime * N, pc);
    else
        NT::forward(r, lds, tid, tb.tw + (size_t)it.prime * N, q);

    // ---- epilogue
    if constexpr (OP == F_COPY || is_modup(OP) || OP == F_SAMPLE || OP == F_INT || (is_relin(OP) && !is_relin_rs(OP))) {
#pragma unroll
        for (int c = 0; c < E; c++) Buf(it.out).st(vo, c * T * 8, r[c]);
    } else if constexpr (OP == F_RESCALE) {
        // it.v: a signed constant added to every slot after the division
        // (a scalar at the output scale on the first polynomial; 0: none)
        const ulonglong2 qi = tb.rescale[(size_t)it.a * tb.n_q + it.prime];
        const u64 add = it.v ? uniform64(reduce_signed(it.v, pc)) : 0;
        const Buf in1(it.in[1]), dst(it.out);
#pragma unroll
        for (int c0 = 0; c0 < E; c0 += kEpiChunk) {
            u64 x[kEpiChunk];
#pragma unroll
            for (int c = 0; c < kEpiChunk; c++) x[c] = in1.ld(vo, (c0 + c) * T * 8);
#pragma unroll
            for (int c = 0; c < kEpiChunk; c++)
                dst.st(vo, (c0 + c) * T * 8, addm(shoup(subm(x[c], r[c0 + c], q), qi.x, qi.y, q), add, q));
        }
    } else if constexpr (is_relin_rs(OP) && FP) {
        // y = (acc' P^-1 - z) q_l^-1 in FP64: |acc' P^-1| < q, |. - z| < 2q,
        // |(.) q_l^-1| < q (multipliers' ratios to q from 1/q, error <= 2^-52)
#pragma clang fp contract(off)
        const ulonglong2 qi = tb.rescale[(size_t)it.a * tb.n_q + it.prime];
        const double qf = pc.qf, qinv = pc.qinvf;
        const double pv = fp_from_u64(pc.pinv), pvq = pv * qinv;
        const double lv = fp_from_u64(qi.x), lvq = lv * qinv;
        const Buf accb(it.in[2]), dst(it.out);
        constexpr int kRC = 4;
#pragma unroll
        for (int c0 = 0; c0 < E; c0 += kRC) {
            u64 x[kRC];
#pragma unroll
            for (int c = 0; c < kRC; c++) x[c] = accb.ld(vo, (c0 + c) * T * 8);
#pragma unroll
            for (int c = 0; c < kRC; c++) {
                const double u = fp_mulmod(fp_from_u64(x[c]), pv, pvq, qf);
                const double w = fp_mulmod(u - fp_from_u64(r[c0 + c]), lv, lvq, qf);
                dst.st(vo, (c0 + c) * T * 8, fp_to_residue(w, pc.qmf, q));
            }
        }
    } else if constexpr (is_relin_rs(OP)) {
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
    } else if constexpr (is_moddown(OP)) {
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

// Waves per SIMD the transform kernels are built for. A workgroup of 2^14
// or 2^13 residues with 32 per thread (8 or 4 waves) whose register count
// would exceed 128 — the inverse transforms, the ModUp / ModDown
// conversions and the rescale — is held to 128 VGPRs, so that two (four) of
// them share a CU and one's memory phases overlap another's arithmetic
// (measured: the 8192-image vision network's ModUp 5.3 -> 4.3 ms, product +
// INTT 1.0 -> 0.8 ms, despite small spills); the other forward kernels fit
// in 128 already and keep the compiler's schedule, as do all other shapes.
template <int LOGN, int LOGE, bool INV, int OP>
constexpr int kWavesPerEu =
    ((LOGN == 14 || LOGN == 13) && LOGE == 5 && (INV || is_modup(OP) || is_moddown(OP) || OP == F_RESCALE)) ? 4
                                                                                                              : 1;

// FP: every item's prime is below 2^50 and the transforms run in FP64
// arithmetic (the host splits a launch by prime class); else 64-bit integer
template <int LOGN, int LOGE, int OP, bool FP>
__global__ void __launch_bounds__(1 << (LOGN - LOGE)) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<LOGN, LOGE, false, OP>)))
k_fwd(DevTables tb, const Item *__restrict__ items, int nitems, u64 seed) {
    __shared__ u32 lds[Ntt<LOGN, LOGE>::LDS_WORDS];
    const int iid = xcd_item(nitems, tb.xcd_remap);
    if (iid < 0) return;
    const Item it = items[iid];
    fwd_item<LOGN, LOGE, OP, FP>(tb, it, lds, seed);
}

// One work item of k_inv (see fwd_item).
template <int LOGN, int LOGE, int OP, bool FP>
__device__ __forceinline__ void inv_item(const DevTables &tb, const Item &it, u32 *lds) {
    using NT = Ntt<LOGN, LOGE>;
    constexpr int N = NT::N, E = NT::E, T = NT::T;
    const u32 tid = threadIdx.x, vo = tid * 8;
    const PrimeConst pc = tb.pc[it.prime];
    const u64 q = pc.q;
    u64 r[E];

    // FP64 product: x y - k q with k the integer nearest to fl(x y) (1/q),
    // |k - x y / q| <= 0.75 for x, y < q < 2^50, so |d| <= 0.75 q, exactly
    constexpr bool kFpMul = FP && OP == I_MUL;
    double d[kFpMul ? E : 1];
    // the epilogue's constant multiplier (same for the whole item), read
    // before the transform into scalar registers
    u64 inv = 0, inv_sh = 0;
    if constexpr (OP == I_SCALE) {
        // b == 0: hat_m^-1 mod p_m for special prime m = a; b == 1: P^-1 mod q;
        // b == 2: hat_i^-1 of ModUp digit block c, position a (a ModUp source)
        const u64 *blk = tb.modup + (size_t)it.c * modup_block_words(tb.alpha, tb.n_prim);
        inv = uniform64(it.b == 1 ? pc.pinv : it.b == 2 ? blk[2 * it.a] : tb.moddown[2 * it.a]);
        inv_sh = uniform64(it.b == 1 ? pc.pinv_sh : it.b == 2 ? blk[2 * it.a + 1] : tb.moddown[2 * it.a + 1]);
    } else if constexpr (OP == I_MUL) {
        // it.v == 1: the ModUp source factor hat_i^-1 (digit block it.c, position it.a)
        if (it.v == 1) {
            const u64 *blk = tb.modup + (size_t)it.c * modup_block_words(tb.alpha, tb.n_prim);
            inv = uniform64(blk[2 * it.a]);
            inv_sh = uniform64(blk[2 * it.a + 1]);
        }
    }
    if constexpr (OP == I_COPY || OP == I_SCALE) {
#pragma unroll
        for (int c = 0; c < E; c++) r[c] = Buf(it.in[0]).ld(vo, c * T * 8);
    } else if constexpr (kFpMul) {
#pragma clang fp contract(off)
        const double qf = pc.qf, qinv = pc.qinvf;
#pragma unroll
        for (int c = 0; c < E; c++) {
            const double x = fp_from_u64(Buf(it.in[0]).ld(vo, c * T * 8));
            const double y = fp_from_u64(Buf(it.in[1]).ld(vo, c * T * 8));
            const double h = x * y;
            const double l = __builtin_fma(x, y, -h);
            const double k = __builtin_fma(h, qinv, kRound) - kRound;
            d[c] = __builtin_fma(-k, qf, h) + l;
        }
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

    if constexpr (kFpMul)
        NT::inverse_fpd(d, r, lds, tid, tb.itwf + (size_t)it.prime * N, pc);
    else if constexpr (FP)
        NT::inverse_fp(r, lds, tid, tb.itwf + (size_t)it.prime * N, pc);
    else
        NT::inverse(r, lds, tid, tb.itw + (size_t)it.prime * N, pc);

    if constexpr (OP == I_MUL) {
        // it.v == 1: store [x * hat_i^-1]_{q_i}, the ModUp input (digit block it.c, position it.a)
        if (it.v == 1) {
#pragma unroll
            for (int c = 0; c < E; c++) r[c] = shoup(r[c], inv, inv_sh, q);
        }
    } else if constexpr (OP == I_SCALE) {
#pragma unroll
        for (int c = 0; c < E; c++) r[c] = shoup(r[c], inv, inv_sh, q);
    }
#pragma unroll
    for (int c = 0; c < E; c++) Buf(it.out).st(vo, c * T * 8, r[c]);
}
template <int LOGN, int LOGE, int OP, bool FP>
__global__ void __launch_bounds__(1 << (LOGN - LOGE)) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<LOGN, LOGE, true, OP>)))
k_inv(DevTables tb, const Item *__restrict__ items, int nitems) {
    __shared__ u32 lds[Ntt<LOGN, LOGE>::LDS_WORDS];
    const int iid = xcd_item(nitems, tb.xcd_remap);
    if (iid < 0) return;
    const Item it = items[iid];
    inv_item<LOGN, LOGE, OP, FP>(tb, it, lds);
}

// ---------------------------------------------------------------------
// Transforms of N = 2^LOGN residues that one workgroup cannot hold in
// registers (N = 2^16), in two in-place passes over the limb:
//   forward: (A) the first stage, which pairs j with j + N/2 under the one
//            twiddle tw[1], as a streaming pass; (B) each half is then a
//            transform of N/2 whose stage s reads tw[(2 + h) 2^s + group]
//            (one workgroup per half h);
//   inverse: (A) the first inverse stage, which pairs 2i with 2i + 1 under
//            itw[N/2 + i], as a streaming pass; (B) each parity class is
//            then an inverse transform of N/2 with the same table indices
//            and the N^-1 merge of the full transform (one workgroup per
//            class, every other word of the limb).
// Only the copy prologue / epilogue (plain NTT / INTT of limbs).
// ---------------------------------------------------------------------
constexpr int kPairsPerThread = 4, kPairThreads = 256;
template <bool FP, bool INV>
__global__ void __launch_bounds__(kPairThreads) k_first_stage(DevTables tb, const Item *__restrict__ items, int nitems) {
    const u32 N = 1u << tb.log_n, H = N >> 1;
    const u32 per = H / (kPairThreads * kPairsPerThread);  // blocks per limb
    const u32 b = blockIdx.x, item = b / per;
    if ((int)item >= nitems) return;
    const Item it = items[item];
    const PrimeConst pc = tb.pc[it.prime];
    u64 *a = it.out;
    const u32 base = (b % per) * (kPairThreads * kPairsPerThread) + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kPairsPerThread; k++) {
        const u32 j = base + k * kPairThreads;
        // forward: (j, j + N/2); inverse: (2j, 2j + 1)
        const u32 ix = INV ? 2 * j : j, iy = INV ? 2 * j + 1 : j + H;
        const u64 X = a[ix], Y = a[iy];
        u64 x2, y2;
        if constexpr (FP) {
#pragma clang fp contract(off)
            const double xd = fp_from_u64(X), yd = fp_from_u64(Y);
            if constexpr (INV) {
                const double2 W = tb.itwf[(size_t)it.prime * N + H + j];
                x2 = fp_to_residue(fp_center(xd + yd, pc.qf, pc.qinvf), pc.qmf, pc.q);
                y2 = fp_to_residue(fp_mulmod(xd - yd, W.x, W.y, pc.qf), pc.qmf, pc.q);
            } else {
                const double2 W = tb.twf[(size_t)it.prime * N + 1];
                const double t = fp_mulmod(yd, W.x, W.y, pc.qf);
                x2 = fp_to_residue(fp_center(xd + t, pc.qf, pc.qinvf), pc.qmf, pc.q);
                y2 = fp_to_residue(fp_center(xd - t, pc.qf, pc.qinvf), pc.qmf, pc.q);
            }
        } else {
            if constexpr (INV) {
                const ulonglong2 W = tb.itw[(size_t)it.prime * N + H + j];
                x2 = addm(X, Y, pc.q);
                y2 = shoup(subm(X, Y, pc.q), W.x, W.y, pc.q);
            } else {
                const ulonglong2 W = tb.tw[(size_t)it.prime * N + 1];
                const u64 t = shoup(Y, W.x, W.y, pc.q);
                x2 = addm(X, t, pc.q);
                y2 = subm(X, t, pc.q);
            }
        }
        a[ix] = x2;
        a[iy] = y2;
    }
}

template <int LOGN, int LOGE, bool FP>
__global__ void __launch_bounds__(1 << (LOGN - 1 - LOGE))
k_fwd_halves(DevTables tb, const Item *__restrict__ items, int nitems) {
    using NT = Ntt<LOGN - 1, LOGE>;
    constexpr int N = 1 << LOGN, H = N / 2, E = NT::E, T = NT::T;
    __shared__ u32 lds[NT::LDS_WORDS];
    const int wid = xcd_item(2 * nitems, tb.xcd_remap);
    if (wid < 0) return;
    const Item it = items[wid >> 1];
    const u32 h = (u32)(wid & 1), tid = threadIdx.x, vo = tid * 8;
    const PrimeConst pc = tb.pc[it.prime];
    const Buf buf(it.out + (size_t)h * H);
    u64 r[E];
#pragma unroll
    for (int c = 0; c < E; c++) r[c] = buf.ld(vo, c * T * 8);
    if constexpr (FP)
        NT::forward_fp(r, lds, tid, tb.twf + (size_t)it.prime * N, pc, 2 + h);
    else
        NT::forward(r, lds, tid, tb.tw + (size_t)it.prime * N, pc.q, 2 + h);
#pragma unroll
    for (int c = 0; c < E; c++) buf.st(vo, c * T * 8, r[c]);
}

template <int LOGN, int LOGE, bool FP>
__global__ void __launch_bounds__(1 << (LOGN - 1 - LOGE))
k_inv_classes(DevTables tb, const Item *__restrict__ items, int nitems) {
    using NT = Ntt<LOGN - 1, LOGE>;
    constexpr int N = 1 << LOGN, E = NT::E, T = NT::T;
    __shared__ u32 lds[NT::LDS_WORDS];
    const int wid = xcd_item(2 * nitems, tb.xcd_remap);
    if (wid < 0) return;
    const Item it = items[wid >> 1];
    const u32 p = (u32)(wid & 1), tid = threadIdx.x, vo = tid * 16 + p * 8;  // class element i at word 2i + p
    const PrimeConst pc = tb.pc[it.prime];
    const Buf buf(it.out);
    u64 r[E];
#pragma unroll
    for (int c = 0; c < E; c++) r[c] = buf.ld(vo, c * T * 16);
    if constexpr (FP)
        NT::inverse_fp(r, lds, tid, tb.itwf + (size_t)it.prime * N, pc);
    else
        NT::inverse(r, lds, tid, tb.itw + (size_t)it.prime * N, pc);
#pragma unroll
    for (int c = 0; c < E; c++) buf.st(vo, c * T * 16, r[c]);
}

// ---------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------
// tb.ntt_fp set: the launch's items all have primes below 2^50 (FP64 engine)
template <int LOGN, int LOGE, int OP>
static hipError_t launch_fwd_t(const DevTables &tb, const Item *items, int n, u64 seed, hipStream_t s) {
    if (tb.ntt_fp)
        hipLaunchKernelGGL((k_fwd<LOGN, LOGE, OP, true>), dim3(xcd_grid(n)), dim3(Ntt<LOGN, LOGE>::T), 0, s, tb,
                           items, n, seed);
    else
        hipLaunchKernelGGL((k_fwd<LOGN, LOGE, OP, false>), dim3(xcd_grid(n)), dim3(Ntt<LOGN, LOGE>::T), 0, s, tb,
                           items, n, seed);
    return hipGetLastError();
}
template <int LOGN, int LOGE, int OP>
static hipError_t launch_inv_t(const DevTables &tb, const Item *items, int n, hipStream_t s) {
    if (tb.ntt_fp)
        hipLaunchKernelGGL((k_inv<LOGN, LOGE, OP, true>), dim3(xcd_grid(n)), dim3(Ntt<LOGN, LOGE>::T), 0, s, tb,
                           items, n);
    else
        hipLaunchKernelGGL((k_inv<LOGN, LOGE, OP, false>), dim3(xcd_grid(n)), dim3(Ntt<LOGN, LOGE>::T), 0, s, tb,
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
// fixed-size conversion variants at N = 2^15 (32 residues per thread, where
// a runtime loop over the digit size spilled); the generic kernels take the
// same items at the other rings, except those of CKKS_FWD_FIXED_SMALL
#define CKKS_FWD_FIXED(LN, LE)                                                        \
    switch (op) {                                                                     \
        case F_MODUP_S1: return launch_fwd_t<LN, LE, F_MODUP_S1>(tb, items, n, seed, s);       \
        case F_MODUP_S2: return launch_fwd_t<LN, LE, F_MODUP_S2>(tb, items, n, seed, s);       \
        case F_MODUP_S3: return launch_fwd_t<LN, LE, F_MODUP_S3>(tb, items, n, seed, s);       \
        case F_MODUP_S4: return launch_fwd_t<LN, LE, F_MODUP_S4>(tb, items, n, seed, s);       \
        case F_RELIN_P1: return launch_fwd_t<LN, LE, F_RELIN_P1>(tb, items, n, seed, s);       \
        case F_RELIN_P2: return launch_fwd_t<LN, LE, F_RELIN_P2>(tb, items, n, seed, s);       \
        case F_RELIN_RS_P1: return launch_fwd_t<LN, LE, F_RELIN_RS_P1>(tb, items, n, seed, s); \
        case F_RELIN_RS_P2: return launch_fwd_t<LN, LE, F_RELIN_RS_P2>(tb, items, n, seed, s); \
        case F_MODDOWN_P1: return launch_fwd_t<LN, LE, F_MODDOWN_P1>(tb, items, n, seed, s);   \
        case F_MODDOWN_P2: return launch_fwd_t<LN, LE, F_MODDOWN_P2>(tb, items, n, seed, s);   \
    }
// below 2^15 (N = 2^13, 2^14); the multi-prime ModUp variants take no
// 60-bit sources in FP64 (the planner sends those items to the integer
// engine), the one-prime-digit variant splits them like the generic kernel
#define CKKS_FWD_FIXED_SMALL(LN, LE)                                                  \
    switch (op) {                                                                     \
        case F_MODUP_S1: return launch_fwd_t<LN, LE, F_MODUP_S1>(tb, items, n, seed, s);       \
        case F_MODUP_S2: return launch_fwd_t<LN, LE, F_MODUP_S2>(tb, items, n, seed, s);       \
        case F_MODUP_S3: return launch_fwd_t<LN, LE, F_MODUP_S3>(tb, items, n, seed, s);       \
        case F_MODUP_S4: return launch_fwd_t<LN, LE, F_MODUP_S4>(tb, items, n, seed, s);       \
        case F_RELIN_P1: return launch_fwd_t<LN, LE, F_RELIN_P1>(tb, items, n, seed, s);       \
        case F_RELIN_P2: return launch_fwd_t<LN, LE, F_RELIN_P2>(tb, items, n, seed, s);       \
        case F_RELIN_RS_P1: return launch_fwd_t<LN, LE, F_RELIN_RS_P1>(tb, items, n, seed, s); \
        case F_RELIN_RS_P2: return launch_fwd_t<LN, LE, F_RELIN_RS_P2>(tb, items, n, seed, s); \
        case F_MODDOWN_P1: return launch_fwd_t<LN, LE, F_MODDOWN_P1>(tb, items, n, seed, s);   \
        case F_MODDOWN_P2: return launch_fwd_t<LN, LE, F_MODDOWN_P2>(tb, items, n, seed, s);   \
    }
#define CKKS_INV_CASE(LN, LE)                                                        \
    case LN:                                                                         \
        switch (op) {                                                                \
            case I_COPY: return launch_inv_t<LN, LE, I_COPY>(tb, items, n, s);             \
            case I_MUL: return launch_inv_t<LN, LE, I_MUL>(tb, items, n, s);               \
            case I_SCALE: return launch_inv_t<LN, LE, I_SCALE>(tb, items, n, s);           \
            case I_DECRYPT: return launch_inv_t<LN, LE, I_DECRYPT>(tb, items, n, s);       \
        }                                                                            \
        break;


// per-ring launchers (one translation unit each)
hipError_t launch_fwd_15(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s);
hipError_t launch_inv_15(const DevTables &tb, int op, const Item *items, int n, hipStream_t s);
hipError_t launch_fwd_15_fixed(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s);
hipError_t launch_fwd_14(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s);
hipError_t launch_inv_14(const DevTables &tb, int op, const Item *items, int n, hipStream_t s);
hipError_t launch_fwd_13(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s);
hipError_t launch_inv_13(const DevTables &tb, int op, const Item *items, int n, hipStream_t s);
hipError_t launch_fwd_small(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s);
hipError_t launch_inv_small(const DevTables &tb, int op, const Item *items, int n, hipStream_t s);
hipError_t launch_fwd_16(const DevTables &tb, int op, const Item *items, int n, u64 seed, hipStream_t s);
hipError_t launch_inv_16(const DevTables &tb, int op, const Item *items, int n, hipStream_t s);
}  // namespace ckks
