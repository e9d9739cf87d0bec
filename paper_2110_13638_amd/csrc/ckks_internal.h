// Internal definitions shared by the host runtime (ckks_runtime.h) and the
// gfx950 kernels (ckks_kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ckks {

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;

constexpr int kMaxPrimes = 64;
constexpr int kMinLogN = 10;
constexpr int kMaxLogN = 16;
// at N = 2^16 a limb does not fit one workgroup: plain transforms (two
// passes) and element-wise operations only
constexpr int kMaxFusedLogN = 15;

// Per-prime constants (one entry per prime index: data primes, then the
// special primes).
struct PrimeConst {
    u64 q;
    u64 two_q;
    u64 br_hi, br_lo;  // floor(2^128 / q) as two words (128-bit Barrett)
    u64 mu;            // floor(2^64 / q) (64-bit Barrett)
    u64 ninv, ninv_sh;     // N^-1 mod q with its Shoup companion
    u64 last_w, last_w_sh; // (psi^-1 table entry 1) * N^-1: merged last inverse stage
    u64 pinv, pinv_sh;     // P^-1 mod q (data primes; P = product of special primes)
    u64 pmod, pmod_sh;     // P mod q
    // FP64 transform constants (used only when q < 2^50): q, 1/q, 2^52 + q,
    // and the merged last inverse stage's N^-1 and last_w with their ratios to q
    double qf, qinvf, qmf;
    double ninvf, ninvqf, last_wf, last_wqf;
};
// primes below this bound may use the FP64 transforms
constexpr u64 kFpPrimeBound = 1ull << 50;

// Device view of the uploaded context tables. Built by the host from the
// device base address; passed by value to every kernel.
struct DevTables {
    const PrimeConst *pc;        // [n_prim]
    const ulonglong2 *tw;        // [n_prim][N] (w, w') forward psi^brv(k)
    const ulonglong2 *itw;       // [n_prim][N] (w, w') inverse: (psi^brv(k))^-1
    const double2 *twf;          // [n_prim][N] (w, w / q) in FP64, forward
    const double2 *itwf;         // [n_prim][N] (w, w / q) in FP64, inverse
    const u64 *modup;            // ModUp blocks, see modup_block()
    const u64 *moddown;          // ModDown block
    const ulonglong2 *rescale;   // [n_q][n_q] (q_l^-1 mod q_i, Shoup)
    u32 log_n, n_q, n_p, n_prim, alpha, n_digits_top;
    // tuning knobs (all settings give bit-identical results)
    u32 ntt_wide;   // 1: 32 residues per thread below N = 2^15 (default 16)
    u32 ew_log;     // log2 of residues per thread in streaming kernels (1..3)
    u32 xcd_remap;  // 1: consecutive work items on one XCD
    u32 fuse_tail;  // 1: HMult's rescale epilogue inside the last NTT
    u32 ip_cts;     // ciphertexts sharing each key load in the inner product (2 or 4)
    u32 lin_mfma;   // 1: dense linear layers on the matrix cores
    u32 ntt_fp;     // context: 1 = transforms of primes below 2^50 in FP64 arithmetic;
                    // per NTT launch: 1 = every item's prime is below 2^50 and takes that engine
};

// ModUp constants for digit j truncated to s primes (1 <= s <= alpha):
// block (j * alpha + s - 1) of size modup_block_words(): first 2*alpha
// words are (inv, inv_sh) pairs for (Q_D / q_i)^-1 mod q_i, then
// alpha x n_prim words of (Q_D / q_i) mod t.
__host__ __device__ inline u32 modup_block_words(u32 alpha, u32 n_prim) {
    return 2 * alpha + alpha * n_prim;
}
// ModDown block: n_p pairs (inv, inv_sh) of (P / p_m)^-1 mod p_m, then
// n_p x n_q words (P / p_m) mod q_i.

// ---------------------------------------------------------------------
// Work-item descriptors (one per workgroup of an NTT-shaped kernel, or a
// unit of an elementwise kernel). Their meaning is per kernel and
// documented next to each kernel.
// ---------------------------------------------------------------------
struct Item {
    const u64 *in[8];
    u64 *out;
    u64 *out2;
    u32 prime;  // prime index of the limb this item produces
    u32 a, b, c;  // small kernel-specific integers
    i64 v;      // kernel-specific signed constant
};

// Elementwise descriptors: one per output limb (or limb pair).
struct EwItem {
    const u64 *x[8];
    u64 *y[3];
    u32 prime;
    u32 op;
    i64 v;
};

// Grouped sparse linear layer: rows that share one column list are one
// group; weights of a group are dense [nrows][ncols] at w_off.
struct LinGroup {
    u32 row0, nrows;   // output rows row0 .. row0 + nrows - 1
    u32 col_off, ncols;  // columns col[col_off .. col_off + ncols - 1]
    u32 w_off, pad;
};
constexpr int kLinRows = 8;  // rows per group (accumulators per thread)

// Dense modular linear layer on the matrix cores (k_linear_mfma): every
// weight is split into kWDig signed base-128 digits and every residue into
// kXDig unsigned base-128 digits; int8 MFMA products of digit planes are
// summed exactly in int32 per digit weight 128^s and recombined before one
// reduction mod q. Valid for |w| <= kWMax and at most kMfmaMaxIn inputs.
constexpr int kWDig = 6, kXDig = 9;
constexpr int64_t kWMax = (int64_t)1 << 40;
constexpr uint32_t kMfmaMaxIn = 40000;

// Key-switch inner product over up to kIpCts ciphertexts of one level that
// share the key: target limb `pos` of the extended basis (prime `prime`).
constexpr int kIpCts = 4;
struct IpItem {
    const u64 *ext[kIpCts];   // ModUp output base of each ciphertext, [digit][E][N]
    u64 *acc[kIpCts];         // accumulator base of each ciphertext, [2][E][N]
    const u64 *own0[kIpCts];  // own digit: the NTT-form input limb, or a1 of a product
    const u64 *own1[kIpCts];  // own digit: b1 of a product, or null
    // a0, b0 of a product (or null): the accumulators of data limbs also
    // receive P (a0 b0) and P (a0 b1 + a1 b0), so that ModDown returns
    // the relinearised product d + floor(acc / P) in one pass
    const u64 *own2[kIpCts];
    const u64 *own3[kIpCts];
    const u64 *key;           // [digits][2][n_prim][N]
    u32 n_ct, prime, beta, own_digit, E, pos;
};

// The same inner product with the key residues of every digit held in
// registers and up to kIpSeqCts ciphertexts processed one after another
// (k_ip_seq; beta <= kIpSeqBeta): each key residue is loaded once for all of
// them while only one ciphertext's sums are live.
constexpr int kIpSeqCts = 16;
constexpr int kIpSeqBeta = 8;
struct IpSeqItem {
    const u64 *ext[kIpSeqCts];
    u64 *acc[kIpSeqCts];
    const u64 *own0[kIpSeqCts];
    const u64 *own1[kIpSeqCts];
    const u64 *own2[kIpSeqCts];
    const u64 *own3[kIpSeqCts];
    const u64 *key;
    u32 n_ct, prime, beta, own_digit, E, pos;
};

// Hoisted rotations with plaintext weights (k_hoist): one item per target
// limb `pos` of the extended basis and up to kHoCts ciphertexts of one
// level. For every rotation i the ModUp'd digits of the ciphertext's second
// polynomial are read through the NTT-domain automorphism g_i and
// multiplied by that rotation's Galois key; P sigma(c0) joins the b-sum on
// data limbs; the weighted sums over all rotations go to acc [2][E][N].
constexpr int kHoCts = 4;
// Staged form: when every rotation maps each aligned block of kHoChunk NTT
// slots onto itself, a workgroup keeps its block of the digits in LDS,
// at most kHoStageRows rows (ciphertexts x digits) of kHoChunk residues.
constexpr unsigned kHoChunk = 256;
constexpr unsigned kHoStageRows = 24;
struct HoItem {
    const u64 *ext[kHoCts];  // ModUp'd digits of c1, [digit][E][N]
    const u64 *c0[kHoCts];   // limb `pos` of c0 (data limbs only)
    const u64 *c1[kHoCts];   // limb 0 of c1 (own-digit limbs)
    u64 *acc[kHoCts];        // [2][E][N]
    const u64 *const *keys;  // [n_rot] Galois key bases ([digits][2][n_prim][N])
    const u32 *galois;       // [n_rot] Galois elements (1 = identity)
    const u64 *pts;          // [n_rot][E][N] plaintexts over Q_l U P (NTT form)
    u32 n_ct, prime, pos, E, L, beta, alpha, n_rot;
};

}  // namespace ckks
