/*
 * ckks.h -- C ABI of libckks_hip.so: RNS-CKKS ciphertext arithmetic for
 * encrypted neural-network inference on AMD Instinct MI355X (gfx950).
 *
 * The operations are those the paper relies on for encrypted inference
 * (Onoufriou, Hanheide, Leontidis, "EDLaaS: Fully Homomorphic Encryption
 * Over Neural Network Graphs", arXiv 2110.13638):
 *   - Sections 2.1 and 3 (FHE background; FHE and deep learning): CKKS
 *     packs N/2 values into one polynomial; ciphertexts that interact must
 *     share parameters and key; every multiplication consumes one prime of
 *     the modulus chain;
 *   - Section 4.1 (FHE parameterisation): the ciphertext container
 *     relinearises after a ciphertext product, rescales, and switches the
 *     higher operand down the modulus chain before a binary op;
 *   - Sections 4.2.2-4.2.3 (CNN, Dense/ANN): conv and dense nodes are sums of
 *     ciphertext-times-weight products plus a bias; activations are
 *     polynomials (the square x^2 is the degree-2 case);
 *   - Algorithms 1-5 (neuronal firing): forward traversal of a
 *     multi-directed graph of such nodes.
 * The integer-level conventions (NTT order, key switching, rounding,
 * randomness) are not fixed by the paper; the ones used here are stated
 * next to each call.
 *
 * Conventions
 *   - Every call returns a status (CKKS_OK = 0 or a negative CKKS_E*).
 *     ckks_last_error() returns a thread-local message for the last
 *     failure. No C++ exception crosses this boundary.
 *   - The library never allocates device memory. Every device buffer
 *     (context tables, keys, ciphertexts, plaintexts, workspace) is owned
 *     by the caller and sized with the *_bytes queries. Host handles
 *     (ckks_ctx, ckks_graph) are created and destroyed by the library.
 *   - "stream" is a hipStream_t passed as void* (NULL = default stream).
 *     Device calls are asynchronous on that stream; argument checks run
 *     on the host before any launch, and a failing check launches nothing.
 *   - Residues are uint64 in [0, q). A polynomial at level l has l+1 limbs
 *     (limb i modulo data prime q_i), each N = 2^log_n residues, contiguous.
 *     Ciphertexts and plaintexts are kept in NTT form: slot k of a limb
 *     holds a(psi^(2 brv(k) + 1)) with psi the smallest primitive 2N-th
 *     root of unity mod q_i (brv = log_n-bit reversal).
 *   - Batched calls take arrays of B descriptors; B = 1 is the plain path.
 *     Unless stated otherwise out may alias the input (in-place).
 *   - The secret key appears only in client-side calls (keygen, decrypt),
 *     matching the semi-honest server of the paper's threat model
 *     (Section 2.3): the server side needs pk, relinearisation and Galois
 *     keys only.
 */
#ifndef CKKS_H
#define CKKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CKKS_OK 0
#define CKKS_EINVAL (-1)  /* bad argument (null pointer, size, range)     */
#define CKKS_ELEVEL (-2)  /* operands at different levels                */
#define CKKS_ESCALE (-3)  /* operands at different scales                */
#define CKKS_EDEPTH (-4)  /* no prime left to rescale / out of levels    */
#define CKKS_ENOKEY (-5)  /* Galois key for the requested step missing   */
#define CKKS_EPARAMS (-6) /* parameters invalid (prime, N, dnum)         */
#define CKKS_ENOMEM (-7)  /* caller buffer (workspace) too small         */
#define CKKS_EDEVICE (-8) /* HIP runtime error                           */

/* thread-local text for the last failing call on this thread */
const char *ckks_last_error(void);

/* ------------------------------------------------------------------ */
/* parameters and context                                               */
/* ------------------------------------------------------------------ */
/* Parameters (the paper's parameter dictionary, Section 4.1 and Algorithm 8: scale,
 * polynomial modulus degree, coefficient modulus chain). q[0] is the base
 * prime that holds the final result, q[1..n_q-1] the primes consumed by
 * rescaling, p[] the key-switching special primes (the last, "special"
 * entry of Algorithm 8's chain). dnum = number of key-switching digits at
 * the top level; each digit is alpha = ceil(n_q / dnum) consecutive data
 * primes (hybrid key switching). Every prime must be 1 mod 2N, distinct,
 * and below 2^61. log_n in [10, 16]; at log_n = 16 only the plain
 * transforms (ckks_ntt, ckks_intt) and element-wise operations run (a 2^16
 * limb takes two workgroups of the 2^15 engine after a streaming first
 * stage); every other device call returns CKKS_EPARAMS. */
typedef struct {
    uint32_t log_n;
    uint32_t n_q;
    const uint64_t *q;
    uint32_t n_p;
    const uint64_t *p;
    uint32_t dnum;
} ckks_params;

typedef struct ckks_ctx ckks_ctx;

/* Prime chain rule used for every configuration: for each requested bit
 * size, in list order, the largest prime below 2^bits that is 1 mod 2N
 * and not already chosen. out[n]. */
int ckks_find_primes(uint32_t log_n, const uint32_t *bits, uint32_t n, uint64_t *out);

/* Algorithm 8 (heuristic parameterisation): maximal group cost c, scale
 * power s, special-prime multiplier p -> bit sizes [s*p, s x c, s*p]
 * (c+2 entries, written to bits_out) and N = 1024 * b / 27 where b
 * doubles from 27 until it covers the bit sum. */
int ckks_parameterise(uint32_t cost, uint32_t scale_bits, double special_mult,
                      uint32_t *bits_out, uint32_t bits_cap, uint32_t *n_bits, uint32_t *log_n);

/* Builds host-side tables (twiddles with Shoup companions, basis
 * conversion constants). No device work. */
int ckks_ctx_create(const ckks_params *params, ckks_ctx **out);
void ckks_ctx_destroy(ckks_ctx *ctx);

/* Device bytes for the context tables, and their upload into a caller
 * buffer of at least that size (256-byte aligned). Must precede every
 * device call. The host copy stays alive until ckks_ctx_destroy. */
size_t ckks_ctx_device_bytes(const ckks_ctx *ctx);
int ckks_ctx_upload(ckks_ctx *ctx, void *dev, void *stream);

uint32_t ckks_ctx_log_n(const ckks_ctx *ctx);
uint32_t ckks_ctx_max_level(const ckks_ctx *ctx);       /* n_q - 1 */
uint32_t ckks_ctx_digits(const ckks_ctx *ctx, uint32_t level); /* ceil((l+1)/alpha) */
/* prime by index: 0..n_q-1 data, n_q.. special. 0 if out of range */
uint64_t ckks_ctx_prime(const ckks_ctx *ctx, uint32_t index);

/* ------------------------------------------------------------------ */
/* objects                                                              */
/* ------------------------------------------------------------------ */
/* Ciphertext: device buffer, poly t limb i at data + (t*limb_stride+i)*N.
 * limb_stride >= level + 1 is the number of limbs allocated per poly, so
 * that switching down the modulus chain (the level matching of Section 4.1)
 * is a change of 'level' only. n_poly is 2, or 3 straight after a
 * tensor product. data (and every plaintext and key buffer) must be
 * 16-byte aligned, as any device allocation is: kernels move residues in
 * pairs. Calls return CKKS_EINVAL for a null or misaligned buffer. */
typedef struct {
    uint64_t *data;
    uint32_t n_poly;
    uint32_t level;
    uint32_t limb_stride;
    uint32_t reserved;
    double scale;
} ckks_ct;

/* Plaintext: device buffer [level+1][N] in NTT form. */
typedef struct {
    uint64_t *data;
    uint32_t level;
    uint32_t reserved;
    double scale;
} ckks_pt;

size_t ckks_ct_bytes(const ckks_ctx *ctx, uint32_t n_poly, uint32_t level);
size_t ckks_pt_bytes(const ckks_ctx *ctx, uint32_t level);

#define CKKS_KEY_SECRET 0 /* [n_q+n_p][N], NTT form over every prime     */
#define CKKS_KEY_PUBLIC 1 /* [2][n_q][N]: (b = -a s + e, a)               */
#define CKKS_KEY_SWITCH 2 /* [digits][2][n_q+n_p][N]: relin or one Galois */
size_t ckks_key_bytes(const ckks_ctx *ctx, int kind);

/* ------------------------------------------------------------------ */
/* serialisation (client <-> server transfer, Section 4: ciphertexts are */
/* encrypted by the client, evaluated by the server, sent back)          */
/* ------------------------------------------------------------------ */
/* Byte format: a 64-byte little-endian header (magic "CKKS", version 1,
 * object kind, log2 N, n_q, n_p, dnum, n_poly, level, key kind, scale as
 * an IEEE double, FNV-1a hash of the prime chain, payload bytes) followed
 * by the residues as u64 [n_poly][level+1][N] (the limb stride of a device
 * ciphertext is not kept). Objects: a ciphertext (obj = ckks_ct *), a
 * plaintext (ckks_pt *), or a key (obj = device pointer to the key, kind
 * given by key_kind; n_poly / level are implied by the kind).
 * ckks_serialize: with host_bytes == NULL stores the size in *n and returns;
 * otherwise copies device -> host on `stream` and waits for it; ENOMEM if
 * *n is smaller than the size (the size is stored in *n).
 * ckks_deserialize: checks the header against ctx (ring, chain hash, dnum:
 * EPARAMS on mismatch; EINVAL for a bad magic, kind or length), copies the
 * residues host -> device into the object's buffer (a ct / pt needs data
 * with room for the stored level: limb_stride >= level + 1, which is
 * checked; level, n_poly and scale are set from the header) and waits. Not
 * allowed while recording (EINVAL). */
#define CKKS_OBJ_CT 0
#define CKKS_OBJ_PT 1
#define CKKS_OBJ_KEY 2
int ckks_serialize(const ckks_ctx *ctx, int obj_kind, const void *obj, int key_kind, void *host_bytes, size_t *n,
                   void *stream);
int ckks_deserialize(const ckks_ctx *ctx, int obj_kind, const void *host_bytes, size_t n, void *obj, int key_kind,
                     void *stream);

/* ------------------------------------------------------------------ */
/* workspace                                                            */
/* ------------------------------------------------------------------ */
#define CKKS_OP_NTT 0        /* count = number of limbs                  */
#define CKKS_OP_ELEMENTWISE 1 /* add, sub, plain and scalar ops, tensor   */
#define CKKS_OP_KEYSWITCH 2  /* relinearize / rotate                     */
#define CKKS_OP_RESCALE 3
#define CKKS_OP_HMULT 4      /* hmult_relin_rescale                      */
#define CKKS_OP_KEYGEN 5
#define CKKS_OP_ENCRYPT 6
#define CKKS_OP_LINEAR 7     /* count = n_out, levels[0] = level, levels[1] = n_in */
/* Workspace bytes for B operations at the given levels (levels[b] for
 * b < B; NULL = every operand at the top level). */
size_t ckks_workspace_bytes(const ckks_ctx *ctx, int op, uint32_t B, const uint32_t *levels);

/* ------------------------------------------------------------------ */
/* NTT primitives (batched over limbs of any prime)                     */
/* ------------------------------------------------------------------ */
/* In place forward / inverse negacyclic NTT of n limbs; limbs[i] points
 * at N residues modulo prime index prime_idx[i]. Output fully reduced. */
int ckks_ntt(const ckks_ctx *ctx, uint64_t *const *limbs, const uint32_t *prime_idx, uint32_t n,
             void *ws, size_t ws_bytes, void *stream);
int ckks_intt(const ckks_ctx *ctx, uint64_t *const *limbs, const uint32_t *prime_idx, uint32_t n,
              void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* client side: keys, encoding, encryption, decryption                  */
/* ------------------------------------------------------------------ */
/* Randomness: Philox4x32-10 keyed by the 64-bit seed, counter =
 * (coefficient index, limb index or 0xFFFFFFFF, object id, domain tag).
 * Ternary = ((w0 * 3) >> 32) - 1; error = centred binomial
 * popcount(w0 & 0x1FFFFF) - popcount(w1 & 0x1FFFFF); uniform = the
 * 128-bit word mod q, drawn directly in the NTT domain. */

/* secret s (ternary, tag 1), written in NTT form over every prime */
int ckks_keygen_secret(const ckks_ctx *ctx, uint64_t seed, uint64_t *sk, void *ws, size_t ws_bytes,
                       void *stream);
/* pk = (-a s + e, a) over the data primes: a tag 2, e tag 3, object 0 */
int ckks_keygen_public(const ckks_ctx *ctx, const uint64_t *sk, uint64_t seed, uint64_t *pk,
                       void *ws, size_t ws_bytes, void *stream);
/* Switching key s^2 -> s (key id 0). For every top-level digit j:
 * a_j uniform (tag 4), e_j error (tag 5), object (key_id << 8) | j,
 * b_j = -a_j s + e_j + [i in digit j] (P mod q_i) s' mod each prime,
 * with P the product of the special primes. */
int ckks_keygen_relin(const ckks_ctx *ctx, const uint64_t *sk, uint64_t seed, uint64_t *rk,
                      void *ws, size_t ws_bytes, void *stream);
/* Switching key sigma_g(s) -> s for Galois element g (odd, < 2N), key id g. */
int ckks_keygen_galois(const ckks_ctx *ctx, const uint64_t *sk, uint32_t galois_elt, uint64_t seed,
                       uint64_t *gk, void *ws, size_t ws_bytes, void *stream);
/* Galois element for a left rotation of the N/2 slots by step (negative
 * = right): 5^(step mod N/2) mod 2N. Conjugation is 2N - 1. */
uint32_t ckks_galois_elt(const ckks_ctx *ctx, int32_t step);

/* Host FP64 encoder (canonical embedding; slot j <-> zeta^(5^j),
 * zeta = exp(i pi / N)): n <= N/2 values (im may be NULL), zero padded,
 * coefficients round_half_away(scale * sigma^-1(z)) into coeffs[N].
 * CKKS_EINVAL when a coefficient would reach 2^62. */
int ckks_encode(const ckks_ctx *ctx, const double *re, const double *im, size_t n, double scale,
                int64_t *coeffs);
/* Host decoder from decrypted residues in coefficient form
 * ([level+1][N], host memory): exact centred CRT lift, then
 * slots = m(zeta^(5^j)) / scale for j < n. im may be NULL. */
int ckks_decode(const ckks_ctx *ctx, const uint64_t *residues, uint32_t level, double scale,
                double *re, double *im, size_t n);
/* Constants (Section 4.2: weights and biases enter conv and dense nodes as
 * plaintext constants). A constant c at scale s is the constant polynomial
 * round_half_away(c * s) (only coefficient 0 nonzero), so its NTT form
 * holds the same residue in every slot of a limb.
 * ckks_encode_scalars: the integers round_half_away(c[k] * scale) for n
 * host values into out[n] (host), the form ckks_multiply_scalar,
 * ckks_add_scalar and the linear layers take. CKKS_EINVAL when a product is
 * not finite or reaches 2^62 in magnitude (nothing after it is written).
 * ckks_encode_scalar: the same constant as its residues per limb,
 * per_limb[i] = round_half_away(c * scale) mod q_i for i <= level (host,
 * level + 1 entries); CKKS_ELEVEL for a level beyond the chain. */
int ckks_encode_scalars(const ckks_ctx *ctx, const double *c, size_t n, double scale, int64_t *out);
int ckks_encode_scalar(const ckks_ctx *ctx, double c, double scale, uint32_t level, uint64_t *per_limb);
/* Integer polynomial (device int64[N]) -> device plaintext in NTT form
 * at out->level; out->scale is left as set by the caller. */
int ckks_pt_load(const ckks_ctx *ctx, const int64_t *coeffs, ckks_pt *out, void *ws,
                 size_t ws_bytes, void *stream);
/* Public-key encryption at pt->level: v ternary (tag 6), e0, e1 errors
 * (tags 7, 8), object obj: ct = (v b + e0 + m, v a + e1). out->scale =
 * pt->scale, out->level = pt->level. */
int ckks_encrypt(const ckks_ctx *ctx, const uint64_t *pk, const ckks_pt *pt, uint64_t seed,
                 uint32_t obj, ckks_ct *out, void *ws, size_t ws_bytes, void *stream);
/* m = c0 + c1 s (+ c2 s^2) in coefficient form into m[level+1][N]
 * (device). */
int ckks_decrypt(const ckks_ctx *ctx, const uint64_t *sk, const ckks_ct *ct, uint64_t *m, void *ws,
                 size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* server side: evaluation (batched, B >= 1)                            */
/* ------------------------------------------------------------------ */
/* Binary ops need equal levels (CKKS_ELEVEL) and bit-equal scales
 * (CKKS_ESCALE); ckks_mod_switch_to lowers the higher operand first. */
int ckks_add(const ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct *out, uint32_t B,
             void *ws, size_t ws_bytes, void *stream);
int ckks_sub(const ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct *out, uint32_t B,
             void *ws, size_t ws_bytes, void *stream);
int ckks_add_plain(const ckks_ctx *ctx, const ckks_ct *a, const ckks_pt *p, ckks_ct *out,
                   uint32_t B, void *ws, size_t ws_bytes, void *stream);
/* ct x pt (Hadamard product of slots); out scale = a.scale * p.scale */
int ckks_multiply_plain(const ckks_ctx *ctx, const ckks_ct *a, const ckks_pt *p, ckks_ct *out,
                        uint32_t B, void *ws, size_t ws_bytes, void *stream);
/* ct x constant: v[b] is the integer constant polynomial round(c * s_c);
 * out scale = a.scale * v_scale[b] */
int ckks_multiply_scalar(const ckks_ctx *ctx, const ckks_ct *a, const int64_t *v,
                         const double *v_scale, ckks_ct *out, uint32_t B, void *ws,
                         size_t ws_bytes, void *stream);
/* ct + constant polynomial v[b] (already at the ciphertext's scale) */
int ckks_add_scalar(const ckks_ctx *ctx, const ckks_ct *a, const int64_t *v, ckks_ct *out,
                    uint32_t B, void *ws, size_t ws_bytes, void *stream);
/* tensor: out (n_poly 3) = (a0 b0, a0 b1 + a1 b0, a1 b1), scale product */
int ckks_multiply(const ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct *out3,
                  uint32_t B, void *ws, size_t ws_bytes, void *stream);
/* hybrid key switch of c2 with the relinearisation key:
 * out = (c0 + ks0, c1 + ks1). ModUp is the approximate basis conversion
 * of each digit; ModDown subtracts the conversion of the special-prime
 * part and multiplies by P^-1. out must not alias in3.
 * rk[b]: device pointer to the relinearisation key of item b. Each client
 * holds its own keys (the threat model of Section 2.3), so items of
 * different clients carry different keys and still share one launch;
 * items with the same key share its loads. CKKS_ENOKEY for a null key. */
int ckks_relinearize(const ckks_ctx *ctx, const uint64_t *const *rk, const ckks_ct *in3, ckks_ct *out,
                     uint32_t B, void *ws, size_t ws_bytes, void *stream);
/* rescale by the top prime q_l: c' = floor((c + floor(q_l/2)) / q_l)
 * coefficient-wise, scale / q_l, level - 1. out may alias in. */
int ckks_rescale(const ckks_ctx *ctx, const ckks_ct *in, ckks_ct *out, uint32_t B, void *ws,
                 size_t ws_bytes, void *stream);
/* rescale, then add the constant v[b] (an integer: a scalar already
 * multiplied by the output scale and rounded, as ckks_encode_scalars gives)
 * to every slot of the first polynomial of out[b]: the bias of a conv or
 * dense layer, which follows its product's rescale (Sections 4.2.2 and
 * 4.2.3). Bit-identical to ckks_rescale then ckks_add_scalar, in one pass
 * over the limbs. CKKS_EINVAL for a null v. */
int ckks_rescale_add_scalar(const ckks_ctx *ctx, const ckks_ct *in, const int64_t *v, ckks_ct *out, uint32_t B,
                            void *ws, size_t ws_bytes, void *stream);
/* modulus-chain level match: a view change (no device work) */
int ckks_mod_switch_to(const ckks_ctx *ctx, ckks_ct *inout, uint32_t level);
/* slot rotation: X -> X^g on both polys, then key switch of the second
 * with the Galois key for g: out = (sigma(c0) + ks0, ks1). Item b uses the
 * Galois element galois_elts[b] (odd, < 2N; see ckks_galois_elt) and the
 * device key gk[b] made for that element (per item, so one launch can
 * rotate ciphertexts of several clients by different steps). EINVAL for a
 * bad element, ENOKEY for a null key. out must not alias in. */
int ckks_rotate(const ckks_ctx *ctx, const uint64_t *const *gk, const uint32_t *galois_elts, const ckks_ct *in,
                ckks_ct *out, uint32_t B, void *ws, size_t ws_bytes, void *stream);
/* Fused, batched HMult + relinearise + rescale (the ciphertext product as
 * the container performs it): out[b] = rescale(relin(a[b] x b[b])),
 * ragged levels allowed. Bit-identical to the three calls in sequence.
 * rk[b]: the relinearisation key of item b (as in ckks_relinearize). */
int ckks_hmult_relin_rescale(const ckks_ctx *ctx, const uint64_t *const *rk, const ckks_ct *a,
                             const ckks_ct *b, ckks_ct *out, uint32_t B, void *ws,
                             size_t ws_bytes, void *stream);
/* The same call without a caller workspace, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * hosts that forbid hipMalloc). Scratch limbs and work-item tables go to a
 * fixed device array of CKKS_NOALLOC_SCRATCH_BYTES inside the library (one
 * per GPU, held until the process ends; its address is looked up on the
 * first call on each device). The call allocates nothing: no device or
 * pinned memory, no events (launch profiling is skipped); work-item tables
 * are copied from pageable host memory. Inputs, outputs and keys are
 * caller-owned device buffers as in ckks_hmult_relin_rescale, whose kernels
 * it runs, with bit-identical results. CKKS_ENOMEM (nothing launched) when
 * the batch's scratch (ckks_workspace_bytes(ctx, CKKS_OP_HMULT, B, levels))
 * exceeds the array (80 MiB: two pairs at N = 2^15 with 16 + 2 primes at
 * the top level, about 39 MiB each). Every call on one GPU shares the array
 * and overwrites what the previous call left there; calls that overlap on
 * one GPU (concurrent streams or host threads) race and must be
 * serialised by the caller. */
#define CKKS_NOALLOC_SCRATCH_BYTES (80u << 20)
int ckks_hmult_relin_rescale_noalloc(const ckks_ctx *ctx, const uint64_t *const *rk, const ckks_ct *a,
                                     const ckks_ct *b, ckks_ct *out, uint32_t B, void *stream);
/* Encrypted linear layer with integer weights (conv and dense of the
 * paper's Sections 4.2.2-4.2.3, weights encoded as constant polynomials):
 * out[j] = sum_i W[j * n_in + i] * in[i]  for j < n_out, W device int64.
 * All inputs at one level and scale; out scale = in.scale * w_scale. */
int ckks_linear(const ckks_ctx *ctx, const ckks_ct *in, uint32_t n_in, const int64_t *W,
                double w_scale, ckks_ct *out, uint32_t n_out, void *ws, size_t ws_bytes,
                void *stream);

/* Sparse form of the same layer (the strided cross-correlation of
 * Section 4.2.2 touches at most k x k inputs per output): row j is
 * sum_{e in [row_ptr[j], row_ptr[j+1])} w[e] * in[col[e]]. Host arrays;
 * consecutive rows with identical column lists are evaluated together so
 * each input residue is loaded once per group. */
size_t ckks_linear_csr_workspace_bytes(const ckks_ctx *ctx, uint32_t n_in, uint32_t n_out, size_t nnz,
                                       uint32_t level);
int ckks_linear_csr(const ckks_ctx *ctx, const ckks_ct *in, uint32_t n_in, uint32_t n_out,
                    const uint32_t *row_ptr, const uint32_t *col, const int64_t *w, double w_scale,
                    ckks_ct *out, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* hoisted rotations with plaintext weights                             */
/* ------------------------------------------------------------------ */
/* The rotation-based matrix-vector product of a dense layer (Section 4.2.3
 * on slot-packed inputs; the diagonal method) with all rotations of one
 * ciphertext sharing a single decomposition. For each input x = (c0, c1)
 * at level l, with D_j the ModUp of digit j of c1 to Q_l U P (NTT form;
 * the digit's own limbs are c1's), sigma_g the NTT-domain automorphism
 * X -> X^g and (b_{g,j}, a_{g,j}) the Galois key of g:
 *   T0 = sum_i pt_i (x) ( sum_j sigma_gi(D_j) (x) b_{gi,j} + P sigma_gi(c0) )
 *   T1 = sum_i pt_i (x) ( sum_j sigma_gi(D_j) (x) a_{gi,j} )
 * over Q_l U P (P sigma(c0) is zero on the special primes; g_i = 1 is the
 * identity and contributes (P c0, P c1)), and out = (ModDown(T0),
 * ModDown(T1)) at level l with scale x.scale * pt_scale: one ModDown per
 * ciphertext for the whole sum. Equals sum_i pt_i (x) rot_{g_i}(x) up to the
 * rounding of ModDown.
 * galois_elts [n_rot] (odd, < 2N; 1 = identity), galois_keys [n_rot]
 * device key pointers (ignored for the identity; ENOKEY when missing),
 * pt_coeffs: device int64 [n_rot][N] integer plaintext coefficients at
 * pt_scale (reduced and transformed to every prime of Q_l U P inside the
 * call). in[b] all at one level (ELEVEL), out[b] must not alias in[b].
 * Workspace: ckks_hoisted_linear_workspace_bytes (ENOMEM when short). */
size_t ckks_hoisted_linear_workspace_bytes(const ckks_ctx *ctx, uint32_t B, uint32_t level, uint32_t n_rot);
int ckks_hoisted_linear(const ckks_ctx *ctx, const ckks_ct *in, ckks_ct *out, uint32_t B, uint32_t n_rot,
                        const uint32_t *galois_elts, const uint64_t *const *galois_keys, const int64_t *pt_coeffs,
                        double pt_scale, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* graph traversal (Algorithms 1-5, forward receptor only)              */
/* ------------------------------------------------------------------ */
/* A multi-directed graph of encrypted layers (Section 4): every edge
 * carries a signal (a list of ciphertexts); a node fires once every
 * in-edge carries one, its inputs are the in-edge signals stacked in edge
 * insertion order (levels matched by switching down to the lowest), and
 * its result is broadcast to all out-edges. Parallel edges are separate
 * edges. Receptors:
 *   INPUT       the run's input ciphertexts (attrs: ckks_input_attrs);
 *   LINEAR      conv / dense: row j = sum_e round(w[e] w_scale) in[col[e]],
 *               rescale, + round(bias[j] * scale) (ckks_linear_attrs);
 *   DIAG_DENSE  rotation-based matvec on each input ciphertext:
 *               sum_i diag_i (x) rot(x, in_steps[i]), rescale, then
 *               x += rot(x, r) for every post step, + bias plaintext;
 *               steps without their own Galois key are composed from
 *               power-of-two keys in non-adjacent form; with `hoisted`
 *               the sum is one ckks_hoisted_linear call (ckks_diag_attrs);
 *   SQUARE      x^2: ckks_hmult_relin_rescale(x, x) on each ciphertext;
 *   POLY        polynomial activation p(x) = sum_k c_k x^k of degree
 *               d >= 1 (Section 4.4: the ReLU approximation
 *               4/(3 pi q) x^2 + x/2 + q/(3 pi), the sigmoid approximation
 *               0.5 + 0.197 x - 0.004 x^3) by Horner's rule on each
 *               ciphertext: h = rescale(x * round(c_d w_scale)); for k =
 *               d-1..1: h += round(c_k scale_h), h = x' (x) h relinearised
 *               and rescaled with x' = x switched down to h's level; then
 *               h += round(c_0 scale_h). Uses d levels (ckks_poly_attrs);
 *   OUTPUT      collects its signal as run outputs (node order). */
typedef struct ckks_graph ckks_graph;
#define CKKS_NODE_INPUT 0
#define CKKS_NODE_LINEAR 1
#define CKKS_NODE_DIAG_DENSE 2
#define CKKS_NODE_SQUARE 3
#define CKKS_NODE_OUTPUT 4
#define CKKS_NODE_POLY 5
typedef struct {
    uint32_t n_ct;
    uint32_t level;
    double scale;
} ckks_input_attrs;
typedef struct {
    uint32_t n_out;
    const uint32_t *row_ptr; /* [n_out + 1] */
    const uint32_t *col;     /* [nnz], index into the node's stacked inputs */
    const double *w;         /* [nnz] */
    double w_scale;          /* weights become round(w * w_scale) */
    const double *bias;      /* [n_out] or NULL */
} ckks_linear_attrs;
typedef struct {
    uint32_t n_diag;
    const int32_t *in_steps;     /* [n_diag], 0 = no rotation */
    const int64_t *diag_coeffs;  /* [n_diag][N] integer plaintexts at pt_scale */
    double pt_scale;
    uint32_t n_post;
    const int32_t *post_steps;   /* [n_post] rotate-and-sum steps */
    const double *bias_slots;    /* [n_bias_slots] or NULL: encoded at plan */
    uint32_t n_bias_slots;
    const int64_t *bias_coeffs;  /* [N] integer plaintext at the output scale, or NULL */
    uint32_t hoisted;            /* 1: all in_steps rotations hoisted (ckks_hoisted_linear);
                                    every nonzero step needs its own Galois key */
} ckks_diag_attrs;
typedef struct {
    uint32_t degree;      /* d >= 1 */
    const double *coeffs; /* [d + 1], c_0 first */
    double w_scale;       /* scale of the constant in the first product */
} ckks_poly_attrs;
int ckks_graph_create(const ckks_ctx *ctx, ckks_graph **out);
void ckks_graph_destroy(ckks_graph *g);
/* attributes are copied */
int ckks_graph_add_node(ckks_graph *g, int kind, const void *attrs, uint32_t *id);
int ckks_graph_add_edge(ckks_graph *g, uint32_t from, uint32_t to);
/* Dry traversal: output count, levels and scales of every node, and the
 * workspace the run needs (all node outputs plus scratch). */
int ckks_graph_plan(ckks_graph *g, size_t *ws_bytes, uint32_t *n_outputs);
/* inputs: the ciphertexts of every INPUT node in node order, at the
 * planned level and scale; outputs receive views into the workspace
 * (valid until the workspace is reused). Galois keys by element. */
int ckks_graph_run(ckks_graph *g, const ckks_ct *inputs, uint32_t n_inputs, ckks_ct *outputs, uint32_t n_outputs,
                   const uint64_t *rk, const uint32_t *galois_elts, const uint64_t *const *galois_keys,
                   uint32_t n_galois, void *ws, size_t ws_bytes, void *stream);

/* Algorithms 6-7 (automatic FHE parameterisation): node cost = depth it
 * consumes (1 for LINEAR, DIAG_DENSE, SQUARE; the degree d for POLY; 0 for
 * INPUT, OUTPUT); every
 * node is labelled with the longest cost from each source that reaches
 * it, OUTPUT nodes are concern nodes where the labelling restarts, and
 * sources meeting at a node are merged into one parameter group whose
 * cost is the largest label reached. Writes the group count, the group of
 * every node (indexed by node id, cap entries; 0xFFFFFFFF for a node no
 * source reaches) and each group's cost, ready for ckks_parameterise. */
int ckks_graph_autohe(ckks_graph *g, uint32_t *n_groups, uint32_t *group_of_node, uint32_t *group_cost,
                      uint32_t cap);

/* ------------------------------------------------------------------ */
/* launch recording (HIP graph capture)                                 */
/* ------------------------------------------------------------------ */
/* Between ckks_record_begin and ckks_record_end, every device call made
 * with ctx still runs as usual, and in addition its kernel launches are
 * recorded. The launch data such calls upload (work descriptors, pointer
 * tables, weight images) goes to the caller's `arena` (device memory,
 * 256-byte aligned) instead of the workspace, so that it outlives the call.
 * ckks_plan_launch re-issues exactly the recorded launches on a stream,
 * with no copy, allocation, memset or host synchronisation, so it can be
 * captured into a HIP graph (stream capture) and replayed: a layer
 * sequence or a batched HMult becomes one graph launch. Every buffer the
 * recorded calls touched (inputs, outputs, keys, workspaces, arena, context
 * tables) must stay allocated at the same address while the plan is used;
 * their contents may change between replays (new inputs in the same
 * buffers give the new results). Host-side results of the recorded calls
 * (output levels and scales) are those of the recording run. Launch shapes
 * (ckks_ctx_set_tuning) are frozen at recording time.
 * ckks_record_begin: EINVAL when already recording or misaligned; a call
 * made while recording fails with ENOMEM if the arena runs out (recording
 * continues; end it and start again with a larger arena).
 * ckks_record_end: returns the plan (owned by the caller, released with
 * ckks_plan_destroy) and the arena bytes used. Not thread safe against
 * other calls on the same context. */
typedef struct ckks_plan ckks_plan;
int ckks_record_begin(ckks_ctx *ctx, void *arena, size_t arena_bytes);
int ckks_record_end(ckks_ctx *ctx, ckks_plan **plan, size_t *arena_used);
int ckks_plan_launch(const ckks_plan *plan, void *stream);
uint32_t ckks_plan_launch_count(const ckks_plan *plan);
void ckks_plan_destroy(ckks_plan *plan);

/* ------------------------------------------------------------------ */
/* tuning                                                               */
/* ------------------------------------------------------------------ */
/* Launch-shape knobs of a context. Every setting computes bit-identical
 * results; only speed differs, so an autotuner may time the variants on
 * the workload at hand and keep the fastest. Settings apply to launches
 * issued after the call (not thread safe against concurrent calls on the
 * same context).
 *   CKKS_TUNE_NTT_WIDE   0 (default): 16 residues per thread in the NTT
 *                        kernels for N < 2^15 (32 at 2^15); 1: 32 residues
 *                        per thread (N in 2^11..2^14 only).
 *   CKKS_TUNE_EW_LOG     log2 of residues per thread in the streaming
 *                        (element-wise, key-switch inner product) kernels:
 *                        1, 2 (default) or 3.
 *   CKKS_TUNE_XCD_REMAP  1 (default): map consecutive NTT work items to one
 *                        XCD (shared L2); 0: plain block order.
 *   CKKS_TUNE_FUSE_TAIL  0 (default): the rescale step of
 *                        ckks_hmult_relin_rescale runs as its own
 *                        element-wise pass; 1: inside the last NTT.
 *   CKKS_TUNE_IP_CTS     ciphertexts of one level that share each key load
 *                        in the key-switch inner product: 4 (default), 2
 *                        (fewer registers, more key traffic) or 16 (key
 *                        residues of every digit held in registers and the
 *                        ciphertexts processed one after another; levels
 *                        with more than 8 digits fall back to 4).
 *   CKKS_TUNE_LIN_MFMA   1 (default): ckks_linear_csr layers whose rows
 *                        share one column list (dense layers), with
 *                        |weight| <= 2^40 and at most 40000 inputs, run on
 *                        the matrix cores (exact int8 digit products);
 *                        0: always the vector-ALU kernel.
 *   CKKS_TUNE_NTT_FP     1 (default): transforms of limbs whose prime is
 *                        below 2^50 use FP64 modular arithmetic (exact
 *                        FMA products, quotients from w/q); 0: 64-bit
 *                        integer arithmetic for every prime.
 * Returns CKKS_EINVAL for an unknown knob or a value out of range. */
enum {
    CKKS_TUNE_NTT_WIDE = 0, CKKS_TUNE_EW_LOG = 1, CKKS_TUNE_XCD_REMAP = 2, CKKS_TUNE_FUSE_TAIL = 3, CKKS_TUNE_IP_CTS = 4,
    CKKS_TUNE_LIN_MFMA = 5, CKKS_TUNE_NTT_FP = 6
};
int ckks_ctx_set_tuning(ckks_ctx *ctx, int knob, int value);
/* Current value of a knob, or -1 for a null context / unknown knob. */
int ckks_ctx_get_tuning(const ckks_ctx *ctx, int knob);

/* ------------------------------------------------------------------ */
/* measurement                                                          */
/* ------------------------------------------------------------------ */
/* Per-launch timing: while enabled, every kernel launch of every call is
 * bracketed by two HIP events recorded on that call's stream (process
 * wide; not thread safe; off by default). */
typedef struct {
    char name[56];   /* kernel family and ring degree, e.g. "ntt_fwd/N=2^15" */
    uint32_t items;  /* work items (workgroups or limbs) in the launch */
    float ms;        /* event-measured duration */
} ckks_launch_record;
int ckks_profile_enable(int on);
/* Waits for the recorded events, writes up to cap records (out may be
 * NULL), the total count to *n, and clears the record list. */
int ckks_profile_collect(ckks_launch_record *out, uint32_t cap, uint32_t *n);

#ifdef __cplusplus
}
#endif
#endif /* CKKS_H */
