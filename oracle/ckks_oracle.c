/*
 * Plain CPU reference for RNS-CKKS ciphertext arithmetic (the oracle).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do. It shares no code, header or table generator
 * with the HIP library.
 *
 * Every routine here is written for obviousness, not speed: residues are
 * u64 in [0, q), every modular product is a 128-bit product followed by
 * the C '%' operator, the NTT is a textbook radix-2 transform of the
 * psi-twisted sequence, and basis conversions are written as the sums
 * that define them.
 *
 * What is computed follows the paper's use of RNS-CKKS (Sections 2.1 and 3,
 * FHE background; Section 4.1, the ciphertext container that relinearises
 * after a ciphertext product and rescales / matches levels before binary
 * operations).
 * The paper defers every integer-level detail to its CKKS backend, so the
 * conventions below are this project's readings of the paper:
 *   - NTT slot k holds a(psi^(2*brv(k)+1)), psi = smallest primitive
 *     2N-th root of unity mod q;
 *   - hybrid key switching with digits of alpha consecutive primes,
 *     approximate ModUp (no correction), floor-style ModDown;
 *   - rescale rounds to nearest: c' = floor((c + floor(q_l/2)) / q_l);
 *   - randomness is Philox4x32-10 keyed by the seed, counter =
 *     (coefficient, limb, object id, domain tag).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;
typedef unsigned __int128 u128;

#define ORC_MAX_PRIMES 64

/* ------------------------------------------------------------------ */
/* scalar modular arithmetic                                            */
/* ------------------------------------------------------------------ */
static u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 addmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + b) % q); }
static u64 submod(u64 a, u64 b, u64 q) { return (u64)(((u128)a + q - b) % q); }
static u64 negmod(u64 a, u64 q) { return a == 0 ? 0 : q - a; }

static u64 powmod(u64 a, u64 e, u64 q)
{
    u64 r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}

/* q prime: Fermat inverse. */
static u64 invmod(u64 a, u64 q) { return powmod(a, q - 2, q); }

/* a signed 64-bit integer reduced into [0, q) */
static u64 reduce_signed(i64 v, u64 q)
{
    if (v >= 0) return (u64)v % q;
    u64 m = ((u64)(-(v + 1)) + 1) % q; /* |v| mod q without overflow */
    return m == 0 ? 0 : q - m;
}

u64 orc_mulmod(u64 a, u64 b, u64 q) { return mulmod(a, b, q); }
u64 orc_powmod(u64 a, u64 e, u64 q) { return powmod(a, e, q); }

/* ------------------------------------------------------------------ */
/* primes and roots (prime choice rule, smallest primitive root)       */
/* ------------------------------------------------------------------ */
/* Deterministic Miller-Rabin for 64-bit n (first 12 prime bases). */
int orc_is_prime(u64 n)
{
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    u64 d = n - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; r++; }
    for (int i = 0; i < 12; i++) {
        u64 x = powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int k = 1; k < r; k++) {
            x = mulmod(x, x, n);
            if (x == n - 1) { comp = 0; break; }
        }
        if (comp) return 0;
    }
    return 1;
}

/* For each requested bit size, in list order, the largest prime below
 * 2^bits that is 1 mod 2N and not already chosen. Returns 0 or -1. */
int orc_find_primes(u32 logn, const u32 *bits, u32 count, u64 *out)
{
    u64 two_n = (u64)2 << logn;
    for (u32 i = 0; i < count; i++) {
        if (bits[i] < 2 || bits[i] > 62) return -1;
        u64 top = ((u64)1 << bits[i]) - 1;
        u64 c = (top / two_n) * two_n + 1;
        if (c > top) c -= two_n;
        for (;;) {
            if (c < two_n) return -1;
            int used = 0;
            for (u32 k = 0; k < i; k++) used |= (out[k] == c);
            if (!used && orc_is_prime(c)) break;
            c -= two_n;
        }
        out[i] = c;
    }
    return 0;
}

/* Smallest primitive 2N-th root of unity modulo q (q = 1 mod 2N). */
u64 orc_min_psi(u64 q, u32 logn)
{
    u64 two_n = (u64)2 << logn;
    u64 n = (u64)1 << logn;
    u64 g = 0;
    for (u64 x = 2; x < q; x++) {
        u64 c = powmod(x, (q - 1) / two_n, q);
        if (powmod(c, n, q) == q - 1) { g = c; break; }
    }
    if (g == 0) return 0;
    /* every primitive 2N-th root is g^k with k odd */
    u64 best = g, g2 = mulmod(g, g, q), cur = g;
    for (u64 k = 1; k < n; k++) {
        cur = mulmod(cur, g2, q);
        if (cur < best) best = cur;
    }
    return best;
}

/* ------------------------------------------------------------------ */
/* oracle context: parameters plus per-prime NTT constants              */
/* ------------------------------------------------------------------ */
typedef struct {
    u32 logn, n_q, n_p, dnum, alpha;
    u64 q[ORC_MAX_PRIMES]; /* data primes then special primes */
    u64 psi[ORC_MAX_PRIMES];
    u64 *psi_pow[ORC_MAX_PRIMES];     /* psi^j, j < N */
    u64 *psi_inv_pow[ORC_MAX_PRIMES]; /* psi^-j, j < N */
    u64 *omega_pow[ORC_MAX_PRIMES];   /* (psi^2)^j, j < N/2 */
    u64 *omega_inv_pow[ORC_MAX_PRIMES];
} orc_ctx;

static u32 brv(u32 x, u32 bits)
{
    u32 r = 0;
    for (u32 i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

void orc_ctx_destroy(orc_ctx *c)
{
    if (!c) return;
    for (u32 i = 0; i < c->n_q + c->n_p; i++) {
        free(c->psi_pow[i]);
        free(c->psi_inv_pow[i]);
        free(c->omega_pow[i]);
        free(c->omega_inv_pow[i]);
    }
    free(c);
}

/* primes: n_q data primes followed by n_p special primes. dnum = number of
 * key-switching digits at the top level; alpha = ceil(n_q / dnum). */
orc_ctx *orc_ctx_create(u32 logn, const u64 *primes, u32 n_q, u32 n_p, u32 dnum)
{
    if (n_q + n_p > ORC_MAX_PRIMES || n_q == 0 || dnum == 0) return NULL;
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    c->logn = logn; c->n_q = n_q; c->n_p = n_p; c->dnum = dnum;
    c->alpha = (n_q + dnum - 1) / dnum;
    u64 n = (u64)1 << logn;
    for (u32 i = 0; i < n_q + n_p; i++) {
        u64 q = primes[i];
        c->q[i] = q;
        u64 psi = orc_min_psi(q, logn);
        if (psi == 0) { orc_ctx_destroy(c); return NULL; }
        c->psi[i] = psi;
        u64 pinv = invmod(psi, q);
        c->psi_pow[i] = (u64 *)malloc(n * sizeof(u64));
        c->psi_inv_pow[i] = (u64 *)malloc(n * sizeof(u64));
        c->omega_pow[i] = (u64 *)malloc(n * sizeof(u64));
        c->omega_inv_pow[i] = (u64 *)malloc(n * sizeof(u64));
        u64 a = 1, b = 1, w = mulmod(psi, psi, q), wi = mulmod(pinv, pinv, q), x = 1, y = 1;
        for (u64 j = 0; j < n; j++) {
            c->psi_pow[i][j] = a; a = mulmod(a, psi, q);
            c->psi_inv_pow[i][j] = b; b = mulmod(b, pinv, q);
            c->omega_pow[i][j] = x; x = mulmod(x, w, q);
            c->omega_inv_pow[i][j] = y; y = mulmod(y, wi, q);
        }
    }
    return c;
}

u64 orc_ctx_psi(const orc_ctx *c, u32 i) { return c->psi[i]; }

/* ------------------------------------------------------------------ */
/* negacyclic NTT (slot k holds a(psi^(2 brv(k) + 1)))                */
/* a_hat[k] = sum_j a[j] psi^((2 brv(k) + 1) j)  (mod q)               */
/* Computed as: twist b[j] = a[j] psi^j, cyclic length-N DFT with       */
/* omega = psi^2 (B[m] = sum_j b[j] omega^(m j)), then a_hat[k] =       */
/* B[brv(k)] since psi^((2m+1) j) = psi^j omega^(m j).                  */
/* ------------------------------------------------------------------ */
static void cyclic_dft(u64 *b, u32 logn, u64 q, const u64 *wpow)
{
    /* iterative radix-2 decimation-in-time: bit-reverse, then butterflies */
    u32 n = 1u << logn;
    for (u32 i = 0; i < n; i++) {
        u32 r = brv(i, logn);
        if (r > i) { u64 t = b[i]; b[i] = b[r]; b[r] = t; }
    }
    for (u32 len = 2; len <= n; len <<= 1) {
        u32 half = len >> 1, step = n / len;
        for (u32 s = 0; s < n; s += len)
            for (u32 j = 0; j < half; j++) {
                u64 w = wpow[(u64)j * step];
                u64 u = b[s + j], v = mulmod(b[s + j + half], w, q);
                b[s + j] = addmod(u, v, q);
                b[s + j + half] = submod(u, v, q);
            }
    }
}

void orc_ntt(const orc_ctx *c, u32 pi, u64 *a)
{
    u32 logn = c->logn, n = 1u << logn;
    u64 q = c->q[pi];
    u64 *b = (u64 *)malloc(n * sizeof(u64));
    for (u32 j = 0; j < n; j++) b[j] = mulmod(a[j] % q, c->psi_pow[pi][j], q);
    cyclic_dft(b, logn, q, c->omega_pow[pi]);
    for (u32 k = 0; k < n; k++) a[k] = b[brv(k, logn)];
    free(b);
}

/* inverse of orc_ntt: undo the output permutation, inverse cyclic DFT
 * (omega^-1, times N^-1), then untwist by psi^-j. */
void orc_intt(const orc_ctx *c, u32 pi, u64 *a)
{
    u32 logn = c->logn, n = 1u << logn;
    u64 q = c->q[pi];
    u64 *b = (u64 *)malloc(n * sizeof(u64));
    for (u32 k = 0; k < n; k++) b[brv(k, logn)] = a[k] % q;
    cyclic_dft(b, logn, q, c->omega_inv_pow[pi]);
    u64 ninv = invmod((u64)n % q, q);
    for (u32 j = 0; j < n; j++) a[j] = mulmod(mulmod(b[j], ninv, q), c->psi_inv_pow[pi][j], q);
    free(b);
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and samplers      */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const u32 ctr_in[4], const u32 key_in[2], u32 out[4])
{
    u32 c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    u32 k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        u64 p0 = (u64)0xD2511F53u * c0;
        u64 p1 = (u64)0xCD9E8D57u * c2;
        u32 hi0 = (u32)(p0 >> 32), lo0 = (u32)p0;
        u32 hi1 = (u32)(p1 >> 32), lo1 = (u32)p1;
        u32 n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* domain tags for the counter's last word */
enum { TAG_SK = 1, TAG_PK_A = 2, TAG_PK_E = 3, TAG_SWK_A = 4, TAG_SWK_E = 5,
       TAG_ENC_V = 6, TAG_ENC_E0 = 7, TAG_ENC_E1 = 8 };
#define NO_LIMB 0xFFFFFFFFu

static void draw(u64 seed, u32 j, u32 limb, u32 obj, u32 tag, u32 w[4])
{
    u32 ctr[4] = {j, limb, obj, tag};
    u32 key[2] = {(u32)seed, (u32)(seed >> 32)};
    orc_philox4x32_10(ctr, key, w);
}

static int popc21(u32 x)
{
    int c = 0;
    x &= (1u << 21) - 1;
    while (x) { c += x & 1u; x >>= 1; }
    return c;
}

void orc_sample_ternary(u64 seed, u32 obj, u32 tag, u32 n, i64 *out)
{
    u32 w[4];
    for (u32 j = 0; j < n; j++) {
        draw(seed, j, NO_LIMB, obj, tag, w);
        out[j] = (i64)(((u64)w[0] * 3u) >> 32) - 1;
    }
}

void orc_sample_cbd(u64 seed, u32 obj, u32 tag, u32 n, i64 *out)
{
    u32 w[4];
    for (u32 j = 0; j < n; j++) {
        draw(seed, j, NO_LIMB, obj, tag, w);
        out[j] = (i64)popc21(w[0]) - (i64)popc21(w[1]);
    }
}

/* uniform residue: the 128-bit integer w3:w2:w1:w0 reduced mod q */
void orc_sample_uniform(u64 seed, u32 obj, u32 tag, u32 limb, u32 n, u64 q, u64 *out)
{
    u32 w[4];
    for (u32 j = 0; j < n; j++) {
        draw(seed, j, limb, obj, tag, w);
        u128 v = ((u128)(((u64)w[3] << 32) | w[2]) << 64) | (((u64)w[1] << 32) | w[0]);
        out[j] = (u64)(v % q);
    }
}

/* ------------------------------------------------------------------ */
/* helpers on residue polynomials                                       */
/* A "poly at level l" is (l+1) limbs of N residues, limb i mod q[i].   */
/* A "key poly" spans all n_q + n_p primes.                             */
/* ------------------------------------------------------------------ */
static u32 nn(const orc_ctx *c) { return 1u << c->logn; }

/* NTT form of a small signed integer polynomial reduced mod prime pi */
static void small_to_ntt(const orc_ctx *c, const i64 *v, u32 pi, u64 *out)
{
    u32 n = nn(c);
    for (u32 j = 0; j < n; j++) out[j] = reduce_signed(v[j], c->q[pi]);
    orc_ntt(c, pi, out);
}

/* Secret key: ternary coefficients (tag SK, object 0) in NTT form over
 * every prime, layout [n_q + n_p][N]. Also returns the coefficients. */
void orc_keygen_secret(const orc_ctx *c, u64 seed, i64 *sk_coeff, u64 *sk_ntt)
{
    u32 n = nn(c);
    orc_sample_ternary(seed, 0, TAG_SK, n, sk_coeff);
    for (u32 i = 0; i < c->n_q + c->n_p; i++) small_to_ntt(c, sk_coeff, i, sk_ntt + (size_t)i * n);
}

/* Public key over the n_q data primes: pk = (b, a), a uniform in the NTT
 * domain, b = -a*s + e. Layout [2][n_q][N]. */
void orc_keygen_public(const orc_ctx *c, const u64 *sk_ntt, u64 seed, u64 *pk)
{
    u32 n = nn(c);
    i64 *e = (i64 *)malloc(n * sizeof(i64));
    u64 *eh = (u64 *)malloc(n * sizeof(u64));
    orc_sample_cbd(seed, 0, TAG_PK_E, n, e);
    for (u32 i = 0; i < c->n_q; i++) {
        u64 q = c->q[i];
        u64 *b = pk + (size_t)i * n, *a = pk + ((size_t)c->n_q + i) * n;
        orc_sample_uniform(seed, 0, TAG_PK_A, i, n, q, a);
        small_to_ntt(c, e, i, eh);
        for (u32 j = 0; j < n; j++)
            b[j] = addmod(negmod(mulmod(a[j], sk_ntt[(size_t)i * n + j], q), q), eh[j], q);
    }
    free(e); free(eh);
}

/* number of digits at level l: ceil((l+1)/alpha) */
u32 orc_digits(const orc_ctx *c, u32 level) { return (level + 1 + c->alpha - 1) / c->alpha; }

/* Switching key from s' (NTT form over all primes, [n_q+n_p][N]) to s.
 * For each top-level digit j: a_j uniform (NTT domain), e_j CBD,
 * b_j = -a_j s + e_j + [i in D_j] * (P mod q_i) * s'  (data primes i),
 * b_j = -a_j s + e_j                                  (special primes).
 * Layout [digits][2][n_q+n_p][N]. key_id selects the randomness stream:
 * object id = (key_id << 8) | j. */
void orc_keygen_switch(const orc_ctx *c, const u64 *sk_ntt, const u64 *sprime_ntt,
                       u64 seed, u32 key_id, u64 *swk)
{
    u32 n = nn(c), tot = c->n_q + c->n_p, dig = orc_digits(c, c->n_q - 1);
    i64 *e = (i64 *)malloc(n * sizeof(i64));
    u64 *eh = (u64 *)malloc(n * sizeof(u64));
    for (u32 j = 0; j < dig; j++) {
        u32 obj = (key_id << 8) | j;
        orc_sample_cbd(seed, obj, TAG_SWK_E, n, e);
        u32 lo = j * c->alpha, hi = lo + c->alpha; /* digit primes [lo, hi) */
        for (u32 i = 0; i < tot; i++) {
            u64 q = c->q[i];
            u64 *b = swk + (((size_t)j * 2 + 0) * tot + i) * n;
            u64 *a = swk + (((size_t)j * 2 + 1) * tot + i) * n;
            orc_sample_uniform(seed, obj, TAG_SWK_A, i, n, q, a);
            small_to_ntt(c, e, i, eh);
            u64 pmod = 1;
            for (u32 m = 0; m < c->n_p; m++) pmod = mulmod(pmod, c->q[c->n_q + m] % q, q);
            int in_digit = (i < c->n_q) && i >= lo && i < hi;
            for (u32 j2 = 0; j2 < n; j2++) {
                u64 v = addmod(negmod(mulmod(a[j2], sk_ntt[(size_t)i * n + j2], q), q), eh[j2], q);
                if (in_digit) v = addmod(v, mulmod(pmod, sprime_ntt[(size_t)i * n + j2], q), q);
                b[j2] = v;
            }
        }
    }
    free(e); free(eh);
}

/* ------------------------------------------------------------------ */
/* automorphism X -> X^g (g odd), defined on coefficients:               */
/* a_j X^j -> a_j X^(j g mod 2N), negated when j g mod 2N >= N.         */
/* On NTT-form input the oracle goes through the coefficient domain.    */
/* ------------------------------------------------------------------ */
static void automorph_coeff(u32 logn, u64 q, u64 g, const u64 *in, u64 *out)
{
    u64 n = (u64)1 << logn, two_n = n << 1;
    for (u64 j = 0; j < n; j++) {
        u64 e = (j * g) % two_n;
        if (e < n) out[e] = in[j];
        else out[e - n] = negmod(in[j], q);
    }
}

void orc_automorph_ntt(const orc_ctx *c, u32 pi, u64 g, const u64 *in, u64 *out)
{
    u32 n = nn(c);
    u64 *t = (u64 *)malloc(n * sizeof(u64));
    memcpy(t, in, n * sizeof(u64));
    orc_intt(c, pi, t);
    automorph_coeff(c->logn, c->q[pi], g, t, out);
    orc_ntt(c, pi, out);
    free(t);
}

/* Galois key for element g: switching key from sigma_g(s) to s, key id g. */
void orc_keygen_galois(const orc_ctx *c, const i64 *sk_coeff, const u64 *sk_ntt, u64 g,
                       u64 seed, u64 *gk)
{
    u32 n = nn(c), tot = c->n_q + c->n_p;
    u64 *sp = (u64 *)malloc((size_t)tot * n * sizeof(u64));
    u64 *tmp = (u64 *)malloc(n * sizeof(u64));
    for (u32 i = 0; i < tot; i++) {
        for (u32 j = 0; j < n; j++) tmp[j] = reduce_signed(sk_coeff[j], c->q[i]);
        automorph_coeff(c->logn, c->q[i], g, tmp, sp + (size_t)i * n);
        orc_ntt(c, i, sp + (size_t)i * n);
    }
    orc_keygen_switch(c, sk_ntt, sp, seed, (u32)g, gk);
    free(sp); free(tmp);
}

/* Relinearisation key: switching key from s^2 to s, key id 0. */
void orc_keygen_relin(const orc_ctx *c, const u64 *sk_ntt, u64 seed, u64 *rk)
{
    u32 n = nn(c), tot = c->n_q + c->n_p;
    u64 *s2 = (u64 *)malloc((size_t)tot * n * sizeof(u64));
    for (u32 i = 0; i < tot; i++)
        for (u32 j = 0; j < n; j++)
            s2[(size_t)i * n + j] = mulmod(sk_ntt[(size_t)i * n + j], sk_ntt[(size_t)i * n + j], c->q[i]);
    orc_keygen_switch(c, sk_ntt, s2, seed, 0, rk);
    free(s2);
}

/* ------------------------------------------------------------------ */
/* encryption / decryption (public key, at the plaintext's level)     */
/* ------------------------------------------------------------------ */
/* pt: NTT form at level l, [l+1][N]. ct out: [2][l+1][N].
 * v ternary (tag ENC_V), e0, e1 CBD (tags ENC_E0, ENC_E1), object obj. */
void orc_encrypt(const orc_ctx *c, const u64 *pk, const u64 *pt, u32 level, u64 seed, u32 obj,
                 u64 *ct)
{
    u32 n = nn(c), L = level + 1;
    i64 *v = (i64 *)malloc(n * sizeof(i64)), *e0 = (i64 *)malloc(n * sizeof(i64)),
        *e1 = (i64 *)malloc(n * sizeof(i64));
    u64 *vh = (u64 *)malloc(n * sizeof(u64)), *e0h = (u64 *)malloc(n * sizeof(u64)),
        *e1h = (u64 *)malloc(n * sizeof(u64));
    orc_sample_ternary(seed, obj, TAG_ENC_V, n, v);
    orc_sample_cbd(seed, obj, TAG_ENC_E0, n, e0);
    orc_sample_cbd(seed, obj, TAG_ENC_E1, n, e1);
    for (u32 i = 0; i < L; i++) {
        u64 q = c->q[i];
        small_to_ntt(c, v, i, vh);
        small_to_ntt(c, e0, i, e0h);
        small_to_ntt(c, e1, i, e1h);
        const u64 *b = pk + (size_t)i * n, *a = pk + ((size_t)c->n_q + i) * n;
        u64 *c0 = ct + (size_t)i * n, *c1 = ct + ((size_t)L + i) * n;
        for (u32 j = 0; j < n; j++) {
            c0[j] = addmod(addmod(mulmod(vh[j], b[j], q), e0h[j], q), pt[(size_t)i * n + j], q);
            c1[j] = addmod(mulmod(vh[j], a[j], q), e1h[j], q);
        }
    }
    free(v); free(e0); free(e1); free(vh); free(e0h); free(e1h);
}

/* m = c0 + c1 s (+ c2 s^2 for three-component input), returned in
 * coefficient form [l+1][N]. */
void orc_decrypt(const orc_ctx *c, const u64 *sk_ntt, const u64 *ct, u32 n_poly, u32 level, u64 *m)
{
    u32 n = nn(c), L = level + 1;
    for (u32 i = 0; i < L; i++) {
        u64 q = c->q[i];
        const u64 *s = sk_ntt + (size_t)i * n;
        for (u32 j = 0; j < n; j++) {
            u64 acc = ct[(size_t)i * n + j];
            u64 sp = s[j];
            for (u32 t = 1; t < n_poly; t++) {
                acc = addmod(acc, mulmod(ct[((size_t)t * L + i) * n + j], sp, q), q);
                sp = mulmod(sp, s[j], q);
            }
            m[(size_t)i * n + j] = acc;
        }
        orc_intt(c, i, m + (size_t)i * n);
    }
}

/* ------------------------------------------------------------------ */
/* residue-wise ciphertext operations                                   */
/* all operands in NTT form at level l; poly p limb i at [(p*(l+1)+i)*N] */
/* ------------------------------------------------------------------ */
void orc_add(const orc_ctx *c, const u64 *a, const u64 *b, u32 n_poly, u32 level, u64 *out)
{
    u32 n = nn(c), L = level + 1;
    for (u32 p = 0; p < n_poly; p++)
        for (u32 i = 0; i < L; i++)
            for (u32 j = 0; j < n; j++) {
                size_t o = ((size_t)p * L + i) * n + j;
                out[o] = addmod(a[o], b[o], c->q[i]);
            }
}

void orc_sub(const orc_ctx *c, const u64 *a, const u64 *b, u32 n_poly, u32 level, u64 *out)
{
    u32 n = nn(c), L = level + 1;
    for (u32 p = 0; p < n_poly; p++)
        for (u32 i = 0; i < L; i++)
            for (u32 j = 0; j < n; j++) {
                size_t o = ((size_t)p * L + i) * n + j;
                out[o] = submod(a[o], b[o], c->q[i]);
            }
}

/* ct + pt: pt added to the first component */
void orc_add_plain(const orc_ctx *c, const u64 *a, const u64 *pt, u32 n_poly, u32 level, u64 *out)
{
    u32 n = nn(c), L = level + 1;
    memcpy(out, a, (size_t)n_poly * L * n * sizeof(u64));
    for (u32 i = 0; i < L; i++)
        for (u32 j = 0; j < n; j++)
            out[(size_t)i * n + j] = addmod(a[(size_t)i * n + j], pt[(size_t)i * n + j], c->q[i]);
}

void orc_mul_plain(const orc_ctx *c, const u64 *a, const u64 *pt, u32 n_poly, u32 level, u64 *out)
{
    u32 n = nn(c), L = level + 1;
    for (u32 p = 0; p < n_poly; p++)
        for (u32 i = 0; i < L; i++)
            for (u32 j = 0; j < n; j++) {
                size_t o = ((size_t)p * L + i) * n + j;
                out[o] = mulmod(a[o], pt[(size_t)i * n + j], c->q[i]);
            }
}

/* multiply by the constant polynomial v (signed integer), i.e. every
 * residue of limb i times v mod q_i (a constant is a constant polynomial) */
void orc_mul_const(const orc_ctx *c, const u64 *a, i64 v, u32 n_poly, u32 level, u64 *out)
{
    u32 n = nn(c), L = level + 1;
    for (u32 p = 0; p < n_poly; p++)
        for (u32 i = 0; i < L; i++) {
            u64 w = reduce_signed(v, c->q[i]);
            for (u32 j = 0; j < n; j++) {
                size_t o = ((size_t)p * L + i) * n + j;
                out[o] = mulmod(a[o], w, c->q[i]);
            }
        }
}

/* add the constant polynomial v to the first component: in the NTT domain
 * a constant polynomial is the same value in every slot */
void orc_add_const(const orc_ctx *c, const u64 *a, i64 v, u32 n_poly, u32 level, u64 *out)
{
    u32 n = nn(c), L = level + 1;
    memcpy(out, a, (size_t)n_poly * L * n * sizeof(u64));
    for (u32 i = 0; i < L; i++) {
        u64 w = reduce_signed(v, c->q[i]);
        for (u32 j = 0; j < n; j++) out[(size_t)i * n + j] = addmod(a[(size_t)i * n + j], w, c->q[i]);
    }
}

/* ct x ct tensor: (a0 b0, a0 b1 + a1 b0, a1 b1), out [3][l+1][N] */
void orc_tensor(const orc_ctx *c, const u64 *a, const u64 *b, u32 level, u64 *out)
{
    u32 n = nn(c), L = level + 1;
    for (u32 i = 0; i < L; i++) {
        u64 q = c->q[i];
        for (u32 j = 0; j < n; j++) {
            size_t o0 = (size_t)i * n + j, o1 = ((size_t)L + i) * n + j;
            u64 a0 = a[o0], a1 = a[o1], b0 = b[o0], b1 = b[o1];
            out[o0] = mulmod(a0, b0, q);
            out[o1] = addmod(mulmod(a0, b1, q), mulmod(a1, b0, q), q);
            out[((size_t)2 * L + i) * n + j] = mulmod(a1, b1, q);
        }
    }
}

/* ------------------------------------------------------------------ */
/* rescale (rounding division by the top prime)                        */
/* c' = floor((c + h) / q_l), h = floor(q_l / 2), per coefficient of the */
/* CRT value; RNS form: r = [c_l + h]_{q_l}, c'_i = (c_i - (r - h)) q_l^-1 */
/* ------------------------------------------------------------------ */
void orc_rescale(const orc_ctx *c, const u64 *in, u32 n_poly, u32 level, u64 *out)
{
    u32 n = nn(c), L = level + 1, Lo = level;
    u64 ql = c->q[level], h = ql >> 1;
    u64 *last = (u64 *)malloc(n * sizeof(u64)), *v = (u64 *)malloc(n * sizeof(u64));
    for (u32 p = 0; p < n_poly; p++) {
        memcpy(last, in + ((size_t)p * L + level) * n, n * sizeof(u64));
        orc_intt(c, level, last);
        for (u32 i = 0; i < Lo; i++) {
            u64 q = c->q[i];
            for (u32 j = 0; j < n; j++) {
                u64 r = addmod(last[j], h, ql);
                /* (r - h) as a signed integer, reduced mod q */
                v[j] = r >= h ? (r - h) % q : negmod((h - r) % q, q);
            }
            orc_ntt(c, i, v);
            u64 qinv = invmod(ql % q, q);
            for (u32 j = 0; j < n; j++) {
                size_t oi = ((size_t)p * L + i) * n + j;
                out[((size_t)p * Lo + i) * n + j] = mulmod(submod(in[oi], v[j], q), qinv, q);
            }
        }
    }
    free(last); free(v);
}

/* level match: keep the first (to+1) limbs of each poly */
void orc_mod_switch(const orc_ctx *c, const u64 *in, u32 n_poly, u32 level, u32 to, u64 *out)
{
    u32 n = nn(c), L = level + 1, Lo = to + 1;
    for (u32 p = 0; p < n_poly; p++)
        memcpy(out + (size_t)p * Lo * n, in + (size_t)p * L * n, (size_t)Lo * n * sizeof(u64));
}

/* ------------------------------------------------------------------ */
/* hybrid key switching (approximate ModUp, floor ModDown)            */
/* ------------------------------------------------------------------ */
/* prime index of target t in the extended basis Q_l U P: t <= l -> data
 * prime t, t > l -> special prime t - (l+1). */
static u32 ext_prime(const orc_ctx *c, u32 level, u32 t)
{
    return t <= level ? t : c->n_q + (t - level - 1);
}

/* ModUp of digit j at level l: x (coefficient form, limbs D_j) to the
 * target prime index pt: sum_{i in D_j} [x_i (Q_D/q_i)^-1]_{q_i} (Q_D/q_i)
 * mod q_pt, written out per coefficient. */
void orc_modup_digit(const orc_ctx *c, const u64 *x_coeff /* limbs lo..hi-1 */, u32 lo, u32 hi,
                     u32 pt, u64 *out)
{
    u32 n = nn(c);
    u64 qt = c->q[pt];
    for (u32 j = 0; j < n; j++) out[j] = 0;
    for (u32 i = lo; i < hi; i++) {
        u64 qi = c->q[i];
        u64 hat_mod_qi = 1, hat_mod_qt = 1;
        for (u32 m = lo; m < hi; m++)
            if (m != i) {
                hat_mod_qi = mulmod(hat_mod_qi, c->q[m] % qi, qi);
                hat_mod_qt = mulmod(hat_mod_qt, c->q[m] % qt, qt);
            }
        u64 hat_inv = invmod(hat_mod_qi, qi);
        for (u32 j = 0; j < n; j++) {
            u64 y = mulmod(x_coeff[(size_t)(i - lo) * n + j], hat_inv, qi);
            out[j] = addmod(out[j], mulmod(y % qt, hat_mod_qt, qt), qt);
        }
    }
}

/* ModDown of a polynomial over Q_l U P (NTT form, [l+1+k][N]) to Q_l:
 * out_i = (a_i - Conv_{P->q_i}([a]_P)) * P^-1 mod q_i. */
void orc_moddown(const orc_ctx *c, const u64 *a, u32 level, u64 *out)
{
    u32 n = nn(c), L = level + 1, k = c->n_p;
    u64 *ap = (u64 *)malloc((size_t)k * n * sizeof(u64)), *conv = (u64 *)malloc(n * sizeof(u64));
    for (u32 m = 0; m < k; m++) {
        memcpy(ap + (size_t)m * n, a + ((size_t)L + m) * n, n * sizeof(u64));
        orc_intt(c, c->n_q + m, ap + (size_t)m * n);
    }
    for (u32 i = 0; i < L; i++) {
        u64 q = c->q[i];
        orc_modup_digit(c, ap, c->n_q, c->n_q + k, i, conv);
        orc_ntt(c, i, conv);
        u64 pmod = 1;
        for (u32 m = 0; m < k; m++) pmod = mulmod(pmod, c->q[c->n_q + m] % q, q);
        u64 pinv = invmod(pmod, q);
        for (u32 j = 0; j < n; j++)
            out[(size_t)i * n + j] = mulmod(submod(a[(size_t)i * n + j], conv[j], q), pinv, q);
    }
    free(ap); free(conv);
}

/* Key switch of d (NTT form at level l, [l+1][N]) with switching key swk
 * ([digits][2][n_q+n_p][N]): returns (ks0, ks1), [2][l+1][N]. */
void orc_keyswitch(const orc_ctx *c, const u64 *d, u32 level, const u64 *swk, u64 *ks)
{
    u32 n = nn(c), L = level + 1, k = c->n_p, E = L + k, tot = c->n_q + c->n_p;
    u32 beta = orc_digits(c, level);
    u64 *dc = (u64 *)malloc((size_t)L * n * sizeof(u64));
    u64 *acc = (u64 *)calloc((size_t)2 * E * n, sizeof(u64));
    u64 *ext = (u64 *)malloc(n * sizeof(u64));
    memcpy(dc, d, (size_t)L * n * sizeof(u64));
    for (u32 i = 0; i < L; i++) orc_intt(c, i, dc + (size_t)i * n);
    for (u32 j = 0; j < beta; j++) {
        u32 lo = j * c->alpha, hi = lo + c->alpha;
        if (hi > L) hi = L;
        for (u32 t = 0; t < E; t++) {
            u32 pt = ext_prime(c, level, t);
            u64 q = c->q[pt];
            if (t >= lo && t < hi) {
                memcpy(ext, d + (size_t)t * n, n * sizeof(u64));
            } else {
                orc_modup_digit(c, dc + (size_t)lo * n, lo, hi, pt, ext);
                orc_ntt(c, pt, ext);
            }
            const u64 *k0 = swk + (((size_t)j * 2 + 0) * tot + pt) * n;
            const u64 *k1 = swk + (((size_t)j * 2 + 1) * tot + pt) * n;
            for (u32 x = 0; x < n; x++) {
                acc[(size_t)t * n + x] = addmod(acc[(size_t)t * n + x], mulmod(ext[x], k0[x], q), q);
                acc[((size_t)E + t) * n + x] =
                    addmod(acc[((size_t)E + t) * n + x], mulmod(ext[x], k1[x], q), q);
            }
        }
    }
    orc_moddown(c, acc, level, ks);
    orc_moddown(c, acc + (size_t)E * n, level, ks + (size_t)L * n);
    free(dc); free(acc); free(ext);
}

/* relinearise a three-component ciphertext: (d0 + ks0(d2), d1 + ks1(d2)) */
void orc_relinearize(const orc_ctx *c, const u64 *ct3, u32 level, const u64 *rk, u64 *out)
{
    u32 n = nn(c), L = level + 1;
    u64 *ks = (u64 *)malloc((size_t)2 * L * n * sizeof(u64));
    orc_keyswitch(c, ct3 + (size_t)2 * L * n, level, rk, ks);
    orc_add(c, ct3, ks, 2, level, out);
    free(ks);
}

/* apply the automorphism g to both components, then key-switch the
 * second with the Galois key for g: (sigma(c0) + ks0, ks1) */
void orc_apply_galois(const orc_ctx *c, const u64 *ct, u32 level, u64 g, const u64 *gk, u64 *out)
{
    u32 n = nn(c), L = level + 1;
    u64 *s0 = (u64 *)malloc((size_t)L * n * sizeof(u64)), *s1 = (u64 *)malloc((size_t)L * n * sizeof(u64));
    u64 *ks = (u64 *)malloc((size_t)2 * L * n * sizeof(u64));
    for (u32 i = 0; i < L; i++) {
        orc_automorph_ntt(c, i, g, ct + (size_t)i * n, s0 + (size_t)i * n);
        orc_automorph_ntt(c, i, g, ct + ((size_t)L + i) * n, s1 + (size_t)i * n);
    }
    orc_keyswitch(c, s1, level, gk, ks);
    for (u32 i = 0; i < L; i++)
        for (u32 j = 0; j < n; j++) {
            out[(size_t)i * n + j] = addmod(s0[(size_t)i * n + j], ks[(size_t)i * n + j], c->q[i]);
            out[((size_t)L + i) * n + j] = ks[((size_t)L + i) * n + j];
        }
    free(s0); free(s1); free(ks);
}

/* HMult followed by relinearisation and rescale: the composition the
 * meta-object performs after a ciphertext product. out [2][l][N]. */
void orc_mul_relin_rescale(const orc_ctx *c, const u64 *a, const u64 *b, u32 level, const u64 *rk,
                           u64 *out)
{
    u32 n = nn(c), L = level + 1;
    u64 *t3 = (u64 *)malloc((size_t)3 * L * n * sizeof(u64));
    u64 *t2 = (u64 *)malloc((size_t)2 * L * n * sizeof(u64));
    orc_tensor(c, a, b, level, t3);
    orc_relinearize(c, t3, level, rk, t2);
    orc_rescale(c, t2, 2, level, out);
    free(t3); free(t2);
}

/* sum_k w_k * ct_k over n ciphertexts (same level, n_poly polys each):
 * the definition of a linear layer with integer weights (each weight a
 * constant polynomial), evaluated residue by residue. */
void orc_lincomb(const orc_ctx *c, const u64 *const *cts, const i64 *w, u32 n, u32 n_poly, u32 level,
                 u64 *out)
{
    u32 nn_ = nn(c), L = level + 1;
    for (u32 p = 0; p < n_poly; p++)
        for (u32 i = 0; i < L; i++) {
            u64 q = c->q[i];
            u64 *o = out + ((size_t)p * L + i) * nn_;
            for (u32 j = 0; j < nn_; j++) o[j] = 0;
            for (u32 k = 0; k < n; k++) {
                u64 wk = reduce_signed(w[k], q);
                const u64 *x = cts[k] + ((size_t)p * L + i) * nn_;
                for (u32 j = 0; j < nn_; j++) o[j] = addmod(o[j], mulmod(x[j], wk, q), q);
            }
        }
}

/* ------------------------------------------------------------------ */
/* Rotations of one ciphertext with plaintext weights, all rotations     */
/* sharing one decomposition (hoisting) and one ModDown (the diagonal    */
/* matrix-vector product of a dense layer, Section 4.2.3):               */
/*   D_j  = ModUp of digit j of c1 to Q_l U P, NTT form (own limbs = c1) */
/*   T0   = sum_i pt_i * ( sum_j sigma_gi(D_j) * b_{gi,j} + P sigma_gi(c0) ) */
/*   T1   = sum_i pt_i * ( sum_j sigma_gi(D_j) * a_{gi,j} )              */
/*   out  = (ModDown(T0), ModDown(T1)),  g = 1: the term pt_i * (P c0, P c1) */
/* pt_i are integer polynomials reduced to every prime of Q_l U P.       */
/* ------------------------------------------------------------------ */
void orc_hoisted_linear(const orc_ctx *c, const u64 *ct, u32 level, u32 n_rot, const u64 *galois,
                        const u64 *const *gks, const i64 *pt_coeffs, u64 *out)
{
    u32 n = nn(c), L = level + 1, k = c->n_p, E = L + k, tot = c->n_q + c->n_p;
    u32 beta = orc_digits(c, level);
    const u64 *c0 = ct, *c1 = ct + (size_t)L * n;
    u64 *dc = (u64 *)malloc((size_t)L * n * sizeof(u64));
    u64 *D = (u64 *)malloc((size_t)beta * E * n * sizeof(u64));
    u64 *T = (u64 *)calloc((size_t)2 * E * n, sizeof(u64));
    u64 *pt = (u64 *)malloc(n * sizeof(u64)), *sd = (u64 *)malloc(n * sizeof(u64));
    u64 *b = (u64 *)malloc(n * sizeof(u64)), *a = (u64 *)malloc(n * sizeof(u64));
    memcpy(dc, c1, (size_t)L * n * sizeof(u64));
    for (u32 i = 0; i < L; i++) orc_intt(c, i, dc + (size_t)i * n);
    for (u32 j = 0; j < beta; j++) {
        u32 lo = j * c->alpha, hi = lo + c->alpha;
        if (hi > L) hi = L;
        for (u32 t = 0; t < E; t++) {
            u64 *dst = D + ((size_t)j * E + t) * n;
            if (t >= lo && t < hi) {
                memcpy(dst, c1 + (size_t)t * n, n * sizeof(u64));
            } else {
                u32 p = ext_prime(c, level, t);
                orc_modup_digit(c, dc + (size_t)lo * n, lo, hi, p, dst);
                orc_ntt(c, p, dst);
            }
        }
    }
    for (u32 r = 0; r < n_rot; r++) {
        u64 g = galois[r];
        for (u32 t = 0; t < E; t++) {
            u32 p = ext_prime(c, level, t);
            u64 q = c->q[p];
            u64 pmod = 1;
            for (u32 m = 0; m < k; m++) pmod = mulmod(pmod, c->q[c->n_q + m] % q, q);
            for (u32 x = 0; x < n; x++) pt[x] = reduce_signed(pt_coeffs[(size_t)r * n + x], q);
            orc_ntt(c, p, pt);
            if (g == 1) {
                if (t >= L) continue; /* P c is zero on the special primes */
                for (u32 x = 0; x < n; x++) {
                    b[x] = mulmod(pmod, c0[(size_t)t * n + x], q);
                    a[x] = mulmod(pmod, c1[(size_t)t * n + x], q);
                }
            } else {
                for (u32 x = 0; x < n; x++) b[x] = a[x] = 0;
                for (u32 j = 0; j < beta; j++) {
                    orc_automorph_ntt(c, p, g, D + ((size_t)j * E + t) * n, sd);
                    const u64 *k0 = gks[r] + (((size_t)j * 2 + 0) * tot + p) * n;
                    const u64 *k1 = gks[r] + (((size_t)j * 2 + 1) * tot + p) * n;
                    for (u32 x = 0; x < n; x++) {
                        b[x] = addmod(b[x], mulmod(sd[x], k0[x], q), q);
                        a[x] = addmod(a[x], mulmod(sd[x], k1[x], q), q);
                    }
                }
                if (t < L) {
                    orc_automorph_ntt(c, p, g, c0 + (size_t)t * n, sd);
                    for (u32 x = 0; x < n; x++) b[x] = addmod(b[x], mulmod(pmod, sd[x], q), q);
                }
            }
            for (u32 x = 0; x < n; x++) {
                T[(size_t)t * n + x] = addmod(T[(size_t)t * n + x], mulmod(pt[x], b[x], q), q);
                T[((size_t)E + t) * n + x] = addmod(T[((size_t)E + t) * n + x], mulmod(pt[x], a[x], q), q);
            }
        }
    }
    orc_moddown(c, T, level, out);
    orc_moddown(c, T + (size_t)E * n, level, out + (size_t)L * n);
    free(dc); free(D); free(T); free(pt); free(sd); free(b); free(a);
}
