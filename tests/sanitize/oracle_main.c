/* Drives every oracle routine once on a small ring (N = 2^10, primes of
 * 60, 40, 40 bits + one 60-bit special prime, and a 4 x 50 + 2 x 60-bit
 * chain with two-prime digits) so that an AddressSanitizer /
 * UndefinedBehaviorSanitizer build can check their memory accesses and
 * integer arithmetic. Exit status 0 when every call returned and a
 * decrypted product is close to the expected value. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;
typedef struct orc_ctx orc_ctx;

int orc_find_primes(u32 logn, const u32 *bits, u32 n, u64 *out);
orc_ctx *orc_ctx_create(u32 logn, const u64 *primes, u32 n_q, u32 n_p, u32 dnum);
void orc_ctx_destroy(orc_ctx *c);
u32 orc_digits(const orc_ctx *c, u32 level);
void orc_ntt(const orc_ctx *c, u32 prime, u64 *a);
void orc_intt(const orc_ctx *c, u32 prime, u64 *a);
void orc_keygen_secret(const orc_ctx *c, u64 seed, i64 *s, u64 *sn);
void orc_keygen_public(const orc_ctx *c, const u64 *sn, u64 seed, u64 *pk);
void orc_keygen_relin(const orc_ctx *c, const u64 *sn, u64 seed, u64 *rk);
void orc_keygen_galois(const orc_ctx *c, const i64 *s, const u64 *sn, u64 g, u64 seed, u64 *gk);
void orc_encrypt(const orc_ctx *c, const u64 *pk, const u64 *pt, u32 level, u64 seed, u32 obj, u64 *ct);
void orc_decrypt(const orc_ctx *c, const u64 *sn, const u64 *ct, u32 n_poly, u32 level, u64 *m);
void orc_tensor(const orc_ctx *c, const u64 *a, const u64 *b, u32 level, u64 *out);
void orc_relinearize(const orc_ctx *c, const u64 *ct3, u32 level, const u64 *rk, u64 *out);
void orc_rescale(const orc_ctx *c, const u64 *a, u32 n_poly, u32 level, u64 *out);
void orc_mul_relin_rescale(const orc_ctx *c, const u64 *a, const u64 *b, u32 level, const u64 *rk, u64 *out);
void orc_apply_galois(const orc_ctx *c, const u64 *ct, u32 level, u64 g, const u64 *gk, u64 *out);
void orc_mul_const(const orc_ctx *c, const u64 *a, i64 v, u32 n_poly, u32 level, u64 *out);
void orc_add_const(const orc_ctx *c, const u64 *a, i64 v, u32 n_poly, u32 level, u64 *out);
void orc_lincomb(const orc_ctx *c, const u64 *const *cts, const i64 *w, u32 n, u32 n_poly, u32 level, u64 *out);
void orc_hoisted_linear(const orc_ctx *c, const u64 *ct, u32 level, u32 n_rot, const u64 *galois,
                        const u64 *const *keys, const i64 *pt, u64 *out);

#define LOGN 10
#define N (1u << LOGN)

static int run_chain(const u32 *bits, u32 n_q, u32 n_p, u32 dnum) {
    u64 primes[8];
    if (orc_find_primes(LOGN, bits, n_q + n_p, primes) != 0) return 1;
    orc_ctx *c = orc_ctx_create(LOGN, primes, n_q, n_p, dnum);
    if (!c) return 2;
    const u32 L = n_q, P = n_q + n_p, top = n_q - 1, D = orc_digits(c, top);
    const size_t key = (size_t)D * 2 * P * N;
    i64 *s = calloc(N, sizeof(i64));
    u64 *sn = calloc((size_t)P * N, 8), *pk = calloc((size_t)2 * L * N, 8), *rk = calloc(key, 8);
    u64 *gk = calloc(key, 8), *gk2 = calloc(key, 8);
    orc_keygen_secret(c, 1, s, sn);
    orc_keygen_public(c, sn, 2, pk);
    orc_keygen_relin(c, sn, 3, rk);
    const u64 g5 = 5, g3 = (5u * 5u * 5u) % (2 * N);
    orc_keygen_galois(c, s, sn, g5, 4, gk);
    orc_keygen_galois(c, s, sn, g3, 5, gk2);
    /* plaintext: the constant 2^30 in every slot (constant polynomial), NTT form */
    u64 *pt = calloc((size_t)L * N, 8);
    for (u32 i = 0; i < L; i++) {
        pt[(size_t)i * N] = (u64)1 << 30;
        orc_ntt(c, i, pt + (size_t)i * N);
    }
    u64 *a = calloc((size_t)2 * L * N, 8), *b = calloc((size_t)2 * L * N, 8), *t3 = calloc((size_t)3 * L * N, 8);
    u64 *r2 = calloc((size_t)2 * L * N, 8), *o = calloc((size_t)2 * L * N, 8), *m = calloc((size_t)L * N, 8);
    orc_encrypt(c, pk, pt, top, 6, 0, a);
    orc_encrypt(c, pk, pt, top, 6, 1, b);
    orc_tensor(c, a, b, top, t3);
    orc_decrypt(c, sn, t3, 3, top, m);
    orc_relinearize(c, t3, top, rk, r2);
    orc_rescale(c, r2, 2, top, o);
    orc_mul_relin_rescale(c, a, b, top, rk, r2);
    if (memcmp(r2, o, (size_t)2 * top * N * 8) != 0) return 3;  /* fused == sequence */
    orc_apply_galois(c, a, top, g5, gk, o);
    orc_mul_const(c, a, -12345, 2, top, o);
    orc_add_const(c, o, 777, 2, top, r2);
    const u64 *cts[3] = {a, b, r2};
    const i64 w[3] = {3, -((i64)1 << 40), 5};
    orc_lincomb(c, cts, w, 3, 2, top, o);
    const u64 gal[3] = {1, g5, g3};
    const u64 *keys[3] = {NULL, gk, gk2};
    i64 *pts = calloc((size_t)3 * N, sizeof(i64));
    for (u32 k = 0; k < 3 * N; k++) pts[k] = (i64)(k % 7) - 3;
    orc_hoisted_linear(c, a, top, 3, gal, keys, pts, o);
    /* decrypt a(x) b(x) relinearised and rescaled: constant term 2^60 / q_top plus noise */
    orc_mul_relin_rescale(c, a, b, top, rk, r2);
    orc_decrypt(c, sn, r2, 2, top - 1, m); /* coefficient form */
    const double want = (double)((u64)1 << 60) / (double)primes[top];
    const u64 q0 = primes[0];
    const u64 v = m[0] > q0 / 2 ? q0 - m[0] : m[0];
    const double err = (double)v - want;
    int rc = (err > 1e4 || err < -1e4) ? 4 : 0;
    free(s); free(sn); free(pk); free(rk); free(gk); free(gk2); free(pt); free(a); free(b); free(t3);
    free(r2); free(o); free(m); free(pts);
    orc_ctx_destroy(c);
    return rc;
}

int main(void) {
    const u32 net[4] = {60, 40, 40, 60};
    const u32 wide[6] = {50, 50, 50, 50, 60, 60};
    int rc = run_chain(net, 3, 1, 3);
    if (rc) { printf("net chain failed: %d\n", rc); return rc; }
    rc = run_chain(wide, 4, 2, 2);
    if (rc) { printf("wide chain failed: %d\n", rc); return rc; }
    printf("oracle driver ok\n");
    return 0;
}
