/* Drives every entry point of the C oracle (oracle/ckks_oracle.c) on a small chain,
 * built with AddressSanitizer and UndefinedBehaviorSanitizer (and LeakSanitizer at
 * exit) by tests/test_sanitizers.py: out-of-bounds accesses, use after free, signed
 * overflow, misaligned or out-of-range shifts and leaked buffers end the run with a
 * report and a non-zero status.  A few cheap identities are checked on the way. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct oc_ctx oc_ctx;
typedef struct oc_ct oc_ct;
oc_ctx *oc_ctx_create(int, int, int, int, int, int, uint64_t);
oc_ctx *oc_ctx_create_ex(int, int, int, int, int, int, uint64_t, int, int, int);
void oc_ctx_free(oc_ctx *);
int oc_ctx_info(const oc_ctx *, int *, int *, int *, int *);
void oc_ctx_primes(const oc_ctx *, uint64_t *);
void oc_ctx_secret(const oc_ctx *, int8_t *);
void oc_set_nonce(oc_ctx *, uint32_t);
uint32_t oc_get_nonce(const oc_ctx *);
int oc_keygen(oc_ctx *, int);
int oc_keygen_galois(oc_ctx *, int, uint64_t);
void oc_ct_free(oc_ct *);
int oc_ct_level(const oc_ct *);
void oc_ct_export(const oc_ctx *, const oc_ct *, uint64_t *);
oc_ct *oc_ct_import(const oc_ctx *, const uint64_t *, int);
void oc_schoolbook(const uint64_t *, const uint64_t *, uint64_t *, int, uint64_t);
void oc_ring_mul(const oc_ctx *, int, const uint64_t *, const uint64_t *, uint64_t *);
oc_ct *oc_encrypt(oc_ctx *, const int64_t *);
void oc_decrypt(const oc_ctx *, const oc_ct *, double *);
oc_ct *oc_add(const oc_ctx *, const oc_ct *, const oc_ct *);
oc_ct *oc_sub(const oc_ctx *, const oc_ct *, const oc_ct *);
oc_ct *oc_mul_int(const oc_ctx *, const oc_ct *, int64_t);
oc_ct *oc_add_const_int(const oc_ctx *, const oc_ct *, int64_t);
oc_ct *oc_drop(const oc_ctx *, const oc_ct *, int);
oc_ct *oc_rescale(const oc_ctx *, const oc_ct *);
oc_ct *oc_mul_int_rescale(const oc_ctx *, const oc_ct *, int64_t);
int oc_keyswitch(const oc_ctx *, const uint64_t *, int, int, uint64_t *, uint64_t *);
oc_ct *oc_mul(const oc_ctx *, const oc_ct *, const oc_ct *);
oc_ct *oc_mul_norescale(const oc_ctx *, const oc_ct *, const oc_ct *);
oc_ct *oc_rotate(const oc_ctx *, const oc_ct *, int);
oc_ct *oc_rotate_gal(const oc_ctx *, const oc_ct *, int, uint64_t);
oc_ct *oc_mul_plain(const oc_ctx *, const oc_ct *, const int64_t *);
oc_ct *oc_modraise(const oc_ctx *, const oc_ct *, int);
oc_ct *oc_rotsum_step(const oc_ctx *, const oc_ct *, int, const int *, const uint64_t *);
oc_ct *oc_rotsum_carried(const oc_ctx *, const oc_ct *, int, const int *, const int *, const uint64_t *);
oc_ct *oc_automorph(const oc_ctx *, const oc_ct *, uint64_t);
int oc_num_threads(void);
void oc_set_num_threads(int);

static int fails = 0;
#define CHECK(c, msg) do { if (!(c)) { fprintf(stderr, "check failed: %s\n", msg); ++fails; } } while (0)

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void) { rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17; return rng; }

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t m) {
    unsigned __int128 r = 1, x = b % m;
    for (; e; e >>= 1, x = x * x % m) if (e & 1) r = r * x % m;
    return (uint64_t)r;
}

int main(void) {
    const int log_n = 10, N = 1 << log_n, n_q = 6;
    oc_set_num_threads(2);
    oc_ctx *C = oc_ctx_create(log_n, n_q, 48, 40, 48, 3, 7);
    CHECK(C != NULL, "context");
    int n, L, alpha, np;
    oc_ctx_info(C, &n, &L, &alpha, &np);
    CHECK(n == N && L == n_q - 1, "info");
    uint64_t *q = malloc(8 * (size_t)np);
    oc_ctx_primes(C, q);
    int8_t *s = malloc((size_t)N);
    oc_ctx_secret(C, s);
    oc_set_nonce(C, 3);
    CHECK(oc_get_nonce(C) == 3, "nonce");
    /* keys: relinearisation, rotations by 2^k, rotation by 3, conjugation; bad index */
    CHECK(oc_keygen(C, 0) == 0, "relin key");
    for (int k = 1; k < log_n; ++k) CHECK(oc_keygen(C, k) == 0, "rotation key");
    CHECK(oc_keygen_galois(C, 20, powmod(5, 3, 2 * (uint64_t)N)) == 0, "galois key");
    CHECK(oc_keygen_galois(C, 21, 2 * (uint64_t)N - 1) == 0, "conjugation key");
    CHECK(oc_keygen(C, 100000) != 0, "key index out of range refused");

    /* ring product against schoolbook on prime 0 */
    uint64_t *a = malloc(8 * (size_t)N), *b = malloc(8 * (size_t)N), *c1 = malloc(8 * (size_t)N),
             *c2 = malloc(8 * (size_t)N);
    for (int i = 0; i < N; ++i) { a[i] = next_u64() % q[0]; b[i] = next_u64() % q[0]; }
    oc_ring_mul(C, 0, a, b, c1);
    oc_schoolbook(a, b, c2, N, q[0]);
    CHECK(memcmp(c1, c2, 8 * (size_t)N) == 0, "ring_mul == schoolbook");

    /* encrypt / decrypt round trip */
    int64_t *m = malloc(8 * (size_t)N), *m2 = malloc(8 * (size_t)N);
    for (int i = 0; i < N; ++i) { m[i] = (int64_t)(next_u64() % (1u << 30)) - (1 << 29); m2[i] = (int64_t)(next_u64() % 64) - 32; }
    oc_ct *x = oc_encrypt(C, m), *y = oc_encrypt(C, m);
    CHECK(x && oc_ct_level(x) == L, "encrypt");
    double *d = malloc(8 * (size_t)N);
    oc_decrypt(C, x, d);
    double e = 0;
    for (int i = 0; i < N; ++i) { double t = d[i] - (double)m[i]; if (t < 0) t = -t; if (t > e) e = t; }
    CHECK(e < 1e4, "decrypt(encrypt(m)) ~ m");

    /* export / import */
    uint64_t *buf = malloc(8 * 2 * (size_t)(L + 1) * N);
    oc_ct_export(C, x, buf);
    oc_ct *xi = oc_ct_import(C, buf, L);
    uint64_t *buf2 = malloc(8 * 2 * (size_t)(L + 1) * N);
    oc_ct_export(C, xi, buf2);
    CHECK(memcmp(buf, buf2, 8 * 2 * (size_t)(L + 1) * N) == 0, "export/import");

    /* every operation once, results freed */
    oc_ct *r[32];
    int k = 0;
    r[k++] = oc_add(C, x, y);
    r[k++] = oc_sub(C, x, y);
    r[k++] = oc_mul_int(C, x, -3);
    r[k++] = oc_add_const_int(C, x, 12345);
    r[k++] = oc_drop(C, x, 2);
    r[k++] = oc_rescale(C, x);
    r[k++] = oc_mul_int_rescale(C, x, 1 << 20);
    r[k++] = oc_mul(C, x, y);
    r[k++] = oc_mul_norescale(C, x, y);
    r[k++] = oc_rotate(C, x, 0);
    r[k++] = oc_rotate(C, x, log_n - 2);
    r[k++] = oc_rotate_gal(C, x, 20, powmod(5, 3, 2 * (uint64_t)N));
    r[k++] = oc_rotate_gal(C, x, 21, 2 * (uint64_t)N - 1);
    r[k++] = oc_mul_plain(C, x, m2);
    r[k++] = oc_automorph(C, x, powmod(5, 3, 2 * (uint64_t)N));
    {
        int kid[3] = {1, 2, 20};
        uint64_t gal[3] = {5, 25 % (2 * (uint64_t)N), powmod(5, 3, 2 * (uint64_t)N)};
        r[k++] = oc_rotsum_step(C, x, 3, kid, gal);
        const int nr2[2] = {2, 1};
        r[k++] = oc_rotsum_carried(C, x, 2, nr2, kid, gal);
        r[k++] = oc_rotsum_carried(C, r[4], 2, nr2, kid, gal);   /* at a lower level */
    }
    oc_ct *low = oc_drop(C, x, 0);
    r[k++] = oc_modraise(C, low, L);
    r[k++] = oc_mul(C, r[5], r[5]);      /* at a lower level */
    r[k++] = oc_rotate(C, r[4], 1);      /* partial digit */
    for (int i = 0; i < k; ++i) CHECK(r[i] != NULL, "operation returned a ciphertext");
    CHECK(oc_rotate(C, x, log_n + 3) == NULL, "rotation without a key refused");
    {
        uint64_t *o0 = malloc(8 * (size_t)(L + 1) * N), *o1 = malloc(8 * (size_t)(L + 1) * N);
        CHECK(oc_keyswitch(C, buf + (size_t)(L + 1) * N, L, 0, o0, o1) == 0, "keyswitch");
        free(o0); free(o1);
    }
    for (int i = 0; i < k; ++i) oc_ct_free(r[i]);
    oc_ct_free(low); oc_ct_free(x); oc_ct_free(y); oc_ct_free(xi);
    free(buf); free(buf2); free(d); free(m); free(m2); free(a); free(b); free(c1); free(c2); free(q); free(s);
    oc_ctx_free(C);

    /* the extended constructor (top primes of another width, sparse secret) and a refusal */
    oc_ctx *B = oc_ctx_create_ex(log_n, 8, 48, 40, 48, 3, 9, 2, 44, 32);
    CHECK(B != NULL, "extended context");
    CHECK(oc_keygen(B, 0) == 0, "extended relin key");
    oc_ctx_free(B);
    CHECK(oc_ctx_create(2, 4, 48, 40, 48, 3, 1) == NULL, "log_n out of range refused");
    CHECK(oc_num_threads() >= 1, "threads");
    if (fails) { fprintf(stderr, "%d checks failed\n", fails); return 1; }
    printf("oracle driver: ok\n");
    return 0;
}
