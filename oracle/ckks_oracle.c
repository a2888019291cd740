/*
 * O2: a plain CPU RNS-CKKS -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load
 * this library.  It shares no code, header, table or constant generator with
 * the HIP path; the two meet only in shared conventions (prime search order,
 * Philox counters and object ids, key layout, rounding rules), each side
 * implementing them on its own from their statement.
 *
 * The paper runs its encrypted experiments in CKKS (Sec. 2.1 properties;
 * Sec. 3.2 SIMD slots and rotations; Alg. 2).  It states no scheme internals,
 * so this file follows the public literature:
 *   - full-RNS CKKS (Cheon, Han, Kim, Kim, Song, SAC 2018): residues per prime,
 *     rescale by the last prime with a centred remainder;
 *   - hybrid key switching with dnum digits (Han, Ki, CT-RSA 2020): digit
 *     decomposition, fast basis conversion up to Q_l u P, key inner product,
 *     division by P;
 *   - Philox4x32-10 (Salmon et al., SC 2011) for every random draw.
 *
 * Representation: every ciphertext polynomial is kept in the COEFFICIENT
 * domain, one residue vector per prime, canonical in [0, q).  A ring product
 * is computed the textbook way: twist by psi^i, cyclic NTT with omega = psi^2,
 * point-wise product, inverse NTT, untwist.  Arithmetic is scalar
 * unsigned __int128 with '%'.  Keys are stored transformed (a cached NTT).
 * OpenMP is used across limbs only.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------- */
/* modular helpers                                                            */
/* ------------------------------------------------------------------------- */
static inline uint64_t mulm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
static inline uint64_t addm(uint64_t a, uint64_t b, uint64_t q) { uint64_t s = a + b; return s >= q ? s - q : s; }
static inline uint64_t subm(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }
static uint64_t powm(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q; a %= q;
    while (e) { if (e & 1) r = mulm(r, a, q); a = mulm(a, a, q); e >>= 1; }
    return r;
}
static uint64_t invm(uint64_t a, uint64_t q) { return powm(a, q - 2, q); } /* q prime */
static inline uint64_t red_i64(int64_t v, uint64_t q) {
    int64_t r = v % (int64_t)q; if (r < 0) r += (int64_t)q; return (uint64_t)r;
}

/* the centred representative of v in [0, q) (in (-q/2, q/2]) reduced modulo p */
static inline uint64_t centred_mod(uint64_t v, uint64_t q, uint64_t p) {
    return v > (q - 1) / 2 ? subm(0, (q - v) % p, p) : v % p;
}
/* deterministic Miller-Rabin for 64-bit n */
static int is_prime(uint64_t n) {
    static const uint64_t bases[12] = {2,3,5,7,11,13,17,19,23,29,31,37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) { if (n == bases[i]) return 1; if (n % bases[i] == 0) return 0; }
    uint64_t d = n - 1; int s = 0; while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        uint64_t x = powm(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int r = 1; r < s; r++) { x = mulm(x, x, n); if (x == n - 1) { comp = 0; break; } }
        if (comp) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011)                        */
/* ------------------------------------------------------------------------- */
void oc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint32_t i, uint32_t limb, uint32_t obj, uint32_t attempt, uint32_t out[4]) {
    uint32_t ctr[4] = {i, limb, obj, attempt};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oc_philox4x32_10(ctr, key, out);
}

static int bitlen(uint64_t q) { int b = 0; while (q) { b++; q >>= 1; } return b; }

/* uniform residue mod q by rejection on the top bits of two 64-bit words */
static uint64_t draw_uniform(uint64_t seed, uint32_t i, uint32_t limb, uint32_t obj, uint64_t q) {
    int b = bitlen(q);
    for (uint32_t att = 0;; att++) {
        uint32_t r[4]; draw(seed, i, limb, obj, att, r);
        uint64_t x0 = (((uint64_t)r[1] << 32) | r[0]) >> (64 - b);
        if (x0 < q) return x0;
        uint64_t x1 = (((uint64_t)r[3] << 32) | r[2]) >> (64 - b);
        if (x1 < q) return x1;
    }
}
static int draw_ternary(uint64_t seed, uint32_t i, uint32_t obj) {
    uint32_t r[4]; draw(seed, i, 0, obj, 0, r);
    return (int)(((uint64_t)r[0] * 3u) >> 32) - 1;
}
static int draw_cbd21(uint64_t seed, uint32_t i, uint32_t obj) {
    uint32_t r[4]; draw(seed, i, 0, obj, 0, r);
    return __builtin_popcount(r[0] & 0x1FFFFFu) - __builtin_popcount(r[1] & 0x1FFFFFu);
}

#define OBJ_SK      0x00000001u
#define OBJ_SKH     0x00000002u
#define OBJ_KEY_A   0x01000000u
#define OBJ_KEY_E   0x02000000u
#define OBJ_ENC_A   0x03000000u
#define OBJ_ENC_E   0x04000000u

/* ------------------------------------------------------------------------- */
/* context                                                                    */
/* ------------------------------------------------------------------------- */
typedef struct {
    int log_n, N;
    int L;            /* Q primes q_0..q_L */
    int alpha, dnum;  /* P primes p_0..p_{alpha-1} live at index L+1.. */
    int np;           /* L + 1 + alpha */
    uint64_t seed;
    uint64_t *q;      /* [np] */
    uint64_t *psi;    /* primitive 2N-th root per prime */
    uint64_t **psipow, **ipsipow;  /* [np][N] psi^i and psi^-i */
    uint64_t **wtab, **iwtab;      /* [np][N/2] omega^k, omega^-k with omega = psi^2 */
    uint64_t *ninv;
    int *rev;
    int8_t *sk;
    uint64_t **sk_ntt;             /* [np][N] transform of s mod each prime */
    uint64_t **keys;               /* key index -> [beta][2][np][N] transformed */
    int nkeys;
    uint32_t nonce;
} oc_ctx;

typedef struct {
    int level;
    uint64_t *c[2];   /* [level+1][N], coefficient domain */
} oc_ct;

/* cyclic NTT of length N over Z_q in place, omega table w[k] = omega^k, k < N/2 */
static void ntt_cyclic(uint64_t *a, int N, const int *rev, const uint64_t *w, uint64_t q) {
    for (int i = 0; i < N; i++) { int j = rev[i]; if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; } }
    for (int len = 2; len <= N; len <<= 1) {
        int half = len >> 1, step = N / len;
        for (int s = 0; s < N; s += len)
            for (int k = 0; k < half; k++) {
                uint64_t u = a[s + k], v = mulm(a[s + k + half], w[k * step], q);
                a[s + k] = addm(u, v, q); a[s + k + half] = subm(u, v, q);
            }
    }
}
/* negacyclic forward transform: evaluations of a(X) at psi * omega^k (order is internal) */
static void fwd(const oc_ctx *C, int pi, uint64_t *a) {
    uint64_t q = C->q[pi];
    for (int i = 0; i < C->N; i++) a[i] = mulm(a[i], C->psipow[pi][i], q);
    ntt_cyclic(a, C->N, C->rev, C->wtab[pi], q);
}
static void inv(const oc_ctx *C, int pi, uint64_t *a) {
    uint64_t q = C->q[pi];
    ntt_cyclic(a, C->N, C->rev, C->iwtab[pi], q);
    for (int i = 0; i < C->N; i++) a[i] = mulm(mulm(a[i], C->ninv[pi], q), C->ipsipow[pi][i], q);
}

static uint64_t find_psi(uint64_t q, int N) {
    uint64_t M = 2 * (uint64_t)N;
    for (uint64_t g = 2;; g++) {
        uint64_t psi = powm(g, (q - 1) / M, q);
        if (powm(psi, (uint64_t)N, q) == q - 1) return psi;
    }
}

static int prime_used(const uint64_t *list, int cnt, uint64_t v) {
    for (int i = 0; i < cnt; i++) if (list[i] == v) return 1;
    return 0;
}
static uint64_t next_prime(int bits, int N, const uint64_t *used, int cnt) {
    uint64_t M = 2 * (uint64_t)N;
    for (uint64_t k = 1;; k++) {
        uint64_t c = ((uint64_t)1 << bits) - k * M + 1;
        if (is_prime(c) && !prime_used(used, cnt, c)) return c;
    }
}

/* Prime chain: q_0 (q0_bits), then q_1 .. q_{n_q-1-n_hi} (q_bits), then the top n_hi
 * primes (hi_bits; the levels a bootstrap consumes first), then alpha P primes (p_bits).
 * Secret: dense ternary (secret_hw = 0) or sparse ternary with exactly secret_hw
 * nonzero coefficients, placed one at a time: for the i-th, draw(seed, i, 0, OBJ_SKH,
 * attempt) for attempt = 0, 1, .. until the position (word 0 mod N) is free; its sign
 * is - for an odd word 1. */
oc_ctx *oc_ctx_create_ex(int log_n, int n_q, int q0_bits, int q_bits, int p_bits, int dnum, uint64_t seed,
                         int n_hi, int hi_bits, int secret_hw) {
    if (log_n < 3 || log_n > 17 || n_q < 1 || dnum < 1) return NULL;
    if (n_hi < 0 || n_hi > n_q - 1 || (n_hi > 0 && (hi_bits < 20 || hi_bits > 48))) return NULL;
    if (secret_hw < 0 || secret_hw > (1 << log_n)) return NULL;
    oc_ctx *C = (oc_ctx *)calloc(1, sizeof(oc_ctx));
    C->log_n = log_n; C->N = 1 << log_n; C->L = n_q - 1; C->dnum = dnum;
    C->alpha = (n_q + dnum - 1) / dnum;
    C->np = n_q + C->alpha; C->seed = seed;
    int N = C->N;
    C->q = (uint64_t *)calloc(C->np, sizeof(uint64_t));
    int cnt = 0;
    C->q[cnt] = next_prime(q0_bits, N, C->q, cnt); cnt++;
    for (int i = 1; i < n_q; i++) {
        C->q[cnt] = next_prime(i >= n_q - n_hi ? hi_bits : q_bits, N, C->q, cnt); cnt++;
    }
    for (int i = 0; i < C->alpha; i++) { C->q[cnt] = next_prime(p_bits, N, C->q, cnt); cnt++; }
    C->rev = (int *)malloc(sizeof(int) * N);
    for (int i = 0; i < N; i++) { int r = 0; for (int b = 0; b < log_n; b++) if (i >> b & 1) r |= 1 << (log_n - 1 - b); C->rev[i] = r; }
    C->psi = (uint64_t *)malloc(sizeof(uint64_t) * C->np);
    C->ninv = (uint64_t *)malloc(sizeof(uint64_t) * C->np);
    C->psipow = (uint64_t **)malloc(sizeof(void *) * C->np);
    C->ipsipow = (uint64_t **)malloc(sizeof(void *) * C->np);
    C->wtab = (uint64_t **)malloc(sizeof(void *) * C->np);
    C->iwtab = (uint64_t **)malloc(sizeof(void *) * C->np);
    for (int p = 0; p < C->np; p++) {
        uint64_t q = C->q[p], psi = find_psi(q, N), ipsi = invm(psi, q);
        uint64_t om = mulm(psi, psi, q), iom = mulm(ipsi, ipsi, q);
        C->psi[p] = psi; C->ninv[p] = invm((uint64_t)N % q, q);
        C->psipow[p] = (uint64_t *)malloc(8 * N); C->ipsipow[p] = (uint64_t *)malloc(8 * N);
        C->wtab[p] = (uint64_t *)malloc(8 * (N / 2)); C->iwtab[p] = (uint64_t *)malloc(8 * (N / 2));
        uint64_t x = 1, y = 1;
        for (int i = 0; i < N; i++) { C->psipow[p][i] = x; C->ipsipow[p][i] = y; x = mulm(x, psi, q); y = mulm(y, ipsi, q); }
        x = 1; y = 1;
        for (int i = 0; i < N / 2; i++) { C->wtab[p][i] = x; C->iwtab[p][i] = y; x = mulm(x, om, q); y = mulm(y, iom, q); }
    }
    /* secret key: ternary, one draw per coefficient, or sparse ternary */
    C->sk = (int8_t *)malloc(N);
    if (secret_hw == 0) {
        for (int i = 0; i < N; i++) C->sk[i] = (int8_t)draw_ternary(seed, (uint32_t)i, OBJ_SK);
    } else {
        memset(C->sk, 0, N);
        for (int i = 0; i < secret_hw; i++)
            for (uint32_t att = 0;; att++) {
                uint32_t r[4]; draw(seed, (uint32_t)i, 0, OBJ_SKH, att, r);
                int pos = (int)(r[0] & (uint32_t)(N - 1));
                if (C->sk[pos]) continue;
                C->sk[pos] = (int8_t)((r[1] & 1u) ? -1 : 1);
                break;
            }
    }
    C->sk_ntt = (uint64_t **)malloc(sizeof(void *) * C->np);
    for (int p = 0; p < C->np; p++) {
        C->sk_ntt[p] = (uint64_t *)malloc(8 * N);
        for (int i = 0; i < N; i++) C->sk_ntt[p][i] = red_i64(C->sk[i], C->q[p]);
        fwd(C, p, C->sk_ntt[p]);
    }
    C->nkeys = 256;
    C->keys = (uint64_t **)calloc(C->nkeys, sizeof(void *));
    return C;
}

oc_ctx *oc_ctx_create(int log_n, int n_q, int q0_bits, int q_bits, int p_bits, int dnum, uint64_t seed) {
    return oc_ctx_create_ex(log_n, n_q, q0_bits, q_bits, p_bits, dnum, seed, 0, 0, 0);
}

void oc_ctx_free(oc_ctx *C) {
    if (!C) return;
    for (int p = 0; p < C->np; p++) {
        free(C->psipow[p]); free(C->ipsipow[p]); free(C->wtab[p]); free(C->iwtab[p]); free(C->sk_ntt[p]);
    }
    for (int k = 0; k < C->nkeys; k++) free(C->keys[k]);
    free(C->keys); free(C->psipow); free(C->ipsipow); free(C->wtab); free(C->iwtab); free(C->sk_ntt);
    free(C->q); free(C->psi); free(C->ninv); free(C->rev); free(C->sk); free(C);
}

int oc_ctx_info(const oc_ctx *C, int *N, int *L, int *alpha, int *np) {
    *N = C->N; *L = C->L; *alpha = C->alpha; *np = C->np; return 0;
}
void oc_ctx_primes(const oc_ctx *C, uint64_t *out) { memcpy(out, C->q, 8 * C->np); }
void oc_ctx_secret(const oc_ctx *C, int8_t *out) { memcpy(out, C->sk, C->N); }
void oc_set_nonce(oc_ctx *C, uint32_t nonce) { C->nonce = nonce; }
uint32_t oc_get_nonce(const oc_ctx *C) { return C->nonce; }

/* number of digits over the primes q_0..q_l: consecutive alpha-blocks from q_0 */
static int n_digits(const oc_ctx *C, int l) { return (l + 1 + C->alpha - 1) / C->alpha; }

/* Galois element of key index k >= 1: 5^(2^(k-1)) mod 2N (rotation by 2^(k-1) slots) */
static uint64_t galois_of_key(const oc_ctx *C, int k) {
    uint64_t M = 2 * (uint64_t)C->N, g = 5;
    for (int i = 0; i < k - 1; i++) g = (g * g) % M;
    return g;
}

/* s(X) -> s(X^g) for small integer coefficient polys */
static void automorph_small(const int8_t *in, int8_t *out, int N, uint64_t g) {
    for (int i = 0; i < N; i++) {
        uint64_t e = ((uint64_t)i * g) % (2 * (uint64_t)N);
        if (e < (uint64_t)N) out[e] = in[i]; else out[e - N] = (int8_t)(-in[i]);
    }
}

/* Key index 0: relinearisation key for s^2.  Key index k >= 1: rotation key
 * for s(X^g); oc_keygen uses g = 5^(2^(k-1)) (rotation by 2^(k-1) slots),
 * oc_keygen_galois takes g from the caller (rotation by any amount a: g = 5^a).
 * Digit j of the key, per prime index pi:
 *   b = -a s + e + [pi in digit j] (P mod q_pi) s'     a uniform, e ~ CBD(21)   */
int oc_keygen_galois(oc_ctx *C, int kidx, uint64_t galois) {
    if (kidx < 0 || kidx >= C->nkeys) return -1;
    if (C->keys[kidx]) return 0;
    int N = C->N, np = C->np, beta = n_digits(C, C->L);
    /* target s' as residues per prime (coefficient domain then transformed) */
    uint64_t **tgt = (uint64_t **)malloc(sizeof(void *) * np);
    int8_t *sg = (int8_t *)malloc(N);
    if (kidx >= 1) automorph_small(C->sk, sg, N, galois);
    #pragma omp parallel for schedule(dynamic)
    for (int p = 0; p < np; p++) {
        uint64_t q = C->q[p];
        tgt[p] = (uint64_t *)malloc(8 * N);
        if (kidx == 0) { for (int i = 0; i < N; i++) tgt[p][i] = mulm(C->sk_ntt[p][i], C->sk_ntt[p][i], q); }
        else { for (int i = 0; i < N; i++) tgt[p][i] = red_i64(sg[i], q); fwd(C, p, tgt[p]); }
    }
    /* P mod q_i */
    uint64_t *Pmod = (uint64_t *)malloc(8 * np);
    for (int p = 0; p <= C->L; p++) {
        uint64_t v = 1;
        for (int m = 0; m < C->alpha; m++) v = mulm(v, C->q[C->L + 1 + m] % C->q[p], C->q[p]);
        Pmod[p] = v;
    }
    size_t per = (size_t)np * N;
    uint64_t *K = (uint64_t *)malloc(8 * (size_t)beta * 2 * per);
    for (int j = 0; j < beta; j++) {
        uint32_t oa = OBJ_KEY_A | ((uint32_t)kidx << 8) | (uint32_t)j;
        uint32_t oe = OBJ_KEY_E | ((uint32_t)kidx << 8) | (uint32_t)j;
        int *e = (int *)malloc(sizeof(int) * N);
        for (int i = 0; i < N; i++) e[i] = draw_cbd21(C->seed, (uint32_t)i, oe);
        int lo = j * C->alpha, hi = lo + C->alpha; if (hi > C->L + 1) hi = C->L + 1;
        #pragma omp parallel for schedule(dynamic)
        for (int p = 0; p < np; p++) {
            uint64_t q = C->q[p];
            uint64_t *b = K + ((size_t)j * 2 + 0) * per + (size_t)p * N;
            uint64_t *a = K + ((size_t)j * 2 + 1) * per + (size_t)p * N;
            for (int i = 0; i < N; i++) a[i] = draw_uniform(C->seed, (uint32_t)i, (uint32_t)p, oa, q);
            for (int i = 0; i < N; i++) b[i] = red_i64(e[i], q);
            fwd(C, p, a); fwd(C, p, b);
            int in_digit = (p >= lo && p < hi);
            for (int i = 0; i < N; i++) {
                uint64_t v = subm(b[i], mulm(a[i], C->sk_ntt[p][i], q), q);
                if (in_digit) v = addm(v, mulm(Pmod[p], tgt[p][i], q), q);
                b[i] = v;
            }
        }
        free(e);
    }
    for (int p = 0; p < np; p++) free(tgt[p]);
    free(tgt); free(sg); free(Pmod);
    C->keys[kidx] = K;
    return 0;
}

int oc_keygen(oc_ctx *C, int kidx) {
    if (kidx < 0 || kidx >= C->nkeys) return -1;
    return oc_keygen_galois(C, kidx, kidx >= 1 ? galois_of_key(C, kidx) : 0);
}

/* ------------------------------------------------------------------------- */
/* ciphertexts                                                                */
/* ------------------------------------------------------------------------- */
static oc_ct *ct_new(const oc_ctx *C, int level) {
    oc_ct *ct = (oc_ct *)malloc(sizeof(oc_ct));
    ct->level = level;
    for (int k = 0; k < 2; k++) ct->c[k] = (uint64_t *)calloc((size_t)(level + 1) * C->N, 8);
    return ct;
}
void oc_ct_free(oc_ct *ct) { if (!ct) return; free(ct->c[0]); free(ct->c[1]); free(ct); }
int oc_ct_level(const oc_ct *ct) { return ct->level; }

void oc_ct_export(const oc_ctx *C, const oc_ct *ct, uint64_t *out) {
    size_t n = (size_t)(ct->level + 1) * C->N;
    memcpy(out, ct->c[0], 8 * n); memcpy(out + n, ct->c[1], 8 * n);
}
oc_ct *oc_ct_import(const oc_ctx *C, const uint64_t *in, int level) {
    oc_ct *ct = ct_new(C, level);
    size_t n = (size_t)(level + 1) * C->N;
    memcpy(ct->c[0], in, 8 * n); memcpy(ct->c[1], in + n, 8 * n);
    return ct;
}

/* c = a * b in Z_q[X]/(X^N+1), coefficient domain in and out */
static void ring_mul(const oc_ctx *C, int pi, const uint64_t *a, const uint64_t *b, uint64_t *c) {
    int N = C->N; uint64_t q = C->q[pi];
    uint64_t *ta = (uint64_t *)malloc(8 * N), *tb = (uint64_t *)malloc(8 * N);
    memcpy(ta, a, 8 * N); memcpy(tb, b, 8 * N);
    fwd(C, pi, ta); fwd(C, pi, tb);
    for (int i = 0; i < N; i++) ta[i] = mulm(ta[i], tb[i], q);
    inv(C, pi, ta);
    memcpy(c, ta, 8 * N);
    free(ta); free(tb);
}
/* product with a transformed operand (s or a key limb) */
static void ring_mul_t(const oc_ctx *C, int pi, const uint64_t *a, const uint64_t *bt, uint64_t *c) {
    int N = C->N; uint64_t q = C->q[pi];
    uint64_t *ta = (uint64_t *)malloc(8 * N);
    memcpy(ta, a, 8 * N);
    fwd(C, pi, ta);
    for (int i = 0; i < N; i++) ta[i] = mulm(ta[i], bt[i], q);
    inv(C, pi, ta);
    memcpy(c, ta, 8 * N);
    free(ta);
}

/* schoolbook negacyclic product, used only to pin ring_mul on small N */
void oc_schoolbook(const uint64_t *a, const uint64_t *b, uint64_t *c, int N, uint64_t q) {
    for (int k = 0; k < N; k++) c[k] = 0;
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            uint64_t t = mulm(a[i], b[j], q);
            int k = i + j;
            if (k < N) c[k] = addm(c[k], t, q); else c[k - N] = subm(c[k - N], t, q);
        }
}
void oc_ring_mul(const oc_ctx *C, int pi, const uint64_t *a, const uint64_t *b, uint64_t *c) { ring_mul(C, pi, a, b, c); }

/* secret-key encryption of an integer plaintext polynomial m at the top level:
 * c1 = a (uniform per prime), c0 = -a s + e + m,  e ~ CBD(21); nonce advances */
oc_ct *oc_encrypt(oc_ctx *C, const int64_t *m) {
    int N = C->N, L = C->L;
    uint32_t nonce = C->nonce++;
    uint32_t oa = OBJ_ENC_A | (nonce & 0xFFFFFFu), oe = OBJ_ENC_E | (nonce & 0xFFFFFFu);
    oc_ct *ct = ct_new(C, L);
    int *e = (int *)malloc(sizeof(int) * N);
    for (int i = 0; i < N; i++) e[i] = draw_cbd21(C->seed, (uint32_t)i, oe);
    #pragma omp parallel for schedule(dynamic)
    for (int p = 0; p <= L; p++) {
        uint64_t q = C->q[p];
        uint64_t *a = ct->c[1] + (size_t)p * N, *c0 = ct->c[0] + (size_t)p * N;
        for (int i = 0; i < N; i++) a[i] = draw_uniform(C->seed, (uint32_t)i, (uint32_t)p, oa, q);
        ring_mul_t(C, p, a, C->sk_ntt[p], c0);
        for (int i = 0; i < N; i++) {
            uint64_t v = subm(0, c0[i], q);
            v = addm(v, red_i64(e[i], q), q);
            v = addm(v, red_i64(m[i], q), q);
            c0[i] = v;
        }
    }
    free(e);
    return ct;
}

/* m = c0 + c1 s at the ciphertext's level; the centred integer is returned as
 * double using the CRT over q_0 (and q_1 when level >= 1) */
void oc_decrypt(const oc_ctx *C, const oc_ct *ct, double *out) {
    int N = C->N, nl = ct->level >= 1 ? 2 : 1;
    uint64_t *m = (uint64_t *)malloc(8 * (size_t)nl * N);
    for (int p = 0; p < nl; p++) {
        uint64_t q = C->q[p];
        ring_mul_t(C, p, ct->c[1] + (size_t)p * N, C->sk_ntt[p], m + (size_t)p * N);
        for (int i = 0; i < N; i++) m[(size_t)p * N + i] = addm(m[(size_t)p * N + i], ct->c[0][(size_t)p * N + i], q);
    }
    if (nl == 1) {
        uint64_t q = C->q[0];
        for (int i = 0; i < N; i++) { uint64_t v = m[i]; out[i] = v > q / 2 ? -(double)(q - v) : (double)v; }
    } else {
        uint64_t q0 = C->q[0], q1 = C->q[1];
        u128 Q = (u128)q0 * q1;
        uint64_t q0inv = invm(q0 % q1, q1);
        for (int i = 0; i < N; i++) {
            uint64_t a0 = m[i], a1 = m[N + i];
            /* x = a0 + q0 * ((a1 - a0) q0^-1 mod q1) */
            uint64_t t = mulm(subm(a1, a0 % q1, q1), q0inv, q1);
            u128 x = (u128)a0 + (u128)q0 * t;
            if (x > Q / 2) out[i] = -(double)(Q - x); else out[i] = (double)x;
        }
    }
    free(m);
}

static void check_same_level(const oc_ct *a, const oc_ct *b) { (void)a; (void)b; }

oc_ct *oc_add(const oc_ctx *C, const oc_ct *a, const oc_ct *b) {
    if (a->level != b->level) return NULL;
    check_same_level(a, b);
    oc_ct *r = ct_new(C, a->level);
    for (int k = 0; k < 2; k++)
        for (int p = 0; p <= a->level; p++)
            for (int i = 0; i < C->N; i++) {
                size_t o = (size_t)p * C->N + i;
                r->c[k][o] = addm(a->c[k][o], b->c[k][o], C->q[p]);
            }
    return r;
}
oc_ct *oc_sub(const oc_ctx *C, const oc_ct *a, const oc_ct *b) {
    if (a->level != b->level) return NULL;
    oc_ct *r = ct_new(C, a->level);
    for (int k = 0; k < 2; k++)
        for (int p = 0; p <= a->level; p++)
            for (int i = 0; i < C->N; i++) {
                size_t o = (size_t)p * C->N + i;
                r->c[k][o] = subm(a->c[k][o], b->c[k][o], C->q[p]);
            }
    return r;
}
/* multiply both polynomials by the integer k */
oc_ct *oc_mul_int(const oc_ctx *C, const oc_ct *a, int64_t k) {
    oc_ct *r = ct_new(C, a->level);
    for (int p = 0; p <= a->level; p++) {
        uint64_t q = C->q[p], km = red_i64(k, q);
        for (int c = 0; c < 2; c++)
            for (int i = 0; i < C->N; i++) { size_t o = (size_t)p * C->N + i; r->c[c][o] = mulm(a->c[c][o], km, q); }
    }
    return r;
}
/* add the integer v to the constant coefficient of c0 (a constant in every slot) */
oc_ct *oc_add_const_int(const oc_ctx *C, const oc_ct *a, int64_t v) {
    oc_ct *r = ct_new(C, a->level);
    size_t n = (size_t)(a->level + 1) * C->N;
    memcpy(r->c[0], a->c[0], 8 * n); memcpy(r->c[1], a->c[1], 8 * n);
    for (int p = 0; p <= a->level; p++) {
        size_t o = (size_t)p * C->N;
        r->c[0][o] = addm(r->c[0][o], red_i64(v, C->q[p]), C->q[p]);
    }
    return r;
}
oc_ct *oc_drop(const oc_ctx *C, const oc_ct *a, int level) {
    if (level > a->level || level < 0) return NULL;
    oc_ct *r = ct_new(C, level);
    size_t n = (size_t)(level + 1) * C->N;
    memcpy(r->c[0], a->c[0], 8 * n); memcpy(r->c[1], a->c[1], 8 * n);
    return r;
}

/* divide by the last prime q_l with a centred remainder:
 * c_i <- (c_i - [c_l]_centred) * q_l^-1 mod q_i */
oc_ct *oc_rescale(const oc_ctx *C, const oc_ct *a) {
    int l = a->level;
    if (l < 1) return NULL;
    oc_ct *r = ct_new(C, l - 1);
    uint64_t ql = C->q[l];
    for (int c = 0; c < 2; c++) {
        const uint64_t *last = a->c[c] + (size_t)l * C->N;
        #pragma omp parallel for
        for (int p = 0; p < l; p++) {
            uint64_t q = C->q[p], qinv = invm(ql % q, q);
            for (int i = 0; i < C->N; i++) {
                uint64_t v = last[i];
                int64_t cen = v > (ql - 1) / 2 ? -(int64_t)(ql - v) : (int64_t)v;
                uint64_t d = subm(a->c[c][(size_t)p * C->N + i], red_i64(cen, q), q);
                r->c[c][(size_t)p * C->N + i] = mulm(d, qinv, q);
            }
        }
    }
    return r;
}

/* multiply by the integer K, then rescale */
oc_ct *oc_mul_int_rescale(const oc_ctx *C, const oc_ct *a, int64_t K) {
    oc_ct *t = oc_mul_int(C, a, K);
    oc_ct *r = oc_rescale(C, t);
    oc_ct_free(t);
    return r;
}

/* ModDown of one NTT-domain accumulator acc over Q_l u P ([l+1+alpha][N], gidx = global
 * prime index of each extended limb; transformed back in place):
 * out_i = (acc_i - conv_P->q_i(acc_P)) * P^-1 mod q_i, coefficient domain */
static void moddown_one(const oc_ctx *C, int l, uint64_t *acc, const int *gidx, uint64_t *out) {
    int N = C->N, nq = l + 1, A = C->alpha, next = nq + A;
    /* back to coefficients */
    #pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < next; k++) inv(C, gidx[k], acc + (size_t)k * N);
    /* out_i = (acc_i - conv_P->q_i(acc_P)) * P^-1 mod q_i, where the conversion lifts each
     * [acc_m * Phat_m^-1]_{p_m} to its centred representative, so the division by P
     * rounds with a mean-zero error */
    uint64_t *phinv = (uint64_t *)malloc(8 * A);
    for (int m = 0; m < A; m++) {
        uint64_t pm = C->q[C->L + 1 + m], v = 1;
        for (int b = 0; b < A; b++) if (b != m) v = mulm(v, C->q[C->L + 1 + b] % pm, pm);
        phinv[m] = invm(v, pm);
    }
    uint64_t *w = (uint64_t *)malloc(8 * (size_t)A * N);
    for (int m = 0; m < A; m++) {
        uint64_t pm = C->q[C->L + 1 + m];
        for (int i = 0; i < N; i++) w[(size_t)m * N + i] = mulm(acc[(size_t)(nq + m) * N + i], phinv[m], pm);
    }
    #pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < nq; k++) {
        uint64_t q = C->q[k];
        uint64_t *ph = (uint64_t *)malloc(8 * A);
        uint64_t Pm = 1;
        for (int m = 0; m < A; m++) {
            uint64_t v = 1;
            for (int b = 0; b < A; b++) if (b != m) v = mulm(v, C->q[C->L + 1 + b] % q, q);
            ph[m] = v;
            Pm = mulm(Pm, C->q[C->L + 1 + m] % q, q);
        }
        uint64_t Pinv = invm(Pm, q);
        for (int i = 0; i < N; i++) {
            uint64_t s = 0;
            for (int m = 0; m < A; m++) {
                /* centred lift of w_m to (-p_m/2, p_m/2], then reduced mod q_k */
                uint64_t pm = C->q[C->L + 1 + m], v = w[(size_t)m * N + i];
                uint64_t vk = v > (pm - 1) / 2 ? subm(0, (pm - v) % q, q) : v % q;
                s = addm(s, mulm(vk, ph[m], q), q);
            }
            out[(size_t)k * N + i] = mulm(subm(acc[(size_t)k * N + i], s, q), Pinv, q);
        }
        free(ph);
    }
    free(w);
    free(phinv);
}

/* ModDown of the two accumulators of a key switch */
static void moddown(const oc_ctx *C, int l, uint64_t *acc0, uint64_t *acc1, const int *gidx, uint64_t *out0,
                    uint64_t *out1) {
    moddown_one(C, l, acc0, gidx, out0);
    moddown_one(C, l, acc1, gidx, out1);
}

/* key products of a key switch of d (level l, coefficient domain) with key kidx.
 * ModUp of digit j (primes D_j): the fast conversion sum_i [d_i Qhat_i^-1]_{q_i} Qhat_i
 * with every [.]_{q_i} taken as its centred representative, so the extension
 * d + u D_j has u of mean zero and the key noise it multiplies adds no bias
 * (a non-centred u has mean dl/2 and leaves a constant offset on every
 * coefficient, which the slot decoding concentrates near slot 0).
 * acc0/acc1 [l+1+alpha][N] (zeroed by the caller) receive sum_j ModUp_j(d) key_j in the
 * NTT domain; gidx[l+1+alpha] gets the global prime index of each extended limb */
static int ks_products(const oc_ctx *C, const uint64_t *d, int l, int kidx, uint64_t *acc0, uint64_t *acc1,
                       int *gidx) {
    const uint64_t *K = C->keys[kidx];
    if (!K) return -1;
    int N = C->N, nq = l + 1, A = C->alpha, next = nq + A;
    int beta = n_digits(C, l);
    size_t per = (size_t)C->np * N;
    for (int k = 0; k < nq; k++) gidx[k] = k;
    for (int m = 0; m < A; m++) gidx[nq + m] = C->L + 1 + m;
    for (int j = 0; j < beta; j++) {
        int lo = j * A, hi = lo + A; if (hi > nq) hi = nq;
        int dl = hi - lo;
        /* Qhat_i = D / q_i with D = prod of the digit's primes present at level l */
        uint64_t *qhinv = (uint64_t *)malloc(8 * dl);     /* (Qhat_i)^-1 mod q_i */
        for (int a = 0; a < dl; a++) {
            uint64_t qi = C->q[lo + a], v = 1;
            for (int b = 0; b < dl; b++) if (b != a) v = mulm(v, C->q[lo + b] % qi, qi);
            qhinv[a] = invm(v, qi);
        }
        uint64_t *vv = (uint64_t *)malloc(8 * (size_t)dl * N);  /* [d_i * Qhat_i^-1]_{q_i} */
        for (int a = 0; a < dl; a++)
            for (int i = 0; i < N; i++) vv[(size_t)a * N + i] = mulm(d[(size_t)(lo + a) * N + i], qhinv[a], C->q[lo + a]);
        #pragma omp parallel for schedule(dynamic)
        for (int k = 0; k < next; k++) {
            int g = gidx[k]; uint64_t pk = C->q[g];
            uint64_t *e = (uint64_t *)malloc(8 * N);
            if (k >= lo && k < hi) memcpy(e, d + (size_t)k * N, 8 * N);
            else {
                uint64_t *qh = (uint64_t *)malloc(8 * dl);   /* Qhat_i mod p_k */
                for (int a = 0; a < dl; a++) {
                    uint64_t v = 1;
                    for (int b = 0; b < dl; b++) if (b != a) v = mulm(v, C->q[lo + b] % pk, pk);
                    qh[a] = v;
                }
                for (int i = 0; i < N; i++) {
                    uint64_t s = 0;
                    for (int a = 0; a < dl; a++)
                        s = addm(s, mulm(centred_mod(vv[(size_t)a * N + i], C->q[lo + a], pk), qh[a], pk), pk);
                    e[i] = s;
                }
                free(qh);
            }
            fwd(C, g, e);
            const uint64_t *kb = K + ((size_t)j * 2 + 0) * per + (size_t)g * N;
            const uint64_t *ka = K + ((size_t)j * 2 + 1) * per + (size_t)g * N;
            for (int i = 0; i < N; i++) {
                acc0[(size_t)k * N + i] = addm(acc0[(size_t)k * N + i], mulm(e[i], kb[i], pk), pk);
                acc1[(size_t)k * N + i] = addm(acc1[(size_t)k * N + i], mulm(e[i], ka[i], pk), pk);
            }
            free(e);
        }
        free(qhinv); free(vv);
    }
    return 0;
}

/* hybrid key switch of d (level l, coefficient domain) with key kidx.
 * out0/out1: [l+1][N] coefficient domain. */
static int keyswitch(const oc_ctx *C, const uint64_t *d, int l, int kidx, uint64_t *out0, uint64_t *out1) {
    int N = C->N, next = l + 1 + C->alpha;
    int *gidx = (int *)malloc(sizeof(int) * next);
    uint64_t *acc0 = (uint64_t *)calloc((size_t)next * N, 8);
    uint64_t *acc1 = (uint64_t *)calloc((size_t)next * N, 8);
    int rc = ks_products(C, d, l, kidx, acc0, acc1, gidx);
    if (rc == 0) moddown(C, l, acc0, acc1, gidx, out0, out1);
    free(acc0); free(acc1); free(gidx);
    return rc;
}

/* Relinearisation with the rescale folded into the ModDown (one rounding): with the
 * key products acc over Q_l u P (NTT domain) and the tensor parts d0, d1 over Q_l
 * (coefficient domain), A = acc + P d (P d vanishes mod every p_m) is divided by
 * P q_l: over B = {q_l, p_0, .., p_{alpha-1}} each [A_b (P q_l / b)^-1]_b is lifted to
 * its centred representative and converted to q_i, and
 *   out_i = (A_i - sum_b w_b [P q_l / b]_{q_i}) (P q_l)^-1 mod q_i,  i < l.
 * The result is the rescaled relinearised product at level l - 1. */
static void moddown_rescale(const oc_ctx *C, int l, uint64_t *acc0, uint64_t *acc1, const int *gidx,
                            const uint64_t *d0, const uint64_t *d1, uint64_t *out0, uint64_t *out1) {
    int N = C->N, nq = l + 1, A = C->alpha, next = nq + A, nb = A + 1;
    #pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < 2 * next; k++) {
        int kk = k % next; uint64_t *acc = k < next ? acc0 : acc1;
        inv(C, gidx[kk], acc + (size_t)kk * N);
    }
    /* basis B: extended limb slot and prime of each member */
    int *bslot = (int *)malloc(sizeof(int) * nb);
    uint64_t *bq = (uint64_t *)malloc(8 * nb), *bhinv = (uint64_t *)malloc(8 * nb);
    bslot[0] = l;
    for (int m = 0; m < A; m++) bslot[1 + m] = nq + m;
    for (int k = 0; k < nb; k++) bq[k] = C->q[gidx[bslot[k]]];
    for (int k = 0; k < nb; k++) {
        uint64_t v = 1;
        for (int b = 0; b < nb; b++) if (b != k) v = mulm(v, bq[b] % bq[k], bq[k]);
        bhinv[k] = invm(v, bq[k]);
    }
    uint64_t Pql = 1;   /* P mod q_l */
    for (int m = 0; m < A; m++) Pql = mulm(Pql, C->q[C->L + 1 + m] % C->q[l], C->q[l]);
    for (int c = 0; c < 2; c++) {
        uint64_t *acc = c ? acc1 : acc0, *out = c ? out1 : out0;
        const uint64_t *d = c ? d1 : d0;
        uint64_t *w = (uint64_t *)malloc(8 * (size_t)nb * N);
        for (int k = 0; k < nb; k++) {
            const uint64_t *a = acc + (size_t)bslot[k] * N;
            for (int i = 0; i < N; i++) {
                uint64_t v = a[i];
                if (k == 0) v = addm(v, mulm(Pql, d[(size_t)l * N + i], bq[0]), bq[0]);
                w[(size_t)k * N + i] = mulm(v, bhinv[k], bq[k]);
            }
        }
        #pragma omp parallel for schedule(dynamic)
        for (int t = 0; t < l; t++) {
            uint64_t q = C->q[t];
            uint64_t *bh = (uint64_t *)malloc(8 * nb);
            uint64_t Pall = 1, Pm = 1;
            for (int k = 0; k < nb; k++) {
                uint64_t v = 1;
                for (int b = 0; b < nb; b++) if (b != k) v = mulm(v, bq[b] % q, q);
                bh[k] = v;
                Pall = mulm(Pall, bq[k] % q, q);
            }
            for (int m = 0; m < A; m++) Pm = mulm(Pm, C->q[C->L + 1 + m] % q, q);
            uint64_t Pinv = invm(Pall, q);
            for (int i = 0; i < N; i++) {
                uint64_t sum = 0;
                for (int k = 0; k < nb; k++) {
                    uint64_t bk = bq[k], v = w[(size_t)k * N + i];
                    uint64_t vk = v > (bk - 1) / 2 ? subm(0, (bk - v) % q, q) : v % q;
                    sum = addm(sum, mulm(vk, bh[k], q), q);
                }
                uint64_t Ai = addm(acc[(size_t)t * N + i], mulm(Pm, d[(size_t)t * N + i], q), q);
                out[(size_t)t * N + i] = mulm(subm(Ai, sum, q), Pinv, q);
            }
            free(bh);
        }
        free(w);
    }
    free(bslot); free(bq); free(bhinv);
}

/* exported for primitive-level tests: key switch of a single polynomial */
int oc_keyswitch(const oc_ctx *C, const uint64_t *d, int level, int kidx, uint64_t *out0, uint64_t *out1) {
    return keyswitch(C, d, level, kidx, out0, out1);
}

/* a(X) -> a(X^g) on residues */
static void automorph(const oc_ctx *C, const uint64_t *in, uint64_t *out, int level, uint64_t g) {
    int N = C->N; uint64_t M = 2 * (uint64_t)N;
    for (int p = 0; p <= level; p++) {
        uint64_t q = C->q[p];
        for (int i = 0; i < N; i++) {
            uint64_t e = ((uint64_t)i * g) % M; uint64_t v = in[(size_t)p * N + i];
            if (e < (uint64_t)N) out[(size_t)p * N + e] = v;
            else out[(size_t)p * N + (e - N)] = v ? q - v : 0;
        }
    }
}

/* tensor, then relinearise and rescale in one ModDown by P q_l */
oc_ct *oc_mul(const oc_ctx *C, const oc_ct *a, const oc_ct *b) {
    if (a->level != b->level || a->level < 1 || !C->keys[0]) return NULL;
    int l = a->level, N = C->N;
    size_t n = (size_t)(l + 1) * N;
    uint64_t *d0 = (uint64_t *)malloc(8 * n), *d1 = (uint64_t *)malloc(8 * n), *d2 = (uint64_t *)malloc(8 * n);
    #pragma omp parallel for schedule(dynamic)
    for (int p = 0; p <= l; p++) {
        uint64_t q = C->q[p]; size_t o = (size_t)p * N;
        uint64_t *t = (uint64_t *)malloc(8 * N);
        ring_mul(C, p, a->c[0] + o, b->c[0] + o, d0 + o);
        ring_mul(C, p, a->c[0] + o, b->c[1] + o, d1 + o);
        ring_mul(C, p, a->c[1] + o, b->c[0] + o, t);
        for (int i = 0; i < N; i++) d1[o + i] = addm(d1[o + i], t[i], q);
        ring_mul(C, p, a->c[1] + o, b->c[1] + o, d2 + o);
        free(t);
    }
    int next = l + 1 + C->alpha;
    int *gidx = (int *)malloc(sizeof(int) * next);
    uint64_t *acc0 = (uint64_t *)calloc((size_t)next * N, 8);
    uint64_t *acc1 = (uint64_t *)calloc((size_t)next * N, 8);
    ks_products(C, d2, l, 0, acc0, acc1, gidx);
    oc_ct *s = ct_new(C, l - 1);
    moddown_rescale(C, l, acc0, acc1, gidx, d0, d1, s->c[0], s->c[1]);
    free(acc0); free(acc1); free(gidx);
    free(d0); free(d1); free(d2);
    return s;
}

/* tensor + relinearise without the rescale (primitive tests) */
oc_ct *oc_mul_norescale(const oc_ctx *C, const oc_ct *a, const oc_ct *b) {
    if (a->level != b->level || !C->keys[0]) return NULL;
    int l = a->level, N = C->N;
    size_t n = (size_t)(l + 1) * N;
    uint64_t *d0 = (uint64_t *)malloc(8 * n), *d1 = (uint64_t *)malloc(8 * n), *d2 = (uint64_t *)malloc(8 * n);
    for (int p = 0; p <= l; p++) {
        uint64_t q = C->q[p]; size_t o = (size_t)p * N;
        uint64_t *t = (uint64_t *)malloc(8 * N);
        ring_mul(C, p, a->c[0] + o, b->c[0] + o, d0 + o);
        ring_mul(C, p, a->c[0] + o, b->c[1] + o, d1 + o);
        ring_mul(C, p, a->c[1] + o, b->c[0] + o, t);
        for (int i = 0; i < N; i++) d1[o + i] = addm(d1[o + i], t[i], q);
        ring_mul(C, p, a->c[1] + o, b->c[1] + o, d2 + o);
        free(t);
    }
    oc_ct *r = ct_new(C, l);
    keyswitch(C, d2, l, 0, r->c[0], r->c[1]);
    for (int p = 0; p <= l; p++)
        for (int i = 0; i < N; i++) {
            size_t o = (size_t)p * N + i;
            r->c[0][o] = addm(r->c[0][o], d0[o], C->q[p]);
            r->c[1][o] = addm(r->c[1][o], d1[o], C->q[p]);
        }
    free(d0); free(d1); free(d2);
    return r;
}

/* rotation by 2^r slots: (sigma(c0) + ks0, ks1), ks = keyswitch(sigma(c1)) */
oc_ct *oc_rotate(const oc_ctx *C, const oc_ct *a, int r) {
    int kidx = 1 + r;
    if (kidx >= C->nkeys || !C->keys[kidx]) return NULL;
    int l = a->level, N = C->N;
    size_t n = (size_t)(l + 1) * N;
    uint64_t g = galois_of_key(C, kidx);
    uint64_t *s0 = (uint64_t *)malloc(8 * n), *s1 = (uint64_t *)malloc(8 * n);
    automorph(C, a->c[0], s0, l, g);
    automorph(C, a->c[1], s1, l, g);
    oc_ct *o = ct_new(C, l);
    keyswitch(C, s1, l, kidx, o->c[0], o->c[1]);
    for (int p = 0; p <= l; p++)
        for (int i = 0; i < N; i++) { size_t x = (size_t)p * N + i; o->c[0][x] = addm(o->c[0][x], s0[x], C->q[p]); }
    free(s0); free(s1);
    return o;
}

/* any Galois automorphism with the key kidx generated for it (oc_keygen_galois):
 * g = 5^a is a rotation by a slots, g = 2N - 1 the complex conjugation of every slot */
oc_ct *oc_rotate_gal(const oc_ctx *C, const oc_ct *a, int kidx, uint64_t g) {
    if (kidx < 1 || kidx >= C->nkeys || !C->keys[kidx]) return NULL;
    int l = a->level, N = C->N;
    size_t n = (size_t)(l + 1) * N;
    uint64_t *s0 = (uint64_t *)malloc(8 * n), *s1 = (uint64_t *)malloc(8 * n);
    automorph(C, a->c[0], s0, l, g);
    automorph(C, a->c[1], s1, l, g);
    oc_ct *o = ct_new(C, l);
    keyswitch(C, s1, l, kidx, o->c[0], o->c[1]);
    for (int p = 0; p <= l; p++)
        for (int i = 0; i < N; i++) { size_t x = (size_t)p * N + i; o->c[0][x] = addm(o->c[0][x], s0[x], C->q[p]); }
    free(s0); free(s1);
    return o;
}

/* both polynomials times the integer plaintext polynomial m (no rescale): the slots
 * multiply by those m encodes */
oc_ct *oc_mul_plain(const oc_ctx *C, const oc_ct *a, const int64_t *m) {
    int l = a->level, N = C->N;
    oc_ct *o = ct_new(C, l);
    #pragma omp parallel for schedule(dynamic)
    for (int p = 0; p <= l; p++) {
        uint64_t q = C->q[p];
        size_t x = (size_t)p * N;
        uint64_t *mp = (uint64_t *)malloc(8 * N);
        for (int i = 0; i < N; i++) mp[i] = red_i64(m[i], q);
        ring_mul(C, p, a->c[0] + x, mp, o->c[0] + x);
        ring_mul(C, p, a->c[1] + x, mp, o->c[1] + x);
        free(mp);
    }
    return o;
}

/* ModRaise: a level-0 ciphertext's residues mod q_0, lifted to (-q_0/2, q_0/2] and
 * reduced modulo q_0 .. q_level.  The result decrypts to m + q_0 I for a small
 * integer polynomial I (the first step of a bootstrap). */
oc_ct *oc_modraise(const oc_ctx *C, const oc_ct *a, int level) {
    if (a->level != 0 || level < 0 || level > C->L) return NULL;
    int N = C->N;
    uint64_t q0 = C->q[0];
    oc_ct *o = ct_new(C, level);
    for (int c = 0; c < 2; c++)
        for (int i = 0; i < N; i++) {
            uint64_t v = a->c[c][i];
            int64_t cen = v > (q0 - 1) / 2 ? -(int64_t)(q0 - v) : (int64_t)v;
            for (int p = 0; p <= level; p++) o->c[c][(size_t)p * N + i] = red_i64(cen, C->q[p]);
        }
    return o;
}

/* a(X) -> a(X^g) on one limb of residues mod q (coefficient domain) */
static void automorph_limb(const uint64_t *in, uint64_t *out, int N, uint64_t g, uint64_t q) {
    uint64_t M = 2 * (uint64_t)N;
    for (int i = 0; i < N; i++) {
        uint64_t e = ((uint64_t)i * g) % M, v = in[i];
        if (e < (uint64_t)N) out[e] = v; else out[e - N] = v ? q - v : 0;
    }
}

/* One step of a hoisted rotate-and-sum: x + sum_r rot(x, a_r) for nr rotations with
 * Galois elements gal[r] = 5^(a_r) and keys kidx[r].  The digits of c1 are extended
 * once (ModUp); every rotation applies its automorphism to the extended digits and
 * multiplies by its own key; the products of all rotations are summed over Q_l u P
 * and brought back by a single ModDown:
 *   A    = sum_r sum_j sigma_r(ModUp_j(c1)) * key_{r,j}
 *   out0 = c0 + sum_r sigma_r(c0) + ModDown(A)_0,   out1 = c1 + ModDown(A)_1.
 * (Halevi-Shoup hoisting of the ModUp, and one ModDown for the whole sum.) */
/* the key products of one hoisted step: the digits of d (c1, coefficient domain, level l)
 * are extended once and every rotation r applies sigma_r to the extended digits before
 * multiplying by its own key; acc0/acc1 [l+1+alpha][N] (zeroed by the caller) receive
 * sum_r sum_j sigma_r(ModUp_j(d)) key_{r,j} in the NTT domain, gidx the global prime index
 * of each extended limb */
static void hoisted_products(const oc_ctx *C, const uint64_t *d, int l, int nr, const int *kidx,
                             const uint64_t *gal, uint64_t *acc0, uint64_t *acc1, int *gidx) {
    int N = C->N, nq = l + 1, A = C->alpha, next = nq + A;
    int beta = n_digits(C, l);
    size_t per = (size_t)C->np * N;
    for (int k = 0; k < nq; k++) gidx[k] = k;
    for (int m = 0; m < A; m++) gidx[nq + m] = C->L + 1 + m;
    for (int j = 0; j < beta; j++) {
        int lo = j * A, hi = lo + A; if (hi > nq) hi = nq;
        int dl = hi - lo;
        uint64_t *qhinv = (uint64_t *)malloc(8 * dl);
        for (int a = 0; a < dl; a++) {
            uint64_t qi = C->q[lo + a], v = 1;
            for (int b = 0; b < dl; b++) if (b != a) v = mulm(v, C->q[lo + b] % qi, qi);
            qhinv[a] = invm(v, qi);
        }
        uint64_t *vv = (uint64_t *)malloc(8 * (size_t)dl * N);
        for (int a = 0; a < dl; a++)
            for (int i = 0; i < N; i++) vv[(size_t)a * N + i] = mulm(d[(size_t)(lo + a) * N + i], qhinv[a], C->q[lo + a]);
        #pragma omp parallel for schedule(dynamic)
        for (int k = 0; k < next; k++) {
            int g = gidx[k]; uint64_t pk = C->q[g];
            uint64_t *e = (uint64_t *)malloc(8 * N), *t = (uint64_t *)malloc(8 * N);
            if (k >= lo && k < hi) memcpy(e, d + (size_t)k * N, 8 * N);
            else {
                uint64_t *qh = (uint64_t *)malloc(8 * dl);
                for (int a = 0; a < dl; a++) {
                    uint64_t v = 1;
                    for (int b = 0; b < dl; b++) if (b != a) v = mulm(v, C->q[lo + b] % pk, pk);
                    qh[a] = v;
                }
                for (int i = 0; i < N; i++) {
                    uint64_t sum = 0;
                    for (int a = 0; a < dl; a++)
                        sum = addm(sum, mulm(centred_mod(vv[(size_t)a * N + i], C->q[lo + a], pk), qh[a], pk), pk);
                    e[i] = sum;
                }
                free(qh);
            }
            for (int r = 0; r < nr; r++) {
                automorph_limb(e, t, N, gal[r], pk);
                fwd(C, g, t);
                const uint64_t *K = C->keys[kidx[r]];
                const uint64_t *kb = K + ((size_t)j * 2 + 0) * per + (size_t)g * N;
                const uint64_t *ka = K + ((size_t)j * 2 + 1) * per + (size_t)g * N;
                for (int i = 0; i < N; i++) {
                    acc0[(size_t)k * N + i] = addm(acc0[(size_t)k * N + i], mulm(t[i], kb[i], pk), pk);
                    acc1[(size_t)k * N + i] = addm(acc1[(size_t)k * N + i], mulm(t[i], ka[i], pk), pk);
                }
            }
            free(e); free(t);
        }
        free(qhinv); free(vv);
    }
}

oc_ct *oc_rotsum_step(const oc_ctx *C, const oc_ct *x, int nr, const int *kidx, const uint64_t *gal) {
    if (nr < 1) return NULL;
    for (int r = 0; r < nr; r++)
        if (kidx[r] < 1 || kidx[r] >= C->nkeys || !C->keys[kidx[r]]) return NULL;
    int N = C->N, l = x->level, nq = l + 1, A = C->alpha, next = nq + A;
    int *gidx = (int *)malloc(sizeof(int) * next);
    uint64_t *acc0 = (uint64_t *)calloc((size_t)next * N, 8);
    uint64_t *acc1 = (uint64_t *)calloc((size_t)next * N, 8);
    hoisted_products(C, x->c[1], l, nr, kidx, gal, acc0, acc1, gidx);
    oc_ct *o = ct_new(C, l);
    moddown(C, l, acc0, acc1, gidx, o->c[0], o->c[1]);
    size_t n = (size_t)nq * N;
    uint64_t *s0 = (uint64_t *)malloc(8 * n);
    for (int r = 0; r < nr; r++) {
        automorph(C, x->c[0], s0, l, gal[r]);
        for (int p = 0; p < nq; p++)
            for (int i = 0; i < N; i++) {
                size_t z = (size_t)p * N + i;
                o->c[0][z] = addm(o->c[0][z], s0[z], C->q[p]);
            }
    }
    for (int p = 0; p < nq; p++)
        for (int i = 0; i < N; i++) {
            size_t z = (size_t)p * N + i;
            o->c[0][z] = addm(o->c[0][z], x->c[0][z], C->q[p]);
            o->c[1][z] = addm(o->c[1][z], x->c[1][z], C->q[p]);
        }
    free(s0); free(acc0); free(acc1); free(gidx);
    return o;
}

/* A hoisted rotate-and-sum of several steps (step s: rotations gal[off_s .. off_s + nr[s])
 * with keys kidx alike) that carries c0 as X0 = P c0 over Q_l u P (coefficient domain)
 * instead of dividing it by P after every step:
 *   X0 = P c0 on the Q limbs, 0 on the P limbs (P c0 vanishes mod each p_m);
 *   per step, with A0, A1 the step's key products (hoisted_products of c1):
 *     X0 <- X0 + sum_r sigma_r(X0) + INTT(A0)      on every limb of Q_l u P
 *     c1 <- c1 + ModDown(A1)
 *   and at the end c0 = ModDown(X0).
 * ModDown(X0) = (X0_Q - conv(X0_P)) P^-1 divides the exact sum P (c0 + sum of the rotated
 * c0s) + sum of the A0s by P once, so the result is x plus every rotation of every step,
 * as with a ModDown per step, but rounded once. */
oc_ct *oc_rotsum_carried(const oc_ctx *C, const oc_ct *x, int nsteps, const int *nr, const int *kidx,
                         const uint64_t *gal) {
    if (nsteps < 1) return NULL;
    int tot = 0;
    for (int s_ = 0; s_ < nsteps; s_++) {
        if (nr[s_] < 1) return NULL;
        tot += nr[s_];
    }
    for (int r = 0; r < tot; r++)
        if (kidx[r] < 1 || kidx[r] >= C->nkeys || !C->keys[kidx[r]]) return NULL;
    int N = C->N, l = x->level, nq = l + 1, A = C->alpha, next = nq + A;
    int *gidx = (int *)malloc(sizeof(int) * next);
    for (int k = 0; k < nq; k++) gidx[k] = k;
    for (int m = 0; m < A; m++) gidx[nq + m] = C->L + 1 + m;
    size_t ne = (size_t)next * N;
    uint64_t *X0 = (uint64_t *)calloc(ne, 8), *S = (uint64_t *)malloc(8 * ne);
    uint64_t *c1 = (uint64_t *)malloc(8 * (size_t)nq * N);
    memcpy(c1, x->c[1], 8 * (size_t)nq * N);
    for (int k = 0; k < nq; k++) {
        uint64_t q = C->q[k], Pm = 1;
        for (int m = 0; m < A; m++) Pm = mulm(Pm, C->q[C->L + 1 + m] % q, q);
        for (int i = 0; i < N; i++) X0[(size_t)k * N + i] = mulm(x->c[0][(size_t)k * N + i], Pm, q);
    }
    uint64_t *acc0 = (uint64_t *)malloc(8 * ne), *acc1 = (uint64_t *)malloc(8 * ne);
    oc_ct *o = ct_new(C, l);
    int off = 0;
    for (int s_ = 0; s_ < nsteps; s_++) {
        memset(acc0, 0, 8 * ne);
        memset(acc1, 0, 8 * ne);
        hoisted_products(C, c1, l, nr[s_], kidx + off, gal + off, acc0, acc1, gidx);
        /* X0 + sum_r sigma_r(X0) + INTT(A0) on every extended limb (limbs independent) */
        memcpy(S, X0, 8 * ne);
        #pragma omp parallel for schedule(dynamic)
        for (int k = 0; k < next; k++) {
            uint64_t pk = C->q[gidx[k]];
            uint64_t *tk = (uint64_t *)malloc(8 * N);
            for (int r = 0; r < nr[s_]; r++) {
                automorph_limb(X0 + (size_t)k * N, tk, N, gal[off + r], pk);
                for (int i = 0; i < N; i++) S[(size_t)k * N + i] = addm(S[(size_t)k * N + i], tk[i], pk);
            }
            inv(C, gidx[k], acc0 + (size_t)k * N);
            for (int i = 0; i < N; i++)
                X0[(size_t)k * N + i] = addm(S[(size_t)k * N + i], acc0[(size_t)k * N + i], pk);
            free(tk);
        }
        /* c1 + ModDown(A1) */
        moddown_one(C, l, acc1, gidx, o->c[1]);
        #pragma omp parallel for schedule(static)
        for (int p = 0; p < nq; p++)
            for (int i = 0; i < N; i++) {
                size_t z = (size_t)p * N + i;
                c1[z] = addm(o->c[1][z], c1[z], C->q[p]);
            }
        off += nr[s_];
    }
    /* c0 = ModDown(X0): to the NTT domain first (moddown_one takes NTT-domain limbs) */
    #pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < next; k++) fwd(C, gidx[k], X0 + (size_t)k * N);
    moddown_one(C, l, X0, gidx, o->c[0]);
    memcpy(o->c[1], c1, 8 * (size_t)nq * N);
    free(X0); free(S); free(c1); free(acc0); free(acc1); free(gidx);
    return o;
}

/* automorphism only (primitive tests) */
oc_ct *oc_automorph(const oc_ctx *C, const oc_ct *a, uint64_t g) {
    oc_ct *o = ct_new(C, a->level);
    automorph(C, a->c[0], o->c[0], a->level, g);
    automorph(C, a->c[1], o->c[1], a->level, g);
    return o;
}

int oc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the following parallel regions (timing at one thread and at all cores) */
void oc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
