/* A plain C client of the encrypted-CutMax library: it sees only include/he.h and host
 * pointers.  Encrypts 1024 toy logits on a 2^12 ring, runs CutMax (Alg. 2) on the
 * device, decrypts, and prints the recovered arg-max next to the plaintext one as
 * "argmax <decrypted> <plaintext> max <value>"; exit status 0 only when they agree.
 * With the argument "boot": bootstraps 2048 values in [-1, 1] from level 3 on a
 * bootstrappable 2^12 chain and prints "boot maxerr <error> level <level>"; exit status 0
 * when the values come back within 1e-3. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "he.h"

static int fail(const char *what, int rc) {
    fprintf(stderr, "%s failed (%d): %s\n", what, rc, he_last_error());
    return 1;
}

static int boot_demo(void) {
    enum { S = 2048 };
    he_params prm = {12, 20, 48, 40, 48, 3, 40.0, 5, 0, NULL, 3, 13, 48, 64};
    he_ctx *ctx = NULL;
    int rc = he_ctx_create(&prm, &ctx);
    if (rc) return fail("he_ctx_create", rc);
    const he_boot_cfg bc = {3, 3, 0, 12, 31, 3, 48.0};
    rc = he_boot_setup(ctx, &bc);
    if (rc) return fail("he_boot_setup", rc);
    double v[S], out[S];
    unsigned s = 777u;
    for (int i = 0; i < S; ++i) {
        s = s * 1103515245u + 12345u;
        v[i] = (double)(s >> 8) / 8388608.0 - 1.0;
    }
    he_ct *ct = NULL, *lo = NULL, *b = NULL;
    if ((rc = he_encrypt(ctx, v, S, 0.0, &ct))) return fail("he_encrypt", rc);
    if ((rc = he_drop(ctx, ct, 3, &lo))) return fail("he_drop", rc);
    if ((rc = he_bootstrap(ctx, lo, 1.0, &b))) return fail("he_bootstrap", rc);
    if ((rc = he_decrypt(ctx, b, out, S))) return fail("he_decrypt", rc);
    uint32_t a, level;
    double scale;
    size_t n;
    he_ct_info(b, &a, &level, &scale, &n);
    double err = 0.0;
    for (int i = 0; i < S; ++i) err = fmax(err, fabs(out[i] - v[i]));
    printf("boot maxerr %.3e level %u\n", err, level);
    he_ct_free(b);
    he_ct_free(lo);
    he_ct_free(ct);
    he_ctx_destroy(ctx);
    return err < 1e-3 ? 0 : 2;
}

int main(int argc, char **argv) {
    if (argc > 1 && argv[1][0] == 'b') return boot_demo();
    enum { N_LOGITS = 1024, T = 4 };
    he_params prm = {12, 36, 40, 30, 40, 3, 30.0, 7, 0, NULL, 3};
    he_ctx *ctx = NULL;
    int rc = he_ctx_create(&prm, &ctx);
    if (rc) return fail("he_ctx_create", rc);

    /* toy logits: a fixed pseudo-random pattern with one clear maximum */
    double x[N_LOGITS];
    unsigned s = 12345u;
    int want = 0;
    for (int i = 0; i < N_LOGITS; ++i) {
        s = s * 1103515245u + 12345u;
        x[i] = ((double)(s >> 8) / 16777216.0 - 0.5) * 3.0;
        if (x[i] > x[want]) want = i;
    }
    x[want] += 1.0;

    he_ct *ct = NULL, *z = NULL;
    rc = he_encrypt(ctx, x, N_LOGITS, 0.0, &ct);
    if (rc) return fail("he_encrypt", rc);

    const uint32_t p[T] = {3, 3, 3, 3};
    const double c[T] = {5.0, 5.0, 5.0, 5.0};
    const double vlo[T] = {0.5, 0.25, 0.3, 0.6}, vhi[T] = {2.0, 0.75, 3.0, 128.0};
    he_cutmax_cfg cfg = {T, p, c, vlo, vhi, 3, NULL, 0, 1.0, 3.0, 3, 0};
    rc = he_cutmax(ctx, &ct, 1, &cfg, &z);
    if (rc) return fail("he_cutmax", rc);

    double out[N_LOGITS];
    rc = he_decrypt(ctx, z, out, N_LOGITS);
    if (rc) return fail("he_decrypt", rc);
    int got = 0;
    for (int i = 1; i < N_LOGITS; ++i)
        if (out[i] > out[got]) got = i;
    printf("argmax %d %d max %.6f\n", got, want, out[got]);

    he_ct_free(z);
    he_ct_free(ct);
    he_ctx_destroy(ctx);
    return got == want ? 0 : 2;
}
