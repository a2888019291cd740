/*
 * he.h -- C ABI of the MI355X encrypted-CutMax library (libcutmax_he.so).
 *
 * The operation is CutMax, the HE-friendly argmax of arXiv 2509.08383
 * (Sec. 3.1, Alg. 1; encrypted form Sec. 3.2, Alg. 2), and the samplers built
 * on it (Sec. 3.3: Gumbel-max and the one-shot nucleus sampler, Alg. 3),
 * evaluated over RNS-CKKS ciphertexts.  The client encrypts its logit vector X, the server returns
 * an encrypted one-hot approximation Z of argmax(X), and only the client
 * decrypts (Sec. 1 and App. A threat model).
 *
 * Conventions shared by every call:
 *   - Every call returns HE_OK (0) or a negative he_status; he_last_error()
 *     gives a thread-local message for the last failure on this thread.
 *   - Handles are opaque; the caller owns every handle it receives and frees
 *     it (he_ct_free, he_ctx_destroy).  A context must outlive its
 *     ciphertexts.  One context = one HIP stream; calls on one context are not
 *     thread-safe.
 *   - Pointer arguments named x, out, limbs, m, g are HOST memory owned by the
 *     caller.  Ciphertexts live in device memory inside their handles.
 *   - Parameters outside the documented ranges return HE_EINVAL; device
 *     failures HE_EDEVICE; allocation failures HE_ENOMEM; a schedule that
 *     needs more levels than the ciphertext has HE_EDEPTH; a constant that
 *     cannot be encoded HE_ERANGE; mismatched handles HE_ESTATE.
 */
#ifndef CUTMAX_HE_H
#define CUTMAX_HE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HE_OK = 0,
    HE_EINVAL = -1,
    HE_ENOMEM = -2,
    HE_EDEVICE = -3,
    HE_EDEPTH = -4,
    HE_ERANGE = -5,
    HE_ESTATE = -6,
    HE_EIO = -7
} he_status;

typedef struct he_ctx he_ctx;
typedef struct he_ct he_ct;

/* CKKS parameters.  log_n in {12, 16}; n_q >= 2 Q primes (levels = n_q - 1);
 * bit sizes in [20, 48] (the kernels compute modulo these primes in the FP64
 * pipe, exact below 2^52, and store evaluation key words in 5 bytes for
 * primes below 2^40 and 6 bytes for the others); dnum >= 1 key-switching digits; log2_scale is the
 * encoding scale Delta = 2^log2_scale; seed keys every random draw
 * (Philox4x32-10).  device: HIP device ordinal.  stream: a hipStream_t the
 * library enqueues on (for example PyTorch's current stream), or NULL for a
 * stream the library creates.  hoist: how rotate-and-sum (Sec. 3.2, App. D)
 * runs: 0 = one rotation by 2^r at a time, each rotation a full key switch
 * followed by an add; h in 1..4 = steps of radix 2^h, x <- x + sum_{r=1}^{2^h-1}
 * rot(x, r k) for k = 1, 2^h, 2^2h, ... (the last step takes the bits left), each
 * step extending the digits of c1 once (ModUp), applying every rotation's
 * automorphism to the extended digits, summing the key products of all its
 * rotations and running one ModDown.  h >= 2 adds rotation keys for the amounts
 * r k that are not powers of two.
 * n_hi, hi_bits: the top n_hi Q primes (q_{L-n_hi+1} .. q_L, the levels a
 * bootstrap consumes first) have hi_bits bits instead of q_bits (n_hi = 0: one
 * size); n_hi < n_q.  secret_hw: 0 = dense ternary secret (one uniform draw in
 * {-1, 0, 1} per coefficient); h > 0 = sparse ternary secret with exactly h
 * nonzero coefficients (a bootstrap's ModRaise error I is bounded by the
 * secret's weight). */
typedef struct {
    uint32_t log_n;
    uint32_t n_q;
    uint32_t q0_bits;
    uint32_t q_bits;
    uint32_t p_bits;
    uint32_t dnum;
    double log2_scale;
    uint64_t seed;
    int device;
    void *stream;
    uint32_t hoist;
    uint32_t n_hi;
    uint32_t hi_bits;
    uint32_t secret_hw;
} he_params;

/* Hyper-parameters of one CutMax call (Alg. 1 inputs p, c, T; Sec. 4.2 uses
 * per-iteration p and c).  All arrays are host memory of length T.
 *   var_lo/var_hi: declared domain of the variance at each iteration; the
 *     inverse square root is evaluated on u = var/var_hi (Sec. 3.2, (ii)).
 *   init_degree/init_coef: power-basis coefficients g_0..g_d (d = init_degree
 *     in 1..4) of the initial guess g(u) ~ u^(-1/2), T rows of d+1 values.
 *     NULL: the library interpolates u^(-1/2) at Chebyshev nodes on
 *     [var_lo/var_hi, 1].
 *   newton_steps: refinements of the initial guess: Newton's
 *     h <- 1.5h - 0.5 u h^3 (2 levels each), or, with HE_REFINE_GOLDSCHMIDT,
 *     Goldschmidt's coupled inverse-square-root iteration (App. B.1 cites it
 *     for invsqr): r = 1.5 - b/2, h <- h r, b <- b r^2 from b = u h^2
 *     (2 levels each plus 1 for the first b).
 *   sum_lo/sum_hi: declared bounds of mean(Y^(T)); the final inverse runs
 *     Goldschmidt's product (App. B.1) with gold_d squarings on
 *     sum/(sum_hi * n).
 *   Bounds of any size are accepted: where var_hi of the next iteration exceeds
 *   2^8 (sum_hi, after the last, 2^4) the iteration's output is prescaled by a
 *   power of two 2^(-e) (the factor 2^(-e/p) on the normalised iterate, no
 *   level), which CutMax's result does not see and which keeps 1/(n sqrt(n v))
 *   and 1/(sum_hi n) within what one constant multiply resolves.
 *   flags: HE_NOISE_PRESCALED (he_topp_sample, he_gumbel_sample: the noise
 *     already carries the temperature); HE_REFINE_GOLDSCHMIDT (see
 *     newton_steps); HE_MASK_PAD: for a zero-padded request (n not dividing
 *     slots), mean, variance and the final sum run over its n logical slots
 *     only (Alg. 1 on the n logits; Sec. 3.2 assumes n = a * slots), so the
 *     first n outputs are CutMax of the logits alone.  The pad slots hold one
 *     common value that a tracker ciphertext follows through the same steps;
 *     the sums subtract (pad count) x tracker, which costs no level.  The pad
 *     slots of the output hold the tracker's iterate, not zeros.  Accuracy
 *     needs pad slots that do not outgrow the logits: encrypt with the mean of
 *     x as pad (he_encrypt with pad = NaN).
 *     HE_BOOT: runs schedules deeper than the chain (the paper's Table 2
 *     schedule T = 4, p = [16, 4, 4, 6], c = [5, 3, 3, 3] needs bootstrapping):
 *     after the normalisation of an iteration, the iterate z is bootstrapped
 *     (he_bootstrap, set up by he_boot_setup) whenever the power step and the
 *     next iteration's moments, or the final normalisation, do not fit in its
 *     levels; the bound passed is |z - 1| <= m sqrt(n - 1) / c (population
 *     moments) times 1.02, m = the maximum of g(u) sqrt(u) over the declared
 *     domain after the refinements (1 for an exact inverse square root).  On a
 *     chain with wider top primes (n_hi > 0) every call runs on the levels
 *     below them. */
typedef struct {
    uint32_t T;
    const uint32_t *p;
    const double *c;
    const double *var_lo;
    const double *var_hi;
    uint32_t init_degree;
    const double *init_coef;
    uint32_t newton_steps;
    double sum_lo;
    double sum_hi;
    uint32_t gold_d;
    uint32_t flags;
    /* HE_REFINE_SCALED only (else ignored, may be NULL): the wide-domain inverse square
     * root the paper's Table 2 schedule needs (Sec. 4, HE CutMax: T = 4, p = [16, 4, 4, 6],
     * c = [5, 3, 3, 3], whose later variances span up to five decades).  Per iteration t,
     * ref_steps[t] = K_t refinements of the guess (0: the guess alone, newton_steps is then
     * ignored); ref_coef holds, iteration after iteration, K_t pairs (a_k, b_k) of
     * x <- x (a_k - b_k x^2), x = g(u) sqrt(u) (b_k > 0); ref_range holds K_t + 1 pairs
     * (l_k, h_k), 0 < l_k <= h_k, bounds of x before step k and after the last, which set the
     * bootstrap bounds.  he_invsqrt_scaled_plan computes all three for a domain.  The
     * refinement runs on E h (the centred, scaled iterate) and on W = b_k x_k^2, never on
     * u^(-1/2) itself: with HE_BOOT, W and E h are bootstrapped in the middle of the
     * refinement when the chain runs short (bounds 1.02 b_k h_k^2 and
     * 1.02 sqrt(n - 1) h_k / c). */
    const uint32_t *ref_steps;
    const double *ref_coef;
    const double *ref_range;
} he_cutmax_cfg;

#define HE_NOISE_PRESCALED 1u
#define HE_REFINE_GOLDSCHMIDT 2u
#define HE_MASK_PAD 4u
#define HE_BOOT 8u
#define HE_REFINE_SCALED 16u

/* Context: prime chain, twiddle and basis-conversion tables, secret key, and
 * the relinearisation and rotation keys (rotation by 2^r slots for every r <
 * log2(slots), and the amounts of the hoisted rotate-and-sum steps), generated
 * on the device.  Roles follow the paper's setting (Sec. 2.1, the CKKS scheme
 * and its properties; App. A, threat model): the secret key stays with the
 * client, which encrypts and decrypts; the server evaluates with the public
 * evaluation keys only (relinearisation for products, Galois keys for the
 * rotations of rotate-and-sum, Sec. 3.2).  One context holds both roles so the
 * library can serve as client and server in one process; a deployment gives
 * the server a context built from the same seed and parameters and never
 * calls he_encrypt/he_decrypt there.
 * prm: host memory, read during the call.  out: receives a new handle owned by
 * the caller (he_ctx_destroy).  Errors: HE_EINVAL for parameters outside the
 * ranges above (no prime of the requested size, too many primes), HE_EDEVICE
 * without a usable GPU, HE_ENOMEM when the keys do not fit in device memory. */
int he_ctx_create(const he_params *prm, he_ctx **out);
void he_ctx_destroy(he_ctx *ctx);

/* Context facts: ring degree, slot count, top level, alpha (P primes) and the
 * prime chain q_0..q_L, p_0..p_{alpha-1} (primes may be NULL; else capacity
 * n_q + alpha entries). */
int he_ctx_info(const he_ctx *ctx, uint32_t *N, uint32_t *slots, uint32_t *L, uint32_t *alpha,
                uint64_t *primes);

/* Client: encrypt n doubles (Sec. 2.1).  n <= slots with slots % n == 0 is
 * replicated; otherwise padded with `pad` to a = ceil(n/slots) ciphertexts
 * (pad = NaN: the mean of x, which keeps masked CutMax accurate, see
 * HE_MASK_PAD).  The handle is at the top level with scale Delta and records n
 * and the pad value.  EINVAL for non-finite values or |x| >= 2^61 / Delta (the
 * encoded coefficients would not fit 64 bits). */
int he_encrypt(he_ctx *ctx, const double *x, size_t n, double pad, he_ct **out);

/* Client: encrypt already-encoded integer plaintexts m[a][N] at `scale`
 * (bit-exact tests feed one encoded plaintext to every implementation).
 * n is the logical length recorded in the handle. */
int he_encrypt_coeffs(he_ctx *ctx, const int64_t *m, uint32_t a, double scale, size_t n,
                      he_ct **out);

/* Records the value of the pad slots (beyond the logical length) of a handle
 * made by he_encrypt_coeffs or he_ct_import (default 0); masked CutMax starts
 * its pad tracker from it.  EINVAL for a non-finite value. */
int he_ct_set_pad(he_ct *ct, double pad);

/* Client: decrypt and decode the first n logical values (Sec. 2.1); n at most
 * a * slots (EINVAL otherwise). */
int he_decrypt(he_ctx *ctx, const he_ct *ct, double *out, size_t n);

/* Server: CutMax over `batch` requests (Alg. 2).  in[r] may hold 1 or more
 * ciphertexts; all requests advance level by level together.  out[r] receives
 * a new handle with the same packing as in[r]. */
int he_cutmax(he_ctx *ctx, he_ct *const *in, size_t batch, const he_cutmax_cfg *cfg, he_ct **out);

/* Server: one-shot nucleus sampling (Alg. 3): CutMax(X + temperature * G),
 * G the client's encrypted Beta(alpha,1) noise (see he_topp_noise). */
int he_topp_sample(he_ctx *ctx, he_ct *const *logits, he_ct *const *noise, size_t batch,
                   double top_p, double temperature, const he_cutmax_cfg *cfg, he_ct **out);

/* Client helper (Alg. 3 lines 1-4): g[i] = u[i]^(1/alpha),
 * alpha = ln(1 - top_p)/ln(top_p), from the caller's uniform draws u. */
int he_topp_noise(double top_p, const double *u, size_t n, double *g);

/* Host helper: the fixed initial guess of the inverse square root (Alg. 2 line 5;
 * Sec. 3.2 (ii) evaluates it on a known domain): the power-basis coefficients
 * coef[0..degree] (host memory, degree + 1 doubles) of the polynomial of degree
 * 1..4 interpolating u^(-1/2) at the Chebyshev nodes of [u_lo, 1], 0 < u_lo < 1,
 * the guess he_cutmax uses when init_coef is NULL.  No GPU needed. */
int he_invsqrt_guess_fit(double u_lo, uint32_t degree, double *coef);

/* Host helper: the wide-domain inverse square root on [u_lo, 1] (HE_REFINE_SCALED): the
 * degree-d Chebyshev guess g (coef, d + 1 doubles, as he_invsqrt_guess_fit), the range
 * [l_0, h_0] of x = g(u) sqrt(u) over the domain (a geometric grid of 20001 points,
 * widened by 1e-3 relative), then K refinements x <- x (a_k - b_k x^2), each chosen for
 * the range it receives so that it maps [l, h] onto [1 - e, 1 + e] with both ends and
 * its maximum at the equioscillation points: a = b (h^2 + h l + l^2),
 * b = 2 / (l h (h + l) + 2 ((h^2 + h l + l^2) / 3)^(3/2)), e = 1 - b l h (h + l).
 * steps: 2K doubles (a_k, b_k); ranges: 2(K + 1) doubles (l_k, h_k).  All host memory.
 * HE_EINVAL for u_lo outside (0, 1), degree outside 1..4, K > 16, or a guess that is not
 * positive on the domain.  No GPU needed. */
int he_invsqrt_scaled_plan(double u_lo, uint32_t degree, uint32_t K, double *coef, double *steps,
                           double *ranges);

/* Server: Gumbel-max sampling (Sec. 3.3, "Using Gumbel Distribution" and the
 * Gumbel-max lemma): CutMax(X + temperature * G), G the client's encrypted
 * Gumbel(0,1) noise (see he_gumbel_noise); the one-hot approximates a draw
 * from softmax(X / temperature).  Same packing, flags (HE_NOISE_PRESCALED) and
 * errors as he_topp_sample; the declared variance domains of cfg must cover
 * X + temperature * G. */
int he_gumbel_sample(he_ctx *ctx, he_ct *const *logits, he_ct *const *noise, size_t batch, double temperature,
                     const he_cutmax_cfg *cfg, he_ct **out);

/* Client helper (Sec. 3.3, Gumbel definition): g[i] = -ln(-ln u[i]) from the
 * caller's uniform draws u[i] in (0, 1). */
int he_gumbel_noise(const double *u, size_t n, double *g);

void he_ct_free(he_ct *ct);
const char *he_last_error(void);

/* Ciphertext facts: ciphertext count a, level, scale, logical length. */
int he_ct_info(const he_ct *ct, uint32_t *a, uint32_t *level, double *scale, size_t *n);

/* Coefficient-domain canonical limbs [a][2][level+1][N] (u64) of a handle;
 * cap is the capacity of `limbs` in words. */
int he_ct_export(he_ctx *ctx, const he_ct *ct, uint64_t *limbs, size_t cap);

/* Import coefficient-domain limbs [a][2][level+1][N]. */
int he_ct_import(he_ctx *ctx, const uint64_t *limbs, uint32_t a, uint32_t level, double scale,
                 size_t n, he_ct **out);

/* Evaluator primitives (single ciphertexts, a == 1, except he_rotsum and he_drop,
 * which act on every ciphertext of a handle independently), each the CKKS
 * operation the encrypted schedule is made of:
 *   he_add, he_sub        element-wise (Sec. 2.1)
 *   he_mul_int            multiply by an integer
 *   he_add_const          add a real constant to every slot
 *   he_mul                tensor, relinearise, rescale
 *   he_rescale            divide by the last prime
 *   he_cmul               multiply by a real constant then rescale; exact != 0
 *                         declares the exact scale, else scale s_want
 *   he_rotate             rotate slots left by 2^r (Sec. 3.2)
 *   he_rotsum             rotate-and-sum over every slot (Sec. 3.2, App. D)
 *   he_drop               drop limbs down to `level`
 * Every handle must belong to ctx; for he_add, he_sub and he_mul the second
 * operand b must also be a single ciphertext of ctx at a's level (HE_EINVAL
 * otherwise, before any kernel runs). */
int he_add(he_ctx *ctx, const he_ct *a, const he_ct *b, he_ct **out);
int he_sub(he_ctx *ctx, const he_ct *a, const he_ct *b, he_ct **out);
int he_mul_int(he_ctx *ctx, const he_ct *a, int64_t k, he_ct **out);
int he_add_const(he_ctx *ctx, const he_ct *a, double c, he_ct **out);
int he_mul(he_ctx *ctx, const he_ct *a, const he_ct *b, he_ct **out);
int he_rescale(he_ctx *ctx, const he_ct *a, he_ct **out);
int he_cmul(he_ctx *ctx, const he_ct *a, double kappa, double s_want, int exact, he_ct **out);
int he_rotate(he_ctx *ctx, const he_ct *a, uint32_t r, he_ct **out);
int he_rotsum(he_ctx *ctx, const he_ct *a, he_ct **out);
int he_drop(he_ctx *ctx, const he_ct *a, uint32_t level, he_ct **out);

/* he_rotsum for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): the same
 * rotate-and-sum, written into the caller's existing handle `out` (from ctx,
 * with as many ciphertexts as a; out may be a itself), whose level, scale and
 * slot count become the result's.  Word for word equal to he_rotsum.  The call
 * allocates nothing: its whole workspace is a static device array of 256 MiB
 * that the library holds on every device it runs on until the process ends
 * (its address is taken once per device by he_ctx_create).  One ciphertext at
 * N = 2^16 needs at most about 215 MiB at any level; a call that needs more returns
 * HE_ENOMEM before any kernel runs.  Every call on one device shares that
 * device's array: calls that overlap on one device (two threads, or two
 * contexts on different streams) race, so serialise them.  The call returns
 * after its kernels have finished.  Errors: HE_EINVAL for null or foreign
 * handles or a count mismatch, HE_ENOMEM as above. */
int he_rotsum_noalloc(he_ctx *ctx, const he_ct *a, he_ct *out);

/* CKKS bootstrapping: a ciphertext whose levels are spent comes back at a high
 * level with the same slot values (the paper runs its deeper CutMax schedules,
 * T = 4 with p up to 16 (Sec. 4, Table 2), with bootstrapping, and App. B.1
 * counts depth because it decides how often a bootstrap runs).  Steps:
 *   ModRaise   level-0 residues, centred, reduced modulo the whole chain: the
 *              plaintext becomes m + q_0 I with |I| <= K;
 *   CoeffToSlot the inverse slot-decoding map as n_cts groups of butterfly
 *              stages, each a baby-step giant-step sum of rotated diagonals
 *              (one level each); one conjugation splits the complex slots into
 *              the two real halves of the coefficient vector;
 *   EvalMod    sin(2 pi x) / (2 pi) removes q_0 I: a degree-cheb_deg Chebyshev
 *              interpolant of cos(2 pi (x - 1/4) / 2^r) in z = 2 y^2 - 1,
 *              then r double-angle steps;
 *   SlotToCoeff the decoding map as n_stc groups.
 * Levels used above the output: n_cts + 1 + ceil(log2(cheb_deg + 1)) + 1 + r + n_stc.
 * K = 0 takes ceil(6 sqrt(h / 12)) for a secret of weight h (the ModRaise
 * overflow of a sparse secret stays below this bound with overwhelming
 * probability); ratio_bits: the message enters EvalMod at q_0 2^-ratio_bits per
 * unit of `bound`, which sets the sine's linearisation error; log2_s_eval: scale of
 * the EvalMod ciphertexts (use the bit size of the primes it runs on).
 * correct_bits = c > 0: every bootstrap runs twice, the second pass on the first's
 * residual x - BTS(x) under the bound bound 2^-c, and adds it back (the error
 * shrinks by about 2^c at twice the time; c must leave the first pass's error below
 * bound 2^-c, and the input must sit below the output level). */
typedef struct {
    uint32_t n_cts;
    uint32_t n_stc;
    uint32_t K;
    uint32_t ratio_bits;
    uint32_t cheb_deg;
    uint32_t r;
    double log2_s_eval;
    uint32_t correct_bits;
} he_boot_cfg;

/* Bootstrap set-up: generates the Galois keys the two linear transforms use
 * (rotation amounts that already have a key keep it; the others take the next
 * free key indices in ascending order of amount, then the conjugation key) and
 * fixes the configuration.  Encoded diagonals are built on first use and kept in
 * device memory.  EINVAL for a configuration whose levels exceed the chain, or
 * whose CoeffToSlot and EvalMod levels (the top n_cts + 2 + ceil(log2(cheb_deg +
 * 1)) + r primes) are not within one bit of log2_s_eval (see he_params.n_hi). */
int he_boot_setup(he_ctx *ctx, const he_boot_cfg *cfg);

/* Bootstrap every ciphertext of `in` (level >= 1, real slot values with
 * |v| <= bound): out receives them at level L - (levels used) with scale Delta.
 * The error grows in proportion to the bound, which is rounded up to a power of
 * 2^(1/8) (each rounded bound keeps one set of encoded SlotToCoeff diagonals in
 * device memory).  ESTATE without he_boot_setup. */
int he_bootstrap(he_ctx *ctx, const he_ct *in, double bound, he_ct **out);

/* Bootstrap primitives (single ciphertexts), each bit-exact against a plain
 * implementation of its definition:
 *   he_keygen_galois  key index kidx for the automorphism X -> X^galois (galois
 *                     odd; 5^a mod 2N rotates by a slots, 2N - 1 conjugates);
 *                     kidx must be the next free index or an existing
 *                     Galois key's (replaced)
 *   he_rotate_gal     automorphism X -> X^galois with key kidx
 *   he_mul_plain      both polynomials times the integer plaintext m[N] (host),
 *                     declared scale = scale * pscale (no rescale)
 *   he_modraise       a level-0 ciphertext lifted to `level`, declared at `scale` */
int he_keygen_galois(he_ctx *ctx, uint32_t kidx, uint64_t galois);
int he_rotate_gal(he_ctx *ctx, const he_ct *a, uint32_t kidx, uint64_t galois, he_ct **out);
int he_mul_plain(he_ctx *ctx, const he_ct *a, const int64_t *m, double pscale, he_ct **out);
int he_modraise(he_ctx *ctx, const he_ct *a, uint32_t level, double scale, he_ct **out);

/* Measurement hooks.
 * he_bench_ntt: `iters` forward+inverse negacyclic NTTs over `vectors`
 *   resident limb vectors (each N words, cycling over the primes); *ms_fwd and
 *   *ms_inv receive the average device time of one forward / one inverse
 *   transform of the whole batch (HIP events on the context stream).
 * he_last_cutmax_ms: device time of the last he_cutmax/he_topp_sample call.
 * he_sync: wait for the context stream. */
int he_bench_ntt(he_ctx *ctx, uint32_t vectors, uint32_t iters, double *ms_fwd, double *ms_inv);
/* he_bench_copy: the library's element-wise copy kernel over `vectors` limb
 *   vectors (N words read and N written each), average device time per launch;
 *   the achievable-bandwidth reference and the calibration of byte counters. */
int he_bench_copy(he_ctx *ctx, uint32_t vectors, uint32_t iters, double *ms);
int he_last_cutmax_ms(const he_ctx *ctx, double *ms);
int he_sync(he_ctx *ctx);

/* Per-kernel timing: between he_profile_begin and he_profile_end every kernel
 * launch is bracketed by HIP events on the stream it is launched on (this adds
 * a little launch overhead).  he_profile_end waits for the stream and writes a
 * JSON object {"kernel": [launches, total_ms], ...} into buf (host, cap bytes).
 * One profile at a time per process. */
int he_profile_begin(he_ctx *ctx);
int he_profile_end(he_ctx *ctx, char *buf, size_t cap);

/* Options: HE_OPT_GRAPH (capture he_cutmax in a HIP graph and replay it for
 * repeated calls of the same shape), HE_OPT_NTT_VARIANT (0 = autotune, k > 0
 * forces variant k), HE_OPT_BOOT_HOIST (2, the default: the baby steps of a
 * bootstrap linear transform share one ModUp and the rotated giant-step sums share
 * one ModDown per 7 rotations; 1: only the baby steps are hoisted, equal word for
 * word to 0: one full key switch per rotation), HE_OPT_WORKSPACE_LIMIT (bytes of
 * device workspace, the per-call buffers and constants, that one call of this
 * context may use; 0, the default, is no limit: a call that needs more returns
 * HE_ENOMEM after its host-side planning, before any allocation or kernel, and
 * leaves the context and its handles usable; setting a limit below what the
 * context holds frees the held workspace, which the next call allocates anew;
 * keys, tables and ciphertext handles are not counted).  Device allocations that
 * fail for lack of memory anywhere in the library return HE_ENOMEM. */
#define HE_OPT_GRAPH 1
#define HE_OPT_NTT_VARIANT 2
#define HE_OPT_BOOT_HOIST 3
#define HE_OPT_WORKSPACE_LIMIT 4
int he_set_option(he_ctx *ctx, int option, int64_t value);

/* NTT autotuner result: the schedule variant chosen for batch buckets of <=4,
 * <=16, <=64, <=256, <=1024, <=4096, ... vectors (n entries, at most 8).  Variant v =
 * 1..6 is a workgroup width ((v - 1) % 3: 4, 8 or 16 sub-transforms per workgroup
 * at N = 2^16, 8, 16 or 32 at 2^12) and a pass-2 twiddle form ((v - 1) / 3: 0 the
 * full table, 1 phase-B twiddles formed as products of a row word and a small-table
 * word); every variant gives the same output word for word. */
int he_ntt_tuning(const he_ctx *ctx, int32_t *variants, uint32_t n);

/* Every candidate the autotuner timed, as JSON in buf (cap bytes, NUL-terminated):
 * {"logN", "variants": [names], "buckets": [{"vectors", "ms": [one forward +
 * inverse pair per variant, best of 3 trials], "choice"}]}.  HE_EINVAL when cap is
 * too small. */
int he_ntt_tuning_report(const he_ctx *ctx, char *buf, size_t cap);

/* ---------------------------------------------------------------------------
 * Learned initial guess for the inverse square root of Alg. 2 line 5 (an
 * addition to the paper's method).  A 1 -> 16 -> 16 -> 1 network with square
 * activations, z = (u - mean)/sd, h1 = W1 z + b1, a1 = h1^2, h2 = W2 a1 + b2,
 * a2 = h2^2, y = W3 . a2 + b3, trained in FP32 on the GPU to minimise the mean
 * of (y sqrt(u) - 1)^2; y is a degree-4 polynomial of u, which he_mlp_to_poly
 * returns for he_cutmax_cfg.init_coef (init_degree = 4).
 * Parameter vector (321 floats): W1[16], b1[16], W2[16][16] (row = output),
 * b2[16], W3[16], b3.  All array arguments are host memory.  Errors of these
 * calls are reported by he_mlp_last_error(). */
typedef struct he_mlp he_mlp;
int he_mlp_create(uint64_t seed, int device, he_mlp **out);
void he_mlp_destroy(he_mlp *mlp);
int he_mlp_set_params(he_mlp *mlp, const float *theta, size_t n, float mean, float sd);
int he_mlp_get_params(const he_mlp *mlp, float *theta, size_t n, float *mean, float *sd);
/* one forward + backward pass over u[m]: mean loss and its gradient (theta order) */
int he_mlp_grad(he_mlp *mlp, const float *u, size_t m, float *loss, float *grad);
int he_mlp_forward(he_mlp *mlp, const float *u, size_t m, float *y);
/* Adam over shuffled mini-batches of u[m] (input normalisation maps [min u, max u] to [-1, 1]),
 * cosine-decayed step size from lr; *final_loss = loss over u afterwards */
int he_mlp_train(he_mlp *mlp, const float *u, size_t m, uint32_t epochs, uint32_t batch, float lr,
                 uint64_t seed, float *final_loss);
/* coef[0..4]: power-basis coefficients of y(u) */
int he_mlp_to_poly(const he_mlp *mlp, double *coef);
/* File form of a trained network (1356 bytes, little-endian): "HEMLPv1\n", uint32
 * parameter count 321 and hidden width 16, float32 mean and sd, the 321 float32
 * weights in the order above, the float64 coefficients c0..c4 of he_mlp_to_poly, and
 * an FNV-1a 64 checksum of everything before it.  he_mlp_save writes it (beside path,
 * then renamed onto it, so readers see the old or the new file whole);
 * he_mlp_load creates a network on `device` from it (weights and normalisation as
 * saved, Adam moments zero); he_mlp_file_poly reads only the coefficients, with no
 * GPU, for he_cutmax_cfg.init_coef.  Reads check size, magic, shape, checksum,
 * finiteness and that the stored coefficients are the collapse of the stored weights
 * (relative 1e-9): HE_EINVAL when they do not, HE_EIO when the file cannot be opened,
 * read, written or renamed. */
int he_mlp_save(const he_mlp *mlp, const char *path);
int he_mlp_load(const char *path, int device, he_mlp **out);
int he_mlp_file_poly(const char *path, double *coef);
/* Training data: plaintext CutMax (Alg. 1) runs on the GPU over synthetic
 * LLM-like logits (vocab tokens zero-padded to `slots`, per-run Gumbel scale
 * ~U[1.5,4.5] and Zipf exponent ~U[0.9,1.3]); var_out[runs][T] receives the
 * population variance entering each iteration, ymean_out[runs] (nullable) the
 * mean of the last iterate. */
int he_variance_log(uint64_t seed, uint32_t runs, uint32_t vocab, uint32_t slots, uint32_t T,
                    uint32_t p, double c, int device, float *var_out, float *ymean_out);
const char *he_mlp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
