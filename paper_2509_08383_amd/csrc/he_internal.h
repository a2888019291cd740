// Internal declarations of the MI355X RNS-CKKS / CutMax library.
//
// Device representation: every residue is an IEEE double holding a canonical
// integer in [0, q), q < 2^49.  Modular products run in the FP64 pipe (full
// rate on CDNA): h = a*b, l = fma(a, b, -h) gives a*b = h + l exactly, the
// quotient is rint(h * (1/q)), and the remainder fma(-quot, q, h) + l is exact
// because every intermediate integer stays below 2^53 (bounds in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace he {

constexpr int kMaxPrimes = 64;

// Pointers to the per-context device tables.
struct DevTables {
    int N, logN, np, L, alpha;
    const double *p;     // [np] primes
    const double *pinv;  // [np] fl(1/p)
    const double *tw;    // [np][N] psi^bitrev(k), canonical
    const double *itw;   // [np][N] psi^-bitrev(k)
    const double *ninv;  // [np] N^-1 mod p
    const double *two32; // [np] 2^32 mod p
    // evaluation-key high parts: bytes per word above the low 32 bits for each prime
    // (1 below 2^40, else 2) and the byte offset of each prime's rows in the high plane
    const int *khb;      // [np] (device)
    const int *khoff;    // [np] (device)
    const int *khb_h;    // [np] the same widths in host memory (byte accounting)
};

// A set of N-word vectors: vector v lives in group g = v / group at slot
// slot[r] (r = v % group) and is reduced modulo prime[r] (identity tables when
// null).  Address = base + g * gstride + slot * N.
struct VecSet {
    double *base;
    int count;
    int group;
    long long gstride;
    const int *slot;
    const int *prime;
};

// Per-vector constant: value = base[(g / gdiv) * stride + r].
struct ConstTab {
    const double *base;
    int gdiv;
    int stride;
};

// An evaluation key of residues below 2^48 with the two polynomials of a digit
// interleaved, stored as two planes.  Low plane: the low 32 bits of word (limb t, digit
// j, position x, polynomial c) at index ((t beta_L + j) N + x) 2 + c.  High plane: the
// bits above 32, in hb = khb[t] bytes (1 for primes below 2^40, 2 for the others), the
// rows of prime t from byte khoff[t] on and word (j, x, c) at khoff[t] + ((j N + x) 2 + c)
// hb.  A lane reads both words of a digit with one 8-byte load and one 2- or 4-byte load
// (5 or 6 bytes a word), and a wave's loads are contiguous.
struct KeyRef {
    const uint32_t *lo;
    const uint8_t *hi;
};

// optional per-kernel profiler: when set, every launch is bracketed by HIP
// events on its stream (see he_profile_begin / he_profile_end)
struct KProf;
extern KProf *g_kprof;
void kprof_mark(const char *name, hipStream_t s, bool end);
void kprof_set_bytes(double algorithmic_bytes);  // for the next launch

#define KLN(name, kern, grid, block, shm, stream, ...)                   \
    do {                                                                 \
        if (g_kprof) kprof_mark(name, stream, false);                    \
        hipLaunchKernelGGL(kern, grid, block, shm, stream, __VA_ARGS__); \
        if (g_kprof) kprof_mark(name, stream, true);                     \
    } while (0)

// NTT schedule tuning (ntt.hip): variant 1..NTT_VARIANTS per (log N, batch bucket)
constexpr int NTT_VARIANTS = 6;
void set_ntt_tuning(int logN, int bucket, int variant);

// ---------------------------------------------------------------- kernels.hip
// in place, or from *src into vs; the inverse multiplies by oscale[r] (per slot)
// instead of N^-1 when oscale is given.  strided_only (inverse, in place): vs already
// holds the first inverse pass (the contiguous-block stages, as a chained forward
// epilogue writes it) and only the second runs.
void launch_ntt(const DevTables &T, const VecSet &vs, bool inverse, int variant, hipStream_t s,
                const VecSet *src = nullptr, const double *oscale = nullptr, bool strided_only = false);

// Forward-NTT prologue: kind 1 loads, for vector (g, r), the centred lift of the
// coefficient-domain word last[g * l_g + j] (modulo ql) reduced modulo prime(r).
// Inverse-NTT prologue (first pass): kind 2 forms, for vector (g, r) = (ciphertext,
// limb), the tensor of ciphertexts a (ta + g ta_ct) and b (tb + tmap[g] tb_ct, tmap
// null: g), polynomial 1 at + ta_poly / + tb_poly: d0 = a0 b0, d1 = a0 b1 + a1 b0,
// d2 = a1 b1 at td + g td_ct + k td_poly + r N; d2 is the word the pass transforms.
struct NttPro {
    int kind;
    const double *last;
    long long l_g;
    double ql;
    const double *ta, *tb;
    long long ta_ct, tb_ct, ta_poly, tb_poly;
    const int *tmap;
    double *td;
    long long td_ct, td_poly;
};
// Forward-NTT epilogue on the transformed word w of vector (g, r), position j:
//   kind 1 (ModDown): out = (in - w) * cst[r] + [m1] add1 + [m2] add2
//   kind 2 (rescale): out = (K in - w) * cst[r], K = kmul[(g >> 1) * kstride + r] or 1
//   kind 3 (ModDown by P q_l): out = (in - w) * cst[r] + add1 * cst2[r]
// with in = in[g * i_g + r N + j], out[g * o_g + r N + j], addk[(g>>1) ak_ct +
// (g&1) ak_poly + r N + j] applied when bit (g & 1) of mk is set.  chain (kind 1): the
// output words also go through the first pass of the inverse NTT (its contiguous-block
// stages, which cover the same blocks) into chain[g * ch_g + r N + j], the input of a
// following inverse NTT's second pass.
struct NttEpi {
    int kind;
    double *out;
    long long o_g;
    const double *in;
    long long i_g;
    const double *add1;
    long long a1_ct, a1_poly;
    int m1;
    const double *add2;
    long long a2_ct, a2_poly;
    int m2;
    const double *cst;
    const double *kmul;
    int kstride;
    const double *cst2;
    // 0: vector groups alternate the two polynomials (group g = 2 ct + poly); 1: every
    // group is polynomial 1 of ciphertext g (the addends are indexed accordingly)
    int poly1;
    double *chain;
    long long ch_g;
};
// passes: 3 both; 2 the second alone (vs holds the first pass's output, as
// launch_moddown_ntt writes it)
void launch_ntt_fused(const DevTables &T, const VecSet &vs, const NttPro &pro, const NttEpi &epi, int variant,
                      hipStream_t s, int passes = 3);
// the second pass of the forward NTT alone (vs holds the first pass's output)
void launch_ntt_fwd_pass2(const DevTables &T, const VecSet &vs, int variant, hipStream_t s);
// the tensor of pro (kind 2) and the first pass of the inverse NTT of its d2 into vs
// (the second pass is launch_ntt(..., strided_only) on vs)
void launch_tensor_intt(const DevTables &T, const VecSet &vs, const NttPro &pro, int variant, hipStream_t s);
void launch_add(const DevTables &T, const VecSet &out, const VecSet &a, const VecSet &b, int sign,
                hipStream_t s);
void launch_copy(const DevTables &T, const VecSet &out, const VecSet &a, hipStream_t s);
void launch_mul_const(const DevTables &T, const VecSet &out, const VecSet &a, ConstTab k,
                      hipStream_t s);
void launch_add_const(const DevTables &T, const VecSet &out, const VecSet &a, ConstTab k,
                      hipStream_t s, int c0only = 0);
void launch_axpy_map(const DevTables &T, const VecSet &out, const VecSet &a, ConstTab k,
                     const VecSet &b, const int *bmap, int bdiv, hipStream_t s);
void launch_sub_mul_map(const DevTables &T, const VecSet &out, const VecSet &a, ConstTab k, const VecSet &b,
                        const int *bmap, int bdiv, hipStream_t s);
void launch_sum_groups(const DevTables &T, const VecSet &out, const VecSet &in, const int *first,
                       const int *cnt, int gdiv, hipStream_t s);
void launch_automorph(const DevTables &T, const VecSet &out, const VecSet &in, uint64_t galois,
                      hipStream_t s);
struct ModUpDigits {
    const double *qhat[8];  // [dl][next] per digit
    int lo[8], dl[8];
};
void launch_modup(const DevTables &T, const double *v, long long vstride, double *ext, long long esb,
                  long long esj, const double *dntt, long long nstride, int cnt, int beta, int next,
                  const int *ext_prime, const ModUpDigits &dg, hipStream_t s);
// ModUp of every digit (as launch_modup, the own slots left unwritten) fused with the
// first pass of the forward NTT of the converted slots; launch_ntt_fwd_pass2 over those
// slots completes the transform
void launch_modup_ntt(const DevTables &T, const double *v, long long vstride, double *ext, long long esb,
                      long long esj, int cnt, int beta, int next, const int *ext_prime, const ModUpDigits &dg,
                      hipStream_t s);
// Where the key products read a digit's own limbs: with p set, limb t <= l of digit
// t / alpha (the NTT-domain input word itself) is read at p + ct * ct_stride + t N
// instead of from the extended digits; p null: every limb from the extended digits.
struct OwnSrc {
    const double *p;
    long long ct_stride;
    int alpha, l;
};
void launch_inner_product(const DevTables &T, const double *ext, long long estride_b,
                          long long estride_j, double *acc0, double *acc1, long long astride,
                          KeyRef key, int betaL, int cnt,
                          int beta, int next, const int *ext_prime, hipStream_t s,
                          const double *dadd = nullptr, long long dct = 0, long long dpoly = 0, int tl = -1,
                          double pmodl = 0.0, const OwnSrc &own = OwnSrc{});
void launch_pack_key(const DevTables &T, const double *src, uint32_t *lo, uint8_t *hi, int beta, int np, int N,
                     hipStream_t s);

// terms of a plaintext-times-ciphertext sum (bootstrap linear transforms): plaintext
// pt[t] ([limbs][N], NTT domain) times ciphertext x[t] (ciphertext c at x + c xct,
// polynomial 1 at + xpoly, limb i at + i N)
constexpr int kMaxLtTerms = 16;
struct LtTerms {
    const double *pt[kMaxLtTerms];
    const double *x[kMaxLtTerms];
    long long xct[kMaxLtTerms];
    long long xpoly[kMaxLtTerms];
    int n;
};
void launch_lt_inner(const DevTables &T, double *out, long long oct, long long opoly, const LtTerms &tm, int cnt,
                     int limbs, hipStream_t s);
// every giant-step sum of one baby-step giant-step linear transform in one pass:
// out[a] = sum_b pt[a][b] * x[b] (pt[a][b] null where giant a has no diagonal for baby b),
// each baby word loaded once for all giants
constexpr int kMaxLtBaby = 8, kMaxLtGiant = 8;
struct LtGiants {
    const double *pt[kMaxLtGiant][kMaxLtBaby];
    const double *x[kMaxLtBaby];
    long long xct[kMaxLtBaby], xpoly[kMaxLtBaby];
    double *out[kMaxLtGiant];
    long long oct, opoly;
    int nb, ng;
};
void launch_lt_giants(const DevTables &T, const LtGiants &g, int cnt, int limbs, hipStream_t s);
// out = sum_t k_t x_t with integer constants (residues kres[(t cnt + c) limbs + i])
void launch_lincomb(const DevTables &T, double *out, long long oct, long long opoly, const LtTerms &tm,
                    const double *kres, int cnt, int limbs, hipStream_t s);

// Basis-conversion grids are one-dimensional and XCD-aware: workgroup b runs on XCD
// b mod 8, and the target blocks of one coefficient block (which all read the same
// input words) are consecutive workgroups of one XCD, so the input is fetched from
// HBM once and re-read from that XCD's L2.  conv_idx returns false for padding
// workgroups.
struct ConvIdx {
    int tb, cb, z;
};
__device__ __forceinline__ bool conv_idx(int b, int ntb, int cblk, int nz, ConvIdx &o) {
    const int slot = b >> 3, c = (slot / ntb) * 8 + (b & 7);
    if (c >= cblk * nz) return false;
    o.tb = slot % ntb;
    o.cb = c % cblk;
    o.z = c / cblk;
    return true;
}
inline dim3 conv_grid(int ntb, int cblk, int nz) { return dim3(8 * ntb * ((cblk * nz + 7) / 8)); }
// smallest compiled digit length that holds dl words
inline int digit_len(int dl) { return dl <= 4 ? 4 : dl <= 8 ? 8 : dl <= 10 ? 10 : dl <= 12 ? 12 : 16; }

// rotations of one hoisted rotate-and-sum step: key and Galois element of each
constexpr int kMaxHoist = 15;
struct RotSet {
    KeyRef key[kMaxHoist];
    uint32_t g[kMaxHoist];
    int nr;
    // with c0: limbs t <= lq also get s0 = c0 + sum_r sigma_r(c0) (c0 + ct c0_ct + t N, s0 alike)
    const double *c0;
    long long c0_ct;
    double *s0;
    long long s0_ct;
    int lq;
    const int *xorder;  // the N/256 x-blocks in the orbit order of g[0] (device)
    int c0_id;          // 1: s0 includes c0 itself (rotate-and-sum), 0: only the rotated copies
    // fold != 0: instead of writing s0, acc0 <- acc0 + s0 on every limb t <= lq (limbs
    // above lq take acc0 alone); c0_mul (per extended limb, may be null) multiplies the
    // sum first (rotate-and-sum carrying P c0 over Q u P between its hoisted steps)
    int fold;
    const double *c0_mul;
    // multi != 0: rotation r acts on its own ciphertext: extended digits ext_r[r] (same
    // strides as ext) and c0 at c0_r[r] (stride c0_ct); s0 = sum_r sigma_r(c0_r)
    int multi;
    const double *ext_r[kMaxHoist];
    const double *c0_r[kMaxHoist];
    OwnSrc own;  // the digits' own limbs (not with multi)
};
void launch_inner_product_rot(const DevTables &T, const double *ext, long long estride_b, long long estride_j,
                              double *acc0, double *acc1, long long astride, const RotSet &rs, int betaL,
                              int cnt, int beta, int next, const int *ext_prime, hipStream_t s);
// inputs: slots in0 .. in0+nin-1 of each group, prime index in_prime[m]; targets
// q_0 .. q_{ntgt-1}; [Bhat_m]_{q_i} = ph[m * phs + i]
struct MdIn {
    int in0, nin;
    const int *in_prime;
    const double *ph;
    int phs, ntgt;
};
// ModDown conversion fused with the first pass of the forward NTT of its output: acc
// holds, at slots in0 .. in0+nin-1 of every group, the coefficient-domain words
// w_m = [A_m Bhat_m^-1]_{b_m} of the basis being divided out (the inverse NTT applied
// the scaling); each is lifted to its centred representative and conv_i = sum_m w_m
// [Bhat_m]_{q_i} for the targets i < ntgt (prime i), transformed by the first pass;
// launch_ntt_fused(..., passes = 2) on conv completes the transform
void launch_moddown_ntt(const DevTables &T, const double *acc, long long astride, double *conv, long long cstride,
                        int groups, const MdIn &md, hipStream_t s);
void launch_sample_uniform(const DevTables &T, const VecSet &out, uint64_t seed, uint32_t obj,
                           const int *gprime, hipStream_t s);
void launch_sample_small(int *out, int N, uint64_t seed, uint32_t obj, int kind, hipStream_t s);
void launch_small_to_res(const DevTables &T, const VecSet &out, const int *v, const int *gprime,
                         hipStream_t s);
void launch_int64_to_res(const DevTables &T, const VecSet &out, const int64_t *m,
                         long long mstride, const int *gprime, hipStream_t s);
void launch_keyb(const DevTables &T, double *b, const double *a, const double *e, const double *s,
                 const double *tgt, const double *pmod, int np, int lo, int hi, hipStream_t st);
void launch_encfinish(const DevTables &T, double *c0, const double *a, const double *e,
                      const double *m, const double *s, long long stride, int limbs, int cnt,
                      long long ctstride, long long mctstride, hipStream_t st);
void launch_decmul(const DevTables &T, double *m, const double *c0, const double *c1,
                   const double *s, int limbs, hipStream_t st);
void launch_square_res(const DevTables &T, double *out, const double *in, int np, hipStream_t st);

// ----------------------------------------------------------------- host math
uint64_t mulmod_u(uint64_t a, uint64_t b, uint64_t q);
uint64_t powmod_u(uint64_t a, uint64_t e, uint64_t q);
uint64_t invmod_u(uint64_t a, uint64_t q);
uint64_t red_i64(int64_t v, uint64_t q);
bool miller_rabin(uint64_t n);
std::vector<uint64_t> gen_primes(int logN, int n_q, int q0_bits, int q_bits, int p_bits,
                                 int alpha, int n_hi = 0, int hi_bits = 0);
void philox_host(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed, uint32_t out[4]);
std::vector<int> sparse_secret(int N, int hw, uint64_t seed, uint32_t obj);
uint64_t find_psi(uint64_t q, int N);
void encode_slots(const double *z, int N, double scale, int64_t *m);
void decode_slots(const double *m, int N, double scale, double *z);
void chebyshev_invsqrt_fit(double u_lo, int degree, double *coef);
bool invsqrt_scaled_plan(double u_lo, int degree, int K, double *coef, double *steps, double *ranges);
int64_t llround_d(double x);

}  // namespace he
