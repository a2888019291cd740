// HIP kernels for gfx950: RNS-CKKS primitives of the encrypted CutMax.
//
// Residues are canonical integers in [0, p) stored as doubles, p < 2^49.
// Modular arithmetic runs in the FP64 pipe:
//   mm(a, b): h = a*b; l = fma(a, b, -h)          (a*b = h + l exactly)
//             k = rint(h * pinv); r = fma(-k, p, h) + l
// For |a| < 2^52 and 0 <= b < p the true quotient a*b/p is below 2^52 in
// magnitude, fl(h*pinv) is within 3*2^-53 relative of it, so |a*b - k*p| is at
// most (0.5 + |a*b/p| * 3 * 2^-53) p; with the bounds used below every
// intermediate is an integer below 2^53 and therefore exact.  red(x) =
// x - rint(x*pinv)*p maps |x| < 2^52 to |x| <= p/2 (plus a negligible
// fraction), canon() to [0, p).
#include "he_internal.h"

namespace he {

#define DEV __device__ __forceinline__

// kernel launch with the optional per-kernel event profiler around it
#define KL(name, kern, grid, block, shm, stream, ...)                 \
    do {                                                              \
        if (g_kprof) kprof_mark(name, stream, false);                 \
        hipLaunchKernelGGL(kern, grid, block, shm, stream, __VA_ARGS__); \
        if (g_kprof) kprof_mark(name, stream, true);                  \
    } while (0)

DEV double mm(double a, double b, double p, double pinv) {
    double h = a * b;
    double l = __builtin_fma(a, b, -h);
    double k = __builtin_rint(h * pinv);
    double r = __builtin_fma(-k, p, h);
    return r + l;
}
DEV double red(double x, double p, double pinv) { return __builtin_fma(-__builtin_rint(x * pinv), p, x); }
DEV double canon(double x, double p, double pinv) {
    double r = red(x, p, pinv);
    return r < 0.0 ? r + p : r;
}
DEV double addm(double a, double b, double p) {  // a, b canonical
    double r = a + b;
    return r >= p ? r - p : r;
}
DEV double subm(double a, double b, double p) {
    double r = a - b;
    return r < 0.0 ? r + p : r;
}

DEV void vs_at(const VecSet &v, int idx, int N, double *&ptr, int &pr, int &g, int &r) {
    g = idx / v.group;
    r = idx - g * v.group;
    int sl = v.slot ? v.slot[r] : r;
    pr = v.prime ? v.prime[r] : r;
    ptr = v.base + (long long)g * v.gstride + (long long)sl * N;
}
DEV double ct_val(const ConstTab &k, int g, int r) { return k.base[(long long)(g / k.gdiv) * k.stride + r]; }

// --------------------------------------------------------------- elementwise
#define EW_PROLOGUE                                          \
    const int x = blockIdx.x * blockDim.x + threadIdx.x;     \
    if (x >= T.N) return;                                    \
    double *po; int pr, g, r;                                \
    vs_at(out, blockIdx.y, T.N, po, pr, g, r);               \
    const double p = T.p[pr];                                \
    (void)p;

static dim3 ew_grid(const DevTables &T, int count) { return dim3((T.N + 255) / 256, count); }

__global__ void k_add(VecSet out, VecSet a, VecSet b, DevTables T, int sign) {
    EW_PROLOGUE
    double *pa, *pb; int q1, q2, g1, r1;
    vs_at(a, blockIdx.y, T.N, pa, q1, g1, r1);
    vs_at(b, blockIdx.y, T.N, pb, q2, g1, r1);
    po[x] = sign > 0 ? addm(pa[x], pb[x], p) : subm(pa[x], pb[x], p);
}
void launch_add(const DevTables &T, const VecSet &out, const VecSet &a, const VecSet &b, int sign,
                hipStream_t s) {
    if (out.count <= 0) return;
    kprof_set_bytes(24.0 * T.N * out.count);
    KL("k_add", k_add, ew_grid(T, out.count), dim3(256), 0, s, out, a, b, T, sign);
}

__global__ void k_copy(VecSet out, VecSet a, DevTables T) {
    EW_PROLOGUE
    double *pa; int q1, g1, r1;
    vs_at(a, blockIdx.y, T.N, pa, q1, g1, r1);
    po[x] = pa[x];
}
void launch_copy(const DevTables &T, const VecSet &out, const VecSet &a, hipStream_t s) {
    if (out.count <= 0) return;
    kprof_set_bytes(16.0 * T.N * out.count);
    KL("k_copy", k_copy, ew_grid(T, out.count), dim3(256), 0, s, out, a, T);
}

__global__ void k_mul_const(VecSet out, VecSet a, ConstTab k, DevTables T) {
    EW_PROLOGUE
    double *pa; int q1, g1, r1;
    vs_at(a, blockIdx.y, T.N, pa, q1, g1, r1);
    const double pinv = T.pinv[pr];
    po[x] = canon(mm(pa[x], ct_val(k, g, r), p, pinv), p, pinv);
}
void launch_mul_const(const DevTables &T, const VecSet &out, const VecSet &a, ConstTab k,
                      hipStream_t s) {
    if (out.count <= 0) return;
    kprof_set_bytes(16.0 * T.N * out.count);
    KL("k_mul_const", k_mul_const, ew_grid(T, out.count), dim3(256), 0, s, out, a, k, T);
}

// adds the constant to every NTT-domain coefficient (a constant polynomial
// evaluates to itself at every root); with c0only the groups are (ciphertext,
// polynomial) pairs and only polynomial 0 gets the constant, polynomial 1 is copied
__global__ void k_add_const(VecSet out, VecSet a, ConstTab k, DevTables T, int c0only) {
    EW_PROLOGUE
    double *pa; int q1, g1, r1;
    vs_at(a, blockIdx.y, T.N, pa, q1, g1, r1);
    po[x] = (c0only && (g & 1)) ? pa[x] : addm(pa[x], ct_val(k, g, r), p);
}
void launch_add_const(const DevTables &T, const VecSet &out, const VecSet &a, ConstTab k,
                      hipStream_t s, int c0only) {
    if (out.count <= 0) return;
    kprof_set_bytes(16.0 * T.N * out.count);
    KL("k_add_const", k_add_const, ew_grid(T, out.count), dim3(256), 0, s, out, a, k, T, c0only);
}

// out = a * k - b[map]   (b group index = bmap[g / bdiv] * bdiv + g % bdiv)
__global__ void k_axpy_map(VecSet out, VecSet a, ConstTab k, VecSet b, const int *bmap, int bdiv,
                           DevTables T) {
    EW_PROLOGUE
    double *pa; int q1, g1, r1;
    vs_at(a, blockIdx.y, T.N, pa, q1, g1, r1);
    const int gb = bmap[g / bdiv] * bdiv + g % bdiv;
    double *pb; int q2, g2, r2;
    vs_at(b, gb * b.group + r, T.N, pb, q2, g2, r2);
    const double pinv = T.pinv[pr];
    po[x] = canon(mm(pa[x], ct_val(k, g, r), p, pinv) - pb[x], p, pinv);
}
void launch_axpy_map(const DevTables &T, const VecSet &out, const VecSet &a, ConstTab k,
                     const VecSet &b, const int *bmap, int bdiv, hipStream_t s) {
    if (out.count <= 0) return;
    kprof_set_bytes(24.0 * T.N * out.count);
    KL("k_axpy_map", k_axpy_map, ew_grid(T, out.count), dim3(256), 0, s, out, a, k, b, bmap, bdiv, T);
}

// out = a - k * b[map]  for the groups whose request has map[g / bdiv] >= 0 (b group
// map * bdiv + g % bdiv), out = a for the others
__global__ void k_sub_mul_map(VecSet out, VecSet a, ConstTab k, VecSet b, const int *bmap, int bdiv, DevTables T) {
    EW_PROLOGUE
    double *pa; int q1, g1, r1;
    vs_at(a, blockIdx.y, T.N, pa, q1, g1, r1);
    const int m = bmap[g / bdiv];
    if (m < 0) {
        po[x] = pa[x];
        return;
    }
    double *pb; int q2, g2, r2;
    vs_at(b, (m * bdiv + g % bdiv) * b.group + r, T.N, pb, q2, g2, r2);
    const double pinv = T.pinv[pr];
    po[x] = canon(pa[x] - mm(pb[x], ct_val(k, g, r), p, pinv), p, pinv);
}
void launch_sub_mul_map(const DevTables &T, const VecSet &out, const VecSet &a, ConstTab k, const VecSet &b,
                        const int *bmap, int bdiv, hipStream_t s) {
    if (out.count <= 0) return;
    kprof_set_bytes(24.0 * T.N * out.count);
    KL("k_sub_mul_map", k_sub_mul_map, ew_grid(T, out.count), dim3(256), 0, s, out, a, k, b, bmap, bdiv, T);
}

// out group g (= req * gdiv + j) = sum over k < cnt[req] of in group (first[req] + k) * gdiv + j
__global__ void k_sum_groups(VecSet out, VecSet in, const int *first, const int *cnt, int gdiv,
                             DevTables T) {
    EW_PROLOGUE
    const int req = g / gdiv, jj = g % gdiv;
    const double pinv = T.pinv[pr];
    double acc = 0.0;
    for (int k = 0; k < cnt[req]; ++k) {
        double *pi; int q1, g1, r1;
        vs_at(in, ((first[req] + k) * gdiv + jj) * in.group + r, T.N, pi, q1, g1, r1);
        acc += pi[x];
    }
    po[x] = canon(acc, p, pinv);
}
void launch_sum_groups(const DevTables &T, const VecSet &out, const VecSet &in, const int *first,
                       const int *cnt, int gdiv, hipStream_t s) {
    if (out.count <= 0) return;
    // the summed words are not known on the host (counts live on the device): every
    // output word with one input word is booked
    kprof_set_bytes(16.0 * T.N * out.count);
    KL("k_sum_groups", k_sum_groups, ew_grid(T, out.count), dim3(256), 0, s, out, in, first, cnt, gdiv, T);
}

// NTT-domain Galois automorphism X -> X^g: out[j] = in[j'] with
// 2 bitrev(j') + 1 = (2 bitrev(j) + 1) g mod 2N.  2N divides 2^32, so the
// product is taken modulo 2^32 and masked.
DEV unsigned aut_src(unsigned j, uint32_t g, int logN) {
    const int sh = 32 - logN;
    const uint32_t t = 2u * (__brev(j) >> sh) + 1u;
    const uint32_t t2 = (t * g) & ((2u << logN) - 1u);
    return __brev((t2 - 1u) >> 1) >> sh;
}
__global__ void k_automorph(VecSet out, VecSet in, uint64_t galois, DevTables T) {
    EW_PROLOGUE
    double *pi; int q1, g1, r1;
    vs_at(in, blockIdx.y, T.N, pi, q1, g1, r1);
    po[x] = pi[aut_src((unsigned)x, (uint32_t)galois, T.logN)];
}
void launch_automorph(const DevTables &T, const VecSet &out, const VecSet &in, uint64_t galois,
                      hipStream_t s) {
    if (out.count <= 0) return;
    kprof_set_bytes(16.0 * T.N * out.count);
    KL("k_automorph", k_automorph, ew_grid(T, out.count), dim3(256), 0, s, out, in, galois, T);
}

// ------------------------------------------------- plaintext products (bootstrap)
// out[c][poly][i] = sum_t pt_t[i] * x_t[c][poly][i] over limbs i < limbs, both
// polynomials: the inner sum of a baby-step giant-step linear transform (each pt_t
// an NTT-domain diagonal, x_t a rotated copy of the input) or, with one term, a
// plaintext product.  Each plaintext word is loaded once for both polynomials of every
// ciphertext (the ciphertexts are a loop inside the thread);
// |sum| <= n (p/2 + 2^44) < 2^52 for n <= kMaxLtTerms.
__global__ __launch_bounds__(256) void k_lt_inner(double *__restrict__ out, long long oct, long long opoly, LtTerms tm,
                                                  int cnt, DevTables T) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T.N) return;
    const int i = blockIdx.y;
    const double p = T.p[i], pinv = T.pinv[i];
    const long long w = (long long)i * T.N + x;
    // every plaintext word once, kept in registers for all ciphertexts of the batch
    double pv[kMaxLtTerms];
#pragma unroll
    for (int t = 0; t < kMaxLtTerms; ++t) pv[t] = t < tm.n ? tm.pt[t][w] : 0.0;
    for (int c = 0; c < cnt; ++c) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int t = 0; t < kMaxLtTerms; ++t) {
            if (t < tm.n) {
                const double *xp = tm.x[t] + c * tm.xct[t] + w;
                a0 += mm(xp[0], pv[t], p, pinv);
                a1 += mm(xp[tm.xpoly[t]], pv[t], p, pinv);
            }
        }
        double *o = out + c * oct + w;
        o[0] = canon(a0, p, pinv);
        o[opoly] = canon(a1, p, pinv);
    }
}
void launch_lt_inner(const DevTables &T, double *out, long long oct, long long opoly, const LtTerms &tm, int cnt,
                     int limbs, hipStream_t s) {
    if (cnt <= 0 || tm.n <= 0) return;
    // each term's plaintext limb once, its two ciphertext polynomials per ciphertext, two words out
    kprof_set_bytes(8.0 * T.N * limbs * ((double)tm.n * (1.0 + 2.0 * cnt) + 2.0 * cnt));
    KL("k_lt_inner", k_lt_inner, dim3((T.N + 255) / 256, limbs), dim3(256), 0, s, out, oct, opoly, tm, cnt, T);
}

// All giant-step sums of a linear transform at once: for each position the words of
// every baby (both polynomials) are loaded once and reused by every giant, which reads
// only its own plaintext words; the per-giant form would re-read the babies once per
// giant.  |sum| <= nb (p/2 + 2^44) < 2^52 for nb <= 8.
__global__ __launch_bounds__(256) void k_lt_giants(LtGiants g, int cnt, DevTables T) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T.N) return;
    const int i = blockIdx.y;
    const double p = T.p[i], pinv = T.pinv[i];
    const long long w = (long long)i * T.N + x;
    for (int c = 0; c < cnt; ++c) {
        double b0[kMaxLtBaby], b1[kMaxLtBaby];
#pragma unroll
        for (int b = 0; b < kMaxLtBaby; ++b) {
            if (b < g.nb) {
                const double *xp = g.x[b] + c * g.xct[b] + w;
                b0[b] = xp[0];
                b1[b] = xp[g.xpoly[b]];
            } else {
                b0[b] = 0.0;
                b1[b] = 0.0;
            }
        }
        for (int a = 0; a < g.ng; ++a) {
            double a0 = 0.0, a1 = 0.0;
#pragma unroll
            for (int b = 0; b < kMaxLtBaby; ++b) {
                const double *pt = g.pt[a][b];
                if (b < g.nb && pt) {
                    const double pv = pt[w];
                    a0 += mm(b0[b], pv, p, pinv);
                    a1 += mm(b1[b], pv, p, pinv);
                }
            }
            double *o = g.out[a] + c * g.oct + w;
            o[0] = canon(a0, p, pinv);
            o[g.opoly] = canon(a1, p, pinv);
        }
    }
}
void launch_lt_giants(const DevTables &T, const LtGiants &g, int cnt, int limbs, hipStream_t s) {
    if (cnt <= 0 || g.ng <= 0 || g.nb <= 0) return;
    int npt = 0;
    for (int a = 0; a < g.ng; ++a)
        for (int b = 0; b < g.nb; ++b) npt += g.pt[a][b] != nullptr;
    // every plaintext once, every baby once per ciphertext, every giant sum written
    kprof_set_bytes(8.0 * T.N * limbs * (npt + 2.0 * cnt * (g.nb + g.ng)));
    KL("k_lt_giants", k_lt_giants, dim3((T.N + 255) / 256, limbs), dim3(256), 0, s, g, cnt, T);
}

// out[c][poly][i] = sum_t k_t[c][i] * x_t[c][poly][i] (integer constants as residues,
// kres[(t cnt + c) limbs + i]), both polynomials, limbs i < limbs: a linear combination
// of ciphertexts at one level before a single rescale.  |sum| < 2^52 for n <= 16.
__global__ __launch_bounds__(256) void k_lincomb(double *__restrict__ out, long long oct, long long opoly, LtTerms tm,
                                                 const double *__restrict__ kres, int cnt, int limbs, DevTables T) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T.N) return;
    const int i = blockIdx.y, c = blockIdx.z;
    const double p = T.p[i], pinv = T.pinv[i];
    const long long w = (long long)i * T.N + x;
    double a0 = 0.0, a1 = 0.0;
    for (int t = 0; t < tm.n; ++t) {
        const double k = kres[((long long)t * cnt + c) * limbs + i];
        const double *xp = tm.x[t] + c * tm.xct[t] + w;
        a0 += mm(xp[0], k, p, pinv);
        a1 += mm(xp[tm.xpoly[t]], k, p, pinv);
    }
    double *o = out + c * oct + w;
    o[0] = canon(a0, p, pinv);
    o[opoly] = canon(a1, p, pinv);
}
void launch_lincomb(const DevTables &T, double *out, long long oct, long long opoly, const LtTerms &tm,
                    const double *kres, int cnt, int limbs, hipStream_t s) {
    if (cnt <= 0 || tm.n <= 0) return;
    kprof_set_bytes(8.0 * T.N * limbs * cnt * 2.0 * (tm.n + 1.0));
    KL("k_lincomb", k_lincomb, dim3((T.N + 255) / 256, limbs, cnt), dim3(256), 0, s, out, oct, opoly, tm, kres, cnt,
       limbs, T);
}

// ------------------------------------------------------------ key switching
// ModUp of every digit j ([lo_j, lo_j+dl_j) of the primes present at the level):
// v holds v_a = [d_{lo+a} * Qhat_a^-1]_{q_{lo+a}} in the coefficient domain (the
// inverse NTT applied that scaling); for every extended slot t outside the digit
// ext_j,t = sum_a v~_a [Qhat_a]_{prime(t)} with v~_a the centred representative of v_a
// (|v~_a| <= q/2); digit slots copy the NTT-domain input.  (The key switch itself runs
// the conversion fused with the NTT, k_modup_ntt; this form serves the extended digits
// the bootstrap's multi-rotation products precompute.)
// Grid: x = blocks of TB target slots (fastest, so the v words of one coefficient
// block stay in L2 across target blocks), y = coefficient blocks, z = (ciphertext,
// digit).  The block's [Qhat_a]_{prime(t)} table and moduli are staged in LDS (every
// lane reads the same word: a broadcast); terms a >= dl and own-digit targets carry
// zero constants, so the DL products of a target run without branches as independent
// chains.  |sum| <= DL (p/2 + 2^44) < 2^52 for DL <= 16.
// (Basis-conversion grids: conv_idx / conv_grid in he_internal.h.)

template <int DL, int TB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_modup(DevTables T, const double *__restrict__ v, long long vstride,
                                               double *__restrict__ ext, long long esb, long long esj,
                                               const double *__restrict__ dntt, long long nstride, int beta,
                                               int next, const int *__restrict__ ext_prime, ModUpDigits dg,
                                               int ntb, int cblk, int nz) {
    __shared__ double sq[DL * TB];
    __shared__ double sp[TB], si[TB];
    ConvIdx ix;
    if (!conv_idx(blockIdx.x, ntb, cblk, nz, ix)) return;
    const int ct = ix.z / beta, j = ix.z - (ix.z / beta) * beta;
    const int lo = dg.lo[j], dl = dg.dl[j];
    const int t0 = ix.tb * TB, tid = threadIdx.x;
    {
        const double *qh = dg.qhat[j];
        for (int i = tid; i < DL * TB; i += blockDim.x) {
            const int a = i / TB, t = t0 + (i - (i / TB) * TB);
            const bool own = t >= lo && t < lo + dl;
            sq[i] = (a < dl && t < next && !own) ? qh[a * next + t] : 0.0;
        }
        if (tid < TB) {
            const int pt = ext_prime[t0 + tid < next ? t0 + tid : 0];
            sp[tid] = T.p[pt];
            si[tid] = T.pinv[pt];
        }
    }
    __syncthreads();
    const int x = ix.cb * blockDim.x + tid;
    if (x >= T.N) return;
    bool need = false;
#pragma unroll
    for (int tt = 0; tt < TB; ++tt) {
        const int t = t0 + tt;
        need |= t < next && !(t >= lo && t < lo + dl);
    }
    // the digit words as centred representatives of [d_i Qhat_i^-1]_{q_i}: the
    // extension d + u D then has u of mean zero, so the key noise it multiplies adds
    // no constant offset to the key-switch output
    double va[DL];
    const double *vp = v + ct * vstride + (long long)lo * T.N + x;
#pragma unroll
    for (int a = 0; a < DL; ++a) {
        const double w = (need && a < dl) ? vp[(long long)a * T.N] : 0.0;
        const double qa = a < dl ? T.p[lo + a] : 1.0;
        va[a] = w > 0.5 * (qa - 1.0) ? w - qa : w;
    }
    double *X = ext + ct * esb + j * esj + x;
#pragma unroll
    for (int tt = 0; tt < TB; ++tt) {
        const int t = t0 + tt;
        if (t >= next) break;
        const double p = sp[tt], pinv = si[tt];
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < DL; ++a) acc += mm(va[a], sq[a * TB + tt], p, pinv);
        if (t >= lo && t < lo + dl) X[(long long)t * T.N] = dntt[ct * nstride + (long long)t * T.N + x];
        else X[(long long)t * T.N] = canon(acc, p, pinv);
    }
}

template <int TB>
static void modup_tb(int DL, int cblk, int nz, hipStream_t s, const DevTables &T, const double *v, long long vstride,
                     double *ext, long long esb, long long esj, const double *dntt, long long nstride, int beta,
                     int next, const int *ext_prime, const ModUpDigits &dg) {
    const int ntb = (next + TB - 1) / TB;
    const dim3 grid = conv_grid(ntb, cblk, nz);
#define MU_CASE(D)                                                                                          \
    case D:                                                                                                 \
        KL("k_modup", (k_modup<D, TB>), grid, dim3(256), 0, s, T, v, vstride, ext, esb, esj, dntt, nstride, \
           beta, next, ext_prime, dg, ntb, cblk, nz);                                                       \
        break;
    switch (DL) { MU_CASE(4) MU_CASE(8) MU_CASE(10) MU_CASE(12) MU_CASE(16) }
#undef MU_CASE
}

void launch_modup(const DevTables &T, const double *v, long long vstride, double *ext, long long esb,
                  long long esj, const double *dntt, long long nstride, int cnt, int beta, int next,
                  const int *ext_prime, const ModUpDigits &dg, hipStream_t s) {
    if (cnt <= 0) return;
    int dmax = 0;
    for (int j = 0; j < beta; ++j) dmax = dg.dl[j] > dmax ? dg.dl[j] : dmax;
    const int DL = digit_len(dmax);
    const int cblk = (T.N + 255) / 256;
    // wide target blocks when they still give a few waves per SIMD
    const bool wide = (long long)((next + 7) / 8) * cblk * cnt * beta >= 2048;
    int lp1 = 0;
    for (int j = 0; j < beta; ++j) lp1 += dg.dl[j];
    // the l+1 digit words in, every extended slot out; the l+1 NTT-domain words in and
    // out again unless skipped
    kprof_set_bytes(8.0 * T.N * cnt * (2.0 * lp1 + (double)beta * next));
    if (wide)
        modup_tb<8>(DL, cblk, cnt * beta, s, T, v, vstride, ext, esb, esj, dntt, nstride, beta, next, ext_prime,
                    dg);
    else
        modup_tb<4>(DL, cblk, cnt * beta, s, T, v, vstride, ext, esb, esj, dntt, nstride, beta, next, ext_prime,
                    dg);
}

// the two words (polynomials 0, 1) of digit j of prime t at position x: hi 2^32 + lo,
// exact (below 2^48); one 8-byte load of the low halves and one aligned 4-byte load of
// the high parts, without a branch: with 2-byte high parts (hb = 1) the dword at x / 2
// holds positions x and x ^ 1 and the lane takes its half
DEV void key_pair(const KeyRef &k, const DevTables &T, int betaL, int t, int j, int N, int x, double &k0,
                  double &k1) {
    // the row offsets are uniform across the wave, the position a 32-bit per-lane index
    const long long row = ((long long)t * betaL + j) * N * 2;
    const uint2 l = ((const uint2 *)(k.lo + row))[(unsigned)x];
    const int hb = T.khb[t];
    const uint32_t *hr = (const uint32_t *)(k.hi + T.khoff[t] + (long long)j * N * 2 * hb);
    const uint32_t w = hr[(unsigned)x >> (2 - hb)] >> (hb == 1 ? 16u * ((unsigned)x & 1u) : 0u);
    const uint32_t m = hb == 1 ? 0xffu : 0xffffu;
    k0 = __builtin_fma((double)(w & m), 4294967296.0, (double)l.x);
    k1 = __builtin_fma((double)((w >> (8 * hb)) & m), 4294967296.0, (double)l.y);
}

// src [beta][2][np][N] doubles -> packed planes with the polynomials interleaved
__global__ void k_pack_key(const double *__restrict__ src, uint32_t *__restrict__ lo, uint8_t *__restrict__ hi,
                           int beta, int np, int N, DevTables T) {
    const size_t per = (size_t)np * N, n = (size_t)beta * 2 * per;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t jc = i / per, pos = i - jc * per;  // jc = 2 j + c, pos = t N + x
        const size_t j = jc >> 1, c = jc & 1, t = pos / (size_t)N, x = pos - t * (size_t)N;
        const size_t o = ((t * (size_t)beta + j) * (size_t)N + x) * 2 + c;
        const uint64_t v = (uint64_t)src[i];
        lo[o] = (uint32_t)v;
        const int hb = T.khb[t];
        const size_t ho = (size_t)T.khoff[t] + ((j * (size_t)N + x) * 2 + c) * (size_t)hb;
        if (hb == 2) *(uint16_t *)(hi + ho) = (uint16_t)(v >> 32);
        else hi[ho] = (uint8_t)(v >> 32);
    }
}
void launch_pack_key(const DevTables &T, const double *src, uint32_t *lo, uint8_t *hi, int beta, int np, int N,
                     hipStream_t s) {
    KL("k_pack_key", k_pack_key, dim3(4096), dim3(256), 0, s, src, lo, hi, beta, np, N, T);
}

// bytes per position of one key row pair (both polynomials, 8 low bytes and 2 hb high
// bytes a slot) summed over the extended slots of a level with `next` slots (the Q
// primes 0..l, then the P primes)
static double key_row_bytes(const DevTables &T, int next) {
    const int l = next - T.alpha - 1;
    double b = 0.0;
    for (int t = 0; t < next; ++t) b += 8.0 + 2.0 * T.khb_h[t <= l ? t : T.L + 1 + (t - l - 1)];
    return b;
}

// the digit whose own limb is extended slot t when the key products read the own limbs
// from the NTT-domain input (ModUp then skipped their copy), else -1; uniform over a
// workgroup, which covers one slot
DEV int own_digit(const OwnSrc &o, int t) { return (o.p && t <= o.l) ? t / o.alpha : -1; }

// acc_c[ct][t] = sum_j ext[ct][j][t] * key[j][c][prime(t)]; the key words are
// read once per (t, x) and reused for every ciphertext of the batch.
// With dadd, slot tl also gets [P]_{q_tl} times the words dadd[ct dct + c dpoly + x]
// (the tensor's d0/d1 at limb tl: the relinearisation with the rescale folded in).
__global__ void k_inner_product(DevTables T, const double *ext, long long esb, long long esj,
                                double *acc0, double *acc1, long long astride, KeyRef key,
                                int betaL, int cnt, int beta, const int *ext_prime,
                                const double *dadd, long long dct, long long dpoly, int tl, double pmodl,
                                OwnSrc own) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T.N) return;
    const int t = blockIdx.y;
    const int oj = own_digit(own, t);
    const int pt = ext_prime[t];
    const double p = T.p[pt], pinv = T.pinv[pt];
    double k0[8], k1[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j < beta) key_pair(key, T, betaL, pt, j, T.N, x, k0[j], k1[j]);
    for (int ct = 0; ct < cnt; ++ct) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j < beta) {
                const double *D = j == oj ? own.p + ct * own.ct_stride : ext + ct * esb + j * esj;
                const double e = D[(long long)t * T.N + x];
                s0 += mm(e, k0[j], p, pinv);
                s1 += mm(e, k1[j], p, pinv);
            }
        }
        if (dadd && t == tl) {
            s0 += mm(dadd[ct * dct + x], pmodl, p, pinv);
            s1 += mm(dadd[ct * dct + dpoly + x], pmodl, p, pinv);
        }
        acc0[ct * astride + (long long)t * T.N + x] = canon(s0, p, pinv);
        acc1[ct * astride + (long long)t * T.N + x] = canon(s1, p, pinv);
    }
}
void launch_inner_product(const DevTables &T, const double *ext, long long estride_b,
                          long long estride_j, double *acc0, double *acc1, long long astride,
                          KeyRef key, int betaL, int cnt,
                          int beta, int next, const int *ext_prime, hipStream_t s, const double *dadd,
                          long long dct, long long dpoly, int tl, double pmodl, const OwnSrc &own) {
    if (cnt <= 0) return;
    // key words (5 or 6 bytes each) once, extended digits and both accumulators per ciphertext
    kprof_set_bytes(T.N * (beta * key_row_bytes(T, next) + 8.0 * next * cnt * (beta + 2.0)));
    KL("k_inner_product", k_inner_product, dim3((T.N + 255) / 256, next), dim3(256), 0, s, T, ext,
                       estride_b, estride_j, acc0, acc1, astride, key, betaL, cnt,
                       beta, ext_prime, dadd, dct, dpoly, tl, pmodl, own);
}

// Inner product of a hoisted rotate-and-sum step: for rotation r with Galois
// element g_r and key K_r, acc_c[ct][t][x] = sum_r sum_j ext[ct][j][t][src_r(x)]
// K_r[j][c][prime(t)][x], the automorphism of the NTT-domain extended digits being
// a gather (src_r = aut_src).  A modular product is below p/2 + 2^43 < 2^47.1 in
// magnitude (p < 2^48), so a partial sum of at most 21 products stays below 2^51.6:
// the sums are reduced once per floor(21 / beta) rotations (beta <= 8).
//
// An automorphism maps every aligned block of 256 NTT positions onto one aligned
// block, and the rotations of a step are powers pi^r of its smallest rotation pi, so
// the sources of x-block X are X, pi(X), .., pi^nr(X).  The grid is one-dimensional
// and XCD-aware: the 8 XCDs take workgroups round-robin (workgroup b runs on XCD
// b mod 8); every XCD is given whole targets t and walks a target's x-blocks in the
// order of their pi-orbits (rs.xorder), so consecutive workgroups on an XCD share all
// but one of their source blocks and re-read them from L2.
// BETA > 0 and NR > 0 fix the digit and rotation counts at compile time: the loop
// over the rotations is unrolled and has no branch, so every gather and key load of a
// ciphertext is issued before the first product waits on one (the loads of a wave are
// then in flight together instead of one rotation at a time).  BETA = 0 or NR = 0 read
// the runtime counts (at most 8 digits).
// c0 + sum_r sigma_r(c0) (g0, below 2^52) on the limbs that have it: written to s0, or
// with rs.fold added to the key-product sum s0 (below 2^51.6), times rs.c0_mul[t] when
// given; returns the new key-product sum (canonical when folded)
DEV double c0_sum(const RotSet &rs, bool wsum, double g0, double s0, int ct, int t, int x, int N, double p,
                  double pinv) {
    if (!wsum) return s0;
    double gc = canon(g0, p, pinv);
    if (!rs.fold) {
        rs.s0[ct * rs.s0_ct + (long long)t * N + x] = gc;
        return s0;
    }
    if (rs.c0_mul) gc = canon(mm(gc, rs.c0_mul[t], p, pinv), p, pinv);
    const double o = canon(s0, p, pinv) + gc;
    return o >= p ? o - p : o;
}
// (with three digits 3 waves per SIMD: at 4 the unrolled form spills to scratch)
template <int BETA, int NR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BETA >= 3 ? 3 : 4))) void k_inner_product_rot(
    DevTables T, const double *__restrict__ ext, long long esb, long long esj, double *__restrict__ acc0,
    double *__restrict__ acc1, long long astride, RotSet rs, int betaL, int cnt, int beta_rt, int next,
    const int *__restrict__ ext_prime, int xblocks) {
    const int beta = BETA > 0 ? BETA : beta_rt;
    const int nr = NR > 0 ? NR : rs.nr;
    constexpr int JM = BETA > 0 ? BETA : 8;
    const int rk = 21 / beta > 0 ? 21 / beta : 1;  // rotations between reductions
    const int b = blockIdx.x, slot = b >> 3;
    const int t = (b & 7) + 8 * (slot / xblocks);
    if (t >= next) return;
    const int x = rs.xorder[slot % xblocks] * blockDim.x + threadIdx.x;
    if (x >= T.N) return;
    const int pt = ext_prime[t];
    const double p = T.p[pt], pinv = T.pinv[pt];
    const bool wsum = rs.c0 && t <= rs.lq;
    const int oj = own_digit(rs.own, t);
    // the unrolled form serves one ciphertext (the key loads then stay inside the
    // rotation chunks instead of being hoisted out of a ciphertext loop)
    const int ncts = BETA > 0 && NR > 0 ? 1 : cnt;
    for (int ct = 0; ct < ncts; ++ct) {
        const double *E = ext + ct * esb + (long long)t * T.N;
        const double *O = oj >= 0 ? rs.own.p + ct * rs.own.ct_stride + (long long)t * T.N : nullptr;
        const double *C0 = wsum ? rs.c0 + ct * rs.c0_ct + (long long)t * T.N : nullptr;
        double s0 = 0.0, s1 = 0.0;
        if (BETA > 0 && NR > 0) {
            constexpr int R = NR > 0 ? NR : 1, J = BETA > 0 ? BETA : 1;
            constexpr int RC = R > (J >= 3 ? 2 : 4) ? (J >= 3 ? 2 : 4) : R;  // rotations whose loads fly together
            double g0 = wsum && rs.c0_id ? C0[x] : 0.0;
#pragma unroll
            for (int r0 = 0; r0 < R; r0 += RC) {
                double e[RC][J], a0[RC][J], a1[RC][J], c[RC];
#pragma unroll
                for (int rr = 0; rr < RC; ++rr) {
                    if (r0 + rr < R) {
                        const unsigned src = aut_src((unsigned)x, rs.g[r0 + rr], T.logN);
#pragma unroll
                        for (int j = 0; j < J; ++j) {
                            e[rr][j] = (j == oj ? O : E + j * esj)[src];
                            key_pair(rs.key[r0 + rr], T, betaL, pt, j, T.N, x, a0[rr][j], a1[rr][j]);
                        }
                        c[rr] = wsum ? C0[src] : 0.0;
                    }
                }
#pragma unroll
                for (int rr = 0; rr < RC; ++rr) {
                    const int r = r0 + rr;
                    if (r < R) {
#pragma unroll
                        for (int j = 0; j < J; ++j) {
                            s0 += mm(e[rr][j], a0[rr][j], p, pinv);
                            s1 += mm(e[rr][j], a1[rr][j], p, pinv);
                        }
                        if ((r + 1) % (21 / J) == 0) {
                            s0 = red(s0, p, pinv);
                            s1 = red(s1, p, pinv);
                        }
                        g0 += c[rr];  // c0 + sum_r sigma_r(c0): at most 16 canonical words, below 2^52
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            s0 = c0_sum(rs, wsum, g0, s0, ct, t, x, T.N, p, pinv);
        } else {
            double g0 = wsum && rs.c0_id ? C0[x] : 0.0;
            for (int r = 0; r < nr; ++r) {
                const unsigned src = aut_src((unsigned)x, rs.g[r], T.logN);
                if (wsum) g0 = red(g0 + C0[src], p, pinv);
                const KeyRef K = rs.key[r];
#pragma unroll
                for (int j = 0; j < JM; ++j) {
                    if (j < beta) {
                        const double e = (j == oj ? O : E + j * esj)[src];
                        double w0, w1;
                        key_pair(K, T, betaL, pt, j, T.N, x, w0, w1);
                        s0 += mm(e, w0, p, pinv);
                        s1 += mm(e, w1, p, pinv);
                    }
                }
                if ((r + 1) % rk == 0) {
                    s0 = red(s0, p, pinv);
                    s1 = red(s1, p, pinv);
                }
            }
            s0 = c0_sum(rs, wsum, g0, s0, ct, t, x, T.N, p, pinv);
        }
        acc0[ct * astride + (long long)t * T.N + x] = canon(s0, p, pinv);
        acc1[ct * astride + (long long)t * T.N + x] = canon(s1, p, pinv);
    }
}
// The same products with every key word of the step held in registers (NR
// rotations, BETA <= 3 digits) and reused for every ciphertext of the batch, on the
// same XCD-aware grid.  Per ciphertext the NR x BETA gathers of the extended digits
// and the NR + 1 gathers of c0 are issued together (no branch between them), then the
// products run.
template <int NR, int BETA>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_inner_product_rot_reg(DevTables T, const double *__restrict__ ext,
                                                               long long esb, long long esj,
                                                               double *__restrict__ acc0, double *__restrict__ acc1,
                                                               long long astride, RotSet rs, int betaL,
                                                               int cnt, int next,
                                                               const int *__restrict__ ext_prime, int xblocks) {
    constexpr int RK = 21 / BETA;  // rotations between reductions
    const int b = blockIdx.x, slot = b >> 3;
    const int t = (b & 7) + 8 * (slot / xblocks);
    if (t >= next) return;
    const int x = rs.xorder[slot % xblocks] * blockDim.x + threadIdx.x;
    if (x >= T.N) return;
    const int pt = ext_prime[t];
    const double p = T.p[pt], pinv = T.pinv[pt];
    double k0[NR][BETA], k1[NR][BETA];
    unsigned src[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        src[r] = aut_src((unsigned)x, rs.g[r], T.logN);
#pragma unroll
        for (int j = 0; j < BETA; ++j) key_pair(rs.key[r], T, betaL, pt, j, T.N, x, k0[r][j], k1[r][j]);
    }
    const bool wsum = rs.c0 && t <= rs.lq;
    // rotations whose gathers are in flight together: with 7 x 3 keys held, chunks of 5
    // fit 3 waves per SIMD without spilling (160 VGPRs)
    constexpr int RCW = BETA >= 3 && NR >= 7 ? 5 : 3;
    constexpr int RC = NR > RCW ? RCW : NR;
    const int oj = own_digit(rs.own, t);
    for (int ct = 0; ct < cnt; ++ct) {
        const double *E = ext + ct * esb + (long long)t * T.N;
        const double *O = oj >= 0 ? rs.own.p + ct * rs.own.ct_stride + (long long)t * T.N : nullptr;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int r0 = 0; r0 < NR; r0 += RC) {
            double e[RC][BETA];
#pragma unroll
            for (int rr = 0; rr < RC; ++rr)
#pragma unroll
                for (int j = 0; j < BETA; ++j)
                    if (r0 + rr < NR) e[rr][j] = (j == oj ? O : E + j * esj)[src[r0 + rr]];
#pragma unroll
            for (int rr = 0; rr < RC; ++rr) {
                const int r = r0 + rr;
                if (r < NR) {
#pragma unroll
                    for (int j = 0; j < BETA; ++j) {
                        s0 += mm(e[rr][j], k0[r][j], p, pinv);
                        s1 += mm(e[rr][j], k1[r][j], p, pinv);
                    }
                    if ((r + 1) % RK == 0) {
                        s0 = red(s0, p, pinv);
                        s1 = red(s1, p, pinv);
                    }
                }
            }
            // keep the next chunk's gathers behind this chunk's products (register budget)
            __builtin_amdgcn_sched_barrier(0);
        }
        acc1[ct * astride + (long long)t * T.N + x] = canon(s1, p, pinv);
        if (wsum) {
            const double *C0 = rs.c0 + ct * rs.c0_ct + (long long)t * T.N;
            double g0 = rs.c0_id ? C0[x] : 0.0;
#pragma unroll
            for (int r = 0; r < NR; ++r) g0 += C0[src[r]];
            s0 = c0_sum(rs, true, g0, s0, ct, t, x, T.N, p, pinv);
        }
        acc0[ct * astride + (long long)t * T.N + x] = canon(s0, p, pinv);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The same products for a step whose automorphisms keep every aligned 256-word block
// within at most NS = 2 blocks: the block an automorphism sends block X to depends only
// on its Galois element mod N/128, so when those residues take at most one value h
// besides 1, the sources of block X are X itself and (NS = 2) one block Y.  Each
// ciphertext's source blocks of the BETA digits and of c0 are staged in LDS with one
// coalesced word per thread and block, and the gathers read LDS: NS (BETA + 1) words per
// position pass through the vector memory path instead of NR (BETA + 1) + 1.  smask bit
// r marks the rotations whose residue is h (sources in Y = the image of X under gh).
// The next ciphertext's words are loaded while the current one's products run (two LDS
// buffers, one barrier per ciphertext).  Every key word of the step stays in registers.
template <int NR, int BETA, int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_inner_product_rot_lds(
    DevTables T, const double *__restrict__ ext, long long esb, long long esj, double *__restrict__ acc0,
    double *__restrict__ acc1, long long astride, RotSet rs, int betaL, int cnt, int next,
    const int *__restrict__ ext_prime, int xblocks, uint32_t gh, uint32_t smask) {
    constexpr int RK = 21 / BETA;  // rotations between reductions
    constexpr int NQ = BETA + 1;   // the digits, then c0
    __shared__ double sw[2][NS][NQ][256];
    const int b = blockIdx.x, slot = b >> 3;
    const int t = (b & 7) + 8 * (slot / xblocks);
    if (t >= next) return;  // uniform over the workgroup
    const int xb = rs.xorder[slot % xblocks], tid = threadIdx.x;
    const int x = xb * 256 + tid;  // N is a multiple of 256: every thread has a position
    const int pt = ext_prime[t];
    const double p = T.p[pt], pinv = T.pinv[pt];
    const bool wsum = rs.c0 && t <= rs.lq;
    // word offset of each staged block: X, then Y
    long long sbo[NS];
    sbo[0] = (long long)xb * 256;
    if (NS == 2) sbo[NS - 1] = (long long)(aut_src((unsigned)xb * 256u, gh, T.logN) >> 8) * 256;
    double k0[NR][BETA], k1[NR][BETA];
    int so[NR];  // LDS word of rotation r's source: block slot * 256 + offset in the block
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const unsigned src = aut_src((unsigned)x, rs.g[r], T.logN);
        so[r] = (NS == 2 && ((smask >> r) & 1) ? 256 : 0) + (int)(src & 255u);
#pragma unroll
        for (int j = 0; j < BETA; ++j) key_pair(rs.key[r], T, betaL, pt, j, T.N, x, k0[r][j], k1[r][j]);
    }
    double w[NS][NQ];
    const int oj = own_digit(rs.own, t);
    auto fetch = [&](int ct) {
        const double *E = ext + ct * esb + (long long)t * T.N + tid;
        const double *O = oj >= 0 ? rs.own.p + ct * rs.own.ct_stride + (long long)t * T.N + tid : nullptr;
        const double *C0 = wsum ? rs.c0 + ct * rs.c0_ct + (long long)t * T.N + tid : nullptr;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
            for (int j = 0; j < BETA; ++j) w[s][j] = (j == oj ? O : E + j * esj)[sbo[s]];
            w[s][BETA] = wsum ? C0[sbo[s]] : 0.0;
        }
    };
    fetch(0);
    for (int ct = 0; ct < cnt; ++ct) {
        const int buf = ct & 1;
        double *L = &sw[buf][0][0][0];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int q = 0; q < NQ; ++q) L[(s * NQ + q) * 256 + tid] = w[s][q];
        __syncthreads();
        if (ct + 1 < cnt) fetch(ct + 1);
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int o = so[r] + (so[r] >> 8) * (NQ - 1) * 256;  // slot s -> (s NQ + j) 256
#pragma unroll
            for (int j = 0; j < BETA; ++j) {
                const double e = L[o + j * 256];
                s0 += mm(e, k0[r][j], p, pinv);
                s1 += mm(e, k1[r][j], p, pinv);
            }
            if ((r + 1) % RK == 0) {
                s0 = red(s0, p, pinv);
                s1 = red(s1, p, pinv);
            }
        }
        acc1[ct * astride + (long long)t * T.N + x] = canon(s1, p, pinv);
        if (wsum) {
            double g0 = rs.c0_id ? L[BETA * 256 + tid] : 0.0;
#pragma unroll
            for (int r = 0; r < NR; ++r) g0 += L[so[r] + (so[r] >> 8) * (NQ - 1) * 256 + BETA * 256];
            s0 = c0_sum(rs, true, g0, s0, ct, t, x, T.N, p, pinv);
        }
        acc0[ct * astride + (long long)t * T.N + x] = canon(s0, p, pinv);
    }
}

// The key products of rotations of different ciphertexts summed in one pass (the giant
// steps of a bootstrap linear transform, whose rotated parts share one ModDown): rotation
// r gathers its own extended digits rs.ext_r[r] and c0 rs.c0_r[r]; otherwise as
// k_inner_product_rot (at most 7 rotations: the partial sums stay below 2^51.6 with one
// reduction per floor(21 / beta) rotations).
template <int BETA>
__global__ __launch_bounds__(256) void k_inner_product_multi(DevTables T, long long esb, long long esj,
                                                             double *__restrict__ acc0, double *__restrict__ acc1,
                                                             long long astride, RotSet rs, int betaL, int cnt,
                                                             int next, const int *__restrict__ ext_prime,
                                                             int xblocks) {
    const int b = blockIdx.x, slot = b >> 3;
    const int t = (b & 7) + 8 * (slot / xblocks);
    if (t >= next) return;
    const int x = rs.xorder[slot % xblocks] * blockDim.x + threadIdx.x;
    if (x >= T.N) return;
    const int pt = ext_prime[t];
    const double p = T.p[pt], pinv = T.pinv[pt];
    const int rk = 21 / BETA;
    const bool wsum = rs.c0_r[0] && t <= rs.lq;
    for (int ct = 0; ct < cnt; ++ct) {
        double s0 = 0.0, s1 = 0.0, g0 = 0.0;
        for (int r = 0; r < rs.nr; ++r) {
            const unsigned src = aut_src((unsigned)x, rs.g[r], T.logN);
            const double *E = rs.ext_r[r] + ct * esb + (long long)t * T.N;
            if (wsum) g0 = red(g0 + rs.c0_r[r][ct * rs.c0_ct + (long long)t * T.N + src], p, pinv);
            const KeyRef K = rs.key[r];
            double e[BETA], a0[BETA], a1[BETA];
#pragma unroll
            for (int j = 0; j < BETA; ++j) {
                e[j] = E[j * esj + src];
                key_pair(K, T, betaL, pt, j, T.N, x, a0[j], a1[j]);
            }
#pragma unroll
            for (int j = 0; j < BETA; ++j) {
                s0 += mm(e[j], a0[j], p, pinv);
                s1 += mm(e[j], a1[j], p, pinv);
            }
            if ((r + 1) % rk == 0) {
                s0 = red(s0, p, pinv);
                s1 = red(s1, p, pinv);
            }
        }
        acc0[ct * astride + (long long)t * T.N + x] = canon(s0, p, pinv);
        acc1[ct * astride + (long long)t * T.N + x] = canon(s1, p, pinv);
        if (wsum) rs.s0[ct * rs.s0_ct + (long long)t * T.N + x] = canon(g0, p, pinv);
    }
}

void launch_inner_product_rot(const DevTables &T, const double *ext, long long estride_b, long long estride_j,
                              double *acc0, double *acc1, long long astride, const RotSet &rs, int betaL,
                              int cnt, int beta, int next, const int *ext_prime, hipStream_t s) {
    if (cnt <= 0) return;
    if (rs.multi) {
        kprof_set_bytes(T.N * (beta * rs.nr * key_row_bytes(T, next) + 8.0 * next * cnt * (beta * rs.nr + 2.0)));
        const int xblocks = (T.N + 255) / 256;
        const dim3 g1(8 * ((next + 7) / 8) * xblocks);
#define IPM_CASE(B)                                                                                            \
    case B:                                                                                                    \
        KL("k_inner_product_multi", k_inner_product_multi<B>, g1, dim3(256), 0, s, T, estride_b, estride_j, acc0, \
           acc1, astride, rs, betaL, cnt, next, ext_prime, xblocks);                                           \
        break;
        switch (beta) { IPM_CASE(1) IPM_CASE(2) IPM_CASE(3) IPM_CASE(4) IPM_CASE(5) IPM_CASE(6) IPM_CASE(7) IPM_CASE(8) }
#undef IPM_CASE
        return;
    }
    // every rotation's key words once; the extended digits and both accumulators
    // once per ciphertext
    kprof_set_bytes(T.N * (beta * rs.nr * key_row_bytes(T, next) + 8.0 * next * cnt * (beta + 2.0)));
    const int xblocks = (T.N + 255) / 256;
    const dim3 g1(8 * ((next + 7) / 8) * xblocks);
    // a step whose Galois elements take at most one residue h != 1 mod N/128 reads its
    // sources from at most two blocks per output block (staged in LDS)
    if (T.logN >= 9 && beta <= 3 && (rs.nr == 7 || rs.nr == 3)) {
        const uint32_t rm = (uint32_t)(T.N / 128);
        uint32_t h = 0, gh = 1, smask = 0;
        bool two = true;
        for (int r = 0; r < rs.nr && two; ++r) {
            const uint32_t res = rs.g[r] % rm;
            if (res == 1u) continue;
            if (h == 0u) {
                h = res;
                gh = rs.g[r];
            }
            if (res != h) two = false;
            smask |= 1u << r;
        }
        if (two) {
#define IPL(R, B, S)                                                                                             \
    if (rs.nr == R && beta == B && (h ? 2 : 1) == S) {                                                           \
        KL("k_inner_product_rot", (k_inner_product_rot_lds<R, B, S>), g1, dim3(256), 0, s, T, ext, estride_b,     \
           estride_j, acc0, acc1, astride, rs, betaL, cnt, next, ext_prime, xblocks, gh, smask);                  \
        return;                                                                                                  \
    }
            IPL(7, 3, 1) IPL(7, 3, 2) IPL(7, 2, 1) IPL(7, 2, 2) IPL(7, 1, 1) IPL(7, 1, 2)
            IPL(3, 3, 1) IPL(3, 3, 2) IPL(3, 2, 1) IPL(3, 2, 2) IPL(3, 1, 1) IPL(3, 1, 2)
#undef IPL
        }
    }
    // a batch holds the step's key words in registers; one ciphertext is bound by the key
    // stream alone, and the lighter kernel keeps more loads in flight
    const bool reg = cnt >= 2 && beta <= 3 && (rs.nr == 7 || rs.nr == 3 || rs.nr == 1);
#define IPR_REG(R, B)                                                                                            \
    if (reg && rs.nr == R && beta == B) {                                                                        \
        KL("k_inner_product_rot", (k_inner_product_rot_reg<R, B>), g1, dim3(256), 0, s, T, ext, estride_b,        \
           estride_j, acc0, acc1, astride, rs, betaL, cnt, next, ext_prime, xblocks);                            \
        return;                                                                                                  \
    }
    IPR_REG(7, 3) IPR_REG(7, 2) IPR_REG(7, 1) IPR_REG(3, 3) IPR_REG(3, 2) IPR_REG(3, 1) IPR_REG(1, 3)
    IPR_REG(1, 2) IPR_REG(1, 1)
#undef IPR_REG
#define IPR(B, R)                                                                                                \
    if (beta == B && (R == 0 || (rs.nr == R && cnt == 1))) {                                                     \
        KL("k_inner_product_rot", (k_inner_product_rot<B, R>), g1, dim3(256), 0, s, T, ext, estride_b, estride_j, \
           acc0, acc1, astride, rs, betaL, cnt, beta, next, ext_prime, xblocks);                                 \
        return;                                                                                                  \
    }
    IPR(3, 7) IPR(2, 7) IPR(1, 7) IPR(3, 3) IPR(2, 3) IPR(1, 3) IPR(3, 1) IPR(2, 1) IPR(1, 1)
    IPR(3, 0) IPR(2, 0) IPR(1, 0)
#undef IPR
    KL("k_inner_product_rot", (k_inner_product_rot<0, 0>), g1, dim3(256), 0, s, T, ext, estride_b, estride_j, acc0,
       acc1, astride, rs, betaL, cnt, beta, next, ext_prime, xblocks);
}

// ---------------------------------------------------------------- sampling
// Philox4x32-10 (Salmon et al., SC 2011), counter (i, prime, obj, attempt).
DEV void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        const uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// uniform residues mod prime(gprime[r]) per vector; coefficient domain
__global__ void k_sample_uniform(VecSet out, uint64_t seed, uint32_t obj, const int *gprime,
                                 DevTables T) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T.N) return;
    double *po; int pr, g, r;
    vs_at(out, blockIdx.y, T.N, po, pr, g, r);
    const int gp = gprime ? gprime[r] : pr;
    const uint64_t q = (uint64_t)T.p[pr];
    const int b = 64 - __clzll((long long)q);
    double val = 0.0;
    for (uint32_t att = 0; att < 4096u; ++att) {
        uint32_t o[4];
        philox((uint32_t)x, (uint32_t)gp, obj, att, (uint32_t)seed, (uint32_t)(seed >> 32), o);
        const uint64_t x0 = ((((uint64_t)o[1]) << 32) | o[0]) >> (64 - b);
        if (x0 < q) { val = (double)x0; break; }
        const uint64_t x1 = ((((uint64_t)o[3]) << 32) | o[2]) >> (64 - b);
        if (x1 < q) { val = (double)x1; break; }
    }
    po[x] = val;
}
void launch_sample_uniform(const DevTables &T, const VecSet &out, uint64_t seed, uint32_t obj,
                           const int *gprime, hipStream_t s) {
    if (out.count <= 0) return;
    KL("k_sample_uniform", k_sample_uniform, ew_grid(T, out.count), dim3(256), 0, s, out, seed, obj, gprime, T);
}

// kind 0: ternary ((o0*3)>>32) - 1; kind 1: centred binomial eta = 21
__global__ void k_sample_small(int *out, int N, uint64_t seed, uint32_t obj, int kind) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    uint32_t o[4];
    philox((uint32_t)x, 0u, obj, 0u, (uint32_t)seed, (uint32_t)(seed >> 32), o);
    if (kind == 0) out[x] = (int)(((uint64_t)o[0] * 3ull) >> 32) - 1;
    else out[x] = __popc(o[0] & 0x1FFFFFu) - __popc(o[1] & 0x1FFFFFu);
}
void launch_sample_small(int *out, int N, uint64_t seed, uint32_t obj, int kind, hipStream_t s) {
    KL("k_sample_small", k_sample_small, dim3((N + 255) / 256), dim3(256), 0, s, out, N, seed, obj, kind);
}

__global__ void k_small_to_res(VecSet out, const int *v, DevTables T) {
    EW_PROLOGUE
    const double pinv = T.pinv[pr];
    po[x] = canon((double)v[x], p, pinv);
}
void launch_small_to_res(const DevTables &T, const VecSet &out, const int *v, const int *gprime,
                         hipStream_t s) {
    (void)gprime;
    if (out.count <= 0) return;
    KL("k_small_to_res", k_small_to_res, ew_grid(T, out.count), dim3(256), 0, s, out, v, T);
}

// int64 coefficients -> residues: m = hi 2^32 + lo
__global__ void k_int64_to_res(VecSet out, const int64_t *m, long long mstride, DevTables T) {
    EW_PROLOGUE
    const double pinv = T.pinv[pr];
    const int64_t v = m[g * mstride + x];
    const double hi = (double)(v >> 32);
    const double lo = (double)(uint32_t)(v & 0xffffffffll);
    po[x] = canon(mm(hi, T.two32[pr], p, pinv) + lo, p, pinv);
}
void launch_int64_to_res(const DevTables &T, const VecSet &out, const int64_t *m,
                         long long mstride, const int *gprime, hipStream_t s) {
    (void)gprime;
    if (out.count <= 0) return;
    KL("k_int64_to_res", k_int64_to_res, ew_grid(T, out.count), dim3(256), 0, s, out, m, mstride, T);
}

// key digit: b = e - a s + [lo <= prime < hi] (P mod q) s'   (NTT domain)
__global__ void k_keyb(DevTables T, double *b, const double *a, const double *e, const double *s,
                       const double *tgt, const double *pmod, int lo, int hi) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T.N) return;
    const int pi = blockIdx.y;
    const double p = T.p[pi], pinv = T.pinv[pi];
    const long long o = (long long)pi * T.N + x;
    double r = e[o] - mm(a[o], s[o], p, pinv);
    if (pi >= lo && pi < hi) r += mm(pmod[pi], tgt[o], p, pinv);
    b[o] = canon(r, p, pinv);
}
void launch_keyb(const DevTables &T, double *b, const double *a, const double *e, const double *s,
                 const double *tgt, const double *pmod, int np, int lo, int hi, hipStream_t st) {
    KL("k_keyb", k_keyb, dim3((T.N + 255) / 256, np), dim3(256), 0, st, T, b, a, e, s, tgt, pmod, lo, hi);
}

// c0 = m + e - a s per (ciphertext, limb)
__global__ void k_encfinish(DevTables T, double *c0, const double *a, const double *e,
                            const double *m, const double *s, int limbs, long long ctstride,
                            long long mctstride) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T.N) return;
    const int ct = blockIdx.y / limbs, li = blockIdx.y % limbs;
    const double p = T.p[li], pinv = T.pinv[li];
    const long long o = (long long)li * T.N + x;
    const double r = m[ct * mctstride + o] + e[o] - mm(a[ct * ctstride + o], s[o], p, pinv);
    c0[ct * ctstride + o] = canon(r, p, pinv);
}
void launch_encfinish(const DevTables &T, double *c0, const double *a, const double *e,
                      const double *m, const double *s, long long stride, int limbs, int cnt,
                      long long ctstride, long long mctstride, hipStream_t st) {
    (void)stride;
    KL("k_encfinish", k_encfinish, dim3((T.N + 255) / 256, cnt * limbs), dim3(256), 0, st, T, c0, a,
                       e, m, s, limbs, ctstride, mctstride);
}

// m = c0 + c1 s on the first `limbs` primes
__global__ void k_decmul(DevTables T, double *m, const double *c0, const double *c1, const double *s) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T.N) return;
    const int li = blockIdx.y;
    const double p = T.p[li], pinv = T.pinv[li];
    const long long o = (long long)li * T.N + x;
    m[o] = canon(c0[o] + mm(c1[o], s[o], p, pinv), p, pinv);
}
void launch_decmul(const DevTables &T, double *m, const double *c0, const double *c1,
                   const double *s, int limbs, hipStream_t st) {
    KL("k_decmul", k_decmul, dim3((T.N + 255) / 256, limbs), dim3(256), 0, st, T, m, c0, c1, s);
}

__global__ void k_square_res(DevTables T, double *out, const double *in) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T.N) return;
    const int pi = blockIdx.y;
    const double p = T.p[pi], pinv = T.pinv[pi];
    const long long o = (long long)pi * T.N + x;
    out[o] = canon(mm(in[o], in[o], p, pinv), p, pinv);
}
void launch_square_res(const DevTables &T, double *out, const double *in, int np, hipStream_t st) {
    KL("k_square_res", k_square_res, dim3((T.N + 255) / 256, np), dim3(256), 0, st, T, out, in);
}

}  // namespace he
