// Batched negacyclic NTT / inverse NTT over RNS limbs for gfx950, with an autotuned
// workgroup width and pass-2 twiddle form.
//
// Forward stage s (m = 2^s, t = N/2m) maps (a_j, a_{j+t}) to
// (a_j + w a_{j+t}, a_j - w a_{j+t}) with w = psi^bitrev(m + j/(2t)) (Cooley-Tukey,
// twiddles merged with the negacyclic twist); output position j holds the evaluation
// at psi^(2 bitrev(j) + 1).  The inverse runs the stages in reverse order with the
// Gentleman-Sande butterfly (x, y) -> (x + y, (x - y) w^-1) and multiplies by N^-1
// (or a caller-supplied per-slot constant that includes N^-1) at the end.
//
// N = 2^(2R) is split into two passes of R = 2H stages: pass 1 runs stages 0..R-1
// on the strided sub-problems {r + SUB k}, pass 2 runs stages R..2R-1 on the
// contiguous blocks {b SUB + k} (SUB = 2^R).  A workgroup holds COLS sub-problems;
// each thread holds E = 2^H words of one sub-problem and runs H stages in registers
// on the high bits of k (phase A) and H stages on the low bits (phase B), exchanging
// through LDS once in between.  Global accesses are made directly from registers
// where the layout is coalesced (phase A side in both passes, phase B side in
// pass 1); pass 2's phase B side goes through LDS.  The LDS tile is skewed so that
// both phases are free of bank conflicts: pass 1 word (c, k) at (k + k/E) COLS + c,
// pass 2 at c (SUB + SUB/E) + k + k/E.
//
// Value bounds: canonical inputs; H lazy CT stages grow |x| below 5p < 2^52, then a
// reduction; GS stages reduce the sum every stage; outputs canonical in [0, p).
#include "he_internal.h"

#include <stdexcept>

namespace he {

#define DEV __device__ __forceinline__

DEV double nmm(double a, double b, double p, double pinv) {
    double h = a * b;
    double l = __builtin_fma(a, b, -h);
    double k = __builtin_rint(h * pinv);
    double r = __builtin_fma(-k, p, h);
    return r + l;
}
DEV double nred(double x, double p, double pinv) { return __builtin_fma(-__builtin_rint(x * pinv), p, x); }
DEV double ncanon(double x, double p, double pinv) {
    double r = nred(x, p, pinv);
    return r < 0.0 ? r + p : r;
}

DEV void nvs_at(const VecSet &v, int idx, int N, double *&ptr, int &pr, int &r, int &g) {
    g = idx / v.group;
    r = idx - g * v.group;
    const int sl = v.slot ? v.slot[r] : r;
    pr = v.prime ? v.prime[r] : r;
    ptr = v.base + (long long)g * v.gstride + (long long)sl * N;
}

// PRO / EPI: fused prologue (forward pass 1 loads) and epilogue (forward pass 2
// stores), see NttPro / NttEpi; EPI 4 is the ModDown epilogue (kind 1) followed by the
// inverse NTT's first pass on the output blocks (epi.chain).  TWF (pass 2): the phase-B twiddles are formed from
// two factors instead of read from the full table: with s = 2H + H + sg the stage and
// low = (th << sg) + g < 2^(s - R), the table entry psi^brev(2^s + (b << (s - R)) + low)
// is tw[2^s + (b << (s - R))] * tw[low] (the three index parts occupy disjoint bits, so
// their bit reversals add), a product of one word per row and one of the first 2^(R-1)
// words; the canonical product equals the table word, so both forms give the same
// output word for word.  pm > 0 (pass 2): blocks walk the vectors prime-major (vector
// y -> group y % pm, slot y / pm), so consecutive vectors share a twiddle row and
// re-read it from L2.
template <int H, int COLS, bool PASS2, bool INV, int PRO, int EPI, int TWF>
__global__ __launch_bounds__(COLS *(1 << H)) void k_ntt(VecSet vs, VecSet src, const double *oscale,
                                                        DevTables T, NttPro pro, NttEpi epi, int pm) {
    constexpr int R = 2 * H, E = 1 << H, TPS = 1 << H, SUB = 1 << R, NT = COLS * TPS;
    constexpr int NN = SUB * SUB, S2 = SUB + SUB / E;
    __shared__ double tile[COLS * S2];
    auto lds = [](int c, int k) { return PASS2 ? c * S2 + k + (k >> H) : (k + (k >> H)) * COLS + c; };

    int vy = blockIdx.y;
    if (pm > 0) vy = (vy % pm) * vs.group + vy / pm;
    double *ptr;
    int pr, r_, g_;
    nvs_at(vs, vy, NN, ptr, pr, r_, g_);
    const double *iptr = ptr;
    if (src.base) {
        double *sp;
        int a1, a2, a3;
        nvs_at(src, vy, NN, sp, a1, a2, a3);
        iptr = sp;
    }
    if (PRO == 1) iptr = pro.last + (long long)g_ * pro.l_g;
    const double p = T.p[pr], pinv = T.pinv[pr];
    const double *tw = (INV ? T.itw : T.tw) + (long long)pr * NN;
    const int cb = blockIdx.x, tid = threadIdx.x;
    int c, th;
    if (PASS2) { th = tid % TPS; c = tid / TPS; } else { c = tid % COLS; th = tid / COLS; }
    const int b = cb * COLS + c;
    auto gidx = [cb](int cc, int k) -> long long {
        return PASS2 ? (long long)(cb * COLS + cc) * SUB + k : (long long)(cb * COLS + cc) + (long long)SUB * k;
    };
    constexpr int soff = PASS2 ? R : 0;
    constexpr int NW = (1 << H) - 1;  // twiddles per phase: 2^sg for stage group sg < H
    // every twiddle of both phases is loaded at the start, so no memory round trip
    // is left between the phases or behind the barrier
    double wa[NW], wb[NW];
#pragma unroll
    for (int sg = 0; sg < H; ++sg) {
        const double row = (PASS2 && TWF) ? tw[(1 << (H + sg + soff)) + (b << (H + sg))] : 0.0;
#pragma unroll
        for (int g = 0; g < (1 << sg); ++g) {
            wa[(1 << sg) - 1 + g] = tw[(1 << (sg + soff)) + (PASS2 ? (b << sg) : 0) + g];
            if (PASS2 && TWF) {
                const int low = (th << sg) + g;
                wb[(1 << sg) - 1 + g] = low == 0 ? row : ncanon(nmm(row, tw[low], p, pinv), p, pinv);
            } else {
                wb[(1 << sg) - 1 + g] = tw[(1 << (H + sg + soff)) + (PASS2 ? (b << (H + sg)) : 0) + (th << sg) + g];
            }
        }
    }
    double v[E];
    constexpr int EW = SUB / TPS;  // words per thread in the coalesced epilogue

    if (!INV) {
        // phase A (high bits of k), loaded straight from global memory
        if (PRO == 1) {
            const double hq = 0.5 * (pro.ql - 1.0);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                double x = iptr[gidx(c, th + TPS * e)];
                x = x > hq ? x - pro.ql : x;
                v[e] = ncanon(x, p, pinv);
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = iptr[gidx(c, th + TPS * e)];
        }
#pragma unroll
        for (int sg = 0; sg < H; ++sg) {
            const int hd = E >> (sg + 1);
#pragma unroll
            for (int g = 0; g < (1 << sg); ++g) {
                const double w = wa[(1 << sg) - 1 + g];
#pragma unroll
                for (int i = 0; i < hd; ++i) {
                    const int e0 = g * 2 * hd + i, e1 = e0 + hd;
                    const double t = nmm(v[e1], w, p, pinv);
                    v[e1] = v[e0] - t;
                    v[e0] = v[e0] + t;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) tile[lds(c, th + TPS * e)] = nred(v[e], p, pinv);
        __syncthreads();
        // epilogue operands, in flight while phase B computes
        double ex[EPI ? EW : 1], es[(EPI == 1 || EPI == 3 || EPI == 4) ? EW : 1];
        long long rN = 0;
        if (EPI) {
            rN = (long long)r_ * NN;
            const double *in = epi.in + (long long)g_ * epi.i_g + rN;
            const int ect = epi.poly1 ? g_ : g_ >> 1, epl = epi.poly1 ? 1 : g_ & 1;
            const bool use1 = epi.add1 && ((epi.m1 >> epl) & 1);
            const bool use2 = epi.add2 && ((epi.m2 >> epl) & 1);
            const double *ad1 = use1 ? epi.add1 + (long long)ect * epi.a1_ct + epl * epi.a1_poly + rN : nullptr;
            const double *ad2 = use2 ? epi.add2 + (long long)ect * epi.a2_ct + epl * epi.a2_poly + rN : nullptr;
#pragma unroll
            for (int i = 0; i < EW; ++i) {
                const int idx = tid + NT * i, k = idx % SUB, cc = idx / SUB;
                const long long j = gidx(cc, k);
                ex[i] = in[j];
                if (EPI == 1 || EPI == 4) es[i] = (use1 ? ad1[j] : 0.0) + (use2 ? ad2[j] : 0.0);
                if (EPI == 3) es[i] = use1 ? ad1[j] : 0.0;
            }
        }
        // phase B (low bits of k)
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = tile[lds(c, th * E + e)];
#pragma unroll
        for (int sg = 0; sg < H; ++sg) {
            const int hd = E >> (sg + 1);
#pragma unroll
            for (int g = 0; g < (1 << sg); ++g) {
                const double w = wb[(1 << sg) - 1 + g];
#pragma unroll
                for (int i = 0; i < hd; ++i) {
                    const int e0 = g * 2 * hd + i, e1 = e0 + hd;
                    const double t = nmm(v[e1], w, p, pinv);
                    v[e1] = v[e0] - t;
                    v[e0] = v[e0] + t;
                }
            }
        }
        if (!PASS2) {
#pragma unroll
            for (int e = 0; e < E; ++e) ptr[gidx(c, th * E + e)] = ncanon(v[e], p, pinv);
        } else {
            // each thread rewrites only the tile words it read in phase B
#pragma unroll
            for (int e = 0; e < E; ++e) tile[lds(c, th * E + e)] = ncanon(v[e], p, pinv);
            __syncthreads();
            if (EPI == 0) {
#pragma unroll
                for (int i = 0; i < EW; ++i) {
                    const int idx = tid + NT * i, k = idx % SUB, cc = idx / SUB;
                    ptr[gidx(cc, k)] = tile[lds(cc, k)];
                }
            } else {
                const double cst = epi.cst[r_];
                const double cst2 = EPI == 3 ? epi.cst2[r_] : 0.0;
                double *out = epi.out + (long long)g_ * epi.o_g + rN;
                const double km = (EPI == 2 && epi.kmul) ? epi.kmul[(long long)(g_ >> 1) * epi.kstride + r_] : 1.0;
#pragma unroll
                for (int i = 0; i < EW; ++i) {
                    const int idx = tid + NT * i, k = idx % SUB, cc = idx / SUB;
                    const double w = tile[lds(cc, k)];
                    double x = ex[i];
                    if (EPI == 2 && epi.kmul) x = nmm(x, km, p, pinv);
                    double o = nmm(x - w, cst, p, pinv);
                    if (EPI == 1 || EPI == 4) o += es[i];
                    if (EPI == 3) o += nmm(es[i], cst2, p, pinv);
                    const double oc = ncanon(o, p, pinv);
                    out[gidx(cc, k)] = oc;
                    if (EPI == 4) tile[lds(cc, k)] = oc;  // the word this thread read
                }
                if (EPI == 4) {
                    // the inverse NTT's first pass on the output blocks (as the inverse
                    // kernel's pass over contiguous blocks runs it, full twiddle table)
                    const double *itw = T.itw + (long long)pr * NN;
#pragma unroll
                    for (int sg = 0; sg < H; ++sg) {
#pragma unroll
                        for (int g = 0; g < (1 << sg); ++g) {
                            wa[(1 << sg) - 1 + g] = itw[(1 << (sg + soff)) + (b << sg) + g];
                            wb[(1 << sg) - 1 + g] = itw[(1 << (H + sg + soff)) + (b << (H + sg)) + (th << sg) + g];
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] = tile[lds(c, th * E + e)];
#pragma unroll
                    for (int sg = H - 1; sg >= 0; --sg) {
                        const int hd = E >> (sg + 1);
#pragma unroll
                        for (int g = 0; g < (1 << sg); ++g) {
                            const double w = wb[(1 << sg) - 1 + g];
#pragma unroll
                            for (int i = 0; i < hd; ++i) {
                                const int e0 = g * 2 * hd + i, e1 = e0 + hd;
                                const double x = v[e0], y = v[e1];
                                v[e0] = nred(x + y, p, pinv);
                                v[e1] = nmm(x - y, w, p, pinv);
                            }
                        }
                    }
                    // each thread rewrites only the tile words it read
#pragma unroll
                    for (int e = 0; e < E; ++e) tile[lds(c, th * E + e)] = nred(v[e], p, pinv);
                    __syncthreads();
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] = tile[lds(c, th + TPS * e)];
#pragma unroll
                    for (int sg = H - 1; sg >= 0; --sg) {
                        const int hd = E >> (sg + 1);
#pragma unroll
                        for (int g = 0; g < (1 << sg); ++g) {
                            const double w = wa[(1 << sg) - 1 + g];
#pragma unroll
                            for (int i = 0; i < hd; ++i) {
                                const int e0 = g * 2 * hd + i, e1 = e0 + hd;
                                const double x = v[e0], y = v[e1];
                                v[e0] = nred(x + y, p, pinv);
                                v[e1] = nmm(x - y, w, p, pinv);
                            }
                        }
                    }
                    double *cp = epi.chain + (long long)g_ * epi.ch_g + rN;
#pragma unroll
                    for (int e = 0; e < E; ++e) cp[gidx(c, th + TPS * e)] = ncanon(v[e], p, pinv);
                }
            }
        }
    } else {
        // phase B first (low bits), stages descending
        if (PASS2 && PRO == 2) {
            // the tensor of the two ciphertexts at this limb; d2 is transformed
            const double *A = pro.ta + (long long)g_ * pro.ta_ct + (long long)r_ * NN;
            const double *B = pro.tb + (long long)(pro.tmap ? pro.tmap[g_] : g_) * pro.tb_ct + (long long)r_ * NN;
            double *D = pro.td + (long long)g_ * pro.td_ct + (long long)r_ * NN;
#pragma unroll
            for (int i = 0; i < EW; ++i) {
                const int idx = tid + NT * i, k = idx % SUB, cc = idx / SUB;
                const long long j = gidx(cc, k);
                const double a0 = A[j], a1 = A[pro.ta_poly + j], b0 = B[j], b1 = B[pro.tb_poly + j];
                const double d2 = ncanon(nmm(a1, b1, p, pinv), p, pinv);
                D[j] = ncanon(nmm(a0, b0, p, pinv), p, pinv);
                D[pro.td_poly + j] = ncanon(nmm(a0, b1, p, pinv) + nmm(a1, b0, p, pinv), p, pinv);
                D[2 * pro.td_poly + j] = d2;
                tile[lds(cc, k)] = d2;
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = tile[lds(c, th * E + e)];
        } else if (PASS2) {
#pragma unroll
            for (int i = 0; i < EW; ++i) {
                const int idx = tid + NT * i, k = idx % SUB, cc = idx / SUB;
                tile[lds(cc, k)] = iptr[gidx(cc, k)];
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = tile[lds(c, th * E + e)];
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = iptr[gidx(c, th * E + e)];
        }
#pragma unroll
        for (int sg = H - 1; sg >= 0; --sg) {
            const int hd = E >> (sg + 1);
#pragma unroll
            for (int g = 0; g < (1 << sg); ++g) {
                const double w = wb[(1 << sg) - 1 + g];
#pragma unroll
                for (int i = 0; i < hd; ++i) {
                    const int e0 = g * 2 * hd + i, e1 = e0 + hd;
                    const double x = v[e0], y = v[e1];
                    v[e0] = nred(x + y, p, pinv);
                    v[e1] = nmm(x - y, w, p, pinv);
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) tile[lds(c, th * E + e)] = nred(v[e], p, pinv);
        __syncthreads();
        // phase A (high bits), stages descending, stored straight to global memory
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = tile[lds(c, th + TPS * e)];
#pragma unroll
        for (int sg = H - 1; sg >= 0; --sg) {
            const int hd = E >> (sg + 1);
#pragma unroll
            for (int g = 0; g < (1 << sg); ++g) {
                const double w = wa[(1 << sg) - 1 + g];
#pragma unroll
                for (int i = 0; i < hd; ++i) {
                    const int e0 = g * 2 * hd + i, e1 = e0 + hd;
                    const double x = v[e0], y = v[e1];
                    v[e0] = nred(x + y, p, pinv);
                    v[e1] = nmm(x - y, w, p, pinv);
                }
            }
        }
        if (!PASS2) {
            const double ni = oscale ? oscale[r_] : T.ninv[pr];
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = nmm(v[e], ni, p, pinv);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) ptr[gidx(c, th + TPS * e)] = ncanon(v[e], p, pinv);
    }
}

// The forward NTT's first pass on one vector's E words held by a thread (canonical,
// at positions c + SUB (th + TPS e) of its COLS-column block): H stages in registers,
// the exchange through the tile, H stages, stored at X[SUB (th E + e)] (X = the
// vector's column c).  Word for word the pass k_ntt runs.  Contains one barrier; the
// caller separates consecutive uses of the tile with another.
template <int H, int COLS>
DEV void pass1_words(double (&x)[1 << H], const double *tw, double p, double pinv, double *tile, int c, int th,
                     double *X) {
    constexpr int E = 1 << H, TPS = 1 << H, SUB = 1 << (2 * H), NW = (1 << H) - 1;
    auto lds = [](int cc, int k) { return (k + (k >> H)) * COLS + cc; };
    double wa[NW], wb[NW];
#pragma unroll
    for (int sg = 0; sg < H; ++sg) {
#pragma unroll
        for (int g = 0; g < (1 << sg); ++g) {
            wa[(1 << sg) - 1 + g] = tw[(1 << sg) + g];
            wb[(1 << sg) - 1 + g] = tw[(1 << (H + sg)) + (th << sg) + g];
        }
    }
#pragma unroll
    for (int sg = 0; sg < H; ++sg) {
        const int hd = E >> (sg + 1);
#pragma unroll
        for (int g = 0; g < (1 << sg); ++g) {
            const double w = wa[(1 << sg) - 1 + g];
#pragma unroll
            for (int i = 0; i < hd; ++i) {
                const int e0 = g * 2 * hd + i, e1 = e0 + hd;
                const double u = nmm(x[e1], w, p, pinv);
                x[e1] = x[e0] - u;
                x[e0] = x[e0] + u;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) tile[lds(c, th + TPS * e)] = nred(x[e], p, pinv);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = tile[lds(c, th * E + e)];
#pragma unroll
    for (int sg = 0; sg < H; ++sg) {
        const int hd = E >> (sg + 1);
#pragma unroll
        for (int g = 0; g < (1 << sg); ++g) {
            const double w = wb[(1 << sg) - 1 + g];
#pragma unroll
            for (int i = 0; i < hd; ++i) {
                const int e0 = g * 2 * hd + i, e1 = e0 + hd;
                const double u = nmm(x[e1], w, p, pinv);
                x[e1] = x[e0] - u;
                x[e0] = x[e0] + u;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) X[(long long)SUB * (th * E + e)] = ncanon(x[e], p, pinv);
}

// ModUp fused into the first pass of the forward NTT of the extended digits.  For
// digit j of ciphertext ct the converted slots are t in [0, lo) u [lo + dl, next); the
// k-th of them is t = k < lo ? k : k + dl.  A workgroup takes COLS columns of the
// first pass (positions c + SUB k, the strided sub-problems) of one (ct, j) and TB
// consecutive converted slots: each thread loads the dl coefficient-domain digit words
// v_a of its E positions once, centres them, accumulates sum_a v~_a [Qhat_a]_{prime(t)}
// for its TB targets (the basis conversion, as k_modup), and runs the pass's stages on
// each target in turn, storing the pass's output; the second pass is the ordinary one.
// The arithmetic is that of k_modup followed by the first pass, word for word.  The
// grid is XCD-aware as the other basis conversions (target blocks of one column block
// consecutive on one XCD, so the digit words are re-read from its L2).
template <int H, int COLS, int DL, int TB>
__global__ __launch_bounds__(COLS *(1 << H)) void k_modup_ntt(DevTables T, const double *__restrict__ v,
                                                               long long vstride, double *__restrict__ ext,
                                                               long long esb, long long esj, int beta, int next,
                                                               const int *__restrict__ ext_prime, ModUpDigits dg,
                                                               int ntb, int cblk, int nz) {
    constexpr int R = 2 * H, E = 1 << H, TPS = 1 << H, SUB = 1 << R, NT = COLS * TPS;
    constexpr int NN = SUB * SUB, S2 = SUB + SUB / E;
    __shared__ double tile[COLS * S2];
    __shared__ double sq[DL * TB];
    __shared__ double sp[TB], si[TB];
    __shared__ int spt[TB];
    ConvIdx ix;
    if (!conv_idx(blockIdx.x, ntb, cblk, nz, ix)) return;  // uniform over the workgroup
    const int ct = ix.z / beta, j = ix.z - (ix.z / beta) * beta;
    const int lo = dg.lo[j], dl = dg.dl[j], ncv = next - dl, k0 = ix.tb * TB;
    if (k0 >= ncv) return;  // uniform
    const int tid = threadIdx.x;
    {
        const double *qh = dg.qhat[j];
        for (int i = tid; i < DL * TB; i += NT) {
            const int a = i / TB, kk = k0 + (i - (i / TB) * TB);
            const int t = kk < lo ? kk : kk + dl;
            sq[i] = (a < dl && kk < ncv) ? qh[a * next + t] : 0.0;
        }
        if (tid < TB) {
            const int kk = k0 + tid, t = kk < lo ? kk : kk + dl;
            const int pt = ext_prime[kk < ncv ? t : 0];
            sp[tid] = T.p[pt];
            si[tid] = T.pinv[pt];
            spt[tid] = pt;
        }
    }
    __syncthreads();
    const int c = tid % COLS, th = tid / COLS;
    const long long col = (long long)ix.cb * COLS + c;
    // the digit words as centred representatives, the conversion of every target
    double acc[TB][E];
#pragma unroll
    for (int tt = 0; tt < TB; ++tt)
#pragma unroll
        for (int e = 0; e < E; ++e) acc[tt][e] = 0.0;
    const double *vp = v + ct * vstride + (long long)lo * NN + col;
#pragma unroll
    for (int a = 0; a < DL; ++a) {
        if (a < dl) {
            const double qa = T.p[lo + a];
            double w[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double u = vp[(long long)a * NN + (long long)SUB * (th + TPS * e)];
                w[e] = u > 0.5 * (qa - 1.0) ? u - qa : u;
            }
#pragma unroll
            for (int tt = 0; tt < TB; ++tt)
#pragma unroll
                for (int e = 0; e < E; ++e) acc[tt][e] += nmm(w[e], sq[a * TB + tt], sp[tt], si[tt]);
        }
    }
#pragma unroll
    for (int tt = 0; tt < TB; ++tt) {
        const int kk = k0 + tt;
        if (kk >= ncv) break;  // uniform
        const int t = kk < lo ? kk : kk + dl;
        const double p = sp[tt], pinv = si[tt];
        double x[E];
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = ncanon(acc[tt][e], p, pinv);
        if (tt > 0) __syncthreads();  // the previous target's tile reads are done
        pass1_words<H, COLS>(x, T.tw + (long long)spt[tt] * NN, p, pinv, tile, c, th,
                             ext + ct * esb + j * esj + (long long)t * NN + col);
    }
}

// ModDown conversion fused into the first pass of the forward NTT of its output: the
// centred lift of the md.nin input limbs of group z (|w| <= p_m / 2), converted to every
// target q_i, i < md.ntgt (|sum| <= AL (p/2 + 2^44) < 2^52 for AL <= 16), then the
// pass, on the grid and with the TB-target blocks of k_modup_ntt.
template <int H, int COLS, int AL, int TB>
__global__ __launch_bounds__(COLS *(1 << H)) void k_moddown_ntt(DevTables T, const double *__restrict__ acc,
                                                                 long long astride, double *__restrict__ conv,
                                                                 long long cstride, MdIn md, int ntb, int cblk,
                                                                 int nz) {
    constexpr int R = 2 * H, E = 1 << H, TPS = 1 << H, SUB = 1 << R, NT = COLS * TPS;
    constexpr int NN = SUB * SUB, S2 = SUB + SUB / E;
    __shared__ double tile[COLS * S2];
    __shared__ double sq[AL * TB];
    __shared__ double sp[TB], si[TB];
    ConvIdx ix;
    if (!conv_idx(blockIdx.x, ntb, cblk, nz, ix)) return;  // uniform over the workgroup
    const int i0 = ix.tb * TB;
    if (i0 >= md.ntgt) return;  // uniform
    const int tid = threadIdx.x;
    for (int k = tid; k < AL * TB; k += NT) {
        const int m = k / TB, i = i0 + (k - (k / TB) * TB);
        sq[k] = (m < md.nin && i < md.ntgt) ? md.ph[m * md.phs + i] : 0.0;
    }
    if (tid < TB) {
        const int i = i0 + tid < md.ntgt ? i0 + tid : 0;
        sp[tid] = T.p[i];
        si[tid] = T.pinv[i];
    }
    __syncthreads();
    const int c = tid % COLS, th = tid / COLS;
    const long long col = (long long)ix.cb * COLS + c;
    double sacc[TB][E];
#pragma unroll
    for (int ii = 0; ii < TB; ++ii)
#pragma unroll
        for (int e = 0; e < E; ++e) sacc[ii][e] = 0.0;
    const double *Ac = acc + ix.z * astride + (long long)md.in0 * NN + col;
#pragma unroll
    for (int m = 0; m < AL; ++m) {
        if (m < md.nin) {
            const double pm = T.p[md.in_prime[m]];
            double w[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double u = Ac[(long long)m * NN + (long long)SUB * (th + TPS * e)];
                w[e] = u > 0.5 * (pm - 1.0) ? u - pm : u;
            }
#pragma unroll
            for (int ii = 0; ii < TB; ++ii)
#pragma unroll
                for (int e = 0; e < E; ++e) sacc[ii][e] += nmm(w[e], sq[m * TB + ii], sp[ii], si[ii]);
        }
    }
#pragma unroll
    for (int ii = 0; ii < TB; ++ii) {
        const int i = i0 + ii;
        if (i >= md.ntgt) break;  // uniform
        const double p = sp[ii], pinv = si[ii];
        double x[E];
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = ncanon(sacc[ii][e], p, pinv);
        if (ii > 0) __syncthreads();  // the previous target's tile reads are done
        pass1_words<H, COLS>(x, T.tw + (long long)i * NN, p, pinv, tile, c, th,
                             conv + ix.z * cstride + (long long)i * NN + col);
    }
}

// tuned schedule per (log N, batch bucket); 0 = not tuned (use the default).  A
// variant v = 1..NTT_VARIANTS is a workgroup width (the (v - 1) % 3 -th of three) and a
// pass-2 twiddle form ((v - 1) / 3: 0 full table, 1 factored phase-B twiddles).
static int g_ntt_tune[2][8];

static int bucket_of(int count) {
    int b = 0;
    while (b < 7 && (4 << (2 * b)) < count) ++b;  // <=4, <=16, <=64, <=256, <=1024, <=4096, ...
    return b;
}

void set_ntt_tuning(int logN, int bucket, int variant) {
    if (bucket >= 0 && bucket < 8) g_ntt_tune[logN == 16 ? 1 : 0][bucket] = variant;
}

// passes: bit 0 the first pass launched (forward: strided; inverse: contiguous blocks),
// bit 1 the second
template <int H, int COLS, int PRO, int EPI, int TWF>
static void ntt_run(const DevTables &T, const VecSet &vs, const VecSet *src, bool inverse, const double *oscale,
                    const NttPro &pro, const NttEpi &epi, hipStream_t s, int passes) {
    constexpr int SUB = 1 << (2 * H), NT = COLS * (1 << H);
    dim3 grid(SUB / COLS, vs.count), block(NT);
    const VecSet none{nullptr, 0, 1, 0, nullptr, nullptr};
    const VecSet first = src ? *src : none;
    // pass 2 walks the vectors prime-major when they form whole groups
    const int pm = (vs.group > 1 && vs.count % vs.group == 0) ? vs.count / vs.group : 0;
    // algorithmic bytes: a limb-NTT reads and writes every word once (2 N 8 bytes), half
    // of it booked to each pass; a fused prologue reads the shared last limb once per
    // group; a fused epilogue adds its element-wise operands (in, addends)
    const double half = 8.0 * SUB * SUB;
    const double nvec = vs.count, ngrp = (vs.count + vs.group - 1) / vs.group;
    // a prologue or epilogue kind of one direction is not instantiated for the other
    if (inverse ? (EPI != 0 || PRO == 1) : PRO == 2)
        throw std::invalid_argument("ntt: prologue or epilogue kind of the other direction");
    if constexpr (PRO != 2) {
        if (!inverse) {
            if (passes & 1) {
                kprof_set_bytes(half * (PRO ? ngrp : nvec));
                KLN(PRO ? "ntt_fwd_pass1_lift" : "ntt_fwd_pass1", (k_ntt<H, COLS, false, false, PRO, 0, 0>), grid,
                    block, 0, s, vs, first, nullptr, T, pro, epi, 0);
            }
            if (!(passes & 2)) return;
            double extra = 0.0;
            if (EPI) {
                extra = 1.0;  // in
                if ((EPI == 1 || EPI == 4) && epi.add1) extra += __builtin_popcount(epi.m1 & 3) * 0.5;
                if ((EPI == 1 || EPI == 4) && epi.add2) extra += __builtin_popcount(epi.m2 & 3) * 0.5;
                if (EPI == 3) extra += 1.0;
                if (EPI == 4) extra += 0.5;  // the chained pass's output
            }
            kprof_set_bytes(half * nvec * (1.0 + extra));
            KLN(EPI == 4   ? "ntt_fwd_pass2_moddown_chain"
                : EPI == 1 ? "ntt_fwd_pass2_moddown"
                : EPI == 2 ? "ntt_fwd_pass2_rescale"
                : EPI == 3 ? "ntt_fwd_pass2_moddown_rescale"
                           : "ntt_fwd_pass2",
                (k_ntt<H, COLS, true, false, 0, EPI, TWF>), grid, block, 0, s, vs, none, nullptr, T, pro, epi, pm);
            return;
        }
    }
    if constexpr (EPI == 0 && PRO != 1) {
        if (passes & 1) {
            // the tensor prologue reads 4 words and writes 3 besides the pass's output
            kprof_set_bytes(half * nvec * (PRO == 2 ? 8.0 : 1.0));
            KLN(PRO == 2 ? "ntt_inv_pass2_tensor" : "ntt_inv_pass2", (k_ntt<H, COLS, true, true, PRO, 0, TWF>), grid,
                block, 0, s, vs, first, nullptr, T, pro, epi, pm);
        }
        if (!(passes & 2)) return;
        kprof_set_bytes(half * nvec);
        KLN("ntt_inv_pass1", (k_ntt<H, COLS, false, true, 0, 0, 0>), grid, block, 0, s, vs, none, oscale, T, pro,
            epi, 0);
    }
}

template <int PRO, int EPI>
static void ntt_dispatch(const DevTables &T, const VecSet &vs, bool inverse, int variant, hipStream_t s,
                         const VecSet *src, const double *oscale, const NttPro &pro, const NttEpi &epi,
                         int passes = 3) {
    if (vs.count <= 0) return;
    int v = variant;
    if (v <= 0) v = g_ntt_tune[T.logN == 16 ? 1 : 0][bucket_of(vs.count)];
    if (v <= 0 || v > NTT_VARIANTS) v = 3;
    const int w = (v - 1) % 3, f = (v - 1) / 3;
#define NTT_CASE(H, C0, C1, C2)                                                                            \
    if (w == 0 && f == 0) ntt_run<H, C0, PRO, EPI, 0>(T, vs, src, inverse, oscale, pro, epi, s, passes);           \
    else if (w == 1 && f == 0) ntt_run<H, C1, PRO, EPI, 0>(T, vs, src, inverse, oscale, pro, epi, s, passes);      \
    else if (w == 2 && f == 0) ntt_run<H, C2, PRO, EPI, 0>(T, vs, src, inverse, oscale, pro, epi, s, passes);      \
    else if (w == 0) ntt_run<H, C0, PRO, EPI, 1>(T, vs, src, inverse, oscale, pro, epi, s, passes);                \
    else if (w == 1) ntt_run<H, C1, PRO, EPI, 1>(T, vs, src, inverse, oscale, pro, epi, s, passes);                \
    else ntt_run<H, C2, PRO, EPI, 1>(T, vs, src, inverse, oscale, pro, epi, s, passes);
    if (T.logN == 16) {
        NTT_CASE(4, 4, 8, 16)
    } else if (T.logN == 12) {
        NTT_CASE(3, 8, 16, 32)
    }
#undef NTT_CASE
}

void launch_ntt(const DevTables &T, const VecSet &vs, bool inverse, int variant, hipStream_t s,
                const VecSet *src, const double *oscale, bool strided_only) {
    const NttPro pro{};
    const NttEpi epi{};
    if (strided_only && (!inverse || src)) throw std::invalid_argument("strided_only: in-place inverse only");
    ntt_dispatch<0, 0>(T, vs, inverse, variant, s, src, oscale, pro, epi, strided_only ? 2 : 3);
}

void launch_ntt_fwd_pass2(const DevTables &T, const VecSet &vs, int variant, hipStream_t s) {
    ntt_dispatch<0, 0>(T, vs, false, variant, s, nullptr, nullptr, NttPro{}, NttEpi{}, 2);
}

template <int H, int COLS, int TB>
static void modup_ntt_run(int DL, const DevTables &T, const double *v, long long vstride, double *ext, long long esb,
                          long long esj, int cnt, int beta, int next, const int *ext_prime, const ModUpDigits &dg,
                          hipStream_t s) {
    int dmin = next;
    for (int j = 0; j < beta; ++j) dmin = dg.dl[j] < dmin ? dg.dl[j] : dmin;
    const int ntb = (next - dmin + TB - 1) / TB, cblk = (1 << (2 * H)) / COLS, nz = cnt * beta;
    const dim3 grid = conv_grid(ntb, cblk, nz);
#define MN_CASE(D)                                                                                                \
    case D:                                                                                                       \
        KLN("k_modup_ntt", (k_modup_ntt<H, COLS, D, TB>), grid, dim3(COLS << H), 0, s, T, v, vstride, ext, esb, \
            esj, beta, next, ext_prime, dg, ntb, cblk, nz);                                                       \
        break;
    switch (DL) { MN_CASE(4) MN_CASE(8) MN_CASE(10) MN_CASE(12) MN_CASE(16) }
#undef MN_CASE
}

void launch_modup_ntt(const DevTables &T, const double *v, long long vstride, double *ext, long long esb,
                      long long esj, int cnt, int beta, int next, const int *ext_prime, const ModUpDigits &dg,
                      hipStream_t s) {
    if (cnt <= 0) return;
    int dmax = 0;
    for (int j = 0; j < beta; ++j) dmax = dg.dl[j] > dmax ? dg.dl[j] : dmax;
    // the l+1 digit words in, every converted slot (after the first pass) out
    kprof_set_bytes(8.0 * T.N * cnt * ((double)beta * next));
    if (T.logN == 16) modup_ntt_run<4, 16, 2>(digit_len(dmax), T, v, vstride, ext, esb, esj, cnt, beta, next,
                                              ext_prime, dg, s);
    else if (T.logN == 12) modup_ntt_run<3, 32, 2>(digit_len(dmax), T, v, vstride, ext, esb, esj, cnt, beta, next,
                                                   ext_prime, dg, s);
    else throw std::invalid_argument("launch_modup_ntt: log N must be 12 or 16");
}

template <int H, int COLS, int TB>
static void moddown_ntt_run(int AL, const DevTables &T, const double *acc, long long astride, double *conv,
                            long long cstride, int groups, const MdIn &md, hipStream_t s) {
    const int ntb = (md.ntgt + TB - 1) / TB, cblk = (1 << (2 * H)) / COLS;
    const dim3 grid = conv_grid(ntb, cblk, groups);
#define MDN_CASE(D)                                                                                                \
    case D:                                                                                                        \
        KLN("k_moddown_ntt", (k_moddown_ntt<H, COLS, D, TB>), grid, dim3(COLS << H), 0, s, T, acc, astride, conv, \
            cstride, md, ntb, cblk, groups);                                                                       \
        break;
    switch (AL) { MDN_CASE(4) MDN_CASE(8) MDN_CASE(10) MDN_CASE(12) MDN_CASE(16) }
#undef MDN_CASE
}

void launch_moddown_ntt(const DevTables &T, const double *acc, long long astride, double *conv, long long cstride,
                        int groups, const MdIn &md, hipStream_t s) {
    if (groups <= 0) return;
    // the inputs in, every target (after the first pass) out
    kprof_set_bytes(8.0 * T.N * groups * (md.nin + md.ntgt));
    if (T.logN == 16 && groups < 8)
        moddown_ntt_run<4, 16, 1>(digit_len(md.nin), T, acc, astride, conv, cstride, groups, md, s);
    else if (T.logN == 16) moddown_ntt_run<4, 16, 2>(digit_len(md.nin), T, acc, astride, conv, cstride, groups, md, s);
    else if (T.logN == 12) moddown_ntt_run<3, 32, 2>(digit_len(md.nin), T, acc, astride, conv, cstride, groups, md, s);
    else throw std::invalid_argument("launch_moddown_ntt: log N must be 12 or 16");
}

void launch_tensor_intt(const DevTables &T, const VecSet &vs, const NttPro &pro, int variant, hipStream_t s) {
    if (pro.kind != 2) throw std::invalid_argument("launch_tensor_intt: tensor prologue expected");
    ntt_dispatch<2, 0>(T, vs, true, variant, s, nullptr, nullptr, pro, NttEpi{}, 1);
}

void launch_ntt_fused(const DevTables &T, const VecSet &vs, const NttPro &pro, const NttEpi &epi, int variant,
                      hipStream_t s, int passes) {
    if (pro.kind == 1 && epi.kind == 2)
        ntt_dispatch<1, 2>(T, vs, false, variant, s, nullptr, nullptr, pro, epi, passes);
    else if (pro.kind == 0 && epi.kind == 1 && epi.chain)
        ntt_dispatch<0, 4>(T, vs, false, variant, s, nullptr, nullptr, pro, epi, passes);
    else if (pro.kind == 0 && epi.kind == 1)
        ntt_dispatch<0, 1>(T, vs, false, variant, s, nullptr, nullptr, pro, epi, passes);
    else if (pro.kind == 1 && epi.kind == 0)
        ntt_dispatch<1, 0>(T, vs, false, variant, s, nullptr, nullptr, pro, epi, passes);
    else if (pro.kind == 0 && epi.kind == 2)
        ntt_dispatch<0, 2>(T, vs, false, variant, s, nullptr, nullptr, pro, epi, passes);
    else if (pro.kind == 0 && epi.kind == 3)
        ntt_dispatch<0, 3>(T, vs, false, variant, s, nullptr, nullptr, pro, epi, passes);
    else ntt_dispatch<0, 0>(T, vs, false, variant, s, nullptr, nullptr, pro, epi, passes);
}

}  // namespace he
