// Host orchestration of the encrypted CutMax on one MI355X: context and
// device key generation, client encrypt/decrypt, the batched CKKS evaluator
// (hybrid key switching, rescale, rotations) and the CutMax schedule of
// Alg. 2 (arXiv 2509.08383, Sec. 3.2) with its Goldschmidt inverse (App. B.1).
//
// Every call runs twice: a dry pass with kernel launches disabled sizes the
// workspace and records every constant the schedule needs (all host-side, in
// IEEE double, in a fixed order); the constants are uploaded once; the real
// pass replays the same sequence and launches the kernels on the context's
// stream.  Nothing is allocated with hipMalloc between the first and the last
// kernel of a call, so a call can be captured in a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include <thread>
#include <tuple>

#include "../../include/he.h"
#include "boot_plan.h"
#include "he_internal.h"

using namespace he;

namespace he {
struct KProf {
    struct Rec { const char *name; hipEvent_t a, b; double bytes; };
    std::vector<Rec> recs;
    double pending = 0;
};
KProf *g_kprof = nullptr;
void kprof_set_bytes(double b) {
    if (g_kprof) g_kprof->pending = b;
}
void kprof_mark(const char *name, hipStream_t s, bool end) {
    if (!end) {
        KProf::Rec r{name, nullptr, nullptr, g_kprof->pending};
        g_kprof->pending = 0;
        hipEventCreate(&r.a);
        hipEventCreate(&r.b);
        hipEventRecord(r.a, s);
        g_kprof->recs.push_back(r);
    } else {
        hipEventRecord(g_kprof->recs.back().b, s);
    }
}
}  // namespace he

namespace {

thread_local std::string g_err;

struct HeError : std::runtime_error {
    int code;
    HeError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess)                                                                  \
            throw HeError(HE_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));          \
    } while (0)

#define REQUIRE(c, code, msg)                 \
    do {                                      \
        if (!(c)) throw HeError(code, msg);   \
    } while (0)

constexpr uint32_t OBJ_SK = 0x00000001u;
constexpr uint32_t OBJ_SKH = 0x00000002u;  // sparse secret positions
constexpr uint32_t OBJ_KEY_A = 0x01000000u;
constexpr uint32_t OBJ_KEY_E = 0x02000000u;
constexpr uint32_t OBJ_ENC_A = 0x03000000u;
constexpr uint32_t OBJ_ENC_E = 0x04000000u;

// bump allocator for the per-call workspace; dry mode only counts
struct Arena {
    char *base = nullptr;
    size_t cap = 0, top = 0, peak = 0;
    bool dry = true;
    void *alloc(size_t bytes) {
        size_t off = (top + 255) & ~(size_t)255;
        top = off + bytes;
        peak = std::max(peak, top);
        if (dry) return (void *)(uintptr_t)(0x100000 + off);
        if (top > cap) throw HeError(HE_ENOMEM, "workspace overflow");
        return base + off;
    }
    size_t mark() const { return top; }
    void release(size_t m) { top = m; }
};

// constants of one call, recorded in the dry pass and uploaded once
struct Pool {
    std::vector<double> dv;
    std::vector<int> iv;
    size_t dpos = 0, ipos = 0;
    double *d_dv = nullptr;
    int *d_iv = nullptr;
    size_t dcap = 0, icap = 0;
    bool dry = true;
    const double *push(const std::vector<double> &v) {
        size_t off = dpos;
        dpos += v.size();
        if (dry) { dv.insert(dv.end(), v.begin(), v.end()); return (const double *)(uintptr_t)(0x200000 + 8 * off); }
        return d_dv + off;
    }
    const int *push(const std::vector<int> &v) {
        size_t off = ipos;
        ipos += v.size();
        if (dry) { iv.insert(iv.end(), v.begin(), v.end()); return (const int *)(uintptr_t)(0x300000 + 4 * off); }
        return d_iv + off;
    }
};

}  // namespace

// ------------------------------------------------------------------ context
struct he_ctx {
    int logN = 0, N = 0, L = 0, alpha = 0, dnum = 0, np = 0, betaL = 0, slots = 0;
    double Delta = 0;
    uint64_t seed = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<uint64_t> q;
    DevTables T{};
    // device tables (one allocation each)
    double *d_tab = nullptr;
    int *d_itab = nullptr;
    double *d_sk = nullptr;  // [np][N] NTT domain
    std::vector<KeyRef> keys;  // packed 40- and 48-bit words (owned)
    std::vector<int> khb_host;  // per prime: high-part bytes of a key word (1 or 2)
    size_t key_hi_bytes = 0;    // bytes of one key's high plane
    // level-indexed conversion tables (device pointers into d_tab / d_itab)
    std::vector<const int *> ext_prime;                 // [L+1] -> [l+1+alpha]
    std::vector<std::vector<const double *>> vinv, qhat;  // [L+1][beta_l]
    std::vector<std::vector<const int *>> ndslot, ndprime;
    std::vector<std::vector<int>> ndcount;
    std::vector<int> ndall;                              // [L+1]: converted limbs over all digits
    std::vector<const int *> ndall_slot, ndall_prime;    // [L+1] -> [ndall]: j*next + t, prime(t)
    const double *phinv = nullptr, *phat = nullptr, *Pinv = nullptr, *qlinv = nullptr, *pmod = nullptr;
    std::vector<const double *> mu_scale;  // [L+1] -> [l+1]: N^-1 Qhat_i^-1 mod q_i at level l
    const double *md_scale = nullptr;      // [alpha]: N^-1 Phat_m^-1 mod p_m
    // ModDown by P q_l (relinearisation with the rescale folded in), per level l >= 1,
    // basis B = {q_l, p_0, .., p_{alpha-1}}:
    std::vector<const double *> mr_scale;  // [alpha+1]: N^-1 Bhat_b^-1 mod b
    std::vector<const double *> mr_phat;   // [alpha+1][l]: Bhat_b mod q_i
    std::vector<const double *> mr_inv;    // [l]: (P q_l)^-1 mod q_i
    std::vector<double> pmod_h;            // [L+1]: P mod q_i (host copy)
    const int *ident = nullptr;   // 0..np-1
    const int *pprime = nullptr;  // L+1 .. L+alpha
    uint32_t nonce = 0;
    Arena arena;
    Pool pool;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = 0;
    int use_graph = 0;
    int ntt_variant = 0;
    // rotate-and-sum: 0 = one rotation at a time, h = hoisted radix-2^h steps
    int hoist = 0;
    std::map<int, int> rot_key;     // rotation amount -> key index
    std::map<int, const int *> xorder;  // smallest amount of a hoisted step -> x-block orbit order
    const int *xorder_id = nullptr;     // x-blocks in natural order (any rotation)
    int boot_hoist = 2;                 // 1: bootstrap baby steps share one ModUp; 2: also one ModDown per giant-step sum
    size_t ws_limit = 0;                // HE_OPT_WORKSPACE_LIMIT: bytes of workspace a call may use (0: no limit)
    std::vector<uint32_t> key_gal;  // key index -> Galois element (0 for relinearisation)
    // graph cache keyed by a signature of the call
    std::map<std::string, hipGraphExec_t> graphs;
    int n_hi = 0, secret_hw = 0;
    std::map<uint64_t, int> gal_key;  // Galois element -> key index (rotations, conjugation)
    // bootstrapping (he_boot_setup): configuration, the butterfly groups of the two
    // linear transforms, EvalMod's Chebyshev coefficients, and the encoded diagonals
    // (device, NTT domain, built on first use) keyed by (transform, group, giant, term,
    // level, plaintext scale bits, multiplier bits)
    struct Boot {
        bool ready = false;
        int n_cts = 3, n_stc = 3, K = 0, ratio_bits = 12, cheb_deg = 31, r = 3, correct_bits = 0;
        double s_eval = 0;
        std::vector<he::Diag> cts, stc;
        std::vector<he::Bsgs> cts_plan, stc_plan;
    } boot;
    std::map<std::tuple<int, int, int, int, int, uint64_t, uint64_t>, double *> pt_cache;
    double *mono_pos = nullptr, *mono_neg = nullptr;  // +X^(N/2), -X^(N/2): NTT residues [np][N]
};

struct he_ct {
    he_ctx *ctx = nullptr;
    double *d = nullptr;  // [a][2][L+1][N]
    uint32_t a = 1, level = 0;
    double scale = 0;
    size_t n = 0;
    double pad = 0;  // value of the slots beyond n (he_encrypt)
};

namespace {

// batch of ciphertexts advancing together: [cnt][2][cap][N]
struct Bt {
    double *d = nullptr;
    int cnt = 0, level = 0, cap = 0;
    std::vector<double> scale;  // per ciphertext
};

// an addend of the key-switch output: word (ct, poly, limb, j) at
// p + ct * ct_stride + poly * poly_stride + limb N + j, on the polys in mask
struct Addend {
    const double *p;
    long long ct, poly;
    int mask;
};

std::vector<std::vector<int>> hoist_steps(int slots, int h);

struct Exec {
    he_ctx *C;
    bool dry;            // sizing pass: fake addresses, no launches
    bool quiet = false;  // replay pass: real addresses, the kernels come from a captured graph
    hipStream_t s;
    const DevTables &T;
    Exec(he_ctx *c, bool d) : C(c), dry(d), s(c->stream), T(c->T) {}
    bool go() const { return !dry && !quiet; }

    double *alloc_d(size_t words) { return (double *)C->arena.alloc(words * 8); }
    Bt new_bt(int cnt, int level) {
        Bt b;
        b.cnt = cnt; b.level = level; b.cap = level + 1;
        b.d = alloc_d((size_t)cnt * 2 * b.cap * C->N);
        b.scale.assign(cnt, 0.0);
        return b;
    }
    long long N() const { return C->N; }
    VecSet vs_all(const Bt &b) const {
        return VecSet{b.d, b.cnt * 2 * (b.level + 1), b.level + 1, (long long)b.cap * C->N, nullptr, nullptr};
    }
    VecSet vs_poly(const Bt &b, int poly) const {
        return VecSet{b.d + (long long)poly * b.cap * C->N, b.cnt * (b.level + 1), b.level + 1,
                      2LL * b.cap * C->N, nullptr, nullptr};
    }
    // residues of per-ciphertext integers for limbs 0..level: [cnt][level+1]
    const double *residues(const std::vector<int64_t> &k, int level) {
        std::vector<double> v((size_t)k.size() * (level + 1));
        for (size_t c = 0; c < k.size(); ++c)
            for (int i = 0; i <= level; ++i) v[c * (level + 1) + i] = (double)red_i64(k[c], C->q[i]);
        return C->pool.push(v);
    }

    // ------------------------------------------------------------- basic ops
    Bt add(const Bt &a, const Bt &b, int sign = 1) {
        REQUIRE(a.level == b.level && a.cnt == b.cnt, HE_ESTATE, "add: level/count mismatch");
        for (int c = 0; c < a.cnt; ++c)
            REQUIRE(std::fabs(a.scale[c] - b.scale[c]) <= 1e-9 * a.scale[c], HE_ERANGE, "add: scale mismatch");
        Bt o = new_bt(a.cnt, a.level);
        o.scale = a.scale;
        if (go()) launch_add(T, vs_all(o), vs_all(a), vs_all(b), sign, s);
        return o;
    }
    void add_inplace(Bt &a, const Bt &b) {
        REQUIRE(a.level == b.level && a.cnt == b.cnt, HE_ESTATE, "add: level/count mismatch");
        for (int c = 0; c < a.cnt; ++c)
            REQUIRE(std::fabs(a.scale[c] - b.scale[c]) <= 1e-9 * a.scale[c], HE_ERANGE, "add: scale mismatch");
        if (go()) launch_add(T, vs_all(a), vs_all(a), vs_all(b), 1, s);
    }
    Bt copy(const Bt &a) {
        Bt o = new_bt(a.cnt, a.level);
        o.scale = a.scale;
        if (go()) launch_copy(T, vs_all(o), vs_all(a), s);
        return o;
    }
    Bt drop(const Bt &a, int level) const {
        REQUIRE(level <= a.level && level >= 0, HE_EDEPTH, "drop: bad level");
        Bt o = a;
        o.level = level;
        return o;
    }
    Bt mul_int(const Bt &a, const std::vector<int64_t> &k) {
        Bt o = new_bt(a.cnt, a.level);
        o.scale = a.scale;
        ConstTab kt{residues(k, a.level), 2, a.level + 1};
        if (go()) launch_mul_const(T, vs_all(o), vs_all(a), kt, s);
        return o;
    }
    Bt add_const(const Bt &a, const std::vector<double> &c) {
        std::vector<int64_t> v(a.cnt);
        for (int i = 0; i < a.cnt; ++i) v[i] = llround_d(c[i] * a.scale[i]);
        Bt o = new_bt(a.cnt, a.level);
        o.scale = a.scale;
        // one launch: the constant onto polynomial 0, polynomial 1 copied
        ConstTab kt{residues(v, a.level), 2, a.level + 1};
        if (go()) launch_add_const(T, vs_all(o), vs_all(a), kt, s, 1);
        return o;
    }
    // D_k = n_k * Y_k - S[map[k]]
    Bt center(const Bt &Y, const Bt &S, const std::vector<int> &cmap, const std::vector<int64_t> &n) {
        REQUIRE(Y.level == S.level, HE_ESTATE, "center: level mismatch");
        for (int c = 0; c < Y.cnt; ++c)
            REQUIRE(std::fabs(Y.scale[c] - S.scale[cmap[c]]) <= 1e-9 * Y.scale[c], HE_ERANGE, "center: scale mismatch");
        Bt o = new_bt(Y.cnt, Y.level);
        o.scale = Y.scale;
        ConstTab kt{residues(n, Y.level), 2, Y.level + 1};
        const int *dmap = C->pool.push(cmap);
        if (go()) launch_axpy_map(T, vs_all(o), vs_all(Y), kt, vs_all(S), dmap, 2, s);
        return o;
    }
    // S_r - k_r * B[map[r]] for the requests with map[r] >= 0, S_r for the others
    Bt sub_mul_map(const Bt &S, const Bt &B, const std::vector<int64_t> &k, const std::vector<int> &map) {
        REQUIRE(S.level == B.level, HE_ESTATE, "sub_mul_map: level mismatch");
        for (int r = 0; r < S.cnt; ++r)
            if (map[r] >= 0)
                REQUIRE(std::fabs(S.scale[r] - B.scale[map[r]]) <= 1e-9 * S.scale[r], HE_ERANGE,
                        "sub_mul_map: scale mismatch");
        Bt o = new_bt(S.cnt, S.level);
        o.scale = S.scale;
        ConstTab kt{residues(k, S.level), 2, S.level + 1};
        const int *dmap = C->pool.push(map);
        if (go()) launch_sub_mul_map(T, vs_all(o), vs_all(S), kt, vs_all(B), dmap, 2, s);
        return o;
    }
    // per-request sums of consecutive ciphertexts
    Bt sum_groups(const Bt &Y, const std::vector<int> &first, const std::vector<int> &cnt) {
        const int R = (int)first.size();
        // one ciphertext per request, in order: the sums are the ciphertexts themselves
        // (a view; its consumers read it and write elsewhere)
        bool ident = R <= Y.cnt;
        for (int r = 0; r < R && ident; ++r) ident = first[r] == r && cnt[r] == 1;
        if (ident) {
            Bt v = Y;
            v.cnt = R;
            v.scale.resize(R);
            return v;
        }
        Bt o = new_bt(R, Y.level);
        for (int r = 0; r < R; ++r) {
            o.scale[r] = Y.scale[first[r]];
            for (int k = 1; k < cnt[r]; ++k)
                REQUIRE(std::fabs(Y.scale[first[r] + k] - o.scale[r]) <= 1e-9 * o.scale[r], HE_ERANGE, "sum: scale mismatch");
        }
        const int *df = C->pool.push(first);
        const int *dc = C->pool.push(cnt);
        if (go()) launch_sum_groups(T, vs_all(o), vs_all(Y), df, dc, 2, s);
        return o;
    }

    // ------------------------------------------------------------- rescale
    // (K a - [K a_l]_centred) / q_l per limb; kres (per ct, limbs 0..l) = K mod q_i, or
    // null for a plain rescale.  The lift of the last limb to the other primes is
    // computed while loading the forward NTT, and the combine happens on its store.
    // With K (the integers behind kres, one per ciphertext) the inverse NTT of the last limb
    // applies K together with N^-1 (INTT(K c) = K INTT(c)), so no separate multiply runs.
    Bt rescale(const Bt &a, const double *kres = nullptr, const std::vector<int64_t> *K = nullptr) {
        const int l = a.level;
        REQUIRE(l >= 1, HE_EDEPTH, "rescale at level 0");
        REQUIRE(!kres == !K, HE_EINVAL, "rescale: residues and integers go together");
        Bt o = new_bt(a.cnt, l - 1);
        for (int c = 0; c < a.cnt; ++c) o.scale[c] = a.scale[c] / (double)C->q[l];
        const size_t m = C->arena.mark();
        const int G = a.cnt * 2;
        const long long N = C->N;
        double *last = alloc_d((size_t)G * N);
        double *lift = alloc_d((size_t)G * l * N);
        const double *kscale = nullptr;
        const int *lprime = nullptr;
        if (kres) {
            // per vector (ciphertext, polynomial): N^-1 K mod q_l
            const uint64_t ql = C->q[l], ninv = invmod_u((uint64_t)N % ql, ql);
            std::vector<double> ks(G);
            for (int g = 0; g < G; ++g) ks[g] = (double)mulmod_u(ninv, red_i64((*K)[g >> 1], ql), ql);
            kscale = C->pool.push(ks);
            lprime = C->pool.push(std::vector<int>(G, l));
        }
        if (go()) {
            VecSet src{a.d + (long long)l * N, G, 1, (long long)a.cap * N, nullptr, C->ident + l};
            if (kres) {
                // one group of G vectors, every one modulo q_l, scaled per vector
                launch_ntt(T, VecSet{last, G, G, 0, nullptr, lprime}, true, C->ntt_variant, s, &src, kscale);
            } else {
                launch_ntt(T, VecSet{last, G, 1, N, nullptr, C->ident + l}, true, C->ntt_variant, s, &src);
            }
            NttPro pro{1, last, N, (double)C->q[l]};
            NttEpi epi{};
            epi.kind = 2;
            epi.out = o.d;
            epi.o_g = (long long)o.cap * N;
            epi.in = a.d;
            epi.i_g = (long long)a.cap * N;
            epi.cst = C->qlinv + (long long)l * (C->L + 1);
            epi.kmul = kres;
            epi.kstride = l + 1;
            launch_ntt_fused(T, VecSet{lift, G * l, l, (long long)l * N, nullptr, nullptr}, pro, epi, C->ntt_variant, s);
        }
        C->arena.release(m);
        return o;
    }

    // ------------------------------------------------------------ key switch
    // d: NTT-domain polynomials [cnt] at `dstride` words apart, limbs 0..l.
    // out (groups ct*2 + poly at ostride) = ModDown(sum_j ModUp_j(d) key_j) + a1 + a2.
    // With rot, the key products are those of a hoisted rotate-and-sum step: every
    // rotation's automorphism applied to the extended digits, its key, summed (kidx unused).
    // With mrescale (relinearisation), a1 holds the tensor's d0/d1 over Q_l and the output
    // is (d + relinearised d2) / q_l at level l - 1: the ModDown divides A = acc + P d by
    // P q_l in one rounding (a2 and rot unused).
    // the extended digits [cnt][beta][next][N] of d (ModUp: inverse NTT with Qhat_i^-1
    // folded in, basis conversion of every digit, one forward NTT of the converted limbs)
    double *modup(const double *d, long long dstride, int cnt, int l) {
        const int A = C->alpha, next = l + 1 + A, beta = (l + 1 + A - 1) / A;
        const long long N = C->N;
        double *ext = alloc_d((size_t)cnt * beta * next * N);
        const size_t m = C->arena.mark();
        double *dcoef = alloc_d((size_t)cnt * (l + 1) * N);
        if (go()) {
            VecSet vd{dcoef, cnt * (l + 1), l + 1, (long long)(l + 1) * N, nullptr, nullptr};
            const VecSet vsrc{const_cast<double *>(d), cnt * (l + 1), l + 1, dstride, nullptr, nullptr};
            launch_ntt(T, vd, true, C->ntt_variant, s, &vsrc, C->mu_scale[l]);
            ModUpDigits dg{};
            for (int j = 0; j < beta; ++j) {
                dg.qhat[j] = C->qhat[l][j];
                dg.lo[j] = j * A;
                dg.dl[j] = std::min(A, l + 1 - j * A);
            }
            launch_modup(T, dcoef, (long long)(l + 1) * N, ext, (long long)beta * next * N, (long long)next * N, d,
                         dstride, cnt, beta, next, C->ext_prime[l], dg, s);
            const int nd = C->ndall[l];
            launch_ntt(T, VecSet{ext, cnt * nd, nd, (long long)beta * next * N, C->ndall_slot[l], C->ndall_prime[l]},
                       false, C->ntt_variant, s);
        }
        C->arena.release(m);
        return ext;
    }

    // ext_pre: the extended digits of d already computed (modup), d unused
    // acc_out (optional): the key-product accumulators [cnt][2][next] go there (and stay
    // after the call) instead of to workspace; md_poly1: the ModDown and the output cover
    // polynomial 1 only (polynomial 0's accumulator is left in acc_out).
    // dbuf: [cnt][l+1][N] for the coefficient-domain digits (the ModUp input) instead of
    // workspace; with dbuf_half it already holds the first inverse-NTT pass of d (written
    // by the previous call's chain_out) and only the second runs, in place.  chain_out
    // (with md_poly1): the output polynomial's first inverse-NTT pass goes there as well
    void keyswitch(const double *d, long long dstride, int cnt, int l, int kidx, double *out, long long ostride,
                   Addend a1 = Addend{nullptr, 0, 0, 0}, Addend a2 = Addend{nullptr, 0, 0, 0},
                   const RotSet *rot = nullptr, bool mrescale = false, const double *ext_pre = nullptr,
                   double *acc_out = nullptr, bool md_poly1 = false, double *dbuf = nullptr,
                   bool dbuf_half = false, double *chain_out = nullptr) {
        const int A = C->alpha, next = l + 1 + A, beta = (l + 1 + A - 1) / A;
        const long long N = C->N;
        const size_t m = C->arena.mark();
        double *dcoef = ext_pre ? nullptr : dbuf ? dbuf : alloc_d((size_t)cnt * (l + 1) * N);
        double *ext = ext_pre ? const_cast<double *>(ext_pre) : alloc_d((size_t)cnt * beta * next * N);
        double *acc = acc_out ? acc_out : alloc_d((size_t)cnt * 2 * next * N);
        double *conv = alloc_d((size_t)cnt * 2 * (l + 1) * N);
        if (go() && !ext_pre) {
            // coefficient-domain digits, already scaled by Qhat_i^-1 (folded into N^-1)
            VecSet vd{dcoef, cnt * (l + 1), l + 1, (long long)(l + 1) * N, nullptr, nullptr};
            const VecSet vsrc{const_cast<double *>(d), cnt * (l + 1), l + 1, dstride, nullptr, nullptr};
            if (dbuf_half) launch_ntt(T, vd, true, C->ntt_variant, s, nullptr, C->mu_scale[l], true);
            else launch_ntt(T, vd, true, C->ntt_variant, s, &vsrc, C->mu_scale[l]);
            ModUpDigits dg{};
            for (int j = 0; j < beta; ++j) {
                dg.qhat[j] = C->qhat[l][j];
                dg.lo[j] = j * A;
                dg.dl[j] = std::min(A, l + 1 - j * A);
            }
            // the basis conversion of every digit inside the first pass of the converted
            // limbs' forward NTT; the digits' own limbs are neither copied nor transformed
            // (the key products read them from d)
            launch_modup_ntt(T, dcoef, (long long)(l + 1) * N, ext, (long long)beta * next * N, (long long)next * N,
                             cnt, beta, next, C->ext_prime[l], dg, s);
            const int nd = C->ndall[l];
            launch_ntt_fwd_pass2(
                T, VecSet{ext, cnt * nd, nd, (long long)beta * next * N, C->ndall_slot[l], C->ndall_prime[l]},
                C->ntt_variant, s);
        }
        if (go()) {
            const OwnSrc own = ext_pre ? OwnSrc{} : OwnSrc{d, dstride, A, l};
            if (rot) {
                RotSet rs = *rot;
                if (!rs.multi) rs.own = own;
                launch_inner_product_rot(T, ext, (long long)beta * next * N, (long long)next * N, acc,
                                         acc + (long long)next * N, 2LL * next * N, rs, C->betaL, cnt, beta,
                                         next, C->ext_prime[l], s);
            } else if (mrescale) {
                launch_inner_product(T, ext, (long long)beta * next * N, (long long)next * N, acc,
                                     acc + (long long)next * N, 2LL * next * N, C->keys[kidx], C->betaL, cnt,
                                     beta, next, C->ext_prime[l], s, a1.p + (long long)l * N, a1.ct, a1.poly, l,
                                     C->pmod_h[l], own);
            } else {
                launch_inner_product(T, ext, (long long)beta * next * N, (long long)next * N, acc,
                                     acc + (long long)next * N, 2LL * next * N, C->keys[kidx], C->betaL, cnt,
                                     beta, next, C->ext_prime[l], s, nullptr, 0, 0, -1, 0.0, own);
            }
            if (mrescale) {
                // B = {q_l, P} to the coefficient domain, scaled by Bhat^-1; convert to q_0..q_{l-1};
                // transform and combine on store: (acc - conv) (P q_l)^-1 + d q_l^-1
                launch_ntt(T, VecSet{acc + (long long)l * N, cnt * 2 * (A + 1), A + 1, (long long)next * N, nullptr,
                                     C->ext_prime[l] + l},
                           true, C->ntt_variant, s, nullptr, C->mr_scale[l]);
                launch_moddown_ntt(T, acc, (long long)next * N, conv, (long long)l * N, cnt * 2,
                                    MdIn{l, A + 1, C->ext_prime[l] + l, C->mr_phat[l], l, l}, s);
                NttEpi epi{};
                epi.kind = 3;
                epi.out = out;
                epi.o_g = ostride;
                epi.in = acc;
                epi.i_g = (long long)next * N;
                epi.add1 = a1.p; epi.a1_ct = a1.ct; epi.a1_poly = a1.poly; epi.m1 = a1.mask;
                epi.cst = C->mr_inv[l];
                epi.cst2 = C->qlinv + (long long)l * (C->L + 1);
                launch_ntt_fused(T, VecSet{conv, cnt * 2 * l, l, (long long)l * N, nullptr, nullptr}, NttPro{}, epi,
                                 C->ntt_variant, s, 2);
                C->arena.release(m);
                return;
            }
            if (md_poly1) {
                // polynomial 1 alone: groups are ciphertexts (stride 2 next N in acc, 2
                // ostride in out)
                double *acc1 = acc + (long long)next * N;
                launch_ntt(T, VecSet{acc1 + (long long)(l + 1) * N, cnt * A, A, 2LL * next * N, nullptr, C->pprime},
                           true, C->ntt_variant, s, nullptr, C->md_scale);
                launch_moddown_ntt(T, acc1, 2LL * next * N, conv, (long long)(l + 1) * N, cnt,
                                    MdIn{l + 1, A, C->pprime, C->phat, C->L + 1, l + 1}, s);
                NttEpi epi{};
                epi.kind = 1;
                epi.poly1 = 1;
                epi.out = out + ostride;
                epi.o_g = 2 * ostride;
                epi.in = acc1;
                epi.i_g = 2LL * next * N;
                epi.add1 = a1.p; epi.a1_ct = a1.ct; epi.a1_poly = a1.poly; epi.m1 = a1.mask;
                epi.add2 = a2.p; epi.a2_ct = a2.ct; epi.a2_poly = a2.poly; epi.m2 = a2.mask;
                epi.cst = C->Pinv;
                epi.chain = chain_out;
                epi.ch_g = (long long)(l + 1) * N;
                launch_ntt_fused(T, VecSet{conv, cnt * (l + 1), l + 1, (long long)(l + 1) * N, nullptr, nullptr},
                                 NttPro{}, epi, C->ntt_variant, s, 2);
                C->arena.release(m);
                return;
            }
            // P slots to the coefficient domain, scaled by Phat_m^-1
            launch_ntt(T, VecSet{acc + (long long)(l + 1) * N, cnt * 2 * A, A, (long long)next * N, nullptr, C->pprime},
                       true, C->ntt_variant, s, nullptr, C->md_scale);
            launch_moddown_ntt(T, acc, (long long)next * N, conv, (long long)(l + 1) * N, cnt * 2,
                                MdIn{l + 1, A, C->pprime, C->phat, C->L + 1, l + 1}, s);
            // transform the conversion and combine on store: (acc - conv) P^-1 + addends
            NttEpi epi{};
            epi.kind = 1;
            epi.out = out;
            epi.o_g = ostride;
            epi.in = acc;
            epi.i_g = (long long)next * N;
            epi.add1 = a1.p; epi.a1_ct = a1.ct; epi.a1_poly = a1.poly; epi.m1 = a1.mask;
            epi.add2 = a2.p; epi.a2_ct = a2.ct; epi.a2_poly = a2.poly; epi.m2 = a2.mask;
            epi.cst = C->Pinv;
            launch_ntt_fused(T, VecSet{conv, cnt * 2 * (l + 1), l + 1, (long long)(l + 1) * N, nullptr, nullptr},
                             NttPro{}, epi, C->ntt_variant, s, 2);
        }
        C->arena.release(m);
    }

    // tensor, relinearise, rescale; b indexed through bmap when given
    Bt mul(const Bt &a, const Bt &b, const std::vector<int> *bmap = nullptr) {
        REQUIRE(a.level == b.level, HE_ESTATE, "mul: level mismatch");
        const int l = a.level;
        REQUIRE(l >= 1, HE_EDEPTH, "mul at level 0");
        const long long N = C->N;
        // tensor, then relinearisation and rescale in one ModDown by P q_l
        Bt o = new_bt(a.cnt, l - 1);
        for (int c = 0; c < a.cnt; ++c) o.scale[c] = (a.scale[c] * b.scale[bmap ? (*bmap)[c] : c]) / (double)C->q[l];
        const size_t m = C->arena.mark();
        double *t = alloc_d((size_t)a.cnt * 3 * (l + 1) * N);
        // the key switch's ModUp input: the first inverse-NTT pass of d2, run by the
        // tensor launch itself on the blocks it forms
        double *dc = alloc_d((size_t)a.cnt * (l + 1) * N);
        const int *dmap = bmap ? C->pool.push(*bmap) : nullptr;
        if (go()) {
            NttPro pro{};
            pro.kind = 2;
            pro.ta = a.d;
            pro.tb = b.d;
            pro.ta_ct = 2LL * a.cap * N;
            pro.tb_ct = 2LL * b.cap * N;
            pro.ta_poly = (long long)a.cap * N;
            pro.tb_poly = (long long)b.cap * N;
            pro.tmap = dmap;
            pro.td = t;
            pro.td_ct = 3LL * (l + 1) * N;
            pro.td_poly = (long long)(l + 1) * N;
            launch_tensor_intt(T, VecSet{dc, a.cnt * (l + 1), l + 1, (long long)(l + 1) * N, nullptr, nullptr}, pro,
                               C->ntt_variant, s);
        }
        keyswitch(t + 2 * (l + 1) * N, 3LL * (l + 1) * N, a.cnt, l, 0, o.d, (long long)o.cap * N,
                  Addend{t, 3LL * (l + 1) * N, (long long)(l + 1) * N, 3}, Addend{nullptr, 0, 0, 0}, nullptr, true,
                  nullptr, nullptr, false, dc, true);
        C->arena.release(m);
        return o;
    }

    // multiply by a real constant then rescale (cm_exact / cm_target)
    Bt cmul(const Bt &a, const std::vector<double> &kappa, const std::vector<double> &s_want, bool exact) {
        const int l = a.level;
        REQUIRE(l >= 1, HE_EDEPTH, "constant multiply at level 0");
        const double q = (double)C->q[l];
        std::vector<int64_t> K(a.cnt);
        for (int c = 0; c < a.cnt; ++c) {
            const double x = ((kappa[c] * s_want[c]) * q) / a.scale[c];
            REQUIRE(std::fabs(x) < 4.0e18, HE_ERANGE, "constant not encodable");
            K[c] = llround_d(x);
            REQUIRE(K[c] != 0 && std::llabs(K[c]) < (1LL << 62), HE_ERANGE, "constant not encodable");
        }
        Bt o = rescale(a, residues(K, l), &K);
        for (int c = 0; c < a.cnt; ++c)
            o.scale[c] = exact ? ((a.scale[c] * (double)K[c]) / q) / kappa[c] : s_want[c];
        return o;
    }

    // rotation by 2^r slots; with `into`, the result is added into that batch in place
    Bt rotate(const Bt &a, int r, Bt *into = nullptr) {
        uint64_t g = 5;
        for (int i = 0; i < r; ++i) g = (g * g) % (2ull * C->N);
        return rotate_gal(a, 1 + r, g, into);
    }

    // automorphism X -> X^g on both polynomials, key switch of sigma(c1) with key
    // kidx: (sigma(c0) + ks0, ks1) [+ into].  The automorphism acts inside the key
    // switch: c1 is extended (ModUp) as it is, the key products gather the extended
    // NTT-domain digits at the automorphism's source positions (the centred extension
    // commutes with the automorphism), and the ModDown epilogue adds sigma(c0), gathered
    // by the same key-product kernel; no separate automorphism pass.
    Bt rotate_gal(const Bt &a, int kidx, uint64_t g, Bt *into = nullptr) {
        REQUIRE(kidx >= 1 && kidx < (int)C->keys.size() && C->keys[kidx].lo, HE_ESTATE, "no such Galois key");
        REQUIRE(C->key_gal[kidx] == (uint32_t)g, HE_ESTATE, "key was generated for another Galois element");
        if (into)
            for (int c = 0; c < a.cnt; ++c)
                REQUIRE(std::fabs(a.scale[c] - into->scale[c]) <= 1e-9 * a.scale[c], HE_ERANGE, "rotate: scale mismatch");
        const int l = a.level;
        const long long N = C->N;
        Bt o;
        if (into) {
            o = *into;
        } else {
            o = new_bt(a.cnt, l);
            o.scale = a.scale;
        }
        const size_t m = C->arena.mark();
        double *ext = modup(a.d + (long long)a.cap * N, 2LL * a.cap * N, a.cnt, l);
        double *s0 = alloc_d((size_t)a.cnt * (l + 1) * N);
        RotSet rs{};
        rs.nr = 1;
        rs.key[0] = C->keys[kidx];
        rs.g[0] = (uint32_t)g;
        rs.xorder = C->xorder_id;
        rs.c0 = a.d;
        rs.c0_ct = 2LL * a.cap * N;
        rs.s0 = s0;
        rs.s0_ct = (long long)(l + 1) * N;
        rs.lq = l;
        rs.c0_id = 0;
        Addend acc{nullptr, 0, 0, 0};
        if (into) acc = Addend{into->d, 2LL * into->cap * N, (long long)into->cap * N, 3};
        keyswitch(nullptr, 0, a.cnt, l, -1, o.d, (long long)o.cap * N, Addend{s0, (long long)(l + 1) * N, 0, 1}, acc,
                  &rs, false, ext);
        C->arena.release(m);
        return o;
    }

    // rotations of one batch by several Galois elements sharing one ModUp: each
    // automorphism acts on the extended NTT-domain digits inside its key products (the
    // extension commutes with the automorphism because the digits are lifted to their
    // centred representatives), one ModDown per rotation; equal to rotate_gal word for word
    std::vector<Bt> rotate_many(const Bt &a, const std::vector<std::pair<int, uint64_t>> &rots) {
        const int l = a.level;
        const long long N = C->N;
        std::vector<Bt> outs;
        for (size_t r = 0; r < rots.size(); ++r) {
            const int kidx = rots[r].first;
            REQUIRE(kidx >= 1 && kidx < (int)C->keys.size() && C->keys[kidx].lo, HE_ESTATE, "no such Galois key");
            REQUIRE(C->key_gal[kidx] == (uint32_t)rots[r].second, HE_ESTATE, "key was generated for another Galois element");
            Bt o = new_bt(a.cnt, l);
            o.scale = a.scale;
            outs.push_back(o);
        }
        if (rots.empty()) return outs;
        const size_t m = C->arena.mark();
        double *ext = modup(a.d + (long long)a.cap * N, 2LL * a.cap * N, a.cnt, l);
        double *s0 = alloc_d((size_t)a.cnt * (l + 1) * N);
        for (size_t r = 0; r < rots.size(); ++r) {
            RotSet rs{};
            rs.nr = 1;
            rs.key[0] = C->keys[rots[r].first];
            rs.g[0] = (uint32_t)rots[r].second;
            rs.xorder = C->xorder_id;
            rs.c0 = a.d;
            rs.c0_ct = 2LL * a.cap * N;
            rs.s0 = s0;
            rs.s0_ct = (long long)(l + 1) * N;
            rs.lq = l;
            rs.c0_id = 0;
            keyswitch(nullptr, 0, a.cnt, l, -1, outs[r].d, (long long)outs[r].cap * N,
                      Addend{s0, (long long)(l + 1) * N, 0, 1}, Addend{nullptr, 0, 0, 0}, &rs, false, ext);
        }
        C->arena.release(m);
        return outs;
    }

    // sum_r rot_{g_r}(x_r) [+ x0] over ciphertexts x_r of one level: every x_r extended
    // once (ModUp), the key products of all rotations summed in one pass (each gathering
    // its own extended digits), one ModDown whose epilogue adds sum_r sigma_r(c0_r) and x0
    Bt rotate_sum_multi(const std::vector<Bt> &xs, const std::vector<std::pair<int, uint64_t>> &rots, const Bt *x0) {
        REQUIRE(!xs.empty() && xs.size() == rots.size() && xs.size() <= 7, HE_EINVAL, "rotate_sum_multi: 1..7 rotations");
        const Bt &a = xs[0];
        const int l = a.level;
        const long long N = C->N;
        for (const Bt &x : xs)
            REQUIRE(x.level == l && x.cnt == a.cnt && x.cap == a.cap, HE_ESTATE, "rotate_sum_multi: shapes differ");
        for (int c = 0; c < a.cnt; ++c) {
            for (const Bt &x : xs)
                REQUIRE(std::fabs(x.scale[c] - a.scale[c]) <= 1e-9 * a.scale[c], HE_ERANGE, "rotate_sum_multi: scales");
            if (x0) REQUIRE(std::fabs(x0->scale[c] - a.scale[c]) <= 1e-9 * a.scale[c], HE_ERANGE, "rotate_sum_multi: scales");
        }
        if (x0) REQUIRE(x0->level == l && x0->cnt == a.cnt, HE_ESTATE, "rotate_sum_multi: addend shape");
        Bt o = new_bt(a.cnt, l);
        o.scale = a.scale;
        const size_t m = C->arena.mark();
        RotSet rs{};
        rs.nr = (int)xs.size();
        rs.multi = 1;
        rs.xorder = C->xorder_id;
        rs.c0_ct = 2LL * a.cap * N;
        rs.s0 = alloc_d((size_t)a.cnt * (l + 1) * N);
        rs.s0_ct = (long long)(l + 1) * N;
        rs.lq = l;
        for (size_t r = 0; r < xs.size(); ++r) {
            const int kidx = rots[r].first;
            REQUIRE(kidx >= 1 && kidx < (int)C->keys.size() && C->keys[kidx].lo, HE_ESTATE, "no such Galois key");
            REQUIRE(C->key_gal[kidx] == (uint32_t)rots[r].second, HE_ESTATE, "key was generated for another Galois element");
            rs.key[r] = C->keys[kidx];
            rs.g[r] = (uint32_t)rots[r].second;
            rs.ext_r[r] = modup(xs[r].d + (long long)xs[r].cap * N, 2LL * xs[r].cap * N, a.cnt, l);
            rs.c0_r[r] = xs[r].d;
        }
        Addend add0{nullptr, 0, 0, 0};
        if (x0) add0 = Addend{x0->d, 2LL * x0->cap * N, (long long)x0->cap * N, 3};
        keyswitch(nullptr, 0, a.cnt, l, -1, o.d, (long long)o.cap * N, Addend{rs.s0, (long long)(l + 1) * N, 0, 1}, add0,
                  &rs, false, rs.ext_r[0]);
        C->arena.release(m);
        return o;
    }

    // sum_t K[t cnt + c] x_t[c] for ciphertexts x_t of one level (integer constants, no
    // rescale), declared at scale s_out
    Bt lincomb(const std::vector<Bt> &xs, const std::vector<int64_t> &K, double s_out) {
        REQUIRE(!xs.empty() && (int)xs.size() <= kMaxLtTerms, HE_EINVAL, "lincomb: 1..16 terms");
        const int l = xs[0].level, cnt = xs[0].cnt;
        REQUIRE((int)K.size() == (int)xs.size() * cnt, HE_EINVAL, "lincomb: constants");
        Bt o = new_bt(cnt, l);
        o.scale.assign(cnt, s_out);
        LtTerms tm{};
        tm.n = (int)xs.size();
        std::vector<double> kr((size_t)xs.size() * cnt * (l + 1));
        for (size_t t = 0; t < xs.size(); ++t) {
            REQUIRE(xs[t].level == l && xs[t].cnt == cnt, HE_ESTATE, "lincomb: shapes differ");
            tm.x[t] = xs[t].d;
            tm.xct[t] = 2LL * xs[t].cap * C->N;
            tm.xpoly[t] = (long long)xs[t].cap * C->N;
            for (int c = 0; c < cnt; ++c)
                for (int i = 0; i <= l; ++i)
                    kr[(t * cnt + c) * (l + 1) + i] = (double)red_i64(K[t * cnt + c], C->q[i]);
        }
        const double *kd = C->pool.push(kr);
        if (go()) launch_lincomb(T, o.d, 2LL * o.cap * C->N, (long long)o.cap * C->N, tm, kd, cnt, l + 1, s);
        return o;
    }

    // both polynomials times a plaintext (NTT-domain residues, limb i at pt + i N),
    // declared scale times pscale, no rescale
    Bt mul_plain(const Bt &a, const double *pt, double pscale) {
        Bt o = new_bt(a.cnt, a.level);
        for (int c = 0; c < a.cnt; ++c) o.scale[c] = a.scale[c] * pscale;
        LtTerms tm{};
        tm.n = 1;
        tm.pt[0] = pt;
        tm.x[0] = a.d;
        tm.xct[0] = 2LL * a.cap * C->N;
        tm.xpoly[0] = (long long)a.cap * C->N;
        if (go()) launch_lt_inner(T, o.d, 2LL * o.cap * C->N, (long long)o.cap * C->N, tm, a.cnt, a.level + 1, s);
        return o;
    }

    // ModRaise: the level-0 residues mod q_0 (coefficient domain), centred and reduced
    // modulo q_0 .. q_level (the lift runs in the forward NTT's loads)
    Bt modraise(const Bt &a, int level, double scale) {
        REQUIRE(a.level == 0, HE_ESTATE, "modraise needs a level-0 ciphertext");
        REQUIRE(level >= 0 && level <= C->L, HE_EINVAL, "modraise: bad level");
        const long long N = C->N;
        const int G = a.cnt * 2;
        Bt o = new_bt(a.cnt, level);
        o.scale.assign(a.cnt, scale);
        const size_t m = C->arena.mark();
        double *last = alloc_d((size_t)G * N);
        if (go()) {
            VecSet src{a.d, G, 1, (long long)a.cap * N, nullptr, C->ident};
            VecSet dst{last, G, 1, N, nullptr, C->ident};
            launch_ntt(T, dst, true, C->ntt_variant, s, &src);
            NttPro pro{1, last, N, (double)C->q[0]};
            launch_ntt_fused(T, VecSet{o.d, G * (level + 1), level + 1, (long long)o.cap * N, nullptr, nullptr}, pro,
                             NttEpi{}, C->ntt_variant, s);
        }
        C->arena.release(m);
        return o;
    }

    // rotate-and-sum over every slot (Sec. 3.2): x <- x + rot(x, 2^r) one rotation at
    // a time, or hoisted steps x <- x + sum_r rot(x, a_r)
    Bt rotsum(const Bt &a) {
        if (C->hoist >= 1) {
            const auto steps = hoist_steps(C->slots, C->hoist);
            Bt o = new_bt(a.cnt, a.level);
            o.scale = a.scale;
            if (steps.size() == 1) {
                const size_t m = C->arena.mark();
                rotsum_step(a, o, steps[0]);
                C->arena.release(m);
                return o;
            }
            // c0 is carried as P c0 over Q_l u P from step to step (in the key products'
            // accumulator of polynomial 0, two buffers used in turn), so only c1 takes a
            // ModDown per step and c0 one at the end; the first step reads a, the others
            // update o's c1 in place
            // dhalf holds every step's ModUp input; each step but the last also writes the
            // first inverse-NTT pass of its output c1 there (chained into its ModDown
            // epilogue, after its own ModUp has read it).
            const int next = a.level + 1 + C->alpha;
            double *accb[2] = {alloc_d((size_t)a.cnt * 2 * next * C->N), alloc_d((size_t)a.cnt * 2 * next * C->N)};
            double *dhalf = alloc_d((size_t)a.cnt * (a.level + 1) * C->N);
            for (size_t k = 0; k < steps.size(); ++k) {
                const size_t m = C->arena.mark();
                const bool last = k + 1 == steps.size();
                rotsum_step_carried(k == 0 ? a : o, o, steps[k], k == 0 ? nullptr : accb[(k - 1) & 1], accb[k & 1],
                                    last, dhalf, k > 0, last ? nullptr : dhalf);
                C->arena.release(m);
            }
            return o;
        }
        Bt o = copy(a);
        int lg = 0;
        while ((1 << lg) < C->slots) ++lg;
        for (int r = 0; r < lg; ++r) {
            const size_t m = C->arena.mark();
            rotate(o, r, &o);
            C->arena.release(m);
        }
        return o;
    }

    // one hoisted step x -> y (y may be x): c1 is extended once, each rotation's
    // automorphism acts on the extended digits inside the key products (where
    // c0 + sum_r sigma_r(c0) is gathered too), one ModDown for all:
    //   y0 = c0 + sum_r sigma_r(c0) + MD_0,  y1 = c1 + MD_1
    void rotsum_step(const Bt &x, const Bt &y, const std::vector<int> &amounts) {
        const int l = x.level;
        const long long N = C->N;
        REQUIRE(!amounts.empty() && (int)amounts.size() <= kMaxHoist, HE_EINVAL, "hoisted step size");
        RotSet rs{};
        rs.nr = (int)amounts.size();
        rs.xorder = C->xorder.at(amounts[0]);
        for (int r = 0; r < rs.nr; ++r) {
            auto it = C->rot_key.find(amounts[r]);
            REQUIRE(it != C->rot_key.end(), HE_ESTATE, "no key for a hoisted rotation");
            rs.key[r] = C->keys[it->second];
            rs.g[r] = C->key_gal[it->second];
        }
        double *s0 = alloc_d((size_t)x.cnt * (l + 1) * N);
        rs.c0 = x.d;
        rs.c0_ct = 2LL * x.cap * N;
        rs.s0 = s0;
        rs.s0_ct = (long long)(l + 1) * N;
        rs.lq = l;
        rs.c0_id = 1;
        keyswitch(x.d + (long long)x.cap * N, 2LL * x.cap * N, x.cnt, l, -1, y.d, (long long)y.cap * N,
                  Addend{s0, (long long)(l + 1) * N, 0, 1}, Addend{x.d, 2LL * x.cap * N, (long long)x.cap * N, 2},
                  &rs);
    }

    // one hoisted step with c0 carried as X0 = P c0 over Q_l u P: the key products fold
    // X0 + sum_r sigma_r(X0) into polynomial 0's accumulator (the first step forms it from
    // x's c0 over Q_l times [P]_{q_i}; P c0 vanishes on the P limbs), so acc0 becomes the
    // next X0; c1 takes its ModDown:  y1 = c1 + MD_1.  The last step takes the ModDown of
    // both polynomials, y0 = MD(X0) = c0 + sum of every step's rotations.
    void rotsum_step_carried(const Bt &x, const Bt &y, const std::vector<int> &amounts, const double *x0,
                             double *acc, bool last, double *dbuf, bool dbuf_half, double *chain_out) {
        const int l = x.level, next = l + 1 + C->alpha;
        const long long N = C->N;
        REQUIRE(!amounts.empty() && (int)amounts.size() <= kMaxHoist, HE_EINVAL, "hoisted step size");
        RotSet rs{};
        rs.nr = (int)amounts.size();
        rs.xorder = C->xorder.at(amounts[0]);
        for (int r = 0; r < rs.nr; ++r) {
            auto it = C->rot_key.find(amounts[r]);
            REQUIRE(it != C->rot_key.end(), HE_ESTATE, "no key for a hoisted rotation");
            rs.key[r] = C->keys[it->second];
            rs.g[r] = C->key_gal[it->second];
        }
        rs.c0_id = 1;
        rs.fold = 1;
        if (x0) {
            rs.c0 = x0;
            rs.c0_ct = 2LL * next * N;
            rs.lq = next - 1;
        } else {
            rs.c0 = x.d;
            rs.c0_ct = 2LL * x.cap * N;
            rs.lq = l;
            rs.c0_mul = C->pmod;
        }
        keyswitch(x.d + (long long)x.cap * N, 2LL * x.cap * N, x.cnt, l, -1, y.d, (long long)y.cap * N,
                  Addend{nullptr, 0, 0, 0}, Addend{x.d, 2LL * x.cap * N, (long long)x.cap * N, 2}, &rs, false,
                  nullptr, acc, !last, dbuf, dbuf_half, chain_out);
    }

    Bt power(const Bt &y, int p) {
        REQUIRE(p >= 1, HE_EINVAL, "power must be >= 1");
        std::vector<Bt> pw{y};
        int nb = 0;
        while ((p >> nb) > 1) ++nb;
        for (int i = 1; i <= nb; ++i) pw.push_back(mul(pw.back(), pw.back()));
        Bt acc;
        bool have = false;
        for (int i = 0; i <= nb; ++i) {
            if (!((p >> i) & 1)) continue;
            if (!have) { acc = pw[i]; have = true; }
            else {
                const int lv = std::min(acc.level, pw[i].level);
                acc = mul(drop(acc, lv), drop(pw[i], lv));
            }
        }
        return acc;
    }
};

// ------------------------------------------------------------- CutMax plan
// n: the slot count the moments run over (a * slots, or the logit count with masked
// padding); npad > 0 gives the request a pad tracker (pad: its starting value)
struct Request { int first, a; int64_t n; int64_t npad = 0; double pad = 0; };

// Goldschmidt's coupled iteration costs one level more than Newton's: its first
// product u h^2 needs h^2 before the update multiplies h
int invsqr_depth(int degree, int newton, bool gold) {
    static const int d[5] = {0, 1, 2, 2, 3};
    return d[degree] + 2 * newton + (gold && newton > 0 ? 1 : 0);
}

// Goldschmidt refinement of h ~ C u^(-1/2) (the inverse-square-root iteration the
// paper's App. B.1 cites): with b = u (h/C)^2 kept as b' = b/2,
//   r_k = 1.5 - b'_k,  h_{k+1} = h_k r_k,  b'_{k+1} = b'_k r_k^2.
// It equals Newton's iteration in exact arithmetic (b_k = u h_k^2 / C^2 is invariant).
// b'_0 is computed at scale Delta; the initial guess's scale is chosen on the host so
// that the last h lands at s_final.
struct GoldPlan { std::vector<double> s_init; };

GoldPlan gold_plan(const he_ctx *C, int lh, int K, const std::vector<double> &s_final) {
    // scale factors of h through the K updates, independent of the starting scale
    const auto &q = C->q;
    const double D = C->Delta;
    double f = 1.0, sb = D, sr = D;
    int lr = lh - 2;
    f = f * sr / (double)q[lr];                     // h_1 = h_0 r_0 at level lh-2
    for (int k = 1; k < K; ++k) {
        const double s_r2 = sr * sr / (double)q[lr];  // r^2 at level lr-1
        sb = sb * s_r2 / (double)q[lr - 1];           // b' at level lr-2
        sr = sb;
        lr -= 2;
        f = f * sr / (double)q[lr];
    }
    GoldPlan g;
    for (double s : s_final) g.s_init.push_back(s / f);
    return g;
}

// h ~ C u^(-1/2): polynomial sum_k coef_k u^k (coefficients times C), then
// Newton steps h <- 1.5 h - (0.5/C^2) u h^3 or Goldschmidt updates; lands at
// scale s_final per ct.
Bt invsqr(Exec &X, const Bt &U, const std::vector<std::vector<double>> &coefC, const std::vector<double> &Cc,
          int newton, bool gold, const std::vector<double> &s_final) {
    const int R = U.cnt, d = (int)coefC[0].size() - 1, lu = U.level;
    const auto &q = X.C->q;
    std::vector<double> S(R);
    if (gold && newton > 0) {
        const int lh0 = lu - invsqr_depth(d, newton, true) + 2 * newton + 1;
        S = gold_plan(X.C, lh0, newton, s_final).s_init;
    } else {
        for (int r = 0; r < R; ++r) S[r] = newton == 0 ? s_final[r] : X.C->Delta;
    }
    auto col = [&](int k) { std::vector<double> v(R); for (int r = 0; r < R; ++r) v[r] = coefC[r][k]; return v; };
    Bt H;
    if (d == 1) {
        H = X.add_const(X.cmul(U, col(1), S, false), col(0));
    } else if (d == 2) {
        Bt U2 = X.mul(U, U);
        Bt T2 = X.cmul(U2, col(2), S, false);
        Bt T1 = X.cmul(X.drop(U, lu - 1), col(1), S, false);
        H = X.add_const(X.add(T2, T1), col(0));
    } else if (d == 3) {
        // two ciphertext products: u^2, then (g_3 u) u^2; g_2 u^2 and g_1 u are
        // constant multiplies landing on the same level
        Bt U2 = X.mul(U, U);
        std::vector<double> sA(R);
        for (int r = 0; r < R; ++r) sA[r] = (S[r] * (double)q[lu - 1]) / U2.scale[r];
        Bt T3 = X.mul(X.cmul(U, col(3), sA, false), U2);
        Bt T2 = X.cmul(U2, col(2), S, false);
        Bt T1 = X.cmul(X.drop(U, lu - 1), col(1), S, false);
        H = X.add_const(X.add(X.add(T3, T2), T1), col(0));
    } else if (d == 4) {
        Bt U2 = X.mul(U, U);
        std::vector<double> sC(R), sD(R);
        for (int r = 0; r < R; ++r) {
            sC[r] = (S[r] * (double)q[lu - 2]) / U2.scale[r];
            sD[r] = (S[r] * (double)q[lu - 2]) / U.scale[r];
        }
        Bt T4 = X.mul(X.cmul(U2, col(4), sC, false), X.drop(U2, lu - 2));
        Bt T3 = X.mul(X.cmul(U2, col(3), sD, false), X.drop(U, lu - 2));
        Bt T2 = X.cmul(X.drop(U2, lu - 2), col(2), S, false);
        Bt T1 = X.cmul(X.drop(U, lu - 2), col(1), S, false);
        H = X.add_const(X.add(X.add(X.add(T4, T3), T2), T1), col(0));
    } else {
        throw HeError(HE_EINVAL, "initial-guess degree must be 1..4");
    }
    if (gold && newton > 0) {
        const int lh = H.level;
        std::vector<double> sA(R), kap(R), c15(R, 1.5);
        Bt G2 = X.mul(H, H);
        for (int r = 0; r < R; ++r) {
            sA[r] = (X.C->Delta * (double)q[lh - 1]) / G2.scale[r];
            kap[r] = 0.5 / (Cc[r] * Cc[r]);
        }
        Bt Bp = X.mul(X.drop(X.cmul(U, kap, sA, false), lh - 1), G2);
        Bt Rk = X.add_const(X.mul_int(Bp, std::vector<int64_t>(R, -1)), c15);
        H = X.mul(X.drop(H, Rk.level), Rk);
        for (int it = 1; it < newton; ++it) {
            Bt R2 = X.mul(Rk, Rk);
            Bp = X.mul(X.drop(Bp, R2.level), R2);
            Rk = X.add_const(X.mul_int(Bp, std::vector<int64_t>(R, -1)), c15);
            H = X.mul(X.drop(H, Rk.level), Rk);
        }
        return H;
    }
    for (int it = 0; it < newton; ++it) {
        std::vector<double> St(R), sA(R), kap(R), c15(R, 1.5);
        for (int r = 0; r < R; ++r) St[r] = it == newton - 1 ? s_final[r] : X.C->Delta;
        const int lh = H.level;
        Bt G2 = X.mul(H, H);
        for (int r = 0; r < R; ++r) {
            sA[r] = (((St[r] * (double)q[lh]) * (double)q[lh - 1]) / H.scale[r]) / G2.scale[r];
            kap[r] = -0.5 / (Cc[r] * Cc[r]);
        }
        Bt A = X.drop(X.cmul(U, kap, sA, false), lh);
        Bt B = X.mul(A, H);
        Bt Tt = X.mul(B, G2);
        Bt L1 = X.drop(X.cmul(H, c15, St, false), lh - 2);
        H = X.add(Tt, L1);
    }
    return H;
}

struct CutmaxCfg {
    int T = 0;
    std::vector<int> p;
    std::vector<double> c, vlo, vhi;
    std::vector<std::vector<double>> coef;  // [T][d+1] unscaled g(u) ~ u^-1/2
    int newton = 0, gold_d = 3;
    bool gold_refine = false;
    double sum_lo = 1, sum_hi = 3;
    bool boot = false;              // bootstrap the normalised iterate when the chain runs short
    std::vector<double> guess_max;  // [T]: max of h(u) sqrt(u) / C over the declared domain
    // [T]: factor on iteration t's normalised iterate, 2^(-e/p_t), so that its output is
    // 2^(-e) times the plain one (vhi[t+1], vlo[t+1] or the sum bounds hold the scaled bounds)
    std::vector<double> gain;
    // scaled refinements (HE_REFINE_SCALED): per iteration the (a_k, b_k) of
    // x <- x (a_k - b_k x^2) and the K+1 ranges (l_k, h_k) of x
    bool scaled = false;
    std::vector<std::vector<std::pair<double, double>>> steps, ranges;
    int ksteps(int t) const { return scaled ? (int)steps[t].size() : 0; }
    // levels of the inverse square root of iteration t (guess and refinements)
    int inv_depth(int t) const;
};

// max over u in [u_lo, 1] of g(u) sqrt(u) after the refinement steps (1 for an exact
// inverse square root): the factor by which |z - 1| can exceed its exact bound
double guess_overshoot(const std::vector<double> &g, double u_lo, int newton) {
    double mx = 0.0;
    const double step = std::pow(1.0 / u_lo, 1.0 / 4000.0);
    double u = u_lo;
    for (int i = 0; i <= 4000; ++i, u = std::min(1.0, u * step)) {
        double y = 0.0;
        for (int k = (int)g.size() - 1; k >= 0; --k) y = y * u + g[k];
        for (int it = 0; it < newton; ++it) y = 1.5 * y - 0.5 * u * y * y * y;
        mx = std::max(mx, std::fabs(y) * std::sqrt(u));
    }
    return mx;
}

int CutmaxCfg::inv_depth(int t) const {
    const int d = (int)coef[t].size() - 1;
    if (scaled) return invsqr_depth(d, 0, false) + 2 * ksteps(t);
    return invsqr_depth(d, newton, gold_refine);
}

// levels an iteration needs before its normalised iterate; a scaled refinement under
// HE_BOOT bootstraps inside itself, so it needs the moments, the guess, W_0 and one level
// left for that bootstrap
int pre_levels(const CutmaxCfg &cf, int t) {
    if (cf.boot && cf.ksteps(t) > 0) return 2 + invsqr_depth((int)cf.coef[t].size() - 1, 0, false) + 3;
    return 2 + cf.inv_depth(t) + 1;
}
int power_levels(int p) {
    int nb = 0;
    while ((p >> nb) > 1) ++nb;
    return nb + (__builtin_popcount(p) > 1 ? 1 : 0);
}

int levels_needed(const CutmaxCfg &cf) {
    int lv = 0;
    for (int t = 0; t < cf.T; ++t) {
        int nb = 0;
        while ((cf.p[t] >> nb) > 1) ++nb;
        lv += 2 + cf.inv_depth(t) + 1 + nb + (__builtin_popcount(cf.p[t]) > 1 ? 1 : 0);
    }
    return lv + cf.gold_d + 3;
}

Bt bootstrap(Exec &X, const Bt &ct, double bound);
int boot_levels(const he_ctx *C);

// z = E h + 1 with h ~ C u^(-1/2) by the scaled refinements of the guess g (the wide-domain
// form), times the iterate's prescale gain (folded into C, and the 1 added is the gain):
// the guess twice from U, C g at the scale that puts Ey = E C g at Delta and
// sqrt(b_0) g at the scale that puts W = b_0 u g^2 = b_0 x_0^2 at Delta; per step
// r = a_k - W (no level), Ey <- Ey r, and unless it is the last step
// W <- (W b_{k+1}/b_k) r^2, the constant multiply landing at the scale that puts the new W
// at Delta (in parallel with r^2: two levels a step); z = Ey + gain.  Ey holds
// (y - mu)/(c sigma) x_k and W holds b_k x_k^2: neither spans the decades u^(-1/2) spans,
// so both can be bootstrapped (HE_BOOT) before a step when the chain runs short.
Bt scaled_normalise(Exec &X, const Bt &U, const Bt &E, const std::vector<Request> &reqs,
                    const std::vector<int> &first, const std::vector<int> &cmap, const CutmaxCfg &cf, int t) {
    he_ctx *C = X.C;
    const auto &q = C->q;
    const int R = (int)reqs.size(), K = cf.ksteps(t), d = (int)cf.coef[t].size() - 1;
    const auto &st = cf.steps[t];
    const auto &rg = cf.ranges[t];
    const int lg = U.level - invsqr_depth(d, 0, false);
    REQUIRE(lg - 2 >= 1, HE_EDEPTH, "chain too short for the refined inverse square root");
    std::vector<double> Cc(R), SH(R), SG(R), one(R, 1.0);
    std::vector<std::vector<double>> coefC(R), coefB(R);
    const double sb0 = std::sqrt(st[0].second);
    double ebound = 0.0;
    for (int r = 0; r < R; ++r) {
        Cc[r] = std::sqrt((double)reqs[r].n) / cf.c[t] * cf.gain[t];
        SH[r] = (C->Delta * (double)q[lg]) / E.scale[first[r]];
        SG[r] = std::sqrt(((C->Delta * (double)q[lg]) * (double)q[lg - 1]) / U.scale[r]);
        for (double g : cf.coef[t]) {
            coefC[r].push_back(g * Cc[r]);
            coefB[r].push_back(g * sb0);
        }
        ebound = std::max(ebound, std::sqrt((double)reqs[r].n - 1.0) / cf.c[t] * cf.gain[t]);
    }
    Bt H0 = invsqr(X, U, coefC, Cc, 0, false, SH);
    Bt G0 = invsqr(X, U, coefB, one, 0, false, SG);
    Bt Ey = X.mul(X.drop(E, lg), H0, &cmap);
    Bt W = X.mul(X.drop(U, lg - 1), X.mul(G0, G0));
    for (int k = 0; k < K; ++k) {
        // W must stay at level 1 or above for a later bootstrap: a step that produces the
        // next W takes two levels, the last step one (its Ey needs a level for the z
        // bootstrap before the power)
        const int need = k + 1 < K ? 3 : 2;
        if (W.level < need) {
            REQUIRE(cf.boot && C->boot.ready, HE_EDEPTH, "scaled refinement needs more levels than the chain has");
            // one bootstrap of W and Ey together: W times the integer m (no level) reaches
            // Ey's bound, and the output's scale times m gives W back, with the error W
            // alone would have had under its own bound
            const double bW = 1.02 * st[k].second * rg[k].second * rg[k].second;
            const double bE = 1.02 * ebound * rg[k].second;
            const int64_t m = std::max<int64_t>(1, (int64_t)std::floor(bE / bW));
            const Bt Wm = m > 1 ? X.mul_int(W, std::vector<int64_t>(R, m)) : W;
            const Bt Ed = X.drop(Ey, W.level);
            Bt J = X.new_bt(R + Ey.cnt, W.level);
            Bt jw = J, je = J;
            jw.cnt = R;
            jw.scale.assign(Wm.scale.begin(), Wm.scale.end());
            je.cnt = Ey.cnt;
            je.d = J.d + (long long)R * 2 * J.cap * C->N;
            je.scale.assign(Ed.scale.begin(), Ed.scale.end());
            for (int i = 0; i < R; ++i) J.scale[i] = Wm.scale[i];
            for (int i = 0; i < Ey.cnt; ++i) J.scale[R + i] = Ed.scale[i];
            if (X.go()) {
                launch_copy(X.T, X.vs_all(jw), X.vs_all(Wm), X.s);
                launch_copy(X.T, X.vs_all(je), X.vs_all(Ed), X.s);
            }
            const Bt B = bootstrap(X, J, std::max(bE, (double)m * bW));
            W = B;
            W.cnt = R;
            W.scale.assign(B.scale.begin(), B.scale.begin() + R);
            for (double &sc : W.scale) sc *= (double)m;
            Ey = B;
            Ey.cnt = (int)B.scale.size() - R;
            Ey.d = B.d + (long long)R * 2 * B.cap * C->N;
            Ey.scale.assign(B.scale.begin() + R, B.scale.end());
        }
        std::vector<double> ak(R, st[k].first);
        Bt Rk = X.add_const(X.mul_int(W, std::vector<int64_t>(R, -1)), ak);
        Ey = X.mul(X.drop(Ey, Rk.level), Rk, &cmap);
        if (k + 1 < K) {
            const int L = W.level;
            std::vector<double> sV(R), kap(R, st[k + 1].second / st[k].second);
            for (int r = 0; r < R; ++r)
                sV[r] = ((C->Delta * (double)q[L]) * (double)q[L - 1]) / (Rk.scale[r] * Rk.scale[r]);
            Bt V = X.cmul(W, kap, sV, false);
            W = X.mul(V, X.mul(Rk, Rk));
        }
    }
    return X.add_const(Ey, std::vector<double>(Ey.cnt, cf.gain[t]));
}

// Alg. 2 on a batch of requests; Y holds every request's ciphertexts.
// Masked padding: the pad slots of a request all hold one value, followed by a
// tracker ciphertext (appended after every request's ciphertexts) that takes the same
// steps; each slot sum subtracts npad x tracker and the variance sum npad x the
// tracker's square, so the moments are those of the first n slots.
Bt cutmax_sched(Exec &X, Bt Y, const std::vector<Request> &reqs, const CutmaxCfg &cf) {
    he_ctx *C = X.C;
    const int R = (int)reqs.size(), total = Y.cnt;
    std::vector<int> first(R), cnt(R), tmap(R, -1);
    std::vector<int64_t> npad(R, 0);
    int ntrk = 0;
    for (int r = 0; r < R; ++r)
        if (reqs[r].npad > 0) { tmap[r] = total + ntrk++; npad[r] = reqs[r].npad; }
    std::vector<int> cmap(total + ntrk);
    std::vector<int64_t> nct(total + ntrk);
    for (int r = 0; r < R; ++r) {
        first[r] = reqs[r].first; cnt[r] = reqs[r].a;
        for (int k = 0; k < reqs[r].a; ++k) { cmap[reqs[r].first + k] = r; nct[reqs[r].first + k] = reqs[r].n; }
        if (tmap[r] >= 0) { cmap[tmap[r]] = r; nct[tmap[r]] = reqs[r].n; }
    }
    // a chain with wider top primes (kept for bootstrapping) runs the schedule on the
    // levels whose primes match the scale
    if (C->n_hi > 0 && Y.level > C->L - C->n_hi) Y = X.drop(Y, C->L - C->n_hi);
    if (cf.boot) {
        REQUIRE(C->boot.ready, HE_ESTATE, "HE_BOOT needs he_boot_setup");
        REQUIRE(pre_levels(cf, 0) + 1 <= Y.level, HE_EDEPTH, "first iteration needs more levels than the ciphertext has");
    } else {
        REQUIRE(levels_needed(cf) <= Y.level, HE_EDEPTH, "schedule needs more levels than the ciphertext has");
    }
    if (ntrk) {
        // trackers start as trivial encryptions of the pad value (0 * ct + pad)
        Bt Ya = X.new_bt(total + ntrk, Y.level);
        for (int k = 0; k < total; ++k) Ya.scale[k] = Y.scale[k];
        Bt main = Ya;
        main.cnt = total;
        main.scale.resize(total);
        if (X.go()) launch_copy(X.T, X.vs_all(main), X.vs_all(Y), X.s);
        std::vector<int64_t> zero(ntrk, 0);
        Bt firsts = X.new_bt(ntrk, Y.level);
        for (int r = 0, i = 0; r < R; ++r)
            if (tmap[r] >= 0) {
                Bt src = Y, dst = firsts;
                src.d = Y.d + (long long)reqs[r].first * 2 * Y.cap * C->N;
                src.cnt = 1;
                dst.d = firsts.d + (long long)i * 2 * firsts.cap * C->N;
                dst.cnt = 1;
                firsts.scale[i] = Y.scale[reqs[r].first];
                if (X.go()) launch_copy(X.T, X.vs_all(dst), X.vs_all(src), X.s);
                ++i;
            }
        std::vector<double> pv;
        for (int r = 0; r < R; ++r)
            if (tmap[r] >= 0) pv.push_back(reqs[r].pad);
        Bt trk = X.add_const(X.mul_int(firsts, zero), pv);
        Bt tdst = Ya;
        tdst.d = Ya.d + (long long)total * 2 * Ya.cap * C->N;
        tdst.cnt = ntrk;
        for (int i = 0; i < ntrk; ++i) Ya.scale[total + i] = trk.scale[i];
        if (X.go()) launch_copy(X.T, X.vs_all(tdst), X.vs_all(trk), X.s);
        Y = Ya;
    }
    // the trackers of a batch, as a view into it (index tmap[r] - total)
    auto trackers = [&](const Bt &B) {
        Bt v = B;
        v.d = B.d + (long long)total * 2 * B.cap * C->N;
        v.cnt = ntrk;
        v.scale.assign(B.scale.begin() + total, B.scale.end());
        return v;
    };
    std::vector<int> tidx(R, -1);
    for (int r = 0; r < R; ++r) tidx[r] = tmap[r] >= 0 ? tmap[r] - total : -1;
    for (int t = 0; t < cf.T; ++t) {
        const size_t mark = C->arena.mark();
        Bt S = X.rotsum(X.sum_groups(Y, first, cnt));
        if (ntrk) S = X.sub_mul_map(S, trackers(Y), npad, tidx);
        Bt D = X.center(Y, S, cmap, nct);
        std::vector<double> kE(Y.cnt), dl(Y.cnt, C->Delta);
        for (int k = 0; k < Y.cnt; ++k) kE[k] = 1.0 / ((double)nct[k] * std::sqrt((double)nct[k] * cf.vhi[t]));
        Bt E = X.cmul(D, kE, dl, true);
        Bt U;
        if (ntrk) {
            // the pad slots' share npad F_R of the variance sum is formed as (sqrt(npad) E_R)^2:
            // the product's noise is then not multiplied by npad (up to 1.2e4 for 151936 logits
            // in 5 ciphertexts), as it would be in npad (E_R^2)
            Bt Em = E;
            Em.cnt = total;
            Em.scale.resize(total);
            const Bt Dt = trackers(D), Et = trackers(E);
            std::vector<double> kt(ntrk), st(ntrk);
            for (int r = 0; r < R; ++r)
                if (tmap[r] >= 0) {
                    kt[tidx[r]] = kE[tmap[r]] * std::sqrt((double)npad[r]);
                    st[tidx[r]] = Et.scale[tidx[r]];
                }
            Bt Ep = X.cmul(Dt, kt, st, false);
            Bt Ft = X.mul(Ep, Ep);
            Bt F = X.mul(Em, Em);
            U = X.sub_mul_map(X.rotsum(X.sum_groups(F, first, cnt)), Ft, std::vector<int64_t>(R, 1), tidx);
        } else {
            Bt F = X.mul(E, E);
            U = X.rotsum(X.sum_groups(F, first, cnt));
        }
        const int lh = U.level - (cf.ksteps(t) > 0 && cf.boot ? 0 : cf.inv_depth(t));
        REQUIRE(lh >= 1, HE_EDEPTH, "chain too short");
        std::vector<double> Cc(R), SH(R);
        std::vector<std::vector<double>> coefC(R);
        for (int r = 0; r < R; ++r) {
            Cc[r] = std::sqrt((double)reqs[r].n) / cf.c[t] * cf.gain[t];
            SH[r] = (C->Delta * (double)C->q[lh]) / E.scale[first[r]];
            for (double g : cf.coef[t]) coefC[r].push_back(g * Cc[r]);
        }
        Bt Yp;
        if (cf.ksteps(t) > 0) {
            Yp = scaled_normalise(X, U, E, reqs, first, cmap, cf, t);
        } else {
            Bt H = invsqr(X, U, coefC, Cc, cf.scaled ? 0 : cf.newton, cf.gold_refine, SH);
            Yp = X.add_const(X.mul(X.drop(E, H.level), H, &cmap), std::vector<double>(Y.cnt, cf.gain[t]));
        }
        if (cf.boot) {
            // bootstrap z when the power and the next iteration's moments (or the final
            // normalisation) do not fit; |z - 1| <= (max h sqrt(u) / C) sqrt(n - 1) / c
            const int need = power_levels(cf.p[t]) + (t + 1 < cf.T ? pre_levels(cf, t + 1) : cf.gold_d + 3);
            if (Yp.level < need) {
                REQUIRE(C->L - boot_levels(C) >= need, HE_EDEPTH, "bootstrapped chain too short for one iteration");
                double bound = 0.0;
                for (int r = 0; r < R; ++r)
                    bound = std::max(bound, 1.0 + cf.guess_max[t] * std::sqrt((double)reqs[r].n - 1.0) / cf.c[t]);
                Yp = bootstrap(X, Yp, 1.02 * bound * cf.gain[t]);
            }
        }
        Bt Yn = X.power(Yp, cf.p[t]);
        // keep the new iterate, drop this iteration's temporaries
        C->arena.release(mark);
        Bt Yk = X.new_bt(Yn.cnt, Yn.level);
        Yk.scale = Yn.scale;
        if (X.go()) launch_copy(X.T, X.vs_all(Yk), X.vs_all(Yn), X.s);
        // Yn's storage was released above but is only overwritten by later
        // allocations; the copy is enqueued before any of them
        Y = Yk;
    }
    std::vector<double> invB(total), dl(total, C->Delta), invBr(R), dlr(R, C->Delta);
    for (int k = 0; k < total; ++k) invB[k] = 1.0 / (cf.sum_hi * (double)nct[k]);
    for (int r = 0; r < R; ++r) invBr[r] = 1.0 / (cf.sum_hi * (double)reqs[r].n);
    Bt S = X.rotsum(X.sum_groups(Y, first, cnt));
    if (ntrk) {
        S = X.sub_mul_map(S, trackers(Y), npad, tidx);
        Y.cnt = total;  // the trackers are done
        Y.scale.resize(total);
    }
    Bt Xs = X.cmul(S, invBr, dlr, true);
    Bt E0 = X.add_const(X.mul_int(Xs, std::vector<int64_t>(R, -1)), std::vector<double>(R, 1.0));
    Bt P = X.add_const(E0, std::vector<double>(R, 1.0));
    Bt Ei = E0;
    for (int i = 0; i < cf.gold_d; ++i) {
        Ei = X.mul(Ei, Ei);
        P = X.mul(X.drop(P, Ei.level), X.add_const(Ei, std::vector<double>(R, 1.0)));
    }
    Bt Yb = X.cmul(Y, invB, dl, true);
    return X.mul(X.drop(Yb, P.level), P, &cmap);
}

// ------------------------------------------------------------ bootstrapping
void gen_keys(he_ctx *C, int from, int to = -1);
static void drop_graphs(he_ctx *C);
void dev_alloc(void **p, size_t bytes, const char *what);
template <class T>
void dev_alloc(T **p, size_t bytes, const char *what);

// NTT-domain residues [limbs][N] of integer polynomials m[k][N] in new device
// allocations (synchronous: set-up, outside any captured call)
std::vector<double *> upload_plains(he_ctx *C, const std::vector<std::vector<int64_t>> &m, int limbs) {
    const int N = C->N;
    std::vector<double *> out;
    int64_t *dm = nullptr;
    dev_alloc(&dm, 8ull * N * std::max<size_t>(1, m.size()), "device buffer");
    try {
        for (size_t k = 0; k < m.size(); ++k) {
            double *pt = nullptr;
            dev_alloc(&pt, 8ull * limbs * N, "device buffer");
            out.push_back(pt);
            HIPCHK(hipMemcpyAsync(dm + k * N, m[k].data(), 8ull * N, hipMemcpyHostToDevice, C->stream));
            const VecSet v{pt, limbs, limbs, 0, nullptr, nullptr};
            launch_int64_to_res(C->T, v, dm + k * N, 0, nullptr, C->stream);
            launch_ntt(C->T, v, false, C->ntt_variant, C->stream);
        }
        HIPCHK(hipStreamSynchronize(C->stream));
        HIPCHK(hipGetLastError());
    } catch (...) {
        hipFree(dm);
        for (double *p : out) hipFree(p);
        throw;
    }
    hipFree(dm);
    return out;
}

int gal_key_of(const he_ctx *C, uint64_t g) {
    auto it = C->gal_key.find(g);
    REQUIRE(it != C->gal_key.end(), HE_ESTATE, "no Galois key for a bootstrap rotation");
    return it->second;
}

uint64_t rot_gal(const he_ctx *C, long long a) {
    const uint64_t M = 2ull * C->N;
    uint64_t g = 1, b = 5;
    for (uint64_t e = (uint64_t)(a % C->slots + C->slots) % C->slots; e; e >>= 1, b = (b * b) % M)
        if (e & 1) g = (g * b) % M;
    return g;
}

uint64_t dbits(double x) { uint64_t u; std::memcpy(&u, &x, 8); return u; }

// sum_d D_d * rot_d(ct) by baby steps rot_{b h0}(ct) and giant steps
// rot_{a B h0}(sum_b rot_{-a B h0}(mult D_d) * rot_{b h0}(ct)), the diagonals encoded
// at rho q_l (l = the input level) and one rescale: output scale = scale * rho.
// The encoded diagonals are made in the dry pass (first use) and cached.
Bt lin_transform(Exec &X, const Bt &ct, const Diag &D, const Bsgs &P, double rho, int kind, int gi, double mult) {
    he_ctx *C = X.C;
    const int s = C->slots, l = ct.level, N = C->N;
    const double pscale = rho * (double)C->q[l];
    using Key = std::tuple<int, int, int, int, int, uint64_t, uint64_t>;
    auto key = [&](int a, int j) { return Key{kind, gi, a, j, l, dbits(pscale), dbits(mult)}; };
    if (X.dry) {
        std::vector<Key> want;
        std::vector<std::pair<int, int>> src;  // (shift, offset d)
        for (const auto &at : P.terms)
            for (size_t j = 0; j < at.second.size(); ++j)
                if (!C->pt_cache.count(key(at.first, (int)j))) {
                    want.push_back(key(at.first, (int)j));
                    src.push_back({(int)(((long long)at.first * P.B * P.h0) % s), at.second[j].second});
                }
        if (!want.empty()) {
            std::vector<std::vector<int64_t>> m(want.size(), std::vector<int64_t>(N));
            const int nth = (int)std::max<size_t>(1, std::min<size_t>(16, std::thread::hardware_concurrency()));
            std::vector<std::string> errs(nth);
            std::vector<std::thread> th;
            for (int w = 0; w < nth; ++w)
                th.emplace_back([&, w]() {
                    try {
                        std::vector<cplx> z(s);
                        for (size_t k = w; k < want.size(); k += nth) {
                            const std::vector<cplx> &dv = D.at(src[k].second);
                            const int sh = src[k].first;
                            // rot_{-shift}(D)[t] = D[t - shift], times the group's multiplier
                            for (int t = 0; t < s; ++t) z[t] = dv[((t - sh) % s + s) % s] * mult;
                            encode_cplx(z, N, pscale, m[k].data());
                        }
                    } catch (const std::exception &e) {
                        errs[w] = e.what();
                    }
                });
            for (auto &t : th) t.join();
            for (const auto &e : errs) REQUIRE(e.empty(), HE_ERANGE, "bootstrap diagonal: " + e);
            std::vector<double *> pts = upload_plains(C, m, l + 1);
            for (size_t k = 0; k < want.size(); ++k) C->pt_cache[want[k]] = pts[k];
        }
    }
    std::map<int, Bt> baby;
    baby[0] = ct;
    if (C->boot_hoist) {
        std::vector<std::pair<int, uint64_t>> rots;
        for (int b : P.babies()) {
            const uint64_t g = rot_gal(C, (long long)b * P.h0);
            rots.push_back({gal_key_of(C, g), g});
        }
        std::vector<Bt> bs = X.rotate_many(ct, rots);
        int i = 0;
        for (int b : P.babies()) baby[b] = bs[i++];
    } else {
        for (int b : P.babies()) {
            const uint64_t g = rot_gal(C, (long long)b * P.h0);
            baby[b] = X.rotate_gal(ct, gal_key_of(C, g), g);
        }
    }
    Bt acc;
    bool have = false;
    std::vector<Bt> rotated;                         // giant sums still to rotate (shared ModDown)
    std::vector<std::pair<int, uint64_t>> rot_keys;
    // with at most 8 babies and 8 giants every giant sum is computed in one pass
    std::map<int, Bt> fused;
    if (C->boot_hoist >= 1 && P.B <= kMaxLtBaby && (int)P.terms.size() <= kMaxLtGiant) {
        LtGiants lg{};
        lg.nb = P.B;
        for (int b = 0; b < P.B; ++b) {
            auto it = baby.find(b);
            const Bt &bx = it != baby.end() ? it->second : ct;
            lg.x[b] = bx.d;
            lg.xct[b] = 2LL * bx.cap * N;
            lg.xpoly[b] = (long long)bx.cap * N;
        }
        int gi = 0;
        for (const auto &at : P.terms) {
            Bt inner = X.new_bt(ct.cnt, l);
            for (int c = 0; c < ct.cnt; ++c) inner.scale[c] = ct.scale[c] * pscale;
            lg.out[gi] = inner.d;
            lg.oct = 2LL * inner.cap * N;
            lg.opoly = (long long)inner.cap * N;
            for (size_t j = 0; j < at.second.size(); ++j)
                lg.pt[gi][at.second[j].first] = X.dry ? nullptr : C->pt_cache.at(key(at.first, (int)j));
            fused[at.first] = inner;
            ++gi;
        }
        lg.ng = gi;
        if (X.go()) launch_lt_giants(X.T, lg, ct.cnt, l + 1, X.s);
    }
    for (const auto &at : P.terms) {
        const long long shift = ((long long)at.first * P.B * P.h0) % s;
        Bt inner = fused.count(at.first) ? fused[at.first] : X.new_bt(ct.cnt, l);
        for (int c = 0; c < ct.cnt; ++c) inner.scale[c] = ct.scale[c] * pscale;
        // chunks of at most kMaxLtTerms terms, summed
        const int nt = fused.count(at.first) ? 0 : (int)at.second.size();
        for (int j0 = 0; j0 < nt; j0 += kMaxLtTerms) {
            Bt part = j0 == 0 ? inner : X.new_bt(ct.cnt, l);
            part.scale = inner.scale;
            LtTerms tm{};
            tm.n = std::min(kMaxLtTerms, nt - j0);
            for (int j = 0; j < tm.n; ++j) {
                const Bt &bx = baby.at(at.second[j0 + j].first);
                double *pt = X.dry ? nullptr : C->pt_cache.at(key(at.first, j0 + j));
                tm.pt[j] = pt;
                tm.x[j] = bx.d;
                tm.xct[j] = 2LL * bx.cap * N;
                tm.xpoly[j] = (long long)bx.cap * N;
            }
            if (X.go())
                launch_lt_inner(X.T, part.d, 2LL * part.cap * N, (long long)part.cap * N, tm, ct.cnt, l + 1, X.s);
            if (j0) X.add_inplace(inner, part);
        }
        if (shift && C->boot_hoist >= 2) {
            const uint64_t g = rot_gal(C, shift);
            rotated.push_back(inner);
            rot_keys.push_back({gal_key_of(C, g), g});
            continue;
        }
        if (shift) {
            const uint64_t g = rot_gal(C, shift);
            if (have) X.rotate_gal(inner, gal_key_of(C, g), g, &acc);
            else acc = X.rotate_gal(inner, gal_key_of(C, g), g);
        } else {
            if (have) X.add_inplace(acc, inner);
            else acc = inner;
        }
        have = true;
    }
    // the rotated giant sums, up to 7 per key switch, one ModDown each
    for (size_t i = 0; i < rotated.size(); i += 7) {
        const size_t e = std::min(rotated.size(), i + 7);
        std::vector<Bt> xs(rotated.begin() + i, rotated.begin() + e);
        std::vector<std::pair<int, uint64_t>> ks(rot_keys.begin() + i, rot_keys.begin() + e);
        acc = X.rotate_sum_multi(xs, ks, have ? &acc : nullptr);
        have = true;
    }
    return X.rescale(acc);
}

// x brought to `level`, declared at `scale`, through one constant product
Bt boot_match(Exec &X, const Bt &x, int level, const std::vector<double> &scale) {
    return X.drop(X.cmul(x, std::vector<double>(x.cnt, 1.0), scale, false), level);
}

// sum_k c_k T_k(z) by baby-step giant-step (Paterson-Stockmeyer in the Chebyshev
// basis): babies T_1..T_7, giants T_8, T_16, .. (T_2k = 2 T_k^2 - 1, T_{m+n} = 2 T_m T_n -
// T_{m-n}); a polynomial of degree >= 8 is split at the largest power of two m <= its
// degree, p = q T_m + r with q_0 = c_m, q_j = 2 c_{m+j}, r_i = c_i - c_{2m-i}
// (T_{m+j} = 2 T_m T_j - T_{m-j}), and the parts are evaluated recursively; a part of
// degree < 8 is a sum of constant multiples of the babies.  Every part is produced at a
// prescribed level and scale, so the sums need no alignment; the result lands at level
// z.level - ceil(log2(deg + 1)) - 1 and scale s_out (the level a plain evaluation of the
// basis reaches), with 11 ciphertext products at degree 31 instead of 30.  Terms with
// |c_k| < 2^-40 (below the scale's noise) are left out.
struct ChebEval {
    Exec &X;
    int R;
    std::map<int, Bt> Tk;
    double eps = std::ldexp(1.0, -40);
    Bt basis(int k) {
        auto it = Tk.find(k);
        if (it != Tk.end()) return it->second;
        const std::vector<int64_t> two(R, 2);
        int m = 1;
        while (2 * m <= k) m *= 2;
        Bt out;
        if (m == k) {
            Bt h = basis(k / 2);
            out = X.add_const(X.mul_int(X.mul(h, h), two), std::vector<double>(R, -1.0));
        } else {
            Bt a = basis(m), b = basis(k - m), c = basis(2 * m - k);
            const int lm = std::min(a.level, b.level);
            Bt P = X.mul_int(X.mul(X.drop(a, lm), X.drop(b, lm)), two);
            Bt c1 = X.drop(X.cmul(c, std::vector<double>(R, 1.0), P.scale, false), P.level);
            out = X.add(P, c1, -1);
        }
        Tk[k] = out;
        return out;
    }
    // sum_i a_i T_i at `level` and scale S; false if every non-constant term vanished
    // (the value is then the constant a_0)
    bool eval(const std::vector<double> &a, int level, double S, Bt &out) {
        int deg = 0;
        for (int i = 1; i < (int)a.size(); ++i)
            if (std::fabs(a[i]) >= eps) deg = i;
        if (deg == 0) return false;
        const std::vector<double> sv(R, S);
        if (deg < 8) {
            // sum_i a_i T_i with one rescale: every T_i at level + 1 times the integer
            // round(a_i S q_{level+1} / s_i), summed (scale S q_{level+1}), rescaled to S
            std::vector<Bt> xs;
            std::vector<int64_t> K;
            const double q1 = (double)X.C->q[level + 1];
            for (int i = 1; i <= deg; ++i) {
                if (std::fabs(a[i]) < eps) continue;
                Bt Ti = basis(i);
                REQUIRE(Ti.level >= level + 1, HE_EDEPTH, "Chebyshev evaluation: baby step too deep");
                xs.push_back(X.drop(Ti, level + 1));
                for (int c = 0; c < R; ++c) {
                    const double k = ((a[i] * S) * q1) / Ti.scale[c];
                    REQUIRE(std::fabs(k) < 4.0e18, HE_ERANGE, "Chebyshev coefficient not encodable");
                    K.push_back(llround_d(k));
                }
            }
            out = X.rescale(X.lincomb(xs, K, S * q1));
            for (int c = 0; c < R; ++c) out.scale[c] = S;
            if (a[0] != 0.0) out = X.add_const(out, std::vector<double>(R, a[0]));
            return true;
        }
        int m = 8;
        while (2 * m <= deg) m *= 2;
        std::vector<double> q(deg - m + 1), r(m);
        q[0] = a[m];
        for (int j = 1; j <= deg - m; ++j) q[j] = 2.0 * a[m + j];
        for (int i = 0; i < m; ++i) r[i] = a[i] - (i >= 1 && 2 * m - i <= deg ? a[2 * m - i] : 0.0);
        Bt G = basis(m);
        REQUIRE(G.level >= level + 1, HE_EDEPTH, "Chebyshev evaluation: giant step too deep");
        Bt QT, Rp;
        Bt Gd = X.drop(G, level + 1);
        const double sq = (S * (double)X.C->q[level + 1]) / G.scale[0];
        if (eval(q, level + 1, sq, QT)) {
            QT = X.mul(QT, Gd);
            for (int c = 0; c < R; ++c) QT.scale[c] = S;  // (sq s_G) / q_{level+1} == S up to rounding
        } else {
            QT = X.drop(X.cmul(G, std::vector<double>(R, q[0]), sv, false), level);
        }
        if (eval(r, level, S, Rp)) out = X.add(QT, Rp);
        else out = r[0] != 0.0 ? X.add_const(QT, std::vector<double>(R, r[0])) : QT;
        return true;
    }
};

Bt cheb_sum(Exec &X, const Bt &z, const std::vector<double> &c, double s_out) {
    int lg = 0;
    while ((1 << lg) < (int)c.size()) ++lg;
    ChebEval E{X, z.cnt};
    E.Tk[1] = z;
    Bt out;
    REQUIRE(E.eval(c, z.level - lg - 1, s_out, out), HE_EINVAL, "EvalMod polynomial is constant");
    return out;
}

std::vector<double> eval_mod_coeffs(const he_ctx *C, double Bk) {
    const double a = 2.0 * M_PI * Bk / std::ldexp(1.0, C->boot.r);
    return cheb_interp([a](double z) { return std::cos(a * std::sqrt(std::max(0.0, (1.0 + z) / 2.0))); },
                       C->boot.cheb_deg);
}

// y = (x - 1/4) / Bk  ->  sin(2 pi x): z = 2 y^2 - 1, Chebyshev sum of
// cos(2 pi (x - 1/4) / 2^r), r double angles
Bt eval_mod(Exec &X, const Bt &y, double Bk) {
    const int R = y.cnt;
    const std::vector<int64_t> two(R, 2);
    const std::vector<double> m1(R, -1.0);
    Bt z = X.add_const(X.mul_int(X.mul(y, y), two), m1);
    Bt v = cheb_sum(X, z, eval_mod_coeffs(X.C, Bk), X.C->boot.s_eval);
    for (int i = 0; i < X.C->boot.r; ++i) v = X.add_const(X.mul_int(X.mul(v, v), two), m1);
    return v;
}

int boot_levels(const he_ctx *C) {
    int lg = 0;
    while ((1 << lg) < C->boot.cheb_deg + 1) ++lg;
    return C->boot.n_cts + 1 + lg + 1 + C->boot.r + C->boot.n_stc;
}

double boot_bk(const he_ctx *C) {
    const int h = C->secret_hw ? C->secret_hw : C->N;
    const int K = C->boot.K > 0 ? C->boot.K : (int)std::ceil(6.0 * std::sqrt(h / 12.0));
    return K + 0.5;
}

// a batch at level >= 1 with real slot values |v| <= bound, back at level
// L - boot_levels with the same values at scale Delta
Bt bootstrap_pass(Exec &X, const Bt &ct, double bound) {
    he_ctx *C = X.C;
    REQUIRE(C->boot.ready, HE_ESTATE, "bootstrap needs he_boot_setup");
    REQUIRE(ct.level >= 1, HE_EDEPTH, "bootstrap input needs a level to spare");
    REQUIRE(bound > 0 && std::isfinite(bound), HE_EINVAL, "bootstrap bound must be positive");
    const int R = ct.cnt, N = C->N;
    const double q0 = (double)C->q[0], Bk = boot_bk(C);
    // the bound rounded up to a power of 2^(1/8): the first SlotToCoeff group's encoded
    // diagonals depend on it, so the cache of encoded diagonals holds a few sets instead
    // of one per distinct bound (at most 9 % more noise than the exact bound)
    bound = std::exp2(std::ceil(std::log2(bound) * 8.0) / 8.0);
    const double s_in = q0 * std::ldexp(1.0, -C->boot.ratio_bits) / bound;
    // to level 0 at scale s_in; the raised plaintext m + q_0 I read at scale q_0 Bk
    Bt c0 = X.cmul(X.drop(ct, 1), std::vector<double>(R, 1.0), std::vector<double>(R, s_in), false);
    Bt U = X.modraise(c0, C->L, q0 * Bk);
    // CoeffToSlot: the slots become (w / (q_0 Bk)) / 2 in bit-reversed order
    const double rho_c = std::pow(C->boot.s_eval / U.scale[0], 1.0 / C->boot.n_cts);
    for (int gi = 0; gi < C->boot.n_cts; ++gi)
        U = lin_transform(X, U, C->boot.cts[gi], C->boot.cts_plan[gi], rho_c, 0, gi,
                          gi == C->boot.n_cts - 1 ? 0.5 : 1.0);
    const uint64_t conj = 2ull * N - 1;
    Bt V = X.rotate_gal(U, gal_key_of(C, conj), conj);
    // real and imaginary halves (times -i), stacked so EvalMod runs once for both
    Bt re = X.add(U, V), im = X.mul_plain(X.add(U, V, -1), C->mono_neg, 1.0);
    Bt Y2 = X.new_bt(2 * R, re.level);
    {
        Bt h0 = Y2, h1 = Y2;
        h0.cnt = R;
        h1.cnt = R;
        h1.d = Y2.d + 2LL * R * Y2.cap * N;
        for (int c = 0; c < R; ++c) { Y2.scale[c] = re.scale[c]; Y2.scale[R + c] = im.scale[c]; }
        if (X.go()) {
            launch_copy(X.T, X.vs_all(h0), X.vs_all(re), X.s);
            launch_copy(X.T, X.vs_all(h1), X.vs_all(im), X.s);
        }
    }
    Bt S = eval_mod(X, X.add_const(Y2, std::vector<double>(2 * R, -0.25 / Bk)), Bk);
    Bt Sre = S, Sim = S;
    Sre.cnt = R;
    Sre.scale.resize(R);
    Sim.cnt = R;
    Sim.d = S.d + 2LL * R * S.cap * N;
    Sim.scale.assign(S.scale.begin() + R, S.scale.end());
    Bt Z = X.add(Sre, X.mul_plain(Sim, C->mono_pos, 1.0));
    // SlotToCoeff, with kappa = q_0 / (2 pi s_in) turning sin(2 pi x) into m / s_in
    const double kappa = q0 / (2.0 * M_PI * s_in);
    const double rho_s = std::pow(C->Delta / Z.scale[0], 1.0 / C->boot.n_stc);
    for (int gi = 0; gi < C->boot.n_stc; ++gi)
        Z = lin_transform(X, Z, C->boot.stc[gi], C->boot.stc_plan[gi], rho_s, 1, gi, gi == 0 ? kappa : 1.0);
    return Z;
}

// With correct_bits = c > 0, a second pass bootstraps the first pass's error and removes
// it: b1 = BTS(x) = x + e1; d = x - b1 = -e1 (|e1| well below bound 2^-c); b2 = BTS(d) =
// -e1 + e2 with e2 in proportion to bound 2^-c; b1 + b2 = x + e2.
Bt bootstrap(Exec &X, const Bt &ct, double bound) {
    he_ctx *C = X.C;
    if (C->boot.correct_bits <= 0) return bootstrap_pass(X, ct, bound);
    const int lb = C->L - boot_levels(C);
    REQUIRE(ct.level >= 1 && ct.level < lb, HE_EDEPTH,
            "error-corrected bootstrap needs an input level between 1 and the output level - 1");
    Bt b1 = bootstrap_pass(X, ct, bound);
    // b1 at the input's scale and level (one constant product), then the residual
    Bt b1s = X.drop(X.cmul(b1, std::vector<double>(ct.cnt, 1.0), ct.scale, false), ct.level);
    Bt d = X.add(ct, b1s, -1);
    Bt b2 = bootstrap_pass(X, d, bound * std::ldexp(1.0, -C->boot.correct_bits));
    return X.add(b1, b2);
}

// every rotation amount (mod slots) of the two linear transforms, ascending
std::vector<int> boot_rotations(const he_ctx *C) {
    std::vector<int> r;
    for (const auto *pl : {&C->boot.cts_plan, &C->boot.stc_plan})
        for (const Bsgs &P : *pl)
            for (int a : P.rotations(C->slots))
                if (a) r.push_back(a);
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    return r;
}

void boot_setup(he_ctx *C, const he_boot_cfg *cfg) {
    REQUIRE(cfg, HE_EINVAL, "null bootstrap configuration");
    int lg = 0;
    while ((1 << lg) < C->slots) ++lg;
    REQUIRE(cfg->n_cts >= 1 && (int)cfg->n_cts <= lg && cfg->n_stc >= 1 && (int)cfg->n_stc <= lg, HE_EINVAL,
            "n_cts and n_stc must lie in [1, log2(slots)]");
    REQUIRE(cfg->cheb_deg >= 2 && cfg->cheb_deg <= 255 && cfg->r <= 8 && cfg->ratio_bits <= 40 && cfg->K <= 4096,
            HE_EINVAL, "bootstrap: cheb_deg in [2, 255], r <= 8, ratio_bits <= 40, K <= 4096");
    REQUIRE(cfg->log2_s_eval >= 20 && cfg->log2_s_eval <= 60, HE_EINVAL, "log2_s_eval in [20, 60]");
    auto &B = C->boot;
    B.ready = false;
    B.n_cts = (int)cfg->n_cts; B.n_stc = (int)cfg->n_stc; B.K = (int)cfg->K; B.ratio_bits = (int)cfg->ratio_bits;
    B.cheb_deg = (int)cfg->cheb_deg; B.r = (int)cfg->r; B.s_eval = std::ldexp(1.0, 0) * std::pow(2.0, cfg->log2_s_eval);
    REQUIRE(cfg->correct_bits <= 30, HE_EINVAL, "correct_bits at most 30");
    B.correct_bits = (int)cfg->correct_bits;
    REQUIRE(boot_levels(C) <= C->L - 1, HE_EINVAL, "bootstrap needs more levels than the chain has");
    // CoeffToSlot and EvalMod rescale by the primes of their levels while keeping the
    // scale near s_eval, so those primes must have about log2(s_eval) bits
    {
        int lg = 0;
        while ((1 << lg) < B.cheb_deg + 1) ++lg;
        const int top = B.n_cts + 1 + lg + 1 + B.r;
        for (int l = C->L; l > C->L - top; --l)
            REQUIRE(std::fabs(std::log2((double)C->q[l]) - cfg->log2_s_eval) < 1.0, HE_EINVAL,
                    "the primes of the levels CoeffToSlot and EvalMod use must have about log2_s_eval bits "
                    "(a chain with n_hi >= n_cts + 2 + ceil(log2(cheb_deg + 1)) + r primes of that size)");
    }
    B.cts = bt_groups(C->slots, B.n_cts, true);
    B.stc = bt_groups(C->slots, B.n_stc, false);
    B.cts_plan.clear();
    B.stc_plan.clear();
    for (const Diag &D : B.cts) B.cts_plan.push_back(bsgs_plan(D, C->slots));
    for (const Diag &D : B.stc) B.stc_plan.push_back(bsgs_plan(D, C->slots));
    // keys: rotation amounts with a key keep it; the others take the next indices in
    // ascending order of amount; the conjugation comes last
    const int from = (int)C->key_gal.size();
    for (int a : boot_rotations(C)) {
        const uint64_t g = rot_gal(C, a);
        if (C->gal_key.count(g)) continue;
        C->gal_key[g] = (int)C->key_gal.size();
        C->key_gal.push_back((uint32_t)g);
    }
    const uint64_t conj = 2ull * C->N - 1;
    if (!C->gal_key.count(conj)) {
        C->gal_key[conj] = (int)C->key_gal.size();
        C->key_gal.push_back((uint32_t)conj);
    }
    gen_keys(C, from);
    drop_graphs(C);
    for (auto &e : C->pt_cache) hipFree(e.second);
    C->pt_cache.clear();
    if (!C->mono_pos) {
        std::vector<std::vector<int64_t>> mono(2, std::vector<int64_t>(C->N, 0));
        mono[0][C->N / 2] = 1;
        mono[1][C->N / 2] = -1;
        std::vector<double *> pts = upload_plains(C, mono, C->L + 1);
        C->mono_pos = pts[0];
        C->mono_neg = pts[1];
    }
    B.ready = true;
}

// ---------------------------------------------------------------- helpers
void set_err(const std::string &m) { g_err = m; }

template <class F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const HeError &e) {
        set_err(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_err("host allocation failed");
        return HE_ENOMEM;
    } catch (const std::exception &e) {
        set_err(e.what());
        return HE_EINVAL;
    }
}

// captured graphs hold workspace and pool addresses: drop them when either moves
static void drop_graphs(he_ctx *C) {
    for (auto &g : C->graphs) hipGraphExecDestroy(g.second);
    C->graphs.clear();
}

// device allocation: out of memory is HE_ENOMEM (the error is cleared so that later
// calls do not see it), any other failure HE_EDEVICE
void dev_alloc(void **p, size_t bytes, const char *what) {
    *p = nullptr;
    const hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) return;
    *p = nullptr;
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory)
        throw HeError(HE_ENOMEM, std::string(what) + ": device out of memory for " + std::to_string(bytes >> 20) + " MiB");
    throw HeError(HE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
template <class T>
void dev_alloc(T **p, size_t bytes, const char *what) {
    void *v = nullptr;
    dev_alloc(&v, bytes, what);
    *p = (T *)v;
}

// device temporaries and events of one host function, released on every exit
// (exceptions included); hipFree waits for the work still using them
struct DevScope {
    std::vector<void *> mem;
    std::vector<hipEvent_t> ev;
    template <class T>
    T *alloc(size_t bytes, const char *what) {
        T *p = nullptr;
        dev_alloc(&p, bytes, what);
        mem.push_back(p);
        return p;
    }
    hipEvent_t event() {
        hipEvent_t e = nullptr;
        HIPCHK(hipEventCreate(&e));
        ev.push_back(e);
        return e;
    }
    ~DevScope() {
        for (hipEvent_t e : ev) hipEventDestroy(e);
        for (void *p : mem) hipFree(p);
    }
};

// frees the workspace and the constant pool (the next call allocates what it needs)
void free_workspace(he_ctx *C) {
    drop_graphs(C);
    if (C->arena.base) hipFree(C->arena.base);
    C->arena.base = nullptr;
    C->arena.cap = 0;
    Pool &P = C->pool;
    if (P.d_dv) hipFree(P.d_dv);
    if (P.d_iv) hipFree(P.d_iv);
    P.d_dv = nullptr;
    P.d_iv = nullptr;
    P.dcap = P.icap = 0;
}

void ensure_workspace(he_ctx *C) {
    Pool &P = C->pool;
    if (C->ws_limit > 0) {
        // checked after the dry pass, before any allocation or kernel of the call
        const size_t need = C->arena.peak + P.dv.size() * 8 + P.iv.size() * 4;
        if (need > C->ws_limit)
            throw HeError(HE_ENOMEM, "workspace limit: the call needs " + std::to_string((need + (1 << 20) - 1) >> 20) +
                                         " MiB, the limit is " + std::to_string(C->ws_limit >> 20) + " MiB");
    }
    if (C->arena.peak > C->arena.cap || P.dv.size() > P.dcap || P.iv.size() > P.icap)
        drop_graphs(C);
    if (C->arena.peak > C->arena.cap) {
        if (C->arena.base) HIPCHK(hipFree(C->arena.base));
        C->arena.base = nullptr;
        C->arena.cap = 0;
        size_t want = C->arena.peak + (64u << 20);
        // under a limit the slack (growth room for later calls) stays within it
        if (C->ws_limit > 0)
            want = std::max(C->arena.peak, std::min(want, C->ws_limit - (P.dv.size() * 8 + P.iv.size() * 4)));
        dev_alloc(&C->arena.base, want, "workspace");
        C->arena.cap = want;
    }
    if (P.dv.size() > P.dcap) {
        if (P.d_dv) HIPCHK(hipFree(P.d_dv));
        P.d_dv = nullptr;
        P.dcap = 0;
        const size_t want = C->ws_limit > 0 ? P.dv.size() : P.dv.size() * 2 + 1024;
        dev_alloc(&P.d_dv, want * 8, "constant pool");
        P.dcap = want;
    }
    if (P.iv.size() > P.icap) {
        if (P.d_iv) HIPCHK(hipFree(P.d_iv));
        P.d_iv = nullptr;
        P.icap = 0;
        const size_t want = C->ws_limit > 0 ? P.iv.size() : P.iv.size() * 2 + 1024;
        dev_alloc(&P.d_iv, want * 4, "constant pool");
        P.icap = want;
    }
    if (!P.dv.empty()) HIPCHK(hipMemcpyAsync(P.d_dv, P.dv.data(), P.dv.size() * 8, hipMemcpyHostToDevice, C->stream));
    if (!P.iv.empty()) HIPCHK(hipMemcpyAsync(P.d_iv, P.iv.data(), P.iv.size() * 4, hipMemcpyHostToDevice, C->stream));
}

// Static scratch of the entry point that allocates nothing (he_rotsum_noalloc): the
// whole workspace of one call (running sum, extended digits, the two key-product
// accumulators that carry c0 between steps, ModDown conversion) and its constants.  One
// ciphertext's rotate-and-sum at N = 2^16 needs about 215 MiB at the top level (30
// primes with 10 special primes).
// Each device holds its own copy, at the address hipGetSymbolAddress gives with that
// device current; host code uses only that address, never the array's name.
constexpr size_t kScratchBytes = 256ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_ptr;  // device ordinal -> address of its scratch

// once per device, with that device current (he_ctx_create)
void scratch_setup(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return;
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    REQUIRE(p != nullptr, HE_EDEVICE, "no address for the static scratch");
    g_scratch_ptr[device] = (unsigned char *)p;
}

unsigned char *scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    REQUIRE(it != g_scratch_ptr.end(), HE_ESTATE, "static scratch not set up on this device");
    return it->second;
}

// dry pass, upload, real pass
template <class Body>
void run2(he_ctx *C, Body &&body) {
    C->arena.dry = true; C->arena.top = 0; C->arena.peak = 0;
    C->pool.dry = true; C->pool.dv.clear(); C->pool.iv.clear(); C->pool.dpos = C->pool.ipos = 0;
    {
        Exec X(C, true);
        body(X);
    }
    ensure_workspace(C);
    C->arena.dry = false; C->arena.top = 0;
    C->pool.dry = false; C->pool.dpos = C->pool.ipos = 0;
    Exec X(C, false);
    body(X);
    HIPCHK(hipGetLastError());
}

he_ct *new_ct(he_ctx *C, uint32_t a) {
    auto *ct = new he_ct;
    ct->ctx = C;
    ct->a = a;
    const size_t words = (size_t)a * 2 * (C->L + 1) * C->N;
    hipError_t e = hipMalloc(&ct->d, words * 8);
    if (e != hipSuccess) { delete ct; throw HeError(HE_ENOMEM, "ciphertext allocation failed"); }
    return ct;
}

// view of a handle as a batch (cap = L+1)
Bt bt_of(const he_ct *ct) {
    Bt b;
    b.d = ct->d; b.cnt = (int)ct->a; b.level = (int)ct->level; b.cap = ct->ctx->L + 1;
    b.scale.assign(ct->a, ct->scale);
    return b;
}

void store_bt(Exec &X, const Bt &b, int first, he_ct *ct) {
    Bt dst = bt_of(ct);
    dst.level = b.level;
    Bt src = b;
    src.d = b.d + (long long)first * 2 * b.cap * X.C->N;
    src.cnt = (int)ct->a;
    if (!X.dry) launch_copy(X.T, X.vs_all(dst), X.vs_all(src), X.s);
    ct->level = (uint32_t)b.level;
    ct->scale = b.scale[first];
}

// --------------------------------------------------------- table building
struct TabBuilder {
    std::vector<double> dv;
    std::vector<int> iv;
    size_t d(const std::vector<double> &v) { size_t o = dv.size(); dv.insert(dv.end(), v.begin(), v.end()); return o; }
    size_t i(const std::vector<int> &v) { size_t o = iv.size(); iv.insert(iv.end(), v.begin(), v.end()); return o; }
};

void build_ctx(he_ctx *C, const he_params *prm) {
    const int N = C->N, L = C->L, A = C->alpha, np = C->np;
    C->q = gen_primes(C->logN, L + 1, (int)prm->q0_bits, (int)prm->q_bits, (int)prm->p_bits, A, (int)prm->n_hi,
                      (int)prm->hi_bits);
    const auto &q = C->q;
    TabBuilder tb;
    std::vector<double> pd(np), pinv(np), ninv(np), two32(np);
    std::vector<double> tw((size_t)np * N), itw((size_t)np * N);
    for (int i = 0; i < np; ++i) {
        pd[i] = (double)q[i];
        pinv[i] = 1.0 / pd[i];
        ninv[i] = (double)invmod_u((uint64_t)N % q[i], q[i]);
        two32[i] = (double)((1ull << 32) % q[i]);
        const uint64_t psi = find_psi(q[i], N), ipsi = invmod_u(psi, q[i]);
        std::vector<uint64_t> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (int k = 1; k < N; ++k) { pw[k] = mulmod_u(pw[k - 1], psi, q[i]); ipw[k] = mulmod_u(ipw[k - 1], ipsi, q[i]); }
        for (int k = 0; k < N; ++k) {
            int r = 0;
            for (int b = 0; b < C->logN; ++b) if ((k >> b) & 1) r |= 1 << (C->logN - 1 - b);
            tw[(size_t)i * N + k] = (double)pw[r];
            itw[(size_t)i * N + k] = (double)ipw[r];
        }
    }
    const size_t o_p = tb.d(pd), o_pinv = tb.d(pinv), o_tw = tb.d(tw), o_itw = tb.d(itw), o_ninv = tb.d(ninv),
                 o_two32 = tb.d(two32);
    // evaluation-key high plane: 1 byte per word above the low 32 bits for primes below
    // 2^40, else 2; each prime's beta_L rows of both polynomials contiguous
    C->khb_host.assign(np, 2);
    std::vector<int> khoff(np);
    size_t hoff = 0;
    for (int i = 0; i < np; ++i) {
        C->khb_host[i] = q[i] < (1ull << 40) ? 1 : 2;
        khoff[i] = (int)hoff;
        hoff += (size_t)C->khb_host[i] * 2 * N * C->betaL;
    }
    REQUIRE(hoff < (1ull << 31), HE_EINVAL, "key plane offsets exceed 32 bits");
    C->key_hi_bytes = hoff;
    const size_t o_khb = tb.i(C->khb_host), o_khoff = tb.i(khoff);
    std::vector<int> ident(np);
    for (int i = 0; i < np; ++i) ident[i] = i;
    const size_t o_ident = tb.i(ident);
    std::vector<int> pprime(A);
    for (int m = 0; m < A; ++m) pprime[m] = L + 1 + m;
    const size_t o_pprime = tb.i(pprime);
    // ModDown constants
    std::vector<double> phinv(A), phat((size_t)A * (L + 1)), Pinv(L + 1), pmod(np, 0.0);
    for (int m = 0; m < A; ++m) {
        const uint64_t pm = q[L + 1 + m];
        uint64_t v = 1;
        for (int b = 0; b < A; ++b) if (b != m) v = mulmod_u(v, q[L + 1 + b] % pm, pm);
        phinv[m] = (double)invmod_u(v, pm);
        for (int i = 0; i <= L; ++i) {
            uint64_t w = 1;
            for (int b = 0; b < A; ++b) if (b != m) w = mulmod_u(w, q[L + 1 + b] % q[i], q[i]);
            phat[(size_t)m * (L + 1) + i] = (double)w;
        }
    }
    for (int i = 0; i <= L; ++i) {
        uint64_t P = 1;
        for (int m = 0; m < A; ++m) P = mulmod_u(P, q[L + 1 + m] % q[i], q[i]);
        Pinv[i] = (double)invmod_u(P, q[i]);
        pmod[i] = (double)P;
    }
    const size_t o_phinv = tb.d(phinv), o_phat = tb.d(phat), o_Pinv = tb.d(Pinv), o_pmod = tb.d(pmod);
    C->pmod_h = pmod;
    std::vector<double> mds(A);
    for (int m = 0; m < A; ++m) {
        const uint64_t pm = q[L + 1 + m];
        mds[m] = (double)mulmod_u((uint64_t)ninv[L + 1 + m], (uint64_t)phinv[m], pm);
    }
    const size_t o_mds = tb.d(mds);
    std::vector<size_t> o_mrs(L + 1, 0), o_mrp(L + 1, 0), o_mri(L + 1, 0);
    for (int l = 1; l <= L; ++l) {
        std::vector<uint64_t> B(A + 1);
        B[0] = q[l];
        for (int m = 0; m < A; ++m) B[1 + m] = q[L + 1 + m];
        std::vector<double> sc(A + 1), ph((size_t)(A + 1) * l), iv(l);
        for (int k = 0; k <= A; ++k) {
            uint64_t v = 1;
            for (int b = 0; b <= A; ++b) if (b != k) v = mulmod_u(v, B[b] % B[k], B[k]);
            const int gk = k == 0 ? l : L + 1 + (k - 1);
            sc[k] = (double)mulmod_u((uint64_t)ninv[gk], invmod_u(v, B[k]), B[k]);
            for (int i = 0; i < l; ++i) {
                uint64_t w = 1;
                for (int b = 0; b <= A; ++b) if (b != k) w = mulmod_u(w, B[b] % q[i], q[i]);
                ph[(size_t)k * l + i] = (double)w;
            }
        }
        for (int i = 0; i < l; ++i) {
            uint64_t w = 1;
            for (int b = 0; b <= A; ++b) w = mulmod_u(w, B[b] % q[i], q[i]);
            iv[i] = (double)invmod_u(w, q[i]);
        }
        o_mrs[l] = tb.d(sc);
        o_mrp[l] = tb.d(ph);
        o_mri[l] = tb.d(iv);
    }
    // rescale: q_l^-1 mod q_i
    std::vector<double> qlinv((size_t)(L + 1) * (L + 1), 0.0);
    for (int l = 1; l <= L; ++l)
        for (int i = 0; i < l; ++i) qlinv[(size_t)l * (L + 1) + i] = (double)invmod_u(q[l] % q[i], q[i]);
    const size_t o_qlinv = tb.d(qlinv);
    // ModUp per level and digit
    std::vector<size_t> o_ext(L + 1), o_mus(L + 1), o_nas(L + 1), o_nap(L + 1);
    C->ndall.assign(L + 1, 0);
    std::vector<std::vector<size_t>> o_vinv(L + 1), o_qhat(L + 1), o_nds(L + 1), o_ndp(L + 1);
    C->ndcount.assign(L + 1, {});
    for (int l = 0; l <= L; ++l) {
        const int next = l + 1 + A, beta = (l + 1 + A - 1) / A;
        std::vector<int> ep(next);
        for (int t = 0; t < next; ++t) ep[t] = t <= l ? t : L + 1 + (t - l - 1);
        o_ext[l] = tb.i(ep);
        std::vector<double> mus(l + 1);
        for (int j = 0; j < beta; ++j) {
            const int lo = j * A, dl = std::min(A, l + 1 - lo);
            std::vector<double> vi(dl), qh((size_t)dl * next);
            for (int a = 0; a < dl; ++a) {
                const uint64_t qi = q[lo + a];
                uint64_t v = 1;
                for (int b = 0; b < dl; ++b) if (b != a) v = mulmod_u(v, q[lo + b] % qi, qi);
                vi[a] = (double)invmod_u(v, qi);
                mus[lo + a] = (double)mulmod_u((uint64_t)ninv[lo + a], (uint64_t)vi[a], qi);
                for (int t = 0; t < next; ++t) {
                    const uint64_t pt = q[ep[t]];
                    uint64_t w = 1;
                    for (int b = 0; b < dl; ++b) if (b != a) w = mulmod_u(w, q[lo + b] % pt, pt);
                    qh[(size_t)a * next + t] = (double)w;
                }
            }
            o_vinv[l].push_back(tb.d(vi));
            o_qhat[l].push_back(tb.d(qh));
            std::vector<int> ns, npr;
            for (int t = 0; t < next; ++t)
                if (!(t >= lo && t < lo + dl)) { ns.push_back(t); npr.push_back(ep[t]); }
            C->ndcount[l].push_back((int)ns.size());
            o_nds[l].push_back(tb.i(ns));
            o_ndp[l].push_back(tb.i(npr));
        }
        o_mus[l] = tb.d(mus);
        // converted limbs of all digits, listed prime by prime: the two or three limbs of one
        // prime are adjacent, so the NTT blocks of one column range that share its twiddle
        // row run back to back on one XCD and re-read the row from its L2
        std::vector<int> as, ap;
        for (int t = 0; t < next; ++t)
            for (int j = 0; j < beta; ++j) {
                const int lo = j * A, dl = std::min(A, l + 1 - lo);
                if (!(t >= lo && t < lo + dl)) { as.push_back(j * next + t); ap.push_back(ep[t]); }
            }
        C->ndall[l] = (int)as.size();
        o_nas[l] = tb.i(as);
        o_nap[l] = tb.i(ap);
    }
    // x-block orders of the hoisted rotate-and-sum steps: the automorphism by
    // g = 5^k (k = the step's smallest rotation) maps aligned 256-blocks onto aligned
    // 256-blocks; list the blocks orbit by orbit
    std::map<int, size_t> o_xord;
    if (C->hoist >= 1) {
        const int nb = N / 256;
        const uint64_t M = 2ull * N;
        auto brev = [&](uint64_t v) {
            uint64_t r = 0;
            for (int b = 0; b < C->logN; ++b) if ((v >> b) & 1) r |= 1ull << (C->logN - 1 - b);
            return r;
        };
        for (const auto &st : hoist_steps(C->slots, C->hoist)) {
            uint64_t g = 1, b5 = 5;
            for (uint64_t e = (uint64_t)st[0]; e; e >>= 1, b5 = (b5 * b5) % M)
                if (e & 1) g = (g * b5) % M;
            std::vector<int> bm(nb), order;
            for (int B = 0; B < nb; ++B) {
                const uint64_t t = (2 * brev((uint64_t)B * 256) + 1) * g % M;
                bm[B] = (int)(brev((t - 1) / 2) / 256);
            }
            std::vector<char> seen(nb, 0);
            for (int B = 0; B < nb; ++B)
                for (int x = B; !seen[x]; x = bm[x]) { seen[x] = 1; order.push_back(x); }
            o_xord[st[0]] = tb.i(order);
        }
    }
    std::vector<int> xid(std::max(1, N / 256));
    for (int B = 0; B < (int)xid.size(); ++B) xid[B] = B;
    const size_t o_xid = tb.i(xid);
    dev_alloc(&C->d_tab, tb.dv.size() * 8, "device buffer");
    dev_alloc(&C->d_itab, tb.iv.size() * 4, "device buffer");
    HIPCHK(hipMemcpy(C->d_tab, tb.dv.data(), tb.dv.size() * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(C->d_itab, tb.iv.data(), tb.iv.size() * 4, hipMemcpyHostToDevice));
    double *D = C->d_tab;
    int *I = C->d_itab;
    C->T = DevTables{N, C->logN, np, L, A, D + o_p, D + o_pinv, D + o_tw, D + o_itw, D + o_ninv, D + o_two32,
                     I + o_khb, I + o_khoff, C->khb_host.data()};
    C->ident = I + o_ident;
    C->pprime = I + o_pprime;
    C->phinv = D + o_phinv; C->phat = D + o_phat; C->Pinv = D + o_Pinv; C->pmod = D + o_pmod;
    C->qlinv = D + o_qlinv;
    C->md_scale = D + o_mds;
    C->mr_scale.assign(L + 1, nullptr);
    C->mr_phat.assign(L + 1, nullptr);
    C->mr_inv.assign(L + 1, nullptr);
    for (int l = 1; l <= L; ++l) {
        C->mr_scale[l] = D + o_mrs[l];
        C->mr_phat[l] = D + o_mrp[l];
        C->mr_inv[l] = D + o_mri[l];
    }
    C->mu_scale.resize(L + 1);
    for (int l = 0; l <= L; ++l) C->mu_scale[l] = D + o_mus[l];
    C->ndall_slot.resize(L + 1);
    C->ndall_prime.resize(L + 1);
    for (int l = 0; l <= L; ++l) {
        C->ndall_slot[l] = I + o_nas[l];
        C->ndall_prime[l] = I + o_nap[l];
    }
    for (const auto &kv : o_xord) C->xorder[kv.first] = I + kv.second;
    C->xorder_id = I + o_xid;
    C->ext_prime.resize(L + 1);
    C->vinv.assign(L + 1, {}); C->qhat.assign(L + 1, {}); C->ndslot.assign(L + 1, {}); C->ndprime.assign(L + 1, {});
    for (int l = 0; l <= L; ++l) {
        C->ext_prime[l] = I + o_ext[l];
        for (size_t j = 0; j < o_vinv[l].size(); ++j) {
            C->vinv[l].push_back(D + o_vinv[l][j]);
            C->qhat[l].push_back(D + o_qhat[l][j]);
            C->ndslot[l].push_back(I + o_nds[l][j]);
            C->ndprime[l].push_back(I + o_ndp[l][j]);
        }
    }
}

// Rotation amounts of the hoisted rotate-and-sum steps with radix 2^h over
// log2(slots) bits: step b covers bits [b, b + hb), hb = min(h, bits left), and
// rotates by r 2^b for r = 1 .. 2^hb - 1.
std::vector<std::vector<int>> hoist_steps(int slots, int h) {
    int lg = 0;
    while ((1 << lg) < slots) ++lg;
    std::vector<std::vector<int>> out;
    for (int b = 0; b < lg;) {
        const int hb = std::min(h, lg - b);
        std::vector<int> st;
        for (int r = 1; r < (1 << hb); ++r) st.push_back(r << b);
        out.push_back(st);
        b += hb;
    }
    return out;
}

// Key plan: index 0 relinearisation; 1 + e rotation by 2^e for every e <
// log2(slots); then, in step order, every other amount of the hoisted steps.
// The Galois element of a rotation by a slots is 5^a mod 2N.
void plan_rotation_keys(he_ctx *C) {
    int lg = 0;
    while ((1 << lg) < C->slots) ++lg;
    const uint64_t M = 2ull * C->N;
    auto gal = [M](int a) {
        uint64_t g = 1, b = 5;
        for (uint64_t e = (uint64_t)a; e; e >>= 1, b = (b * b) % M)
            if (e & 1) g = (g * b) % M;
        return (uint32_t)g;
    };
    C->rot_key.clear();
    C->gal_key.clear();
    C->key_gal.assign(1, 0u);
    for (int e = 0; e < lg; ++e) {
        C->rot_key[1 << e] = (int)C->key_gal.size();
        C->key_gal.push_back(gal(1 << e));
    }
    if (C->hoist >= 1)
        for (const auto &st : hoist_steps(C->slots, C->hoist))
            for (int a : st)
                if (!C->rot_key.count(a)) {
                    C->rot_key[a] = (int)C->key_gal.size();
                    C->key_gal.push_back(gal(a));
                }
}

// evaluation keys from index `from` on (key_gal[k]: 0 = relinearisation, else the
// Galois element), generated on the device; an existing key at such an index is replaced
void gen_keys(he_ctx *C, int from, int to) {
    const int N = C->N, np = C->np;
    const DevTables &T = C->T;
    hipStream_t s = C->stream;
    const int nkeys = (int)C->key_gal.size();
    if (to < 0 || to > nkeys) to = nkeys;
    if (from >= to) return;
    const size_t per = (size_t)np * N, kw = (size_t)C->betaL * 2 * per;
    DevScope tmp;
    int *dsmall = tmp.alloc<int>(sizeof(int) * N, "key generation");
    double *te = tmp.alloc<double>(8ull * per, "key generation");
    double *tg = tmp.alloc<double>(8ull * per, "key generation");
    double *tk = tmp.alloc<double>(8ull * kw, "key generation");  // one key as doubles, packed after generation
    const VecSet all_sk{C->d_sk, np, np, 0, nullptr, nullptr};
    C->keys.resize(nkeys, KeyRef{nullptr, nullptr});
    for (int k = from; k < to; ++k) {
        if (C->keys[k].lo) {
            HIPCHK(hipStreamSynchronize(s));
            hipFree(const_cast<uint32_t *>(C->keys[k].lo));
            hipFree(const_cast<uint8_t *>(C->keys[k].hi));
            C->keys[k] = KeyRef{nullptr, nullptr};
        }
        uint32_t *klo = nullptr;
        uint8_t *khi = nullptr;
        // each plane owned by the context as soon as it exists (freed with it on any failure)
        dev_alloc(&klo, 4ull * kw, "evaluation key");
        C->keys[k] = KeyRef{klo, nullptr};
        dev_alloc(&khi, C->key_hi_bytes, "evaluation key");
        C->keys[k].hi = khi;
        if (k == 0) launch_square_res(T, tg, C->d_sk, np, s);
        else {
            launch_automorph(T, VecSet{tg, np, np, 0, nullptr, nullptr}, all_sk, C->key_gal[k], s);
            C->gal_key[C->key_gal[k]] = k;
        }
        for (int j = 0; j < C->betaL; ++j) {
            const uint32_t oa = OBJ_KEY_A | ((uint32_t)k << 8) | (uint32_t)j;
            const uint32_t oe = OBJ_KEY_E | ((uint32_t)k << 8) | (uint32_t)j;
            double *kb = tk + (size_t)j * 2 * per, *ka = kb + per;
            const VecSet va{ka, np, np, 0, nullptr, nullptr}, ve{te, np, np, 0, nullptr, nullptr};
            launch_sample_uniform(T, va, C->seed, oa, nullptr, s);
            launch_ntt(T, va, false, 0, s);
            launch_sample_small(dsmall, N, C->seed, oe, 1, s);
            launch_small_to_res(T, ve, dsmall, nullptr, s);
            launch_ntt(T, ve, false, 0, s);
            const int lo = j * C->alpha, hi = std::min(lo + C->alpha, C->L + 1);
            launch_keyb(T, kb, ka, te, C->d_sk, tg, C->pmod, np, lo, hi, s);
        }
        launch_pack_key(T, tk, klo, khi, C->betaL, np, N, s);
    }
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
}

// secret key (dense ternary from one draw per coefficient, or sparse ternary placed
// on the host) and every evaluation key of the CutMax schedule
void keygen(he_ctx *C) {
    const int N = C->N, np = C->np;
    DevScope tmp;
    int *dsmall = tmp.alloc<int>(sizeof(int) * N, "secret key");
    dev_alloc(&C->d_sk, 8ull * np * N, "secret key");
    const VecSet all_sk{C->d_sk, np, np, 0, nullptr, nullptr};
    if (C->secret_hw > 0) {
        const std::vector<int> sk = sparse_secret(N, C->secret_hw, C->seed, OBJ_SKH);
        HIPCHK(hipMemcpyAsync(dsmall, sk.data(), sizeof(int) * N, hipMemcpyHostToDevice, C->stream));
    } else {
        launch_sample_small(dsmall, N, C->seed, OBJ_SK, 0, C->stream);
    }
    launch_small_to_res(C->T, all_sk, dsmall, nullptr, C->stream);
    launch_ntt(C->T, all_sk, false, 0, C->stream);
    HIPCHK(hipStreamSynchronize(C->stream));
    plan_rotation_keys(C);
    gen_keys(C, 0);
}

// NTT autotuner: times every schedule variant (workgroup width x pass-2 twiddle
// form, NTT_VARIANTS in all) of the forward + inverse transform on random residues at
// one batch size per bucket (about 4, 16, 64, 256, 1024 and 4096 vectors, whole groups of
// the chain's primes as the evaluator's batches are) and keeps the fastest per bucket
// (larger batches use the 4096 choice).  Every candidate's time is kept for
// he_ntt_tuning_report.  Runs once per process and ring degree.
constexpr int kTuneBuckets = 6;
int g_tuned_logN[2] = {0, 0};
int g_tuned_choice[2][8];
int g_tuned_count[2][kTuneBuckets];
double g_tuned_ms[2][kTuneBuckets][NTT_VARIANTS];

void autotune_ntt(he_ctx *C) {
    const int li = C->logN == 16 ? 1 : 0;
    if (!g_tuned_logN[li]) {
        const int target[kTuneBuckets] = {4, 16, 64, 256, 1024, 4096};
        const int N = C->N, grp = C->L + 1;
        DevScope tmp;
        double *buf = tmp.alloc<double>(8ull * target[kTuneBuckets - 1] * N, "NTT autotuner");
        const hipEvent_t a = tmp.event(), b = tmp.event();
        for (int ci = 0; ci < kTuneBuckets; ++ci) {
            const int g = std::min(target[ci], grp), cnt = (target[ci] / g) * g;
            g_tuned_count[li][ci] = cnt;
            const VecSet vs{buf, cnt, g, (long long)g * N, nullptr, nullptr};
            launch_sample_uniform(C->T, vs, 99, 0x7E000000u, nullptr, C->stream);
            double best = 1e30;
            int bestv = 3;
            for (int v = 1; v <= NTT_VARIANTS; ++v) {
                launch_ntt(C->T, vs, false, v, C->stream);
                launch_ntt(C->T, vs, true, v, C->stream);
                // the best of 3 trials of 4 transform pairs each (small batches vary from
                // run to run by a few microseconds)
                double vbest = 1e30;
                for (int trial = 0; trial < 3; ++trial) {
                    HIPCHK(hipEventRecord(a, C->stream));
                    for (int rep = 0; rep < 4; ++rep) {
                        launch_ntt(C->T, vs, false, v, C->stream);
                        launch_ntt(C->T, vs, true, v, C->stream);
                    }
                    HIPCHK(hipEventRecord(b, C->stream));
                    HIPCHK(hipEventSynchronize(b));
                    float ms = 0;
                    HIPCHK(hipEventElapsedTime(&ms, a, b));
                    vbest = std::min(vbest, ms / 4.0);
                }
                g_tuned_ms[li][ci][v - 1] = vbest;
                if (vbest < best) { best = vbest; bestv = v; }
            }
            g_tuned_choice[li][ci] = bestv;
        }
        for (int bk = kTuneBuckets; bk < 8; ++bk) g_tuned_choice[li][bk] = g_tuned_choice[li][kTuneBuckets - 1];
        g_tuned_logN[li] = 1;
    }
    for (int bk = 0; bk < 8; ++bk) set_ntt_tuning(C->logN, bk, g_tuned_choice[li][bk]);
}

// encryption of already-encoded integer plaintexts m[a][N] (host memory)
void encrypt_coeffs_impl(he_ctx *C, const int64_t *m, uint32_t a, double scale, he_ct *ct) {
    const int N = C->N, L = C->L;
    const size_t words = (size_t)a * N;
    run2(C, [&](Exec &X) {
        int64_t *dm = (int64_t *)C->arena.alloc(words * 8);
        double *mres = X.alloc_d((size_t)a * (L + 1) * N);
        double *e = X.alloc_d((size_t)(L + 1) * N);
        int *small = (int *)C->arena.alloc(sizeof(int) * N);
        if (X.dry) return;
        HIPCHK(hipMemcpyAsync(dm, m, words * 8, hipMemcpyHostToDevice, C->stream));
        const VecSet vm{mres, (int)a * (L + 1), L + 1, (long long)(L + 1) * N, nullptr, nullptr};
        launch_int64_to_res(C->T, vm, dm, N, nullptr, C->stream);
        launch_ntt(C->T, vm, false, C->ntt_variant, C->stream);
        for (uint32_t c = 0; c < a; ++c) {
            const uint32_t nonce = C->nonce + c;
            double *c0 = ct->d + (size_t)c * 2 * (L + 1) * N, *c1 = c0 + (size_t)(L + 1) * N;
            const VecSet v1{c1, L + 1, L + 1, 0, nullptr, nullptr};
            launch_sample_uniform(C->T, v1, C->seed, OBJ_ENC_A | (nonce & 0xFFFFFFu), nullptr, C->stream);
            launch_ntt(C->T, v1, false, C->ntt_variant, C->stream);
            const VecSet ve{e, L + 1, L + 1, 0, nullptr, nullptr};
            launch_sample_small(small, N, C->seed, OBJ_ENC_E | (nonce & 0xFFFFFFu), 1, C->stream);
            launch_small_to_res(C->T, ve, small, nullptr, C->stream);
            launch_ntt(C->T, ve, false, C->ntt_variant, C->stream);
            launch_encfinish(C->T, c0, c1, e, mres + (size_t)c * (L + 1) * N, C->d_sk, 0, L + 1, 1, 0, 0, C->stream);
        }
    });
    HIPCHK(hipStreamSynchronize(C->stream));
    C->nonce += a;
    ct->level = (uint32_t)L;
    ct->scale = scale;
}

CutmaxCfg parse_cfg(he_ctx *C, const he_cutmax_cfg *cfg) {
    REQUIRE(cfg && cfg->T >= 1 && cfg->T <= 64 && cfg->p && cfg->c && cfg->var_lo && cfg->var_hi, HE_EINVAL,
            "cutmax cfg: T, p, c, var_lo, var_hi are required");
    CutmaxCfg cf;
    cf.T = (int)cfg->T;
    const int d = cfg->init_degree ? (int)cfg->init_degree : 3;
    REQUIRE(d >= 1 && d <= 4, HE_EINVAL, "init_degree must be 1..4");
    for (int t = 0; t < cf.T; ++t) {
        REQUIRE(cfg->p[t] >= 1 && cfg->p[t] <= 255, HE_EINVAL, "p out of range");
        REQUIRE(cfg->c[t] > 0 && cfg->var_hi[t] > 0 && cfg->var_lo[t] > 0 && cfg->var_lo[t] < cfg->var_hi[t],
                HE_EINVAL, "c and the variance domain must be positive with var_lo < var_hi");
        cf.p.push_back((int)cfg->p[t]);
        cf.c.push_back(cfg->c[t]);
        cf.vlo.push_back(cfg->var_lo[t]);
        cf.vhi.push_back(cfg->var_hi[t]);
        std::vector<double> g(d + 1);
        if (cfg->init_coef) for (int k = 0; k <= d; ++k) g[k] = cfg->init_coef[t * (d + 1) + k];
        else chebyshev_invsqrt_fit(cfg->var_lo[t] / cfg->var_hi[t], d, g.data());
        cf.coef.push_back(g);
    }
    cf.newton = (int)cfg->newton_steps;
    cf.gold_refine = (cfg->flags & HE_REFINE_GOLDSCHMIDT) != 0;
    cf.gold_d = (int)cfg->gold_d;
    REQUIRE(cfg->sum_hi > 0 && cfg->sum_lo >= 0 && cfg->sum_lo < cfg->sum_hi, HE_EINVAL, "bad sum domain");
    cf.sum_lo = cfg->sum_lo;
    cf.sum_hi = cfg->sum_hi;
    cf.boot = (cfg->flags & HE_BOOT) != 0;
    cf.scaled = (cfg->flags & HE_REFINE_SCALED) != 0;
    if (cf.scaled) {
        REQUIRE(cfg->ref_steps && cfg->ref_range && !cf.gold_refine, HE_EINVAL,
                "HE_REFINE_SCALED needs ref_steps and ref_range (and excludes HE_REFINE_GOLDSCHMIDT)");
        size_t ic = 0, ir = 0;
        cf.steps.resize(cf.T);
        cf.ranges.resize(cf.T);
        for (int t = 0; t < cf.T; ++t) {
            const int K = (int)cfg->ref_steps[t];
            REQUIRE(K >= 0 && K <= 16 && (K == 0 || cfg->ref_coef), HE_EINVAL, "ref_steps: 0..16 per iteration");
            for (int k = 0; k < K; ++k, ic += 2) {
                const double a = cfg->ref_coef[ic], b = cfg->ref_coef[ic + 1];
                REQUIRE(std::isfinite(a) && std::isfinite(b) && b > 0 && a > 0, HE_EINVAL, "ref_coef: a, b > 0");
                cf.steps[t].push_back({a, b});
            }
            for (int k = 0; k <= K; ++k, ir += 2) {
                const double l = cfg->ref_range[ir], h = cfg->ref_range[ir + 1];
                // (a plan converged to double precision gives l == h)
                REQUIRE(std::isfinite(l) && std::isfinite(h) && l > 0 && l <= h, HE_EINVAL, "ref_range: 0 < l <= h");
                cf.ranges[t].push_back({l, h});
            }
        }
    }
    // CutMax is unchanged when its iterate is multiplied by a positive constant (the next
    // moments' normalisation or the final division removes it), while deep schedules reach
    // variances near 1e12 (p = 16 after the first iteration), whose 1 / (n sqrt(n v)) lies
    // below the 1/q that one constant multiply resolves.  Iteration t's output is therefore
    // prescaled by 2^(-e), e the least exponent that brings the next variance bound under
    // 2^8 (the mean bound under 2^4 before the final division), through the factor
    // 2^(-e/p) on the normalised iterate before the power: no level, and bounds already
    // that small keep e = 0 and the plain arithmetic.
    cf.gain.assign(cf.T, 1.0);
    for (int t = 0; t < cf.T; ++t) {
        int e = 0;
        if (t + 1 < cf.T) {
            while (std::ldexp(cf.vhi[t + 1], -2 * e) > 256.0) ++e;
            cf.vhi[t + 1] = std::ldexp(cf.vhi[t + 1], -2 * e);
            cf.vlo[t + 1] = std::ldexp(cf.vlo[t + 1], -2 * e);
        } else {
            while (std::ldexp(cf.sum_hi, -e) > 16.0) ++e;
            cf.sum_hi = std::ldexp(cf.sum_hi, -e);
            cf.sum_lo = std::ldexp(cf.sum_lo, -e);
        }
        if (e > 0) cf.gain[t] = std::pow(2.0, -(double)e / (double)cf.p[t]);
    }
    // (host work on every call, so only where a bootstrap bound needs it)
    for (int t = 0; t < cf.T; ++t) {
        if (cf.ksteps(t) > 0) cf.guess_max.push_back(cf.ranges[t].back().second);
        else cf.guess_max.push_back(cf.boot ? guess_overshoot(cf.coef[t], cf.vlo[t] / cf.vhi[t], cf.scaled ? 0 : cf.newton)
                                            : 1.0);
    }
    (void)C;
    return cf;
}

// runs CutMax over the requests (optionally after the nucleus noise add)
int cutmax_impl(he_ctx *C, he_ct *const *in, he_ct *const *noise, size_t batch, const he_cutmax_cfg *cfg,
                double temperature, he_ct **out) {
    REQUIRE(C && in && out && batch >= 1, HE_EINVAL, "null argument");
    CutmaxCfg cf = parse_cfg(C, cfg);
    std::vector<Request> reqs;
    int total = 0;
    int level = -1;
    for (size_t r = 0; r < batch; ++r) {
        REQUIRE(in[r] && in[r]->ctx == C, HE_ESTATE, "ciphertext from another context");
        if (noise) REQUIRE(noise[r] && noise[r]->ctx == C && noise[r]->a == in[r]->a, HE_ESTATE, "noise mismatch");
        if (level < 0) level = (int)in[r]->level;
        REQUIRE((int)in[r]->level == level, HE_ESTATE, "requests at different levels");
        Request q{total, (int)in[r]->a, (int64_t)in[r]->a * C->slots};
        // masked padding for a zero-padded request (a replicated one has exact moments)
        const int64_t nr = (int64_t)in[r]->n;
        const bool replicated = in[r]->a == 1 && nr >= 1 && nr <= C->slots && C->slots % nr == 0;
        if ((cfg->flags & HE_MASK_PAD) && !replicated && nr >= 1 && nr < q.n) {
            q.npad = q.n - nr;
            q.n = nr;
            q.pad = in[r]->pad;
        }
        reqs.push_back(q);
        total += (int)in[r]->a;
    }
    const bool prescaled = cfg->flags & HE_NOISE_PRESCALED;
    std::vector<he_ct *> outs(batch, nullptr);
    try {
        for (size_t r = 0; r < batch; ++r) {
            outs[r] = new_ct(C, in[r]->a);
            outs[r]->n = in[r]->n;
        }
        hipEvent_t e0 = C->ev0, e1 = C->ev1;
        // the kernel sequence of the schedule depends only on the structure of the
        // call (constants are read from the pool at run time), so a captured graph
        // replays any later call with the same structure and workspace
        const bool use_graph = C->use_graph && !g_kprof;
        std::string gkey;
        if (use_graph) {
            gkey = "L" + std::to_string(level) + (noise ? (prescaled ? "np" : "nt") : "") + "T" +
                   std::to_string(cf.T) + "n" + std::to_string(cf.newton) + (cf.gold_refine ? "G" : "") + "g" + std::to_string(cf.gold_d);
            // bootstrapped calls read encoded diagonals chosen by the bound (n, c, guess)
            if (cf.boot) {
                char b[64];
                gkey += "B";
                for (int t = 0; t < cf.T; ++t) {
                    std::snprintf(b, sizeof b, "c%.17g/%.17g/%.17g", cf.c[t], cf.guess_max[t], cf.gain[t]);
                    gkey += b;
                }
                for (auto &r : reqs) gkey += "n" + std::to_string(r.n);
            }
            for (auto &r : reqs) gkey += "a" + std::to_string(r.a) + (r.npad > 0 ? "m" : "");
            for (int t = 0; t < cf.T; ++t)
                gkey += "p" + std::to_string(cf.p[t]) + "d" + std::to_string(cf.coef[t].size());
            // scaled refinements: their step counts fix the launches, and under HE_BOOT their
            // ranges fix the bootstrap bounds
            if (cf.scaled) {
                char b[64];
                for (int t = 0; t < cf.T; ++t) {
                    gkey += "k" + std::to_string(cf.ksteps(t));
                    if (cf.boot)
                        for (int k = 0; k < cf.ksteps(t); ++k) {
                            std::snprintf(b, sizeof b, "/%.17g:%.17g", cf.steps[t][k].second, cf.ranges[t][k].second);
                            gkey += b;
                        }
                }
            }
        }
        run2(C, [&](Exec &X) {
            Bt Y = X.new_bt(total, level);
            Bt G;
            if (noise) G = X.new_bt(total, level);
            for (size_t r = 0; r < batch; ++r) {
                Bt src = bt_of(in[r]);
                Bt dst = Y;
                dst.d = Y.d + (long long)reqs[r].first * 2 * Y.cap * C->N;
                dst.cnt = (int)in[r]->a;
                for (int k = 0; k < dst.cnt; ++k) Y.scale[reqs[r].first + k] = in[r]->scale;
                if (!X.dry) launch_copy(X.T, X.vs_all(dst), X.vs_all(src), X.s);
                if (noise) {
                    Bt gs = bt_of(noise[r]);
                    Bt gd = G;
                    gd.d = G.d + (long long)reqs[r].first * 2 * G.cap * C->N;
                    gd.cnt = dst.cnt;
                    REQUIRE(noise[r]->level == (uint32_t)level, HE_ESTATE, "noise level mismatch");
                    for (int k = 0; k < dst.cnt; ++k) G.scale[reqs[r].first + k] = noise[r]->scale;
                    if (!X.dry) launch_copy(X.T, X.vs_all(gd), X.vs_all(gs), X.s);
                }
            }
            if (!X.dry) HIPCHK(hipEventRecord(e0, X.s));
            hipGraphExec_t gexec = nullptr;
            bool capture = false;
            std::string key;
            if (!X.dry && use_graph) {
                char ptrs[96];
                std::snprintf(ptrs, sizeof ptrs, "@%p/%p/%p", (void *)C->arena.base, (void *)C->pool.d_dv,
                              (void *)C->pool.d_iv);
                key = gkey + ptrs;
                auto it = C->graphs.find(key);
                if (it != C->graphs.end()) {
                    gexec = it->second;
                    X.quiet = true;
                } else {
                    capture = true;
                    HIPCHK(hipStreamBeginCapture(X.s, hipStreamCaptureModeRelaxed));
                }
            }
            Bt Z;
            try {
                if (noise) {
                    if (prescaled) {
                        Y = X.add(Y, G);
                    } else {
                        std::vector<double> tau(total, temperature);
                        Bt Gs = X.cmul(G, tau, Y.scale, false);
                        Y = X.add(X.drop(Y, Gs.level), Gs);
                    }
                }
                Z = cutmax_sched(X, Y, reqs, cf);
            } catch (...) {
                if (capture) {
                    hipGraph_t g = nullptr;
                    hipStreamEndCapture(X.s, &g);
                    if (g) hipGraphDestroy(g);
                }
                throw;
            }
            if (capture) {
                hipGraph_t g = nullptr;
                HIPCHK(hipStreamEndCapture(X.s, &g));
                HIPCHK(hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0));
                hipGraphDestroy(g);
                C->graphs[key] = gexec;
            }
            if (gexec) {
                X.quiet = false;
                HIPCHK(hipGraphLaunch(gexec, X.s));
            }
            if (!X.dry) HIPCHK(hipEventRecord(e1, X.s));
            for (size_t r = 0; r < batch; ++r) store_bt(X, Z, reqs[r].first, outs[r]);
        });
        HIPCHK(hipStreamSynchronize(C->stream));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, C->ev0, C->ev1));
        C->last_ms = ms;
    } catch (...) {
        for (auto *o : outs) if (o) { hipFree(o->d); delete o; }
        throw;
    }
    for (size_t r = 0; r < batch; ++r) out[r] = outs[r];
    return HE_OK;
}

// evaluator primitive on a single ciphertext, or (multi) on every ciphertext of a
// handle independently
template <class F>
int prim(he_ctx *C, const he_ct *a, he_ct **out, F &&f, bool multi = false) {
    return guarded([&]() {
        REQUIRE(C && a && out && a->ctx == C, HE_EINVAL, "null or foreign argument");
        REQUIRE(a->a == 1 || multi, HE_EINVAL, "primitive ops take single ciphertexts");
        he_ct *o = new_ct(C, a->a);
        o->n = a->n;
        try {
            run2(C, [&](Exec &X) {
                Bt r = f(X);
                store_bt(X, r, 0, o);
            });
            HIPCHK(hipStreamSynchronize(C->stream));
        } catch (...) {
            hipFree(o->d);
            delete o;
            throw;
        }
        *out = o;
        return HE_OK;
    });
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

const char *he_last_error(void) { return g_err.c_str(); }

int he_ctx_create(const he_params *prm, he_ctx **out) {
    return guarded([&]() {
        REQUIRE(prm && out, HE_EINVAL, "null argument");
        REQUIRE(prm->log_n == 12 || prm->log_n == 16, HE_EINVAL, "log_n must be 12 or 16");
        REQUIRE(prm->n_q >= 2 && prm->n_q <= 48 && prm->dnum >= 1, HE_EINVAL, "n_q in [2,48], dnum >= 1");
        REQUIRE(prm->q0_bits >= 20 && prm->q0_bits <= 48 && prm->q_bits >= 20 && prm->q_bits <= 48 &&
                    prm->p_bits >= 20 && prm->p_bits <= 48,
                HE_EINVAL, "prime sizes must lie in [20, 48] bits");
        REQUIRE(prm->log2_scale >= 10 && prm->log2_scale <= 60, HE_EINVAL, "log2_scale out of range");
        auto C = std::make_unique<he_ctx>();
        C->logN = (int)prm->log_n;
        C->N = 1 << C->logN;
        C->slots = C->N / 2;
        C->L = (int)prm->n_q - 1;
        C->dnum = (int)prm->dnum;
        C->alpha = ((int)prm->n_q + C->dnum - 1) / C->dnum;
        C->np = (int)prm->n_q + C->alpha;
        REQUIRE(C->np <= kMaxPrimes && C->alpha <= 15, HE_EINVAL, "too many primes (alpha <= 15)");
        C->betaL = ((int)prm->n_q + C->alpha - 1) / C->alpha;
        REQUIRE(C->betaL <= 8, HE_EINVAL, "at most 8 digits");
        REQUIRE(prm->hoist <= 4, HE_EINVAL, "hoist must be 0..4");
        C->hoist = (int)prm->hoist;
        REQUIRE(prm->n_hi < prm->n_q && (prm->n_hi == 0 || (prm->hi_bits >= 20 && prm->hi_bits <= 48)), HE_EINVAL,
                "n_hi < n_q and hi_bits in [20, 48]");
        REQUIRE(prm->secret_hw <= (1u << prm->log_n), HE_EINVAL, "secret_hw at most N");
        C->n_hi = (int)prm->n_hi;
        C->secret_hw = (int)prm->secret_hw;
        C->Delta = std::ldexp(1.0, 0) * std::pow(2.0, prm->log2_scale);
        C->seed = prm->seed;
        C->device = prm->device;
        int ndev = 0;
        HIPCHK(hipGetDeviceCount(&ndev));
        REQUIRE(ndev > 0, HE_EDEVICE, "no HIP device");
        REQUIRE(prm->device >= 0 && prm->device < ndev, HE_EINVAL, "bad device ordinal");
        HIPCHK(hipSetDevice(prm->device));
        scratch_setup(prm->device);
        if (prm->stream) C->stream = (hipStream_t)prm->stream;
        else { HIPCHK(hipStreamCreateWithFlags(&C->stream, hipStreamNonBlocking)); C->own_stream = true; }
        HIPCHK(hipEventCreate(&C->ev0));
        HIPCHK(hipEventCreate(&C->ev1));
        build_ctx(C.get(), prm);
        autotune_ntt(C.get());
        keygen(C.get());
        *out = C.release();
        return HE_OK;
    });
}

void he_ctx_destroy(he_ctx *C) {
    if (!C) return;
    hipSetDevice(C->device);
    if (C->stream) hipStreamSynchronize(C->stream);
    for (auto &g : C->graphs) hipGraphExecDestroy(g.second);
    for (const KeyRef &k : C->keys) {
        hipFree(const_cast<uint32_t *>(k.lo));
        hipFree(const_cast<uint8_t *>(k.hi));
    }
    hipFree(C->d_sk); hipFree(C->d_tab); hipFree(C->d_itab);
    for (auto &e : C->pt_cache) hipFree(e.second);
    if (C->mono_pos) hipFree(C->mono_pos);
    if (C->mono_neg) hipFree(C->mono_neg);
    if (C->arena.base) hipFree(C->arena.base);
    if (C->pool.d_dv) hipFree(C->pool.d_dv);
    if (C->pool.d_iv) hipFree(C->pool.d_iv);
    if (C->ev0) hipEventDestroy(C->ev0);
    if (C->ev1) hipEventDestroy(C->ev1);
    if (C->own_stream) hipStreamDestroy(C->stream);
    delete C;
}

int he_ctx_info(const he_ctx *C, uint32_t *N, uint32_t *slots, uint32_t *L, uint32_t *alpha, uint64_t *primes) {
    if (!C) { g_err = "null context"; return HE_EINVAL; }
    if (N) *N = (uint32_t)C->N;
    if (slots) *slots = (uint32_t)C->slots;
    if (L) *L = (uint32_t)C->L;
    if (alpha) *alpha = (uint32_t)C->alpha;
    if (primes) std::memcpy(primes, C->q.data(), 8 * C->q.size());
    return HE_OK;
}

int he_encrypt_coeffs(he_ctx *C, const int64_t *m, uint32_t a, double scale, size_t n, he_ct **out) {
    return guarded([&]() {
        REQUIRE(C && m && out && a >= 1 && scale > 0, HE_EINVAL, "bad argument");
        HIPCHK(hipSetDevice(C->device));
        he_ct *ct = new_ct(C, a);
        ct->n = n;
        try {
            encrypt_coeffs_impl(C, m, a, scale, ct);
        } catch (...) {
            hipFree(ct->d);
            delete ct;
            throw;
        }
        *out = ct;
        return HE_OK;
    });
}

int he_encrypt(he_ctx *C, const double *x, size_t n, double pad, he_ct **out) {
    return guarded([&]() {
        REQUIRE(C && x && out && n >= 1, HE_EINVAL, "bad argument");
        // every encoded coefficient stays below 2^62 when |x| * Delta < 2^61
        const double xmax = std::ldexp(1.0, 61) / C->Delta;
        for (size_t i = 0; i < n; ++i)
            REQUIRE(std::isfinite(x[i]) && std::fabs(x[i]) < xmax, HE_EINVAL, "values must be finite and below 2^61 / Delta");
        const size_t s = (size_t)C->slots;
        std::vector<double> packed;
        uint32_t a;
        if (std::isnan(pad)) {
            double sum = 0;
            for (size_t i = 0; i < n; ++i) sum += x[i];
            pad = sum / (double)n;
        }
        REQUIRE(std::isfinite(pad) && std::fabs(pad) < xmax, HE_EINVAL, "pad must be finite and below 2^61 / Delta");
        if (n <= s && s % n == 0) {
            a = 1;
            packed.resize(s);
            for (size_t i = 0; i < s; ++i) packed[i] = x[i % n];
        } else {
            a = (uint32_t)((n + s - 1) / s);
            packed.assign((size_t)a * s, pad);
            std::memcpy(packed.data(), x, n * 8);
        }
        std::vector<int64_t> m((size_t)a * C->N);
        for (uint32_t c = 0; c < a; ++c) encode_slots(packed.data() + (size_t)c * s, C->N, C->Delta, m.data() + (size_t)c * C->N);
        const int rc = he_encrypt_coeffs(C, m.data(), a, C->Delta, n, out);
        if (rc == HE_OK) (*out)->pad = pad;
        return rc;
    });
}

int he_ct_set_pad(he_ct *ct, double pad) {
    if (!ct || !std::isfinite(pad)) { g_err = "bad argument"; return HE_EINVAL; }
    ct->pad = pad;
    return HE_OK;
}

int he_decrypt(he_ctx *C, const he_ct *ct, double *out, size_t n) {
    return guarded([&]() {
        REQUIRE(C && ct && out && ct->ctx == C, HE_EINVAL, "bad argument");
        REQUIRE(n <= (size_t)ct->a * (size_t)C->slots, HE_EINVAL, "more values than the handle's slots");
        HIPCHK(hipSetDevice(C->device));
        const int N = C->N, nl = ct->level >= 1 ? 2 : 1;
        const size_t s = (size_t)C->slots;
        std::vector<double> res((size_t)nl * N), slotv((size_t)ct->a * s), mc(N);
        double *dm = nullptr;
        dev_alloc(&dm, 8ull * nl * N, "device buffer");
        try {
            for (uint32_t c = 0; c < ct->a; ++c) {
                const double *c0 = ct->d + (size_t)c * 2 * (C->L + 1) * N, *c1 = c0 + (size_t)(C->L + 1) * N;
                launch_decmul(C->T, dm, c0, c1, C->d_sk, nl, C->stream);
                launch_ntt(C->T, VecSet{dm, nl, nl, 0, nullptr, nullptr}, true, C->ntt_variant, C->stream);
                HIPCHK(hipMemcpyAsync(res.data(), dm, 8ull * nl * N, hipMemcpyDeviceToHost, C->stream));
                HIPCHK(hipStreamSynchronize(C->stream));
                const uint64_t q0 = C->q[0];
                if (nl == 1) {
                    for (int i = 0; i < N; ++i) {
                        const uint64_t v = (uint64_t)res[i];
                        mc[i] = v > q0 / 2 ? -(double)(q0 - v) : (double)v;
                    }
                } else {
                    const uint64_t q1 = C->q[1];
                    const unsigned __int128 Q = (unsigned __int128)q0 * q1;
                    const uint64_t q0inv = invmod_u(q0 % q1, q1);
                    for (int i = 0; i < N; ++i) {
                        const uint64_t a0 = (uint64_t)res[i], a1 = (uint64_t)res[N + i];
                        const uint64_t d = a1 >= a0 % q1 ? a1 - a0 % q1 : a1 + q1 - a0 % q1;
                        const uint64_t t = mulmod_u(d, q0inv, q1);
                        const unsigned __int128 v = (unsigned __int128)a0 + (unsigned __int128)q0 * t;
                        mc[i] = v > Q / 2 ? -(double)(Q - v) : (double)v;
                    }
                }
                decode_slots(mc.data(), N, ct->scale, slotv.data() + (size_t)c * s);
            }
        } catch (...) {
            hipFree(dm);
            throw;
        }
        hipFree(dm);
        const size_t total = (size_t)ct->a * s;
        for (size_t i = 0; i < n; ++i) out[i] = slotv[i % total];
        return HE_OK;
    });
}

int he_cutmax(he_ctx *C, he_ct *const *in, size_t batch, const he_cutmax_cfg *cfg, he_ct **out) {
    return guarded([&]() {
        REQUIRE(C, HE_EINVAL, "null context");
        HIPCHK(hipSetDevice(C->device));
        return cutmax_impl(C, in, nullptr, batch, cfg, 1.0, out);
    });
}

int he_topp_sample(he_ctx *C, he_ct *const *logits, he_ct *const *noise, size_t batch, double top_p,
                   double temperature, const he_cutmax_cfg *cfg, he_ct **out) {
    return guarded([&]() {
        REQUIRE(C && noise, HE_EINVAL, "null argument");
        REQUIRE(top_p > 0 && top_p < 1 && temperature > 0, HE_EINVAL, "top_p in (0,1), temperature > 0");
        HIPCHK(hipSetDevice(C->device));
        return cutmax_impl(C, logits, noise, batch, cfg, temperature, out);
    });
}

int he_topp_noise(double top_p, const double *u, size_t n, double *g) {
    return guarded([&]() {
        REQUIRE(u && g && top_p > 0 && top_p < 1, HE_EINVAL, "bad argument");
        const double alpha = std::log(1.0 - top_p) / std::log(top_p);
        for (size_t i = 0; i < n; ++i) {
            REQUIRE(u[i] > 0 && u[i] <= 1, HE_EINVAL, "uniform draws must lie in (0, 1]");
            g[i] = std::pow(u[i], 1.0 / alpha);
        }
        return HE_OK;
    });
}

int he_gumbel_sample(he_ctx *C, he_ct *const *logits, he_ct *const *noise, size_t batch, double temperature,
                     const he_cutmax_cfg *cfg, he_ct **out) {
    return guarded([&]() {
        REQUIRE(C && noise, HE_EINVAL, "null argument");
        REQUIRE(temperature > 0, HE_EINVAL, "temperature > 0");
        HIPCHK(hipSetDevice(C->device));
        return cutmax_impl(C, logits, noise, batch, cfg, temperature, out);
    });
}

int he_gumbel_noise(const double *u, size_t n, double *g) {
    return guarded([&]() {
        REQUIRE(u && g, HE_EINVAL, "bad argument");
        for (size_t i = 0; i < n; ++i) {
            REQUIRE(u[i] > 0 && u[i] < 1, HE_EINVAL, "uniform draws must lie in (0, 1)");
            g[i] = -std::log(-std::log(u[i]));
        }
        return HE_OK;
    });
}

int he_invsqrt_guess_fit(double u_lo, uint32_t degree, double *coef) {
    return guarded([&]() {
        REQUIRE(coef && u_lo > 0 && u_lo < 1 && degree >= 1 && degree <= 4, HE_EINVAL,
                "u_lo in (0, 1), degree 1..4, coef non-null");
        chebyshev_invsqrt_fit(u_lo, (int)degree, coef);
        return HE_OK;
    });
}

int he_invsqrt_scaled_plan(double u_lo, uint32_t degree, uint32_t K, double *coef, double *steps, double *ranges) {
    return guarded([&]() {
        REQUIRE(coef && ranges && (K == 0 || steps) && u_lo > 0 && u_lo < 1 && degree >= 1 && degree <= 4 && K <= 16,
                HE_EINVAL, "u_lo in (0, 1), degree 1..4, K <= 16, non-null outputs");
        REQUIRE(invsqrt_scaled_plan(u_lo, (int)degree, (int)K, coef, steps, ranges), HE_EINVAL,
                "the guess is not positive on the domain");
        return HE_OK;
    });
}

void he_ct_free(he_ct *ct) {
    if (!ct) return;
    if (ct->d) hipFree(ct->d);
    delete ct;
}

int he_ct_info(const he_ct *ct, uint32_t *a, uint32_t *level, double *scale, size_t *n) {
    if (!ct) { g_err = "null ciphertext"; return HE_EINVAL; }
    if (a) *a = ct->a;
    if (level) *level = ct->level;
    if (scale) *scale = ct->scale;
    if (n) *n = ct->n;
    return HE_OK;
}

int he_ct_export(he_ctx *C, const he_ct *ct, uint64_t *limbs, size_t cap) {
    return guarded([&]() {
        REQUIRE(C && ct && limbs && ct->ctx == C, HE_EINVAL, "bad argument");
        HIPCHK(hipSetDevice(C->device));
        const int N = C->N, l = (int)ct->level;
        const size_t need = (size_t)ct->a * 2 * (l + 1) * N;
        REQUIRE(cap >= need, HE_EINVAL, "export buffer too small");
        double *tmp = nullptr;
        dev_alloc(&tmp, need * 8, "device buffer");
        std::vector<double> h(need);
        try {
            const VecSet dst{tmp, (int)ct->a * 2 * (l + 1), l + 1, (long long)(l + 1) * N, nullptr, nullptr};
            const VecSet src{ct->d, (int)ct->a * 2 * (l + 1), l + 1, (long long)(C->L + 1) * N, nullptr, nullptr};
            launch_copy(C->T, dst, src, C->stream);
            launch_ntt(C->T, dst, true, C->ntt_variant, C->stream);
            HIPCHK(hipMemcpyAsync(h.data(), tmp, need * 8, hipMemcpyDeviceToHost, C->stream));
            HIPCHK(hipStreamSynchronize(C->stream));
        } catch (...) {
            hipFree(tmp);
            throw;
        }
        hipFree(tmp);
        for (size_t i = 0; i < need; ++i) limbs[i] = (uint64_t)h[i];
        return HE_OK;
    });
}

int he_ct_import(he_ctx *C, const uint64_t *limbs, uint32_t a, uint32_t level, double scale, size_t n,
                 he_ct **out) {
    return guarded([&]() {
        REQUIRE(C && limbs && out && a >= 1 && (int)level <= C->L, HE_EINVAL, "bad argument");
        REQUIRE(std::isfinite(scale) && scale > 0, HE_EINVAL, "scale must be positive and finite");
        HIPCHK(hipSetDevice(C->device));
        const int N = C->N, l = (int)level;
        const size_t words = (size_t)a * 2 * (l + 1) * N;
        std::vector<double> h(words);
        for (size_t i = 0; i < words; ++i) {
            const int limb = (int)((i / N) % (l + 1));
            REQUIRE(limbs[i] < C->q[limb], HE_EINVAL, "limb value not canonical");
            h[i] = (double)limbs[i];
        }
        he_ct *ct = new_ct(C, a);
        double *tmp = nullptr;
        try {
            dev_alloc(&tmp, words * 8, "device buffer");
            HIPCHK(hipMemcpyAsync(tmp, h.data(), words * 8, hipMemcpyHostToDevice, C->stream));
            const VecSet src{tmp, (int)a * 2 * (l + 1), l + 1, (long long)(l + 1) * N, nullptr, nullptr};
            launch_ntt(C->T, src, false, C->ntt_variant, C->stream);
            const VecSet dst{ct->d, (int)a * 2 * (l + 1), l + 1, (long long)(C->L + 1) * N, nullptr, nullptr};
            launch_copy(C->T, dst, src, C->stream);
            HIPCHK(hipStreamSynchronize(C->stream));
        } catch (...) {
            if (tmp) hipFree(tmp);
            hipFree(ct->d);
            delete ct;
            throw;
        }
        hipFree(tmp);
        ct->level = level;
        ct->scale = scale;
        ct->n = n;
        *out = ct;
        return HE_OK;
    });
}

int he_add(he_ctx *C, const he_ct *a, const he_ct *b, he_ct **out) {
    // b is read with this context's ring degree and limb stride: it must belong to C
    if (!b || b->ctx != C || b->a != 1 || (a && b->level != a->level)) {
        g_err = "bad operand (null, from another context, several ciphertexts or another level)";
        return HE_EINVAL;
    }
    return prim(C, a, out, [&](Exec &X) { return X.add(bt_of(a), bt_of(b)); });
}
int he_sub(he_ctx *C, const he_ct *a, const he_ct *b, he_ct **out) {
    // b is read with this context's ring degree and limb stride: it must belong to C
    if (!b || b->ctx != C || b->a != 1 || (a && b->level != a->level)) {
        g_err = "bad operand (null, from another context, several ciphertexts or another level)";
        return HE_EINVAL;
    }
    return prim(C, a, out, [&](Exec &X) { return X.add(bt_of(a), bt_of(b), -1); });
}
int he_mul_int(he_ctx *C, const he_ct *a, int64_t k, he_ct **out) {
    return prim(C, a, out, [&](Exec &X) { return X.mul_int(bt_of(a), {k}); });
}
int he_add_const(he_ctx *C, const he_ct *a, double c, he_ct **out) {
    return prim(C, a, out, [&](Exec &X) { return X.add_const(bt_of(a), {c}); });
}
int he_mul(he_ctx *C, const he_ct *a, const he_ct *b, he_ct **out) {
    // b is read with this context's ring degree and limb stride: it must belong to C
    if (!b || b->ctx != C || b->a != 1 || (a && b->level != a->level)) {
        g_err = "bad operand (null, from another context, several ciphertexts or another level)";
        return HE_EINVAL;
    }
    return prim(C, a, out, [&](Exec &X) { return X.mul(bt_of(a), bt_of(b)); });
}
int he_rescale(he_ctx *C, const he_ct *a, he_ct **out) {
    return prim(C, a, out, [&](Exec &X) { return X.rescale(bt_of(a)); });
}
int he_cmul(he_ctx *C, const he_ct *a, double kappa, double s_want, int exact, he_ct **out) {
    return prim(C, a, out, [&](Exec &X) { return X.cmul(bt_of(a), {kappa}, {s_want}, exact != 0); });
}
int he_rotate(he_ctx *C, const he_ct *a, uint32_t r, he_ct **out) {
    if (C && (1u << r) >= (uint32_t)C->slots) { g_err = "rotation index too large"; return HE_EINVAL; }
    return prim(C, a, out, [&](Exec &X) { return X.rotate(bt_of(a), (int)r); });
}
int he_rotsum(he_ctx *C, const he_ct *a, he_ct **out) {
    return prim(C, a, out, [&](Exec &X) { return X.rotsum(bt_of(a)); }, true);
}
int he_rotsum_noalloc(he_ctx *C, const he_ct *a, he_ct *out) {
    return guarded([&]() {
        REQUIRE(C && a && out && a->ctx == C && out->ctx == C, HE_EINVAL, "null or foreign argument");
        REQUIRE(out->a == a->a, HE_EINVAL, "out must hold as many ciphertexts as a");
        unsigned char *base = scratch_of(C->device);
        HIPCHK(hipSetDevice(C->device));
        // this call's workspace and constants live in the scratch; the context's own
        // (hipMalloc'd) arena and pool are set aside and restored afterwards
        struct Restore {
            he_ctx *C;
            Arena a;
            Pool p;
            ~Restore() { C->arena = a; C->pool = std::move(p); }
        } keep{C, C->arena, std::move(C->pool)};
        C->arena = Arena{};
        C->pool = Pool{};
        {
            Exec X(C, true);
            (void)X.rotsum(bt_of(a));
        }
        const size_t dbytes = (C->pool.dv.size() * 8 + 255) & ~(size_t)255;
        const size_t ibytes = (C->pool.iv.size() * 4 + 255) & ~(size_t)255;
        const size_t need = ((C->arena.peak + 255) & ~(size_t)255) + dbytes + ibytes;
        if (need > kScratchBytes)
            throw HeError(HE_ENOMEM, "he_rotsum_noalloc: the call needs " + std::to_string(need >> 20) +
                                         " MiB of scratch; the static scratch holds " +
                                         std::to_string(kScratchBytes >> 20) + " MiB");
        const size_t wcap = kScratchBytes - dbytes - ibytes;
        C->arena.base = (char *)base;
        C->arena.cap = wcap;
        C->arena.dry = false;
        C->arena.top = 0;
        C->pool.d_dv = (double *)(base + wcap);
        C->pool.d_iv = (int *)(base + wcap + dbytes);
        C->pool.dcap = dbytes / 8;
        C->pool.icap = ibytes / 4;
        C->pool.dry = false;
        C->pool.dpos = C->pool.ipos = 0;
        if (!C->pool.dv.empty())
            HIPCHK(hipMemcpyAsync(C->pool.d_dv, C->pool.dv.data(), C->pool.dv.size() * 8, hipMemcpyHostToDevice,
                                  C->stream));
        if (!C->pool.iv.empty())
            HIPCHK(hipMemcpyAsync(C->pool.d_iv, C->pool.iv.data(), C->pool.iv.size() * 4, hipMemcpyHostToDevice,
                                  C->stream));
        Exec X(C, false);
        Bt r = X.rotsum(bt_of(a));
        store_bt(X, r, 0, out);
        out->n = a->n;
        out->pad = a->pad;
        HIPCHK(hipGetLastError());
        // the scratch is free again when the call returns
        HIPCHK(hipStreamSynchronize(C->stream));
        return HE_OK;
    });
}
int he_drop(he_ctx *C, const he_ct *a, uint32_t level, he_ct **out) {
    return prim(C, a, out, [&](Exec &X) { return X.copy(X.drop(bt_of(a), (int)level)); }, true);
}

int he_boot_setup(he_ctx *C, const he_boot_cfg *cfg) {
    return guarded([&]() {
        REQUIRE(C, HE_EINVAL, "null context");
        HIPCHK(hipSetDevice(C->device));
        boot_setup(C, cfg);
        return HE_OK;
    });
}

int he_bootstrap(he_ctx *C, const he_ct *in, double bound, he_ct **out) {
    return prim(C, in, out, [&](Exec &X) { return bootstrap(X, bt_of(in), bound); }, true);
}

int he_keygen_galois(he_ctx *C, uint32_t kidx, uint64_t galois) {
    return guarded([&]() {
        REQUIRE(C, HE_EINVAL, "null context");
        REQUIRE((galois & 1) && galois > 1 && galois < 2ull * C->N, HE_EINVAL, "Galois element must be odd in (1, 2N)");
        if (kidx < C->key_gal.size()) {
            REQUIRE(kidx >= 1 && C->key_gal[kidx] == (uint32_t)galois, HE_EINVAL,
                    "key index taken by another key (use the next free index)");
            return HE_OK;
        }
        REQUIRE(kidx == C->key_gal.size(), HE_EINVAL, "key index must be the next free index");
        REQUIRE(kidx < 0x10000u, HE_EINVAL, "too many keys");
        HIPCHK(hipSetDevice(C->device));
        C->key_gal.push_back((uint32_t)galois);
        try {
            gen_keys(C, (int)kidx);
        } catch (...) {
            C->key_gal.pop_back();
            C->keys.resize(C->key_gal.size());
            throw;
        }
        drop_graphs(C);
        return HE_OK;
    });
}

int he_rotate_gal(he_ctx *C, const he_ct *a, uint32_t kidx, uint64_t galois, he_ct **out) {
    return prim(C, a, out, [&](Exec &X) { return X.rotate_gal(bt_of(a), (int)kidx, galois); });
}

int he_mul_plain(he_ctx *C, const he_ct *a, const int64_t *m, double pscale, he_ct **out) {
    return prim(C, a, out, [&](Exec &X) {
        REQUIRE(m && std::isfinite(pscale) && pscale > 0, HE_EINVAL, "mul_plain: null plaintext or bad scale");
        const int l = (int)a->level, N = C->N;
        int64_t *dm = (int64_t *)C->arena.alloc(8ull * N);
        double *pt = X.alloc_d((size_t)(l + 1) * N);
        if (X.go()) {
            HIPCHK(hipMemcpyAsync(dm, m, 8ull * N, hipMemcpyHostToDevice, C->stream));
            const VecSet v{pt, l + 1, l + 1, 0, nullptr, nullptr};
            launch_int64_to_res(C->T, v, dm, 0, nullptr, C->stream);
            launch_ntt(C->T, v, false, C->ntt_variant, C->stream);
        }
        return X.mul_plain(bt_of(a), pt, pscale);
    });
}

int he_modraise(he_ctx *C, const he_ct *a, uint32_t level, double scale, he_ct **out) {
    return prim(C, a, out, [&](Exec &X) {
        REQUIRE(std::isfinite(scale) && scale > 0, HE_EINVAL, "modraise: bad scale");
        return X.modraise(bt_of(a), (int)level, scale);
    });
}

int he_bench_ntt(he_ctx *C, uint32_t vectors, uint32_t iters, double *ms_fwd, double *ms_inv) {
    return guarded([&]() {
        REQUIRE(C && vectors >= 1 && iters >= 1 && ms_fwd && ms_inv, HE_EINVAL, "bad argument");
        HIPCHK(hipSetDevice(C->device));
        const int N = C->N;
        DevScope tmp;
        double *buf = tmp.alloc<double>(8ull * vectors * N, "NTT measurement");
        const hipEvent_t a = tmp.event(), b = tmp.event(), c = tmp.event();
        const int grp = std::min<int>((int)vectors, C->L + 1);
        const VecSet vs{buf, (int)vectors, grp, (long long)grp * N, nullptr, nullptr};
        launch_sample_uniform(C->T, vs, 12345, 0x7F000000u, nullptr, C->stream);
        launch_ntt(C->T, vs, false, C->ntt_variant, C->stream);
        launch_ntt(C->T, vs, true, C->ntt_variant, C->stream);
        double tf = 0, ti = 0;
        for (uint32_t it = 0; it < iters; ++it) {
            HIPCHK(hipEventRecord(a, C->stream));
            launch_ntt(C->T, vs, false, C->ntt_variant, C->stream);
            HIPCHK(hipEventRecord(b, C->stream));
            launch_ntt(C->T, vs, true, C->ntt_variant, C->stream);
            HIPCHK(hipEventRecord(c, C->stream));
            HIPCHK(hipEventSynchronize(c));
            float f1 = 0, f2 = 0;
            HIPCHK(hipEventElapsedTime(&f1, a, b));
            HIPCHK(hipEventElapsedTime(&f2, b, c));
            tf += f1; ti += f2;
        }
        *ms_fwd = tf / iters;
        *ms_inv = ti / iters;
        return HE_OK;
    });
}

int he_bench_copy(he_ctx *C, uint32_t vectors, uint32_t iters, double *ms) {
    return guarded([&]() {
        REQUIRE(C && vectors >= 1 && iters >= 1 && ms, HE_EINVAL, "bad argument");
        HIPCHK(hipSetDevice(C->device));
        const int N = C->N;
        DevScope tmp;
        double *buf = tmp.alloc<double>(16ull * vectors * N, "copy measurement");
        const hipEvent_t a = tmp.event(), b = tmp.event();
        const int grp = std::min<int>((int)vectors, C->L + 1);
        const VecSet src{buf, (int)vectors, grp, (long long)grp * N, nullptr, nullptr};
        const VecSet dst{buf + (size_t)vectors * N, (int)vectors, grp, (long long)grp * N, nullptr, nullptr};
        launch_sample_uniform(C->T, src, 777, 0x7D000000u, nullptr, C->stream);
        launch_copy(C->T, dst, src, C->stream);
        HIPCHK(hipEventRecord(a, C->stream));
        for (uint32_t it = 0; it < iters; ++it) launch_copy(C->T, dst, src, C->stream);
        HIPCHK(hipEventRecord(b, C->stream));
        HIPCHK(hipEventSynchronize(b));
        float f = 0;
        HIPCHK(hipEventElapsedTime(&f, a, b));
        *ms = f / iters;
        return HE_OK;
    });
}

int he_last_cutmax_ms(const he_ctx *C, double *ms) {
    if (!C || !ms) { g_err = "null argument"; return HE_EINVAL; }
    *ms = C->last_ms;
    return HE_OK;
}

int he_sync(he_ctx *C) {
    return guarded([&]() {
        REQUIRE(C, HE_EINVAL, "null context");
        HIPCHK(hipStreamSynchronize(C->stream));
        return HE_OK;
    });
}

int he_profile_begin(he_ctx *C) {
    return guarded([&]() {
        REQUIRE(C, HE_EINVAL, "null context");
        REQUIRE(!g_kprof, HE_ESTATE, "a profile is already running");
        HIPCHK(hipSetDevice(C->device));
        g_kprof = new KProf;
        return HE_OK;
    });
}

int he_profile_end(he_ctx *C, char *buf, size_t cap) {
    return guarded([&]() {
        REQUIRE(C && buf && cap > 2, HE_EINVAL, "bad argument");
        REQUIRE(g_kprof, HE_ESTATE, "no profile running");
        KProf *P = g_kprof;
        g_kprof = nullptr;
        HIPCHK(hipStreamSynchronize(C->stream));
        struct Agg { long n = 0; double ms = 0, bytes = 0; };
        std::map<std::string, Agg> agg;
        for (auto &r : P->recs) {
            float ms = 0;
            hipEventElapsedTime(&ms, r.a, r.b);
            auto &e = agg[r.name];
            e.n += 1;
            e.ms += ms;
            e.bytes += r.bytes;
            hipEventDestroy(r.a);
            hipEventDestroy(r.b);
        }
        delete P;
        std::string js = "{";
        for (auto &kv : agg) {
            char tmp[256];
            std::snprintf(tmp, sizeof tmp, "%s\"%s\": [%ld, %.6f, %.1f]", js.size() > 1 ? ", " : "",
                          kv.first.c_str(), kv.second.n, kv.second.ms, kv.second.bytes);
            js += tmp;
        }
        js += "}";
        REQUIRE(js.size() + 1 <= cap, HE_EINVAL, "profile buffer too small");
        std::memcpy(buf, js.c_str(), js.size() + 1);
        return HE_OK;
    });
}

int he_ntt_tuning(const he_ctx *C, int32_t *variants, uint32_t n) {
    if (!C || !variants) { g_err = "null argument"; return HE_EINVAL; }
    const int li = C->logN == 16 ? 1 : 0;
    for (uint32_t i = 0; i < n && i < 8; ++i) variants[i] = g_tuned_choice[li][i];
    return HE_OK;
}

int he_ntt_tuning_report(const he_ctx *C, char *buf, size_t cap) {
    if (!C || !buf || cap == 0) { g_err = "null argument"; return HE_EINVAL; }
    const int li = C->logN == 16 ? 1 : 0;
    const int w[3] = {C->logN == 16 ? 4 : 8, C->logN == 16 ? 8 : 16, C->logN == 16 ? 16 : 32};
    std::string js = "{\"logN\":" + std::to_string(C->logN) + ",\"variants\":[";
    for (int v = 1; v <= NTT_VARIANTS; ++v) {
        js += std::string(v > 1 ? "," : "") + "\"" + std::to_string(w[(v - 1) % 3]) + " sub-transforms per workgroup, " +
              ((v - 1) / 3 ? "factored" : "table") + " pass-2 twiddles\"";
    }
    js += "],\"buckets\":[";
    for (int b = 0; b < kTuneBuckets; ++b) {
        char tmp[64];
        js += std::string(b ? "," : "") + "{\"vectors\":" + std::to_string(g_tuned_count[li][b]) + ",\"ms\":[";
        for (int v = 0; v < NTT_VARIANTS; ++v) {
            std::snprintf(tmp, sizeof tmp, "%s%.5f", v ? "," : "", g_tuned_ms[li][b][v]);
            js += tmp;
        }
        js += "],\"choice\":" + std::to_string(g_tuned_choice[li][b]) + "}";
    }
    js += "]}";
    if (js.size() + 1 > cap) { g_err = "buffer too small"; return HE_EINVAL; }
    std::memcpy(buf, js.c_str(), js.size() + 1);
    return HE_OK;
}

int he_set_option(he_ctx *C, int option, int64_t value) {
    if (!C) { g_err = "null context"; return HE_EINVAL; }
    if (option == HE_OPT_GRAPH) { C->use_graph = (int)value; return HE_OK; }
    if (option == HE_OPT_NTT_VARIANT) {
        if (value < 0 || value > NTT_VARIANTS) { g_err = "NTT variant out of range"; return HE_EINVAL; }
        C->ntt_variant = (int)value;
        drop_graphs(C);  // captured graphs hold the previous variant's kernels
        return HE_OK;
    }
    if (option == HE_OPT_BOOT_HOIST) {
        C->boot_hoist = value <= 0 ? 0 : (value >= 2 ? 2 : 1);
        drop_graphs(C);  // captured graphs hold the other launch sequence
        return HE_OK;
    }
    if (option == HE_OPT_WORKSPACE_LIMIT) {
        if (value < 0) { g_err = "workspace limit must be >= 0"; return HE_EINVAL; }
        C->ws_limit = (size_t)value;
        // memory held beyond the new limit is returned now
        const size_t held = C->arena.cap + C->pool.dcap * 8 + C->pool.icap * 4;
        if (C->ws_limit > 0 && held > C->ws_limit)
            return guarded([&]() {
                HIPCHK(hipStreamSynchronize(C->stream));
                free_workspace(C);
                return HE_OK;
            });
        return HE_OK;
    }
    g_err = "unknown option";
    return HE_EINVAL;
}

}  // extern "C"
