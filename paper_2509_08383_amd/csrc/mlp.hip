// Learned initial guess for the encrypted inverse square root (Alg. 2 line 5):
// a 1 -> 16 -> 16 -> 1 network with square activations, trained in FP32 on the GPU
// by hand-written forward/backward/Adam kernels, then collapsed on the host into the
// degree-4 polynomial in u that the encrypted schedule evaluates.
//
//   z = (u - m)/s,  h1 = W1 z + b1,  a1 = h1^2,  h2 = W2 a1 + b2,  a2 = h2^2,
//   y = W3 . a2 + b3,   loss = mean (y sqrt(u) - 1)^2   (relative error of 1/sqrt(u))
//
// Parameter layout (321 floats): W1[16], b1[16], W2[16][16] (row = output unit), b2[16],
// W3[16], b3.
//
// The training set is the variances of plaintext CutMax runs (Alg. 1) on synthetic
// LLM-like logits, generated here by k_var_log: one workgroup per run, logits
// x_i = s G_i - z ln(i+1) (i < vocab; 0 in pad slots) with G_i Gumbel(0,1) from
// Philox4x32-10 and per-run s ~ U[1.5, 4.5], z ~ U[0.9, 1.3].  Giving token i the rank
// i+1 is equivalent in distribution to a random rank permutation because the G_i are
// i.i.d.  Every iterate is recomputed from x_i and the scalar statistics of the
// earlier iterations, so nothing per slot is stored.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <random>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/he.h"
#include "he_internal.h"
#include "mlp_file.h"

namespace {

constexpr int HID = he::kMlpHidden;
constexpr int NP = he::kMlpParams;  // 321
constexpr int MB = 128;                                    // samples per block

__global__ __launch_bounds__(MB) void k_mlp_fwd_bwd(const float *u, int m, const float *theta, float mean,
                                                    float sdv, float inv_count, float *grad, float *loss,
                                                    float *yout) {
    __shared__ float th[NP];
    __shared__ float s_z[MB], s_dy[MB], s_a1[MB][HID], s_dh1[MB][HID], s_a2[MB][HID], s_dh2[MB][HID];
    for (int i = threadIdx.x; i < NP; i += MB) th[i] = theta[i];
    __syncthreads();
    const float *W1 = th, *b1 = th + HID, *W2 = th + 2 * HID, *b2 = th + 2 * HID + HID * HID;
    const float *W3 = b2 + HID, b3 = W3[HID];
    const int t = threadIdx.x, idx = blockIdx.x * MB + t;
    const bool live = idx < m;
    const float uu = live ? u[idx] : 1.0f;
    const float z = (uu - mean) / sdv;
    float h1[HID], a1[HID], h2[HID], a2[HID];
#pragma unroll
    for (int k = 0; k < HID; ++k) { h1[k] = W1[k] * z + b1[k]; a1[k] = h1[k] * h1[k]; }
    float y = b3;
#pragma unroll
    for (int j = 0; j < HID; ++j) {
        float acc = b2[j];
#pragma unroll
        for (int k = 0; k < HID; ++k) acc += W2[j * HID + k] * a1[k];
        h2[j] = acc;
        a2[j] = acc * acc;
        y += W3[j] * a2[j];
    }
    const float su = sqrtf(uu);
    const float r = y * su - 1.0f;
    if (yout && live) yout[idx] = y;
    const float dy = live ? 2.0f * r * su * inv_count : 0.0f;
    float dh2[HID];
#pragma unroll
    for (int j = 0; j < HID; ++j) dh2[j] = dy * W3[j] * 2.0f * h2[j];
#pragma unroll
    for (int k = 0; k < HID; ++k) {
        float da1 = 0.0f;
#pragma unroll
        for (int j = 0; j < HID; ++j) da1 += dh2[j] * W2[j * HID + k];
        s_dh1[t][k] = da1 * 2.0f * h1[k];
        s_a1[t][k] = a1[k];
        s_a2[t][k] = a2[k];
        s_dh2[t][k] = dh2[k];
    }
    s_z[t] = z;
    s_dy[t] = dy;
    if (loss) {
        float l = live ? r * r : 0.0f;
        for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off);
        if ((t & 63) == 0) atomicAdd(loss, l);
    }
    __syncthreads();
    if (!grad) return;
    for (int p = t; p < NP; p += MB) {
        float s = 0.0f;
        if (p < HID) { for (int i = 0; i < MB; ++i) s += s_dh1[i][p] * s_z[i]; }
        else if (p < 2 * HID) { const int k = p - HID; for (int i = 0; i < MB; ++i) s += s_dh1[i][k]; }
        else if (p < 2 * HID + HID * HID) {
            const int q = p - 2 * HID, j = q / HID, k = q % HID;
            for (int i = 0; i < MB; ++i) s += s_dh2[i][j] * s_a1[i][k];
        } else if (p < 3 * HID + HID * HID) { const int j = p - 2 * HID - HID * HID; for (int i = 0; i < MB; ++i) s += s_dh2[i][j]; }
        else if (p < 4 * HID + HID * HID) { const int j = p - 3 * HID - HID * HID; for (int i = 0; i < MB; ++i) s += s_dy[i] * s_a2[i][j]; }
        else { for (int i = 0; i < MB; ++i) s += s_dy[i]; }
        atomicAdd(grad + p, s);
    }
}

__global__ void k_fill(float *x, int n, float v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// Adam (Kingma and Ba, 2015) on every parameter
__global__ void k_adam(float *theta, const float *grad, float *m1, float *m2, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float a = b1 * m1[i] + (1.0f - b1) * g;
    const float v = b2 * m2[i] + (1.0f - b2) * g * g;
    m1[i] = a;
    m2[i] = v;
    theta[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// ----------------------------------------------------- plaintext CutMax statistics
__device__ inline void philox_m(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

constexpr int VT = 256;

__device__ inline double block_sum(double v, double *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < VT / 64; ++i) s += sh[i];
    return s;
}

// var_out[run][t] = population variance of the iterate entering iteration t;
// ysum_out[run] = mean of the last iterate
__global__ __launch_bounds__(VT) void k_var_log(uint64_t seed, int run0, int vocab, int slots, int T, int p,
                                                double c, float *var_out, float *ymean_out) {
    __shared__ double sh[VT / 64];
    const int run = run0 + blockIdx.x;
    uint32_t o[4];
    philox_m(0u, (uint32_t)run, 0x6D000000u, 0u, (uint32_t)seed, (uint32_t)(seed >> 32), o);
    const double sc = 1.5 + 3.0 * ((o[0] + 0.5) / 4294967296.0);
    const double zf = 0.9 + 0.4 * ((o[1] + 0.5) / 4294967296.0);
    double mu[8], isd[8];
    const double n = (double)slots;
    for (int t = 0; t <= T; ++t) {
        double s1 = 0.0, s2 = 0.0;
        for (int i = threadIdx.x; i < slots; i += VT) {
            double y = 0.0;
            if (i < vocab) {
                philox_m((uint32_t)i, (uint32_t)run, 0x6E000000u, 0u, (uint32_t)seed, (uint32_t)(seed >> 32), o);
                const double uu = (o[0] + 0.5) / 4294967296.0;
                y = sc * (-log(-log(uu))) - zf * log((double)(i + 1));
            }
            for (int k = 0; k < t; ++k) {
                const double zz = (y - mu[k]) * isd[k] / c + 1.0;
                double pw = zz;
                for (int e = 1; e < p; ++e) pw *= zz;
                y = pw;
            }
            s1 += y;
            s2 += y * y;
        }
        const double S1 = block_sum(s1, sh);
        const double S2 = block_sum(s2, sh);
        const double m = S1 / n, var = S2 / n - m * m;
        if (t < T) {
            mu[t] = m;
            isd[t] = 1.0 / sqrt(var);
            if (threadIdx.x == 0) var_out[(size_t)run * T + t] = (float)var;
        } else if (threadIdx.x == 0 && ymean_out) {
            ymean_out[run] = (float)m;
        }
    }
}

thread_local std::string g_merr;

struct MErr : std::runtime_error {
    int code;
    MErr(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};
#define MCHK(x)                                                                                           \
    do {                                                                                                  \
        hipError_t e_ = (x);                                                                              \
        if (e_ != hipSuccess) throw MErr(HE_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));     \
    } while (0)

template <class F>
int mguard(F &&f) {
    try {
        return f();
    } catch (const MErr &e) {
        g_merr = e.what();
        return e.code;
    } catch (const std::exception &e) {
        g_merr = e.what();
        return HE_EINVAL;
    }
}

}  // namespace

struct he_mlp {
    int device = 0;
    hipStream_t s = nullptr;
    float *d_theta = nullptr, *d_grad = nullptr, *d_m1 = nullptr, *d_m2 = nullptr, *d_loss = nullptr;
    float *d_u = nullptr, *d_y = nullptr;
    size_t cap = 0;
    float mean = 0.5f, sd = 0.25f;
    int step = 0;
};

static void ensure_cap(he_mlp *M, size_t m) {
    if (m <= M->cap) return;
    if (M->d_u) hipFree(M->d_u);
    if (M->d_y) hipFree(M->d_y);
    MCHK(hipMalloc(&M->d_u, m * 4));
    MCHK(hipMalloc(&M->d_y, m * 4));
    M->cap = m;
}

static void fill(he_mlp *M, float *x, int n, float v) {
    hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, M->s, x, n, v);
}

extern "C" {

const char *he_mlp_last_error(void) { return g_merr.c_str(); }

int he_mlp_create(uint64_t seed, int device, he_mlp **out) {
    return mguard([&]() {
        if (!out) throw MErr(HE_EINVAL, "null argument");
        auto *M = new he_mlp;
        M->device = device;
        MCHK(hipSetDevice(device));
        MCHK(hipStreamCreateWithFlags(&M->s, hipStreamNonBlocking));
        MCHK(hipMalloc(&M->d_theta, NP * 4));
        MCHK(hipMalloc(&M->d_grad, NP * 4));
        MCHK(hipMalloc(&M->d_m1, NP * 4));
        MCHK(hipMalloc(&M->d_m2, NP * 4));
        MCHK(hipMalloc(&M->d_loss, 4));
        std::mt19937_64 rng(seed);
        std::normal_distribution<float> nd(0.0f, 1.0f);
        std::vector<float> th(NP);
        for (int k = 0; k < HID; ++k) { th[k] = 0.5f * nd(rng); th[HID + k] = 0.5f * nd(rng); }
        for (int i = 0; i < HID * HID; ++i) th[2 * HID + i] = 0.25f * nd(rng);
        for (int j = 0; j < HID; ++j) th[2 * HID + HID * HID + j] = 0.25f * nd(rng);
        for (int j = 0; j < HID; ++j) th[3 * HID + HID * HID + j] = 0.05f * nd(rng);
        th[NP - 1] = 1.0f;
        MCHK(hipMemcpy(M->d_theta, th.data(), NP * 4, hipMemcpyHostToDevice));
        fill(M, M->d_m1, NP, 0.0f);
        fill(M, M->d_m2, NP, 0.0f);
        MCHK(hipStreamSynchronize(M->s));
        *out = M;
        return HE_OK;
    });
}

void he_mlp_destroy(he_mlp *M) {
    if (!M) return;
    hipSetDevice(M->device);
    hipStreamSynchronize(M->s);
    hipFree(M->d_theta); hipFree(M->d_grad); hipFree(M->d_m1); hipFree(M->d_m2); hipFree(M->d_loss);
    if (M->d_u) hipFree(M->d_u);
    if (M->d_y) hipFree(M->d_y);
    hipStreamDestroy(M->s);
    delete M;
}

int he_mlp_set_params(he_mlp *M, const float *theta, size_t n, float mean, float sd) {
    return mguard([&]() {
        if (!M || !theta || n != (size_t)NP || !(sd > 0)) throw MErr(HE_EINVAL, "bad argument");
        MCHK(hipSetDevice(M->device));
        MCHK(hipMemcpy(M->d_theta, theta, NP * 4, hipMemcpyHostToDevice));
        M->mean = mean;
        M->sd = sd;
        return HE_OK;
    });
}

int he_mlp_get_params(const he_mlp *M, float *theta, size_t n, float *mean, float *sd) {
    return mguard([&]() {
        if (!M || !theta || n != (size_t)NP) throw MErr(HE_EINVAL, "bad argument");
        MCHK(hipSetDevice(M->device));
        MCHK(hipMemcpy(theta, M->d_theta, NP * 4, hipMemcpyDeviceToHost));
        if (mean) *mean = M->mean;
        if (sd) *sd = M->sd;
        return HE_OK;
    });
}

int he_mlp_grad(he_mlp *M, const float *u, size_t m, float *loss, float *grad) {
    return mguard([&]() {
        if (!M || !u || !loss || !grad || m == 0) throw MErr(HE_EINVAL, "bad argument");
        MCHK(hipSetDevice(M->device));
        ensure_cap(M, m);
        MCHK(hipMemcpyAsync(M->d_u, u, m * 4, hipMemcpyHostToDevice, M->s));
        fill(M, M->d_grad, NP, 0.0f);
        fill(M, M->d_loss, 1, 0.0f);
        hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((m + MB - 1) / MB), dim3(MB), 0, M->s, M->d_u, (int)m, M->d_theta,
                           M->mean, M->sd, 1.0f / (float)m, M->d_grad, M->d_loss, (float *)nullptr);
        MCHK(hipMemcpyAsync(grad, M->d_grad, NP * 4, hipMemcpyDeviceToHost, M->s));
        MCHK(hipMemcpyAsync(loss, M->d_loss, 4, hipMemcpyDeviceToHost, M->s));
        MCHK(hipStreamSynchronize(M->s));
        *loss /= (float)m;
        return HE_OK;
    });
}

int he_mlp_forward(he_mlp *M, const float *u, size_t m, float *y) {
    return mguard([&]() {
        if (!M || !u || !y || m == 0) throw MErr(HE_EINVAL, "bad argument");
        MCHK(hipSetDevice(M->device));
        ensure_cap(M, m);
        MCHK(hipMemcpyAsync(M->d_u, u, m * 4, hipMemcpyHostToDevice, M->s));
        hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((m + MB - 1) / MB), dim3(MB), 0, M->s, M->d_u, (int)m, M->d_theta,
                           M->mean, M->sd, 0.0f, (float *)nullptr, (float *)nullptr, M->d_y);
        MCHK(hipMemcpyAsync(y, M->d_y, m * 4, hipMemcpyDeviceToHost, M->s));
        MCHK(hipStreamSynchronize(M->s));
        return HE_OK;
    });
}

// Adam over shuffled mini-batches; the input normalisation (mean, sd) is taken from
// the data.  *final_loss is the loss over the whole set after training.
int he_mlp_train(he_mlp *M, const float *u, size_t m, uint32_t epochs, uint32_t batch, float lr, uint64_t seed,
                 float *final_loss) {
    return mguard([&]() {
        if (!M || !u || m == 0 || batch == 0 || epochs == 0 || !final_loss) throw MErr(HE_EINVAL, "bad argument");
        MCHK(hipSetDevice(M->device));
        ensure_cap(M, m);
        // the data range maps to z in [-1, 1] (keeps z^4 well conditioned for heavy tails)
        float lo = u[0], hi = u[0];
        for (size_t i = 1; i < m; ++i) { lo = std::min(lo, u[i]); hi = std::max(hi, u[i]); }
        M->mean = 0.5f * (lo + hi);
        M->sd = std::max(1e-12f, 0.5f * (hi - lo));
        std::vector<float> sh(u, u + m);
        std::mt19937_64 rng(seed);
        for (size_t i = m - 1; i > 0; --i) std::swap(sh[i], sh[std::uniform_int_distribution<size_t>(0, i)(rng)]);
        MCHK(hipMemcpyAsync(M->d_u, sh.data(), m * 4, hipMemcpyHostToDevice, M->s));
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        for (uint32_t ep = 0; ep < epochs; ++ep) {
            // cosine decay of the step size over the run
            for (size_t off = 0; off < m; off += batch) {
                const size_t nb = std::min<size_t>(batch, m - off);
                const double prog = (ep + (double)off / m) / epochs;
                const float lr_t = (float)(lr * 0.5 * (1.0 + std::cos(M_PI * prog)));
                fill(M, M->d_grad, NP, 0.0f);
                hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((nb + MB - 1) / MB), dim3(MB), 0, M->s, M->d_u + off, (int)nb,
                                   M->d_theta, M->mean, M->sd, 1.0f / (float)nb, M->d_grad, (float *)nullptr,
                                   (float *)nullptr);
                ++M->step;
                const float c1 = 1.0f - std::pow(b1, (float)M->step), c2 = 1.0f - std::pow(b2, (float)M->step);
                hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, M->s, M->d_theta, M->d_grad,
                                   M->d_m1, M->d_m2, NP, lr_t, b1, b2, eps, c1, c2);
            }
        }
        fill(M, M->d_loss, 1, 0.0f);
        hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((m + MB - 1) / MB), dim3(MB), 0, M->s, M->d_u, (int)m, M->d_theta,
                           M->mean, M->sd, 0.0f, (float *)nullptr, M->d_loss, (float *)nullptr);
        MCHK(hipMemcpyAsync(final_loss, M->d_loss, 4, hipMemcpyDeviceToHost, M->s));
        MCHK(hipStreamSynchronize(M->s));
        MCHK(hipGetLastError());
        *final_loss /= (float)m;
        return HE_OK;
    });
}

// y(u) as a power-basis polynomial c0..c4, expanded in FP64 from the trained weights
int he_mlp_to_poly(const he_mlp *M, double *coef) {
    return mguard([&]() {
        if (!M || !coef) throw MErr(HE_EINVAL, "bad argument");
        MCHK(hipSetDevice(M->device));
        std::vector<float> th(NP);
        MCHK(hipMemcpy(th.data(), M->d_theta, NP * 4, hipMemcpyDeviceToHost));
        he::mlp_poly(th.data(), M->mean, M->sd, coef);
        return HE_OK;
    });
}

int he_mlp_save(const he_mlp *M, const char *path) {
    return mguard([&]() {
        if (!M || !path) throw MErr(HE_EINVAL, "bad argument");
        MCHK(hipSetDevice(M->device));
        MCHK(hipStreamSynchronize(M->s));
        std::vector<float> th(NP);
        MCHK(hipMemcpy(th.data(), M->d_theta, NP * 4, hipMemcpyDeviceToHost));
        std::string err;
        const int rc = he::mlp_file_write(path, th.data(), M->mean, M->sd, &err);
        if (rc != HE_OK) throw MErr(rc, err);
        return HE_OK;
    });
}

int he_mlp_load(const char *path, int device, he_mlp **out) {
    return mguard([&]() {
        if (!path || !out) throw MErr(HE_EINVAL, "bad argument");
        std::vector<float> th(NP);
        float mean = 0, sd = 1;
        std::string err;
        const int rc = he::mlp_file_read(path, th.data(), &mean, &sd, nullptr, &err);
        if (rc != HE_OK) throw MErr(rc, err);
        he_mlp *M = nullptr;
        int c = he_mlp_create(0, device, &M);
        if (c != HE_OK) return c;
        c = he_mlp_set_params(M, th.data(), NP, mean, sd);
        if (c != HE_OK) { he_mlp_destroy(M); return c; }
        *out = M;
        return (int)HE_OK;
    });
}

int he_mlp_file_poly(const char *path, double *coef) {
    return mguard([&]() {
        if (!path || !coef) throw MErr(HE_EINVAL, "bad argument");
        std::string err;
        const int rc = he::mlp_file_read(path, nullptr, nullptr, nullptr, coef, &err);
        if (rc != HE_OK) throw MErr(rc, err);
        return HE_OK;
    });
}

// variances of `runs` plaintext CutMax runs (see k_var_log); var_out[runs][T] and the
// mean of the last iterate ymean_out[runs] (may be null), host memory
int he_variance_log(uint64_t seed, uint32_t runs, uint32_t vocab, uint32_t slots, uint32_t T, uint32_t p, double c,
                    int device, float *var_out, float *ymean_out) {
    return mguard([&]() {
        if (!var_out || runs == 0 || T == 0 || T > 8 || vocab == 0 || slots < vocab || p == 0 || !(c > 0))
            throw MErr(HE_EINVAL, "bad argument");
        MCHK(hipSetDevice(device));
        float *dv = nullptr, *dm = nullptr;
        MCHK(hipMalloc(&dv, (size_t)runs * T * 4));
        MCHK(hipMalloc(&dm, (size_t)runs * 4));
        const int chunk = 65535;
        for (uint32_t r0 = 0; r0 < runs; r0 += chunk) {
            const int nr = (int)std::min<uint32_t>(chunk, runs - r0);
            hipLaunchKernelGGL(k_var_log, dim3(nr), dim3(VT), 0, 0, seed, (int)r0, (int)vocab, (int)slots, (int)T,
                               (int)p, c, dv, dm);
        }
        MCHK(hipDeviceSynchronize());
        MCHK(hipGetLastError());
        MCHK(hipMemcpy(var_out, dv, (size_t)runs * T * 4, hipMemcpyDeviceToHost));
        if (ymean_out) MCHK(hipMemcpy(ymean_out, dm, (size_t)runs * 4, hipMemcpyDeviceToHost));
        hipFree(dv);
        hipFree(dm);
        return HE_OK;
    });
}

}  // extern "C"
