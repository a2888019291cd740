// Probe of the HBM read rate the rotation key products can reach: S key streams per
// limb (each word a uint2 low part and a uint32 high part, as the packed keys), read once
// per position, in the library's row layout (one row per rotation and digit) and in a
// layout where the S rows of each 64-position wave block are contiguous; the row layout
// with 2-byte high parts on limbs 1..29 (the 40-bit primes of the top level of the
// secure set: a lane reads the dword of positions x and x ^ 1 and takes its half, as
// the library does); and a 1 GiB copy.
// Every access is in bounds: rows x N words, N = 65536, S <= 42, 40 limbs.
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       paper_2509_08383_amd/probes/key_streams.hip -o /tmp/key_streams && /tmp/key_streams
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>
#define CHK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("err %s line %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

template <int S>
__global__ __launch_bounds__(256) void rows(const uint2 *lo, const uint32_t *hi, double *out, int N, int limbs) {
    const int x = blockIdx.x * 256 + threadIdx.x;  // position
    const int t = blockIdx.y;                      // limb
    if (x >= N || t >= limbs) return;
    double s = 0;
#pragma unroll
    for (int r = 0; r < S; ++r) {
        const long long row = ((long long)t * S + r) * N;
        const uint2 l = lo[row + x];
        const uint32_t h = hi[row + x];
        s += (double)l.x + (double)l.y + (double)h;
    }
    out[(long long)t * N + x] = s;
}
// wave-blocked: for limb t, position block xb (64 positions), rows r: lo at
// ((t * (N/64) + xb) * S + r) * 64 + lane, same for hi
template <int S>
__global__ __launch_bounds__(256) void blocked(const uint2 *lo, const uint32_t *hi, double *out, int N, int limbs) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int t = blockIdx.y;
    if (x >= N || t >= limbs) return;
    const int xb = x >> 6, lane = x & 63;
    double s = 0;
    const long long base = ((long long)t * (N / 64) + xb) * S * 64 + lane;
#pragma unroll
    for (int r = 0; r < S; ++r) {
        const uint2 l = lo[base + r * 64];
        const uint32_t h = hi[base + r * 64];
        s += (double)l.x + (double)l.y + (double)h;
    }
    out[(long long)t * N + x] = s;
}
// rows, with 2-byte high parts on limbs [nlo, nhi]: the high row of such a limb holds N/2
// dwords (two positions each)
template <int S>
__global__ __launch_bounds__(256) void mixed(const uint2 *lo, const uint32_t *hi, double *out, int N, int limbs,
                                             int nlo, int nhi) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int t = blockIdx.y;
    if (x >= N || t >= limbs) return;
    const bool nr = t >= nlo && t <= nhi;
    double s = 0;
#pragma unroll
    for (int r = 0; r < S; ++r) {
        const long long row = ((long long)t * S + r) * N;
        const uint2 l = lo[row + x];
        const uint32_t h = hi[row + (nr ? (x >> 1) : x)] >> (nr ? 16u * ((unsigned)x & 1u) : 0u);
        s += (double)l.x + (double)l.y + (double)h;
    }
    out[(long long)t * N + x] = s;
}
__global__ void copyk(const double4 *a, double4 *b, long long n) {
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

template <int S>
int run(int limbs, const uint2 *lo, const uint32_t *hi, double *out, int N) {
    hipEvent_t a, b;
    CHK(hipEventCreate(&a)); CHK(hipEventCreate(&b));
    dim3 grid(N / 256, limbs);
    float best1 = 1e9, best2 = 1e9, best3 = 1e9;
    const int nlo = 1, nhi = limbs >= 30 ? 29 : limbs - 1;
    for (int it = 0; it < 6; ++it) {
        CHK(hipEventRecord(a));
        hipLaunchKernelGGL(rows<S>, grid, dim3(256), 0, 0, lo, hi, out, N, limbs);
        CHK(hipEventRecord(b)); CHK(hipEventSynchronize(b));
        float ms; CHK(hipEventElapsedTime(&ms, a, b)); if (it) best1 = ms < best1 ? ms : best1;
        CHK(hipEventRecord(a));
        hipLaunchKernelGGL(blocked<S>, grid, dim3(256), 0, 0, lo, hi, out, N, limbs);
        CHK(hipEventRecord(b)); CHK(hipEventSynchronize(b));
        CHK(hipEventElapsedTime(&ms, a, b)); if (it) best2 = ms < best2 ? ms : best2;
        CHK(hipEventRecord(a));
        hipLaunchKernelGGL(mixed<S>, grid, dim3(256), 0, 0, lo, hi, out, N, limbs, nlo, nhi);
        CHK(hipEventRecord(b)); CHK(hipEventSynchronize(b));
        CHK(hipEventElapsedTime(&ms, a, b)); if (it) best3 = ms < best3 ? ms : best3;
    }
    const double bytes = (double)limbs * N * (S * 12.0 + 8.0);
    const int nn = nhi - nlo + 1;
    const double bytes3 = (double)N * (limbs * (S * 12.0 + 8.0) - nn * S * 2.0);
    printf("S=%2d limbs=%d  rows: %.1f us %.0f GB/s   blocked: %.1f us %.0f GB/s   5-byte rows on %d limbs: %.1f us "
           "%.0f GB/s\n",
           S, limbs, best1 * 1e3, bytes / best1 / 1e6, best2 * 1e3, bytes / best2 / 1e6, nn, best3 * 1e3,
           bytes3 / best3 / 1e6);
    return 0;
}

int main() {
    const int N = 65536, limbs = 40, SMAX = 42;
    const size_t words = (size_t)limbs * SMAX * N;
    uint2 *lo; uint32_t *hi; double *out;
    CHK(hipMalloc(&lo, words * 8)); CHK(hipMalloc(&hi, words * 4)); CHK(hipMalloc(&out, (size_t)limbs * N * 8));
    CHK(hipMemset(lo, 1, words * 8)); CHK(hipMemset(hi, 1, words * 4));
    // copy reference: 1 GiB
    {
        const long long n = (1ll << 30) / 32;
        double4 *A, *B;
        CHK(hipMalloc(&A, n * 32)); CHK(hipMalloc(&B, n * 32));
        CHK(hipMemset(A, 0, n * 32));
        hipEvent_t a, b; CHK(hipEventCreate(&a)); CHK(hipEventCreate(&b));
        float best = 1e9;
        for (int it = 0; it < 5; ++it) {
            CHK(hipEventRecord(a));
            hipLaunchKernelGGL(copyk, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, A, B, n);
            CHK(hipEventRecord(b)); CHK(hipEventSynchronize(b));
            float ms; CHK(hipEventElapsedTime(&ms, a, b)); if (it) best = ms < best ? ms : best;
        }
        printf("copy 1 GiB: %.0f GB/s (read+write)\n", 2.0 * n * 32 / best / 1e6);
        CHK(hipFree(A)); CHK(hipFree(B));
    }
    if (run<1>(limbs, lo, hi, out, N)) return 1;
    if (run<6>(limbs, lo, hi, out, N)) return 1;
    if (run<21>(limbs, lo, hi, out, N)) return 1;
    if (run<42>(limbs, lo, hi, out, N / 2)) return 1;
    CHK(hipDeviceSynchronize());
    return 0;
}
