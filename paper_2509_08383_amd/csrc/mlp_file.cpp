// File form of the learned initial guess (he_mlp_save / he_mlp_load / he_mlp_file_poly):
// the trained weights, the input normalisation and the degree-4 polynomial they collapse
// to, so that a serving process can read the polynomial (he_cutmax_cfg.init_coef)
// without a GPU and a training process can resume from the weights.  Host code only.
//
// Layout (little-endian, 1356 bytes):
//   0     char[8]   "HEMLPv1\n"
//   8     uint32    parameter count (321)      12  uint32  hidden width (16)
//   16    float32   mean                       20  float32 sd
//   24    float32   theta[321]  (W1, b1, W2 row-major by output, b2, W3, b3)
//   1308  float64   poly[5]     (power basis in u)
//   1348  uint64    FNV-1a 64 of bytes 0..1347
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/he.h"
#include "mlp_file.h"

namespace he {
namespace {

constexpr char kMagic[8] = {'H', 'E', 'M', 'L', 'P', 'v', '1', '\n'};
constexpr size_t kBodyBytes = 8 + 4 + 4 + 4 + 4 + 4 * (size_t)kMlpParams + 8 * 5;
constexpr size_t kFileBytes = kBodyBytes + 8;

uint64_t fnv1a64(const unsigned char *p, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

template <class T>
void put(std::vector<unsigned char> &b, size_t off, T v) {
    std::memcpy(b.data() + off, &v, sizeof v);
}
template <class T>
T get(const std::vector<unsigned char> &b, size_t off) {
    T v;
    std::memcpy(&v, b.data() + off, sizeof v);
    return v;
}

}  // namespace

void mlp_poly(const float *th, double mean, double sd, double coef[5]) {
    const int H = kMlpHidden, NP = kMlpParams;
    // z = (u - mean)/sd = z0 + z1 u; a1_k = (W1_k z + b1_k)^2 is a quadratic in u
    const double z0 = -mean / sd, z1 = 1.0 / sd;
    double y[5] = {0, 0, 0, 0, 0};
    std::vector<double> A1(3 * H);
    for (int k = 0; k < H; ++k) {
        const double l0 = th[k] * z0 + th[H + k], l1 = th[k] * z1;
        A1[3 * k] = l0 * l0;
        A1[3 * k + 1] = 2 * l0 * l1;
        A1[3 * k + 2] = l1 * l1;
    }
    // h2_j = W2_j . a1 + b2_j (quadratic), y = sum_j W3_j h2_j^2 + b3 (quartic)
    for (int j = 0; j < H; ++j) {
        double h[3] = {th[2 * H + H * H + j], 0, 0};
        for (int k = 0; k < H; ++k)
            for (int d = 0; d < 3; ++d) h[d] += (double)th[2 * H + j * H + k] * A1[3 * k + d];
        const double w = th[3 * H + H * H + j];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) y[a + b] += w * h[a] * h[b];
    }
    y[0] += th[NP - 1];
    for (int d = 0; d < 5; ++d) coef[d] = y[d];
}

int mlp_file_write(const char *path, const float *theta, float mean, float sd, std::string *err) {
    std::vector<unsigned char> b(kFileBytes, 0);
    std::memcpy(b.data(), kMagic, 8);
    put<uint32_t>(b, 8, (uint32_t)kMlpParams);
    put<uint32_t>(b, 12, (uint32_t)kMlpHidden);
    put<float>(b, 16, mean);
    put<float>(b, 20, sd);
    std::memcpy(b.data() + 24, theta, 4 * (size_t)kMlpParams);
    double poly[5];
    mlp_poly(theta, mean, sd, poly);
    std::memcpy(b.data() + 24 + 4 * (size_t)kMlpParams, poly, sizeof poly);
    put<uint64_t>(b, kBodyBytes, fnv1a64(b.data(), kBodyBytes));
    // written beside the target and renamed over it, so a reader never sees half a file
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) { *err = "cannot open " + tmp + " for writing"; return HE_EIO; }
    const bool ok = std::fwrite(b.data(), 1, b.size(), f) == b.size();
    if (std::fclose(f) != 0 || !ok) {
        std::remove(tmp.c_str());
        *err = "short write to " + tmp;
        return HE_EIO;
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        *err = std::string("cannot rename onto ") + path;
        return HE_EIO;
    }
    return HE_OK;
}

int mlp_file_read(const char *path, float *theta, float *mean, float *sd, double poly[5], std::string *err) {
    FILE *f = std::fopen(path, "rb");
    if (!f) { *err = std::string("cannot open ") + path; return HE_EIO; }
    std::vector<unsigned char> b(kFileBytes + 1);
    const size_t got = std::fread(b.data(), 1, b.size(), f);
    std::fclose(f);
    if (got != kFileBytes) {
        *err = std::string(path) + ": " + std::to_string(got) + " bytes, expected " + std::to_string(kFileBytes);
        return HE_EINVAL;
    }
    b.resize(kFileBytes);
    if (std::memcmp(b.data(), kMagic, 8) != 0) { *err = std::string(path) + ": not a learned-guess file"; return HE_EINVAL; }
    if (get<uint32_t>(b, 8) != (uint32_t)kMlpParams || get<uint32_t>(b, 12) != (uint32_t)kMlpHidden) {
        *err = std::string(path) + ": network shape differs from this library's";
        return HE_EINVAL;
    }
    if (get<uint64_t>(b, kBodyBytes) != fnv1a64(b.data(), kBodyBytes)) {
        *err = std::string(path) + ": checksum mismatch";
        return HE_EINVAL;
    }
    const float m = get<float>(b, 16), s = get<float>(b, 20);
    std::vector<float> th(kMlpParams);
    std::memcpy(th.data(), b.data() + 24, 4 * (size_t)kMlpParams);
    double p[5], q[5];
    std::memcpy(p, b.data() + 24 + 4 * (size_t)kMlpParams, sizeof p);
    bool finite = std::isfinite(m) && std::isfinite(s) && s > 0;
    for (float v : th) finite = finite && std::isfinite(v);
    if (!finite) { *err = std::string(path) + ": non-finite weights or sd <= 0"; return HE_EINVAL; }
    // the stored polynomial must be the collapse of the stored weights
    mlp_poly(th.data(), m, s, q);
    double scale = 0.0;
    for (int d = 0; d < 5; ++d) scale = std::fmax(scale, std::fabs(q[d]));
    for (int d = 0; d < 5; ++d)
        if (!(std::fabs(p[d] - q[d]) <= 1e-9 * scale)) {
            *err = std::string(path) + ": stored polynomial is not the collapse of the stored weights";
            return HE_EINVAL;
        }
    if (theta) std::memcpy(theta, th.data(), 4 * (size_t)kMlpParams);
    if (mean) *mean = m;
    if (sd) *sd = s;
    if (poly) std::memcpy(poly, p, sizeof p);
    return HE_OK;
}

}  // namespace he
