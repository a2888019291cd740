// Host-only helpers of the learned initial guess: the collapse of the network to its
// degree-4 polynomial and the file form of the trained weights (layout in mlp_file.cpp).
#pragma once
#include <string>

namespace he {

constexpr int kMlpHidden = 16;
constexpr int kMlpParams = kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden + 1;  // 321

// y(u) of the network with weights th and input normalisation (mean, sd), expanded in FP64
// into power-basis coefficients coef[0..4]
void mlp_poly(const float *th, double mean, double sd, double coef[5]);
// HE_OK, or HE_EIO (open, read, write or rename failed) or HE_EINVAL (the content is not
// a valid file) with *err set; the read checks the size, magic, shape, checksum, finiteness
// and that the stored polynomial is the collapse of the stored weights.  Output pointers
// of the read may be null.
int mlp_file_write(const char *path, const float *theta, float mean, float sd, std::string *err);
int mlp_file_read(const char *path, float *theta, float *mean, float *sd, double poly[5], std::string *err);

}  // namespace he
