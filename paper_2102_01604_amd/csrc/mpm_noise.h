// mpm_noise.h -- kernels of the noise estimation (paper Sec. 2.7): per image a
// histogram of the magnitudes and a two-class Rician mixture fitted to it.
#pragma once

#include "mpm_kernels.h"

namespace mpm {

constexpr int NOISE_MAX_BINS = 4096;
constexpr int NOISE_FIT_DOUBLES = 10;  // per image: pi0 pi1 nu0 nu1 sigma0 sigma1 mean0 mean1 nll ok

int noise_blocks(int64_t N);
// maxbits [I]: the largest finite value >= 0 of each image as FP32 bits (the
// caller zeroes it first; 0 if no value is > 0).
hipError_t launch_image_max(hipStream_t s, int dtype, const void *X, int64_t N, int I, uint32_t *maxbits);
// counts [I][nbins] (zeroed by the caller): finite values >= 0 binned over
// [0, max] with the bin floor(x * (nbins / max)) taken in FP32, the top value
// in the last bin.
hipError_t launch_image_hist(hipStream_t s, int dtype, const void *X, int64_t N, int I, int nbins,
                             const uint32_t *maxbits, uint32_t *counts);
// fits [I][NOISE_FIT_DOUBLES]: n_iter EM iterations per image, one workgroup
// each (class 0 the background, nu0 = 0); ok = 0 if the values do not split.
hipError_t launch_rice_em(hipStream_t s, const uint32_t *counts, const uint32_t *maxbits, int I, int nbins,
                          int n_iter, double *fits);

}  // namespace mpm
