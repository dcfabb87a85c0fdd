// mpm_kernels.h -- host-callable launchers of libmpm's kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpm_device.h"

namespace mpm {

enum Dtype { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2 };

// Every launcher returns the hipError_t of its launch.
struct LaunchCtx {
    hipStream_t stream;
};

// --- voxelwise kernels (k_voxel.hip) ---
hipError_t launch_fill_maps(const LaunchCtx &c, float *maps, int64_t N, const float y0[4]);
hipError_t launch_fill(const LaunchCtx &c, float *p, int64_t n, float v);
hipError_t launch_simulate(const LaunchCtx &c, const DevProto &P, const float *maps, const float *b1,
                           const float *noise, int dtype, void *out, int64_t N);
// per-image sums and counts of the finite echo values (+ the b1 sum in row
// 2I) -> partials[(2I+1)][nblk]
hipError_t launch_echo_sums(const LaunchCtx &c, const DevProto &P, int dtype, const void *X,
                            const float *b1, int64_t N, double *partials, int nblk);
int echo_sums_blocks(int64_t N);
// ML fit: n_gn steps per voxel, echoes register-resident.  partials rows:
// [0..n_gn] NLL before each step / final, then degenerate, nonfinite, increases
hipError_t launch_ml_fit(const LaunchCtx &c, const DevProto &P, int dtype, const void *X,
                         const float *b1, const float *bm, float *maps, int64_t N, int n_gn, int loading,
                         double *partials, int nblk);
int ml_fit_blocks(int64_t N);
// per-image offsets of reduced-precision storage
struct EchoOffsets {
    float v[MAXI];
};
// dst[i][n] = round(src[i][n] - off.v[i]) in dtype (F16 / BF16); *overflow +=
// the finite inputs whose stored value is not finite
hipError_t launch_pack_echoes(const LaunchCtx &c, int I, int64_t N, const float *src, int dtype, void *dst,
                              const EchoOffsets &off, unsigned int *overflow);
// out[r] = sum over b < ncols of in[r*ncols + b] (fixed order)
hipError_t launch_reduce_rows(const LaunchCtx &c, const double *in, int nrows, int ncols, double *out);

}  // namespace mpm
