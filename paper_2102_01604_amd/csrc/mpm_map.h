// mpm_map.h -- shared declarations of the MAP (JTV) kernels and their host driver.
#pragma once

#include <hip/hip_runtime.h>

#include "mpm_kernels.h"

namespace mpm {

constexpr int TILE_X = 64;   // voxels along x per workgroup (one wavefront)
constexpr int TILE_Y = 4;    // rows along y per workgroup
constexpr int MAX_TRIALS = 8;  // step sizes 1, 1/2, ..., 1/128 evaluated by one accept pass

struct Grid3 {
    int nx, ny, nz;
    int gx, gy;   // tiles along x and y
    int64_t N;
};

inline Grid3 make_grid3(int64_t nx, int64_t ny, int64_t nz)
{
    Grid3 g;
    g.nx = (int)nx;
    g.ny = (int)ny;
    g.nz = (int)nz;
    g.gx = (int)((nx + TILE_X - 1) / TILE_X);
    g.gy = (int)((ny + TILE_Y - 1) / TILE_Y);
    g.N = nx * ny * nz;
    return g;
}

// Device-resident scalars of the MAP iteration (FP64).
struct MapCtl {
    double F;           // F_w at the current maps
    double yLy;         // y^T L y at the current maps
    double gamma, gamma0, alpha_pend, beta;
    double step;        // accepted step length of this Newton step (0: none)
    double nll_cur;     // NLL at the current maps
    double jtv;         // smoothed JTV at the last weight refresh
    double nll_final, degenerate, nonfinite;
    int gn_stop;        // remaining Newton steps of this outer loop are skipped
    int cg_stop;        // remaining CG iterations of this Newton step are skipped
    int delta_valid;    // the delta buffer holds a CG partial sum
    int p_buf;          // buffer holding the last search direction
    int cg_done, gn_done, rejected, pad;
};

enum { FIN_LIK = 0, FIN_A = 1, FIN_B = 2, FIN_ACCEPT = 3, FIN_W = 4, FIN_STATS = 5 };

struct MapArgs {
    Grid3 g;
    DevProto P;
    int dtype;
    const void *X;
    const float *b1;
    float *Y;      // maps [4][N]
    float *w;      // JTV weights [N]
    float *H;      // packed loaded Hessian [10][N]
    float *R, *Z, *P0, *P1, *D;  // CG vectors [4][N]
    float lam[4];
    float eps;
    int loading;
    MapCtl *ctl;
    double *partials;   // [MAX_TRIALS + 2][nblk]
    double *trace;      // device copy of the objective trace
};

hipError_t launch_ctl_init(hipStream_t s, MapCtl *ctl, double *trace, int trace_len);
hipError_t launch_lik(hipStream_t s, const MapArgs &a);
hipError_t launch_cg_a(hipStream_t s, const MapArgs &a, int it);
hipError_t launch_cg_b(hipStream_t s, const MapArgs &a, int it);
hipError_t launch_accept(hipStream_t s, const MapArgs &a, int ntrial);
hipError_t launch_update(hipStream_t s, const MapArgs &a);
hipError_t launch_weights(hipStream_t s, const MapArgs &a, int prior_on);
hipError_t launch_final(hipStream_t s, const MapArgs &a, float *var, float *mom);
hipError_t launch_fin(hipStream_t s, const MapArgs &a, int stage, int arg, double cg_stop_rel, int ntrial,
                      int accept_off);

}  // namespace mpm
