// mpm_map.h -- shared declarations of the MAP (JTV) kernels and their host driver.
#pragma once

#include <hip/hip_runtime.h>

#include "mpm_kernels.h"

namespace mpm {

constexpr int TILE_X = 64;   // voxels along x per workgroup (one wavefront)
constexpr int TILE_Y = 4;    // rows along y per workgroup (256 threads)
constexpr int MAX_TRIALS = 8;  // step sizes 1, 1/2, ..., 1/128 of the acceptance test
constexpr int TALL_Y = 16;            // rows of a CG-sweep tile (1024 threads)
constexpr int TALL_WORKGROUPS = 2048; // 4 rounds of 2 workgroups per CU

// Stencil kernels walk columns: a workgroup owns a TILE_X x TILE_Y tile of
// the x-y plane and a run of zc consecutive planes.
struct Grid3 {
    int nx, ny, nz;
    int gx, gy, gz;  // tiles along x and y, z-runs along z
    int zc;          // planes per z-run
    int ty;          // tile rows along y (threads per workgroup = TILE_X * ty)
    int64_t N;
};

constexpr int TARGET_WORKGROUPS = 8192;  // 32 per CU: short enough columns, many workgroups in flight

// Number of column workgroups to aim for; MPM_STENCIL_WORKGROUPS overrides it
// (a tuning knob: longer columns mean fewer z-halo planes, fewer workgroups).
int stencil_workgroups();

inline Grid3 make_grid3(int64_t nx, int64_t ny, int64_t nz, int ty = TILE_Y, int64_t target = 0)
{
    Grid3 g;
    g.nx = (int)nx;
    g.ny = (int)ny;
    g.nz = (int)nz;
    g.ty = ty;
    g.gx = (int)((nx + TILE_X - 1) / TILE_X);
    g.gy = (int)((ny + ty - 1) / ty);
    int64_t tiles = (int64_t)g.gx * g.gy;
    if (target <= 0) target = stencil_workgroups();
    int64_t zc = (tiles * nz + target - 1) / target;
    if (zc < 1) zc = 1;
    if (zc > 32) zc = 32;
    if (zc > nz) zc = nz;
    g.zc = (int)zc;
    g.gz = (int)((nz + zc - 1) / zc);
    g.N = nx * ny * nz;
    return g;
}

inline int grid_blocks(const Grid3 &g) { return (int)((int64_t)g.gx * g.gy * g.gz); }

// The same grid walked one plane per workgroup (for the echo-heavy kernels,
// where more independent workgroups hide the arithmetic better).
inline Grid3 plane_grid(Grid3 g)
{
    g.zc = 1;
    g.gz = g.nz;
    return g;
}

// Loaded Hessian of every voxel, split into coalesced vector arrays:
// d = (00, 11, 22, 33), o = (01, 02, 03, 12), r = (13, 23).
struct HessArrays {
    float4 *d;
    float4 *o;
    float2 *r;
};

// Device-resident scalars of the MAP iteration (FP64).
struct MapCtl {
    double F;           // F_w at the current maps
    double yLy;         // y^T L y at the current maps
    double gamma, gamma0, alpha_pend, beta;
    double step;        // accepted step length of this Newton step (0: none)
    double nll_cur;     // NLL at the current maps
    double jtv;         // smoothed JTV at the last weight refresh
    double nll_final, degenerate, nonfinite;
    double c1, c2;      // delta.(L y) and delta.(L delta) of the current step
    int gn_stop;        // remaining Newton steps of this outer loop are skipped
    int cg_stop;        // remaining CG iterations of this Newton step are skipped
    int delta_valid;    // the delta buffer holds a CG partial sum
    int p_buf;          // buffer holding the last search direction
    int cg_done, gn_done, rejected;
    int accept_more;    // the full step was rejected: evaluate the halvings
};

enum { FIN_LIK = 0, FIN_A = 1, FIN_B = 2, FIN_ACCEPT = 3, FIN_W = 4, FIN_STATS = 5, FIN_ACCEPT2 = 6 };

struct MapArgs {
    Grid3 g;
    DevProto P;
    int dtype;
    const void *X;
    const float *b1;
    float *Y;      // maps [4][N]
    float *w;      // JTV weights [N]
    Grid3 gp;      // one plane per workgroup
    Grid3 gt;      // tall tiles (TILE_X x TALL_Y) for the CG sweeps
    Grid3 gv;      // CG sweep B: one voxel per thread, tiles of TILE_X x cg_b_rows() (plane grid)
    HessArrays H;  // loaded Hessian per voxel
    float4 *R, *Z, *P0, *P1, *D;  // CG vectors, one float4 per voxel
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
hipError_t launch_accept(hipStream_t s, const MapArgs &a);
hipError_t launch_accept2(hipStream_t s, const MapArgs &a, int ntrial);
hipError_t launch_update(hipStream_t s, const MapArgs &a);
hipError_t launch_weights(hipStream_t s, const MapArgs &a, int prior_on);
hipError_t launch_final(hipStream_t s, const MapArgs &a, float *var, float *mom);
int cg_a_blocks(const MapArgs &a);  // workgroups (partials) of CG sweep A
int cg_b_blocks(const MapArgs &a);  // ... and of sweep B
int cg_b_rows();                    // tile rows of sweep B
int tall_workgroups();
hipError_t launch_fin(hipStream_t s, const MapArgs &a, int stage, int arg, int nblk, double cg_stop_rel,
                      int ntrial, int accept_off);

}  // namespace mpm
