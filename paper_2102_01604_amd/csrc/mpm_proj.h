// mpm_proj.h -- spatial projection (paper Sec. 2.4, "Spatial projection"):
// each contrast is acquired on its own grid; the log-parameter maps (and b1)
// live on the reconstruction grid and are resliced ("pulled") into every
// acquisition space, where the likelihood is evaluated; gradients and loaded
// Hessian blocks are sent back with the adjoint ("pushed").
//
// Reslicing: acquisition voxel (i, j, k) lies at reconstruction coordinates
// r = A (i, j, k, 1)^T; trilinear interpolation with replicated borders
// (corner indices clamped, so the weights of a voxel sum to 1); acquisition
// voxels with r outside [-1/2, n_d - 1/2] on some axis d lie outside the
// reconstruction field of view and carry no observation.  Push of the loaded
// Hessian: P~_n = sum_m Psi_mn P~_m, the block-diagonal majoriser of
// Psi^T P~ Psi (rows of Psi sum to 1).
#pragma once

#include <cmath>

#include "../../include/mpm.h"
#include "mpm_map.h"

namespace mpm {

struct ProjSpace {
    int mx, my, mz;
    int64_t M;        // mx * my * mz
    double A[12];     // acquisition index -> reconstruction coordinates (row-major 3x4)
    double Ainv[12];  // reconstruction coordinates -> acquisition index
    double rA0[3];    // 1 / A[d][0], or 0 where |A[d][0]| < 1e-12 (no bound on i from axis d)
};

// Host: the space with its inverse affine (validated invertible beforehand).
inline ProjSpace make_proj_space(const mpm_space &sp)
{
    ProjSpace S;
    S.mx = (int)sp.nx;
    S.my = (int)sp.ny;
    S.mz = (int)sp.nz;
    S.M = sp.nx * sp.ny * sp.nz;
    const double *a = sp.affine;
    for (int k = 0; k < 12; k++) S.A[k] = a[k];
    const double R[9] = {a[0], a[1], a[2], a[4], a[5], a[6], a[8], a[9], a[10]};
    const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                       R[2] * (R[3] * R[7] - R[4] * R[6]);
    const double inv[9] = {(R[4] * R[8] - R[5] * R[7]) / det, (R[2] * R[7] - R[1] * R[8]) / det,
                           (R[1] * R[5] - R[2] * R[4]) / det, (R[5] * R[6] - R[3] * R[8]) / det,
                           (R[0] * R[8] - R[2] * R[6]) / det, (R[2] * R[3] - R[0] * R[5]) / det,
                           (R[3] * R[7] - R[4] * R[6]) / det, (R[1] * R[6] - R[0] * R[7]) / det,
                           (R[0] * R[4] - R[1] * R[3]) / det};
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) S.Ainv[4 * r + c] = inv[3 * r + c];
        S.Ainv[4 * r + 3] = -(inv[3 * r] * a[3] + inv[3 * r + 1] * a[7] + inv[3 * r + 2] * a[11]);
    }
    for (int d = 0; d < 3; d++) S.rA0[d] = std::fabs(a[4 * d]) < 1e-12 ? 0.0 : 1.0 / a[4 * d];
    return S;
}

// Position of acquisition voxel (i, j, k) on the reconstruction grid g, the
// field-of-view test, and its 8 corners and trilinear weights.  Pull and push
// both call this, so they use the same weights.
struct Corners {
    int64_t idx[8];
    float w[8];
};

__device__ __forceinline__ bool proj_corners(const Grid3 &g, const ProjSpace &S, int i, int j, int k, Corners &cr)
{
    const int nd[3] = {g.nx, g.ny, g.nz};
    float t[3];
    int lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double r = S.A[4 * d] * i + S.A[4 * d + 1] * j + S.A[4 * d + 2] * k + S.A[4 * d + 3];
        if (!(r >= -0.5 && r <= nd[d] - 0.5)) return false;
        const double f = floor(r);
        t[d] = (float)(r - f);
        lo[d] = max((int)f, 0);
        hi[d] = min((int)f + 1, nd[d] - 1);
    }
#pragma unroll
    for (int c = 0; c < 8; c++) {
        const int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
        cr.idx[c] = (int64_t)(bx ? hi[0] : lo[0]) + (int64_t)g.nx * ((by ? hi[1] : lo[1]) + (int64_t)g.ny * (bz ? hi[2] : lo[2]));
        cr.w[c] = (bx ? t[0] : 1.0f - t[0]) * (by ? t[1] : 1.0f - t[1]) * (bz ? t[2] : 1.0f - t[2]);
    }
    return true;
}

// Blocks of one contrast's acquisition voxels: gradient and loaded Hessian.
struct ProjBlocks {
    float4 *G;
    HessArrays H;
};

struct ProjPushArgs {
    int C;
    ProjSpace S[MAXC];
    ProjBlocks B[MAXC];
};

// Recon-space blocks after the push, read by the MAP kernels in place of the
// echoes (VoxelEchoes<Pushed, 0, 0>).
struct Pushed {};
struct PushedProto {
    const float4 *G;
    HessArrays H;
};

// The pushed blocks as the MAP kernels' echo source: g and the loaded Hessian
// are read, the NLL lives in the acquisition-space partials (0 here).
template <>
struct VoxelEchoes<Pushed, 0, 0> {
    using Proto = PushedProto;
    using Consts = const void *;
    int64_t n;
    static __device__ __forceinline__ Consts stage(const Proto &) { return nullptr; }
    __device__ __forceinline__ void load(const Proto &, const Pushed *, int64_t, int64_t n_, float, float = 1.0f)
    {
        n = n_;
    }
    template <bool PLUS>
    __device__ __forceinline__ float lik(const Proto &P, Consts, const float *, int, bool, float g[4],
                                         float H[10]) const
    {
        vload(P.G, n, g);
        load_H(P.H, n, H);
        return 0.0f;
    }
    __device__ __forceinline__ float nll(const Proto &, Consts, const float *) const { return 0.0f; }
};

// One contrast of a projected likelihood launch.
struct ProjContrast {
    ProjSpace S;
    DevProto P;       // the protocol restricted to this contrast
    const void *X;    // its first image (images of M voxels, back to back)
    ProjBlocks B;
    int ext_col;      // first partial column of this contrast in the extra rows
};

// Acquisition space: pull, likelihood blocks, NLL partial (extra row 0), at
// the current maps, or at the trial point Yt (from launch_trial_point) when
// Yt is given.  gated (current maps): return when the control block says the
// Newton step is skipped or the blocks are current (the previous step took its
// full step).
hipError_t launch_proj_lik(hipStream_t s, const MapArgs &m, const ProjContrast &pc, double *ext, int gated,
                           const float4 *Yt = nullptr);
// Yt = y - delta_f [N] (float4 per reconstruction voxel), gated like the step.
hipError_t launch_trial_point(hipStream_t s, const MapArgs &m, float4 *Yt);
// NLL at y - 2^-h delta_f for h in [h0, h1) (extra rows h); h0 > 0 runs only
// after the full step was rejected.
hipError_t launch_proj_nll(hipStream_t s, const MapArgs &m, const ProjContrast &pc, double *ext, int ext_stride,
                           int h0, int h1);
// Column grid of an acquisition space; its workgroups are the partial columns
// of one contrast's launch.
inline Grid3 proj_grid(const ProjSpace &S) { return make_grid3(S.mx, S.my, S.mz); }
int proj_blocks(const ProjSpace &S);
// Reconstruction space: gather every contrast's blocks -> G [N], H.
hipError_t launch_proj_push(hipStream_t s, const MapArgs &m, const ProjPushArgs &pa, float4 *G, HessArrays H);
// Psi^T stored by reconstruction voxel: rows ci * N + n (contrast-major),
// row pointers row[0 .. C N], entries (m, bits of w) in the order of the
// direct push; at most 8 entries per acquisition voxel.
struct PsiT {
    int64_t *row;
    int2 *ent;
};
int64_t psi_scan_blocks(int64_t rows);  // scratch int64 values of the build's scan
hipError_t launch_psi_build(hipStream_t s, const Grid3 &g, const ProjPushArgs &pa, const PsiT &psi, int64_t *scan_tmp);
hipError_t launch_proj_push_csr(hipStream_t s, const MapArgs &m, const ProjPushArgs &pa, const PsiT &psi, float4 *G,
                                HessArrays H);
// Pulled maps [4][M] and b1 [M] (NaN outside the field of view).
hipError_t launch_proj_pull(hipStream_t s, const Grid3 &g, const ProjSpace &S, const float *Y, const float *b1,
                            float *Yp, float *bp);

// MAP kernels on pushed blocks (k_map.hip); the extra rows carry the NLL.
hipError_t launch_lik_pushed(hipStream_t s, const MapArgs &a, const PushedProto &pp);
hipError_t launch_accept_pushed(hipStream_t s, const MapArgs &a, const PushedProto &pp);
hipError_t launch_final_pushed(hipStream_t s, const MapArgs &a, const PushedProto &pp, float *var, float *mom);

}  // namespace mpm
