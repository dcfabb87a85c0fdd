// k_proj.hip -- kernels of the spatial projection (paper Sec. 2.4, "Spatial
// projection"); the reslicing convention is in mpm_proj.h.
//
//   k_proj_lik   acquisition space, one launch per contrast: pull y and b1,
//                likelihood block of the contrast's echoes (NLL, g, loaded
//                Hessian) -> per-voxel blocks and an NLL partial;
//   k_proj_nll   acquisition space: NLL at trial steps y - 2^-h delta_f;
//   k_proj_push  reconstruction space: gather every contrast's blocks,
//                g_n = sum_m Psi_mn g_m, P~_n = sum_m Psi_mn P~_m, in a fixed
//                order (deterministic, no atomics): a voxel visits the
//                acquisition voxels inside the inverse-affine image of its
//                interpolation support;
//   k_proj_pull  pulled maps and b1 of one space (for simulation).
#include "mpm_proj.h"

namespace mpm {

// Block sums of v[0..NV) written to base[k * stride + blockIdx.x].
template <int NV>
__device__ __forceinline__ void write_rows(double (&v)[NV], double *__restrict__ base, int stride)
{
    __shared__ double lds[NV][NWAVE];
    block_sum<NV>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) base[(int64_t)k * stride + blockIdx.x] = v[k];
    }
}

__device__ __forceinline__ void acq_index(const ProjSpace &S, int64_t m, int &i, int &j, int &k)
{
    i = (int)(m % S.mx);
    j = (int)((m / S.mx) % S.my);
    k = (int)(m / ((int64_t)S.mx * S.my));
}

// Pulled maps and b1 at the corners cr.
__device__ __forceinline__ void pull_y_b1(const Grid3 &g, const Corners &cr, const float *__restrict__ Y,
                                          const float *__restrict__ b1, float y[4], float &b)
{
#pragma unroll
    for (int a = 0; a < 4; a++) y[a] = 0.0f;
    b = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; c++) {
#pragma unroll
        for (int a = 0; a < 4; a++) y[a] += cr.w[c] * Y[a * g.N + cr.idx[c]];
        b += cr.w[c] * (b1 ? b1[cr.idx[c]] : 1.0f);
    }
}

template <typename T, int CM1, int EM, bool PLUS>
__global__ __launch_bounds__(BLOCK) void k_proj_lik(Grid3 g, ProjSpace S, typename VoxelEchoes<T, CM1, EM>::Proto P,
                                                    const T *__restrict__ X, const float *__restrict__ Y,
                                                    const float *__restrict__ b1, int loading, ProjBlocks B,
                                                    const MapCtl *__restrict__ ctl, int gated,
                                                    double *__restrict__ ext)
{
    if (gated && ctl->gn_stop) return;
    const auto K = VoxelEchoes<T, CM1, EM>::stage(P);
    const int64_t m = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double part[1] = {0.0};
    if (m < S.M) {
        int i, j, k;
        acq_index(S, m, i, j, k);
        float gl[4] = {0.f, 0.f, 0.f, 0.f}, H[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        Corners cr;
        if (proj_corners(g, S, i, j, k, cr)) {
            float y[4], b;
            pull_y_b1(g, cr, Y, b1, y, b);
            VoxelEchoes<T, CM1, EM> ve;
            ve.load(P, X, S.M, m, b);
            part[0] = ve.template lik<PLUS>(P, K, y, loading, true, gl, H);
        }
        vstore_nt(B.G, m, gl);
        store_H(B.H, m, H);
    }
    write_rows<1>(part, ext, 0);
}

template <typename T, int CM1, int EM>
__global__ __launch_bounds__(BLOCK) void k_proj_nll(Grid3 g, ProjSpace S, typename VoxelEchoes<T, CM1, EM>::Proto P,
                                                    const T *__restrict__ X, const float *__restrict__ Y,
                                                    const float *__restrict__ b1, const float4 *__restrict__ D,
                                                    const float4 *__restrict__ P0, const float4 *__restrict__ P1,
                                                    int h0, int h1, const MapCtl *__restrict__ ctl,
                                                    double *__restrict__ ext, int ext_stride)
{
    if (ctl->gn_stop || (h0 > 0 && !ctl->accept_more)) return;
    const DeltaF getd{D, ctl->p_buf ? P1 : P0, (float)ctl->alpha_pend, ctl->delta_valid != 0};
    const auto K = VoxelEchoes<T, CM1, EM>::stage(P);
    const int64_t m = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double part[MAX_TRIALS];
#pragma unroll
    for (int h = 0; h < MAX_TRIALS; h++) part[h] = 0.0;
    if (m < S.M) {
        int i, j, k;
        acq_index(S, m, i, j, k);
        Corners cr;
        if (proj_corners(g, S, i, j, k, cr)) {
            float y[4], b, dl[4] = {0.f, 0.f, 0.f, 0.f};
            pull_y_b1(g, cr, Y, b1, y, b);
#pragma unroll
            for (int c = 0; c < 8; c++) {
                float dv[4];
                getd(cr.idx[c], dv);
#pragma unroll
                for (int a = 0; a < 4; a++) dl[a] += cr.w[c] * dv[a];
            }
            VoxelEchoes<T, CM1, EM> ve;
            ve.load(P, X, S.M, m, b);
            float step = ldexpf(1.0f, -h0);
#pragma unroll 1
            for (int h = h0; h < h1; h++) {
                float yt[4];
#pragma unroll
                for (int a = 0; a < 4; a++) yt[a] = y[a] - step * dl[a];
                const float v = ve.nll(P, K, yt);
#pragma unroll
                for (int q = 0; q < MAX_TRIALS; q++)
                    if (q == h) part[q] = v;
                step *= 0.5f;
            }
        }
    }
    __shared__ double lds[MAX_TRIALS][NWAVE];
    block_sum<MAX_TRIALS>(part, lds);
    if (threadIdx.x == 0)
        for (int h = h0; h < h1; h++) ext[(int64_t)h * ext_stride + blockIdx.x] = part[h];
}

// Weight of reconstruction voxel n = (x, y, z) in the pull of acquisition voxel
// (i, j, k): the sum of the weights of those of its corners that are n (same
// per-axis factors, multiplied in the same order as proj_corners).
__device__ __forceinline__ float proj_weight_at(const Grid3 &g, const ProjSpace &S, int i, int j, int k,
                                                const int n[3])
{
    const int nd[3] = {g.nx, g.ny, g.nz};
    float w = 1.0f;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double r = S.A[4 * d] * i + S.A[4 * d + 1] * j + S.A[4 * d + 2] * k + S.A[4 * d + 3];
        if (!(r >= -0.5 && r <= nd[d] - 0.5)) return 0.0f;
        const double f = floor(r);
        const float t = (float)(r - f);
        const int lo = max((int)f, 0), hi = min((int)f + 1, nd[d] - 1);
        const float wd = (lo == n[d] ? 1.0f - t : 0.0f) + (hi == n[d] ? t : 0.0f);
        if (wd == 0.0f) return 0.0f;
        w = d == 0 ? wd : w * wd;
    }
    return w;
}

__global__ __launch_bounds__(BLOCK) void k_proj_push(Grid3 g, ProjPushArgs A, float4 *__restrict__ G, HessArrays H)
{
    const Col c = locate_col(g);
    if (!c.act) return;
    const int64_t n = c.base + (int64_t)c.z0 * c.sxy;
    const int nv[3] = {c.x, c.y, c.z0};
    const int nd[3] = {g.nx, g.ny, g.nz};
    float gs[4] = {0.f, 0.f, 0.f, 0.f}, Hs[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    // interpolation support of n on each axis, within the field of view
    double lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        lo[d] = fmax(nv[d] - 1.0, -0.5);
        hi[d] = fmin(nv[d] + 1.0, nd[d] - 0.5);
    }
    for (int ci = 0; ci < A.C; ci++) {
        const ProjSpace &S = A.S[ci];
        const int md[3] = {S.mx, S.my, S.mz};
        // acquisition-index bounding box of the inverse image of the support
        double amin[3] = {1e300, 1e300, 1e300}, amax[3] = {-1e300, -1e300, -1e300};
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const double p[3] = {q & 1 ? hi[0] : lo[0], q & 2 ? hi[1] : lo[1], q & 4 ? hi[2] : lo[2]};
#pragma unroll
            for (int d = 0; d < 3; d++) {
                const double a = S.Ainv[4 * d] * p[0] + S.Ainv[4 * d + 1] * p[1] + S.Ainv[4 * d + 2] * p[2] +
                                 S.Ainv[4 * d + 3];
                amin[d] = fmin(amin[d], a);
                amax[d] = fmax(amax[d], a);
            }
        }
        int b0[3], b1[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            b0[d] = (int)fmax(floor(amin[d]), 0.0);
            b1[d] = (int)fmin(ceil(amax[d]), md[d] - 1.0);
        }
        const ProjBlocks &B = A.B[ci];
        for (int kk = b0[2]; kk <= b1[2]; kk++)
            for (int jj = b0[1]; jj <= b1[1]; jj++)
                for (int ii = b0[0]; ii <= b1[0]; ii++) {
                    const float w = proj_weight_at(g, S, ii, jj, kk, nv);
                    if (w == 0.0f) continue;
                    const int64_t m = (int64_t)ii + (int64_t)S.mx * (jj + (int64_t)S.my * kk);
                    float gm[4], Hm[10];
                    vload(B.G, m, gm);
                    load_H(B.H, m, Hm);
#pragma unroll
                    for (int a = 0; a < 4; a++) gs[a] += w * gm[a];
#pragma unroll
                    for (int e = 0; e < 10; e++) Hs[e] += w * Hm[e];
                }
    }
    vstore_nt(G, n, gs);
    store_H(H, n, Hs);
}

__global__ __launch_bounds__(BLOCK) void k_proj_pull(Grid3 g, ProjSpace S, const float *__restrict__ Y,
                                                     const float *__restrict__ b1, float *__restrict__ Yp,
                                                     float *__restrict__ bp)
{
    const int64_t m = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (m >= S.M) return;
    int i, j, k;
    acq_index(S, m, i, j, k);
    Corners cr;
    float y[4] = {NAN, NAN, NAN, NAN}, b = NAN;
    if (proj_corners(g, S, i, j, k, cr)) pull_y_b1(g, cr, Y, b1, y, b);
#pragma unroll
    for (int a = 0; a < 4; a++) Yp[a * S.M + m] = y[a];
    bp[m] = b;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int proj_blocks(int64_t M) { return (int)((M + BLOCK - 1) / BLOCK); }

template <typename T, int CM1, int EM>
static hipError_t lik_one(hipStream_t s, const MapArgs &m, const ProjContrast &pc, double *ext, int gated, bool plus)
{
    const T *X = (const T *)pc.X;
    const auto P = ProtoArg<T, CM1, EM>::make(pc.P, X, pc.S.M);
    dim3 grid(proj_blocks(pc.S.M)), blk(BLOCK);
    if (plus)
        hipLaunchKernelGGL((k_proj_lik<T, CM1, EM, true>), grid, blk, 0, s, m.g, pc.S, P, X, m.Y, m.b1, m.loading,
                           pc.B, m.ctl, gated, ext + pc.ext_col);
    else
        hipLaunchKernelGGL((k_proj_lik<T, CM1, EM, false>), grid, blk, 0, s, m.g, pc.S, P, X, m.Y, m.b1, m.loading,
                           pc.B, m.ctl, gated, ext + pc.ext_col);
    return hipGetLastError();
}

template <typename T, int CM1, int EM>
static hipError_t nll_one(hipStream_t s, const MapArgs &m, const ProjContrast &pc, double *ext, int stride, int h0,
                          int h1)
{
    const T *X = (const T *)pc.X;
    const auto P = ProtoArg<T, CM1, EM>::make(pc.P, X, pc.S.M);
    hipLaunchKernelGGL((k_proj_nll<T, CM1, EM>), dim3(proj_blocks(pc.S.M)), dim3(BLOCK), 0, s, m.g, pc.S, P, X, m.Y,
                       m.b1, m.D, m.P0, m.P1, h0, h1, m.ctl, ext + pc.ext_col, stride);
    return hipGetLastError();
}

// echo storage x echo count of the contrast (registers for <= 8 or <= 16)
#define PROJ_DISPATCH(FN, ...)                                                                            \
    do {                                                                                                  \
        const int ne = pc.P.first[1] - pc.P.first[0];                                                     \
        if (m.dtype == DT_F32)                                                                            \
            return ne <= 8 ? FN<float, 1, 8>(__VA_ARGS__)                                                 \
                           : ne <= 16 ? FN<float, 1, 16>(__VA_ARGS__) : FN<float, 0, 0>(__VA_ARGS__);     \
        if (m.dtype == DT_F16)                                                                            \
            return ne <= 8 ? FN<F16, 1, 8>(__VA_ARGS__)                                                   \
                           : ne <= 16 ? FN<F16, 1, 16>(__VA_ARGS__) : FN<F16, 0, 0>(__VA_ARGS__);         \
        return ne <= 8 ? FN<BF16, 1, 8>(__VA_ARGS__)                                                      \
                       : ne <= 16 ? FN<BF16, 1, 16>(__VA_ARGS__) : FN<BF16, 0, 0>(__VA_ARGS__);           \
    } while (0)

hipError_t launch_proj_lik(hipStream_t s, const MapArgs &m, const ProjContrast &pc, double *ext, int gated)
{
    PROJ_DISPATCH(lik_one, s, m, pc, ext, gated, m.loading == 2);
}

hipError_t launch_proj_nll(hipStream_t s, const MapArgs &m, const ProjContrast &pc, double *ext, int ext_stride,
                           int h0, int h1)
{
    PROJ_DISPATCH(nll_one, s, m, pc, ext, ext_stride, h0, h1);
}

hipError_t launch_proj_push(hipStream_t s, const MapArgs &m, const ProjPushArgs &pa, float4 *G, HessArrays H)
{
    hipLaunchKernelGGL(k_proj_push, dim3((unsigned)grid_blocks(m.gp)), dim3(BLOCK), 0, s, m.gp, pa, G, H);
    return hipGetLastError();
}

hipError_t launch_proj_pull(hipStream_t s, const Grid3 &g, const ProjSpace &S, const float *Y, const float *b1,
                            float *Yp, float *bp)
{
    hipLaunchKernelGGL(k_proj_pull, dim3(proj_blocks(S.M)), dim3(BLOCK), 0, s, g, S, Y, b1, Yp, bp);
    return hipGetLastError();
}

}  // namespace mpm
