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
//   k_psi_*      the same enumeration stored once as a sparse Psi^T, and
//   k_proj_push_csr  the push through it (what a fit runs every step);
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

// Pulled trial maps (float4 per reconstruction voxel) and b1 at the corners cr.
__device__ __forceinline__ void pull_yt_b1(const Grid3 &g, const Corners &cr, const float4 *__restrict__ Yt,
                                           const float *__restrict__ b1, float y[4], float &b)
{
#pragma unroll
    for (int a = 0; a < 4; a++) y[a] = 0.0f;
    b = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; c++) {
        const float4 v = Yt[cr.idx[c]];
        y[0] += cr.w[c] * v.x;
        y[1] += cr.w[c] * v.y;
        y[2] += cr.w[c] * v.z;
        y[3] += cr.w[c] * v.w;
        b += cr.w[c] * (b1 ? b1[cr.idx[c]] : 1.0f);
    }
}

// Trial point y - delta_f of the current Newton step, one float4 per voxel,
// for the trial likelihood's pull.
__global__ __launch_bounds__(BLOCK) void k_trial_point(int64_t N, const float *__restrict__ Y,
                                                      const float4 *__restrict__ D, const float4 *__restrict__ P0,
                                                      const float4 *__restrict__ P1, const MapCtl *__restrict__ ctl,
                                                      float4 *__restrict__ Yt)
{
    if (ctl->gn_stop) return;
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= N) return;
    const DeltaF getd{D, ctl->p_buf ? P1 : P0, (float)ctl->alpha_pend, ctl->delta_valid != 0};
    float d[4];
    getd(n, d);
    Yt[n] = make_float4(Y[n] - d[0], Y[N + n] - d[1], Y[2 * N + n] - d[2], Y[3 * N + n] - d[3]);
}

// Acquisition-space kernels walk columns of their own grid ga (a 64 x 4 tile
// of the x-y plane, a run of planes along z; workgroups XCD-contiguous), so
// the reconstruction voxels that consecutive planes pull from stay in cache.
//
// k_proj_lik evaluates the blocks at the current maps (TRIAL = false) or at
// the trial point y - delta_f of the current Newton step (TRIAL = true: its
// NLL decides the acceptance, and when the full step is taken its blocks are
// those of the next step).  gated (current maps, at the start of a step): skip
// when the step is skipped, or when the previous step took its full step, so
// that the blocks from its trial point are current.
template <typename T, int CM1, int EM, bool PLUS, bool TRIAL>
__global__ __launch_bounds__(BLOCK) void k_proj_lik(Grid3 g, Grid3 ga, ProjSpace S,
                                                    typename VoxelEchoes<T, CM1, EM>::Proto P,
                                                    const T *__restrict__ X, const float *__restrict__ Y,
                                                    const float *__restrict__ b1, int loading, ProjBlocks B,
                                                    const MapCtl *__restrict__ ctl, int gated,
                                                    double *__restrict__ ext, const float4 *__restrict__ Yt)
{
    if (TRIAL ? ctl->gn_stop != 0 : gated && (ctl->gn_stop || ctl->step == 1.0)) return;
    const auto K = VoxelEchoes<T, CM1, EM>::stage(P);
    const Col c = locate_col(ga);
    double part[1] = {0.0};
    if (c.act) {
        for (int k = c.z0; k < c.z1; k++) {
            const int64_t m = c.base + (int64_t)k * c.sxy;
            float gl[4] = {0.f, 0.f, 0.f, 0.f}, H[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            Corners cr;
            if (proj_corners(g, S, c.x, c.y, k, cr)) {
                float y[4], b;
                if (TRIAL)
                    pull_yt_b1(g, cr, Yt, b1, y, b);
                else
                    pull_y_b1(g, cr, Y, b1, y, b);
                VoxelEchoes<T, CM1, EM> ve;
                ve.load(P, X, S.M, m, b);
                part[0] += ve.template lik<PLUS>(P, K, y, loading, true, gl, H);
            }
            vstore_nt(B.G, m, gl);
            store_H(B.H, m, H);
        }
    }
    write_rows<1>(part, ext, 0);
}

template <typename T, int CM1, int EM>
__global__ __launch_bounds__(BLOCK) void k_proj_nll(Grid3 g, Grid3 ga, ProjSpace S,
                                                    typename VoxelEchoes<T, CM1, EM>::Proto P,
                                                    const T *__restrict__ X, const float *__restrict__ Y,
                                                    const float *__restrict__ b1, const float4 *__restrict__ D,
                                                    const float4 *__restrict__ P0, const float4 *__restrict__ P1,
                                                    int h0, int h1, const MapCtl *__restrict__ ctl,
                                                    double *__restrict__ ext, int ext_stride)
{
    if (ctl->gn_stop || (h0 > 0 && !ctl->accept_more)) return;
    const DeltaF getd{D, ctl->p_buf ? P1 : P0, (float)ctl->alpha_pend, ctl->delta_valid != 0};
    const auto K = VoxelEchoes<T, CM1, EM>::stage(P);
    const Col c = locate_col(ga);
    double part[MAX_TRIALS];
#pragma unroll
    for (int h = 0; h < MAX_TRIALS; h++) part[h] = 0.0;
    if (c.act) {
        for (int k = c.z0; k < c.z1; k++) {
            const int64_t m = c.base + (int64_t)k * c.sxy;
            Corners cr;
            if (!proj_corners(g, S, c.x, c.y, k, cr)) continue;
            float y[4], b, dl[4] = {0.f, 0.f, 0.f, 0.f};
            pull_y_b1(g, cr, Y, b1, y, b);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                float dv[4];
                getd(cr.idx[q], dv);
#pragma unroll
                for (int a = 0; a < 4; a++) dl[a] += cr.w[q] * dv[a];
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
                    if (q == h) part[q] += v;
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

// Acquisition-index bounding box [b0, b1] (clamped to the space) of the
// inverse image of the box [lo, hi] of reconstruction coordinates.
__device__ __forceinline__ void preimage_box(const ProjSpace &S, const double lo[3], const double hi[3], int b0[3],
                                             int b1[3])
{
    const int md[3] = {S.mx, S.my, S.mz};
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
#pragma unroll
    for (int d = 0; d < 3; d++) {
        b0[d] = (int)fmax(floor(amin[d]), 0.0);
        b1[d] = (int)fmin(ceil(amax[d]), md[d] - 1.0);
    }
}

// The acquisition voxels m of space S whose pull weight at reconstruction
// voxel nv is nonzero, with that weight, in a fixed order: visit(m, w).
// Candidates are the rows (jj, kk) of the preimage box of nv's interpolation
// support in ascending order and, along each row, the i for which every
// coordinate of A (i, jj, kk) lies in the support (an interval per axis with
// A[d][0] != 0; a superset after floor/ceil, the weight test decides).
template <class Visit>
__device__ __forceinline__ void push_visit(const Grid3 &g, const ProjSpace &S, const int nv[3], Visit visit)
{
    const int nd[3] = {g.nx, g.ny, g.nz};
    double lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        lo[d] = fmax(nv[d] - 1.0, -0.5);
        hi[d] = fmin(nv[d] + 1.0, nd[d] - 0.5);
    }
    int b0[3], b1[3];
    preimage_box(S, lo, hi, b0, b1);
    for (int kk = b0[2]; kk <= b1[2]; kk++)
        for (int jj = b0[1]; jj <= b1[1]; jj++) {
            double ilo = b0[0], ihi = b1[0];
#pragma unroll
            for (int d = 0; d < 3; d++) {
                if (S.rA0[d] == 0.0) continue;
                const double c0 = S.A[4 * d + 1] * jj + S.A[4 * d + 2] * kk + S.A[4 * d + 3];
                const double p = (lo[d] - c0) * S.rA0[d], q = (hi[d] - c0) * S.rA0[d];
                ilo = fmax(ilo, fmin(p, q));
                ihi = fmin(ihi, fmax(p, q));
            }
            // ilo >= b0[0] and ihi <= b1[0] already; clamp the far ends before
            // the conversion so it stays in range
            const int i0 = (int)floor(fmin(ilo, b1[0] + 1.0)), i1 = (int)ceil(fmax(ihi, b0[0] - 1.0));
            for (int ii = i0; ii <= min(i1, b1[0]); ii++) {
                const float w = proj_weight_at(g, S, ii, jj, kk, nv);
                if (w != 0.0f) visit((int64_t)ii + (int64_t)S.mx * (jj + (int64_t)S.my * kk), w);
            }
        }
}

__device__ __forceinline__ void recon_index(const Grid3 &g, int64_t n, int nv[3])
{
    nv[0] = (int)(n % g.nx);
    nv[1] = (int)((n / g.nx) % g.ny);
    nv[2] = (int)(n / ((int64_t)g.nx * g.ny));
}

__device__ __forceinline__ void push_add(float w, const float gm[4], const float Hm[10], float gs[4], float Hs[10])
{
#pragma unroll
    for (int a = 0; a < 4; a++) gs[a] += w * gm[a];
#pragma unroll
    for (int e = 0; e < 10; e++) Hs[e] += w * Hm[e];
}

// Direct push: each reconstruction voxel enumerates its candidates (used
// where the blocks are pushed once, e.g. for the variance).
__global__ __launch_bounds__(BLOCK) void k_proj_push(Grid3 g, ProjPushArgs A, float4 *__restrict__ G, HessArrays H)
{
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= g.N) return;
    int nv[3];
    recon_index(g, n, nv);
    float gs[4] = {0.f, 0.f, 0.f, 0.f}, Hs[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int ci = 0; ci < A.C; ci++) {
        const ProjBlocks &B = A.B[ci];
        push_visit(g, A.S[ci], nv, [&](int64_t m, float w) {
            float gm[4], Hm[10];
            vload(B.G, m, gm);
            load_H_cached(B.H, m, Hm);
            push_add(w, gm, Hm, gs, Hs);
        });
    }
    vstore_nt(G, n, gs);
    store_H(H, n, Hs);
}

// Psi^T as a sparse matrix, built once per fit (the spaces do not change):
// row ci * N + n holds the (m, w) pairs of contrast ci at voxel n in the
// enumeration order, so a push through it sums in the same order as the
// direct push.  Counts first (into row[1 + r]), an in-place inclusive scan,
// then the fill.
__global__ __launch_bounds__(BLOCK) void k_psi_count(Grid3 g, ProjPushArgs A, int64_t *__restrict__ row)
{
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= g.N) return;
    int nv[3];
    recon_index(g, n, nv);
    if (n == 0) row[0] = 0;
    for (int ci = 0; ci < A.C; ci++) {
        int64_t cnt = 0;
        push_visit(g, A.S[ci], nv, [&](int64_t, float) { cnt++; });
        row[1 + ci * g.N + n] = cnt;
    }
}

__global__ __launch_bounds__(BLOCK) void k_psi_fill(Grid3 g, ProjPushArgs A, const int64_t *__restrict__ row,
                                                   int2 *__restrict__ ent)
{
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= g.N) return;
    int nv[3];
    recon_index(g, n, nv);
    for (int ci = 0; ci < A.C; ci++) {
        int64_t p = row[ci * g.N + n];
        const int64_t end = row[ci * g.N + n + 1];
        push_visit(g, A.S[ci], nv, [&](int64_t m, float w) {
            if (p < end) ent[p] = make_int2((int)m, __float_as_int(w));
            p++;
        });
    }
}

// In-place inclusive scan of v[0, n): chunk sums, an exclusive scan of the
// chunk sums by one workgroup, then each chunk rescanned with its offset.
constexpr int SCAN_PER_THREAD = 16;
constexpr int SCAN_CHUNK = BLOCK * SCAN_PER_THREAD;

__device__ __forceinline__ int64_t block_excl_scan(int64_t x, int64_t *total)
{
    __shared__ int64_t sh[BLOCK];
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < BLOCK; off <<= 1) {
        const int64_t t = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    const int64_t incl = sh[threadIdx.x];
    *total = sh[BLOCK - 1];
    __syncthreads();
    return incl - x;
}

__global__ __launch_bounds__(BLOCK) void k_scan_sums(const int64_t *__restrict__ v, int64_t n, int64_t *__restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    int64_t s = 0;
    for (int k = 0; k < SCAN_PER_THREAD; k++)
        if (base + k < n) s += v[base + k];
    int64_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(BLOCK) void k_scan_top(int64_t *__restrict__ sums, int64_t nb)
{
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += BLOCK) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t x = b < nb ? sums[b] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(x, &tot);
        if (b < nb) sums[b] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(BLOCK) void k_scan_apply(int64_t *__restrict__ v, int64_t n,
                                                      const int64_t *__restrict__ offs)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    int64_t loc[SCAN_PER_THREAD];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; k++) {
        loc[k] = base + k < n ? v[base + k] : 0;
        s += loc[k];
    }
    int64_t tot;
    int64_t run = offs[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; k++) {
        run += loc[k];
        if (base + k < n) v[base + k] = run;
    }
}

// Push through the stored Psi^T: columns of the reconstruction grid (64 x 4
// tiles, XCD-contiguous; measured faster than 8 x 8 x 4 bricks); per contrast,
// entries in chunks of four (their blocks loaded together, then added in row
// order).
constexpr int PUSH_CHUNK = 8;  // entries whose blocks are loaded together (4: 1.60 ms, 8: 1.46, 12: 1.67 per whole-brain push)

__global__ __launch_bounds__(BLOCK) void k_proj_push_csr(Grid3 g, ProjPushArgs A, const int64_t *__restrict__ row,
                                                        const int2 *__restrict__ ent, float4 *__restrict__ G,
                                                        HessArrays H)
{
    const Col c = locate_col(g);
    if (!c.act) return;
    for (int z = c.z0; z < c.z1; z++) {
        const int64_t n = c.base + (int64_t)z * c.sxy;
        float gs[4] = {0.f, 0.f, 0.f, 0.f}, Hs[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        // the next contrast's row bounds are loaded while this one is gathered
        int64_t p0 = row[n], p1 = row[n + 1];
        for (int ci = 0; ci < A.C; ci++) {
            const ProjBlocks &B = A.B[ci];
            int64_t q0 = 0, q1 = 0;
            if (ci + 1 < A.C) {
                q0 = row[(ci + 1) * g.N + n];
                q1 = row[(ci + 1) * g.N + n + 1];
            }
            for (int64_t p = p0; p < p1; p += PUSH_CHUNK) {
                int2 e[PUSH_CHUNK];
#pragma unroll
                for (int q = 0; q < PUSH_CHUNK; q++) e[q] = ent[p + q < p1 ? p + q : p0];
                float gm[PUSH_CHUNK][4], Hm[PUSH_CHUNK][10];
#pragma unroll
                for (int q = 0; q < PUSH_CHUNK; q++) {
                    vload(B.G, e[q].x, gm[q]);
                    load_H_cached(B.H, e[q].x, Hm[q]);
                }
#pragma unroll
                for (int q = 0; q < PUSH_CHUNK; q++)
                    if (p + q < p1) push_add(__int_as_float(e[q].y), gm[q], Hm[q], gs, Hs);
            }
            p0 = q0;
            p1 = q1;
        }
        vstore_nt(G, n, gs);
        store_H(H, n, Hs);
    }
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
int proj_blocks(const ProjSpace &S) { return grid_blocks(proj_grid(S)); }

template <typename T, int CM1, int EM>
static hipError_t lik_one(hipStream_t s, const MapArgs &m, const ProjContrast &pc, double *ext, int gated, bool plus,
                          const float4 *Yt)
{
    const T *X = (const T *)pc.X;
    const auto P = ProtoArg<T, CM1, EM>::make(pc.P, X, pc.S.M);
    const Grid3 ga = proj_grid(pc.S);
    dim3 grid(grid_blocks(ga)), blk(BLOCK);
#define PROJ_LIK(PL, TR)                                                                                       \
    hipLaunchKernelGGL((k_proj_lik<T, CM1, EM, PL, TR>), grid, blk, 0, s, m.g, ga, pc.S, P, X, m.Y, m.b1,     \
                       m.loading, pc.B, m.ctl, gated, ext + pc.ext_col, Yt)
    if (plus) {
        if (Yt)
            PROJ_LIK(true, true);
        else
            PROJ_LIK(true, false);
    } else {
        if (Yt)
            PROJ_LIK(false, true);
        else
            PROJ_LIK(false, false);
    }
#undef PROJ_LIK
    return hipGetLastError();
}

template <typename T, int CM1, int EM>
static hipError_t nll_one(hipStream_t s, const MapArgs &m, const ProjContrast &pc, double *ext, int stride, int h0,
                          int h1)
{
    const T *X = (const T *)pc.X;
    const auto P = ProtoArg<T, CM1, EM>::make(pc.P, X, pc.S.M);
    const Grid3 ga = proj_grid(pc.S);
    hipLaunchKernelGGL((k_proj_nll<T, CM1, EM>), dim3(grid_blocks(ga)), dim3(BLOCK), 0, s, m.g, ga, pc.S, P, X,
                       m.Y, m.b1, m.D, m.P0, m.P1, h0, h1, m.ctl, ext + pc.ext_col, stride);
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

hipError_t launch_proj_lik(hipStream_t s, const MapArgs &m, const ProjContrast &pc, double *ext, int gated,
                           const float4 *Yt)
{
    PROJ_DISPATCH(lik_one, s, m, pc, ext, gated, m.loading == 2, Yt);
}

hipError_t launch_trial_point(hipStream_t s, const MapArgs &m, float4 *Yt)
{
    hipLaunchKernelGGL(k_trial_point, dim3((unsigned)((m.g.N + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, m.g.N, m.Y,
                       m.D, m.P0, m.P1, m.ctl, Yt);
    return hipGetLastError();
}

hipError_t launch_proj_nll(hipStream_t s, const MapArgs &m, const ProjContrast &pc, double *ext, int ext_stride,
                           int h0, int h1)
{
    PROJ_DISPATCH(nll_one, s, m, pc, ext, ext_stride, h0, h1);
}

static unsigned voxel_blocks(int64_t N) { return (unsigned)((N + BLOCK - 1) / BLOCK); }

hipError_t launch_proj_push(hipStream_t s, const MapArgs &m, const ProjPushArgs &pa, float4 *G, HessArrays H)
{
    hipLaunchKernelGGL(k_proj_push, dim3(voxel_blocks(m.g.N)), dim3(BLOCK), 0, s, m.g, pa, G, H);
    return hipGetLastError();
}

int64_t psi_scan_blocks(int64_t rows) { return (rows + SCAN_CHUNK - 1) / SCAN_CHUNK; }

hipError_t launch_psi_build(hipStream_t s, const Grid3 &g, const ProjPushArgs &pa, const PsiT &psi, int64_t *scan_tmp)
{
    const int64_t rows = (int64_t)pa.C * g.N;
    const unsigned nb = (unsigned)psi_scan_blocks(rows);
    hipLaunchKernelGGL(k_psi_count, dim3(voxel_blocks(g.N)), dim3(BLOCK), 0, s, g, pa, psi.row);
    hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(BLOCK), 0, s, psi.row + 1, rows, scan_tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BLOCK), 0, s, scan_tmp, (int64_t)nb);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(BLOCK), 0, s, psi.row + 1, rows, scan_tmp);
    hipLaunchKernelGGL(k_psi_fill, dim3(voxel_blocks(g.N)), dim3(BLOCK), 0, s, g, pa, psi.row, psi.ent);
    return hipGetLastError();
}

hipError_t launch_proj_push_csr(hipStream_t s, const MapArgs &m, const ProjPushArgs &pa, const PsiT &psi, float4 *G,
                                HessArrays H)
{
    hipLaunchKernelGGL(k_proj_push_csr, dim3((unsigned)grid_blocks(m.g)), dim3(BLOCK), 0, s, m.g, pa, psi.row,
                       psi.ent, G, H);
    return hipGetLastError();
}

hipError_t launch_proj_pull(hipStream_t s, const Grid3 &g, const ProjSpace &S, const float *Y, const float *b1,
                            float *Yp, float *bp)
{
    hipLaunchKernelGGL(k_proj_pull, dim3(voxel_blocks(S.M)), dim3(BLOCK), 0, s, g, S, Y, b1, Yp, bp);
    return hipGetLastError();
}

}  // namespace mpm
