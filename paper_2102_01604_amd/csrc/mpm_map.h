// mpm_map.h -- shared declarations of the MAP (JTV) kernels and their host driver.
#pragma once

#include <hip/hip_runtime.h>

#include "mpm_kernels.h"

namespace mpm {

constexpr int TILE_X = 64;   // voxels along x per workgroup (one wavefront)
constexpr int TILE_Y = 4;    // rows along y per workgroup (256 threads)
constexpr int MAX_TRIALS = 8;  // step sizes 1, 1/2, ..., 1/128 of the acceptance test
// A step is accepted when F_w rises by at most ACCEPT_REL |F_w|: the objective
// is a sum of single-precision voxel terms, whose rounding makes differences
// below about 1e-11 |F_w| (larger for small volumes) indistinguishable from 0.
constexpr double ACCEPT_REL = 1e-9;
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
    double gam[2];      // r.z of CG iteration k in slot k & 1 (the sweeps' own finalising)
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
    // early stopping on the gain of a step (Newton) or an outer loop
    double F_loop0;     // F_w before the first Newton step of this outer loop
    double obj_first, obj_prev;  // objective at the end of the first / previous outer loop
    int n_obj;          // outer loops ended so far
    int outer_done;     // outer loops run
    int outer_stop;     // the remaining outer loops are skipped
    int tol_stop;       // the accepted step ends this outer loop (set after its update)
    int spec_ready;     // the accept pass evaluated the next likelihood pass at the taken full step
};

// ---------------------------------------------------------------------------
// Column walk.  A workgroup owns a TILE_X x TILE_Y tile of the x-y plane and
// the planes [z0, z1); each thread walks its own (x, y) column.  The values
// at z - 1, z, z + 1 of the thread's own column rotate through registers; the
// four in-plane neighbours are loaded (they are L2-resident: adjacent tiles of
// the same z-run are processed by the same XCD at the same time).
// ---------------------------------------------------------------------------
struct Col {
    int x, y, z0, z1;
    bool act;
    bool xm, xp, ym, yp;  // in-plane neighbours inside the grid
    int64_t base;         // voxel index of (x, y, 0)
    int64_t sxy;          // plane stride
};

// L: the workgroup's index among the T workgroups that walk grid g (its
// blockIdx.x and gridDim.x, unless one launch serves several volumes).
__device__ __forceinline__ Col locate_col(const Grid3 &g, int L, int T)
{
    const int q = T >> 3, r = T & 7, j = L & 7;
    const int lid = j * q + min(j, r) + (L >> 3);  // XCD-contiguous workgroup index
    const int bx = lid % g.gx;
    const int t2 = lid / g.gx;
    const int by = t2 % g.gy;
    const int bz = t2 / g.gy;
    Col c;
    c.x = bx * TILE_X + (threadIdx.x & (TILE_X - 1));
    c.y = by * g.ty + (threadIdx.x / TILE_X);
    c.z0 = bz * g.zc;
    c.z1 = min(c.z0 + g.zc, g.nz);
    c.act = c.x < g.nx && c.y < g.ny;
    c.xm = c.x > 0;
    c.xp = c.x < g.nx - 1;
    c.ym = c.y > 0;
    c.yp = c.y < g.ny - 1;
    c.sxy = (int64_t)g.nx * g.ny;
    c.base = c.act ? (int64_t)c.x + (int64_t)g.nx * c.y : 0;
    return c;
}

__device__ __forceinline__ Col locate_col(const Grid3 &g) { return locate_col(g, blockIdx.x, gridDim.x); }

template <class Visit>
__device__ __forceinline__ void for_inplane(const Col &c, int64_t n, int nx, Visit visit)
{
    if (c.xm) visit(n - 1);
    if (c.xp) visit(n + 1);
    if (c.ym) visit(n - nx);
    if (c.yp) visit(n + nx);
}

// ---------------------------------------------------------------------------
// device helpers shared by the MAP kernels
// ---------------------------------------------------------------------------
// Block sums of v written to partials[k * T + L] (workgroup L of T).
template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], double *__restrict__ partials, int L, int T)
{
    __shared__ double lds[NV][NWAVE];
    block_sum<NV>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) partials[(int64_t)k * T + L] = v[k];
    }
}

template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], double *__restrict__ partials)
{
    write_partials<NV>(v, partials, blockIdx.x, gridDim.x);
}

// Non-temporal access for arrays that a kernel streams exactly once (no
// stencil reuse), so they do not evict the stencil operands' halos from L2.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void vload_nt(const float4 *__restrict__ a, int64_t n, float v[4])
{
    const v4f t = __builtin_nontemporal_load((const v4f *)(a + n));
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
    v[3] = t.w;
}

__device__ __forceinline__ void vstore_nt(float4 *__restrict__ a, int64_t n, const float v[4])
{
    const v4f t = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(t, (v4f *)(a + n));
}

__device__ __forceinline__ void vload(const float4 *__restrict__ a, int64_t n, float v[4])
{
    const float4 t = a[n];
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
    v[3] = t.w;
}

__device__ __forceinline__ void vstore(float4 *__restrict__ a, int64_t n, const float v[4])
{
    a[n] = make_float4(v[0], v[1], v[2], v[3]);
}

// packed symmetric index: 0:00 1:01 2:02 3:03 4:11 5:12 6:13 7:22 8:23 9:33;
// stored as d = (00, 11, 22, 33), o = (01, 02, 03, 12), r = (13, 23)
__device__ __forceinline__ void unpack_H(const v4f d, const v4f o, const v2f r, float H[10])
{
    H[0] = d.x;
    H[4] = d.y;
    H[7] = d.z;
    H[9] = d.w;
    H[1] = o.x;
    H[2] = o.y;
    H[3] = o.z;
    H[5] = o.w;
    H[6] = r.x;
    H[8] = r.y;
}

__device__ __forceinline__ void load_H(const HessArrays &h, int64_t n, float H[10])
{
    unpack_H(__builtin_nontemporal_load((const v4f *)(h.d + n)), __builtin_nontemporal_load((const v4f *)(h.o + n)),
             __builtin_nontemporal_load((const v2f *)(h.r + n)), H);
}

// Cached load, for blocks that several threads gather (the projection's push).
__device__ __forceinline__ void load_H_cached(const HessArrays &h, int64_t n, float H[10])
{
    const float4 d = h.d[n], o = h.o[n];
    const float2 r = h.r[n];
    unpack_H(v4f{d.x, d.y, d.z, d.w}, v4f{o.x, o.y, o.z, o.w}, v2f{r.x, r.y}, H);
}

__device__ __forceinline__ void store_H(const HessArrays &h, int64_t n, const float H[10])
{
    const v4f d = {H[0], H[4], H[7], H[9]};
    const v4f o = {H[1], H[2], H[3], H[5]};
    const v2f r = {H[6], H[8]};
    __builtin_nontemporal_store(d, (v4f *)(h.d + n));
    __builtin_nontemporal_store(o, (v4f *)(h.o + n));
    __builtin_nontemporal_store(r, (v2f *)(h.r + n));
}

// delta_f = delta + alpha_pend p_last at voxel m
struct DeltaF {
    const float4 *__restrict__ D;
    const float4 *__restrict__ Pl;
    float alpha;
    bool dvalid;
    __device__ __forceinline__ void operator()(int64_t m, float v[4]) const
    {
        float4 t = dvalid ? D[m] : make_float4(0.f, 0.f, 0.f, 0.f);
        if (alpha != 0.0f) {
            const float4 p = Pl[m];
            t.x += alpha * p.x;
            t.y += alpha * p.y;
            t.z += alpha * p.z;
            t.w += alpha * p.w;
        }
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        v[3] = t.w;
    }
};

enum {
    FIN_LIK = 0, FIN_A = 1, FIN_B = 2, FIN_ACCEPT = 3, FIN_W = 4, FIN_STATS = 5, FIN_ACCEPT2 = 6, FIN_STOP = 7,
    FIN_ACCEPT_SPEC = 8
};

struct MapArgs {
    Grid3 g;
    DevProto P;
    int dtype;
    const void *X;
    const float *b1;
    const float *bm;  // net receive field [N] or NULL
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
    double *partials;   // [MAX_TRIALS + 2][pstride]
    int pstride;        // row stride of partials (the largest workgroup count of any grid)
    int nb_a, nb_b;     // workgroups (partials) of CG sweeps A and B
    // The CG sweeps finalise each other: sweep B reduces sweep A's partials
    // (row 0) and sweep A the previous sweep B's (row 1) itself, in every
    // workgroup and in the finaliser's order, instead of a one-workgroup
    // finaliser launch between them.  Used where the partials are few.
    int fold;
    double cg_stop_rel;
    double *trace;      // device copy of the objective trace
    double tol_gn, tol_outer;  // early-stopping tolerances (0: fixed counts)
};

hipError_t launch_ctl_init(hipStream_t s, MapCtl *ctl, double *trace, int trace_len);
hipError_t launch_lik(hipStream_t s, const MapArgs &a);
hipError_t launch_cg_a(hipStream_t s, const MapArgs &a, int it);
hipError_t launch_cg_b(hipStream_t s, const MapArgs &a, int it);
hipError_t launch_accept(hipStream_t s, const MapArgs &a);
// k_accept that also evaluates the next Newton step's likelihood pass at the
// full step (that step must follow in the same outer loop)
hipError_t launch_accept_spec(hipStream_t s, const MapArgs &a);
hipError_t launch_accept2(hipStream_t s, const MapArgs &a, int ntrial);
hipError_t launch_update(hipStream_t s, const MapArgs &a);
hipError_t launch_weights(hipStream_t s, const MapArgs &a, int prior_on);
hipError_t launch_final(hipStream_t s, const MapArgs &a, float *var, float *mom);
int cg_a_blocks(const MapArgs &a);  // workgroups (partials) of CG sweep A
int cg_b_blocks(const MapArgs &a);  // ... and of sweep B
int cg_b_rows();                    // tile rows of sweep B
int tall_workgroups();
// Extra partial rows added to a finaliser's sums (the acquisition-space NLL
// of a projected fit): row k at p + k * stride, cols columns, rows rows.
struct ExtRows {
    const double *p = nullptr;
    int stride = 0, cols = 0, rows = 0;
};
hipError_t launch_fin(hipStream_t s, const MapArgs &a, int stage, int arg, int nblk, double cg_stop_rel,
                      int ntrial, int accept_off, const ExtRows &ext = ExtRows(), int row = 0);
// Folded CG finalising is used when both sweeps have at most this many
// workgroups: about one round of resident workgroups, so the reduction at the
// start of a sweep adds its latency once (≈2 us) against the ≈5.6 us of a
// finaliser launch saved.  Measured on 64^3 MAP fits (256 partials per sweep):
// 53 vs 61 ms; with 2048 partials (96 x 128 x 128) the reduction in every
// workgroup of four rounds cost more than the launch (271 vs 254 ms), and in
// batched launches, which share one finaliser launch among their volumes, it
// did not pay either (16 x 64^3: 0.56 vs 0.54 s), so batches do not fold.
constexpr int FOLD_MAX_PARTIALS = 512;

// ---------------------------------------------------------------------------
// Batched launches: one launch of a MAP kernel serves several volumes (their
// own grids, buffers, priors and control blocks) that run the same schedule
// in lockstep.  Volume v owns the workgroups [start[k][v], start[k][v] +
// count[k][v]) of a launch over grid kind k; each start is a multiple of 8,
// so a volume's workgroups meet the XCDs exactly as in a launch of its own,
// and each workgroup runs the single-volume kernel body with its index L and
// count T within its volume: every partial sum, and so every result, is the
// one of the volume fitted alone.
// ---------------------------------------------------------------------------
constexpr int MAX_BATCH = 64;
enum BatchKind { BK_PLANE = 0, BK_TALL = 1, BK_CGB = 2, BK_COL = 3, BK_UPD = 4, BK_N = 5, BK_NONE = -1 };

struct BatchTab {
    int n;
    int start[BK_N][MAX_BATCH + 1];  // start[k][n]: workgroups of the whole launch
    int count[BK_N][MAX_BATCH];
};

// Host-side description of one batched fit's device tables.
struct BatchLaunch {
    int n = 0;
    int dtype = 0, shape = 0, loading = 0;
    int total[BK_N] = {};
    const BatchTab *tab = nullptr;  // device
    const void *vols = nullptr;     // device array of per-volume descriptors (batch_desc_bytes each)
};

// Bytes of one per-volume descriptor for echo storage dtype and register
// shape (echo_shape), and writing descriptor v of a host array of them.
size_t batch_desc_bytes(int dtype, int shape);
void fill_batch_desc(void *host, int v, const MapArgs &m, int prior_on, int dtype, int shape);
// Fills the workgroup table of the batch from the volumes' grids.
void fill_batch_tab(BatchTab &t, const MapArgs *m, int n, int total[BK_N]);

hipError_t launch_ctl_init_batch(hipStream_t s, const BatchLaunch &b, int trace_len);
hipError_t launch_lik_batch(hipStream_t s, const BatchLaunch &b);
hipError_t launch_cg_a_batch(hipStream_t s, const BatchLaunch &b, int it);
hipError_t launch_cg_b_batch(hipStream_t s, const BatchLaunch &b, int it);
hipError_t launch_accept_batch(hipStream_t s, const BatchLaunch &b);
hipError_t launch_accept2_batch(hipStream_t s, const BatchLaunch &b, int ntrial);
hipError_t launch_update_batch(hipStream_t s, const BatchLaunch &b);
hipError_t launch_weights_batch(hipStream_t s, const BatchLaunch &b);
hipError_t launch_final_batch(hipStream_t s, const BatchLaunch &b);
// kind: the grid whose per-volume workgroup count is the partial count
// (BK_NONE: no partials)
hipError_t launch_fin_batch(hipStream_t s, const BatchLaunch &b, int stage, int arg, int kind, double cg_stop_rel,
                            int ntrial, int accept_off, double tol_gn, double tol_outer, int row = 0);

}  // namespace mpm
