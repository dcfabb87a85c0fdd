// k_map.hip -- kernels of the JTV-regularised (MAP) fit, paper Sec. 2.5-2.7.
//
// One GN step is: lik (likelihood block + L y + CG start), n_cg x (cg_a, cg_b),
// accept (objective at every trial step), update.  Every kernel reads its
// control scalars from a device-resident MapCtl written by the one-workgroup
// "fin_*" kernels that follow each reduction, so the host never waits inside
// a fit.  Reductions are two-stage and fixed-order (deterministic).
//
// Voxel mapping: the echo kernels (lik, accept, final) give each thread one
// voxel of a 64 x 4 tile of one z-plane; the stencil-only kernels walk z-runs
// of such tiles, and the CG sweeps z-runs of 64 x 16 tiles.  The 1-D workgroup
// index is remapped so that each of the 8 XCDs receives a contiguous run of
// tiles (neighbouring tiles and planes share stencil halos in that XCD's L2).
#include <cstdlib>
#include <cstring>

#include "mpm_proj.h"

namespace mpm {

__device__ __forceinline__ void load4(const float *__restrict__ a, int64_t N, int64_t n, float v[4])
{
#pragma unroll
    for (int k = 0; k < 4; k++) v[k] = a[k * N + n];
}

__device__ __forceinline__ void store4(float *__restrict__ a, int64_t N, int64_t n, const float v[4])
{
#pragma unroll
    for (int k = 0; k < 4; k++) a[k * N + n] = v[k];
}

__device__ __forceinline__ void copy4(float d[4], const float s[4])
{
#pragma unroll
    for (int k = 0; k < 4; k++) d[k] = s[k];
}

// One edge of the L stencil (paper Sec. 2.5): adds (w_n + w_m)(v_n - v_m) to
// acc and (w_n + w_m) to d = diag(G^T W G)_n.
__device__ __forceinline__ void edge(float wn, float wm, const float vn[4], const float vm[4], float acc[4], float &d)
{
    const float f = wn + wm;
    d += f;
#pragma unroll
    for (int k = 0; k < 4; k++) acc[k] += f * (vn[k] - vm[k]);
}

__device__ __forceinline__ double dot4(const float a[4], const float b[4])
{
    return (double)a[0] * b[0] + (double)a[1] * b[1] + (double)a[2] * b[2] + (double)a[3] * b[3];
}

__device__ __forceinline__ void symv4(const float H[10], const float p[4], float q[4])
{
#pragma unroll
    for (int i = 0; i < 4; i++) {
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < 4; j++) s += H[sym(i, j)] * p[j];
        q[i] = s;
    }
}

// z = M^{-1} r with M = H + diag(lam_k d) (block-Jacobi preconditioner of
// paper Sec. 2.6) and the degenerate-voxel rule (z = 0).
__device__ __forceinline__ bool precond(const float H[10], const float lam[4], float d, const float r[4],
                                        float z[4])
{
    float M[10];
#pragma unroll
    for (int k = 0; k < 10; k++) M[k] = H[k];
    M[0] += lam[0] * d;
    M[4] += lam[1] * d;
    M[7] += lam[2] * d;
    M[9] += lam[3] * d;
    return solve_sym4(M, r, z);
}

constexpr int FIN_THREADS = 1024;

// Sum of row[0..ncols) in a fixed order; four independent accumulators per
// thread keep several loads in flight.  The result is valid in every thread.
__device__ __forceinline__ double reduce_row(const double *__restrict__ row, int ncols, double *lds)
{
    const int t = threadIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = t;
    for (; b + 3 * FIN_THREADS < ncols; b += 4 * FIN_THREADS) {
        a0 += row[b];
        a1 += row[b + FIN_THREADS];
        a2 += row[b + 2 * FIN_THREADS];
        a3 += row[b + 3 * FIN_THREADS];
    }
    for (; b < ncols; b += FIN_THREADS) a0 += row[b];
    double v = wave_sum((a0 + a1) + (a2 + a3));
    if ((t & 63) == 0) lds[t >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < FIN_THREADS / 64; i++) r += lds[i];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// control block
// ---------------------------------------------------------------------------
__global__ void k_ctl_init(MapCtl *ctl, double *trace, int trace_len)
{
    int t = threadIdx.x;
    if (t == 0) {
        MapCtl c = {};
        *ctl = c;
    }
    for (int i = t; i < trace_len; i += blockDim.x) trace[i] = __builtin_nan("");
}

// ---------------------------------------------------------------------------
// lik: likelihood block, L y, b = g + L y, and the CG start r = b,
// z = M^{-1} r.  One voxel per thread.  Partials: NLL, y.Ly, r.z
// ---------------------------------------------------------------------------
template <bool PLUS, typename T, int CM, int EM>
__device__ __forceinline__ void lik_body(const Grid3 &g, const typename VoxelEchoes<T, CM, EM>::Proto &P,
                                         const T *__restrict__ X, const float *__restrict__ b1,
                                         const float *__restrict__ bm,
                                         const float *__restrict__ Y, const float *__restrict__ w, float l0, float l1,
                                         float l2, float l3, int loading, const HessArrays &Hs,
                                         float4 *__restrict__ R, float4 *__restrict__ Z,
                                         const MapCtl *__restrict__ ctl, double *__restrict__ partials, int L,
                                         int T_)
{
    // (spec_ready: the previous step's accept pass already computed all of
    // this at the maps now current, see accept_spec_body)
    if (ctl->gn_stop || ctl->spec_ready) return;
    const int64_t N = g.N;
    const float lam[4] = {l0, l1, l2, l3};
    const Col c = locate_col(g, L, T_);
    const auto K = VoxelEchoes<T, CM, EM>::stage(P);
    double part[3] = {0.0, 0.0, 0.0};
    if (c.act) {
        const int64_t n = c.base + (int64_t)c.z0 * c.sxy;
        VoxelEchoes<T, CM, EM> ve;
        ve.load(P, X, N, n, b1 ? b1[n] : 1.0f, bm ? bm[n] : 1.0f);
        float y0[4];
        load4(Y, N, n, y0);
        const float w0 = w[n];
        float acc[4] = {0.f, 0.f, 0.f, 0.f}, d = 0.f;
        const auto nb = [&](int64_t m) {
            float vm[4];
            load4(Y, N, m, vm);
            edge(w0, w[m], y0, vm, acc, d);
        };
        for_inplane(c, n, g.nx, nb);
        if (c.z0 > 0) nb(n - c.sxy);
        if (c.z0 < g.nz - 1) nb(n + c.sxy);
        float gr[4], H[10], r[4], zz[4];
        const float nll = ve.template lik<PLUS>(P, K, y0, loading, true, gr, H);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            acc[k] *= lam[k];  // (L y)_k
            r[k] = gr[k] + acc[k];
        }
        precond(H, lam, d, r, zz);
        store_H(Hs, n, H);
        vstore_nt(R, n, r);
        vstore_nt(Z, n, zz);
        part[0] = nll;
        part[1] = dot4(y0, acc);
        part[2] = dot4(r, zz);
    }
    write_partials<3>(part, partials, L, T_);
}

#define LIK_PARAMS                                                                                           \
    Grid3 g, typename VoxelEchoes<T, CM, EM>::Proto P, const T *__restrict__ X, const float *__restrict__ b1, \
        const float *__restrict__ bm,                                                                        \
        const float *__restrict__ Y, const float *__restrict__ w, float l0, float l1, float l2, float l3,       \
        int loading, HessArrays Hs, float4 *__restrict__ R, float4 *__restrict__ Z,                             \
        const MapCtl *__restrict__ ctl, double *__restrict__ partials
#define LIK_ARGS g, P, X, b1, bm, Y, w, l0, l1, l2, l3, loading, Hs, R, Z, ctl, partials

template <typename T, int CM, int EM>
__global__ __launch_bounds__(BLOCK) void k_lik(LIK_PARAMS)
{
    lik_body<false, T, CM, EM>(LIK_ARGS, blockIdx.x, gridDim.x);
}
template <typename T, int CM, int EM>  // Proposed+ loading
__global__ __launch_bounds__(BLOCK) void k_lik_plus(LIK_PARAMS)
{
    lik_body<true, T, CM, EM>(LIK_ARGS, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// CG sweeps (paper Sec. 2.6, preconditioned CG on (H + L) delta = g + L y).
//   sweep A (iteration it): p = z + beta p_old, q = (H + L) p, partial p.q,
//                           and the deferred update delta += alpha_{it-1} p_old;
//   sweep B (iteration it): q = (H + L) p recomputed, r -= alpha q,
//                           z = M^{-1} r, partial r.z.
// Sweep A: a workgroup of TILE_X x TALL_Y threads owns a TILE_X x TALL_Y tile
// and walks its z-run; each plane of the stencil operand (p and w) is staged in LDS
// (double-buffered, one barrier per plane), so in-plane neighbours inside the
// tile come from LDS and only the tile's rim reads neighbours from memory
// (those reads mostly hit L2: arrays streamed once use non-temporal accesses
// and leave L2 to the stencil operands).
// ---------------------------------------------------------------------------
constexpr int TALL_THREADS = TILE_X * TALL_Y;

struct TallLds {
    float4 p[2][TALL_Y][TILE_X];
    float w[2][TALL_Y][TILE_X];
};

// Neighbours of (tx, ty) at plane buffer `buf`: inside the tile from LDS,
// across the tile rim from memory through get(m, v, wm).
template <class GetMem>
__device__ __forceinline__ void tall_neighbours(const Col &c, const Grid3 &g, int64_t n, int tx, int ty,
                                                const TallLds &L, int buf, float w0, const float p0[4],
                                                GetMem get, float acc[4], float &d)
{
    auto from_lds = [&](int yy, int xx) {
        const float4 v = L.p[buf][yy][xx];
        const float vm[4] = {v.x, v.y, v.z, v.w};
        edge(w0, L.w[buf][yy][xx], p0, vm, acc, d);
    };
    auto from_mem = [&](int64_t m) {
        float vm[4], wm;
        get(m, vm, wm);
        edge(w0, wm, p0, vm, acc, d);
    };
    if (c.xm) {
        if (tx > 0) from_lds(ty, tx - 1);
        else from_mem(n - 1);
    }
    if (c.xp) {
        if (tx < TILE_X - 1) from_lds(ty, tx + 1);
        else from_mem(n + 1);
    }
    if (c.ym) {
        if (ty > 0) from_lds(ty - 1, tx);
        else from_mem(n - g.nx);
    }
    if (c.yp) {
        if (ty < TALL_Y - 1) from_lds(ty + 1, tx);
        else from_mem(n + g.nx);
    }
}

// Folded finalising of the CG sweeps (MapArgs::fold): the partials of the
// previous sweep, their count, and CG's relative stop level.
struct CgFold {
    int on;
    int nblk_prev;
    const double *prev;
    double cg_stop_rel;
};

template <bool FOLD>
__device__ __forceinline__ void cg_a_body(const Grid3 &g, int it, const HessArrays &Hs, const float *__restrict__ w,
                                          float l0, float l1, float l2, float l3, const float4 *__restrict__ Z,
                                          const float4 *__restrict__ Pold, float4 *__restrict__ Pnew,
                                          float4 *__restrict__ D, MapCtl *ctl, double *__restrict__ partials,
                                          const CgFold &fold, int Lb, int Tb)
{
    if (ctl->gn_stop || ctl->cg_stop) return;
    __shared__ TallLds L;
    const float lam[4] = {l0, l1, l2, l3};
    float beta = 0.0f;
    if (FOLD && it > 0) {
        // the finaliser of the previous sweep B, in every workgroup (same
        // fixed order, so every workgroup gets the same value); the first
        // workgroup records it for the kernels after this one
        __shared__ double red[FIN_THREADS / 64];
        const double gn = reduce_row(fold.prev, fold.nblk_prev, red);
        const double gold = ctl->gam[(it - 1) & 1];
        const bool stop = !(gn > fold.cg_stop_rel * ctl->gamma0) || !(gn > 0.0);
        if (Lb == 0 && threadIdx.x == 0) {
            ctl->cg_done++;
            if (stop) ctl->cg_stop = 1;
            ctl->beta = gn / gold;
            ctl->gamma = gn;
            ctl->gam[it & 1] = gn;
        }
        if (stop) return;
        beta = (float)(gn / gold);
    } else if (it > 0) {
        beta = (float)ctl->beta;
    }
    const float alpha_prev = (float)ctl->alpha_pend;
    const Col c = locate_col(g, Lb, Tb);
    const int tx = threadIdx.x & (TILE_X - 1), ty = threadIdx.x / TILE_X;
    auto getp = [&](int64_t m, float p[4], float po[4]) {
        vload(Z, m, p);
        if (it > 0) {
            vload(Pold, m, po);
#pragma unroll
            for (int k = 0; k < 4; k++) p[k] += beta * po[k];
        }
    };
    auto getmem = [&](int64_t m, float p[4], float &wm) {
        float po[4];
        getp(m, p, po);
        wm = w[m];
    };
    double part[1] = {0.0};
    int64_t n = c.base + (int64_t)c.z0 * c.sxy;
    float pm[4] = {0.f, 0.f, 0.f, 0.f}, p0[4] = {0.f, 0.f, 0.f, 0.f}, pp[4] = {0.f, 0.f, 0.f, 0.f};
    float po0[4] = {0.f, 0.f, 0.f, 0.f}, pop[4] = {0.f, 0.f, 0.f, 0.f}, tmp[4];
    float wm = 0.f, w0 = 0.f, wp = 0.f;
    if (c.act) {
        if (c.z0 > 0) {
            getp(n - c.sxy, pm, tmp);
            wm = w[n - c.sxy];
        }
        getp(n, p0, po0);
        w0 = w[n];
    }
    for (int z = c.z0; z < c.z1; z++, n += c.sxy) {
        const int buf = (z - c.z0) & 1;
        const bool hzp = z < g.nz - 1;
        if (c.act && hzp) {
            getp(n + c.sxy, pp, pop);
            wp = w[n + c.sxy];
        }
        L.p[buf][ty][tx] = make_float4(p0[0], p0[1], p0[2], p0[3]);
        L.w[buf][ty][tx] = w0;
        __syncthreads();
        if (c.act) {
            float acc[4] = {0.f, 0.f, 0.f, 0.f}, d = 0.f;
            tall_neighbours(c, g, n, tx, ty, L, buf, w0, p0, getmem, acc, d);
            if (z > 0) edge(w0, wm, p0, pm, acc, d);
            if (hzp) edge(w0, wp, p0, pp, acc, d);
            float H[10], q[4];
            load_H(Hs, n, H);
            symv4(H, p0, q);
#pragma unroll
            for (int k = 0; k < 4; k++) q[k] += lam[k] * acc[k];
            vstore_nt(Pnew, n, p0);
            if (it == 1) {
                float dl[4];
#pragma unroll
                for (int k = 0; k < 4; k++) dl[k] = alpha_prev * po0[k];
                vstore_nt(D, n, dl);
            } else if (it >= 2) {
                float dl[4];
                vload_nt(D, n, dl);
#pragma unroll
                for (int k = 0; k < 4; k++) dl[k] += alpha_prev * po0[k];
                vstore_nt(D, n, dl);
            }
            part[0] += dot4(p0, q);
        }
        copy4(pm, p0);
        copy4(p0, pp);
        copy4(po0, pop);
        wm = w0;
        w0 = wp;
    }
    __shared__ double lds_part[1][TALL_THREADS / 64];
    {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        double s = wave_sum(part[0]);
        if (lane == 0) lds_part[0][wid] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < TALL_THREADS / 64; i++) t += lds_part[0][i];
            partials[Lb] = t;
        }
    }
}

template <bool FOLD>
__global__ __launch_bounds__(TALL_THREADS) void k_cg_a(Grid3 g, int it, HessArrays Hs,
                                                            const float *__restrict__ w, float l0, float l1, float l2,
                                                            float l3, const float4 *__restrict__ Z,
                                                            const float4 *__restrict__ Pold, float4 *__restrict__ Pnew,
                                                            float4 *__restrict__ D, MapCtl *ctl,
                                                            double *__restrict__ partials, CgFold fold)
{
    cg_a_body<FOLD>(g, it, Hs, w, l0, l1, l2, l3, Z, Pold, Pnew, D, ctl, partials, fold, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Sweep B gives each thread one voxel of a TILE_X x CGB_Y tile of one plane and
// reads every neighbour of p through L2 (no LDS, no barriers; the plane grid's
// XCD-contiguous order keeps neighbouring planes in that XCD's L2).  Measured
// on the whole-brain volume this beats the column walk for sweep B (228 vs
// 244 us: many more, shorter workgroups), while sweep A, whose stencil operand
// p = z + beta p_old costs two loads per neighbour, keeps the column walk.
// ---------------------------------------------------------------------------
constexpr int CGB_Y = 16;
constexpr int CGB_THREADS = TILE_X * CGB_Y;
// the folded finalising reduces in the finaliser's own order (reduce_row)
static_assert(TALL_THREADS == FIN_THREADS && CGB_THREADS == FIN_THREADS, "CG sweeps run FIN_THREADS threads");

template <int THREADS>
__device__ __forceinline__ void write_partial1(double v, double *__restrict__ partials, int L)
{
    __shared__ double lds[THREADS / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const double s = wave_sum(v);
    if (lane == 0) lds[wid] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < THREADS / 64; i++) t += lds[i];
        partials[L] = t;
    }
}

template <bool FOLD>
__device__ __forceinline__ void cg_b_body(const Grid3 &g, int it, const HessArrays &Hs, const float *__restrict__ w,
                                          float l0, float l1, float l2, float l3, const float4 *__restrict__ Pc,
                                          float4 *__restrict__ R, float4 *__restrict__ Z, MapCtl *ctl,
                                          double *__restrict__ partials, const CgFold &fold, int L, int T)
{
    if (ctl->gn_stop || ctl->cg_stop) return;
    const float lam[4] = {l0, l1, l2, l3};
    float alpha;
    if (FOLD) {
        // the finaliser of sweep A of this iteration, in every workgroup
        __shared__ double red[FIN_THREADS / 64];
        const double pq = reduce_row(fold.prev, fold.nblk_prev, red);
        const bool stop = !(pq > 0.0);
        const double a = stop ? 0.0 : ctl->gam[it & 1] / pq;
        if (L == 0 && threadIdx.x == 0) {
            if (it >= 1) ctl->delta_valid = 1;
            ctl->p_buf = it & 1;
            ctl->alpha_pend = a;
            if (stop) ctl->cg_stop = 1;
        }
        if (stop) return;
        alpha = (float)a;
    } else {
        alpha = (float)ctl->alpha_pend;
    }
    const Col c = locate_col(g, L, T);
    double part = 0.0;
    if (c.act) {
        const int64_t n = c.base + (int64_t)c.z0 * c.sxy;
        float p0[4];
        vload(Pc, n, p0);
        const float w0 = w[n];
        float acc[4] = {0.f, 0.f, 0.f, 0.f}, d = 0.f;
        const auto nb = [&](int64_t m) {
            float vm[4];
            vload(Pc, m, vm);
            edge(w0, w[m], p0, vm, acc, d);
        };
        for_inplane(c, n, g.nx, nb);
        if (c.z0 > 0) nb(n - c.sxy);
        if (c.z0 < g.nz - 1) nb(n + c.sxy);
        float H[10], q[4], r[4], zz[4];
        load_H(Hs, n, H);
        symv4(H, p0, q);
        vload_nt(R, n, r);
#pragma unroll
        for (int k = 0; k < 4; k++) r[k] -= alpha * (q[k] + lam[k] * acc[k]);
        precond(H, lam, d, r, zz);
        vstore_nt(R, n, r);
        vstore_nt(Z, n, zz);
        part = dot4(r, zz);
    }
    write_partial1<CGB_THREADS>(part, partials, L);
}

template <bool FOLD>
__global__ __launch_bounds__(CGB_THREADS) void k_cg_b(Grid3 g, int it, HessArrays Hs, const float *__restrict__ w,
                                                         float l0, float l1, float l2, float l3,
                                                         const float4 *__restrict__ Pc, float4 *__restrict__ R,
                                                         float4 *__restrict__ Z, MapCtl *ctl,
                                                         double *__restrict__ partials, CgFold fold)
{
    cg_b_body<FOLD>(g, it, Hs, w, l0, l1, l2, l3, Pc, R, Z, ctl, partials, fold, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// accept, pass 1: the NLL at the full step y - delta_f and the prior pieces
// c1 = delta_f.(L y), c2 = delta_f.(L delta_f), so that
// F_w(y - t delta_f) = NLL(y - t delta_f) + (y.Ly - 2 t c1 + t^2 c2) / 2.
// One voxel per thread.  Partials: NLL_0, c1, c2
// ---------------------------------------------------------------------------
#define ACCEPT_PARAMS                                                                                        \
    Grid3 g, typename VoxelEchoes<T, CM, EM>::Proto P, const T *__restrict__ X, const float *__restrict__ b1, \
        const float *__restrict__ bm, const float *__restrict__ Y, const float *__restrict__ w, float l0,       \
        float l1, float l2, float l3, const float4 *__restrict__ D, const float4 *__restrict__ P0,              \
        const float4 *__restrict__ P1, const MapCtl *__restrict__ ctl, double *__restrict__ partials
#define ACCEPT_ARGS g, P, X, b1, bm, Y, w, l0, l1, l2, l3, D, P0, P1, ctl, partials

template <typename T, int CM, int EM>
__device__ __forceinline__ void accept_body(ACCEPT_PARAMS, int L, int T_)
{
    if (ctl->gn_stop) return;
    const int64_t N = g.N;
    const float lam[4] = {l0, l1, l2, l3};
    const DeltaF getd{D, ctl->p_buf ? P1 : P0, (float)ctl->alpha_pend, ctl->delta_valid != 0};
    const Col c = locate_col(g, L, T_);
    const auto K = VoxelEchoes<T, CM, EM>::stage(P);
    double part[3] = {0.0, 0.0, 0.0};
    if (c.act) {
        const int64_t n = c.base + (int64_t)c.z0 * c.sxy;
        VoxelEchoes<T, CM, EM> ve;
        ve.load(P, X, N, n, b1 ? b1[n] : 1.0f, bm ? bm[n] : 1.0f);
        float y0[4], d0[4];
        load4(Y, N, n, y0);
        getd(n, d0);
        const float w0 = w[n];
        float ay[4] = {0.f, 0.f, 0.f, 0.f}, ad[4] = {0.f, 0.f, 0.f, 0.f}, d = 0.f, d2 = 0.f;
        const auto nb = [&](int64_t m) {
            float vm[4], um[4];
            load4(Y, N, m, vm);
            getd(m, um);
            const float wmm = w[m];
            edge(w0, wmm, y0, vm, ay, d);
            edge(w0, wmm, d0, um, ad, d2);
        };
        for_inplane(c, n, g.nx, nb);
        if (c.z0 > 0) nb(n - c.sxy);
        if (c.z0 < g.nz - 1) nb(n + c.sxy);
        float yt[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            ay[k] *= lam[k];
            ad[k] *= lam[k];
            yt[k] = y0[k] - d0[k];
        }
        part[0] = ve.nll(P, K, yt);
        part[1] = dot4(d0, ay);
        part[2] = dot4(d0, ad);
    }
    write_partials<3>(part, partials, L, T_);
}

template <typename T, int CM, int EM>
__global__ __launch_bounds__(BLOCK) void k_accept(ACCEPT_PARAMS)
{
    accept_body<T, CM, EM>(ACCEPT_ARGS, blockIdx.x, gridDim.x);
}

// accept, pass 1, when the next Newton step follows in the same outer loop:
// besides the partials of k_accept it evaluates that step's likelihood pass
// (k_lik) at the full step.  If the full step is taken the maps become
// y - delta_f exactly (the update subtracts 1 * delta_f) and the weights stay,
// so H, r and z written here, and the partial rows 3 (y.Ly) and 4 (r.z) beside
// the NLL in row 0, are what k_lik would compute after the update, bit for bit
// (the same operations in the same order: the neighbours' maps are formed as
// y_m - delta_m like the update forms them, the NLL of the likelihood
// evaluation equals that of the NLL-only one).  The finaliser then marks them
// valid and the next k_lik returns at once.  H, r and z are dead at this point
// of a step (the halved trials and the update read y, delta_f and the echoes).
// Partials: NLL, c1, c2, y.Ly and r.z at the full step.
#define ACCEPT_SPEC_PARAMS                                                                                   \
    Grid3 g, typename VoxelEchoes<T, CM, EM>::Proto P, const T *__restrict__ X, const float *__restrict__ b1, \
        const float *__restrict__ bm, const float *__restrict__ Y, const float *__restrict__ w, float l0,       \
        float l1, float l2, float l3, const float4 *__restrict__ D, const float4 *__restrict__ P0,              \
        const float4 *__restrict__ P1, int loading, HessArrays Hs, float4 *__restrict__ R,                      \
        float4 *__restrict__ Z, const MapCtl *__restrict__ ctl, double *__restrict__ partials
#define ACCEPT_SPEC_ARGS g, P, X, b1, bm, Y, w, l0, l1, l2, l3, D, P0, P1, loading, Hs, R, Z, ctl, partials

template <bool PLUS, typename T, int CM, int EM>
__device__ __forceinline__ void accept_spec_body(ACCEPT_SPEC_PARAMS, int L, int T_)
{
    if (ctl->gn_stop) return;
    const int64_t N = g.N;
    const float lam[4] = {l0, l1, l2, l3};
    const DeltaF getd{D, ctl->p_buf ? P1 : P0, (float)ctl->alpha_pend, ctl->delta_valid != 0};
    const Col c = locate_col(g, L, T_);
    const auto K = VoxelEchoes<T, CM, EM>::stage(P);
    double part[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (c.act) {
        const int64_t n = c.base + (int64_t)c.z0 * c.sxy;
        VoxelEchoes<T, CM, EM> ve;
        ve.load(P, X, N, n, b1 ? b1[n] : 1.0f, bm ? bm[n] : 1.0f);
        float y0[4], d0[4], yt[4];
        load4(Y, N, n, y0);
        getd(n, d0);
#pragma unroll
        for (int k = 0; k < 4; k++) yt[k] = y0[k] - d0[k];
        const float w0 = w[n];
        float ay[4] = {0.f, 0.f, 0.f, 0.f}, ad[4] = {0.f, 0.f, 0.f, 0.f}, at[4] = {0.f, 0.f, 0.f, 0.f};
        float d = 0.f, d2 = 0.f, d3 = 0.f;
        const auto nb = [&](int64_t m) {
            float vm[4], um[4], tm[4];
            load4(Y, N, m, vm);
            getd(m, um);
#pragma unroll
            for (int k = 0; k < 4; k++) tm[k] = vm[k] - um[k];
            const float wmm = w[m];
            edge(w0, wmm, y0, vm, ay, d);
            edge(w0, wmm, d0, um, ad, d2);
            edge(w0, wmm, yt, tm, at, d3);
        };
        for_inplane(c, n, g.nx, nb);
        if (c.z0 > 0) nb(n - c.sxy);
        if (c.z0 < g.nz - 1) nb(n + c.sxy);
        float gr[4], H[10], r[4], zz[4];
        const float nll = ve.template lik<PLUS>(P, K, yt, loading, true, gr, H);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            ay[k] *= lam[k];
            ad[k] *= lam[k];
            at[k] *= lam[k];  // (L y) at the full step
            r[k] = gr[k] + at[k];
        }
        precond(H, lam, d, r, zz);
        store_H(Hs, n, H);
        vstore_nt(R, n, r);
        vstore_nt(Z, n, zz);
        part[0] = nll;
        part[1] = dot4(d0, ay);
        part[2] = dot4(d0, ad);
        part[3] = dot4(yt, at);
        part[4] = dot4(r, zz);
    }
    write_partials<5>(part, partials, L, T_);
}

template <typename T, int CM, int EM>
__global__ __launch_bounds__(BLOCK) void k_accept_spec(ACCEPT_SPEC_PARAMS)
{
    accept_spec_body<false, T, CM, EM>(ACCEPT_SPEC_ARGS, blockIdx.x, gridDim.x);
}
template <typename T, int CM, int EM>  // Proposed+ loading
__global__ __launch_bounds__(BLOCK) void k_accept_spec_plus(ACCEPT_SPEC_PARAMS)
{
    accept_spec_body<true, T, CM, EM>(ACCEPT_SPEC_ARGS, blockIdx.x, gridDim.x);
}

// accept, pass 2 (only after the full step was rejected): the NLL at the
// halved steps y - 2^-h delta_f, h = 1 .. ntrial-1.  Column grid (returns at
// once in the common case, so few workgroups).  Partial row h.
#define ACCEPT2_PARAMS                                                                                       \
    Grid3 g, typename VoxelEchoes<T, CM, EM>::Proto P, const T *__restrict__ X, const float *__restrict__ b1, \
        const float *__restrict__ bm, const float *__restrict__ Y, const float4 *__restrict__ D,               \
        const float4 *__restrict__ P0, const float4 *__restrict__ P1, int ntrial, const MapCtl *__restrict__ ctl, \
        double *__restrict__ partials
#define ACCEPT2_ARGS g, P, X, b1, bm, Y, D, P0, P1, ntrial, ctl, partials

template <typename T, int CM, int EM>
__device__ __forceinline__ void accept2_body(ACCEPT2_PARAMS, int L, int T_)
{
    if (ctl->gn_stop || !ctl->accept_more) return;
    const int64_t N = g.N;
    const DeltaF getd{D, ctl->p_buf ? P1 : P0, (float)ctl->alpha_pend, ctl->delta_valid != 0};
    const Col c = locate_col(g, L, T_);
    const auto K = VoxelEchoes<T, CM, EM>::stage(P);
    double part[MAX_TRIALS];
#pragma unroll
    for (int h = 0; h < MAX_TRIALS; h++) part[h] = 0.0;
    if (c.act) {
        for (int z = c.z0; z < c.z1; z++) {
            const int64_t n = c.base + (int64_t)z * c.sxy;
            VoxelEchoes<T, CM, EM> ve;
            ve.load(P, X, N, n, b1 ? b1[n] : 1.0f, bm ? bm[n] : 1.0f);
            float y[4], df[4];
            load4(Y, N, n, y);
            getd(n, df);
            float step = 0.5f;
#pragma unroll 1
            for (int h = 1; h < ntrial; h++) {
                float yt[4];
#pragma unroll
                for (int k = 0; k < 4; k++) yt[k] = y[k] - step * df[k];
                const float v = ve.nll(P, K, yt);
#pragma unroll
                for (int j = 1; j < MAX_TRIALS; j++)
                    if (j == h) part[j] += v;
                step *= 0.5f;
            }
        }
    }
    write_partials<MAX_TRIALS>(part, partials, L, T_);
}

template <typename T, int CM, int EM>
__global__ __launch_bounds__(BLOCK) void k_accept2(ACCEPT2_PARAMS)
{
    accept2_body<T, CM, EM>(ACCEPT2_ARGS, blockIdx.x, gridDim.x);
}

// y -= step * delta_f (voxels L * BLOCK + thread)
__device__ __forceinline__ void update_body(int64_t N, float *__restrict__ Y, const float4 *__restrict__ D,
                                            const float4 *__restrict__ P0, const float4 *__restrict__ P1,
                                            const MapCtl *__restrict__ ctl, int L)
{
    if (ctl->gn_stop || ctl->step == 0.0) return;
    const float step = (float)ctl->step;
    const DeltaF getd{D, ctl->p_buf ? P1 : P0, (float)ctl->alpha_pend, ctl->delta_valid != 0};
    int64_t n = (int64_t)L * BLOCK + threadIdx.x;
    if (n >= N) return;
    float df[4];
    getd(n, df);
#pragma unroll
    for (int k = 0; k < 4; k++) Y[k * N + n] -= step * df[k];
}

__global__ __launch_bounds__(BLOCK) void k_update(int64_t N, float *__restrict__ Y, const float4 *__restrict__ D,
                                                  const float4 *__restrict__ P0, const float4 *__restrict__ P1,
                                                  const MapCtl *__restrict__ ctl)
{
    update_body(N, Y, D, P0, P1, ctl, blockIdx.x);
}

// ---------------------------------------------------------------------------
// JTV weights (paper Sec. 2.5, eq. bound): q_n = sum_k lam_k ||G_n y_k||^2,
// w_n = (q_n + eps^2)^(-1/2).  Partial: sum_n sqrt(q_n + eps^2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void weights_body(const Grid3 &g, const float *__restrict__ Y, float l0, float l1,
                                             float l2, float l3, float eps, int prior_on, float *__restrict__ w,
                                             double *__restrict__ partials, int L, int T)
{
    const int64_t N = g.N;
    const float lam[4] = {l0, l1, l2, l3};
    const Col c = locate_col(g, L, T);
    double part[1] = {0.0};
    if (c.act) {
        int64_t n = c.base + (int64_t)c.z0 * c.sxy;
        if (!prior_on) {
            for (int z = c.z0; z < c.z1; z++, n += c.sxy) w[n] = 0.0f;
        } else {
            float ym[4], y0[4], yp[4];
            if (c.z0 > 0) load4(Y, N, n - c.sxy, ym);
            load4(Y, N, n, y0);
            for (int z = c.z0; z < c.z1; z++, n += c.sxy) {
                const bool hzp = z < g.nz - 1;
                if (hzp) load4(Y, N, n + c.sxy, yp);
                float acc[4] = {0.f, 0.f, 0.f, 0.f};
                auto sq = [&](const float vm[4]) {
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        const float dk = vm[k] - y0[k];
                        acc[k] += dk * dk;
                    }
                };
                for_inplane(c, n, g.nx, [&](int64_t m) {
                    float vm[4];
                    load4(Y, N, m, vm);
                    sq(vm);
                });
                if (z > 0) sq(ym);
                if (hzp) sq(yp);
                float q = 0.f;
#pragma unroll
                for (int k = 0; k < 4; k++) q += lam[k] * acc[k];
                const float root = sqrtf(q + eps * eps);
                w[n] = root > 0.f ? 1.0f / root : 0.0f;
                part[0] += root;
                copy4(ym, y0);
                copy4(y0, yp);
            }
        }
    }
    write_partials<1>(part, partials, L, T);
}

__global__ __launch_bounds__(BLOCK) void k_weights(Grid3 g, const float *__restrict__ Y, float l0, float l1,
                                                   float l2, float l3, float eps, int prior_on,
                                                   float *__restrict__ w, double *__restrict__ partials)
{
    weights_body(g, Y, l0, l1, l2, l3, eps, prior_on, w, partials, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// final statistics at the fitted maps: NLL, degenerate M blocks, non-finite
// voxels.  With var != NULL also the Laplace variance of paper Sec. 3.6 (and
// with mom != NULL the log-normal moments of r1 and t1).
// ---------------------------------------------------------------------------
template <bool PLUS, typename T, int CM, int EM>
__device__ __forceinline__ void final_body(const Grid3 &g, const typename VoxelEchoes<T, CM, EM>::Proto &P,
                                           const T *__restrict__ X, const float *__restrict__ b1,
                                           const float *__restrict__ bm,
                                           const float *__restrict__ Y, const float *__restrict__ w, float l0,
                                           float l1, float l2, float l3, int loading, float *__restrict__ var,
                                           float *__restrict__ mom, double *__restrict__ partials, int L, int T_)
{
    const int64_t N = g.N;
    const float lam[4] = {l0, l1, l2, l3};
    const Col c = locate_col(g, L, T_);
    const auto K = VoxelEchoes<T, CM, EM>::stage(P);
    double part[3] = {0.0, 0.0, 0.0};
    if (c.act) {
        const int64_t n = c.base + (int64_t)c.z0 * c.sxy;
        VoxelEchoes<T, CM, EM> ve;
        ve.load(P, X, N, n, b1 ? b1[n] : 1.0f, bm ? bm[n] : 1.0f);
        const float w0 = w[n];
        float d = 0.f;
        for_inplane(c, n, g.nx, [&](int64_t m) { d += w0 + w[m]; });
        if (c.z0 > 0) d += w0 + w[n - c.sxy];
        if (c.z0 < g.nz - 1) d += w0 + w[n + c.sxy];
        float y[4], gr[4], H[10];
        load4(Y, N, n, y);
        const float nll = ve.template lik<PLUS>(P, K, y, loading, true, gr, H);
        float M[10];
#pragma unroll
        for (int k = 0; k < 10; k++) M[k] = H[k];
        M[0] += lam[0] * d;
        M[4] += lam[1] * d;
        M[7] += lam[2] * d;
        M[9] += lam[3] * d;
        const float e0[4] = {1.f, 0.f, 0.f, 0.f};
        float tmp[4];
        const bool degen = solve_sym4(M, e0, tmp);
        bool bad = false;
#pragma unroll
        for (int k = 0; k < 4; k++) bad |= !(fabsf(y[k]) < INFINITY);
        part[0] = nll;
        part[1] = degen ? 1.0 : 0.0;
        part[2] = bad ? 1.0 : 0.0;
        if (var) {
            const float dg[4] = {M[0], M[4], M[7], M[9]};
            const float maxd = fmaxf(fmaxf(dg[0], dg[1]), fmaxf(dg[2], dg[3]));
            float vv[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                float e[4] = {0.f, 0.f, 0.f, 0.f}, col[4];
                e[k] = 1.0f;
                const bool frozen = !(dg[k] > FROZEN_REL * maxd);
                const bool dk = solve_sym4(M, e, col);
                vv[k] = (frozen || dk) ? INFINITY : col[k];
                var[k * N + n] = vv[k];
            }
            if (mom) {
                const float ev = expf(vv[1]);
                const float er = expf(y[1]), et = expf(-y[1]);
                mom[n] = sqrtf(ev) * er;
                mom[N + n] = (ev - 1.0f) * ev * er * er;
                mom[2 * N + n] = sqrtf(ev) * et;
                mom[3 * N + n] = (ev - 1.0f) * ev * et * et;
            }
        }
    }
    write_partials<3>(part, partials, L, T_);
}

#define FINAL_PARAMS                                                                                         \
    Grid3 g, typename VoxelEchoes<T, CM, EM>::Proto P, const T *__restrict__ X, const float *__restrict__ b1, \
        const float *__restrict__ bm,                                                                        \
        const float *__restrict__ Y, const float *__restrict__ w, float l0, float l1, float l2, float l3,       \
        int loading, float *__restrict__ var, float *__restrict__ mom, double *__restrict__ partials
#define FINAL_ARGS g, P, X, b1, bm, Y, w, l0, l1, l2, l3, loading, var, mom, partials

template <typename T, int CM, int EM>
__global__ __launch_bounds__(BLOCK) void k_final(FINAL_PARAMS)
{
    final_body<false, T, CM, EM>(FINAL_ARGS, blockIdx.x, gridDim.x);
}
template <typename T, int CM, int EM>  // Proposed+ loading
__global__ __launch_bounds__(BLOCK) void k_final_plus(FINAL_PARAMS)
{
    final_body<true, T, CM, EM>(FINAL_ARGS, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// one-workgroup finalisers: fixed-order reduction of the partials, then the
// scalar logic of the step
// ---------------------------------------------------------------------------
// Early stopping (reading of the gain in Sec. 2.7): a step from F to Fn ends
// its outer loop when its decrease is below tol times the decrease since the
// loop's first F_w (or there was none); the flag takes effect after the
// step's update.
__device__ __forceinline__ void stop_on_gain(MapCtl &c, double F, double Fn, double tol)
{
    if (!(tol > 0.0)) return;
    const double den = c.F_loop0 - Fn;
    if (!(den > 0.0) || F - Fn < tol * den) c.tol_stop = 1;
}

__device__ __forceinline__ void fin_body(int stage, int arg, int nblk, const double *__restrict__ partials,
                                         MapCtl *__restrict__ ctl, double *__restrict__ trace, double cg_stop_rel,
                                         int ntrial, int accept_off, const ExtRows &ext, double tol_gn,
                                         double tol_outer)
{
    __shared__ double lds[FIN_THREADS / 64];
    const bool gated = (stage == FIN_W || stage == FIN_STATS) ? false : (ctl->gn_stop != 0);
    if (gated) return;
    if ((stage == FIN_A || stage == FIN_B) && ctl->cg_stop) return;
    if (stage == FIN_ACCEPT2 && !ctl->accept_more) return;
    double s[MAX_TRIALS];
    const int rows = (stage == FIN_LIK || stage == FIN_ACCEPT || stage == FIN_ACCEPT_SPEC || stage == FIN_STATS) ? 3
                     : stage == FIN_ACCEPT2                                          ? MAX_TRIALS
                     : stage == FIN_STOP                                             ? 0
                                                                                     : 1;
    // the likelihood pass evaluated by the accept pass: rows 0, 3, 4
    const bool spec = stage == FIN_LIK && ctl->spec_ready;
    for (int k = 0; k < rows; k++)
        s[k] = reduce_row(partials + (int64_t)(spec && k > 0 ? k + 2 : k) * nblk, nblk, lds);
    for (int k = 0; k < rows && k < ext.rows; k++) s[k] += reduce_row(ext.p + (int64_t)k * ext.stride, ext.cols, lds);
    if (threadIdx.x != 0) return;
    MapCtl &c = *ctl;
    switch (stage) {
    case FIN_LIK:  // arg: trace slot for "F before step 0" or -1
        c.nll_cur = s[0];
        c.yLy = s[1];
        c.F = s[0] + 0.5 * s[1];
        c.gamma = c.gamma0 = s[2];
        c.gam[0] = s[2];
        c.alpha_pend = 0.0;
        c.beta = 0.0;
        c.step = 0.0;
        c.delta_valid = 0;
        c.p_buf = 0;
        c.accept_more = 0;
        c.cg_stop = !(s[2] > 0.0);
        c.spec_ready = 0;
        if (arg >= 0) {  // the first Newton step of an outer loop
            trace[arg] = c.F;
            c.F_loop0 = c.F;
        }
        break;
    case FIN_A: {  // arg: CG iteration
        const double pq = s[0];
        if (arg >= 1) c.delta_valid = 1;
        c.p_buf = arg & 1;
        if (!(pq > 0.0)) {
            c.cg_stop = 1;
            c.alpha_pend = 0.0;
        } else {
            c.alpha_pend = c.gamma / pq;
        }
        break;
    }
    case FIN_B: {
        const double gn = s[0];
        c.cg_done++;
        if (!(gn > cg_stop_rel * c.gamma0) || !(gn > 0.0)) c.cg_stop = 1;
        c.beta = gn / c.gamma;
        c.gamma = gn;
        break;
    }
    case FIN_ACCEPT:         // full step; arg: trace slot for "F after this step"
    case FIN_ACCEPT_SPEC: {  // the same, after k_accept_spec
        c.c1 = s[1];
        c.c2 = s[2];
        const double F0 = s[0] + 0.5 * (c.yLy - 2.0 * c.c1 + c.c2);
        if (accept_off || F0 <= c.F + ACCEPT_REL * fabs(c.F)) {
            stop_on_gain(c, c.F, F0, tol_gn);
            c.step = 1.0;
            c.spec_ready = stage == FIN_ACCEPT_SPEC;
            c.nll_cur = s[0];
            c.F = F0;
            c.gn_done++;
            if (arg >= 0) trace[arg] = F0;
        } else if (ntrial > 1) {
            c.accept_more = 1;
        } else {
            c.step = 0.0;
            c.gn_stop = 1;
            c.rejected++;
        }
        break;
    }
    case FIN_ACCEPT2: {  // halved steps
        double t = 0.5;
        int chosen = -1;
        double Fc = 0.0;
        for (int h = 1; h < ntrial; h++) {
            const double Fh = s[h] + 0.5 * (c.yLy - 2.0 * t * c.c1 + t * t * c.c2);
            if (Fh <= c.F + ACCEPT_REL * fabs(c.F)) {
                chosen = h;
                Fc = Fh;
                break;
            }
            t *= 0.5;
        }
        c.accept_more = 0;
        if (chosen >= 0) {
            stop_on_gain(c, c.F, Fc, tol_gn);
            c.step = t;
            c.nll_cur = s[chosen];
            c.F = Fc;
            c.gn_done++;
            if (arg >= 0) trace[arg] = Fc;
        } else {
            c.step = 0.0;
            c.gn_stop = 1;
            c.rejected++;
        }
        break;
    }
    case FIN_W: {  // the end of an outer loop; arg: its trace slot or -1
        const bool stopped = c.outer_stop != 0;
        const double O = c.nll_cur + s[0];
        c.jtv = s[0];
        if (!stopped) {
            if (arg >= 0) trace[arg] = O;
            c.outer_done++;
            if (c.n_obj == 0) {
                c.obj_first = O;
            } else if (tol_outer > 0.0) {
                const double den = c.obj_first - O;
                if (!(den > 0.0) || c.obj_prev - O < tol_outer * den) c.outer_stop = 1;
            }
            c.obj_prev = O;
            c.n_obj++;
        }
        c.gn_stop = c.outer_stop;
        c.tol_stop = 0;
        c.spec_ready = 0;  // the weights changed (or the loop stopped before using it)
        break;
    }
    case FIN_STOP:  // after the update of a step that ended its outer loop
        if (c.tol_stop) {
            c.gn_stop = 1;
            c.tol_stop = 0;
        }
        break;
    case FIN_STATS:
        c.nll_final = s[0];
        c.degenerate = s[1];
        c.nonfinite = s[2];
        break;
    }
}

__global__ __launch_bounds__(FIN_THREADS) void k_fin(int stage, int arg, int nblk,
                                                     const double *__restrict__ partials, MapCtl *__restrict__ ctl,
                                                     double *__restrict__ trace, double cg_stop_rel, int ntrial,
                                                     int accept_off, ExtRows ext, double tol_gn, double tol_outer)
{
    fin_body(stage, arg, nblk, partials, ctl, trace, cg_stop_rel, ntrial, accept_off, ext, tol_gn, tol_outer);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static dim3 cols(const Grid3 &g) { return dim3((unsigned)grid_blocks(g)); }

hipError_t launch_ctl_init(hipStream_t s, MapCtl *ctl, double *trace, int trace_len)
{
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(BLOCK), 0, s, ctl, trace, trace_len);
    return hipGetLastError();
}

// Launch KERNEL<T, CM, EM>(G, protocol, X, ...) for the echo storage type T
// and the register shape (CM, EM) of the protocol (echo_shape).
#define LAUNCH_ONE(KERNEL, T, CM, EM, G, ...)                                                          \
    hipLaunchKernelGGL((KERNEL<T, CM, EM>), cols(G), dim3(BLOCK), 0, s, G,                             \
                       (ProtoArg<T, CM, EM>::make(a.P, (const T *)a.X, a.g.N)), (const T *)a.X, __VA_ARGS__)

#define LAUNCH_SHAPED(KERNEL, T, G, ...)                                     \
    do {                                                                     \
        switch (echo_shape(a.P)) {                                           \
        case 1: LAUNCH_ONE(KERNEL, T, 4, 8, G, __VA_ARGS__); break;          \
        case 2: LAUNCH_ONE(KERNEL, T, 4, 16, G, __VA_ARGS__); break;         \
        case 3: LAUNCH_ONE(KERNEL, T, 8, 8, G, __VA_ARGS__); break;          \
        default: LAUNCH_ONE(KERNEL, T, 0, 0, G, __VA_ARGS__); break;         \
        }                                                                    \
    } while (0)

#define DISPATCH_T(KERNEL, G, ...)                                           \
    do {                                                                     \
        if (a.dtype == DT_F32) {                                             \
            using T = float;                                                 \
            LAUNCH_SHAPED(KERNEL, T, G, __VA_ARGS__);                        \
        } else if (a.dtype == DT_F16) {                                      \
            using T = F16;                                                   \
            LAUNCH_SHAPED(KERNEL, T, G, __VA_ARGS__);                        \
        } else {                                                             \
            using T = BF16;                                                  \
            LAUNCH_SHAPED(KERNEL, T, G, __VA_ARGS__);                        \
        }                                                                    \
    } while (0)

hipError_t launch_lik(hipStream_t s, const MapArgs &a)
{
    const float *l = a.lam;
    if (a.loading == 2)
        DISPATCH_T(k_lik_plus, a.gp, a.b1, a.bm, a.Y, a.w, l[0], l[1], l[2], l[3], a.loading, a.H, a.R, a.Z, a.ctl,
                   a.partials);
    else
        DISPATCH_T(k_lik, a.gp, a.b1, a.bm, a.Y, a.w, l[0], l[1], l[2], l[3],
                   a.loading, a.H, a.R, a.Z, a.ctl, a.partials);
    return hipGetLastError();
}

// With folded finalising sweep A writes partial row 0 and reads sweep B's
// row 1; sweep B the other way round.
static CgFold fold_a(const MapArgs &a)
{
    return CgFold{a.fold, a.nb_b, a.partials + a.pstride, a.cg_stop_rel};
}

static CgFold fold_b(const MapArgs &a)
{
    return CgFold{a.fold, a.nb_a, a.partials, a.cg_stop_rel};
}

hipError_t launch_cg_a(hipStream_t s, const MapArgs &a, int it)
{
    const float *l = a.lam;
    const float4 *pold = (it & 1) ? a.P0 : a.P1;
    float4 *pnew = (it & 1) ? a.P1 : a.P0;
    if (a.fold)
        hipLaunchKernelGGL(k_cg_a<true>, cols(a.gt), dim3(TALL_THREADS), 0, s, a.gt, it, a.H, a.w, l[0], l[1], l[2],
                           l[3], a.Z, pold, pnew, a.D, a.ctl, a.partials, fold_a(a));
    else
        hipLaunchKernelGGL(k_cg_a<false>, cols(a.gt), dim3(TALL_THREADS), 0, s, a.gt, it, a.H, a.w, l[0], l[1], l[2],
                           l[3], a.Z, pold, pnew, a.D, a.ctl, a.partials, fold_a(a));
    return hipGetLastError();
}

hipError_t launch_cg_b(hipStream_t s, const MapArgs &a, int it)
{
    const float *l = a.lam;
    const float4 *pc = (it & 1) ? a.P1 : a.P0;
    if (a.fold)
        hipLaunchKernelGGL(k_cg_b<true>, cols(a.gv), dim3(CGB_THREADS), 0, s, a.gv, it, a.H, a.w, l[0], l[1], l[2],
                           l[3], pc, a.R, a.Z, a.ctl, a.partials + a.pstride, fold_b(a));
    else
        hipLaunchKernelGGL(k_cg_b<false>, cols(a.gv), dim3(CGB_THREADS), 0, s, a.gv, it, a.H, a.w, l[0], l[1], l[2],
                           l[3], pc, a.R, a.Z, a.ctl, a.partials, fold_b(a));
    return hipGetLastError();
}

int cg_a_blocks(const MapArgs &a) { return grid_blocks(a.gt); }
int cg_b_blocks(const MapArgs &a) { return grid_blocks(a.gv); }
int cg_b_rows() { return CGB_Y; }

hipError_t launch_accept(hipStream_t s, const MapArgs &a)
{
    const float *l = a.lam;
    DISPATCH_T(k_accept, a.gp, a.b1, a.bm, a.Y, a.w, l[0], l[1], l[2], l[3], a.D, a.P0, a.P1, a.ctl,
               a.partials);
    return hipGetLastError();
}

hipError_t launch_accept_spec(hipStream_t s, const MapArgs &a)
{
    const float *l = a.lam;
    if (a.loading == 2)
        DISPATCH_T(k_accept_spec_plus, a.gp, a.b1, a.bm, a.Y, a.w, l[0], l[1], l[2], l[3], a.D, a.P0, a.P1,
                   a.loading, a.H, a.R, a.Z, a.ctl, a.partials);
    else
        DISPATCH_T(k_accept_spec, a.gp, a.b1, a.bm, a.Y, a.w, l[0], l[1], l[2], l[3], a.D, a.P0, a.P1, a.loading,
                   a.H, a.R, a.Z, a.ctl, a.partials);
    return hipGetLastError();
}

hipError_t launch_accept2(hipStream_t s, const MapArgs &a, int ntrial)
{
    DISPATCH_T(k_accept2, a.g, a.b1, a.bm, a.Y, a.D, a.P0, a.P1, ntrial, a.ctl, a.partials);
    return hipGetLastError();
}

hipError_t launch_update(hipStream_t s, const MapArgs &a)
{
    int nb = (int)((a.g.N + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_update, dim3(nb), dim3(BLOCK), 0, s, a.g.N, a.Y, a.D, a.P0, a.P1, a.ctl);
    return hipGetLastError();
}

hipError_t launch_weights(hipStream_t s, const MapArgs &a, int prior_on)
{
    const float *l = a.lam;
    hipLaunchKernelGGL(k_weights, cols(a.g), dim3(BLOCK), 0, s, a.g, a.Y, l[0], l[1], l[2], l[3], a.eps, prior_on,
                       a.w, a.partials);
    return hipGetLastError();
}

hipError_t launch_final(hipStream_t s, const MapArgs &a, float *var, float *mom)
{
    const float *l = a.lam;
    if (a.loading == 2)
        DISPATCH_T(k_final_plus, a.gp, a.b1, a.bm, a.Y, a.w, l[0], l[1], l[2], l[3], a.loading, var, mom, a.partials);
    else
        DISPATCH_T(k_final, a.gp, a.b1, a.bm, a.Y, a.w, l[0], l[1], l[2], l[3], a.loading, var, mom, a.partials);
    return hipGetLastError();
}

hipError_t launch_fin(hipStream_t s, const MapArgs &a, int stage, int arg, int nblk, double cg_stop_rel,
                      int ntrial, int accept_off, const ExtRows &ext, int row)
{
    hipLaunchKernelGGL(k_fin, dim3(1), dim3(FIN_THREADS), 0, s, stage, arg, nblk, a.partials + (int64_t)row * a.pstride,
                       a.ctl, a.trace, cg_stop_rel, ntrial, accept_off, ext, a.tol_gn, a.tol_outer);
    return hipGetLastError();
}

// --- the MAP kernels on pushed blocks (projected fits) ---
hipError_t launch_lik_pushed(hipStream_t s, const MapArgs &a, const PushedProto &pp)
{
    const float *l = a.lam;
    hipLaunchKernelGGL((k_lik<Pushed, 0, 0>), cols(a.gp), dim3(BLOCK), 0, s, a.gp, pp, (const Pushed *)nullptr,
                       (const float *)nullptr, (const float *)nullptr,
                       a.Y, a.w, l[0], l[1], l[2], l[3], a.loading, a.H, a.R, a.Z, a.ctl,
                       a.partials);
    return hipGetLastError();
}

hipError_t launch_accept_pushed(hipStream_t s, const MapArgs &a, const PushedProto &pp)
{
    const float *l = a.lam;
    hipLaunchKernelGGL((k_accept<Pushed, 0, 0>), cols(a.gp), dim3(BLOCK), 0, s, a.gp, pp, (const Pushed *)nullptr,
                       (const float *)nullptr, (const float *)nullptr,
                       a.Y, a.w, l[0], l[1], l[2], l[3], a.D, a.P0, a.P1, a.ctl, a.partials);
    return hipGetLastError();
}

hipError_t launch_final_pushed(hipStream_t s, const MapArgs &a, const PushedProto &pp, float *var, float *mom)
{
    const float *l = a.lam;
    hipLaunchKernelGGL((k_final<Pushed, 0, 0>), cols(a.gp), dim3(BLOCK), 0, s, a.gp, pp, (const Pushed *)nullptr,
                       (const float *)nullptr, (const float *)nullptr,
                       a.Y, a.w, l[0], l[1], l[2], l[3], a.loading, var, mom, a.partials);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched launches (several volumes per launch; see BatchTab)
// ---------------------------------------------------------------------------
template <typename Proto>
struct VolDesc {
    MapArgs m;
    int prior_on;
    Proto proto;
};

// Volume of workgroup b in a launch over grid kind k, and the workgroup's
// index L and count T within that volume; -1 for the alignment padding.
__device__ __forceinline__ int batch_volume(const BatchTab *__restrict__ tab, int k, int b, int &L, int &T)
{
    int lo = 0, hi = tab->n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tab->start[k][mid] <= b) lo = mid;
        else hi = mid;
    }
    L = b - tab->start[k][lo];
    T = tab->count[k][lo];
    return L < T ? lo : -1;
}

__global__ void k_ctl_init_batch(const VolDesc<DevProto> *__restrict__ vols, size_t stride, int trace_len)
{
    const MapArgs &m = ((const VolDesc<DevProto> *)((const char *)vols + stride * blockIdx.x))->m;
    if (threadIdx.x == 0) {
        MapCtl c = {};
        *m.ctl = c;
    }
    for (int i = threadIdx.x; i < trace_len; i += blockDim.x) m.trace[i] = __builtin_nan("");
}

// The descriptor of volume v: element v of an array of VolDesc<Proto>.
template <typename Proto>
__device__ __forceinline__ const VolDesc<Proto> &vol_at(const void *vols, int v)
{
    return ((const VolDesc<Proto> *)vols)[v];
}

template <bool PLUS, typename T, int CM, int EM>
__global__ __launch_bounds__(BLOCK) void k_lik_batch(const BatchTab *__restrict__ tab, const void *__restrict__ vols)
{
    int L, Tn;
    const int v = batch_volume(tab, BK_PLANE, blockIdx.x, L, Tn);
    if (v < 0) return;
    const auto &d = vol_at<typename VoxelEchoes<T, CM, EM>::Proto>(vols, v);
    const MapArgs &m = d.m;
    lik_body<PLUS, T, CM, EM>(m.gp, d.proto, (const T *)m.X, m.b1, m.bm, m.Y, m.w, m.lam[0], m.lam[1], m.lam[2],
                              m.lam[3], m.loading, m.H, m.R, m.Z, m.ctl, m.partials, L, Tn);
}

__global__ __launch_bounds__(TALL_THREADS) void k_cg_a_batch(const BatchTab *__restrict__ tab,
                                                                const void *__restrict__ vols, size_t stride, int it)
{
    int L, Tn;
    const int v = batch_volume(tab, BK_TALL, blockIdx.x, L, Tn);
    if (v < 0) return;
    const MapArgs &m = ((const VolDesc<DevProto> *)((const char *)vols + stride * v))->m;
    const float4 *pold = (it & 1) ? m.P0 : m.P1;
    float4 *pnew = (it & 1) ? m.P1 : m.P0;
    cg_a_body<false>(m.gt, it, m.H, m.w, m.lam[0], m.lam[1], m.lam[2], m.lam[3], m.Z, pold, pnew, m.D, m.ctl,
                     m.partials, CgFold{0, 0, nullptr, 0.0}, L, Tn);
}

__global__ __launch_bounds__(CGB_THREADS) void k_cg_b_batch(const BatchTab *__restrict__ tab,
                                                               const void *__restrict__ vols, size_t stride, int it)
{
    int L, Tn;
    const int v = batch_volume(tab, BK_CGB, blockIdx.x, L, Tn);
    if (v < 0) return;
    const MapArgs &m = ((const VolDesc<DevProto> *)((const char *)vols + stride * v))->m;
    const float4 *pc = (it & 1) ? m.P1 : m.P0;
    cg_b_body<false>(m.gv, it, m.H, m.w, m.lam[0], m.lam[1], m.lam[2], m.lam[3], pc, m.R, m.Z, m.ctl, m.partials,
                     CgFold{0, 0, nullptr, 0.0}, L, Tn);
}

template <typename T, int CM, int EM>
__global__ __launch_bounds__(BLOCK) void k_accept_batch(const BatchTab *__restrict__ tab,
                                                        const void *__restrict__ vols)
{
    int L, Tn;
    const int v = batch_volume(tab, BK_PLANE, blockIdx.x, L, Tn);
    if (v < 0) return;
    const auto &d = vol_at<typename VoxelEchoes<T, CM, EM>::Proto>(vols, v);
    const MapArgs &m = d.m;
    accept_body<T, CM, EM>(m.gp, d.proto, (const T *)m.X, m.b1, m.bm, m.Y, m.w, m.lam[0], m.lam[1], m.lam[2],
                           m.lam[3], m.D, m.P0, m.P1, m.ctl, m.partials, L, Tn);
}

template <typename T, int CM, int EM>
__global__ __launch_bounds__(BLOCK) void k_accept2_batch(const BatchTab *__restrict__ tab,
                                                         const void *__restrict__ vols, int ntrial)
{
    int L, Tn;
    const int v = batch_volume(tab, BK_COL, blockIdx.x, L, Tn);
    if (v < 0) return;
    const auto &d = vol_at<typename VoxelEchoes<T, CM, EM>::Proto>(vols, v);
    const MapArgs &m = d.m;
    accept2_body<T, CM, EM>(m.g, d.proto, (const T *)m.X, m.b1, m.bm, m.Y, m.D, m.P0, m.P1, ntrial, m.ctl,
                            m.partials, L, Tn);
}

__global__ __launch_bounds__(BLOCK) void k_update_batch(const BatchTab *__restrict__ tab,
                                                        const void *__restrict__ vols, size_t stride)
{
    int L, Tn;
    const int v = batch_volume(tab, BK_UPD, blockIdx.x, L, Tn);
    if (v < 0) return;
    const MapArgs &m = ((const VolDesc<DevProto> *)((const char *)vols + stride * v))->m;
    update_body(m.g.N, m.Y, m.D, m.P0, m.P1, m.ctl, L);
}

__global__ __launch_bounds__(BLOCK) void k_weights_batch(const BatchTab *__restrict__ tab,
                                                         const void *__restrict__ vols, size_t stride)
{
    int L, Tn;
    const int v = batch_volume(tab, BK_COL, blockIdx.x, L, Tn);
    if (v < 0) return;
    const VolDesc<DevProto> &d = *(const VolDesc<DevProto> *)((const char *)vols + stride * v);
    const MapArgs &m = d.m;
    weights_body(m.g, m.Y, m.lam[0], m.lam[1], m.lam[2], m.lam[3], m.eps, d.prior_on, m.w, m.partials, L, Tn);
}

template <bool PLUS, typename T, int CM, int EM>
__global__ __launch_bounds__(BLOCK) void k_final_batch(const BatchTab *__restrict__ tab,
                                                       const void *__restrict__ vols)
{
    int L, Tn;
    const int v = batch_volume(tab, BK_PLANE, blockIdx.x, L, Tn);
    if (v < 0) return;
    const auto &d = vol_at<typename VoxelEchoes<T, CM, EM>::Proto>(vols, v);
    const MapArgs &m = d.m;
    final_body<PLUS, T, CM, EM>(m.gp, d.proto, (const T *)m.X, m.b1, m.bm, m.Y, m.w, m.lam[0], m.lam[1], m.lam[2],
                                m.lam[3], m.loading, nullptr, nullptr, m.partials, L, Tn);
}

// one workgroup per volume
__global__ __launch_bounds__(FIN_THREADS) void k_fin_batch(const BatchTab *__restrict__ tab,
                                                           const void *__restrict__ vols, size_t stride, int stage,
                                                           int arg, int kind, int row, double cg_stop_rel,
                                                           int ntrial, int accept_off, double tol_gn,
                                                           double tol_outer)
{
    const int v = blockIdx.x;
    const MapArgs &m = ((const VolDesc<DevProto> *)((const char *)vols + stride * v))->m;
    const int nblk = kind >= 0 ? tab->count[kind][v] : 0;
    fin_body(stage, arg, nblk, m.partials + (int64_t)row * m.pstride, m.ctl, m.trace, cg_stop_rel, ntrial,
             accept_off, ExtRows(), tol_gn, tol_outer);
}

// --- host side of the batched launches ---
template <typename T, int CM, int EM>
static size_t desc_bytes_of()
{
    return sizeof(VolDesc<typename VoxelEchoes<T, CM, EM>::Proto>);
}

template <typename T, int CM, int EM>
static void fill_desc_of(void *host, int v, const MapArgs &m, int prior_on)
{
    using Proto = typename VoxelEchoes<T, CM, EM>::Proto;
    VolDesc<Proto> *d = (VolDesc<Proto> *)host + v;
    memset((void *)d, 0, sizeof(*d));
    d->m = m;
    d->prior_on = prior_on;
    d->proto = ProtoArg<T, CM, EM>::make(m.P, (const T *)m.X, m.g.N);
}

#define BATCH_SHAPED(FN, T, ...)                                  \
    do {                                                          \
        switch (shape) {                                          \
        case 1: FN<T, 4, 8>(__VA_ARGS__); break;                  \
        case 2: FN<T, 4, 16>(__VA_ARGS__); break;                 \
        case 3: FN<T, 8, 8>(__VA_ARGS__); break;                  \
        default: FN<T, 0, 0>(__VA_ARGS__); break;                 \
        }                                                         \
    } while (0)
#define BATCH_TYPED(FN, ...)                                      \
    do {                                                          \
        if (dtype == DT_F32) BATCH_SHAPED(FN, float, __VA_ARGS__); \
        else if (dtype == DT_F16) BATCH_SHAPED(FN, F16, __VA_ARGS__); \
        else BATCH_SHAPED(FN, BF16, __VA_ARGS__);                 \
    } while (0)

template <typename T, int CM, int EM>
static void desc_bytes_into(size_t *out)
{
    *out = desc_bytes_of<T, CM, EM>();
}

size_t batch_desc_bytes(int dtype, int shape)
{
    size_t b = 0;
    BATCH_TYPED(desc_bytes_into, &b);
    return b;
}

void fill_batch_desc(void *host, int v, const MapArgs &m, int prior_on, int dtype, int shape)
{
    BATCH_TYPED(fill_desc_of, host, v, m, prior_on);
}

void fill_batch_tab(BatchTab &t, const MapArgs *m, int n, int total[BK_N])
{
    memset(&t, 0, sizeof(t));
    t.n = n;
    for (int k = 0; k < BK_N; k++) {
        int at = 0;
        for (int v = 0; v < n; v++) {
            const MapArgs &a = m[v];
            const int c = k == BK_PLANE ? grid_blocks(a.gp)
                          : k == BK_TALL ? grid_blocks(a.gt)
                          : k == BK_CGB  ? grid_blocks(a.gv)
                          : k == BK_COL  ? grid_blocks(a.g)
                                         : (int)((a.g.N + BLOCK - 1) / BLOCK);
            t.start[k][v] = at;
            t.count[k][v] = c;
            at += (c + 7) & ~7;  // the next volume starts on an XCD boundary
        }
        t.start[k][n] = at;
        total[k] = at;
    }
}

hipError_t launch_ctl_init_batch(hipStream_t s, const BatchLaunch &b, int trace_len)
{
    const size_t stride = batch_desc_bytes(b.dtype, b.shape);
    hipLaunchKernelGGL(k_ctl_init_batch, dim3(b.n), dim3(BLOCK), 0, s, (const VolDesc<DevProto> *)b.vols, stride,
                       trace_len);
    return hipGetLastError();
}

template <typename T, int CM, int EM>
static void lik_batch_of(hipStream_t s, const BatchLaunch &b)
{
    if (b.loading == 2)
        hipLaunchKernelGGL((k_lik_batch<true, T, CM, EM>), dim3(b.total[BK_PLANE]), dim3(BLOCK), 0, s, b.tab, b.vols);
    else
        hipLaunchKernelGGL((k_lik_batch<false, T, CM, EM>), dim3(b.total[BK_PLANE]), dim3(BLOCK), 0, s, b.tab,
                           b.vols);
}

hipError_t launch_lik_batch(hipStream_t s, const BatchLaunch &b)
{
    const int dtype = b.dtype, shape = b.shape;
    BATCH_TYPED(lik_batch_of, s, b);
    return hipGetLastError();
}

hipError_t launch_cg_a_batch(hipStream_t s, const BatchLaunch &b, int it)
{
    hipLaunchKernelGGL(k_cg_a_batch, dim3(b.total[BK_TALL]), dim3(TALL_THREADS), 0, s, b.tab, b.vols,
                       batch_desc_bytes(b.dtype, b.shape), it);
    return hipGetLastError();
}

hipError_t launch_cg_b_batch(hipStream_t s, const BatchLaunch &b, int it)
{
    hipLaunchKernelGGL(k_cg_b_batch, dim3(b.total[BK_CGB]), dim3(CGB_THREADS), 0, s, b.tab, b.vols,
                       batch_desc_bytes(b.dtype, b.shape), it);
    return hipGetLastError();
}

template <typename T, int CM, int EM>
static void accept_batch_of(hipStream_t s, const BatchLaunch &b)
{
    hipLaunchKernelGGL((k_accept_batch<T, CM, EM>), dim3(b.total[BK_PLANE]), dim3(BLOCK), 0, s, b.tab, b.vols);
}

hipError_t launch_accept_batch(hipStream_t s, const BatchLaunch &b)
{
    const int dtype = b.dtype, shape = b.shape;
    BATCH_TYPED(accept_batch_of, s, b);
    return hipGetLastError();
}

template <typename T, int CM, int EM>
static void accept2_batch_of(hipStream_t s, const BatchLaunch &b, int ntrial)
{
    hipLaunchKernelGGL((k_accept2_batch<T, CM, EM>), dim3(b.total[BK_COL]), dim3(BLOCK), 0, s, b.tab, b.vols,
                       ntrial);
}

hipError_t launch_accept2_batch(hipStream_t s, const BatchLaunch &b, int ntrial)
{
    const int dtype = b.dtype, shape = b.shape;
    BATCH_TYPED(accept2_batch_of, s, b, ntrial);
    return hipGetLastError();
}

hipError_t launch_update_batch(hipStream_t s, const BatchLaunch &b)
{
    hipLaunchKernelGGL(k_update_batch, dim3(b.total[BK_UPD]), dim3(BLOCK), 0, s, b.tab, b.vols,
                       batch_desc_bytes(b.dtype, b.shape));
    return hipGetLastError();
}

hipError_t launch_weights_batch(hipStream_t s, const BatchLaunch &b)
{
    hipLaunchKernelGGL(k_weights_batch, dim3(b.total[BK_COL]), dim3(BLOCK), 0, s, b.tab, b.vols,
                       batch_desc_bytes(b.dtype, b.shape));
    return hipGetLastError();
}

template <typename T, int CM, int EM>
static void final_batch_of(hipStream_t s, const BatchLaunch &b)
{
    if (b.loading == 2)
        hipLaunchKernelGGL((k_final_batch<true, T, CM, EM>), dim3(b.total[BK_PLANE]), dim3(BLOCK), 0, s, b.tab,
                           b.vols);
    else
        hipLaunchKernelGGL((k_final_batch<false, T, CM, EM>), dim3(b.total[BK_PLANE]), dim3(BLOCK), 0, s, b.tab,
                           b.vols);
}

hipError_t launch_final_batch(hipStream_t s, const BatchLaunch &b)
{
    const int dtype = b.dtype, shape = b.shape;
    BATCH_TYPED(final_batch_of, s, b);
    return hipGetLastError();
}

hipError_t launch_fin_batch(hipStream_t s, const BatchLaunch &b, int stage, int arg, int kind, double cg_stop_rel,
                            int ntrial, int accept_off, double tol_gn, double tol_outer, int row)
{
    hipLaunchKernelGGL(k_fin_batch, dim3(b.n), dim3(FIN_THREADS), 0, s, b.tab, b.vols,
                       batch_desc_bytes(b.dtype, b.shape), stage, arg, kind, row, cg_stop_rel, ntrial, accept_off,
                       tol_gn, tol_outer);
    return hipGetLastError();
}

}  // namespace mpm
