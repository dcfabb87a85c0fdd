// k_map.hip -- kernels of the JTV-regularised (MAP) fit, paper Sec. 2.5-2.7.
//
// One GN step is: lik (likelihood block + L y + CG start), n_cg x (cg_a, cg_b),
// accept (objective at every trial step), update.  Every kernel reads its
// control scalars from a device-resident MapCtl written by the one-workgroup
// "fin_*" kernels that follow each reduction, so the host never waits inside
// a fit.  Reductions are two-stage and fixed-order (deterministic).
//
// Voxel mapping: workgroups of 64 x 4 threads cover 64 x 4 tiles of one
// z-plane; the 1-D workgroup index is remapped so that each of the 8 XCDs
// receives a contiguous run of tiles (consecutive tiles share stencil halos
// in that XCD's L2).
#include "mpm_map.h"

namespace mpm {

// ---------------------------------------------------------------------------
// voxel location and the 6-neighbour stencil (unit spacing, zero difference
// across the border)
// ---------------------------------------------------------------------------
struct Vox {
    int x, y, z;
    int64_t n;
    bool act;
};

__device__ __forceinline__ Vox locate(const Grid3 &g)
{
    const int L = blockIdx.x, T = gridDim.x;
    const int q = T >> 3, r = T & 7, j = L & 7;
    const int lid = j * q + min(j, r) + (L >> 3);  // XCD-contiguous tile index
    const int bx = lid % g.gx;
    const int t2 = lid / g.gx;
    const int by = t2 % g.gy;
    const int bz = t2 / g.gy;
    Vox v;
    v.x = bx * TILE_X + (threadIdx.x & (TILE_X - 1));
    v.y = by * TILE_Y + (threadIdx.x / TILE_X);
    v.z = bz;
    v.act = v.x < g.nx && v.y < g.ny;
    v.n = v.act ? (int64_t)v.x + (int64_t)g.nx * ((int64_t)v.y + (int64_t)g.ny * v.z) : 0;
    return v;
}

// The in-bounds neighbour offsets of a voxel (count in *cnt).
__device__ __forceinline__ int neighbours(const Grid3 &g, const Vox &v, int64_t off[6])
{
    int c = 0;
    const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
    if (v.x > 0) off[c++] = -1;
    if (v.x < g.nx - 1) off[c++] = 1;
    if (v.y > 0) off[c++] = -sy;
    if (v.y < g.ny - 1) off[c++] = sy;
    if (v.z > 0) off[c++] = -sz;
    if (v.z < g.nz - 1) off[c++] = sz;
    return c;
}

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

// (L v)_k[n] = lam_k * sum_m (w_n + w_m)(v_k[n] - v_k[m]) and
// d_n = sum_m (w_n + w_m) = diag(G^T W G)_n   (paper Sec. 2.5).
// get(m, vm) fetches the field at voxel m.
template <class Get>
__device__ __forceinline__ void apply_L(const int64_t off[6], int cnt, int64_t n, const float *__restrict__ w,
                                        float wn, const float own[4], const float lam[4], Get get,
                                        float out[4], float &d)
{
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    float dd = 0.f;
    for (int j = 0; j < cnt; j++) {
        const int64_t m = n + off[j];
        const float f = wn + w[m];
        float vm[4];
        get(m, vm);
        dd += f;
#pragma unroll
        for (int k = 0; k < 4; k++) acc[k] += f * (own[k] - vm[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; k++) out[k] = lam[k] * acc[k];
    d = dd;
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

template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], double *__restrict__ partials)
{
    __shared__ double lds[NV][NWAVE];
    block_sum<NV>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) partials[(int64_t)k * gridDim.x + blockIdx.x] = v[k];
    }
}

// Likelihood block of one voxel: NLL, gradient and loaded Hessian summed over
// all echoes (paper eq. precond with the Sec. 2.4 derivatives).  X is read
// once per call.
template <typename T>
__device__ __forceinline__ float lik_block(const DevProto &P, const T *__restrict__ X, int64_t N, int64_t n,
                                           float b, const float y[4], int loading, float g[4], float H[10])
{
    Params p = decode(y);
    float nll = 0.f;
#pragma unroll
    for (int k = 0; k < 4; k++) g[k] = 0.f;
#pragma unroll
    for (int k = 0; k < 10; k++) H[k] = 0.f;
    for (int c = 0; c < P.C; c++) {
        ContrastK K = contrast_factors(p, P.tr[c], make_angle(P.flip[c] * b), P.mt[c]);
        EchoAcc acc;
        for (int i = P.first[c]; i < P.first[c + 1]; i++) {
            const float te = P.te[i];
            const float s = K.s0 * __expf(-p.r2 * te);
            acc.add(s, load_echo(X + (int64_t)i * N + n), te, P.wgt[i], p.r2);
        }
        nll += 0.5f * acc.L;
        accumulate_contrast(acc, K, p.r2, loading, g, H);
    }
    return nll;
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
// z = M^{-1} r.  Partials: NLL, y.Ly, r.z
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_lik(Grid3 g, DevProto P, const T *__restrict__ X,
                                               const float *__restrict__ b1, const float *__restrict__ Y,
                                               const float *__restrict__ w, float l0, float l1, float l2,
                                               float l3, int loading, float *__restrict__ Hs,
                                               float *__restrict__ R, float *__restrict__ Z,
                                               const MapCtl *__restrict__ ctl, double *__restrict__ partials)
{
    if (ctl->gn_stop) return;
    const int64_t N = g.N;
    const float lam[4] = {l0, l1, l2, l3};
    Vox v = locate(g);
    double part[3] = {0.0, 0.0, 0.0};
    if (v.act) {
        int64_t off[6];
        int cnt = neighbours(g, v, off);
        float y[4], Ly[4], d;
        load4(Y, N, v.n, y);
        const float wn = w[v.n];
        apply_L(off, cnt, v.n, w, wn, y, lam, [&](int64_t m, float vm[4]) { load4(Y, N, m, vm); }, Ly, d);
        float gr[4], H[10];
        float nll = lik_block(P, X, N, v.n, b1 ? b1[v.n] : 1.0f, y, loading, gr, H);
        float r[4], z[4];
#pragma unroll
        for (int k = 0; k < 4; k++) r[k] = gr[k] + Ly[k];
        precond(H, lam, d, r, z);
#pragma unroll
        for (int k = 0; k < 10; k++) Hs[k * N + v.n] = H[k];
        store4(R, N, v.n, r);
        store4(Z, N, v.n, z);
        part[0] = nll;
        part[1] = (double)y[0] * Ly[0] + (double)y[1] * Ly[1] + (double)y[2] * Ly[2] + (double)y[3] * Ly[3];
        part[2] = (double)r[0] * z[0] + (double)r[1] * z[1] + (double)r[2] * z[2] + (double)r[3] * z[3];
    }
    write_partials<3>(part, partials);
}

// ---------------------------------------------------------------------------
// CG sweep A (iteration i): p = z + beta p_old, q = (H + L) p, partial p.q;
// the deferred update delta += alpha_{i-1} p_old.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_cg_a(Grid3 g, int it, const float *__restrict__ Hs,
                                                const float *__restrict__ w, float l0, float l1, float l2,
                                                float l3, const float *__restrict__ Z,
                                                const float *__restrict__ Pold, float *__restrict__ Pnew,
                                                float *__restrict__ D, const MapCtl *__restrict__ ctl,
                                                double *__restrict__ partials)
{
    if (ctl->gn_stop || ctl->cg_stop) return;
    const int64_t N = g.N;
    const float lam[4] = {l0, l1, l2, l3};
    const float beta = it > 0 ? (float)ctl->beta : 0.0f;
    const float alpha_prev = (float)ctl->alpha_pend;
    Vox v = locate(g);
    double part[1] = {0.0};
    if (v.act) {
        int64_t off[6];
        int cnt = neighbours(g, v, off);
        auto getp = [&](int64_t m, float pm[4]) {
            load4(Z, N, m, pm);
            if (it > 0) {
#pragma unroll
                for (int k = 0; k < 4; k++) pm[k] += beta * Pold[k * N + m];
            }
        };
        float p[4], po[4] = {0.f, 0.f, 0.f, 0.f};
        load4(Z, N, v.n, p);
        if (it > 0) {
            load4(Pold, N, v.n, po);
#pragma unroll
            for (int k = 0; k < 4; k++) p[k] += beta * po[k];
        }
        float Lp[4], d, H[10], q[4];
        apply_L(off, cnt, v.n, w, w[v.n], p, lam, getp, Lp, d);
#pragma unroll
        for (int k = 0; k < 10; k++) H[k] = Hs[k * N + v.n];
        symv4(H, p, q);
#pragma unroll
        for (int k = 0; k < 4; k++) q[k] += Lp[k];
        store4(Pnew, N, v.n, p);
        if (it == 1) {
            float dl[4];
#pragma unroll
            for (int k = 0; k < 4; k++) dl[k] = alpha_prev * po[k];
            store4(D, N, v.n, dl);
        } else if (it >= 2) {
            float dl[4];
            load4(D, N, v.n, dl);
#pragma unroll
            for (int k = 0; k < 4; k++) dl[k] += alpha_prev * po[k];
            store4(D, N, v.n, dl);
        }
        part[0] = (double)p[0] * q[0] + (double)p[1] * q[1] + (double)p[2] * q[2] + (double)p[3] * q[3];
    }
    write_partials<1>(part, partials);
}

// ---------------------------------------------------------------------------
// CG sweep B (iteration i): q = (H + L) p recomputed, r -= alpha q,
// z = M^{-1} r, partial r.z
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_cg_b(Grid3 g, const float *__restrict__ Hs,
                                                const float *__restrict__ w, float l0, float l1, float l2,
                                                float l3, const float *__restrict__ Pc, float *__restrict__ R,
                                                float *__restrict__ Z, const MapCtl *__restrict__ ctl,
                                                double *__restrict__ partials)
{
    if (ctl->gn_stop || ctl->cg_stop) return;
    const int64_t N = g.N;
    const float lam[4] = {l0, l1, l2, l3};
    const float alpha = (float)ctl->alpha_pend;
    Vox v = locate(g);
    double part[1] = {0.0};
    if (v.act) {
        int64_t off[6];
        int cnt = neighbours(g, v, off);
        float p[4], Lp[4], d, H[10], q[4], r[4], z[4];
        load4(Pc, N, v.n, p);
        apply_L(off, cnt, v.n, w, w[v.n], p, lam, [&](int64_t m, float pm[4]) { load4(Pc, N, m, pm); }, Lp, d);
#pragma unroll
        for (int k = 0; k < 10; k++) H[k] = Hs[k * N + v.n];
        symv4(H, p, q);
        load4(R, N, v.n, r);
#pragma unroll
        for (int k = 0; k < 4; k++) r[k] -= alpha * (q[k] + Lp[k]);
        precond(H, lam, d, r, z);
        store4(R, N, v.n, r);
        store4(Z, N, v.n, z);
        part[0] = (double)r[0] * z[0] + (double)r[1] * z[1] + (double)r[2] * z[2] + (double)r[3] * z[3];
    }
    write_partials<1>(part, partials);
}

// ---------------------------------------------------------------------------
// accept: with delta_f = delta + alpha_pend p_last, the NLL at every trial
// y - 2^-h delta_f (h < ntrial) and the quadratic pieces delta_f.(L y),
// delta_f.(L delta_f) of the prior.  Partials: NLL_0..NLL_{ntrial-1}, c1, c2
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_accept(Grid3 g, DevProto P, const T *__restrict__ X,
                                                  const float *__restrict__ b1, const float *__restrict__ Y,
                                                  const float *__restrict__ w, float l0, float l1, float l2,
                                                  float l3, const float *__restrict__ D,
                                                  const float *__restrict__ P0, const float *__restrict__ P1,
                                                  int ntrial, const MapCtl *__restrict__ ctl,
                                                  double *__restrict__ partials)
{
    if (ctl->gn_stop) return;
    const int64_t N = g.N;
    const float lam[4] = {l0, l1, l2, l3};
    const float alpha = (float)ctl->alpha_pend;
    const bool dvalid = ctl->delta_valid;
    const float *__restrict__ Pl = ctl->p_buf ? P1 : P0;
    Vox v = locate(g);
    double part[MAX_TRIALS + 2];
#pragma unroll
    for (int h = 0; h < MAX_TRIALS + 2; h++) part[h] = 0.0;
    if (v.act) {
        int64_t off[6];
        int cnt = neighbours(g, v, off);
        auto getd = [&](int64_t m, float dm[4]) {
#pragma unroll
            for (int k = 0; k < 4; k++)
                dm[k] = (dvalid ? D[k * N + m] : 0.0f) + (alpha != 0.0f ? alpha * Pl[k * N + m] : 0.0f);
        };
        float y[4], df[4], Ly[4], Ld[4], d;
        load4(Y, N, v.n, y);
        getd(v.n, df);
        const float wn = w[v.n];
        apply_L(off, cnt, v.n, w, wn, y, lam, [&](int64_t m, float vm[4]) { load4(Y, N, m, vm); }, Ly, d);
        apply_L(off, cnt, v.n, w, wn, df, lam, getd, Ld, d);
        part[MAX_TRIALS] = (double)df[0] * Ly[0] + (double)df[1] * Ly[1] + (double)df[2] * Ly[2] + (double)df[3] * Ly[3];
        part[MAX_TRIALS + 1] =
            (double)df[0] * Ld[0] + (double)df[1] * Ld[1] + (double)df[2] * Ld[2] + (double)df[3] * Ld[3];
        const float b = b1 ? b1[v.n] : 1.0f;
        Params pt[MAX_TRIALS];
        float step = 1.0f;
#pragma unroll
        for (int h = 0; h < MAX_TRIALS; h++) {
            float yt[4];
#pragma unroll
            for (int k = 0; k < 4; k++) yt[k] = y[k] - step * df[k];
            pt[h] = decode(yt);
            step *= 0.5f;
        }
        float nll[MAX_TRIALS];
#pragma unroll
        for (int h = 0; h < MAX_TRIALS; h++) nll[h] = 0.f;
        for (int c = 0; c < P.C; c++) {
            const Angle an = make_angle(P.flip[c] * b);
            float s0[MAX_TRIALS];
#pragma unroll
            for (int h = 0; h < MAX_TRIALS; h++)
                if (h < ntrial) s0[h] = contrast_factors(pt[h], P.tr[c], an, P.mt[c]).s0;
            for (int i = P.first[c]; i < P.first[c + 1]; i++) {
                const float x = load_echo(X + (int64_t)i * N + v.n);
                const float te = P.te[i], wi = P.wgt[i];
#pragma unroll
                for (int h = 0; h < MAX_TRIALS; h++) {
                    if (h < ntrial) {
                        const float res = s0[h] * __expf(-pt[h].r2 * te) - x;
                        nll[h] += 0.5f * wi * res * res;
                    }
                }
            }
        }
#pragma unroll
        for (int h = 0; h < MAX_TRIALS; h++) part[h] = nll[h];
    }
    write_partials<MAX_TRIALS + 2>(part, partials);
}

// y -= step * (delta + alpha_pend p_last)
__global__ __launch_bounds__(BLOCK) void k_update(int64_t N, float *__restrict__ Y, const float *__restrict__ D,
                                                  const float *__restrict__ P0, const float *__restrict__ P1,
                                                  const MapCtl *__restrict__ ctl)
{
    if (ctl->gn_stop || ctl->step == 0.0) return;
    const float step = (float)ctl->step;
    const float alpha = (float)ctl->alpha_pend;
    const bool dvalid = ctl->delta_valid;
    const float *__restrict__ Pl = ctl->p_buf ? P1 : P0;
    int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= N) return;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        float df = (dvalid ? D[k * N + n] : 0.0f) + (alpha != 0.0f ? alpha * Pl[k * N + n] : 0.0f);
        Y[k * N + n] -= step * df;
    }
}

// ---------------------------------------------------------------------------
// JTV weights (paper Sec. 2.5, eq. bound): q_n = sum_k lam_k ||G_n y_k||^2,
// w_n = (q_n + eps^2)^(-1/2).  Partial: sum_n sqrt(q_n + eps^2)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_weights(Grid3 g, const float *__restrict__ Y, float l0, float l1,
                                                   float l2, float l3, float eps, int prior_on,
                                                   float *__restrict__ w, double *__restrict__ partials)
{
    const int64_t N = g.N;
    const float lam[4] = {l0, l1, l2, l3};
    Vox v = locate(g);
    double part[1] = {0.0};
    if (v.act) {
        float wn = 0.0f;
        if (prior_on) {
            int64_t off[6];
            int cnt = neighbours(g, v, off);
            float y[4], q = 0.f;
            load4(Y, N, v.n, y);
            float acc[4] = {0.f, 0.f, 0.f, 0.f};
            for (int j = 0; j < cnt; j++) {
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const float dk = Y[k * N + v.n + off[j]] - y[k];
                    acc[k] += dk * dk;
                }
            }
#pragma unroll
            for (int k = 0; k < 4; k++) q += lam[k] * acc[k];
            const float root = sqrtf(q + eps * eps);
            wn = root > 0.f ? 1.0f / root : 0.0f;
            part[0] = root;
        }
        w[v.n] = wn;
    }
    write_partials<1>(part, partials);
}

// ---------------------------------------------------------------------------
// final statistics at the fitted maps: NLL, degenerate M blocks, non-finite
// voxels.  Also used (with var != NULL) for the Laplace variance of Sec. 3.6.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_final(Grid3 g, DevProto P, const T *__restrict__ X,
                                                 const float *__restrict__ b1, const float *__restrict__ Y,
                                                 const float *__restrict__ w, float l0, float l1, float l2,
                                                 float l3, int loading, float *__restrict__ var,
                                                 float *__restrict__ mom, double *__restrict__ partials)
{
    const int64_t N = g.N;
    const float lam[4] = {l0, l1, l2, l3};
    Vox v = locate(g);
    double part[3] = {0.0, 0.0, 0.0};
    if (v.act) {
        int64_t off[6];
        int cnt = neighbours(g, v, off);
        float y[4];
        load4(Y, N, v.n, y);
        const float wn = w[v.n];
        float d = 0.f;
        for (int j = 0; j < cnt; j++) d += wn + w[v.n + off[j]];
        float gr[4], H[10];
        float nll = lik_block(P, X, N, v.n, b1 ? b1[v.n] : 1.0f, y, loading, gr, H);
        float M[10];
#pragma unroll
        for (int k = 0; k < 10; k++) M[k] = H[k];
        M[0] += lam[0] * d;
        M[4] += lam[1] * d;
        M[7] += lam[2] * d;
        M[9] += lam[3] * d;
        const float e0[4] = {1.f, 0.f, 0.f, 0.f};
        float tmp[4];
        bool degen = solve_sym4(M, e0, tmp);
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
                var[k * N + v.n] = vv[k];
            }
            if (mom) {
                const float ev = expf(vv[1]);
                const float er = expf(y[1]), et = expf(-y[1]);
                mom[v.n] = sqrtf(ev) * er;
                mom[N + v.n] = (ev - 1.0f) * ev * er * er;
                mom[2 * N + v.n] = sqrtf(ev) * et;
                mom[3 * N + v.n] = (ev - 1.0f) * ev * et * et;
            }
        }
    }
    write_partials<3>(part, partials);
}

// ---------------------------------------------------------------------------
// one-workgroup finalisers: fixed-order reduction of the partials, then the
// scalar logic of the step
// ---------------------------------------------------------------------------
__device__ __forceinline__ double reduce_row(const double *__restrict__ row, int ncols, double *lds_tmp)
{
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < ncols; b += BLOCK) v[0] += row[b];
    __shared__ double lds[1][NWAVE];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) *lds_tmp = v[0];
    __syncthreads();
    double r = *lds_tmp;
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(BLOCK) void k_fin(int stage, int arg, int nblk, const double *__restrict__ partials,
                                               MapCtl *__restrict__ ctl, double *__restrict__ trace,
                                               double cg_stop_rel, int ntrial, int accept_off)
{
    __shared__ double tmp;
    const bool gated = (stage == FIN_W || stage == FIN_STATS) ? false : (ctl->gn_stop != 0);
    if (gated) return;
    if ((stage == FIN_A || stage == FIN_B) && ctl->cg_stop) return;
    double s[MAX_TRIALS + 2];
    int rows = stage == FIN_LIK ? 3 : stage == FIN_ACCEPT ? MAX_TRIALS + 2 : stage == FIN_STATS ? 3 : 1;
    for (int k = 0; k < rows; k++) s[k] = reduce_row(partials + (int64_t)k * nblk, nblk, &tmp);
    if (threadIdx.x != 0) return;
    MapCtl &c = *ctl;
    switch (stage) {
    case FIN_LIK:  // arg: trace slot for "F before step 0" or -1
        c.nll_cur = s[0];
        c.yLy = s[1];
        c.F = s[0] + 0.5 * s[1];
        c.gamma = c.gamma0 = s[2];
        c.alpha_pend = 0.0;
        c.beta = 0.0;
        c.step = 0.0;
        c.delta_valid = 0;
        c.p_buf = 0;
        c.cg_stop = !(s[2] > 0.0);
        if (arg >= 0) trace[arg] = c.F;
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
    case FIN_ACCEPT: {  // arg: trace slot for "F after this step"
        const double c1 = s[MAX_TRIALS], c2 = s[MAX_TRIALS + 1];
        double t = 1.0;
        int chosen = -1;
        double Fc = 0.0;
        for (int h = 0; h < ntrial; h++) {
            const double Fh = s[h] + 0.5 * (c.yLy - 2.0 * t * c1 + t * t * c2);
            if (accept_off || Fh <= c.F) {
                chosen = h;
                Fc = Fh;
                break;
            }
            t *= 0.5;
        }
        if (chosen >= 0) {
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
    case FIN_W:  // arg: trace slot for "objective at the end of the outer loop" or -1
        c.jtv = s[0];
        if (arg >= 0) trace[arg] = c.nll_cur + s[0];
        c.gn_stop = 0;
        break;
    case FIN_STATS:
        c.nll_final = s[0];
        c.degenerate = s[1];
        c.nonfinite = s[2];
        break;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static dim3 tiles(const Grid3 &g) { return dim3((unsigned)((int64_t)g.gx * g.gy * g.nz)); }

hipError_t launch_ctl_init(hipStream_t s, MapCtl *ctl, double *trace, int trace_len)
{
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(BLOCK), 0, s, ctl, trace, trace_len);
    return hipGetLastError();
}

hipError_t launch_lik(hipStream_t s, const MapArgs &a)
{
    const float *l = a.lam;
#define LIK_ARGS a.g, a.P, (const T *)a.X, a.b1, a.Y, a.w, l[0], l[1], l[2], l[3], a.loading, a.H, a.R, a.Z, a.ctl, a.partials
    if (a.dtype == DT_F32) {
        using T = float;
        hipLaunchKernelGGL(k_lik<T>, tiles(a.g), dim3(BLOCK), 0, s, LIK_ARGS);
    } else if (a.dtype == DT_F16) {
        using T = F16;
        hipLaunchKernelGGL(k_lik<T>, tiles(a.g), dim3(BLOCK), 0, s, LIK_ARGS);
    } else {
        using T = BF16;
        hipLaunchKernelGGL(k_lik<T>, tiles(a.g), dim3(BLOCK), 0, s, LIK_ARGS);
    }
#undef LIK_ARGS
    return hipGetLastError();
}

hipError_t launch_cg_a(hipStream_t s, const MapArgs &a, int it)
{
    const float *l = a.lam;
    const float *pold = (it & 1) ? a.P0 : a.P1;
    float *pnew = (it & 1) ? a.P1 : a.P0;
    hipLaunchKernelGGL(k_cg_a, tiles(a.g), dim3(BLOCK), 0, s, a.g, it, a.H, a.w, l[0], l[1], l[2], l[3], a.Z,
                       pold, pnew, a.D, a.ctl, a.partials);
    return hipGetLastError();
}

hipError_t launch_cg_b(hipStream_t s, const MapArgs &a, int it)
{
    const float *l = a.lam;
    const float *pc = (it & 1) ? a.P1 : a.P0;
    hipLaunchKernelGGL(k_cg_b, tiles(a.g), dim3(BLOCK), 0, s, a.g, a.H, a.w, l[0], l[1], l[2], l[3], pc, a.R,
                       a.Z, a.ctl, a.partials);
    return hipGetLastError();
}

hipError_t launch_accept(hipStream_t s, const MapArgs &a, int ntrial)
{
    const float *l = a.lam;
#define ACC_ARGS a.g, a.P, (const T *)a.X, a.b1, a.Y, a.w, l[0], l[1], l[2], l[3], a.D, a.P0, a.P1, ntrial, a.ctl, a.partials
    if (a.dtype == DT_F32) {
        using T = float;
        hipLaunchKernelGGL(k_accept<T>, tiles(a.g), dim3(BLOCK), 0, s, ACC_ARGS);
    } else if (a.dtype == DT_F16) {
        using T = F16;
        hipLaunchKernelGGL(k_accept<T>, tiles(a.g), dim3(BLOCK), 0, s, ACC_ARGS);
    } else {
        using T = BF16;
        hipLaunchKernelGGL(k_accept<T>, tiles(a.g), dim3(BLOCK), 0, s, ACC_ARGS);
    }
#undef ACC_ARGS
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
    hipLaunchKernelGGL(k_weights, tiles(a.g), dim3(BLOCK), 0, s, a.g, a.Y, l[0], l[1], l[2], l[3], a.eps,
                       prior_on, a.w, a.partials);
    return hipGetLastError();
}

hipError_t launch_final(hipStream_t s, const MapArgs &a, float *var, float *mom)
{
    const float *l = a.lam;
#define FIN_ARGS a.g, a.P, (const T *)a.X, a.b1, a.Y, a.w, l[0], l[1], l[2], l[3], a.loading, var, mom, a.partials
    if (a.dtype == DT_F32) {
        using T = float;
        hipLaunchKernelGGL(k_final<T>, tiles(a.g), dim3(BLOCK), 0, s, FIN_ARGS);
    } else if (a.dtype == DT_F16) {
        using T = F16;
        hipLaunchKernelGGL(k_final<T>, tiles(a.g), dim3(BLOCK), 0, s, FIN_ARGS);
    } else {
        using T = BF16;
        hipLaunchKernelGGL(k_final<T>, tiles(a.g), dim3(BLOCK), 0, s, FIN_ARGS);
    }
#undef FIN_ARGS
    return hipGetLastError();
}

hipError_t launch_fin(hipStream_t s, const MapArgs &a, int stage, int arg, double cg_stop_rel, int ntrial,
                      int accept_off)
{
    int nblk = (int)((int64_t)a.g.gx * a.g.gy * a.g.nz);
    hipLaunchKernelGGL(k_fin, dim3(1), dim3(BLOCK), 0, s, stage, arg, nblk, a.partials, a.ctl, a.trace,
                       cg_stop_rel, ntrial, accept_off);
    return hipGetLastError();
}

}  // namespace mpm
