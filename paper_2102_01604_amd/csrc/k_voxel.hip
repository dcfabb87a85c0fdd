// k_voxel.hip -- voxelwise kernels of libmpm: forward model, per-image means,
// the maximum-likelihood fit (SPGR-ML) and a fixed-order row reduction.
#include <algorithm>

#include "mpm_stream.h"
#include "mpm_voxelwise.h"

namespace mpm {

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_fill_maps(float *maps, int64_t N, float y0, float y1,
                                                     float y2, float y3)
{
    int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= N) return;
    maps[n] = y0;
    maps[N + n] = y1;
    maps[2 * N + n] = y2;
    maps[3 * N + n] = y3;
}

hipError_t launch_fill_maps(const LaunchCtx &c, float *maps, int64_t N, const float y0[4])
{
    int nb = (int)((N + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_fill_maps, dim3(nb), dim3(BLOCK), 0, c.stream, maps, N, y0[0], y0[1], y0[2],
                       y0[3]);
    return hipGetLastError();
}

__global__ __launch_bounds__(BLOCK) void k_fill(float *p, int64_t n, float v)
{
    int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill(const LaunchCtx &c, float *p, int64_t n, float v)
{
    if (n <= 0) return hipSuccess;
    int nb = (int)((n + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_fill, dim3(nb), dim3(BLOCK), 0, c.stream, p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// forward model: out[i][n] = s_i(y_n) + sigma_i * noise[i][n]
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_simulate(DevProto P, const float *__restrict__ maps,
                                                    const float *__restrict__ b1,
                                                    const float *__restrict__ noise, T *__restrict__ out,
                                                    int64_t N)
{
    int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= N) return;
    float y[4] = {maps[n], maps[N + n], maps[2 * N + n], maps[3 * N + n]};
    float b = b1 ? b1[n] : 1.0f;
    Params p = decode(y);
    for (int c = 0; c < P.C; c++) {
        ContrastK K = contrast_factors(p, P.tr[c], make_angle(P.flip[c] * b), P.mt[c]);
        for (int i = P.first[c]; i < P.first[c + 1]; i++) {
            float s = K.s0 * __expf(-p.r2 * P.te[i]);
            if (noise) s += rsqrtf(P.wgt[i]) * noise[(int64_t)i * N + n];
            store_echo(out + (int64_t)i * N + n, s);
        }
    }
}

hipError_t launch_simulate(const LaunchCtx &c, const DevProto &P, const float *maps, const float *b1,
                           const float *noise, int dtype, void *out, int64_t N)
{
    int nb = (int)((N + BLOCK - 1) / BLOCK);
    if (dtype == DT_F32)
        hipLaunchKernelGGL(k_simulate<float>, dim3(nb), dim3(BLOCK), 0, c.stream, P, maps, b1, noise,
                           (float *)out, N);
    else if (dtype == DT_F16)
        hipLaunchKernelGGL(k_simulate<F16>, dim3(nb), dim3(BLOCK), 0, c.stream, P, maps, b1, noise,
                           (F16 *)out, N);
    else
        hipLaunchKernelGGL(k_simulate<BF16>, dim3(nb), dim3(BLOCK), 0, c.stream, P, maps, b1, noise,
                           (BF16 *)out, N);
    return hipGetLastError();
}

// forward model with a protocol per voxel (tr, flip [C][N], te [I][N]); a
// voxel whose protocol is invalid gets NaN
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_simulate_pv(DevProto P, PVArrays A, const float *__restrict__ maps,
                                                       const float *__restrict__ noise, T *__restrict__ out,
                                                       int64_t N)
{
    int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= N) return;
    float y[4] = {maps[n], maps[N + n], maps[2 * N + n], maps[3 * N + n]};
    Params p = decode(y);
    bool ok = true;
    for (int c = 0; c < P.C; c++) ok = ok && pv_valid(A.tr[(int64_t)c * N + n], A.flip[(int64_t)c * N + n]);
    for (int i = 0; i < P.I; i++) {
        const float t = A.te[(int64_t)i * N + n];
        ok = ok && t >= 0.0f && t < INFINITY;
    }
    for (int c = 0; c < P.C; c++) {
        ContrastK K = contrast_factors(p, A.tr[(int64_t)c * N + n], make_angle(A.flip[(int64_t)c * N + n]), P.mt[c]);
        for (int i = P.first[c]; i < P.first[c + 1]; i++) {
            float s = K.s0 * __expf(-p.r2 * A.te[(int64_t)i * N + n]);
            if (noise) s += rsqrtf(P.wgt[i]) * noise[(int64_t)i * N + n];
            store_echo(out + (int64_t)i * N + n, ok ? s : NAN);
        }
    }
}

hipError_t launch_simulate_pv(const LaunchCtx &c, const DevProto &P, const PVArrays &A, const float *maps,
                              const float *noise, int dtype, void *out, int64_t N)
{
    int nb = (int)((N + BLOCK - 1) / BLOCK);
    if (dtype == DT_F32)
        hipLaunchKernelGGL(k_simulate_pv<float>, dim3(nb), dim3(BLOCK), 0, c.stream, P, A, maps, noise, (float *)out,
                           N);
    else if (dtype == DT_F16)
        hipLaunchKernelGGL(k_simulate_pv<F16>, dim3(nb), dim3(BLOCK), 0, c.stream, P, A, maps, noise, (F16 *)out, N);
    else
        hipLaunchKernelGGL(k_simulate_pv<BF16>, dim3(nb), dim3(BLOCK), 0, c.stream, P, A, maps, noise, (BF16 *)out,
                           N);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-image sums (for the default initialisation) in one streaming pass over
// the echoes: grid (nblk, I + 1).  Workgroup row i < I reads image i once and
// writes partial row i (sum of its finite values) and row I + i (their count);
// row I reads b1 and writes row 2I (its sum).  Non-finite echoes are missing
// observations.  Every partial is an FP64 sum in a fixed order.
// ---------------------------------------------------------------------------
int echo_sums_blocks(int64_t N)
{
    const int64_t per = (int64_t)BLOCK * 64;  // values per workgroup and pass
    return (int)std::min<int64_t>(std::max<int64_t>((N + per - 1) / per, 1), 128);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_echo_sums(int I, const T *__restrict__ X,
                                                     const float *__restrict__ b1, int64_t N,
                                                     double *__restrict__ partials)
{
    __shared__ double lds[2][NWAVE];
    const int row = blockIdx.y;
    double v[2] = {0.0, 0.0};
    if (row < I) {
        for_each_value(X + (int64_t)row * N, N, [&](float x) {
            if (fabsf(x) < INFINITY) {
                v[0] += (double)x;
                v[1] += 1.0;
            }
        });
    } else if (b1) {
        for_each_value(b1, N, [&](float x) { v[0] += (double)x; });
    } else if (blockIdx.x == 0 && threadIdx.x == 0) {
        v[0] = (double)N;  // b1 = 1 everywhere
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        const int64_t nb = gridDim.x;
        if (row < I) {
            partials[(int64_t)row * nb + blockIdx.x] = v[0];
            partials[(int64_t)(I + row) * nb + blockIdx.x] = v[1];
        } else {
            partials[(int64_t)2 * I * nb + blockIdx.x] = v[0];
        }
    }
}

hipError_t launch_echo_sums(const LaunchCtx &c, const DevProto &P, int dtype, const void *X,
                            const float *b1, int64_t N, double *partials, int nblk)
{
    dim3 g(nblk, P.I + 1);
    if (dtype == DT_F32)
        hipLaunchKernelGGL(k_echo_sums<float>, g, dim3(BLOCK), 0, c.stream, P.I, (const float *)X, b1, N,
                           partials);
    else if (dtype == DT_F16)
        hipLaunchKernelGGL(k_echo_sums<F16>, g, dim3(BLOCK), 0, c.stream, P.I, (const F16 *)X, b1, N,
                           partials);
    else
        hipLaunchKernelGGL(k_echo_sums<BF16>, g, dim3(BLOCK), 0, c.stream, P.I, (const BF16 *)X, b1, N,
                           partials);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reduced-precision storage with per-image offsets: dst = round(src - off_i);
// counts finite inputs whose stored difference is not finite (overflow)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_pack_echoes(const float *__restrict__ src, T *__restrict__ dst, int64_t N,
                                                       EchoOffsets off, unsigned int *__restrict__ overflow)
{
    const int i = blockIdx.y;
    const float o = off.v[i];
    const float *s = src + (int64_t)i * N;
    T *d = dst + (int64_t)i * N;
    unsigned int bad = 0;
    for (int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x; n < N; n += (int64_t)gridDim.x * BLOCK) {
        const float x = s[n];
        store_echo(d + n, x - o);
        const float back = load_echo(d + n);
        bad += (fabsf(x) < INFINITY && !(fabsf(back) < INFINITY)) ? 1u : 0u;
    }
    if (bad) atomicAdd(overflow, bad);
}

hipError_t launch_pack_echoes(const LaunchCtx &c, int I, int64_t N, const float *src, int dtype, void *dst,
                              const EchoOffsets &off, unsigned int *overflow)
{
    const int64_t want = (N + BLOCK - 1) / BLOCK;
    dim3 g((unsigned)(want < 1024 ? want : 1024), (unsigned)I);
    if (dtype == DT_F16)
        hipLaunchKernelGGL(k_pack_echoes<F16>, g, dim3(BLOCK), 0, c.stream, src, (F16 *)dst, N, off, overflow);
    else
        hipLaunchKernelGGL(k_pack_echoes<BF16>, g, dim3(BLOCK), 0, c.stream, src, (BF16 *)dst, N, off, overflow);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fixed-order reduction of rows: one workgroup per row
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_reduce_rows(const double *__restrict__ in, int ncols,
                                                       double *__restrict__ out)
{
    __shared__ double lds[1][NWAVE];
    const double *row = in + (int64_t)blockIdx.x * ncols;
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < ncols; b += BLOCK) v[0] += row[b];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = v[0];
}

hipError_t launch_reduce_rows(const LaunchCtx &c, const double *in, int nrows, int ncols, double *out)
{
    hipLaunchKernelGGL(k_reduce_rows, dim3(nrows), dim3(BLOCK), 0, c.stream, in, ncols, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ML fit (paper Sec. 2.3-2.4): each thread owns one voxel and runs all n_gn
// Newton-like steps y <- y - P~^{-1} g.  Protocols of at most CM contrasts x
// EM echoes keep the echoes in registers; CM = EM = 0 re-reads them from
// memory at every step (any protocol).
// ---------------------------------------------------------------------------
int ml_fit_blocks(int64_t N) { return (int)((N + BLOCK - 1) / BLOCK); }

// Waves per SIMD asked of the compiler: with up to 32 echo slots the kernel
// fits in 168 registers (3 waves) with 6 spilled (measured on the whole-brain
// volume, 4 x 8 slots: 6.0 ms at 2 waves, 5.0 ms at 3); the larger register
// shapes would spill 46-101 and keep the compiler's choice.
template <int CM, int EM>
constexpr int ml_min_waves() { return CM * EM > 0 && CM * EM <= 32 ? 3 : 1; }

template <typename T, int CM, int EM, bool PLUS>
__global__ __launch_bounds__(BLOCK, (ml_min_waves<CM, EM>())) void k_ml_fit(typename VoxelEchoes<T, CM, EM>::Proto P, const T *__restrict__ X,
                                                  const float *__restrict__ b1, const float *__restrict__ bm,
                                                  float *__restrict__ maps,
                                                  int64_t N, int n_gn, int loading,
                                                  double *__restrict__ partials)
{
    __shared__ double lds[1][NWAVE];
    const int nblk = gridDim.x;
    int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool active = n < N;
    const int64_t nn = active ? n : 0;

    const auto K = VoxelEchoes<T, CM, EM>::stage(P);
    VoxelEchoes<T, CM, EM> ve;
    ve.load(P, X, N, nn, b1 ? b1[nn] : 1.0f, bm ? bm[nn] : 1.0f);
    float y[4] = {maps[nn], maps[N + nn], maps[2 * N + nn], maps[3 * N + nn]};

    float prev_nll = 0.0f;
    double cnt_inc = 0.0, degen = 0.0;
    for (int it = 0; it <= n_gn; it++) {
        const bool last = (it == n_gn);
        float g[4], H[10];
        const float nll = ve.template lik<PLUS>(P, K, y, loading, !last, g, H);
        if (it > 0 && nll > prev_nll * (1.0f + 1e-5f)) cnt_inc += 1.0;
        prev_nll = nll;
        double v[1] = {active ? (double)nll : 0.0};
        block_sum<1>(v, lds);
        if (threadIdx.x == 0) partials[(int64_t)it * nblk + blockIdx.x] = v[0];
        __syncthreads();
        if (last) break;
        float step[4];
        bool bad = solve_sym4(H, g, step);
        degen = bad ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < 4; k++) y[k] -= step[k];
    }
    double fin = 0.0;
#pragma unroll
    for (int k = 0; k < 4; k++) fin += (fabsf(y[k]) < INFINITY) ? 0.0 : 1.0;
    double st[3] = {active ? (n_gn > 0 ? degen : 0.0) : 0.0, (active && fin > 0.0) ? 1.0 : 0.0,
                    active ? cnt_inc : 0.0};
    __shared__ double lds3[3][NWAVE];
    block_sum<3>(st, lds3);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; k++) partials[(int64_t)(n_gn + 1 + k) * nblk + blockIdx.x] = st[k];
    if (active) {
        maps[n] = y[0];
        maps[N + n] = y[1];
        maps[2 * N + n] = y[2];
        maps[3 * N + n] = y[3];
    }
}

template <typename T, bool PLUS>
static hipError_t ml_launch(const LaunchCtx &c, const DevProto &P, const T *X, const float *b1, const float *bm,
                              float *maps, int64_t N, int n_gn, int loading, double *partials, int nblk)
{
    dim3 g(nblk), b(BLOCK);
    const int shape = echo_shape(P);
    if (shape == 1)
        hipLaunchKernelGGL((k_ml_fit<T, 4, 8, PLUS>), g, b, 0, c.stream, (ProtoArg<T, 4, 8>::make(P, X, N)), X, b1, bm,
                           maps, N, n_gn, loading, partials);
    else if (shape == 2)
        hipLaunchKernelGGL((k_ml_fit<T, 4, 16, PLUS>), g, b, 0, c.stream, (ProtoArg<T, 4, 16>::make(P, X, N)),
                           X, b1, bm,
                           maps, N, n_gn, loading, partials);
    else if (shape == 3)
        hipLaunchKernelGGL((k_ml_fit<T, 8, 8, PLUS>), g, b, 0, c.stream, (ProtoArg<T, 8, 8>::make(P, X, N)), X, b1, bm,
                           maps, N, n_gn, loading, partials);
    else
        hipLaunchKernelGGL((k_ml_fit<T, 0, 0, PLUS>), g, b, 0, c.stream, (ProtoArg<T, 0, 0>::make(P, X, N)), X, b1, bm,
                           maps, N, n_gn, loading, partials);
    return hipGetLastError();
}

template <typename T>
static hipError_t ml_dispatch(const LaunchCtx &c, const DevProto &P, const T *X, const float *b1, const float *bm,
                              float *maps, int64_t N, int n_gn, int loading, double *partials, int nblk)
{
    return loading == 2 ? ml_launch<T, true>(c, P, X, b1, bm, maps, N, n_gn, loading, partials, nblk)
                        : ml_launch<T, false>(c, P, X, b1, bm, maps, N, n_gn, loading, partials, nblk);
}

hipError_t launch_ml_fit(const LaunchCtx &c, const DevProto &P, int dtype, const void *X,
                         const float *b1, const float *bm, float *maps, int64_t N, int n_gn, int loading,
                         double *partials, int nblk)
{
    if (dtype == DT_F32)
        return ml_dispatch(c, P, (const float *)X, b1, bm, maps, N, n_gn, loading, partials, nblk);
    if (dtype == DT_F16)
        return ml_dispatch(c, P, (const F16 *)X, b1, bm, maps, N, n_gn, loading, partials, nblk);
    return ml_dispatch(c, P, (const BF16 *)X, b1, bm, maps, N, n_gn, loading, partials, nblk);
}

// ---------------------------------------------------------------------------
// ML fit with a protocol per voxel (paper Sec. 3.1): the same Newton-like
// steps per thread; per voxel the count of steps after which its NLL rose
// (more than 1e-5 relative, or finite to non-finite) and the final NLL.
// Partials per workgroup: final NLL, degenerate, non-finite, rises.  BASIS
// selects the parameters the steps act on: 0 the log/logit ones, 1 the rates
// (A, R1, R2*, MTsat), 2 the times (A, T1, T2*, MTsat), kept in their domain
// by basis_step.
// ---------------------------------------------------------------------------
template <typename T, int CM, int EM, bool PLUS, int BASIS>
__global__ __launch_bounds__(BLOCK) void k_ml_fit_pv(DevProto P, PVArrays A, const T *__restrict__ X,
                                                     float *__restrict__ maps, int64_t N, int n_gn, int loading,
                                                     int32_t *__restrict__ incr, float *__restrict__ nll_out,
                                                     double *__restrict__ partials)
{
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool active = n < N;
    const int64_t nn = active ? n : 0;
    const auto W = VoxelEchoesPV<T, CM, EM>::stage(P);
    VoxelEchoesPV<T, CM, EM> ve;
    ve.load(P, A, X, N, nn);
    float y[4] = {maps[nn], maps[N + nn], maps[2 * N + nn], maps[3 * N + nn]};
    float prev = 0.0f, cur = NAN;
    int cnt = 0;
    bool degen = false;
    if (ve.ok) {
        for (int it = 0; it <= n_gn; it++) {
            const bool last = (it == n_gn);
            float g[4], H[10];
            if (BASIS == 0)
                cur = ve.template lik<PLUS>(P, W, y, loading, !last, g, H);
            else
                cur = ve.template lik_basis<PLUS, BASIS>(P, W, y, loading, !last, g, H);
            if (it > 0 && (cur > prev * (1.0f + 1e-5f) || (fabsf(prev) < INFINITY && !(fabsf(cur) < INFINITY))))
                cnt++;
            prev = cur;
            if (last) break;
            float step[4];
            degen = solve_sym4(H, g, step);
#pragma unroll
            for (int k = 0; k < 4; k++) y[k] = BASIS == 0 ? y[k] - step[k] : basis_step(k, y[k], step[k]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; k++) y[k] = NAN;
    }
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 4; k++) fin = fin && fabsf(y[k]) < INFINITY;
    double st[4] = {active ? (double)cur : 0.0, (active && n_gn > 0 && degen) ? 1.0 : 0.0,
                    (active && !fin) ? 1.0 : 0.0, active ? (double)cnt : 0.0};
    __shared__ double lds[4][NWAVE];
    block_sum<4>(st, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; k++) partials[(int64_t)k * gridDim.x + blockIdx.x] = st[k];
    if (active) {
        maps[n] = y[0];
        maps[N + n] = y[1];
        maps[2 * N + n] = y[2];
        maps[3 * N + n] = y[3];
        if (incr) incr[n] = cnt;
        if (nll_out) nll_out[n] = cur;
    }
}

template <typename T, bool PLUS, int BASIS>
static hipError_t ml_pv_launch(const LaunchCtx &c, const DevProto &P, const PVArrays &A, const T *X, float *maps,
                               int64_t N, int n_gn, int loading, int32_t *incr, float *nll, double *partials)
{
    dim3 g(ml_fit_blocks(N)), b(BLOCK);
    int emax = 0;
    for (int k = 0; k < P.C; k++) emax = std::max(emax, P.first[k + 1] - P.first[k]);
#define PV_LAUNCH(CM, EM)                                                                                          \
    hipLaunchKernelGGL((k_ml_fit_pv<T, CM, EM, PLUS, BASIS>), g, b, 0, c.stream, P, A, X, maps, N, n_gn, loading, \
                       incr, nll, partials)
    if (P.C <= 4 && emax <= 5)
        PV_LAUNCH(4, 5);
    else if (P.C <= 4 && emax <= 6)
        PV_LAUNCH(4, 6);
    else if (P.C <= 4 && emax <= 8)
        PV_LAUNCH(4, 8);
    else if (P.C <= 8 && emax <= 8)
        PV_LAUNCH(8, 8);
    else
        PV_LAUNCH(0, 0);
#undef PV_LAUNCH
    return hipGetLastError();
}

template <typename T, int BASIS>
static hipError_t ml_pv_loading(const LaunchCtx &c, const DevProto &P, const PVArrays &A, const T *X, float *maps,
                                int64_t N, int n_gn, int loading, int32_t *incr, float *nll, double *partials)
{
    return loading == 2 ? ml_pv_launch<T, true, BASIS>(c, P, A, X, maps, N, n_gn, loading, incr, nll, partials)
                        : ml_pv_launch<T, false, BASIS>(c, P, A, X, maps, N, n_gn, loading, incr, nll, partials);
}

template <typename T>
static hipError_t ml_pv_dispatch(const LaunchCtx &c, const DevProto &P, const PVArrays &A, const T *X, float *maps,
                                 int64_t N, int n_gn, int loading, int basis, int32_t *incr, float *nll,
                                 double *partials)
{
    if (basis == 1) return ml_pv_loading<T, 1>(c, P, A, X, maps, N, n_gn, loading, incr, nll, partials);
    if (basis == 2) return ml_pv_loading<T, 2>(c, P, A, X, maps, N, n_gn, loading, incr, nll, partials);
    return ml_pv_loading<T, 0>(c, P, A, X, maps, N, n_gn, loading, incr, nll, partials);
}

hipError_t launch_ml_fit_pv(const LaunchCtx &c, const DevProto &P, const PVArrays &A, int dtype, const void *X,
                            float *maps, int64_t N, int n_gn, int loading, int basis, int32_t *incr, float *nll,
                            double *partials)
{
    if (dtype == DT_F32)
        return ml_pv_dispatch(c, P, A, (const float *)X, maps, N, n_gn, loading, basis, incr, nll, partials);
    if (dtype == DT_F16)
        return ml_pv_dispatch(c, P, A, (const F16 *)X, maps, N, n_gn, loading, basis, incr, nll, partials);
    return ml_pv_dispatch(c, P, A, (const BF16 *)X, maps, N, n_gn, loading, basis, incr, nll, partials);
}

}  // namespace mpm
