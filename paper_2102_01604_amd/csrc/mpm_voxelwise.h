// mpm_voxelwise.h -- the ML fit and forward model with a protocol per voxel
// (the convergence experiment of paper Sec. 3.1): device building blocks and
// the launchers of k_voxel.hip.
#pragma once

#include "mpm_kernels.h"

namespace mpm {

// ---------------------------------------------------------------------------
// Per-voxel protocols (the convergence experiment of Sec. 3.1): the contrast /
// echo structure, MT flags and weights of DevProto are shared; TR and flip
// angle per contrast and TE per echo are arrays over voxels (tr, flip [C][N],
// te [I][N]; DevProto's tr, flip, te are unused).  With CM, EM > 0 the
// voxel's echoes, echo times, TRs and flip-angle terms are held in registers
// (slots past a contrast's last echo repeat it with weight 0, so the echo
// loops carry no tests); CM = EM = 0 reads them at every evaluation.  The
// per-echo arithmetic is the shared-protocol one.
// ---------------------------------------------------------------------------
struct PVArrays {
    const float *tr, *flip, *te;
};

__device__ __forceinline__ bool pv_valid(float tr, float flip)
{
    return tr > 0.0f && tr < INFINITY && flip > 0.0f && flip < 3.14159265358979f;
}

typedef const volatile __attribute__((address_space(3))) float lds_f32;

// ---------------------------------------------------------------------------
// Rate and time representations (the representation comparison of Sec. 3.1):
// the steps act on th = (A, R1, R2*, MTsat) (BASIS 1) or (A, T1, T2*, MTsat)
// (BASIS 2, R = 1/T).  With E = exp(-R1 TR), q = 1 - delta, w = q cos(alpha),
// D = 1 - w E the signal is s = A F G, F = sin(alpha) q (1 - E) / D,
// G = exp(-R2* TE), and
//   dF/dR1 = TR E sin(alpha) q (1 - w) / D^2,
//   d2F/dR1^2 = -TR (dF/dR1) (1 + w E) / D,        1 + w E = 2 - D,
//   dF/ddelta = -sin(alpha) (1 - E) / D^2,
//   d2F/ddelta^2 = 2 sin(alpha) (1 - E) cos(alpha) E / D^3,
//   d2F/dR1 ddelta = TR E sin(alpha) (w (1 - E) - (1 - w)) / D^3,
// with 1 - E, 1 - w and D formed without cancellation as in
// contrast_factors.  A parameter u with R = rho(u) brings the factors
// j = rho'(u) and jp = rho''(u): 1 and 0 (rate), -R^2 and 2 R^3 (time).
// Per echo every derivative is G times per-contrast constants times a power of
// TE, so one contrast's echoes reduce to the sums of BasisAcc.
// ---------------------------------------------------------------------------
struct BasisK {
    float F, Fu, Fuu, Fd, Fud, Fdd;  // F and its derivatives in th[1] and delta
};

__device__ __forceinline__ BasisK basis_factors(float r1, float j1, float j1p, float dl_, float tr, const Angle &an,
                                                int mt)
{
    const float dl = mt ? dl_ : 0.0f;
    const float ome = -expm1f(-r1 * tr);   // 1 - E
    const float e1 = 1.0f - ome;           // E
    const float omw = an.omc + dl * an.ca;  // 1 - w
    const float D = ome + e1 * omw;         // 1 - w E
    const float iD = 1.0f / D;
    const float t = tr * e1 * an.sa * iD * iD;  // TR E sin(alpha) / D^2
    const float F1 = t * (1.0f - dl) * omw;
    const float F11 = -tr * F1 * (2.0f - D) * iD;
    BasisK k;
    k.F = an.sa * (1.0f - dl) * ome * iD;
    k.Fu = F1 * j1;
    k.Fuu = F11 * j1 * j1 + F1 * j1p;
    k.Fd = mt ? -an.sa * ome * iD * iD : 0.0f;
    k.Fdd = mt ? 2.0f * an.sa * ome * an.ca * e1 * iD * iD * iD : 0.0f;
    k.Fud = mt ? t * ((1.0f - omw) * ome - omw) * iD * j1 : 0.0f;
    return k;
}

// Sums over one contrast's echoes (weights w = 1/sigma^2, residual r = s - x):
//   R0 = sum w r G, R1 = .. TE;  A0 = sum w G^2, A1 = .. TE, A2 = .. TE^2;
//   B0 = sum w |r| G, BT = .. TE, BQ = sum w |r| G TE |TE j2^2 - j2p|
// (BQ carries |d2G/du2^2| / G, whose sign can change with TE in the time
// basis).  A non-finite x is a missing observation and adds exactly 0.
struct BasisAcc {
    float R0 = 0.f, R1 = 0.f, A0 = 0.f, A1 = 0.f, A2 = 0.f, B0 = 0.f, BT = 0.f, BQ = 0.f, L = 0.f;
    __device__ __forceinline__ void add(float G, float s, float x, float te, float tq, float w)
    {
        const bool ok = fabsf(x) < INFINITY;
        const float wv = ok ? w : 0.0f;
        const float res = s - (ok ? x : 0.0f);
        const float wr = wv * res;
        const float wrg = wr * G;
        R0 += wrg;
        R1 = fmaf(wrg, te, R1);
        const float wg2 = wv * G * G;
        A0 += wg2;
        A1 = fmaf(wg2, te, A1);
        A2 = fmaf(wg2 * te, te, A2);
        const float awrg = fabsf(wrg);
        B0 += awrg;
        BT = fmaf(awrg, te, BT);
        BQ = fmaf(awrg, tq, BQ);
        L = fmaf(wr, res, L);
    }
};

// One contrast's share of g and of the loaded Hessian (H packed upper
// triangle 00 01 02 03 11 12 13 22 23 33).  grad s = G (v0, v1, TE v2, v3)
// with v = (F, A Fu, -A F j2, A Fd).  Loading: PLUS the absolute row sums of
// the second-derivative matrix, else 0 = |diag|, 1 = none.
template <bool PLUS>
__device__ __forceinline__ void basis_contrast(const BasisAcc &e, const BasisK &K, float a, float j2, int loading,
                                               float g[4], float H[10])
{
    const float v0 = K.F, v1 = a * K.Fu, v2 = -a * K.F * j2, v3 = a * K.Fd;
    g[0] += v0 * e.R0;
    g[1] += v1 * e.R0;
    g[2] += v2 * e.R1;
    g[3] += v3 * e.R0;
    H[0] += v0 * v0 * e.A0;
    H[1] += v0 * v1 * e.A0;
    H[2] += v0 * v2 * e.A1;
    H[3] += v0 * v3 * e.A0;
    H[4] += v1 * v1 * e.A0;
    H[5] += v1 * v2 * e.A1;
    H[6] += v1 * v3 * e.A0;
    H[7] += v2 * v2 * e.A2;
    H[8] += v2 * v3 * e.A1;
    H[9] += v3 * v3 * e.A0;
    const float aF = fabsf(a * K.F), aFuu = fabsf(a * K.Fuu), aFud = fabsf(a * K.Fud), aFdd = fabsf(a * K.Fdd);
    if (PLUS) {
        const float fu = fabsf(K.Fu), fd = fabsf(K.Fd), aj = fabsf(j2);
        const float f2 = fabsf(K.F) * aj, w1 = fabsf(v1) * aj, w3 = fabsf(v3) * aj;
        H[0] += e.B0 * (fu + fd) + e.BT * f2;
        H[4] += e.B0 * (fu + aFuu + aFud) + e.BT * w1;
        H[7] += e.BT * (f2 + w1 + w3) + aF * e.BQ;
        H[9] += e.B0 * (fd + aFud + aFdd) + e.BT * w3;
    } else if (loading == 0) {
        H[4] += aFuu * e.B0;
        H[7] += aF * e.BQ;
        H[9] += aFdd * e.B0;
    }
}

// Rate values and chain factors of th[1], th[2] in basis BASIS.
template <int BASIS>
struct BasisRates {
    float r1, r2, j1, j1p, j2, j2p;
    __device__ __forceinline__ explicit BasisRates(const float th[4])
    {
        if (BASIS == 2) {
            r1 = 1.0f / th[1];
            r2 = 1.0f / th[2];
            j1 = -r1 * r1;
            j1p = -2.0f * r1 * j1;
            j2 = -r2 * r2;
            j2p = -2.0f * r2 * j2;
        } else {
            r1 = th[1];
            r2 = th[2];
            j1 = j2 = 1.0f;
            j1p = j2p = 0.0f;
        }
    }
};

// Newton-like update of one parameter in the rate / time basis: a step that
// would take A, R1 (T1) or R2* (T2*) to <= 0, or MTsat out of (0, 1), moves
// the parameter halfway to that boundary instead.
__device__ __forceinline__ float basis_step(int k, float u, float step)
{
    const float v = u - step;
    if (!(fabsf(v) < INFINITY)) return v;
    if (!(v > 0.0f)) return 0.5f * u;
    if (k == 3 && !(v < 1.0f)) return 0.5f * (1.0f + u);
    return v;
}

template <typename T, int CM, int EM>
struct VoxelEchoesPV {
    using Consts = lds_f32 *;
    float x[CM][EM], te[CM][EM], tr[CM];
    Angle an[CM];
    bool ok;

    // The weight 1/sigma^2 of each slot (c, e) in LDS, read back at each use
    // (held in scalar registers they spill).  Every thread calls this first;
    // it ends with a barrier.
    static __device__ __forceinline__ Consts stage(const DevProto &P)
    {
        __shared__ float tab[CM * EM];
        if (threadIdx.x == 0) {
            for (int c = 0; c < CM; c++)
                for (int e = 0; e < EM; e++)
                    tab[c * EM + e] = c < P.C && e < P.first[c + 1] - P.first[c] ? P.wgt[P.first[c] + e] : 0.0f;
        }
        __syncthreads();
        return (lds_f32 *)tab;
    }

    __device__ __forceinline__ void load(const DevProto &P, const PVArrays &A, const T *__restrict__ X, int64_t N,
                                         int64_t n)
    {
        ok = true;
#pragma unroll
        for (int c = 0; c < CM; c++) {
            if (c < P.C) {
                const int ne = P.first[c + 1] - P.first[c];
                tr[c] = A.tr[(int64_t)c * N + n];
                const float f = A.flip[(int64_t)c * N + n];
                ok = ok && pv_valid(tr[c], f);
                an[c] = make_angle(f);
#pragma unroll
                for (int e = 0; e < EM; e++) {
                    // slots past the last echo repeat it (weight 0 in the table)
                    const int64_t i = P.first[c] + (e < ne ? e : ne - 1);
                    x[c][e] = load_echo(X + i * N + n);
                    te[c][e] = A.te[i * N + n];
                    ok = ok && te[c][e] >= 0.0f && te[c][e] < INFINITY;
                }
            }
        }
    }

    template <bool PLUS>
    __device__ __forceinline__ float lik(const DevProto &P, Consts W, const float y[4], int loading, bool grad,
                                         float g[4], float H[10]) const
    {
        const Params p = decode(y);
        const float k2 = -p.r2 * 1.4426950f;  // exp(-r2 te) = 2^(k2 te)
        float nll = 0.f;
#pragma unroll
        for (int k = 0; k < 4; k++) g[k] = 0.f;
#pragma unroll
        for (int k = 0; k < 10; k++) H[k] = 0.f;
#pragma unroll
        for (int c = 0; c < CM; c++) {
            if (c < P.C) {
                const ContrastK F = contrast_factors(p, tr[c], an[c], P.mt[c]);
                EchoAcc acc;
#pragma unroll
                for (int e = 0; e < EM; e++) {
                    const float t = te[c][e];
                    acc.add(F.s0 * __builtin_amdgcn_exp2f(k2 * t), x[c][e], t, t * t, W[c * EM + e], p.r2);
                }
                nll += 0.5f * acc.L;
                if (grad) accumulate_contrast<PLUS>(acc, F, p.r2, loading, g, H);
            }
        }
        return nll;
    }

    // The same in the rate (BASIS 1) or time (BASIS 2) representation.
    template <bool PLUS, int BASIS>
    __device__ __forceinline__ float lik_basis(const DevProto &P, Consts W, const float th[4], int loading,
                                               bool grad, float g[4], float H[10]) const
    {
        const BasisRates<BASIS> b(th);
        const float k2 = -b.r2 * 1.4426950f, j2sq = b.j2 * b.j2;
        float nll = 0.f;
#pragma unroll
        for (int k = 0; k < 4; k++) g[k] = 0.f;
#pragma unroll
        for (int k = 0; k < 10; k++) H[k] = 0.f;
#pragma unroll
        for (int c = 0; c < CM; c++) {
            if (c < P.C) {
                const BasisK K = basis_factors(b.r1, b.j1, b.j1p, th[3], tr[c], an[c], P.mt[c]);
                const float s0 = th[0] * K.F;
                BasisAcc acc;
#pragma unroll
                for (int e = 0; e < EM; e++) {
                    const float t = te[c][e];
                    const float G = __builtin_amdgcn_exp2f(k2 * t);
                    acc.add(G, s0 * G, x[c][e], t, t * fabsf(fmaf(t, j2sq, -b.j2p)), W[c * EM + e]);
                }
                nll += 0.5f * acc.L;
                if (grad) basis_contrast<PLUS>(acc, K, th[0], b.j2, loading, g, H);
            }
        }
        return nll;
    }
};

template <typename T>
struct VoxelEchoesPV<T, 0, 0> {
    using Consts = const void *;
    const T *__restrict__ X;
    PVArrays A;
    int64_t N, n;
    bool ok;

    static __device__ __forceinline__ Consts stage(const DevProto &) { return nullptr; }

    __device__ __forceinline__ void load(const DevProto &P, const PVArrays &A_, const T *__restrict__ X_, int64_t N_,
                                         int64_t n_)
    {
        X = X_;
        A = A_;
        N = N_;
        n = n_;
        ok = true;
        for (int c = 0; c < P.C; c++) ok = ok && pv_valid(A.tr[(int64_t)c * N + n], A.flip[(int64_t)c * N + n]);
        for (int i = 0; i < P.I; i++) {
            const float t = A.te[(int64_t)i * N + n];
            ok = ok && t >= 0.0f && t < INFINITY;
        }
    }

    template <bool PLUS>
    __device__ __forceinline__ float lik(const DevProto &P, Consts, const float y[4], int loading, bool grad,
                                         float g[4], float H[10]) const
    {
        const Params p = decode(y);
        const float k2 = -p.r2 * 1.4426950f;
        float nll = 0.f;
#pragma unroll
        for (int k = 0; k < 4; k++) g[k] = 0.f;
#pragma unroll
        for (int k = 0; k < 10; k++) H[k] = 0.f;
        for (int c = 0; c < P.C; c++) {
            const ContrastK K = contrast_factors(p, A.tr[(int64_t)c * N + n], make_angle(A.flip[(int64_t)c * N + n]),
                                                 P.mt[c]);
            EchoAcc acc;
            for (int i = P.first[c]; i < P.first[c + 1]; i++) {
                const float t = A.te[(int64_t)i * N + n];
                acc.add(K.s0 * __builtin_amdgcn_exp2f(k2 * t), load_echo(X + (int64_t)i * N + n), t, t * t, P.wgt[i],
                        p.r2);
            }
            nll += 0.5f * acc.L;
            if (grad) accumulate_contrast<PLUS>(acc, K, p.r2, loading, g, H);
        }
        return nll;
    }

    template <bool PLUS, int BASIS>
    __device__ __forceinline__ float lik_basis(const DevProto &P, Consts, const float th[4], int loading, bool grad,
                                               float g[4], float H[10]) const
    {
        const BasisRates<BASIS> b(th);
        const float k2 = -b.r2 * 1.4426950f, j2sq = b.j2 * b.j2;
        float nll = 0.f;
#pragma unroll
        for (int k = 0; k < 4; k++) g[k] = 0.f;
#pragma unroll
        for (int k = 0; k < 10; k++) H[k] = 0.f;
        for (int c = 0; c < P.C; c++) {
            const BasisK K = basis_factors(b.r1, b.j1, b.j1p, th[3], A.tr[(int64_t)c * N + n],
                                           make_angle(A.flip[(int64_t)c * N + n]), P.mt[c]);
            const float s0 = th[0] * K.F;
            BasisAcc acc;
            for (int i = P.first[c]; i < P.first[c + 1]; i++) {
                const float t = A.te[(int64_t)i * N + n];
                const float G = __builtin_amdgcn_exp2f(k2 * t);
                acc.add(G, s0 * G, load_echo(X + (int64_t)i * N + n), t, t * fabsf(fmaf(t, j2sq, -b.j2p)),
                        P.wgt[i]);
            }
            nll += 0.5f * acc.L;
            if (grad) basis_contrast<PLUS>(acc, K, th[0], b.j2, loading, g, H);
        }
        return nll;
    }
};

hipError_t launch_simulate_pv(const LaunchCtx &c, const DevProto &P, const PVArrays &A, const float *maps,
                              const float *noise, int dtype, void *out, int64_t N);
// ML fit with a protocol per voxel (tr, flip [C][N], te [I][N]); partials
// [4][ml_fit_blocks(N)]: final NLL, degenerate, non-finite, NLL rises.
// basis: 0 log/logit parameters, 1 rate, 2 time (maps in that basis).
hipError_t launch_ml_fit_pv(const LaunchCtx &c, const DevProto &P, const PVArrays &A, int dtype, const void *X,
                            float *maps, int64_t N, int n_gn, int loading, int basis, int32_t *incr, float *nll,
                            double *partials);

}  // namespace mpm
