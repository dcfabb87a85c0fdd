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
};

hipError_t launch_simulate_pv(const LaunchCtx &c, const DevProto &P, const PVArrays &A, const float *maps,
                              const float *noise, int dtype, void *out, int64_t N);
// ML fit with a protocol per voxel (tr, flip [C][N], te [I][N]); partials
// [4][ml_fit_blocks(N)]: final NLL, degenerate, non-finite, NLL rises.
hipError_t launch_ml_fit_pv(const LaunchCtx &c, const DevProto &P, const PVArrays &A, int dtype, const void *X,
                            float *maps, int64_t N, int n_gn, int loading, int32_t *incr, float *nll,
                            double *partials);

}  // namespace mpm
