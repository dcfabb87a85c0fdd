// mpm_device.h -- device-side building blocks of libmpm (gfx950).
//
// FP32 forms of the SPGR signal model and its derivatives (paper Sec. 2.1,
// Sec. 2.4), the Jacobi-scaled 4x4 solve with the degenerate-voxel rule, echo
// loads for FP32/FP16/BF16 storage and FP64 block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpm {

constexpr int MAXC = 8;
constexpr int MAXI = 64;
constexpr int BLOCK = 256;          // threads per workgroup (4 wave64)
constexpr int NWAVE = BLOCK / 64;

// Degenerate-voxel rule: a parameter whose Hessian diagonal is <= FROZEN_REL
// times the largest one takes no step; a Jacobi-scaled Cholesky pivot below
// PIVOT_MIN makes the whole voxel take no step.
constexpr float FROZEN_REL = 1e-30f;
constexpr float PIVOT_MIN = 1e-6f;

// Protocol constants, passed by value as a kernel argument.
struct DevProto {
    int C, I;
    int first[MAXC + 1];      // first image of each contrast
    float tr[MAXC];
    float flip[MAXC];
    int mt[MAXC];
    float te[MAXI];
    float wgt[MAXI];          // 1 / sigma_i^2
};

// ---------------------------------------------------------------------------
// echo storage
// ---------------------------------------------------------------------------
struct F16 { uint16_t v; };
struct BF16 { uint16_t v; };

__device__ __forceinline__ float load_echo(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float load_echo(const F16 *p)
{
    uint16_t b = __builtin_nontemporal_load(&p->v);
    _Float16 h;
    __builtin_memcpy(&h, &b, 2);
    return (float)h;
}
__device__ __forceinline__ float load_echo(const BF16 *p)
{
    uint32_t b = (uint32_t)__builtin_nontemporal_load(&p->v) << 16;
    float f;
    __builtin_memcpy(&f, &b, 4);
    return f;
}

__device__ __forceinline__ void store_echo(float *p, float v) { *p = v; }
__device__ __forceinline__ void store_echo(F16 *p, float v)
{
    _Float16 h = (_Float16)v;  // round to nearest even
    __builtin_memcpy(&p->v, &h, 2);
}
__device__ __forceinline__ void store_echo(BF16 *p, float v)
{
    uint32_t u;
    __builtin_memcpy(&u, &v, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) {
        p->v = (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));  // inf / quiet nan
        return;
    }
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    p->v = (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// signal model
// ---------------------------------------------------------------------------
struct Params {
    float a, r1, r2, dl;  // A, R1, R2*, MTsat
};

__device__ __forceinline__ Params decode(const float y[4])
{
    Params p;
    p.a = __expf(y[0]);
    p.r1 = __expf(y[1]);
    p.r2 = __expf(y[2]);
    p.dl = 1.0f / (1.0f + __expf(-y[3]));
    return p;
}

// Per-(voxel, contrast) factors of the signal and its log-parameter
// derivatives.  With E = exp(-r1 TR), omega = (1 - delta) cos(alpha):
//   s(TE)        = s0 * exp(-r2 TE)
//   ds/d log a   = s,            d2s = s
//   ds/d log r1  = phi * s,      d2s = kap * phi * s
//   ds/d log r2  = -TE r2 s,     d2s = (1 - TE r2)(-TE r2) s
//   ds/d logit d = psi * s,      d2s = mu * psi * s      (MT contrasts)
// 1 - E, 1 - omega, 1 - omega E and 1 - cos(alpha) E are formed without
// cancellation (expm1 and 2 sin^2(alpha/2)), which FP32 needs at TR = 25 ms.
struct ContrastK {
    float s0, phi, psi, kap, mu;
};

// Flip-angle terms of one (voxel, contrast), computed once per voxel.
struct Angle {
    float sa, ca, omc;  // sin(alpha), cos(alpha), 1 - cos(alpha) = 2 sin^2(alpha/2)
};

__device__ __forceinline__ Angle make_angle(float alpha)
{
    Angle a;
    sincosf(alpha, &a.sa, &a.ca);
    float sh = sinf(0.5f * alpha);
    a.omc = 2.0f * sh * sh;
    return a;
}

__device__ __forceinline__ ContrastK contrast_factors(const Params &p, float tr, const Angle &an, int mt)
{
    float dl = mt ? p.dl : 0.0f;
    float x = p.r1 * tr;
    float ome = -expm1f(-x);                    // 1 - E
    float e1 = 1.0f - ome;                      // E
    float one_m_omega = an.omc + dl * an.ca;    // 1 - (1 - delta) cos(alpha)
    float den = ome + e1 * one_m_omega;         // 1 - omega E
    float inv_den = 1.0f / den;
    ContrastK k;
    k.s0 = p.a * an.sa * (1.0f - dl) * ome * inv_den;
    k.phi = x * one_m_omega * e1 * inv_den / ome;
    k.kap = 1.0f - x * (2.0f - den) * inv_den;  // 1 + omega E = 2 - den
    k.psi = -dl * inv_den;
    k.mu = 2.0f * (1.0f - dl) * (ome + e1 * an.omc) * inv_den - 1.0f;
    return k;
}

// ---------------------------------------------------------------------------
// Per-voxel likelihood block for one contrast, factored over echoes.
//
// With v_i = (1, phi, -TE_i r2, psi) the gradient of s_i is s_i v_i, so
//   sum_i w res s v                = (R0, phi R0, -r2 R1, psi R0)
//   sum_i w s^2 v v^T              from A0 = sum w s^2, A1 = .. TE, A2 = .. TE^2
//   sum_i w |res| |d2 s_i| (diag)  = (B0, |kap phi| B0, r2 B2, |mu psi| B0)
// with B0 = sum w |res s|, B2 = sum w |res s| TE |1 - TE r2|  (paper Sec. 2.3
// eq. precond applied to the Sec. 2.4 derivatives, weights 1/sigma_i^2).
// ---------------------------------------------------------------------------
struct EchoAcc {
    float R0 = 0.f, R1 = 0.f, A0 = 0.f, A1 = 0.f, A2 = 0.f, B0 = 0.f, B2 = 0.f, L = 0.f;
    __device__ __forceinline__ void add(float s, float x, float te, float w, float r2)
    {
        if (!(fabsf(x) < INFINITY)) return;  // missing observation
        float res = s - x;
        float wr = w * res;
        float ws = w * s;
        float wrs = wr * s;
        R0 += wrs;
        R1 += wrs * te;
        float ws2 = ws * s;
        A0 += ws2;
        A1 += ws2 * te;
        A2 += ws2 * te * te;
        float ab = fabsf(wrs);
        B0 += ab;
        B2 += ab * te * fabsf(1.0f - te * r2);
        L += wr * res;
    }
};

__device__ __forceinline__ void accumulate_contrast(const EchoAcc &e, const ContrastK &K, float r2,
                                                    int loading, float g[4], float H[10])
{
    g[0] += e.R0;
    g[1] += K.phi * e.R0;
    g[2] -= r2 * e.R1;
    g[3] += K.psi * e.R0;
    H[0] += e.A0;
    H[1] += K.phi * e.A0;
    H[2] -= r2 * e.A1;
    H[3] += K.psi * e.A0;
    H[4] += K.phi * K.phi * e.A0;
    H[5] -= r2 * K.phi * e.A1;
    H[6] += K.phi * K.psi * e.A0;
    H[7] += r2 * r2 * e.A2;
    H[8] -= r2 * K.psi * e.A1;
    H[9] += K.psi * K.psi * e.A0;
    if (loading == 0) {
        H[0] += e.B0;
        H[4] += fabsf(K.kap * K.phi) * e.B0;
        H[7] += r2 * e.B2;
        H[9] += fabsf(K.mu * K.psi) * e.B0;
    }
}

// ---------------------------------------------------------------------------
// packed symmetric 4x4: 0:00 1:01 2:02 3:03 4:11 5:12 6:13 7:22 8:23 9:33
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int sym(int i, int j)
{
    return i <= j ? (i == 0 ? j : i == 1 ? 3 + j : i == 2 ? 5 + j : 9) : sym(j, i);
}

// out = P^{-1} g.  Returns true when the voxel is degenerate (out = 0).
__device__ __forceinline__ bool solve_sym4(const float P[10], const float g[4], float out[4])
{
    float dg[4] = {P[0], P[4], P[7], P[9]};
    float maxd = fmaxf(fmaxf(dg[0], dg[1]), fmaxf(dg[2], dg[3]));
    bool bad = !(maxd > 0.0f) || !(maxd < INFINITY);
#pragma unroll
    for (int k = 0; k < 4; k++) bad |= !(fabsf(g[k]) < INFINITY);
    float D[4];
    bool fz[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        fz[k] = !(dg[k] > FROZEN_REL * maxd);
        D[k] = fz[k] ? 0.0f : rsqrtf(dg[k]);
    }
    float S[4][4], rhs[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            float v = D[i] * P[sym(i, j)] * D[j];
            S[i][j] = (fz[i] || fz[j]) ? (i == j ? 1.0f : 0.0f) : v;
        }
        rhs[i] = fz[i] ? 0.0f : D[i] * g[i];
    }
    float L[4][4], inv[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        float piv = S[j][j];
#pragma unroll
        for (int m = 0; m < j; m++) piv -= L[j][m] * L[j][m];
        bad |= !(piv >= PIVOT_MIN);
        piv = fmaxf(piv, PIVOT_MIN);
        const float ij = rsqrtf(piv);  // 1 / L_jj
        L[j][j] = piv * ij;
        inv[j] = ij;
#pragma unroll
        for (int i = j + 1; i < 4; i++) {
            float v = S[i][j];
#pragma unroll
            for (int m = 0; m < j; m++) v -= L[i][m] * L[j][m];
            L[i][j] = v * inv[j];
        }
    }
    float t[4], u[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        float v = rhs[i];
#pragma unroll
        for (int m = 0; m < i; m++) v -= L[i][m] * t[m];
        t[i] = v * inv[i];
    }
#pragma unroll
    for (int i = 3; i >= 0; i--) {
        float v = t[i];
#pragma unroll
        for (int m = i + 1; m < 4; m++) v -= L[m][i] * u[m];
        u[i] = v * inv[i];
    }
#pragma unroll
    for (int k = 0; k < 4; k++) out[k] = bad ? 0.0f : D[k] * u[k];
    return bad;
}

// ---------------------------------------------------------------------------
// FP64 reductions (fixed order: deterministic for a given launch shape)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of v over the workgroup; the result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*lds)[NWAVE])
{
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        double s = wave_sum(v[k]);
        if (lane == 0) lds[k][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < NWAVE; w++) s += lds[k][w];
            v[k] = s;
        }
    }
}

}  // namespace mpm
