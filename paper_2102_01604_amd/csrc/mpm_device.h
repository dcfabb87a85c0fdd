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
    float off[MAXI];          // offset added to each stored value (reduced-precision storage)
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

// A stored value plus its image's offset (reduced-precision storage only: FP32
// echoes carry no offsets, so their path has no extra instruction).
template <typename T>
__device__ __forceinline__ float decode_echo(const T *p, float off)
{
    return load_echo(p) + off;
}
template <>
__device__ __forceinline__ float decode_echo(const float *p, float)
{
    return load_echo(p);
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
    p.dl = __builtin_amdgcn_rcpf(1.0f + __expf(-y[3]));
    return p;
}

// Per-(voxel, contrast) factors of the signal and its log-parameter
// derivatives.  With E = exp(-r1 TR), omega = (1 - delta) cos(alpha):
//   s(TE)        = s0 * exp(-r2 TE)
//   ds/d log a   = s,            d2s = s
//   ds/d log r1  = phi * s,      d2s = kap * phi * s
//   ds/d log r2  = -TE r2 s,     d2s = (1 - TE r2)(-TE r2) s
//   ds/d logit d = psi * s,      d2s = mu * psi * s      (MT contrasts)
//   cross terms:  d2s/d log a d(.) = ds/d(.),  d2s/d log r2 d(.) = -TE r2 ds/d(.),
//                 d2s/d log r1 d logit d = chi * s
// 1 - E, 1 - omega, 1 - omega E and 1 - cos(alpha) E are formed without
// cancellation (expm1 and 2 sin^2(alpha/2)), which FP32 needs at TR = 25 ms.
struct ContrastK {
    float s0, phi, psi, kap, mu, chi;
};

// Flip-angle terms of one (voxel, contrast), computed once per voxel, all
// from the half angle h = alpha / 2:
//   sin(alpha) = 2 sin(h) cos(h),  cos(alpha) = 1 - 2 sin^2(h),
//   1 - cos(alpha) = 2 sin^2(h)  (no cancellation for small flip angles).
// sin(h) and cos(h): h = r + q pi/2 with integer q and |r| <= pi/4 (pi/2 split
// in two parts, so r is exact to FP32 rounding for |h| < 1e4), then the Taylor
// series of sin r and cos r, truncated where the next term is below 1e-11,
// and the quadrant identities.  Flip angles up to pi/2 (h <= pi/4) give q = 0.
struct Angle {
    float sa, ca, omc;  // sin(alpha), cos(alpha), 1 - cos(alpha)
};

__device__ __forceinline__ Angle make_angle(float alpha)
{
    const float h = 0.5f * alpha;
    const float q = rintf(h * 0.63661977f);  // 2 / pi
    const float r = fmaf(q, 4.3711388e-8f, fmaf(-q, 1.5707964f, h));  // h - q pi/2, pi/2 = 1.5707964 - 4.3711388e-8
    const float u = r * r;
    // sin r = r (1 - u/3! + u^2/5! - u^3/7! + u^4/9! - u^5/11!)
    float ps = -2.5052108e-8f;
    ps = fmaf(ps, u, 2.7557319e-6f);
    ps = fmaf(ps, u, -1.9841270e-4f);
    ps = fmaf(ps, u, 8.3333333e-3f);
    ps = fmaf(ps, u, -1.6666667e-1f);
    const float sr = fmaf(r * u, ps, r);
    // cos r = 1 - u/2! + u^2/4! - u^3/6! + u^4/8! - u^5/10! + u^6/12!
    float pc = 2.0876757e-9f;
    pc = fmaf(pc, u, -2.7557319e-7f);
    pc = fmaf(pc, u, 2.4801587e-5f);
    pc = fmaf(pc, u, -1.3888889e-3f);
    pc = fmaf(pc, u, 4.1666667e-2f);
    pc = fmaf(pc, u, -0.5f);
    const float cr = fmaf(u, pc, 1.0f);
    const int iq = (int)q & 3;
    const float sh = iq == 0 ? sr : iq == 1 ? cr : iq == 2 ? -sr : -cr;
    const float ch = iq == 0 ? cr : iq == 1 ? -sr : iq == 2 ? -cr : sr;
    Angle a;
    a.omc = 2.0f * sh * sh;
    a.sa = 2.0f * sh * ch;
    a.ca = 1.0f - a.omc;
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
    float inv_den = __builtin_amdgcn_rcpf(den);
    ContrastK k;
    k.s0 = p.a * an.sa * (1.0f - dl) * ome * inv_den;
    k.phi = x * one_m_omega * e1 * inv_den * __builtin_amdgcn_rcpf(ome);
    k.kap = 1.0f - x * (2.0f - den) * inv_den;  // 1 + omega E = 2 - den
    k.psi = -dl * inv_den;
    k.mu = 2.0f * (1.0f - dl) * (ome + e1 * an.omc) * inv_den - 1.0f;
    // d2s/d log r1 d logit delta = chi s (not printed in the paper; the cross
    // derivative of the same factorisation): -x E delta ((1 - w) - w (1 - E))
    // / ((1 - E)(1 - w E)^2) with w = (1 - delta) cos(alpha)
    k.chi = -x * e1 * dl * (one_m_omega - (1.0f - one_m_omega) * ome) * inv_den * inv_den * __builtin_amdgcn_rcpf(ome);
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
// eq. precond applied to the Sec. 2.4 derivatives, weights 1/sigma_i^2).  The
// Proposed+ loading (absolute row sums of d2s) also needs BT = sum w |res s| TE.
// ---------------------------------------------------------------------------
struct EchoAcc {
    float R0 = 0.f, R1 = 0.f, A0 = 0.f, A1 = 0.f, A2 = 0.f, B0 = 0.f, BT = 0.f, B2 = 0.f, L = 0.f;
    // One echo: model value s, observation x at echo time te (te2 = te^2),
    // weight w.  A non-finite x is a missing observation: its weight and value
    // are replaced by 0, so every term it adds is exactly 0.
    __device__ __forceinline__ void add(float s, float x, float te, float te2, float w, float r2)
    {
        const bool ok = fabsf(x) < INFINITY;
        const float wv = ok ? w : 0.0f;
        const float res = s - (ok ? x : 0.0f);
        const float wr = wv * res;
        const float ws = wv * s;
        const float wrs = wr * s;
        R0 += wrs;
        R1 = fmaf(wrs, te, R1);
        const float ws2 = ws * s;
        A0 += ws2;
        A1 = fmaf(ws2, te, A1);
        A2 = fmaf(ws2, te2, A2);
        B0 += fabsf(wrs);
        BT = fmaf(fabsf(wrs), te, BT);
        B2 = fmaf(fabsf(wrs), fabsf(fmaf(-te2, r2, te)), B2);  // te |1 - te r2|, te >= 0
        L = fmaf(wr, res, L);
    }
};

// The same echo's contribution to sum w res^2 (value only, same arithmetic
// as EchoAcc::L).
__device__ __forceinline__ float nll_add(float s, float x, float w, float L)
{
    const bool ok = fabsf(x) < INFINITY;
    const float res = s - (ok ? x : 0.0f);
    return fmaf((ok ? w : 0.0f) * res, res, L);
}

// PLUS: the Proposed+ loading (loading is then ignored); otherwise loading 0
// (|diag|) or 1 (none).  Without PLUS, BT and chi are never read, so the
// compiler drops their arithmetic.
template <bool PLUS>
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
    if (PLUS) {  // absolute row sums of d2s (Proposed+)
        const float ap = fabsf(K.phi), as = fabsf(K.psi), ac = fabsf(K.chi), rt = r2 * e.BT;
        H[0] += e.B0 * (1.0f + ap + as) + rt;
        H[4] += e.B0 * (ap + fabsf(K.kap * K.phi) + ac) + rt * ap;
        H[7] += r2 * (e.BT * (1.0f + ap + as) + e.B2);
        H[9] += e.B0 * (as + ac + fabsf(K.mu * K.psi)) + rt * as;
    } else if (loading == 0) {  // |diag of d2s|
        H[0] += e.B0;
        H[4] += fabsf(K.kap * K.phi) * e.B0;
        H[7] += r2 * e.B2;
        H[9] += fabsf(K.mu * K.psi) * e.B0;
    }
}

// ---------------------------------------------------------------------------
// The echoes of one voxel and its likelihood terms.
//
// Protocols of at most CM contrasts with at most EM echoes each use a table
// with one slot (c, e) per contrast and echo at fixed offsets of the kernel
// arguments (ShapedProto), and keep the voxel's echoes in registers, x[c][e],
// with every load issued before any arithmetic uses them.  Slots past the last
// echo of a contrast repeat its last image with weight 0: they read valid
// memory and add exactly 0, so the per-echo loops carry no guards.  Other
// protocols use DevProto and read each echo inside the per-echo loop.  Both
// evaluate the same per-echo arithmetic:
//   K = stage(P): per-workgroup constants (called by every thread first);
//   lik<PLUS>(P, K, y, loading, grad, g, H): NLL; with grad also g and the
//       loaded Hessian (paper Sec. 2.3 eq. precond with the Sec. 2.4
//       derivatives; PLUS selects the Proposed+ loading);
//   nll(P, K, y): the NLL alone (bitwise equal to lik's).
// ---------------------------------------------------------------------------
template <typename T, int CM, int EM>
struct ShapedProto {
    int C;
    uint32_t stride;          // bytes between consecutive images (N * sizeof(T))
    const T *base[CM];        // first image of contrast c
    int last[CM];             // echo index of the last image of contrast c
    float tr[CM], flip[CM];
    int mt[CM];
    float te[CM][EM], te2[CM][EM], wgt[CM][EM];
    float off[CM][EM];        // offset added to each stored value (FP16 / BF16 storage)
};

// Host: the slot table of protocol P for echoes X [I][N] (N < 2^30).  Needs
// at most CM contrasts of at most EM echoes.
template <typename T, int CM, int EM>
inline ShapedProto<T, CM, EM> make_shaped(const DevProto &P, const T *X, int64_t N)
{
    ShapedProto<T, CM, EM> s = {};
    s.C = P.C;
    s.stride = (uint32_t)(N * (int64_t)sizeof(T));
    for (int c = 0; c < CM; c++) {
        const bool on = c < P.C;
        const int ne = on ? P.first[c + 1] - P.first[c] : 1;
        s.base[c] = X + (on ? (int64_t)P.first[c] * N : 0);
        s.last[c] = ne - 1;
        s.tr[c] = on ? P.tr[c] : 1.0f;
        s.flip[c] = on ? P.flip[c] : 0.0f;
        s.mt[c] = on ? P.mt[c] : 0;
        for (int e = 0; e < EM; e++) {
            const int i = on ? P.first[c] + (e < ne ? e : ne - 1) : 0;
            s.te[c][e] = P.te[i];
            s.te2[c][e] = P.te[i] * P.te[i];
            s.wgt[c][e] = on && e < ne ? P.wgt[i] : 0.0f;
            s.off[c][e] = P.off[i];
        }
    }
    return s;
}

typedef float slot4 __attribute__((ext_vector_type(4)));  // te, te^2, weight, 0 of one slot
typedef const volatile __attribute__((address_space(3))) slot4 lds_slot4;

template <typename T, int CM, int EM>
struct VoxelEchoes {
    using Proto = ShapedProto<T, CM, EM>;
    using Consts = lds_slot4 *;
    float x[CM][EM];
    Angle an[CM];
    float bm;  // net receive field of the voxel (multiplies its signal)

    // Stage the per-slot constants in LDS, read back at each use (volatile:
    // one broadcast LDS read per slot and evaluation, instead of holding all
    // of them in scalar registers).  Every thread of the workgroup calls this
    // before load; it ends with a barrier.
    static __device__ __forceinline__ Consts stage(const Proto &P)
    {
        __shared__ slot4 tab[CM * EM];
        if (threadIdx.x == 0) {
#pragma unroll
            for (int c = 0; c < CM; c++)
#pragma unroll
                for (int e = 0; e < EM; e++) tab[c * EM + e] = slot4{P.te[c][e], P.te2[c][e], P.wgt[c][e], 0.0f};
        }
        __syncthreads();
        return (lds_slot4 *)tab;
    }

    // n: voxel index; byte offsets n * sizeof(T) fit 32 bits (N < 2^30); b, bm_:
    // transmit and receive fields of the voxel
    __device__ __forceinline__ void load(const Proto &P, const T *__restrict__, int64_t, int64_t n, float b,
                                         float bm_ = 1.0f)
    {
        bm = bm_;
        const uint32_t off = (uint32_t)n * (uint32_t)sizeof(T);
#pragma unroll
        for (int c = 0; c < CM; c++) {
            if (c < P.C) {
                const char *img0 = (const char *)P.base[c] + off;
#pragma unroll
                for (int e = 0; e < EM; e++) {
                    const uint64_t k = (uint64_t)(e < P.last[c] ? e : P.last[c]);  // slots past the last echo
                    x[c][e] = decode_echo((const T *)(img0 + k * P.stride), P.off[c][e]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CM; c++)
            if (c < P.C) an[c] = make_angle(P.flip[c] * b);
    }

    template <bool PLUS>
    __device__ __forceinline__ float lik(const Proto &P, Consts K, const float y[4], int loading, bool grad,
                                         float g[4], float H[10]) const
    {
        Params p = decode(y);
        p.a *= bm;  // the receive field multiplies the whole signal (Sec. 2.4)
        const float k2 = -p.r2 * 1.4426950f;  // exp(-r2 te) = 2^(k2 te)
        float nll = 0.f;
#pragma unroll
        for (int k = 0; k < 4; k++) g[k] = 0.f;
#pragma unroll
        for (int k = 0; k < 10; k++) H[k] = 0.f;
#pragma unroll
        for (int c = 0; c < CM; c++) {
            if (c < P.C) {
                const ContrastK F = contrast_factors(p, P.tr[c], an[c], P.mt[c]);
                EchoAcc acc;
#pragma unroll
                for (int e = 0; e < EM; e++) {
                    const slot4 k = K[c * EM + e];
                    acc.add(F.s0 * __builtin_amdgcn_exp2f(k2 * k.x), x[c][e], k.x, k.y, k.z, p.r2);
                }
                nll += 0.5f * acc.L;
                if (grad) accumulate_contrast<PLUS>(acc, F, p.r2, loading, g, H);
            }
        }
        return nll;
    }

    __device__ __forceinline__ float nll(const Proto &P, Consts K, const float y[4]) const
    {
        Params p = decode(y);
        p.a *= bm;  // the receive field multiplies the whole signal (Sec. 2.4)
        const float k2 = -p.r2 * 1.4426950f;
        float v = 0.f;
#pragma unroll
        for (int c = 0; c < CM; c++) {
            if (c < P.C) {
                const float s0 = contrast_factors(p, P.tr[c], an[c], P.mt[c]).s0;
                float L = 0.f;
#pragma unroll
                for (int e = 0; e < EM; e++) {
                    const slot4 k = K[c * EM + e];
                    L = nll_add(s0 * __builtin_amdgcn_exp2f(k2 * k.x), x[c][e], k.z, L);
                }
                v += 0.5f * L;
            }
        }
        return v;
    }
};

template <typename T>
struct VoxelEchoes<T, 0, 0> {
    using Proto = DevProto;
    using Consts = const void *;
    const T *__restrict__ X;
    int64_t N, n;
    float b, bm;

    static __device__ __forceinline__ Consts stage(const Proto &) { return nullptr; }

    __device__ __forceinline__ void load(const Proto &, const T *__restrict__ X_, int64_t N_, int64_t n_, float b_,
                                         float bm_ = 1.0f)
    {
        X = X_;
        N = N_;
        n = n_;
        b = b_;
        bm = bm_;
    }

    template <bool PLUS>
    __device__ __forceinline__ float lik(const Proto &P, Consts, const float y[4], int loading, bool grad,
                                         float g[4], float H[10]) const
    {
        Params p = decode(y);
        p.a *= bm;  // the receive field multiplies the whole signal (Sec. 2.4)
        const float k2 = -p.r2 * 1.4426950f;
        float nll = 0.f;
#pragma unroll
        for (int k = 0; k < 4; k++) g[k] = 0.f;
#pragma unroll
        for (int k = 0; k < 10; k++) H[k] = 0.f;
        for (int c = 0; c < P.C; c++) {
            const ContrastK K = contrast_factors(p, P.tr[c], make_angle(P.flip[c] * b), P.mt[c]);
            EchoAcc acc;
            for (int i = P.first[c]; i < P.first[c + 1]; i++) {
                const float te = P.te[i];
                acc.add(K.s0 * __builtin_amdgcn_exp2f(k2 * te), decode_echo(X + (int64_t)i * N + n, P.off[i]), te,
                        te * te, P.wgt[i], p.r2);
            }
            nll += 0.5f * acc.L;
            if (grad) accumulate_contrast<PLUS>(acc, K, p.r2, loading, g, H);
        }
        return nll;
    }

    __device__ __forceinline__ float nll(const Proto &P, Consts, const float y[4]) const
    {
        Params p = decode(y);
        p.a *= bm;  // the receive field multiplies the whole signal (Sec. 2.4)
        const float k2 = -p.r2 * 1.4426950f;
        float v = 0.f;
        for (int c = 0; c < P.C; c++) {
            const float s0 = contrast_factors(p, P.tr[c], make_angle(P.flip[c] * b), P.mt[c]).s0;
            float L = 0.f;
            for (int i = P.first[c]; i < P.first[c + 1]; i++)
                L = nll_add(s0 * __builtin_amdgcn_exp2f(k2 * P.te[i]), decode_echo(X + (int64_t)i * N + n, P.off[i]),
                            P.wgt[i], L);
            v += 0.5f * L;
        }
        return v;
    }
};

// Register shape of a protocol: 1 = at most 4 contrasts x 8 echoes, 2 = 4 x 16,
// 3 = 8 x 8, 0 = any other protocol (echoes read from memory echo by echo).
inline int echo_shape(const DevProto &P)
{
    int emax = 0;
    for (int c = 0; c < P.C; c++) emax = emax > P.first[c + 1] - P.first[c] ? emax : P.first[c + 1] - P.first[c];
    if (P.C <= 4 && emax <= 8) return 1;
    if (P.C <= 4 && emax <= 16) return 2;
    if (emax <= 8) return 3;
    return 0;
}

// Host: the kernel-argument form of the protocol for register shape (CM, EM).
template <typename T, int CM, int EM>
struct ProtoArg {
    static ShapedProto<T, CM, EM> make(const DevProto &P, const T *X, int64_t N)
    {
        return make_shaped<T, CM, EM>(P, X, N);
    }
};
template <typename T>
struct ProtoArg<T, 0, 0> {
    static DevProto make(const DevProto &P, const T *, int64_t) { return P; }
};

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
