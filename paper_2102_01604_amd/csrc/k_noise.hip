// k_noise.hip -- noise estimation kernels (paper Sec. 2.7): the largest value
// and the histogram of every magnitude image (two streaming passes over the
// echoes), then a two-class Rician mixture fitted to each histogram by EM.
//
// Mixture: class 0 is the background (air, no signal: a Rician with nu = 0),
// class 1 a Rician with free nu.  With the phase of each value as the latent
// variable, the EM step over the bin centres c (counts n) is
//   E: r_k(c) = pi_k p_k(c) / sum_j pi_j p_j(c),
//      log p_k(c) = log c - 2 log s_k - (c - nu_k)^2 / (2 s_k^2) + log(e^-z I0(z)),
//      z = c nu_k / s_k^2, and the posterior mean of cos(phase) I1(z) / I0(z);
//   M: pi_k = N_k / N, nu_1 = sum n r_1 c I1/I0 / N_1,
//      s_k^2 = (sum n r_k c^2 / N_k - nu_k^2) / 2.
// It starts from the split of the histogram at its mean.
#include <cmath>

#include "mpm_noise.h"
#include "mpm_stream.h"

namespace mpm {

constexpr int NOISE_THREADS = 256;  // streaming passes

int noise_blocks(int64_t N)
{
    // enough workgroups per image to fill the chip with 22 images, few enough
    // that merging the per-workgroup histograms stays cheap
    const int64_t want = (N + (int64_t)NOISE_THREADS * 256 - 1) / ((int64_t)NOISE_THREADS * 256);
    return (int)std::min<int64_t>(std::max<int64_t>(want, 1), 64);
}

__device__ __forceinline__ bool observed(float v) { return v >= 0.0f && v < INFINITY; }

template <typename T>
__global__ __launch_bounds__(NOISE_THREADS) void k_image_max(const T *__restrict__ X, int64_t N,
                                                            uint32_t *__restrict__ maxbits)
{
    const int i = blockIdx.y;
    float m = 0.0f;
    for_each_value(X + (int64_t)i * N, N, [&](float v) {
        if (observed(v)) m = fmaxf(m, v);
    });
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    __shared__ float wm[NOISE_THREADS / 64];
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NOISE_THREADS / 64; w++) m = fmaxf(m, wm[w]);
        // for values >= 0 the order of the FP32 bit patterns is the order of the values
        atomicMax(maxbits + i, __float_as_uint(m));
    }
}

template <typename T>
__global__ __launch_bounds__(NOISE_THREADS) void k_image_hist(const T *__restrict__ X, int64_t N, int nbins,
                                                             const uint32_t *__restrict__ maxbits,
                                                             uint32_t *__restrict__ counts)
{
    const int i = blockIdx.y;
    const float mx = __uint_as_float(maxbits[i]);
    if (!(mx > 0.0f)) return;  // uniform per workgroup
    __shared__ uint32_t h[NOISE_MAX_BINS];
    for (int b = threadIdx.x; b < nbins; b += NOISE_THREADS) h[b] = 0u;
    __syncthreads();
    const float scale = (float)nbins / mx;  // correctly rounded FP32 division
    for_each_value(X + (int64_t)i * N, N, [&](float v) {
        if (observed(v)) {
            const int b = (int)(v * scale);
            atomicAdd(&h[b < nbins ? b : nbins - 1], 1u);
        }
    });
    __syncthreads();
    uint32_t *out = counts + (int64_t)i * nbins;
    for (int b = threadIdx.x; b < nbins; b += NOISE_THREADS)
        if (h[b]) atomicAdd(out + b, h[b]);
}

// e^-z I0(z) and e^-z I1(z), z >= 0, in FP64: the ascending power series of
// I0 and I1 below z = 20, above it the asymptotic (Hankel) expansion
//   I_v(z) ~ e^z / sqrt(2 pi z) sum_k a_k,  a_k / a_{k-1} = ((2k - 1)^2 - 4 v^2) / (8 k z),
// until a term falls below 1e-17 of its sum, at most 40 terms (at z >= 20 the
// terms keep shrinking at least that far).
// Reciprocals the series divide by, 1/k^2, 1/(k (k+1)) and 1/k, formed at
// compile time (correctly rounded), so the loops multiply instead.
struct InvTable {
    double sq[100], kk1[100], k[41];
};
constexpr InvTable make_inv_table()
{
    InvTable t{};
    for (int k = 1; k < 100; k++) {
        t.sq[k] = 1.0 / ((double)k * (double)k);
        t.kk1[k] = 1.0 / ((double)k * (double)(k + 1));
    }
    for (int k = 1; k <= 40; k++) t.k[k] = 1.0 / (double)k;
    return t;
}
__constant__ InvTable c_inv = make_inv_table();

__device__ void bessel_i01e(double z, double &i0e, double &i1e)
{
    if (z < 20.0) {
        const double q = 0.25 * z * z;
        double t0 = 1.0, t1 = 0.5 * z, s0 = 1.0, s1 = 0.5 * z;
        for (int k = 1; k < 100; k++) {
            t0 *= q * c_inv.sq[k];
            t1 *= q * c_inv.kk1[k];
            s0 += t0;
            s1 += t1;
            if (t0 <= 1e-17 * s0 && t1 <= 1e-17 * s1) break;
        }
        const double e = exp(-z);
        i0e = s0 * e;
        i1e = s1 * e;
    } else {
        const double r = 0.125 / z;
        double a0 = 1.0, a1 = 1.0, s0 = 1.0, s1 = 1.0;
        for (int k = 1; k <= 40; k++) {
            const double m = (double)(2 * k - 1) * (double)(2 * k - 1);
            a0 *= m * r * c_inv.k[k];
            a1 *= (m - 4.0) * r * c_inv.k[k];
            s0 += a0;
            s1 += a1;
            if (fabs(a0) <= 1e-17 * s0 && fabs(a1) <= 1e-17 * s1) break;
        }
        const double f = 1.0 / sqrt(6.283185307179586 * z);
        i0e = f * s0;
        i1e = f * s1;
    }
}

// Sum of NV values over a workgroup of EM_THREADS threads; the result is
// valid in thread 0 (fixed order).
constexpr int EM_THREADS = 1024;
constexpr int EM_WAVES = EM_THREADS / 64;
constexpr int EM_PER = NOISE_MAX_BINS / EM_THREADS;  // bins per thread

template <int NV>
__device__ __forceinline__ void em_sum(double (&v)[NV], double (*lds)[EM_WAVES])
{
    static_assert(NV <= 8 && EM_WAVES == 16, "wave 0 sums 8 x 16 partial sums");
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        const double t = wave_sum(v[k]);
        if (lane == 0) lds[k][wid] = t;
    }
    __syncthreads();
    if (wid == 0) {
        // lane = 8 k + g sums waves 2g and 2g + 1 of value k, then the 8 lanes
        // of value k combine (fixed order); lane 0 collects the NV results
        const int k = lane >> 3, g = lane & 7;
        double t = k < NV ? lds[k][2 * g] + lds[k][2 * g + 1] : 0.0;
        t += __shfl_xor(t, 1, 64);
        t += __shfl_xor(t, 2, 64);
        t += __shfl_xor(t, 4, 64);
#pragma unroll
        for (int q = 0; q < NV; q++) {
            const double r = __shfl(t, 8 * q, 64);
            if (lane == 0) v[q] = r;
        }
    }
}

// One workgroup per image; thread t owns bins t, t + EM_THREADS, ...
__global__ __launch_bounds__(EM_THREADS) void k_rice_em(const uint32_t *__restrict__ counts,
                                                       const uint32_t *__restrict__ maxbits, int nbins, int n_iter,
                                                       double *__restrict__ fits)
{
    const int i = blockIdx.x;
    double *out = fits + (int64_t)i * NOISE_FIT_DOUBLES;
    const float mx = __uint_as_float(maxbits[i]);
    if (!(mx > 0.0f)) {  // uniform per workgroup
        if (threadIdx.x == 0)
            for (int k = 0; k < NOISE_FIT_DOUBLES; k++) out[k] = 0.0;
        return;
    }
    const float scale = (float)nbins / mx;
    const double width = 1.0 / (double)scale;
    double cnt[EM_PER], cen[EM_PER], lcen[EM_PER];
    const uint32_t *h = counts + (int64_t)i * nbins;
#pragma unroll
    for (int j = 0; j < EM_PER; j++) {
        const int b = threadIdx.x + j * EM_THREADS;
        cnt[j] = b < nbins ? (double)h[b] : 0.0;
        cen[j] = ((double)b + 0.5) * width;
        lcen[j] = log(cen[j]);
    }
    __shared__ double red[8][EM_WAVES];
    __shared__ double par[8];  // pi0 pi1 nu1 s0 s1 ok tot
    // start: the histogram split at the mean of its values
    {
        double v[2] = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < EM_PER; j++) {
            v[0] += cnt[j];
            v[1] += cnt[j] * cen[j];
        }
        em_sum<2>(v, red);
        if (threadIdx.x == 0) {
            par[0] = v[0];
            par[1] = v[1] / v[0];
        }
        __syncthreads();
        const double tot = par[0], m = par[1];
        double u[6] = {0, 0, 0, 0, 0, 0};  // weight, sum, sum of squares: lower part, then upper
#pragma unroll
        for (int j = 0; j < EM_PER; j++) {
            const int k = cen[j] < m ? 0 : 3;
            u[k] += cnt[j];
            u[k + 1] += cnt[j] * cen[j];
            u[k + 2] += cnt[j] * cen[j] * cen[j];
        }
        __syncthreads();
        em_sum<6>(u, red);
        if (threadIdx.x == 0) {
            const bool ok = u[0] > 0.0 && u[3] > 0.0;
            par[5] = ok ? 1.0 : 0.0;
            par[6] = tot;
            if (ok) {
                par[0] = u[0] / tot;
                par[1] = u[3] / tot;
                par[2] = u[4] / u[3];
                par[3] = sqrt(0.5 * u[2] / u[0]);
                const double var = u[5] / u[3] - par[2] * par[2];
                par[4] = sqrt(var > width * width ? var : width * width);
            }
        }
        __syncthreads();
    }
    if (par[5] == 0.0) {  // uniform: read after the barrier
        if (threadIdx.x == 0)
            for (int k = 0; k < NOISE_FIT_DOUBLES; k++) out[k] = 0.0;
        return;
    }
    const double tot = par[6];
    for (int it = 0;; it++) {
        const double lp0 = log(par[0]), lp1 = log(par[1]), nu1 = par[2], s0 = par[3], s1 = par[4];
        const double ls0 = 2.0 * log(s0), ls1 = 2.0 * log(s1), h0 = 0.5 / (s0 * s0), h1 = 0.5 / (s1 * s1);
        double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // N0 N1 Sx0 Sx1 Sx2_0 Sx2_1 Sxa1 NLL
#pragma unroll
        for (int j = 0; j < EM_PER; j++) {
            if (cnt[j] == 0.0) continue;
            const double c = cen[j], lc = lcen[j];
            double i0e, i1e;
            bessel_i01e(c * nu1 * 2.0 * h1, i0e, i1e);
            const double w0 = lp0 + lc - ls0 - c * c * h0;
            const double w1 = lp1 + lc - ls1 - (c - nu1) * (c - nu1) * h1 + log(i0e);
            const double top = fmax(w0, w1);
            const double lse = top + log(exp(w0 - top) + exp(w1 - top));
            const double r0 = cnt[j] * exp(w0 - lse), r1 = cnt[j] * exp(w1 - lse);
            v[0] += r0;
            v[1] += r1;
            v[2] += r0 * c;
            v[3] += r1 * c;
            v[4] += r0 * c * c;
            v[5] += r1 * c * c;
            v[6] += r1 * c * (i1e / i0e);
            v[7] -= cnt[j] * lse;
        }
        em_sum<8>(v, red);
        if (threadIdx.x == 0) {
            if (it == n_iter) {
                out[0] = par[0];
                out[1] = par[1];
                out[2] = 0.0;
                out[3] = nu1;
                out[4] = s0;
                out[5] = s1;
                out[6] = v[2] / v[0];
                out[7] = v[3] / v[1];
                out[8] = v[7];
                out[9] = 1.0;
            } else {
                par[0] = v[0] / tot;
                par[1] = v[1] / tot;
                par[2] = v[6] / v[1];
                par[3] = sqrt(0.5 * v[4] / v[0]);
                par[4] = sqrt(0.5 * (v[5] / v[1] - par[2] * par[2]));
            }
        }
        __syncthreads();
        if (it == n_iter) break;
    }
}

template <typename T>
static hipError_t max_t(hipStream_t s, const void *X, int64_t N, int I, uint32_t *maxbits)
{
    hipLaunchKernelGGL(k_image_max<T>, dim3(noise_blocks(N), I), dim3(NOISE_THREADS), 0, s, (const T *)X, N,
                       maxbits);
    return hipGetLastError();
}

hipError_t launch_image_max(hipStream_t s, int dtype, const void *X, int64_t N, int I, uint32_t *maxbits)
{
    if (dtype == DT_F32) return max_t<float>(s, X, N, I, maxbits);
    if (dtype == DT_F16) return max_t<F16>(s, X, N, I, maxbits);
    return max_t<BF16>(s, X, N, I, maxbits);
}

template <typename T>
static hipError_t hist_t(hipStream_t s, const void *X, int64_t N, int I, int nbins, const uint32_t *maxbits,
                         uint32_t *counts)
{
    hipLaunchKernelGGL(k_image_hist<T>, dim3(noise_blocks(N), I), dim3(NOISE_THREADS), 0, s, (const T *)X, N, nbins,
                       maxbits, counts);
    return hipGetLastError();
}

hipError_t launch_image_hist(hipStream_t s, int dtype, const void *X, int64_t N, int I, int nbins,
                             const uint32_t *maxbits, uint32_t *counts)
{
    if (dtype == DT_F32) return hist_t<float>(s, X, N, I, nbins, maxbits, counts);
    if (dtype == DT_F16) return hist_t<F16>(s, X, N, I, nbins, maxbits, counts);
    return hist_t<BF16>(s, X, N, I, nbins, maxbits, counts);
}

hipError_t launch_rice_em(hipStream_t s, const uint32_t *counts, const uint32_t *maxbits, int I, int nbins,
                          int n_iter, double *fits)
{
    hipLaunchKernelGGL(k_rice_em, dim3(I), dim3(EM_THREADS), 0, s, counts, maxbits, nbins, n_iter, fits);
    return hipGetLastError();
}

}  // namespace mpm
