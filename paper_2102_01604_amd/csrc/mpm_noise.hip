// mpm_noise.hip -- mpm_estimate_noise: the noise level and the constant
// initial maps from the echoes, as paper Sec. 2.7 obtains them.
#include <cmath>
#include <cstring>

#include "mpm_api_internal.h"
#include "mpm_noise.h"

using namespace mpm;

extern "C" mpm_status mpm_estimate_noise(const mpm_protocol *protocol, const mpm_grid *grid, mpm_dtype dtype,
                                         const void *echoes, const float *b1, int32_t nbins, int32_t n_iter,
                                         double *sigma_image, double *sigma_contrast, double *fg_mean,
                                         double *init_const, mpm_rice_fit *fits, uint32_t *hist, void *stream)
{
    clear_error();
    int64_t N;
    mpm_status st;
    if (!protocol) return fail(MPM_ERR_INVALID_ARG, "protocol is NULL");
    mpm_protocol p = *protocol;  // sigma is what is estimated: not read
    for (int i = 0; i < MPM_MAX_IMAGES; i++) p.sigma[i] = 1.0;
    if ((st = check_protocol(&p)) || (st = check_grid(grid, &N)) || (st = check_dtype(dtype))) return st;
    if (!echoes) return fail(MPM_ERR_INVALID_ARG, "echoes must be a device pointer");
    if (!sigma_image || !sigma_contrast || !fg_mean || !init_const)
        return fail(MPM_ERR_INVALID_ARG, "sigma_image, sigma_contrast, fg_mean and init_const must be host pointers");
    if (nbins < 16 || nbins > NOISE_MAX_BINS)
        return fail(MPM_ERR_INVALID_ARG, "nbins must be in [16, %d]", NOISE_MAX_BINS);
    if (n_iter < 0 || n_iter > 100000) return fail(MPM_ERR_INVALID_ARG, "n_iter must be in [0, 100000]");
    if (!has_mt(&p)) return fail(MPM_ERR_UNSUPPORTED, "the four-parameter model needs at least one MT contrast");
    const DevProto P = to_dev(&p);
    const int I = P.I;
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> f((size_t)I * NOISE_FIT_DOUBLES);
    double b1m = 1.0;
    {
        Workspace ws(s);
        Prof prof(s);
        uint32_t *maxbits = nullptr, *counts = nullptr;
        double *dfits = nullptr;
        if (ws.alloc((void **)&maxbits, sizeof(uint32_t) * I) != hipSuccess ||
            ws.alloc((void **)&counts, sizeof(uint32_t) * (size_t)I * nbins) != hipSuccess ||
            ws.alloc((void **)&dfits, sizeof(double) * f.size()) != hipSuccess)
            return fail(MPM_ERR_OUT_OF_MEMORY, "noise estimation: workspace allocation failed");
        hipError_t e = hipMemsetAsync(maxbits, 0, sizeof(uint32_t) * I, s);
        if (e == hipSuccess) e = hipMemsetAsync(counts, 0, sizeof(uint32_t) * (size_t)I * nbins, s);
        const double xb = (double)N * I * dtype_size(dtype);
        if (e == hipSuccess)
            e = prof.launch("image_max", xb, [&] { return launch_image_max(s, dtype, echoes, N, I, maxbits); });
        if (e == hipSuccess)
            e = prof.launch("image_hist", xb,
                            [&] { return launch_image_hist(s, dtype, echoes, N, I, nbins, maxbits, counts); });
        if (e == hipSuccess)
            e = prof.launch("rice_em", 0.0,
                            [&] { return launch_rice_em(s, counts, maxbits, I, nbins, n_iter, dfits); });
        if (e == hipSuccess)
            e = hipMemcpyAsync(f.data(), dfits, sizeof(double) * f.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && hist)
            e = hipMemcpyAsync(hist, counts, sizeof(uint32_t) * (size_t)I * nbins, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        prof.collect();
        if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "noise estimation: %s", hipGetErrorString(e));
        if (b1) {
            DevProto none;
            memset(&none, 0, sizeof(none));
            std::vector<double> unused;
            if ((st = image_means(ws, prof, none, dtype, nullptr, b1, N, unused, b1m))) return st;
        }
    }
    for (int i = 0; i < I; i++)
        if (f[(size_t)i * NOISE_FIT_DOUBLES + 9] != 1.0)
            return fail(MPM_ERR_UNSUPPORTED, "image %d: its values do not split into background and signal", i);
    for (int i = 0; i < I; i++) {
        const double *r = &f[(size_t)i * NOISE_FIT_DOUBLES];
        const int bg = r[6] <= r[7] ? 0 : 1;  // the class with the lower mean
        sigma_image[i] = r[4 + bg];
        fg_mean[i] = r[7 - bg];
        if (fits) {
            for (int k = 0; k < 2; k++) {
                fits[i].pi[k] = r[k];
                fits[i].nu[k] = r[2 + k];
                fits[i].sigma[k] = r[4 + k];
                fits[i].mean[k] = r[6 + k];
            }
            fits[i].nll = r[8];
        }
    }
    for (int c = 0; c < P.C; c++) {
        const int first = P.first[c], ne = P.first[c + 1] - first;
        double lv = 0.0;
        for (int e = 0; e < ne; e++) lv += std::log(sigma_image[first + e] * sigma_image[first + e]);
        sigma_contrast[c] = std::sqrt(std::exp(lv / ne));
    }
    float y0[4];
    if ((st = default_init_from_means(&p, fg_mean, b1m, y0))) return st;
    for (int k = 0; k < 4; k++) init_const[k] = y0[k];
    return MPM_OK;
}
