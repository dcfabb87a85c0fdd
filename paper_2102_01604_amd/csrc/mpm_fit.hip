// mpm_fit.hip -- host orchestration of the ML and MAP fits.
#include <cmath>
#include <cstring>

#include "mpm_api_internal.h"

namespace mpm {

// ---------------------------------------------------------------------------
// ML: one launch runs every Newton-like step of every voxel; a fixed-order
// reduction then gives the NLL trace and the report counters.
// ---------------------------------------------------------------------------
mpm_status fit_ml(const FitArgs &a, Workspace &ws, Prof &prof, mpm_report &rep, double *trace, int trace_len)
{
    const int n_gn = a.opt->n_gn;
    const int rows = n_gn + 4;
    const int nblk = ml_fit_blocks(a.N);
    double *part = nullptr, *sums = nullptr;
    if (ws.alloc((void **)&part, sizeof(double) * (size_t)rows * nblk) != hipSuccess ||
        ws.alloc((void **)&sums, sizeof(double) * rows) != hipSuccess)
        return fail(MPM_ERR_OUT_OF_MEMORY, "ML workspace allocation failed");
    LaunchCtx c{a.stream};
    double bytes = (double)a.N * ((double)a.P.I * dtype_size(a.dtype) + (a.b1 ? 4.0 : 0.0) + 32.0);
    hipError_t e = prof.launch("ml_fit", bytes, [&] {
        return launch_ml_fit(c, a.P, a.dtype, a.X, a.b1, a.maps, a.N, n_gn, a.opt->loading, part, nblk);
    });
    if (e == hipSuccess) e = launch_reduce_rows(c, part, rows, nblk, sums);
    std::vector<double> h(rows);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), sums, sizeof(double) * rows, hipMemcpyDeviceToHost, a.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(a.stream);
    if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "ML fit: %s", hipGetErrorString(e));
    for (int i = 0; i <= n_gn && i < trace_len; i++) trace[i] = h[i];
    rep.nll = rep.objective = h[n_gn];
    rep.jtv = 0.0;
    rep.gn_done = n_gn;
    rep.degenerate_voxels = (int64_t)llround(h[n_gn + 1]);
    rep.nonfinite_voxels = (int64_t)llround(h[n_gn + 2]);
    rep.nll_increases = (int64_t)llround(h[n_gn + 3]);
    return MPM_OK;
}

}  // namespace mpm
