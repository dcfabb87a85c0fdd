// mpm_fit.hip -- the ML fit as a job, and the shared initialisation step.
#include <cmath>
#include <cstring>

#include "mpm_api_internal.h"

namespace mpm {

PinnedBuf::~PinnedBuf()
{
    if (p) (void)hipHostFree(p);
}

hipError_t PinnedBuf::alloc(size_t bytes) { return hipHostMalloc(&p, bytes ? bytes : 8, hipHostMallocDefault); }

mpm_status enqueue_init(const FitArgs &a, Workspace &ws, Prof &prof)
{
    const mpm_options *opt = a.opt;
    if (opt->init_kind == MPM_INIT_FROM_MAPS) return MPM_OK;
    float y0[4];
    if (opt->init_kind == MPM_INIT_CONST) {
        for (int k = 0; k < 4; k++) y0[k] = (float)opt->init_const[k];
    } else {
        std::vector<double> mean;
        double b1m;
        mpm_status st;
        if (!a.spaces) {
            if ((st = image_means(ws, prof, a.P, a.dtype, a.X, a.b1, a.N, mean, b1m))) return st;
        } else {
            // projected: each image's mean over its own space; b1 over the reconstruction grid
            const char *X = (const char *)a.X;
            double unused;
            for (int c = 0; c < a.P.C; c++) {
                const DevProto Pc = sub_proto(a.P, c);
                const int64_t M = space_voxels(a.spaces[c]);
                std::vector<double> mc;
                if ((st = image_means(ws, prof, Pc, a.dtype, X, nullptr, M, mc, unused))) return st;
                mean.insert(mean.end(), mc.begin(), mc.end());
                X += (int64_t)Pc.I * M * (int64_t)dtype_size(a.dtype);
            }
            b1m = 1.0;
            if (a.b1) {
                DevProto none;
                memset(&none, 0, sizeof(none));
                std::vector<double> m0;
                if ((st = image_means(ws, prof, none, a.dtype, nullptr, a.b1, a.N, m0, b1m))) return st;
            }
        }
        if ((st = default_init_from_means(a.proto, mean.data(), b1m, y0))) return st;
    }
    LaunchCtx c{a.stream};
    hipError_t e = launch_fill_maps(c, a.maps, a.N, y0);
    if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "init: %s", hipGetErrorString(e));
    return MPM_OK;
}

// ---------------------------------------------------------------------------
// ML (paper Sec. 2.3-2.4): one launch runs every Newton-like step of every
// voxel; a fixed-order reduction then gives the NLL trace and the report
// counters, copied to pinned host memory on the stream.
// ---------------------------------------------------------------------------
struct MlJob : FitJob {
    FitArgs a;
    Workspace &ws;
    Prof &prof;
    int piece = 0, rows = 0, nblk = 0;
    double *part = nullptr, *sums = nullptr;
    PinnedBuf host;

    MlJob(const FitArgs &a_, Workspace &ws_, Prof &prof_) : a(a_), ws(ws_), prof(prof_) {}

    mpm_status setup()
    {
        rows = a.opt->n_gn + 4;
        nblk = ml_fit_blocks(a.N);
        if (ws.alloc((void **)&part, sizeof(double) * (size_t)rows * nblk) != hipSuccess ||
            ws.alloc((void **)&sums, sizeof(double) * rows) != hipSuccess ||
            host.alloc(sizeof(double) * rows) != hipSuccess)
            return fail(MPM_ERR_OUT_OF_MEMORY, "ML workspace allocation failed");
        return MPM_OK;
    }

    mpm_status enqueue_next(bool *more) override
    {
        if (piece++ == 0) {
            *more = true;
            return enqueue_init(a, ws, prof);
        }
        *more = false;
        LaunchCtx c{a.stream};
        const int n_gn = a.opt->n_gn;
        double bytes = (double)a.N * ((double)a.P.I * dtype_size(a.dtype) + (a.b1 ? 4.0 : 0.0) + 32.0);
        hipError_t e = prof.launch("ml_fit", bytes, [&] {
            return launch_ml_fit(c, a.P, a.dtype, a.X, a.b1, a.maps, a.N, n_gn, a.opt->loading, part, nblk);
        });
        if (e == hipSuccess) e = launch_reduce_rows(c, part, rows, nblk, sums);
        if (e == hipSuccess)
            e = hipMemcpyAsync(host.p, sums, sizeof(double) * rows, hipMemcpyDeviceToHost, a.stream);
        if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "ML fit: %s", hipGetErrorString(e));
        return MPM_OK;
    }

    mpm_status collect(mpm_report &rep, double *trace, int trace_len) override
    {
        const int n_gn = a.opt->n_gn;
        const double *h = (const double *)host.p;
        for (int i = 0; i <= n_gn && i < trace_len; i++) trace[i] = h[i];
        memset(&rep, 0, sizeof(rep));
        rep.nll = rep.objective = h[n_gn];
        rep.gn_done = n_gn;
        rep.degenerate_voxels = (int64_t)llround(h[n_gn + 1]);
        rep.nonfinite_voxels = (int64_t)llround(h[n_gn + 2]);
        rep.nll_increases = (int64_t)llround(h[n_gn + 3]);
        return MPM_OK;
    }
};

std::unique_ptr<FitJob> make_ml_job(const FitArgs &a, Workspace &ws, Prof &prof, mpm_status *st)
{
    std::unique_ptr<MlJob> j(new MlJob(a, ws, prof));
    *st = j->setup();
    if (*st) return nullptr;
    return std::unique_ptr<FitJob>(j.release());
}

}  // namespace mpm
