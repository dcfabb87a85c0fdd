// mpm_fit.hip -- the ML fit as a job, and the shared initialisation step.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "mpm_api_internal.h"
#include "mpm_voxelwise.h"

namespace mpm {

PinnedBuf::~PinnedBuf()
{
    if (p) (void)hipHostFree(p);
}

hipError_t PinnedBuf::alloc(size_t bytes) { return hipHostMalloc(&p, bytes ? bytes : 8, hipHostMallocDefault); }

InitStage::~InitStage()
{
    if (ev) (void)hipEventDestroy(ev);
}

static mpm_status fill_maps(const FitArgs &a, const float y0[4])
{
    LaunchCtx c{a.stream};
    hipError_t e = launch_fill_maps(c, a.maps, a.N, y0);
    if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "init: %s", hipGetErrorString(e));
    return MPM_OK;
}

mpm_status InitStage::start(const FitArgs &a, Workspace &ws, Prof &prof)
{
    const mpm_options *opt = a.opt;
    if (opt->init_kind == MPM_INIT_FROM_MAPS) return MPM_OK;
    if (opt->init_kind == MPM_INIT_CONST) {
        float y0[4];
        for (int k = 0; k < 4; k++) y0[k] = (float)opt->init_const[k];
        return fill_maps(a, y0);
    }
    // default: the sums of every image (projected: each over its own space)
    // and of b1 over the reconstruction grid
    auto add = [&](const DevProto &P, const void *X, const float *b1, int64_t N) -> mpm_status {
        Seg sg{P, N, nullptr, rows};
        mpm_status st = enqueue_image_sums(ws, prof, P, a.dtype, X, b1, N, &sg.dev);
        if (st) return st;
        segs.push_back(sg);
        rows += image_sum_rows(P);
        return MPM_OK;
    };
    mpm_status st;
    if (!a.spaces) {
        if ((st = add(a.P, a.X, a.b1, a.N))) return st;
    } else {
        const char *X = (const char *)a.X;
        for (int c = 0; c < a.P.C; c++) {
            const DevProto Pc = sub_proto(a.P, c);
            const int64_t M = space_voxels(a.spaces[c]);
            if ((st = add(Pc, X, nullptr, M))) return st;
            X += (int64_t)Pc.I * M * (int64_t)dtype_size(a.dtype);
        }
        if (a.b1) {
            DevProto none;
            memset(&none, 0, sizeof(none));
            if ((st = add(none, nullptr, a.b1, a.N))) return st;
        }
    }
    pending = true;
    if (a.no_pinned) return MPM_OK;
    hipError_t e = host.alloc(sizeof(double) * rows);
    for (size_t k = 0; k < segs.size() && e == hipSuccess; k++)
        e = hipMemcpyAsync((double *)host.p + segs[k].at, segs[k].dev, sizeof(double) * image_sum_rows(segs[k].P),
                           hipMemcpyDeviceToHost, a.stream);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, a.stream);
    if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "init: %s", hipGetErrorString(e));
    return MPM_OK;
}

bool InitStage::ready() const { return !pending || !ev || hipEventQuery(ev) != hipErrorNotReady; }

mpm_status InitStage::finish(const FitArgs &a)
{
    if (!pending) return MPM_OK;
    pending = false;
    std::vector<double> local;
    const double *h;
    hipError_t e = hipSuccess;
    if (ev) {
        e = hipEventSynchronize(ev);
        h = (const double *)host.p;
    } else {
        // no pinned staging: copies on the fit's stream, then wait for them
        local.resize(rows);
        for (size_t k = 0; k < segs.size() && e == hipSuccess; k++)
            e = hipMemcpyAsync(local.data() + segs[k].at, segs[k].dev, sizeof(double) * image_sum_rows(segs[k].P),
                               hipMemcpyDeviceToHost, a.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(a.stream);
        h = local.data();
    }
    if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "init: %s", hipGetErrorString(e));
    std::vector<double> mean;
    double b1m = 1.0;
    for (const Seg &sg : segs) {
        std::vector<double> m;
        double b;
        image_means_from_sums(sg.P, sg.N, h + sg.at, m, b);
        mean.insert(mean.end(), m.begin(), m.end());
        // b1 comes with the images on one grid; projected fits sum it on its own
        if (!a.spaces || sg.P.I == 0) b1m = b;
    }
    float y0[4];
    mpm_status st = default_init_from_means(a.proto, mean.data(), b1m, y0);
    if (st) return st;
    return fill_maps(a, y0);
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
    InitStage init;

    bool ready() const override { return init.ready(); }

    MlJob(const FitArgs &a_, Workspace &ws_, Prof &prof_) : a(a_), ws(ws_), prof(prof_) {}

    mpm_status setup()
    {
        rows = a.opt->n_gn + 4;
        nblk = ml_fit_blocks(a.N);
        if (ws.alloc((void **)&part, sizeof(double) * (size_t)rows * nblk) != hipSuccess ||
            ws.alloc((void **)&sums, sizeof(double) * rows) != hipSuccess ||
            (!a.no_pinned && host.alloc(sizeof(double) * rows) != hipSuccess))
            return fail(MPM_ERR_OUT_OF_MEMORY, "ML workspace allocation failed");
        return MPM_OK;
    }

    mpm_status enqueue_next(bool *more) override
    {
        if (piece++ == 0) {
            *more = true;
            return init.start(a, ws, prof);
        }
        mpm_status st = init.finish(a);
        if (st) return st;
        *more = false;
        LaunchCtx c{a.stream};
        const int n_gn = a.opt->n_gn;
        const float *bm = a.opt->b1_receive;
        double bytes = (double)a.N * ((double)a.P.I * dtype_size(a.dtype) + (a.b1 ? 4.0 : 0.0) + (bm ? 4.0 : 0.0) +
                                      32.0);
        hipError_t e = prof.launch("ml_fit", bytes, [&] {
            return launch_ml_fit(c, a.P, a.dtype, a.X, a.b1, bm, a.maps, a.N, n_gn, a.opt->loading, part, nblk);
        });
        if (e == hipSuccess) e = launch_reduce_rows(c, part, rows, nblk, sums);
        if (e == hipSuccess && !a.no_pinned)
            e = hipMemcpyAsync(host.p, sums, sizeof(double) * rows, hipMemcpyDeviceToHost, a.stream);
        if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "ML fit: %s", hipGetErrorString(e));
        return MPM_OK;
    }

    mpm_status collect(mpm_report &rep, double *trace, int trace_len) override
    {
        const int n_gn = a.opt->n_gn;
        double tail[4];  // final NLL, degenerate, non-finite, increases (rows n_gn .. n_gn + 3)
        if (a.no_pinned) {
            // the NLL trace straight into trace
            const int nt = std::min(n_gn + 1, trace_len);
            hipError_t e = hipMemcpy(tail, sums + n_gn, sizeof(tail), hipMemcpyDeviceToHost);
            if (e == hipSuccess && nt > 0) e = hipMemcpy(trace, sums, sizeof(double) * nt, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "ML fit: %s", hipGetErrorString(e));
        } else {
            const double *h = (const double *)host.p;
            for (int i = 0; i <= n_gn && i < trace_len; i++) trace[i] = h[i];
            for (int k = 0; k < 4; k++) tail[k] = h[n_gn + k];
        }
        memset(&rep, 0, sizeof(rep));
        rep.nll = rep.objective = tail[0];
        rep.gn_done = n_gn;
        rep.degenerate_voxels = (int64_t)llround(tail[1]);
        rep.nonfinite_voxels = (int64_t)llround(tail[2]);
        rep.nll_increases = (int64_t)llround(tail[3]);
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

// ---------------------------------------------------------------------------
// ML fit with a protocol per voxel (paper Sec. 3.1 convergence experiment).
// ---------------------------------------------------------------------------
namespace mpm {
// The shared structure of per-voxel protocols as a protocol (TR, flip and TE
// are per voxel: placeholders here), validated; *I: number of images.
static mpm_status voxelwise_shape(const mpm_voxel_protocols *vp, int64_t n_voxels, mpm_protocol &p, int *I)
{
    if (!vp) return fail(MPM_ERR_INVALID_ARG, "protocols is NULL");
    if (vp->n_contrasts < 1 || vp->n_contrasts > MPM_MAX_CONTRASTS)
        return fail(MPM_ERR_INVALID_ARG, "n_contrasts=%d outside [1, %d]", vp->n_contrasts, MPM_MAX_CONTRASTS);
    memset(&p, 0, sizeof(p));
    p.n_contrasts = vp->n_contrasts;
    *I = 0;
    for (int c = 0; c < vp->n_contrasts; c++) {
        p.n_echoes[c] = vp->n_echoes[c];
        p.mt[c] = vp->mt[c];
        p.tr_s[c] = 1.0;
        p.flip_rad[c] = 0.1;
        if (vp->n_echoes[c] >= 1 && *I + vp->n_echoes[c] <= MPM_MAX_IMAGES) *I += vp->n_echoes[c];
    }
    for (int i = 0; i < *I; i++) p.sigma[i] = vp->sigma[i];
    mpm_status st;
    if ((st = check_protocol(&p))) return st;
    if (n_voxels < 1 || n_voxels > ((int64_t)1 << 34))
        return fail(MPM_ERR_INVALID_ARG, "n_voxels=%lld outside [1, 2^34]", (long long)n_voxels);
    if (!vp->tr_s || !vp->flip_rad || !vp->te_s)
        return fail(MPM_ERR_INVALID_ARG, "tr_s, flip_rad and te_s must be device pointers");
    return MPM_OK;
}
}  // namespace mpm

extern "C" mpm_status mpm_simulate_voxelwise(const mpm_voxel_protocols *vp, int64_t n_voxels, const float *maps,
                                             const float *noise, mpm_dtype out_dtype, void *out, void *stream)
{
    using namespace mpm;
    clear_error();
    mpm_protocol p;
    int I;
    mpm_status st;
    if ((st = voxelwise_shape(vp, n_voxels, p, &I)) || (st = check_dtype(out_dtype))) return st;
    if (!maps || !out) return fail(MPM_ERR_INVALID_ARG, "maps and out must be device pointers");
    hipStream_t s = (hipStream_t)stream;
    Prof prof(s);
    LaunchCtx c{s};
    const DevProto P = to_dev(&p);
    const PVArrays A{vp->tr_s, vp->flip_rad, vp->te_s};
    hipError_t e = prof.launch("simulate_pv", (double)n_voxels * (16.0 + 8.0 * p.n_contrasts +
                                                                    I * (4.0 + dtype_size(out_dtype) + (noise ? 4.0 : 0.0))),
                               [&] { return launch_simulate_pv(c, P, A, maps, noise, out_dtype, out, n_voxels); });
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    prof.collect();
    if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "simulate: %s", hipGetErrorString(e));
    return MPM_OK;
}

extern "C" mpm_status mpm_fit_voxelwise(const mpm_voxel_protocols *vp, int64_t n_voxels, mpm_dtype dtype,
                                        const void *echoes, const mpm_options *opt, float *maps,
                                        int32_t *nll_increases, float *nll, mpm_report *report, void *stream)
{
    using namespace mpm;
    clear_error();
    mpm_protocol p;
    int I;
    mpm_status st;
    if ((st = voxelwise_shape(vp, n_voxels, p, &I)) || (st = check_dtype(dtype))) return st;
    if (!echoes || !maps) return fail(MPM_ERR_INVALID_ARG, "echoes and maps must be device pointers");
    if (!opt) return fail(MPM_ERR_INVALID_ARG, "options is NULL");
    if (opt->mode != MPM_ML) return fail(MPM_ERR_INVALID_ARG, "mpm_fit_voxelwise is an ML fit (mode %d)", opt->mode);
    if (opt->n_gn < 0 || opt->n_gn > 100000) return fail(MPM_ERR_INVALID_ARG, "n_gn must be in [0, 100000]");
    if (opt->loading != MPM_LOAD_PROPOSED && opt->loading != MPM_LOAD_GN && opt->loading != MPM_LOAD_PROPOSED_PLUS)
        return fail(MPM_ERR_INVALID_ARG, "unknown loading %d", opt->loading);
    if (opt->flags != 0) return fail(MPM_ERR_INVALID_ARG, "flags must be 0");
    if (opt->start_outer != 0) return fail(MPM_ERR_INVALID_ARG, "start_outer is a MAP option (0 for ML)");
    if (opt->b1_receive) return fail(MPM_ERR_UNSUPPORTED, "b1_receive is not supported by the per-voxel-protocol fit");
    if (opt->echo_offset) return fail(MPM_ERR_UNSUPPORTED, "echo_offset is not supported by the per-voxel-protocol fit");
    if (opt->init_kind == MPM_INIT_DEFAULT)
        return fail(MPM_ERR_UNSUPPORTED, "the default initialisation needs one protocol for all voxels");
    if (opt->init_kind != MPM_INIT_CONST && opt->init_kind != MPM_INIT_FROM_MAPS)
        return fail(MPM_ERR_INVALID_ARG, "unknown init_kind %d", opt->init_kind);
    if (opt->init_kind == MPM_INIT_CONST)
        for (int k = 0; k < 4; k++)
            if (!std::isfinite(opt->init_const[k])) return fail(MPM_ERR_INVALID_ARG, "init_const[%d] is not finite", k);
    if (opt->basis != MPM_BASIS_LOG && opt->basis != MPM_BASIS_RATE && opt->basis != MPM_BASIS_TIME)
        return fail(MPM_ERR_INVALID_ARG, "unknown basis %d", opt->basis);
    if (opt->basis != MPM_BASIS_LOG && opt->init_kind == MPM_INIT_CONST) {
        const double *c = opt->init_const;
        if (!(c[0] > 0.0 && c[1] > 0.0 && c[2] > 0.0 && c[3] > 0.0 && c[3] < 1.0))
            return fail(MPM_ERR_INVALID_ARG, "init_const must lie in the basis' domain (A, R or T > 0, 0 < MTsat < 1)");
    }
    if (!has_mt(&p)) return fail(MPM_ERR_UNSUPPORTED, "the four-parameter model needs at least one MT contrast");

    const int64_t N = n_voxels;
    const DevProto P = to_dev(&p);
    const PVArrays A{vp->tr_s, vp->flip_rad, vp->te_s};
    hipStream_t s = (hipStream_t)stream;
    const int nblk = ml_fit_blocks(N);
    mpm_report rep;
    memset(&rep, 0, sizeof(rep));
    {
        Workspace ws(s);
        Prof prof(s);
        PinnedBuf host;
        double *part = nullptr, *sums = nullptr;
        if (ws.alloc((void **)&part, sizeof(double) * 4 * (size_t)nblk) != hipSuccess ||
            ws.alloc((void **)&sums, sizeof(double) * 4) != hipSuccess || host.alloc(sizeof(double) * 4) != hipSuccess)
            return fail(MPM_ERR_OUT_OF_MEMORY, "voxelwise fit: workspace allocation failed");
        LaunchCtx c{s};
        hipError_t e = hipSuccess;
        if (opt->init_kind == MPM_INIT_CONST) {
            float y0[4];
            for (int k = 0; k < 4; k++) y0[k] = (float)opt->init_const[k];
            e = launch_fill_maps(c, maps, N, y0);
        }
        const double bytes = (double)N * ((double)I * (dtype_size(dtype) + 4.0) + 8.0 * p.n_contrasts + 32.0 +
                                          (nll_increases ? 4.0 : 0.0) + (nll ? 4.0 : 0.0));
        if (e == hipSuccess)
            e = prof.launch("ml_fit_pv", bytes, [&] {
                return launch_ml_fit_pv(c, P, A, dtype, echoes, maps, N, opt->n_gn, opt->loading, opt->basis,
                                        nll_increases, nll, part);
            });
        if (e == hipSuccess) e = launch_reduce_rows(c, part, 4, nblk, sums);
        if (e == hipSuccess) e = hipMemcpyAsync(host.p, sums, sizeof(double) * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        prof.collect();
        if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "voxelwise fit: %s", hipGetErrorString(e));
        const double *h = (const double *)host.p;
        rep.nll = rep.objective = h[0];
        rep.gn_done = opt->n_gn;
        rep.degenerate_voxels = (int64_t)llround(h[1]);
        rep.nonfinite_voxels = (int64_t)llround(h[2]);
        rep.nll_increases = (int64_t)llround(h[3]);
    }
    if (report) *report = rep;
    return MPM_OK;
}
