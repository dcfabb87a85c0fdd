// mpm_api_internal.h -- host-side helpers shared by libmpm's C-ABI sources.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <memory>
#include <vector>

#include "../../include/mpm.h"
#include "mpm_kernels.h"

namespace mpm {

mpm_status fail(mpm_status st, const char *fmt, ...);
void clear_error();
int n_images(const mpm_protocol *p);
mpm_status check_protocol(const mpm_protocol *p);
mpm_status check_grid(const mpm_grid *g, int64_t *N);
mpm_status check_dtype(int dtype);
bool has_mt(const mpm_protocol *p);
// Device form of a protocol; echo_offset: host float [I] or NULL (zeros).
DevProto to_dev(const mpm_protocol *p, const float *echo_offset = nullptr);
// echo_offset of the options: only with reduced-precision storage, finite.
mpm_status check_echo_offset(const mpm_protocol *p, int dtype, const float *echo_offset);
size_t dtype_size(int dtype);
mpm_status default_init_from_means(const mpm_protocol *p, const double *mean, double b1_mean, float y0[4]);
// Spatial projection: validation of the spaces, the device protocol restricted
// to contrast c, and the voxel count of a space.
mpm_status check_spaces(const mpm_protocol *p, const mpm_space *spaces);
DevProto sub_proto(const DevProto &P, int c);
inline int64_t space_voxels(const mpm_space &s) { return s.nx * s.ny * s.nz; }

// Launch wrapper: counts launches and algorithmic bytes per kernel name and,
// when timing is enabled, brackets sampled launches with events on `stream`.
struct Prof {
    struct Pending {
        int id;
        hipEvent_t a, b;
    };
    hipStream_t stream;
    std::vector<Pending> pend;
    explicit Prof(hipStream_t s) : stream(s) {}
    ~Prof();
    hipError_t launch(const char *name, double bytes, const std::function<hipError_t()> &fn);
    void collect();
};

// Stream-ordered device allocations released (and synchronised) on scope
// exit.  Given a fixed device region instead, alloc carves 256-byte aligned
// pieces out of it and allocates nothing; a request beyond its end fails with
// hipErrorOutOfMemory and records in `need` the bytes it would have taken.
struct Workspace {
    hipStream_t stream;
    std::vector<void *> bufs;
    char *arena = nullptr;
    size_t cap = 0, used = 0, need = 0;
    explicit Workspace(hipStream_t s) : stream(s) {}
    Workspace(hipStream_t s, void *region, size_t bytes) : stream(s), arena((char *)region), cap(bytes) {}
    ~Workspace();
    hipError_t alloc(void **p, size_t bytes);
};

struct FitArgs {
    const mpm_protocol *proto;
    DevProto P;
    int dtype;
    const void *X;
    const float *b1;
    const mpm_options *opt;
    float *maps;
    int64_t N, nx, ny, nz;
    hipStream_t stream;
    const mpm_space *spaces = nullptr;  // per-contrast acquisition spaces (projected fit) or NULL
    // no pinned host staging: collect() reads the results from device memory
    // with synchronous copies (the stream has completed by then)
    bool no_pinned = false;
};

// Pinned host buffer (freed with the owner).
struct PinnedBuf {
    void *p = nullptr;
    ~PinnedBuf();
    hipError_t alloc(size_t bytes);
};

// Per-image sums reduced on the device in FP64 (fixed order): rows 0..I-1 the
// sums of each image's finite values, I..2I-1 their counts, 2I the sum of b1
// (N without b1).  enqueue_image_sums leaves them in a workspace buffer of
// image_sum_rows(P) doubles; image_means_from_sums turns a host copy into the
// per-image means (each image's storage offset added) and the mean b1.
int image_sum_rows(const DevProto &P);
mpm_status enqueue_image_sums(Workspace &ws, Prof &prof, const DevProto &P, int dtype, const void *X,
                              const float *b1, int64_t N, double **sums);
void image_means_from_sums(const DevProto &P, int64_t N, const double *sums, std::vector<double> &mean,
                           double &b1m);
// Both, with one stream synchronisation.
mpm_status image_means(Workspace &ws, Prof &prof, const DevProto &P, int dtype, const void *X,
                       const float *b1, int64_t N, std::vector<double> &mean, double &b1m);

// The initial maps of a fit, in two halves so that a caller driving several
// fits never waits for the device: start() writes constant maps at once or,
// for the default initialisation, enqueues the image sums and their copy to
// pinned host memory (to device memory only, when the fit has no pinned
// staging); ready() says whether that copy has landed; finish() waits for it
// if it has not, computes the starting point on the host and enqueues the fill
// of the maps.  Given maps need neither half.
struct InitStage {
    InitStage() = default;
    InitStage(const InitStage &) = delete;
    InitStage &operator=(const InitStage &) = delete;
    ~InitStage();
    mpm_status start(const FitArgs &a, Workspace &ws, Prof &prof);
    bool ready() const;
    mpm_status finish(const FitArgs &a);
    bool pending = false;

  private:
    struct Seg {
        DevProto P;
        int64_t N;
        double *dev;  // workspace rows
        size_t at;    // first row in the host copy
    };
    std::vector<Seg> segs;
    size_t rows = 0;
    PinnedBuf host;
    hipEvent_t ev = nullptr;
};
size_t map_workspace_floats_per_voxel();

// A fit enqueued piece by piece on one stream (a piece is the whole ML fit,
// or the initialisation, one Newton-like step or the finalisation of a MAP
// fit).  collect() reads the results once all enqueued work has completed.
struct FitJob {
    virtual ~FitJob() {}
    // false while the next piece waits for host data still in flight (the
    // default initialisation); enqueue_next would then block until it lands
    virtual bool ready() const { return true; }
    virtual mpm_status enqueue_next(bool *more) = 0;
    virtual mpm_status collect(mpm_report &rep, double *trace, int trace_len) = 0;
};
std::unique_ptr<FitJob> make_ml_job(const FitArgs &a, Workspace &ws, Prof &prof, mpm_status *st);
std::unique_ptr<FitJob> make_map_job(const FitArgs &a, Workspace &ws, Prof &prof, mpm_status *st);

// Several JTV-MAP fits of one schedule enqueued together, every kernel launch
// serving all of them (batched launches); collect_item reads fit i's results
// once all enqueued work has completed.
struct BatchJob {
    virtual ~BatchJob() {}
    virtual bool ready() const { return true; }
    virtual mpm_status enqueue_next(bool *more) = 0;
    virtual mpm_status collect_item(int i, mpm_report &rep, double *trace, int trace_len) = 0;
};
std::unique_ptr<BatchJob> make_batch_job(const std::vector<FitArgs> &a, Workspace &ws, Prof &prof,
                                         mpm_status *st);
// Whether MAP fit b can share batched launches with fit a (same schedule,
// echo storage and register shape; no spatial projection).
bool batch_compatible(const FitArgs &a, const FitArgs &b);

// Runs a whole fit on a.stream with workspace ws and blocks until it is done.
mpm_status run_fit(const FitArgs &a, Workspace &ws, mpm_report *report, double *trace, int trace_len);

// Host-side validation shared by mpm_fit and the server.
mpm_status check_fit_args(const mpm_protocol *protocol, const mpm_grid *grid, int dtype, const void *echoes,
                          const mpm_options *opt, const float *maps, int64_t *N);

}  // namespace mpm
