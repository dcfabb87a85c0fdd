// mpm_api_internal.h -- host-side helpers shared by libmpm's C-ABI sources.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
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
DevProto to_dev(const mpm_protocol *p);
size_t dtype_size(int dtype);
mpm_status default_init_from_means(const mpm_protocol *p, const double *mean, double b1_mean, float y0[4]);

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

// Stream-ordered device allocations released (and synchronised) on scope exit.
struct Workspace {
    hipStream_t stream;
    std::vector<void *> bufs;
    explicit Workspace(hipStream_t s) : stream(s) {}
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
};

mpm_status image_means(Workspace &ws, Prof &prof, const DevProto &P, int dtype, const void *X,
                       const float *b1, int64_t N, std::vector<double> &mean, double &b1m);
mpm_status fit_ml(const FitArgs &a, Workspace &ws, Prof &prof, mpm_report &rep, double *trace,
                  int trace_len);
mpm_status fit_map(const FitArgs &a, Workspace &ws, Prof &prof, mpm_report &rep, double *trace,
                   int trace_len);
size_t map_workspace_floats_per_voxel();

}  // namespace mpm
