// mpm_noalloc.hip -- mpm_fit_noalloc: the fit of mpm_fit with its whole
// workspace in a fixed device array, for callers that cannot allocate.
//
// The array lives in the library's code object; each device that runs the
// library holds its own copy at its own address until the process ends.  In
// host code its name stands for a host-side shadow, not for device memory, so
// the device address is taken once per device with hipGetSymbolAddress and
// only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "mpm_api_internal.h"

using namespace mpm;

namespace {

static __device__ __align__(256) unsigned char scratch[MPM_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_addr_mu;
void *g_addr[MAX_DEVICES];             // device address of scratch, per device
std::mutex g_call_mu[MAX_DEVICES];     // one fit at a time per device

// Device address of this device's scratch (the current device).
mpm_status scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(g_addr_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MPM_ERR_DEVICE, "mpm_fit_noalloc: scratch address: %s", hipGetErrorString(e));
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return MPM_OK;
}

}  // namespace

extern "C" mpm_status mpm_fit_noalloc(const mpm_protocol *protocol, const mpm_grid *grid, mpm_dtype dtype,
                                      const void *echoes, const float *b1, const mpm_options *opt, float *maps,
                                      mpm_report *report, double *trace, int32_t trace_len, void *stream)
{
    clear_error();
    int64_t N;
    mpm_status st = check_fit_args(protocol, grid, dtype, echoes, opt, maps, &N);
    if (st) return st;
    if (trace_len < 0 || (trace_len > 0 && !trace)) return fail(MPM_ERR_INVALID_ARG, "trace is NULL");
    for (int i = 0; i < trace_len; i++) trace[i] = NAN;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(MPM_ERR_DEVICE, "mpm_fit_noalloc: no HIP device");
    if (dev >= MAX_DEVICES) return fail(MPM_ERR_UNSUPPORTED, "mpm_fit_noalloc: device %d beyond %d", dev, MAX_DEVICES);
    void *base = nullptr;
    if ((st = scratch_address(dev, &base))) return st;
    std::lock_guard<std::mutex> lk(g_call_mu[dev]);  // held until the workspace's stream has drained
    hipStream_t s = (hipStream_t)stream;
    FitArgs a{protocol, to_dev(protocol, opt->echo_offset), dtype, echoes, b1, opt, maps, N,
              grid->nx, grid->ny, grid->nz, s};
    a.no_pinned = true;
    Workspace ws(s, base, MPM_NOALLOC_SCRATCH_BYTES);
    st = run_fit(a, ws, report, trace, trace_len);
    if (st == MPM_ERR_OUT_OF_MEMORY && ws.need > 0)
        return fail(MPM_ERR_OUT_OF_MEMORY,
                    "mpm_fit_noalloc: this fit needs more than the library's fixed %zu-byte scratch "
                    "(%zu bytes or more; a MAP fit takes about 124 bytes per voxel)",
                    (size_t)MPM_NOALLOC_SCRATCH_BYTES, ws.need);
    return st;
}
