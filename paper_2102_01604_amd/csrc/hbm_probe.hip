// hbm_probe.hip -- achievable HBM bandwidth of plain streaming kernels on this
// GPU, the ceiling against which the MAP sweeps' measured rates are read.
//
// Four float4 streams over 2 GiB buffers (far beyond every cache level), each
// a grid-stride loop bounded by the element count, with non-temporal loads and
// stores as the sweeps use them:
//   read   1 stream in            copy   1 in, 1 out
//   write  1 stream out           mix    3 in, 2 out (a CG-update-like mix)
// Each is timed with HIP events (2 warm-up launches, then the median of 8) at
// 1024 threads per workgroup for several grid sizes; one JSON line per stream
// reports the best median.  Usage: hbm_probe [GiB per buffer, default 2].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

typedef float v4 __attribute__((ext_vector_type(4)));

#define CHECK(x)                                                                              \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            std::fprintf(stderr, "hbm_probe: %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            std::exit(1);                                                                     \
        }                                                                                     \
    } while (0)

__global__ __launch_bounds__(1024) void k_read(const v4 *__restrict__ a, size_t n, float *__restrict__ sink)
{
    v4 s = {0.f, 0.f, 0.f, 0.f};
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        s += __builtin_nontemporal_load(a + i);
    const float t = s.x + s.y + s.z + s.w;
    if (t == 1234.5f) sink[blockIdx.x] = t;  // the buffers hold zeros: keeps the loads, never stores
}

__global__ __launch_bounds__(1024) void k_write(v4 *__restrict__ a, size_t n)
{
    const v4 v = {0.f, 0.f, 0.f, 0.f};
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(v, a + i);
}

__global__ __launch_bounds__(1024) void k_copy(const v4 *__restrict__ a, v4 *__restrict__ b, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

__global__ __launch_bounds__(1024) void k_mix(const v4 *__restrict__ a, v4 *__restrict__ b, v4 *__restrict__ c,
                                              size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const v4 x = __builtin_nontemporal_load(a + i);
        const v4 y = __builtin_nontemporal_load(b + i);
        const v4 z = __builtin_nontemporal_load(c + i);
        __builtin_nontemporal_store(x + 0.5f * y, b + i);
        __builtin_nontemporal_store(z - 0.25f * x, c + i);
    }
}

int main(int argc, char **argv)
{
    const double gib = argc > 1 ? std::atof(argv[1]) : 2.0;
    if (!(gib >= 0.0625 && gib <= 16.0)) {
        std::fprintf(stderr, "hbm_probe: buffer size must be in [1/16, 16] GiB\n");
        return 2;
    }
    const size_t bytes = (size_t)(gib * (1u << 30)) & ~(size_t)4095;
    const size_t n = bytes / sizeof(v4);
    v4 *a, *b, *c;
    float *sink;
    CHECK(hipMalloc(&a, bytes));
    CHECK(hipMalloc(&b, bytes));
    CHECK(hipMalloc(&c, bytes));
    CHECK(hipMalloc(&sink, 1 << 20));
    CHECK(hipMemset(a, 0, bytes));
    CHECK(hipMemset(b, 0, bytes));
    CHECK(hipMemset(c, 0, bytes));
    CHECK(hipDeviceSynchronize());
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const int grids[] = {1024, 2048, 4096, 8192, 16384};  // sink holds >= 16384 floats

    auto run = [&](const char *name, double moved, auto launch) {
        double best = 0.0;
        int best_grid = 0;
        for (int grid : grids) {
            std::vector<float> ms;
            for (int r = 0; r < 10; r++) {
                CHECK(hipEventRecord(e0));
                launch(grid);
                CHECK(hipGetLastError());
                CHECK(hipEventRecord(e1));
                CHECK(hipEventSynchronize(e1));
                float t;
                CHECK(hipEventElapsedTime(&t, e0, e1));
                if (r >= 2) ms.push_back(t);
            }
            std::sort(ms.begin(), ms.end());
            const double gbps = moved / (ms[ms.size() / 2] * 1e-3) / 1e9;
            if (gbps > best) {
                best = gbps;
                best_grid = grid;
            }
        }
        std::printf("{\"stream\": \"%s\", \"GBps\": %.1f, \"bytes\": %.0f, \"workgroups\": %d, \"threads\": 1024}\n",
                    name, best, moved, best_grid);
        std::fflush(stdout);
    };
    run("read", (double)bytes, [&](int g) { hipLaunchKernelGGL(k_read, dim3(g), dim3(1024), 0, 0, a, n, sink); });
    run("write", (double)bytes, [&](int g) { hipLaunchKernelGGL(k_write, dim3(g), dim3(1024), 0, 0, b, n); });
    run("copy", 2.0 * bytes, [&](int g) { hipLaunchKernelGGL(k_copy, dim3(g), dim3(1024), 0, 0, a, b, n); });
    run("mix_3r_2w", 5.0 * bytes, [&](int g) { hipLaunchKernelGGL(k_mix, dim3(g), dim3(1024), 0, 0, a, b, c, n); });
    CHECK(hipDeviceSynchronize());
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    CHECK(hipFree(c));
    CHECK(hipFree(sink));
    return 0;
}
