// valu_probe.hip -- achievable VALU issue rate of this GPU for the instruction
// mixes of the voxelwise kernels: the ceiling against which the measured
// instruction rates of the ML fits are read.
//
// Each thread runs 8 independent dependency chains for a fixed number of
// steps (enough resident wavefronts to hide the latency), and writes one sum:
//   fma    v_fma_f32 (non-packed FP32: packed FP32 is disabled at compile time)
//   exp2   v_exp_f32 (transcendental)
// Timed with HIP events (2 warm-up launches, then the median of 8); one JSON
// line per mix with the rate in wave64 instructions per clock per CU, lane
// instructions per second, and FLOP/s for the FMA mix.
// Usage: valu_probe [clock GHz, default 2.4].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                                       \
    do {                                                                                               \
        hipError_t e_ = (x);                                                                           \
        if (e_ != hipSuccess) {                                                                        \
            std::fprintf(stderr, "valu_probe: %s at line %d\n", hipGetErrorString(e_), __LINE__);       \
            std::exit(1);                                                                              \
        }                                                                                              \
    } while (0)

constexpr int CHAINS = 8;

__global__ __launch_bounds__(256) void k_fma(int steps, float m, float c, float *__restrict__ out)
{
    float a[CHAINS];
#pragma unroll
    for (int k = 0; k < CHAINS; k++) a[k] = (float)(threadIdx.x + k);
    for (int s = 0; s < steps; s++) {
#pragma unroll
        for (int k = 0; k < CHAINS; k++) a[k] = fmaf(a[k], m, c);
    }
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < CHAINS; k++) t += a[k];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_exp2(int steps, float m, float c, float *__restrict__ out)
{
    float a[CHAINS];
#pragma unroll
    for (int k = 0; k < CHAINS; k++) a[k] = 1e-3f * (float)(threadIdx.x + k);
    for (int s = 0; s < steps; s++) {
#pragma unroll
        for (int k = 0; k < CHAINS; k++) a[k] = __builtin_amdgcn_exp2f(a[k] * m) - c;
    }
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < CHAINS; k++) t += a[k];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = t;
}

int main(int argc, char **argv)
{
    const double ghz = argc > 1 ? std::atof(argv[1]) : 2.4;
    int dev = 0, cus = 0;
    CHECK(hipGetDevice(&dev));
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = cus * 32, threads = 256, steps = 20000;  // 32 wavefronts per CU
    float *out = nullptr;
    CHECK(hipMalloc(&out, sizeof(float) * (size_t)blocks * threads));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    for (int mix = 0; mix < 2; mix++) {
        std::vector<float> ms;
        for (int r = 0; r < 10; r++) {
            CHECK(hipEventRecord(e0));
            if (mix == 0)
                hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(threads), 0, 0, steps, 0.999f, 1e-3f, out);
            else
                hipLaunchKernelGGL(k_exp2, dim3(blocks), dim3(threads), 0, 0, steps, 0.5f, 0.9f, out);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(e1));
            CHECK(hipEventSynchronize(e1));
            float t = 0.0f;
            CHECK(hipEventElapsedTime(&t, e0, e1));
            if (r >= 2) ms.push_back(t);
        }
        std::sort(ms.begin(), ms.end());
        const double t = 0.5 * (ms[3] + ms[4]) * 1e-3;
        // the mix's own instructions (the loop's counter and branch aside)
        const double lane_insts = (double)blocks * threads * steps * CHAINS * (mix == 0 ? 1.0 : 2.0);
        const double wave_per_clk_cu = lane_insts / 64.0 / t / (ghz * 1e9) / cus;
        std::printf("{\"mix\": \"%s\", \"seconds\": %.6f, \"lane_insts_per_s\": %.4g, "
                    "\"wave64_insts_per_clock_per_cu\": %.3f, \"cus\": %d, \"clock_ghz\": %.2f%s}\n",
                    mix == 0 ? "fma" : "exp2_and_sub", t, lane_insts / t, wave_per_clk_cu, cus, ghz,
                    mix == 0 ? "" : ", \"note\": \"each step is one v_exp_f32 and one subtraction\"");
        if (mix == 0) std::printf("{\"mix\": \"fma\", \"TFLOPs\": %.2f}\n", 2.0 * lane_insts / t / 1e12);
    }
    CHECK(hipFree(out));
    return 0;
}
