// mpm_stream.h -- streaming reads of whole echo images: 16-byte loads of the
// aligned middle of an image (several in flight per thread), single values at
// its ragged ends.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "mpm_device.h"

namespace mpm {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The values of T held in one 16-byte word (V of them), unpacked from registers.
template <typename T>
struct Unpack;
template <>
struct Unpack<float> {
    static constexpr int V = 4;
    static __device__ __forceinline__ float get(const u32x4 &w, int e) { return __uint_as_float(w[e]); }
};
__device__ __forceinline__ uint32_t half_bits(const u32x4 &w, int e)
{
    const uint32_t u = w[e >> 1];
    return (e & 1) ? u >> 16 : u & 0xffffu;
}
template <>
struct Unpack<F16> {
    static constexpr int V = 8;
    static __device__ __forceinline__ float get(const u32x4 &w, int e)
    {
        const uint16_t b = (uint16_t)half_bits(w, e);
        _Float16 h;
        __builtin_memcpy(&h, &b, 2);
        return (float)h;
    }
};
template <>
struct Unpack<BF16> {
    static constexpr int V = 8;
    static __device__ __forceinline__ float get(const u32x4 &w, int e)
    {
        return __uint_as_float(half_bits(w, e) << 16);
    }
};

// Calls f(v) for every value of one image x [N]: the 16-byte aligned middle
// with 16-byte loads (four in flight per thread), the ragged ends one value
// at a time.  Work is spread over the workgroups of grid dimension x.
template <typename T, typename F>
__device__ __forceinline__ void for_each_value(const T *__restrict__ x, int64_t N, F &&f)
{
    constexpr int V = Unpack<T>::V;  // values per 16-byte load
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    const int64_t mis = (int64_t)(((uintptr_t)x >> (sizeof(T) == 4 ? 2 : 1)) & (V - 1));
    const int64_t head = mis ? std::min<int64_t>(V - mis, N) : 0;
    const int64_t nvec = (N - head) / V;
    for (int64_t n = tid; n < head; n += nth) f(load_echo(x + n));
    const u32x4 *xv = (const u32x4 *)(x + head);
    int64_t q = tid;
    for (; q + 3 * nth < nvec; q += 4 * nth) {
        u32x4 w[4];
#pragma unroll
        for (int u = 0; u < 4; u++) w[u] = __builtin_nontemporal_load(xv + q + u * nth);
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int e = 0; e < V; e++) f(Unpack<T>::get(w[u], e));
    }
    for (; q < nvec; q += nth) {
        const u32x4 w = __builtin_nontemporal_load(xv + q);
#pragma unroll
        for (int e = 0; e < V; e++) f(Unpack<T>::get(w, e));
    }
    for (int64_t n = head + nvec * V + tid; n < N; n += nth) f(load_echo(x + n));
}

}  // namespace mpm
