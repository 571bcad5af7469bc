// Roofline probes used by the benchmark: the rate of independent random
// 64-byte-sector reads over a buffer far larger than the caches (the gather
// roofline of a hop), and a plain streaming copy of known size (bandwidth,
// and the reference for scaling hardware byte counters).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__device__ __forceinline__ uint64_t mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Each thread issues `iters` independent 16-byte loads, each from a random
// 64-byte-aligned sector of buf (n_sectors sectors).
__global__ void __launch_bounds__(256) k_gather(const uint4* __restrict__ buf, uint64_t n_sectors,
                                                uint64_t seed, int iters,
                                                unsigned int* __restrict__ sink) {
    uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t x = mix(seed ^ (tid * 0x9E3779B97F4A7C15ull));
    unsigned int acc = 0;
#pragma unroll 8
    for (int i = 0; i < iters; ++i) {
        x += 0x9E3779B97F4A7C15ull;
        uint64_t s = __umul64hi(mix(x), n_sectors);
        uint4 v = buf[s * 4];
        acc ^= v.x ^ v.w;
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

__global__ void __launch_bounds__(256) k_copy(const uint4* __restrict__ in, uint4* __restrict__ out,
                                              uint64_t n) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = in[i];
}

}  // namespace

extern "C" {

// Random-sector gather over buf (bytes, multiple of 64): threads x iters
// loads on stream. Returns 0 or a hipError_t.
int probe_gather(const void* buf, uint64_t bytes, uint64_t threads, int iters, uint64_t seed,
                 void* sink, void* stream) {
    uint64_t blocks = (threads + 255) / 256;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const uint4*)buf, bytes / 64, seed, iters, (unsigned int*)sink);
    return (int)hipGetLastError();
}

// Copy bytes (multiple of 16) from in to out on stream.
int probe_copy(const void* in, void* out, uint64_t bytes, void* stream) {
    uint64_t n = bytes / 16;
    hipLaunchKernelGGL(k_copy, dim3(256 * 8 * 4), dim3(256), 0, (hipStream_t)stream,
                       (const uint4*)in, (uint4*)out, n);
    return (int)hipGetLastError();
}

}  // extern "C"
