// Tally probe: a measuring instrument for the transport's int64 tally
// atomics (not part of the method).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mcx {

// int64 atomic adds of 1 spread uniformly over an image (pixel of
// add i from a 32-bit integer hash of i and the seed, scaled to the image by a
// high multiply), a grid-stride loop with nothing else in it.
__device__ __forceinline__ uint32_t probe_hash(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(256) atomic_probe_kernel(unsigned long long *img, uint32_t n_pix,
                                                           unsigned long long n, uint32_t seed) {
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride) {
        const uint32_t h = probe_hash((uint32_t)i ^ seed ^ ((uint32_t)(i >> 32) * 0x9E3779B9u));
        atomicAdd(img + __umulhi(h, n_pix), 1ull);
    }
}

hipError_t launch_atomic_probe(unsigned long long *img, uint32_t n_pix, unsigned long long n,
                               uint32_t seed, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(atomic_probe_kernel, dim3(grid), dim3(256), 0, stream, img, n_pix, n, seed);
    return hipGetLastError();
}

}  // namespace mcx
