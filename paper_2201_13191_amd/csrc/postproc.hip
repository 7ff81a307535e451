// Scatter-image post-processing of the paper's correction loop (section
// II-C-3 dual interpolation, II-C-4 smoothing): Savitzky-Golay smoothing
// (separable, rows then columns, mirrored edges) and Keys cubic up-sampling
// (a = -0.5, pixel centres aligned, clamped edges), plus the fixed-point
// tally to float conversion.  Small stencil kernels bound by memory traffic;
// one thread per output pixel, rows contiguous across a wave.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mcx {

constexpr int kMaxSgWindow = 31;

struct SgCoeffs {
    float c[kMaxSgWindow];
};

__device__ __forceinline__ int mirror_index(int i, int n) {
    if (n == 1) return 0;
    const int period = 2 * (n - 1);
    i %= period;
    if (i < 0) i += period;
    return i < n ? i : period - i;
}

// along x when `along_x`, else along y; fp32 sum in window order
__global__ void savgol_kernel(const float *in, float *out, int nx, int ny, int half,
                              SgCoeffs co, int along_x) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= nx || y >= ny) return;
    float s = 0.0f;
    if (along_x) {
        const float *row = in + (size_t)y * nx;
        for (int k = -half; k <= half; ++k) s += co.c[k + half] * row[mirror_index(x + k, nx)];
    } else {
        for (int k = -half; k <= half; ++k)
            s += co.c[k + half] * in[(size_t)mirror_index(y + k, ny) * nx + x];
    }
    out[(size_t)y * nx + x] = s;
}

__device__ __forceinline__ float keys_weight(float t) {
    t = fabsf(t);
    const float a = -0.5f;
    if (t <= 1.0f) return ((a + 2.0f) * t - (a + 3.0f)) * t * t + 1.0f;
    if (t < 2.0f) return ((a * t - 5.0f * a) * t + 8.0f * a) * t - 4.0f * a;
    return 0.0f;
}

// output (x, y) of an (nx*f) x (ny*f) image from the nx x ny input: separable
// 4 x 4 cubic convolution at input coordinate (i + 0.5)/f - 0.5
__global__ void upsample_kernel(const float *in, float *out, int nx, int ny, int f) {
    const int ox = blockIdx.x * blockDim.x + threadIdx.x;
    const int oy = blockIdx.y;
    const int mx = nx * f, my = ny * f;
    if (ox >= mx || oy >= my) return;
    const float ux = ((float)ox + 0.5f) / (float)f - 0.5f;
    const float uy = ((float)oy + 0.5f) / (float)f - 0.5f;
    const int x0 = (int)floorf(ux), y0 = (int)floorf(uy);
    float acc = 0.0f;
    for (int m = y0 - 1; m <= y0 + 2; ++m) {
        const float wy = keys_weight(uy - (float)m);
        const float *row = in + (size_t)min(max(m, 0), ny - 1) * nx;
        float r = 0.0f;
        for (int n = x0 - 1; n <= x0 + 2; ++n) r += keys_weight(ux - (float)n) * row[min(max(n, 0), nx - 1)];
        acc += wy * r;
    }
    out[(size_t)oy * mx + ox] = acc;
}

__global__ void tally_to_float_kernel(const long long *in, float *out, uint64_t n, double scale) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (float)((double)in[i] * scale);
}

hipError_t launch_savgol(const float *in, float *out, float *tmp, int nx, int ny, int window,
                         const float *coeffs, hipStream_t s) {
    SgCoeffs co{};
    for (int i = 0; i < window; ++i) co.c[i] = coeffs[i];
    const dim3 block(256), grid((nx + 255) / 256, ny);
    hipLaunchKernelGGL(savgol_kernel, grid, block, 0, s, in, tmp, nx, ny, window / 2, co, 1);
    hipLaunchKernelGGL(savgol_kernel, grid, block, 0, s, (const float *)tmp, out, nx, ny,
                       window / 2, co, 0);
    return hipGetLastError();
}

hipError_t launch_upsample(const float *in, float *out, int nx, int ny, int f, hipStream_t s) {
    const dim3 block(256), grid((nx * f + 255) / 256, ny * f);
    hipLaunchKernelGGL(upsample_kernel, grid, block, 0, s, in, out, nx, ny, f);
    return hipGetLastError();
}

// out[y][x] = alpha * in[flip_y ? ny-1-y : y][flip_x ? nx-1-x : x] + beta * out[y][x]
// (mirror images of a map, optionally accumulated; out is not read when beta
// is 0): training pairs are augmented with them and predictions averaged
__global__ void flip2d_kernel(const float *in, float *out, int nx, int ny, int fx, int fy,
                              float alpha, float beta) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= nx) return;
    const int sx = fx ? nx - 1 - x : x, sy = fy ? ny - 1 - y : y;
    const size_t o = (size_t)y * nx + x;
    const float v = alpha * in[(size_t)sy * nx + sx];
    out[o] = beta != 0.0f ? v + beta * out[o] : v;
}

hipError_t launch_flip2d(const float *in, float *out, int nx, int ny, int fx, int fy, float alpha,
                         float beta, hipStream_t s) {
    hipLaunchKernelGGL(flip2d_kernel, dim3((nx + 255) / 256, ny), dim3(256), 0, s, in, out, nx,
                       ny, fx, fy, alpha, beta);
    return hipGetLastError();
}

hipError_t launch_tally_to_float(const int64_t *in, float *out, uint64_t n, double scale,
                                 hipStream_t s) {
    uint64_t grid = (n + 255) / 256;
    if (grid > 8192) grid = 8192;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL(tally_to_float_kernel, dim3((unsigned)grid), dim3(256), 0, s,
                       (const long long *)in, out, n, scale);
    return hipGetLastError();
}

}  // namespace mcx
