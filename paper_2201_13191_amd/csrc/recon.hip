// Reconstruction side of the iterative scatter correction (section II-E and its
// flowchart): line integrals of the measured intensities, the Feldkamp-Davis-
// Kress filtered backprojection of the projector's circular orbit, a histogram
// for Otsu's threshold, volume to density, and eq. (8),
// c = a - ln(Ip / (Ip + Is)).  All of it is bandwidth-light next to the
// Monte Carlo: the filter is a row convolution staged in LDS, the
// backprojection one thread per voxel over all angles.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mcx {

struct FdkGeom {
    double R, D;           // source to axis, source to panel
    double pu, pv;         // panel pitch
    int nu, nv, n_ang;
};

// a = -ln(I / I0), I0 per panel pixel (n0 of them, repeated for each projection)
__global__ void line_integrals_kernel(const float *I, uint64_t n, const float *I0, uint64_t n0,
                                      float *a) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double v = (double)I[i];
        v = v > 1e-30 ? v : 1e-30;
        a[i] = (float)(-log(v / (double)I0[i % n0]));
    }
}

// eq. (8)
__global__ void scatter_correct_kernel(const float *a, const float *ip, const float *is,
                                       uint64_t n, float *c) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double p = (double)ip[i];
        c[i] = (float)((double)a[i] - log(p / (p + (double)is[i])));
    }
}

// One block per panel row of one projection: the row, cosine-weighted on the
// virtual panel through the axis (coordinates scaled by R / D), is staged in
// LDS; each thread convolves it with the discrete Ram-Lak kernel of the virtual
// pitch t at its own pixels (fp64 sums): h(0) = 1/(4 t^2), h(odd d) =
// -1/(d pi t)^2, times t.
__global__ void fdk_filter_kernel(const float *proj, FdkGeom g, float *q) {
    extern __shared__ double row[];
    const int r = blockIdx.x % g.nv, i = blockIdx.x / g.nv;
    const double s = g.R / g.D, t = g.pu * s;
    const double b = (-(double)g.nv * g.pv / 2 + (r + 0.5) * g.pv) * s;
    const float *src = proj + ((size_t)i * g.nv + r) * g.nu;
    for (int k = threadIdx.x; k < g.nu; k += blockDim.x) {
        const double a = (-(double)g.nu * g.pu / 2 + (k + 0.5) * g.pu) * s;
        row[k] = (double)src[k] * (g.R / sqrt(g.R * g.R + a * a + b * b));
    }
    __syncthreads();
    const double pi = 3.141592653589793;
    for (int j = threadIdx.x; j < g.nu; j += blockDim.x) {
        double acc = row[j] * (1.0 / (4.0 * t * t));
        // odd offsets: j - k = +-1, +-3, ...
        for (int d = 1; d < g.nu; d += 2) {
            const double w = -1.0 / ((d * pi * t) * (d * pi * t));
            double x = 0.0;
            if (j - d >= 0) x += row[j - d];
            if (j + d < g.nu) x += row[j + d];
            acc += w * x;
        }
        q[((size_t)i * g.nv + r) * g.nu + j] = (float)(acc * t);
    }
}

// One thread per voxel: f = 1/2 (2 pi / n) sum_i R^2 / L^2 q_i(a, b), the
// filtered projections read by bilinear interpolation between pixel centres
// (zero outside the panel); cos/sin of the angles precomputed per block in LDS.
__global__ void fdk_backproject_kernel(const float *q, FdkGeom g, int nx, int ny, int nz,
                                       double h, float *vol) {
    extern __shared__ double cs[];   // [2 * n_ang]
    for (int i = threadIdx.x; i < g.n_ang; i += blockDim.x) {
        double sb, cb;
        sincos(2.0 * 3.141592653589793 * i / g.n_ang, &sb, &cb);
        cs[2 * i] = cb;
        cs[2 * i + 1] = sb;
    }
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (int64_t)nx * ny * nz) return;
    const int ix = (int)(v % nx), iy = (int)((v / nx) % ny), iz = (int)(v / ((int64_t)nx * ny));
    const double X = (ix + 0.5) * h - nx * h / 2, Y = (iy + 0.5) * h - ny * h / 2,
                 Z = (iz + 0.5) * h - nz * h / 2;
    const double s = g.R / g.D;
    double f = 0.0;
    for (int i = 0; i < g.n_ang; ++i) {
        const double cb = cs[2 * i], sb = cs[2 * i + 1];
        const double L = g.R - (X * cb + Y * sb);
        const double av = g.R * (-X * sb + Y * cb) / L;
        const double bv = g.R * Z / L;
        const double fu = (av / s + g.nu * g.pu / 2) / g.pu - 0.5;
        const double fv = (bv / s + g.nv * g.pv / 2) / g.pv - 0.5;
        // off the panel by more than a pixel: no contribution (also keeps the
        // integer conversions below in range)
        if (!(fu > -2.0 && fu < g.nu + 1.0 && fv > -2.0 && fv < g.nv + 1.0)) continue;
        const double u0 = floor(fu), v0 = floor(fv);
        const double wu = fu - u0, wv = fv - v0;
        const int iu = (int)u0, iv = (int)v0;
        const float *qi = q + (size_t)i * g.nv * g.nu;
        double val = 0.0;
        if (iv >= 0 && iv < g.nv) {
            if (iu >= 0 && iu < g.nu) val += (double)qi[(size_t)iv * g.nu + iu] * ((1 - wu) * (1 - wv));
            if (iu + 1 >= 0 && iu + 1 < g.nu) val += (double)qi[(size_t)iv * g.nu + iu + 1] * (wu * (1 - wv));
        }
        if (iv + 1 >= 0 && iv + 1 < g.nv) {
            if (iu >= 0 && iu < g.nu) val += (double)qi[(size_t)(iv + 1) * g.nu + iu] * ((1 - wu) * wv);
            if (iu + 1 >= 0 && iu + 1 < g.nu) val += (double)qi[(size_t)(iv + 1) * g.nu + iu + 1] * (wu * wv);
        }
        f += (g.R * g.R) / (L * L) * val;
    }
    vol[v] = (float)(0.5 * (2.0 * 3.141592653589793 / g.n_ang) * f);
}

// counts of x in [lo, hi) in `bins` equal bins, bin floor((x - lo) / (hi - lo) * bins)
__global__ void histogram_kernel(const float *x, uint64_t n, double lo, double hi, int bins,
                                 unsigned int *hist) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double k = floor(((double)x[i] - lo) / (hi - lo) * bins);
        if (k >= 0.0 && k < (double)bins) atomicAdd(hist + (int)k, 1u);
    }
}

__global__ void zero_u32_kernel(unsigned int *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// voxels with mu >= threshold: `material` with density mu / (0.1 mu/rho) rounded
// to multiples of step (half to even); the others air
__global__ void to_density_kernel(const float *mu, uint64_t n, double threshold, double mu_rho,
                                  int material, double air_rho, double step, uint8_t *ids,
                                  float *rho) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double m = (double)mu[i];
        const bool obj = m >= threshold;
        ids[i] = obj ? (uint8_t)material : (uint8_t)0;
        rho[i] = (float)(obj ? __builtin_rint(m / (0.1 * mu_rho) / step) * step : air_rho);
    }
}

static unsigned grid_for(uint64_t n) {
    uint64_t g = (n + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

hipError_t launch_line_integrals(const float *I, uint64_t n, const float *I0, uint64_t n0,
                                 float *a, hipStream_t s) {
    hipLaunchKernelGGL(line_integrals_kernel, dim3(grid_for(n)), dim3(256), 0, s, I, n, I0, n0, a);
    return hipGetLastError();
}

hipError_t launch_scatter_correct(const float *a, const float *ip, const float *is, uint64_t n,
                                  float *c, hipStream_t s) {
    hipLaunchKernelGGL(scatter_correct_kernel, dim3(grid_for(n)), dim3(256), 0, s, a, ip, is, n, c);
    return hipGetLastError();
}

hipError_t launch_fdk(const float *proj, double R, double D, double pu, double pv, int nu, int nv,
                      int n_ang, float *q, int nx, int ny, int nz, double h, float *vol,
                      hipStream_t s) {
    const FdkGeom g{R, D, pu, pv, nu, nv, n_ang};
    hipLaunchKernelGGL(fdk_filter_kernel, dim3((unsigned)(n_ang * nv)), dim3(256),
                       (size_t)nu * sizeof(double), s, proj, g, q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nvox = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL(fdk_backproject_kernel, dim3((unsigned)((nvox + 255) / 256)), dim3(256),
                       (size_t)2 * n_ang * sizeof(double), s, q, g, nx, ny, nz, h, vol);
    return hipGetLastError();
}

hipError_t launch_histogram(const float *x, uint64_t n, double lo, double hi, int bins,
                            unsigned int *hist, hipStream_t s) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((bins + 255) / 256)), dim3(256), 0, s,
                       hist, bins);
    hipLaunchKernelGGL(histogram_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, lo, hi, bins,
                       hist);
    return hipGetLastError();
}

hipError_t launch_to_density(const float *mu, uint64_t n, double threshold, double mu_rho,
                             int material, double air_rho, double step, uint8_t *ids, float *rho,
                             hipStream_t s) {
    hipLaunchKernelGGL(to_density_kernel, dim3(grid_for(n)), dim3(256), 0, s, mu, n, threshold,
                       mu_rho, material, air_rho, step, ids, rho);
    return hipGetLastError();
}

}  // namespace mcx
