// Analog Monte Carlo photon transport on gfx950: cone-beam point source,
// fixed-step march through a voxel object, photoelectric / Rayleigh (eq. (2))
// / Compton (eq. (1), Kahn's method) events, primary and scatter tallies on a
// flat panel (arXiv 2201.13191, section II-A; step size section II-C-2).
//
// Execution model: a persistent grid.  Each lane carries one photon; a wave
// refills its dead lanes from a global photon counter with one atomic per
// wave (ballot + popcount + prefix count), so lanes never wait for the
// wave's longest history.  Each scheduling round (1) starts flights for
// lanes that need one, (2) marches every flying lane up to
// `steps_per_round` fixed steps, (3) handles the lanes whose flight ended:
// an interaction (type draw, angle sampling, rotation) or an exit (panel
// crossing and tally).
//
// Reproducibility: every photon owns a Philox4x32-10 stream (key = seed,
// counter = photon id, draw index / 4), all fp32 state is updated with
// separately rounded operations (built with -ffp-contract=off), the samplers
// use fp64 with correctly rounded + - * / and round once, transcendentals
// are fp64 rounded to fp32, and tallies are int64 fixed point added with
// atomics.  A photon's history therefore does not depend on which lane,
// wave or round runs it, and images do not depend on the launch shape.
#include <hip/hip_runtime.h>

#include "kernel_params.hpp"

namespace mcx {

// ------------------------------------------------------------------ RNG
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// odd multiples of 2^-24 in (0, 1): exact in fp32
__device__ __forceinline__ float unit_float(uint32_t x) {
    return (float)(2u * (x >> 9) + 1u) * 5.9604644775390625e-8f;
}

struct PhotonStream {
    uint32_t id_lo, id_hi, key0, key1;
    uint32_t next;     // index of the next draw
    uint32_t cached;   // block index held in blk
    uint4 blk;

    __device__ void reset(uint64_t photon, uint32_t k0, uint32_t k1) {
        id_lo = (uint32_t)photon;
        id_hi = (uint32_t)(photon >> 32);
        key0 = k0;
        key1 = k1;
        next = 0;
        cached = 0xFFFFFFFFu;
    }
    __device__ uint32_t raw() {
        const uint32_t b = next >> 2;
        if (b != cached) {
            blk = philox4x32_10(make_uint4(id_lo, id_hi, b, 0u), key0, key1);
            cached = b;
        }
        const uint32_t w = next & 3u;
        ++next;
        return w == 0u ? blk.x : (w == 1u ? blk.y : (w == 2u ? blk.z : blk.w));
    }
    __device__ float u() { return unit_float(raw()); }
};

// ------------------------------------------------------------------ tables
__device__ __forceinline__ float grid_lerp(const float *t, int J, float e) {
    const float x = e - 1.0f;
    int j = (int)x;
    j = j < 0 ? 0 : (j > J - 2 ? J - 2 : j);
    const float f = x - (float)j;
    return t[j] + f * (t[j + 1] - t[j]);
}

// per-lane linear attenuation per material at energy e, mm^-1 per g/cm^3
__device__ __forceinline__ void material_mu(const KParams &p, float e, float *mm, int stride) {
    for (int m = 0; m < p.n_mat; ++m) {
        const int o = m * p.J;
        const float a = grid_lerp(p.pe + o, p.J, e);
        const float b = grid_lerp(p.coh + o, p.J, e);
        const float c = grid_lerp(p.inc + o, p.J, e);
        mm[m * stride] = ((a + b) + c) * 0.1f;
    }
}

// ------------------------------------------------------------------ samplers
// Kahn's rejection method for the Klein-Nishina polar angle: x = E/E' drawn
// from one of two branches and accepted against the KN shape.
__device__ void sample_compton(PhotonStream &s, float e, float &ct, float &e_out) {
    const double a = (double)e / 510.99895;
    const double top = 1.0 + 2.0 * a;
    const double branch = top / (9.0 + 2.0 * a);
    double x;
    for (;;) {
        const double r1 = (double)s.u();
        const double r2 = (double)s.u();
        const double r3 = (double)s.u();
        if (r1 <= branch) {
            x = 1.0 + 2.0 * a * r2;
            if (r3 <= 4.0 * (1.0 / x - 1.0 / (x * x))) break;
        } else {
            x = top / (1.0 + 2.0 * a * r2);
            const double c = 1.0 - (x - 1.0) / a;
            if (r3 <= 0.5 * (c * c + 1.0 / x)) break;
        }
    }
    e_out = (float)((double)e / x);
    ct = (float)(1.0 - (x - 1.0) / a);
}

// Rayleigh polar angle: v = sin^2(theta/2)/lambda^2 inverted from the
// (1 + b v)^-4 form-factor weight, accepted with (1 + cos^2)/2 evaluated on
// the fp32 cosine.
__device__ float sample_rayleigh(PhotonStream &s, float e, double b) {
    const double t = (double)e / 12.398419843320026;
    const double V = t * t;
    const double W = 1.0 + b * V;
    const double ymin = 1.0 / (W * W * W);
    for (;;) {
        const double r1 = (double)s.u();
        const double r2 = (double)s.u();
        const double y = 1.0 - r1 * (1.0 - ymin);
        const double v = (1.0 / cbrt(y) - 1.0) / b;
        const float cf = (float)(1.0 - 2.0 * v / V);
        const double cd = (double)cf;
        if (r2 <= 0.5 * (1.0 + cd * cd)) return cf;
    }
}

__device__ __forceinline__ void scatter_direction(float &dx, float &dy, float &dz, float ct,
                                                  float cp, float sp) {
    const float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
    float nx, ny, nz;
    if (fabsf(dz) < 0.99999f) {
        const float t = sqrtf(1.0f - dz * dz);
        nx = st * ((dx * dz) * cp - dy * sp) / t + dx * ct;
        ny = st * ((dy * dz) * cp + dx * sp) / t + dy * ct;
        nz = dz * ct - (st * cp) * t;
    } else {
        nx = st * cp;
        ny = st * sp;
        nz = dz >= 0.0f ? ct : -ct;
    }
    const float inv = 1.0f / sqrtf((nx * nx + ny * ny) + nz * nz);
    dx = nx * inv;
    dy = ny * inv;
    dz = nz * inv;
}

__device__ __forceinline__ uint32_t pick_bin(const KParams &p, uint32_t x) {
    int lo = 0, hi = p.n_bins - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((uint64_t)x < p.thr[mid]) hi = mid; else lo = mid + 1;
    }
    return (uint32_t)lo;
}

// ------------------------------------------------------------------ geometry
__device__ __forceinline__ bool box_entry(const KParams &p, const float o[3], const float d[3],
                                          float &tin, float &tout) {
    float t0 = 0.0f, t1 = __builtin_inff();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0f) {
            const float inv = 1.0f / d[a];
            const float ta = (p.lo[a] - o[a]) * inv;
            const float tb = (p.hi[a] - o[a]) * inv;
            const float tn = ta < tb ? ta : tb;
            const float tf = ta < tb ? tb : ta;
            if (tn > t0) t0 = tn;
            if (tf < t1) t1 = tf;
        } else if (o[a] < p.lo[a] || o[a] > p.hi[a]) {
            return false;
        }
    }
    tin = t0;
    tout = t1;
    return t0 < t1;
}

__device__ __forceinline__ bool panel_hit(const KParams &p, const float o[3], const float d[3],
                                          int &iu, int &iv) {
    const ProjFrame &F = p.F;
    const float den = (d[0] * F.ax[0] + d[1] * F.ax[1]) + d[2] * F.ax[2];
    if (!(den > 0.0f)) return false;
    const float rel = ((o[0] - F.S[0]) * F.ax[0] + (o[1] - F.S[1]) * F.ax[1]) +
                      (o[2] - F.S[2]) * F.ax[2];
    const float td = (p.sdd - rel) / den;
    const float w0 = (o[0] + td * d[0]) - F.D[0];
    const float w1 = (o[1] + td * d[1]) - F.D[1];
    const float w2 = (o[2] + td * d[2]) - F.D[2];
    const float u = (w0 * F.eu[0] + w1 * F.eu[1]) + w2 * F.eu[2];
    const float v = (w0 * F.ev[0] + w1 * F.ev[1]) + w2 * F.ev[2];
    const float fu = (u + F.hu) / p.pu;
    const float fv = (v + F.hv) / p.pv;
    if (!(fu >= 0.0f && fu < (float)p.nu && fv >= 0.0f && fv < (float)p.nv)) return false;
    iu = (int)fu;
    iv = (int)fv;
    return true;
}

// ------------------------------------------------------------------ kernels
enum : int { kStHist, kStSteps, kStFlights, kStPhoto, kStRayl, kStCompt, kStPrim, kStScat,
             kStCut, kStCap, kStCount };

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <bool STATS, bool DEBUG>
__global__ void __launch_bounds__(256) transport_kernel(const KParams p) {
    extern __shared__ float lds_mu[];        // [n_mat][blockDim]: lane-private columns
    const int bs = blockDim.x;
    float *mm = lds_mu + threadIdx.x;
    const int lane = (int)__lane_id();

    bool alive = false, flying = false, exhausted = false;
    PhotonStream rng;
    uint64_t pid = 0;
    float e = 0.0f;
    float o[3] = {0.0f, 0.0f, 0.0f}, d[3] = {0.0f, 0.0f, 0.0f};
    float pin[3], q[3], g[3];
    float len = 0.0f, tau = 0.0f, tau_star = 0.0f;
    uint32_t k = 0;
    int n_int = 0, mat = 0;
    unsigned long long st[kStCount] = {};
    uint32_t h_steps = 0;
    uint8_t h_first = 0;

    for (;;) {
        // ---- refill dead lanes: one atomic per wave
        if (!exhausted) {
            const unsigned long long dead = __ballot(!alive);
            if (dead) {
                const unsigned nd = (unsigned)__popcll(dead);
                const int leader = __ffsll(dead) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(p.counter, (unsigned long long)nd);
                base = __shfl(base, leader);
                if (base + nd >= p.n) exhausted = true;
                if (!alive) {
                    const unsigned long long below = dead & ((1ull << lane) - 1ull);
                    const unsigned long long idx = base + (unsigned long long)__popcll(below);
                    if (idx < p.n) {
                        pid = p.first + idx;
                        rng.reset(pid, p.key0, p.key1);
                        e = p.e_bin[pick_bin(p, rng.raw())];
                        const float ct = 1.0f - rng.u() * p.F.omc;
                        const float stt = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
                        double sphi, cphi;
                        sincos(6.283185307179586 * (double)rng.u(), &sphi, &cphi);
                        const float cp = (float)cphi, sp = (float)sphi;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            d[a] = (ct * p.F.ax[a] + (stt * cp) * p.F.eu[a]) +
                                   (stt * sp) * p.F.ev[a];
                            o[a] = p.F.S[a];
                        }
                        material_mu(p, e, mm, bs);
                        n_int = 0;
                        alive = true;
                        flying = false;
                        h_steps = 0;
                        h_first = 0;
                        if (STATS) ++st[kStHist];
                    }
                }
            }
        }
        if (!__any(alive)) break;

        int event = 0;   // 1 interaction, 2 left the object or missed it
        // ---- start flights
        if (alive && !flying) {
            float tin, tout;
            if (box_entry(p, o, d, tin, tout)) {
                tau_star = (float)(-log((double)rng.u()));
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    pin[a] = o[a] + d[a] * tin;
                    q[a] = (pin[a] - p.lo[a]) * p.inv_h;
                    g[a] = d[a] * p.inv_h;
                }
                len = tout - tin;
                tau = 0.0f;
                k = 0;
                flying = true;
                if (STATS) ++st[kStFlights];
            } else {
                event = 2;
            }
        }
        // ---- march
        if (flying) {
            for (int it = 0; it < p.steps_per_round; ++it) {
                const float a0 = (float)k * p.step;
                if (!(a0 < len)) {
                    event = 2;
                    break;
                }
                float b = a0 + p.step;
                if (b > len) b = len;
                const float dk = b - a0;
                const float s = 0.5f * (a0 + b);
                int ix = (int)(q[0] + g[0] * s);
                int iy = (int)(q[1] + g[1] * s);
                int iz = (int)(q[2] + g[2] * s);
                ix = min(max(ix, 0), p.nx - 1);
                iy = min(max(iy, 0), p.ny - 1);
                iz = min(max(iz, 0), p.nz - 1);
                const int v = (iz * p.ny + iy) * p.nx + ix;
                const int id = p.ids[v];
                const float mu = p.rho[v] * mm[id * bs];
                const float x = mu * dk;
                const float tn = tau + x;
                if (DEBUG) ++h_steps;
                if (STATS) ++st[kStSteps];
                if (tn >= tau_star) {
                    const float si = a0 + (tau_star - tau) / mu;
#pragma unroll
                    for (int a = 0; a < 3; ++a) o[a] = pin[a] + d[a] * si;
                    mat = id;
                    event = 1;
                    break;
                }
                tau = tn;
                ++k;
            }
        }
        if (event) flying = false;
        int end = -1;
        // ---- interaction
        if (event == 1) {
            const int off = mat * p.J;
            const float a = grid_lerp(p.pe + off, p.J, e);
            const float b = grid_lerp(p.coh + off, p.J, e);
            const float c = grid_lerp(p.inc + off, p.J, e);
            const float tot = (a + b) + c;
            const float xs = rng.u() * tot;
            if ((p.flags & 1u) || xs < a) {
                if (STATS) ++st[kStPhoto];
                if (DEBUG && n_int == 0) h_first = 1;
                end = 3;
            } else {
                float ct, e2;
                if (xs < a + b) {
                    ct = sample_rayleigh(rng, e, p.rayl_b[mat]);
                    e2 = e;
                    if (STATS) ++st[kStRayl];
                    if (DEBUG && n_int == 0) h_first = 2;
                } else {
                    sample_compton(rng, e, ct, e2);
                    if (STATS) ++st[kStCompt];
                    if (DEBUG && n_int == 0) h_first = 3;
                }
                double sphi, cphi;
                sincos(6.283185307179586 * (double)rng.u(), &sphi, &cphi);
                scatter_direction(d[0], d[1], d[2], ct, (float)cphi, (float)sphi);
                ++n_int;
                if (e2 < 1.0f) {
                    if (STATS) ++st[kStCut];
                    end = 4;
                } else if (n_int >= kMaxScatterings) {
                    if (STATS) ++st[kStCap];
                    end = 5;
                } else if (e2 != e) {
                    e = e2;
                    material_mu(p, e, mm, bs);
                }
            }
        } else if (event == 2) {
            // ---- panel
            int iu, iv;
            if (panel_hit(p, o, d, iu, iv)) {
                const float w = grid_lerp(p.eta, p.J, e);
                const long long t = (long long)rintf(w * 1048576.0f);
                if (n_int == 0) {
                    atomicAdd(p.prim + (size_t)iv * p.nu + iu, (unsigned long long)t);
                    if (STATS) ++st[kStPrim];
                    end = 0;
                } else {
                    const int su = iu / p.bu, sv = iv / p.bv;
                    atomicAdd(p.scat + (size_t)sv * p.snu + su, (unsigned long long)t);
                    if (STATS) ++st[kStScat];
                    end = 1;
                }
            } else {
                end = 2;
            }
        }
        if (end >= 0) {
            if (DEBUG) {
                const uint64_t r = pid - p.first;
                if (p.dbg_nint) p.dbg_nint[r] = (uint16_t)n_int;
                if (p.dbg_steps) p.dbg_steps[r] = h_steps;
                if (p.dbg_end) p.dbg_end[r] = (uint8_t)end;
                if (p.dbg_first) p.dbg_first[r] = h_first;
            }
            alive = false;
        }
    }
    if (STATS) {
#pragma unroll
        for (int i = 0; i < kStCount; ++i) {
            const unsigned long long sum = wave_sum(st[i]);
            if (lane == 0 && sum) atomicAdd(p.stats + i, sum);
        }
    }
}

__global__ void sample_kernel(const KParams p, int process, int material, float e_kev,
                              uint64_t n, float *cos_out, float *e_out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    PhotonStream s;
    s.reset(i, p.key0, p.key1);
    if (process == 0) {
        e_out[i] = p.e_bin[pick_bin(p, s.raw())];
    } else if (process == 3) {
        (void)s.raw();
        cos_out[i] = 1.0f - s.u() * p.F.omc;
    } else if (process == 1) {
        cos_out[i] = sample_rayleigh(s, e_kev, p.rayl_b[material]);
        if (e_out) e_out[i] = e_kev;
    } else {
        float ct, e2;
        sample_compton(s, e_kev, ct, e2);
        cos_out[i] = ct;
        if (e_out) e_out[i] = e2;
    }
}

hipError_t launch_transport(const KParams &p, int grid, int block, bool stats, bool debug,
                            hipStream_t stream) {
    const size_t lds = (size_t)p.n_mat * block * sizeof(float);
    if (debug)
        hipLaunchKernelGGL((transport_kernel<false, true>), dim3(grid), dim3(block), lds, stream,
                           p);
    else if (stats)
        hipLaunchKernelGGL((transport_kernel<true, false>), dim3(grid), dim3(block), lds, stream,
                           p);
    else
        hipLaunchKernelGGL((transport_kernel<false, false>), dim3(grid), dim3(block), lds, stream,
                           p);
    return hipGetLastError();
}

hipError_t launch_sample(const KParams &p, int process, int material, float e_kev, uint64_t n,
                         float *cos_out, float *e_out, hipStream_t stream) {
    const int block = 256;
    const uint64_t grid = (n + block - 1) / block;
    hipLaunchKernelGGL(sample_kernel, dim3((unsigned)grid), dim3(block), 0, stream, p, process,
                       material, e_kev, n, cos_out, e_out);
    return hipGetLastError();
}

int transport_blocks_per_cu(int block, int n_mat, bool stats) {
    int nb = 0;
    const size_t lds = (size_t)n_mat * block * sizeof(float);
    if (stats)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, transport_kernel<true, false>,
                                                           block, lds);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, transport_kernel<false, false>,
                                                           block, lds);
    return nb > 0 ? nb : 1;
}

}  // namespace mcx
