// Analog Monte Carlo photon transport on gfx950: cone-beam point source,
// fixed-step march through a voxel object, photoelectric / Rayleigh (eq. (2))
// / Compton (eq. (1), Kahn's method) events, primary and scatter tallies on a
// flat panel (arXiv 2201.13191, section II-A; step size section II-C-2).
//
// Execution model: a persistent grid.  Each lane carries one photon; a wave
// refills its dead lanes from a global photon counter with one atomic per
// wave (ballot + popcount + prefix count), so lanes never wait for the
// wave's longest history.  Each scheduling round handles, together, every
// lane waiting for an event -- interactions (type draw, angle sampling in
// fp64, rotation), panel crossings (int64 tally), refills and births, new
// flights -- and then marches all flying lanes until `event_batch` lanes are
// waiting again.  Batching keeps the expensive event code from running for
// one or two lanes at a time.
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
        // each 32x32 -> 64-bit product in one multiply-add (both halves)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                       (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
    }
    return c;
}

// odd multiples of 2^-24 in (0, 1): exact in fp32
__device__ __forceinline__ float unit_float(uint32_t x) {
    return (float)(2u * (x >> 9) + 1u) * 5.9604644775390625e-8f;
}

// A photon's stream: counter (photon id, block, 0).  PSEUDO: the stream of
// pseudo-particle i of the photon's n-th scattering, counter
// (photon id, n, (i + 1) * 2^12 + block).
template <bool PSEUDO>
struct StreamT {
    uint32_t id_lo, id_hi, key0, key1;
    uint32_t next;     // index of the next draw
    uint32_t cached;   // block index held in w0 .. w3
    uint32_t w0, w1, w2, w3;
    uint32_t n, tag;   // PSEUDO only

    __device__ void reset(uint64_t photon, uint32_t k0, uint32_t k1) {
        id_lo = (uint32_t)photon;
        id_hi = (uint32_t)(photon >> 32);
        key0 = k0;
        key1 = k1;
        next = 0;
        cached = 0xFFFFFFFFu;
    }
    __device__ void reset_pseudo(uint64_t photon, uint32_t k0, uint32_t k1, uint32_t scat,
                                 uint32_t i) {
        reset(photon, k0, k1);
        n = scat;
        tag = (i + 1u) << 12;
    }
    __device__ __forceinline__ uint4 block(uint32_t b) const {
        return PSEUDO ? philox4x32_10(make_uint4(id_lo, id_hi, n, tag | b), key0, key1)
                      : philox4x32_10(make_uint4(id_lo, id_hi, b, 0u), key0, key1);
    }
    __device__ uint32_t raw() {
        const uint32_t b = next >> 2;
        if (b != cached) {
            const uint4 blk = block(b);
            w0 = blk.x;
            w1 = blk.y;
            w2 = blk.z;
            w3 = blk.w;
            cached = b;
        }
        // word (next & 3) from all four words and masks: no selected or indexed
        // access into the stream, which would keep the stream in scratch memory
        const uint32_t i = next & 3u;
        ++next;
        return (w0 & (0u - (uint32_t)(i == 0u))) | (w1 & (0u - (uint32_t)(i == 1u))) |
               (w2 & (0u - (uint32_t)(i == 2u))) | (w3 & (0u - (uint32_t)(i == 3u)));
    }
    __device__ float u() { return unit_float(raw()); }
    // the next N words (N <= 4) with a single block computation: they lie in
    // the cached block and the one after it, or, from a block boundary, all in
    // one new block (the cached block always holds the last word drawn)
    template <int N>
    __device__ __forceinline__ void draw(uint32_t (&r)[N]) {
        static_assert(N >= 1 && N <= 4, "one block at most");
        const uint32_t sh = next & 3u;
        const uint32_t b0 = next >> 2, b1 = (next + (uint32_t)N - 1u) >> 2;
        const bool fresh = b0 != cached;
        const bool straddle = !fresh && b1 != b0;
        uint32_t x0 = w0, x1 = w1, x2 = w2, x3 = w3;   // the block before the new one
        if (fresh || straddle) {
            const uint32_t b = fresh ? b0 : b1;
            const uint4 blk = block(b);
            w0 = blk.x;
            w1 = blk.y;
            w2 = blk.z;
            w3 = blk.w;
            cached = b;
        }
        if (!straddle) {
            x0 = w0;
            x1 = w1;
            x2 = w2;
            x3 = w3;
        }
        // words sh .. sh + N - 1 of the window x0 .. x3, w0 .. w3, by a
        // two-stage shift (by sh & 1, then by sh & 2).  Each stage picks whole
        // words with a byte permute, which keeps the window in registers
        // (a select between its elements becomes an indexed scratch access).
        const uint32_t x[8] = {x0, x1, x2, x3, w0, w1, w2, w3};
        const uint32_t p1 = (sh & 1u) ? 0x07060504u : 0x03020100u;
        const uint32_t p2 = (sh & 2u) ? 0x07060504u : 0x03020100u;
        uint32_t y[N + 2];
#pragma unroll
        for (int i = 0; i < N + 2; ++i) y[i] = __builtin_amdgcn_perm(x[i + 1], x[i], p1);
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] = __builtin_amdgcn_perm(y[i + 2], y[i], p2);
        next += (uint32_t)N;
    }
};
using PhotonStream = StreamT<false>;
using PseudoStream = StreamT<true>;

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
// Rayleigh polar angle: v = sin^2(theta/2)/lambda^2 inverted from the
// (1 + b v)^-4 form-factor weight, accepted with (1 + cos^2)/2 evaluated on
// the fp32 cosine.  One trial (two draws); the cosine is set either way.
template <class S>
__device__ __forceinline__ bool rayleigh_trial(S &s, float e, double b, float &cf) {
    const double t = (double)e / 12.398419843320026;
    const double V = t * t;
    const double W = 1.0 + b * V;
    const double ymin = 1.0 / (W * W * W);
    uint32_t w[2];
    s.draw(w);
    const double r1 = (double)unit_float(w[0]);
    const double r2 = (double)unit_float(w[1]);
    const double y = 1.0 - r1 * (1.0 - ymin);
    const double v = (1.0 / cbrt(y) - 1.0) / b;
    cf = (float)(1.0 - 2.0 * v / V);
    const double cd = (double)cf;
    return r2 <= 0.5 * (1.0 + cd * cd);
}

template <class S>
__device__ float sample_rayleigh(S &s, float e, double b) {
    float cf;
    while (!rayleigh_trial(s, e, b, cf)) {
    }
    return cf;
}

// Kahn's rejection method for the Klein-Nishina polar angle: x = E / E_KN drawn
// from one of two branches and accepted against the KN shape.  One trial
// (three draws); false when rejected.
__device__ __forceinline__ bool kahn_trial(PhotonStream &s, double a, double &x) {
    const double top = 1.0 + 2.0 * a;
    const double branch = top / (9.0 + 2.0 * a);
    uint32_t w[3];
    s.draw(w);
    const double r1 = (double)unit_float(w[0]);
    const double r2 = (double)unit_float(w[1]);
    const double r3 = (double)unit_float(w[2]);
    if (r1 <= branch) {
        x = 1.0 + 2.0 * a * r2;
        return r3 <= 4.0 * (1.0 / x - 1.0 / (x * x));
    }
    x = top / (1.0 + 2.0 * a * r2);
    const double c = 1.0 - (x - 1.0) / a;
    return r3 <= 0.5 * (c * c + 1.0 / x);
}

// ------------------------------------------------------------------ binding effects
// Eq. (1)'s incoherent scattering function and the Doppler broadening of the
// Compton line, from one orbital model: every electron in a 1s-like orbital of
// the Rayleigh form factor's screening radius r_Z, so S/Z = 1 - (1 + b x^2)^-4
// (b and x as for the form factor) and the Compton profile is
// J(p_z) ~ (1 + (p_z / p0)^2)^-3 with p0 = hbar / r_Z.  S applies by rejection:
// a rejected collision is a null collision that leaves the photon as it was,
// and the tables stay Klein-Nishina, so the effective cross section and the
// angular law are both exact.  Doppler: s = |p_z| / p0 from the envelope
// (1 + s)^-2 by inversion (s = a / (1 - a)), accepted with
// (1 + s)^2 / (M (1 + s^2)^3), M above the ratio's maximum; E'/E is the root in
// (0, 1) of the impulse-approximation relation between p_z, the Compton ratio
// tau = E_KN / E and the cosine, a draw without one drawn again (the draws with
// p_z < 0 always have one when tau < 1).
constexpr double kDopplerEnvelope = 1.3064;

__device__ __forceinline__ double incoh_sf(double b, double V, double om) {
    const double w = 1.0 + b * (0.5 * V * om);
    const double w2 = w * w;
    return 1.0 - 1.0 / (w2 * w2);
}

// E'/E at the Compton ratio ratio_kn = E / E_KN and 1 - cos = om.  The
// discriminant is written as t ((1 - tau)^2 + tau om (2 - t tau (2 - om))),
// free of the cancellation of (1 - t tau mu)^2 - (1 - t tau^2)(1 - t) near the
// forward direction (where that form can round below zero for every draw).
// Without momentum transfer the line is not shifted.  A trial succeeds with
// probability above 0.2, so the cap of kDopplerMaxTrials trials (then the
// unbroadened ratio) is reached with probability below 1e-24; it bounds the
// loop.
constexpr int kDopplerMaxTrials = 256;

template <class S>
__device__ double sample_doppler(S &s, double pz, double ratio_kn, double om) {
    const double tau = 1.0 / ratio_kn;
    const double omt = (ratio_kn - 1.0) / ratio_kn;
    if (!(tau < 1.0) || !(omt > 0.0)) return 1.0;
    const double mu = 1.0 - om;
    for (int k = 0; k < kDopplerMaxTrials; ++k) {
        uint32_t w[2];
        s.draw(w);
        const double v = 2.0 * (double)unit_float(w[0]) - 1.0;
        const double u2 = (double)unit_float(w[1]);
        const double a = fabs(v);
        const double sm = a / (1.0 - a);
        const double s2 = 1.0 + sm * sm;
        if (!(u2 * kDopplerEnvelope <= ((1.0 + sm) * (1.0 + sm)) / ((s2 * s2) * s2))) continue;
        const double P = (v < 0.0 ? -sm : sm) * pz;
        const double t = P * P;
        const double c1 = 1.0 - (t * tau) * mu;
        const double c2 = 1.0 - (t * tau) * tau;
        const double disc = t * (omt * omt + tau * om * (2.0 - (t * tau) * (2.0 - om)));
        if (!(c2 > 0.0) || !(disc >= 0.0)) continue;
        const double root = sqrt(disc);
        const double x = tau * ((P < 0.0 ? c1 - root : c1 + root) / c2);
        if (x > 0.0 && x < 1.0) return x;
    }
    return tau;
}

// One Compton collision: Kahn's angle and, in the BIND variants, the binding
// effects p.phys asks for: (bit 0) acceptance with S/Z -- false for a null
// collision, the outputs untouched -- and (bit 1) the broadened energy.
template <bool BIND>
__device__ bool compton_collision(PhotonStream &s, const KParams &p, int mat, float e, float &ct,
                                  float &e_out) {
    const double a = (double)e / 510.99895;
    double x;
    while (!kahn_trial(s, a, x)) {
    }
    if (BIND && (p.phys & 1u)) {
        const double t = (double)e / 12.398419843320026;
        const double u = (double)s.u();
        if (!(u <= incoh_sf(p.rayl_b[mat], t * t, (x - 1.0) / a))) return false;
    }
    ct = (float)(1.0 - (x - 1.0) / a);
    if (BIND && (p.phys & 2u))
        e_out = (float)((double)e * sample_doppler(s, p.pz_scale[mat], x, (x - 1.0) / a));
    else
        e_out = (float)((double)e / x);
    return true;
}

// ------------------------------------------------------------------ point detector
// K(a) = sigma_KN / (pi r_e^2) at a = E / mc^2: the integral over the scattering
// cosine of the bracket of eq. (1) (S = 1), which normalises the Compton law of
// eq. (4).  Its Taylor series below a = 0.1, where the closed form cancels.
__device__ double kn_norm(const KParams &p, double a) {
    if (a < 0.1) {
        double s = p.kn_series[kKnTerms - 1];
        for (int i = kKnTerms - 2; i >= 0; --i) s = s * a + p.kn_series[i];
        return s;
    }
    const double d = 1.0 + 2.0 * a;
    const double ln = log1p(2.0 * a);
    const double first = (1.0 + a) / (a * a) * (2.0 * (1.0 + a) / d - ln / a);
    return 2.0 * ((first + ln / (2.0 * a)) - (1.0 + 3.0 * a) / (d * d));
}

// (1/V) int_0^V (1 + cos^2) (1 + b v)^-4 dv at B = b V: eq. (2) with the screened
// form factor integrated over the scattering cosine (per Z^2 and 2 pi r_e^2),
// which normalises the Rayleigh law of eq. (5).  Power series below B = 0.1.
__device__ double coherent_shape(const KParams &p, double B) {
    if (B < 0.1) {
        double s = p.coh_series[kCohTerms - 1];
        for (int i = kCohTerms - 2; i >= 0; --i) s = s * B + p.coh_series[i];
        return s;
    }
    const double r1 = 1.0 / (1.0 + B);
    const double r2 = r1 * r1;
    const double r3 = r2 * r1;
    const double m0 = (1.0 - r3) / 3.0;
    const double m1 = 1.0 / 6.0 - r2 / 2.0 + r3 / 3.0;
    const double m2 = 1.0 / 3.0 - r1 + r2 - r3 / 3.0;
    return 2.0 * m0 / B - 4.0 * m1 / (B * B) + 4.0 * m2 / (B * B * B);
}

// the direction rotated by polar angle (cosine ct, sine st) and azimuth
// (cosine cp, sine sp), renormalised
__device__ __forceinline__ void rotate_direction(float &dx, float &dy, float &dz, float ct,
                                                 float st, float cp, float sp) {
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

// first bin k with x < thr[k]: the guide table gives the first candidate of
// x's top-byte bucket, a short scan finds the bin (thr[n_bins-1] = 2^32)
__device__ __forceinline__ uint32_t pick_bin(const KParams &p, uint32_t x) {
    uint32_t k = p.guide[x >> 24];
    while ((uint64_t)x >= p.thr[k]) ++k;
    return k;
}

// ------------------------------------------------------------------ geometry
__device__ __forceinline__ bool box_entry(const VoxelGrid &p, const float o[3], const float d[3],
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

__device__ __forceinline__ bool panel_hit(const KParams &p, const ProjFrame &F, const float o[3],
                                          const float d[3], int &iu, int &iv) {
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

// birth direction inside the cone that circumscribes the panel: cos theta
// uniform on [cos theta_max, 1], azimuth uniform (two draws)
__device__ __forceinline__ void cone_direction(const ProjFrame &F, PhotonStream &rng, float d[3]) {
    const float ct = 1.0f - rng.u() * F.omc;
    const float stt = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
    double sphi, cphi;
    sincos(6.283185307179586 * (double)rng.u(), &sphi, &cphi);
    const float cp = (float)cphi, sp = (float)sphi;
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = (ct * F.ax[a] + (stt * cp) * F.eu[a]) + (stt * sp) * F.ev[a];
}

// ------------------------------------------------------------------ kernels
enum : int { kStHist, kStSteps, kStFlights, kStPhoto, kStRayl, kStCompt, kStPrim, kStScat,
             kStCut, kStCap, kStSkipped, kStPdScores, kStPdKilled, kStPdSteps, kStNull, kStCount };

// optical-depth increments on the grid of 2^-32: fp64 sums of them are exact,
// so a run of equal increments can be added at once
__device__ __forceinline__ double on_grid(double x) {
    return __builtin_rint(x * 4294967296.0) * 2.3283064365386963e-10;
}

constexpr float kSkipMargin = 1.0f / 64.0f;   // voxels kept from a uniform region's faces
#ifndef MCX_MIN_SKIP
#define MCX_MIN_SKIP 4
#endif
constexpr uint32_t kMinSkip = MCX_MIN_SKIP;  // shortest run taken at once


#ifndef MCX_PREFETCH
#define MCX_PREFETCH 8
#endif
constexpr int kPrefetch = MCX_PREFETCH;   // march steps whose voxel loads are issued together
// An unclamped group reads up to kPrefetch - 1 step centres past a flight's last
// step; with steps of at most one voxel those lie within the edge copies.
static_assert(kPrefetch + 1 <= kEdgePad, "unclamped gathers would read past the edge copies");
constexpr int kLdsHeader = 256 + 64;   // floats: palette densities, then 256 palette ids

// the value lane `src` (wave-uniform) holds, read into a scalar register
// without a trip through LDS
__device__ __forceinline__ unsigned long long lane_value(unsigned long long v, int src) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// byte offset of voxel (ix, iy, iz) in the bricked arrays,
//   (iz>>2)*slab + (iy>>2)*row + (ix>>3)*128 + (iz&3)*32 + (iy&3)*8 + (ix&7),
// regrouped as ix + 120*(ix>>3) + 8*iy + (row-32)*(iy>>2) + 32*iz + (slab-128)*(iz>>2)
// so that each axis costs one shift and one 24-bit multiply-add (the runtime
// keeps row-32 and slab-128 below 2^24)
__device__ __forceinline__ uint32_t brick_offset(const VoxelGrid &p, uint32_t ix, uint32_t iy,
                                                 uint32_t iz) {
    uint32_t o = __umul24(ix >> 3, 120u) + ix;
    o += __umul24(iy >> 2, p.ry) + (iy << 3);
    o += __umul24(iz >> 2, p.rz) + (iz << 5);
    return o;
}

// number of march steps of a chord of length len: the count of k >= 0 with
// (float)k * step < len (an increasing sequence), from the quotient's estimate
__device__ __forceinline__ uint32_t step_count(float len, float step) {
    if (!(len > 0.0f)) return 0u;
    uint32_t n = (uint32_t)(len / step);
    while (n > 0u && !((float)(n - 1u) * step < len)) --n;
    while ((float)n * step < len) ++n;
    return n;
}

// voxel index along one axis: truncation of the voxel coordinate clamped to
// [0, n - 1]; clamping the float first is the same as clamping the integer
// and needs one median instruction
__device__ __forceinline__ uint32_t voxel_index(float c, float cmax) {
    return (uint32_t)__builtin_amdgcn_fmed3f(c, 0.0f, cmax);
}

// voxel index along one axis without the upper clamp: v_cvt_u32_f32 itself
// saturates (negative and NaN to 0), which C's conversion does not promise
__device__ __forceinline__ uint32_t saturated_index(float c) {
    uint32_t i;
    asm("v_cvt_u32_f32 %0, %1" : "=v"(i) : "v"(c));
    return i;
}

// A pointer taken from a descriptor copied out of memory (a batch's object or
// job table) is a generic pointer to the compiler, which then issues flat
// accesses; these always address device memory, and saying so gives global
// ones (with a scalar base when the pointer is uniform).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *dev(const T *q) {
    return (const __attribute__((address_space(1))) T *)q;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *dev_rw(T *q) {
    return (__attribute__((address_space(1))) T *)q;
}

// uniform-cell word of the cell holding the (clamped) voxel of centre q
__device__ __forceinline__ uint32_t cell_word(const VoxelGrid &g, const float q[3]) {
    const uint32_t cx = voxel_index(q[0], g.cmax[0]) >> kCellLog;
    const uint32_t cy = voxel_index(q[1], g.cmax[1]) >> kCellLog;
    const uint32_t cz = voxel_index(q[2], g.cmax[2]) >> kCellLog;
    return dev(g.cells)[__umul24(__umul24(cz, (uint32_t)g.ncy) + cy, (uint32_t)g.ncx) + cx];
}

// MODE: layout of the single object (ignored for batches, where each lane
// follows the layout of its own job's object).  BATCH: run the job table.
// BIND: the binding-effect samplers are compiled in (launched when p.phys is
// non-zero); without them the default path keeps its register budget.
template <int MODE, bool BATCH, bool STATS, bool DEBUG, bool PD, bool BIND>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((PD || STATS || DEBUG) ? 1 : 3)))
transport_kernel(const KParams p) {
    static_assert(!PD || (!BATCH && !DEBUG), "point-detector scoring: single projections only");
    // LDS: palette densities [256] | palette ids [256 bytes] (single object only) |
    // lane-private columns: mu per material [n_mat][bs] (fp32), then the
    // optical-depth increment of a full step per palette entry [n_pal][bs]
    // (fp64) for per-lane palette tables
    extern __shared__ float lds[];
    float *s_pal_rho = lds;
    uint8_t *s_pal_id = (uint8_t *)(lds + 256);
    const int bs = blockDim.x;
    float *mm = lds + kLdsHeader + threadIdx.x;
    double *inc_pal = (double *)(lds + kLdsHeader + p.n_mat * bs) + threadIdx.x;
    const uint32_t bs8 = (uint32_t)bs * 8u;   // byte stride between a lane's fp64 entries
    const double step32 = (double)p.step * 4294967296.0;
    const int lane = (int)__lane_id();
    if (!BATCH && MODE != kGeneric) {
        for (int i = threadIdx.x; i < p.G.n_pal; i += bs) {
            s_pal_rho[i] = p.G.pal_rho[i];
            s_pal_id[i] = p.G.pal_id[i];
        }
        __syncthreads();
    }

    // the lane's voxel object: the kernel's own for a single projection; in a
    // batch the index of the job's object.  with_grid(active, f) runs f(grid)
    // for the active lanes once per distinct object among them (almost always
    // one), with the descriptor read by scalar loads from the constant address
    // space, so a batch keeps no per-lane copy of it in vector registers.
    int gi = 0;
    using ConstWord = const __attribute__((address_space(4))) uint32_t;
    static_assert(sizeof(VoxelGrid) % 4 == 0, "descriptor copied word by word");
    auto with_grid = [&](bool active, auto f) __attribute__((always_inline)) {
        if (!BATCH) {
            if (active) f(p.G);
            return;
        }
        unsigned long long todo = __ballot(active);
        while (todo) {
            const int leader = __ffsll(todo) - 1;
            const int g = __builtin_amdgcn_readlane(gi, leader);
            // read in control flow uniform across the wave (inside the
            // divergent branch below it would become vector loads)
            VoxelGrid gs;
            ConstWord *src = (ConstWord *)(p.grids + g);
            uint32_t *dst = (uint32_t *)&gs;
#pragma unroll
            for (int w = 0; w < (int)(sizeof(VoxelGrid) / 4); ++w) dst[w] = src[w];
            const bool mine = active && gi == g;
            if (mine) f(gs);
            todo &= ~__ballot(mine);
        }
    };
    int job = 0;          // batch: the lane's job
    int cur_job = 0;      // batch: the job this wave refills from
    // the descriptor of job j (wave-uniform j) by scalar loads
    static_assert(sizeof(JobDesc) % 4 == 0, "descriptor copied word by word");
    auto job_desc = [&](int j) __attribute__((always_inline)) {
        JobDesc jd;
        ConstWord *src = (ConstWord *)(p.jobs + j);
        uint32_t *dst = (uint32_t *)&jd;
#pragma unroll
        for (int w = 0; w < (int)(sizeof(JobDesc) / 4); ++w) dst[w] = src[w];
        return jd;
    };
    // with_job(active, f): f(frame, primary image, scatter image) for the
    // active lanes, once per distinct job among them (as with_grid)
    auto with_job = [&](bool active, auto f) __attribute__((always_inline)) {
        if (!BATCH) {
            if (active) f(p.F, p.prim, p.scat);
            return;
        }
        unsigned long long todo = __ballot(active);
        while (todo) {
            const int leader = __ffsll(todo) - 1;
            const int j = __builtin_amdgcn_readlane(job, leader);
            const JobDesc jd = job_desc(j);      // uniform control flow: scalar loads
            const bool mine = active && job == j;
            if (mine) f(jd.F, jd.prim, jd.scat);
            todo &= ~__ballot(mine);
        }
    };

    bool alive = false, flying = false, exhausted = false;
    // the wave's reserved photon ids [res_next, res_end) (single projections:
    // relative to first; batches: of job res_job); a reservation takes p.chunk
    // ids from the launch's (or the job's) counter, so the counter, which every
    // wave updates, sees one atomic per chunk rather than one per refill
    uint64_t res_next = 0, res_end = 0;
    int res_job = 0;      // batch: the job of the reserved ids
    uint32_t rounds = 0;     // scheduling rounds of this wave (cancellation checks)
    PhotonStream rng;
    uint64_t pid = 0;
    float e = 0.0f;
    float o[3] = {0.0f, 0.0f, 0.0f}, d[3] = {0.0f, 0.0f, 0.0f};
    float c0[3], q[3], G[3], ig[3];
    float tin = 0.0f, last = 0.0f;
    double tau = 0.0, ts = 0.0;
    uint32_t k = 0, nsteps = 0;
    uint32_t cellw = 0;   // uniform-cell word at the centre of step k (0: none known)
    float tab_e = -1.0f;  // energy of the lane's LDS attenuation tables (-1: none yet)
    // Between flights, three flight variables hold what the next flight
    // needs, without registers of their own: `last` the polar cosine of the
    // pending turn (birth: into the cone; scattering: away from the old
    // direction), `nsteps` the azimuth's draw, and `ts` the draw of the next
    // flight's optical depth (the word after the azimuth's), as a double.
    bool turn = false;
    float &dir_ct = last;
    uint32_t &phi_w = nsteps;
    int n_int = 0, mat = 0;
    int n_coll = 0;     // scatterings and null collisions: point-detector counters
    unsigned long long st[kStCount] = {};
    uint32_t h_steps = 0;
    uint8_t h_first = 0;

    // attenuation at the photon's energy: per material, and the full-step
    // optical-depth increment per palette entry
    auto refresh_mu = [&](float energy, const VoxelGrid &gr) __attribute__((always_inline)) {
        material_mu(p, energy, mm, bs);
        if (BATCH ? gr.layout == kPaletteLane : MODE == kPaletteLane) {
            // the palette (the same for every lane) by scalar loads, so each
            // entry costs one LDS read of the lane's material column; the ids
            // are read four to a word (the id array holds 256 entries)
            using ConstF = const __attribute__((address_space(4))) float;
            using ConstW = const __attribute__((address_space(4))) uint32_t;
            const ConstF *rho = (const ConstF *)gr.pal_rho;
            const ConstW *ids = (const ConstW *)gr.pal_id;
            for (int c = 0; c < gr.n_pal; ++c) {
                const int id = (int)((ids[c >> 2] >> (8 * (c & 3))) & 0xFFu);
                const float mu = rho[c] * mm[id * bs];
                inc_pal[c * bs] = __builtin_rint((double)mu * step32) * 2.3283064365386963e-10;
            }
        }
    };
    // a new photon: energy bin, direction in the cone, position at the source
    auto birth = [&](uint64_t photon, uint32_t k0, uint32_t k1, const ProjFrame &F)
        __attribute__((always_inline)) {
        pid = photon;
        rng.reset(pid, k0, k1);
        // the first block: energy bin, the cone's polar cosine and azimuth,
        // and the first flight's optical depth
        uint32_t w[4];
        rng.draw(w);
        e = p.e_bin[pick_bin(p, w[0])];
        dir_ct = 1.0f - unit_float(w[1]) * F.omc;
        phi_w = w[2];
        ts = (double)w[3];
        turn = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) o[a] = F.S[a];
        tab_e = -1.0f;    // tables are rebuilt when the first flight starts
        n_int = 0;
        n_coll = 0;
        alive = true;
        flying = false;
        if (DEBUG) {
            h_steps = 0;
            h_first = 0;
        }
        if (STATS) ++st[kStHist];
    };

    // point-detector scoring (PD): the next pseudo-particle of the lane's
    // scattering event (-1: none pending), its process, the flight in progress
    // being a pseudo-particle's chord, and that pseudo-particle's unattenuated
    // score and scatter bin
    int pd_i = -1;
    bool pd_rayl = false, pd_flight = false;
    double pd_x0 = 0.0;
    uint32_t pd_bin = 0;
    const double pd_area = (double)((float)p.nu * p.pu) * (double)((float)p.nv * p.pv);

    // the march of a new flight along `dir` from o, entering at tin and leaving
    // at tout: voxel coordinates of the first step's nominal centre, the
    // per-step increment, the step count and the last step's length
    auto start_march = [&](const VoxelGrid &gr, const float dir[3], float tout)
        __attribute__((always_inline)) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float pin = o[a] + dir[a] * tin;
            G[a] = (dir[a] * gr.inv_h) * p.step;
            c0[a] = (pin - gr.lo[a]) * gr.inv_h + 0.5f * G[a];
            q[a] = c0[a] + 0.0f * G[a];
            ig[a] = 1.0f / G[a];
        }
        const float len = tout - tin;
        nsteps = step_count(len, p.step);
        last = nsteps ? len - (float)(nsteps - 1u) * p.step : 0.0f;
        tau = 0.0;
        cellw = gr.cells != nullptr ? cell_word(gr, q) : 0u;
        k = 0;
        flying = true;
    };

    // the interaction type at (material, E): 0 photoelectric (or any
    // interaction without scattering), 1 Rayleigh, 2 Compton
    auto interaction_type = [&]() __attribute__((always_inline)) -> int {
        const int off = mat * p.J;
        const float a = grid_lerp(p.pe + off, p.J, e);
        const float b = grid_lerp(p.coh + off, p.J, e);
        const float c = grid_lerp(p.inc + off, p.J, e);
        const float tot = (a + b) + c;
        const float xs = rng.u() * tot;
        if ((p.flags & 1u) || xs < a) {
            if (STATS) ++st[kStPhoto];
            if (DEBUG && n_int == 0) h_first = 1;
            return 0;
        }
        return xs < a + b ? 1 : 2;
    };
    // the photon scatters: polar angle by the process's sampler, then the
    // azimuth's and the next flight's draws; cut-offs end the history
    auto scatter = [&](bool rayleigh, int &end) __attribute__((always_inline)) {
        float ct = 1.0f, e2 = e;
        bool real = true;
        if (rayleigh) {
            ct = sample_rayleigh(rng, e, p.rayl_b[mat]);
            e2 = e;
            if (STATS) ++st[kStRayl];
            if (DEBUG && n_int == 0) h_first = 2;
        } else {
            real = compton_collision<BIND>(rng, p, mat, e, ct, e2);
            if (STATS) {
                st[kStCompt] += real ? 1ull : 0ull;
                st[kStNull] += real ? 0ull : 1ull;
            }
            if (DEBUG && n_int == 0 && real) h_first = 3;
        }
        uint32_t w[2];
        rng.draw(w);
        ts = (double)w[1];
        if constexpr (BIND) ++n_coll;
        if (!real) return;      // null collision: a new flight along the same line
        dir_ct = ct;
        phi_w = w[0];
        turn = true;
        ++n_int;
        if (e2 < 1.0f) {
            if (STATS) ++st[kStCut];
            end = 4;
            turn = false;
        } else if (n_int >= kMaxScatterings) {
            if (STATS) ++st[kStCap];
            end = 5;
            turn = false;
        } else {
            e = e2;
        }
    };

    // point detector, eq. (3)-(5): the pseudo-particle pd_i of the photon's
    // n_int-th scattering at o (incoming direction d, energy e) picks a uniform
    // point on the panel from its own Philox block (counter photon id, n_int,
    // pd_i + 1; the photon's draws use counters ending in 0) and scores
    // eta(E') p(lambda) cos(gamma) A / (2 pi R^2 split) exp(-tau), tau the
    // optical depth at E' from o to the object's exit.  Roulette below
    // pd_rr (section II-C-1).  Returns true when the chord's march started;
    // false when the pseudo-particle needs none (killed, below 1 keV, or
    // scored at once because it leaves the object without a step).
    auto pd_score = [&](double tau_chord) __attribute__((always_inline)) {
        const double x = pd_x0 * exp(-tau_chord);
        const long long t = (long long)__builtin_rint(x * 1048576.0);
        if (t != 0)
            __hip_atomic_fetch_add(dev_rw(p.scat) + pd_bin, (unsigned long long)t,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (STATS) ++st[kStPdScores];
    };
    auto pd_start = [&]() __attribute__((always_inline)) -> bool {
        const ProjFrame &F = p.F;
        if (p.pd_mode == 2 && pd_rayl) {
            // mixed estimator: a Rayleigh pseudo-particle draws its direction
            // from the Rayleigh law (its own stream) and scores eta(E) / split
            // exp(-tau) where that line crosses the panel
            PseudoStream ps;
            ps.reset_pseudo(pid, p.key0, p.key1, (uint32_t)(BIND ? n_coll : n_int),
                            (uint32_t)pd_i);
            const float ct = sample_rayleigh(ps, e, p.rayl_b[mat]);
            double sphi, cphi;
            sincos(6.283185307179586 * (double)ps.u(), &sphi, &cphi);
            float om[3] = {d[0], d[1], d[2]};
            rotate_direction(om[0], om[1], om[2], ct, sqrtf(fmaxf(0.0f, 1.0f - ct * ct)),
                             (float)cphi, (float)sphi);
            int iu, iv;
            if (!panel_hit(p, F, o, om, iu, iv)) return false;
            double x0 = (double)grid_lerp(p.eta, p.J, e) / (double)p.pd_split;
            const double u_rr = (double)ps.u();
            if (p.pd_rr > 0.0 && x0 < p.pd_rr) {
                if (u_rr < x0 / p.pd_rr) {
                    x0 = p.pd_rr;
                } else {
                    if (STATS) ++st[kStPdKilled];
                    return false;
                }
            }
            pd_x0 = x0;
            pd_bin = (uint32_t)((iv / p.bv) * p.snu + iu / p.bu);
            float tout;
            if (!box_entry(p.G, o, om, tin, tout)) {
                pd_score(0.0);
                return false;
            }
            if (tab_e != e) {
                refresh_mu(e, p.G);
                tab_e = e;
            }
            start_march(p.G, om, tout);
            ts = __builtin_inf();
            pd_flight = true;
            if (STATS) ++st[kStFlights];
            return true;
        }
        const uint4 w = philox4x32_10(make_uint4((uint32_t)pid, (uint32_t)(pid >> 32),
                                                 (uint32_t)(BIND ? n_coll : n_int),
                                                 (uint32_t)pd_i + 1u),
                                      p.key0, p.key1);
        const float fu = unit_float(w.x) * (float)p.nu;
        const float fv = unit_float(w.y) * (float)p.nv;
        int iu = (int)fu, iv = (int)fv;
        iu = iu > p.nu - 1 ? p.nu - 1 : iu;
        iv = iv > p.nv - 1 ? p.nv - 1 : iv;
        const float uu = fu * p.pu - F.hu, vv = fv * p.pv - F.hv;
        float dq[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) dq[a] = ((F.D[a] + uu * F.eu[a]) + vv * F.ev[a]) - o[a];
        const double r2 =
            ((double)dq[0] * dq[0] + (double)dq[1] * dq[1]) + (double)dq[2] * dq[2];
        const double dist = sqrt(r2);
        double lam =
            (((double)d[0] * dq[0] + (double)d[1] * dq[1]) + (double)d[2] * dq[2]) / dist;
        lam = lam > 1.0 ? 1.0 : (lam < -1.0 ? -1.0 : lam);
        const double cg =
            (((double)F.ax[0] * dq[0] + (double)F.ax[1] * dq[1]) + (double)F.ax[2] * dq[2]) /
            dist;
        float e2;
        double pdf;
        if (!pd_rayl) {
            // eq. (4): Klein-Nishina per unit cosine, at the Compton energy
            const double alpha = (double)e / 510.99895;
            const double ratio = 1.0 + alpha * (1.0 - lam);
            const double r = 1.0 / ratio;
            e2 = (float)((double)e / ratio);
            pdf = r * r * ((r + ratio) - (1.0 - lam * lam)) / kn_norm(p, alpha);
            if (BIND && (p.phys & 1u)) {
                // the law's deficit under S/Z is the null collisions' share
                const double t = (double)e / 12.398419843320026;
                pdf *= incoh_sf(p.rayl_b[mat], t * t, 1.0 - lam);
            }
            if (BIND && (p.phys & 2u)) {
                // the broadened energy towards the point, from the
                // pseudo-particle's own stream
                PseudoStream ps;
                ps.reset_pseudo(pid, p.key0, p.key1, (uint32_t)n_coll, (uint32_t)pd_i);
                e2 = (float)((double)e * sample_doppler(ps, p.pz_scale[mat], ratio, 1.0 - lam));
            }
        } else {
            // eq. (5): (1 + lambda^2) F^2 per unit cosine, energy unchanged
            const double t = (double)e / 12.398419843320026;
            const double V = t * t;
            const double b = p.rayl_b[mat];
            const double wv = 1.0 + b * ((1.0 - lam) * 0.5 * V);
            e2 = e;
            pdf = (1.0 + lam * lam) / (((wv * wv) * wv) * wv) / (2.0 * coherent_shape(p, b * V));
        }
        if (e2 < 1.0f) return false;      // such a photon would be killed
        const double eta = (double)grid_lerp(p.eta, p.J, e2);
        double x0 = (((eta * pdf) * cg) * pd_area) /
                    ((6.283185307179586 * r2) * (double)p.pd_split);
        if (p.pd_rr > 0.0 && x0 < p.pd_rr) {
            if ((double)unit_float(w.z) < x0 / p.pd_rr) {
                x0 = p.pd_rr;
            } else {
                if (STATS) ++st[kStPdKilled];
                return false;
            }
        }
        pd_x0 = x0;
        pd_bin = (uint32_t)((iv / p.bv) * p.snu + iu / p.bu);
        float om[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) om[a] = (float)((double)dq[a] / dist);
        float tout;
        if (!box_entry(p.G, o, om, tin, tout)) {
            pd_score(0.0);
            return false;
        }
        if (tab_e != e2) {
            refresh_mu(e2, p.G);
            tab_e = e2;
        }
        start_march(p.G, om, tout);
        ts = __builtin_inf();
        pd_flight = true;
        if (STATS) ++st[kStFlights];
        return true;
    };

    // pending: 1 interaction, 2 reaches the panel plane (left or missed the box),
    // 3 a pseudo-particle's chord left the object
    int event = 0;
    for (;;) {
        int end = -1;
        // ---- 1. interactions of lanes whose flight ended inside the object
        if constexpr (!PD) {
            if (event == 1) {
                event = 0;
                const int kind = interaction_type();
                if (kind == 0)
                    end = 3;
                else
                    scatter(kind == 1, end);
            }
        } else {
            // with the point detector a scattering event first scores its
            // pseudo-particles (each one's chord marched like a flight, with
            // tau* infinite), and the photon scatters after the last one
            bool do_scatter = false, rayl = false;
            if (event == 1) {
                event = 0;
                const int kind = interaction_type();
                if (kind == 0) {
                    end = 3;
                } else if (n_int + 1 < kMaxScatterings) {
                    pd_i = 0;
                    pd_rayl = kind == 1;
                } else {
                    do_scatter = true;      // the scattered photon is not transported
                    rayl = kind == 1;
                }
            }
            if (pd_i >= 0 && !flying) {
                if (event == 3) {
                    event = 0;
                    pd_flight = false;
                    pd_score(tau);
                    ++pd_i;
                }
                while (pd_i < p.pd_split && !pd_start()) ++pd_i;
                if (pd_i >= p.pd_split) {
                    pd_i = -1;
                    do_scatter = true;
                    rayl = pd_rayl;
                }
            }
            if (do_scatter) scatter(rayl, end);
        }
        // ---- 2. panel crossings
        with_job(event == 2, [&](const ProjFrame &F, unsigned long long *prim,
                                 unsigned long long *scat) __attribute__((always_inline)) {
            event = 0;
            int iu, iv;
            if (panel_hit(p, F, o, d, iu, iv)) {
                const float w = grid_lerp(p.eta, p.J, e);
                const long long t = (long long)rintf(w * 1048576.0f);
                if (n_int == 0) {
                    __hip_atomic_fetch_add(dev_rw(prim) + (size_t)iv * p.nu + iu,
                                           (unsigned long long)t, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    end = 0;
                } else {
                    // with the point detector the scatter image holds its scores only
                    if (!PD) {
                        const int su = iu / p.bu, sv = iv / p.bv;
                        __hip_atomic_fetch_add(dev_rw(scat) + (size_t)sv * p.snu + su,
                                               (unsigned long long)t, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    }
                    end = 1;
                }
                if (STATS) {
                    // both counters, added to by value (an index chosen per lane
                    // would put the counters in scratch memory)
                    st[kStPrim] += n_int == 0 ? 1ull : 0ull;
                    st[kStScat] += n_int == 0 ? 0ull : 1ull;
                }
            } else {
                end = 2;
            }
        });
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
        // ---- 3. refill dead lanes from the wave's reserved photon ids
        // A cancellation request (a flag in host memory, read every 64th round
        // of a wave) ends the launch's intake: the photons in flight, and the
        // ids a wave has reserved, finish.
        if (!exhausted && p.cancel != nullptr && (++rounds & 63u) == 0u) {
            int flag = 0;
            if (lane == 0)
                flag = __hip_atomic_load(p.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (__builtin_amdgcn_readfirstlane(flag) != 0) exhausted = true;
        }
        if (!BATCH) {
            // dead lanes take the reserved ids in lane order, then a new chunk's
            // when the reservation runs short.  Reserved ids are always used up
            // (also after a cancellation, which only stops new reservations),
            // so the photons a launch runs are the prefix [0, counter).
            const unsigned long long dead = __ballot(!alive);
            const unsigned nd = (unsigned)__popcll(dead);
            const uint64_t avail = res_end - res_next;
            uint64_t cb = 0, ce = 0;
            if (nd > 0 && avail < nd && !exhausted) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(p.counter, (unsigned long long)p.chunk);
                base = lane_value(base, 0);
                if (base >= p.n) {
                    exhausted = true;
                } else {
                    cb = base;
                    ce = p.n - base < p.chunk ? p.n : base + p.chunk;
                }
            }
            if (!alive) {
                const uint64_t rank = (uint64_t)__popcll(dead & ((1ull << lane) - 1ull));
                if (rank < avail)
                    birth(p.first + res_next + rank, p.key0, p.key1, p.F);
                else if (rank - avail < ce - cb)
                    birth(p.first + cb + (rank - avail), p.key0, p.key1, p.F);
            }
            if (avail >= nd) {
                res_next += nd;
            } else if (ce > cb) {
                const uint64_t used = (uint64_t)nd - avail;
                res_next = used < ce - cb ? cb + used : ce;
                res_end = ce;
            } else {
                res_next = res_end;
            }
        } else {
            // batches: the reservation belongs to job res_job; a new one takes
            // p.chunk ids of the current job, moving to the next job when this
            // one has none left
            unsigned long long dead = __ballot(!alive);
            while (dead) {
                const uint64_t avail = res_end - res_next;
                if (avail > 0) {
                    const JobDesc rd = job_desc(__builtin_amdgcn_readfirstlane(res_job));
                    const unsigned nd = (unsigned)__popcll(dead);
                    if (!alive) {
                        const uint64_t rank = (uint64_t)__popcll(dead & ((1ull << lane) - 1ull));
                        if (rank < avail) {
                            job = res_job;
                            gi = rd.grid;
                            birth(res_next + rank, rd.key0, rd.key1, rd.F);
                        }
                    }
                    res_next += avail < nd ? avail : nd;
                    dead = __ballot(!alive);
                    continue;
                }
                if (exhausted) break;
                const int cj = __builtin_amdgcn_readfirstlane(cur_job);
                const JobDesc cd = job_desc(cj);
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(p.job_counters + cj, (unsigned long long)p.chunk);
                base = lane_value(base, 0);
                if (base < cd.n) {
                    res_job = cj;
                    res_next = base;
                    res_end = cd.n - base < p.chunk ? cd.n : base + p.chunk;
                } else if (cur_job + 1 < p.n_jobs) {
                    ++cur_job;          // the current job has no photons left
                } else {
                    exhausted = true;
                }
            }
        }
        if (!__any(alive)) break;

        // ---- 3b. new directions of born and scattered photons, with one
        //          azimuth evaluation for both
        float cp = 0.0f, sp = 0.0f, stt = 0.0f;
        if (turn) {
            double sphi, cphi;
            sincos(6.283185307179586 * (double)unit_float(phi_w), &sphi, &cphi);
            cp = (float)cphi;
            sp = (float)sphi;
            stt = sqrtf(fmaxf(0.0f, 1.0f - dir_ct * dir_ct));
            if (n_int != 0) rotate_direction(d[0], d[1], d[2], dir_ct, stt, cp, sp);
        }
        with_job(turn && n_int == 0, [&](const ProjFrame &F, unsigned long long *,
                                         unsigned long long *) __attribute__((always_inline)) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                d[a] = (dir_ct * F.ax[a] + (stt * cp) * F.eu[a]) + (stt * sp) * F.ev[a];
        });
        turn = false;

        // ---- 4. start flights (new photons and scattered ones); the LDS tables
        //         are rebuilt first if the energy changed since the last flight
        with_grid(alive && !flying && event == 0, [&](const VoxelGrid &gr) __attribute__((always_inline)) {
            float tout;
            if (box_entry(gr, o, d, tin, tout)) {
                if (tab_e != e) {
                    refresh_mu(e, gr);
                    tab_e = e;
                }
                ts = (double)(float)(-log((double)unit_float((uint32_t)ts)));
                start_march(gr, d, tout);
                if (STATS) ++st[kStFlights];
            } else {
                event = 2;
            }
        });
        // ---- 5. march until `event_batch` lanes wait for an event (or none flies).
        //         A lane whose step centre lies in a uniform region first takes
        //         the run of identical steps ahead of it at once.  Then each group
        //         issues the voxel loads of kPrefetch consecutive steps (centres
        //         re-anchored every 4 steps, added up in between) together with
        //         the uniform-cell word at the centre after the group, and
        //         consumes the steps in order without branches: the optical depth
        //         (fp64, exact) and the step index advance by selection, the step
        //         that reaches tau* is recorded, and the interaction point or the
        //         exit follows the group.
        static_assert(kPrefetch % 4 == 0, "groups hold whole anchor periods");
        // march(each_object): the loop of groups; each_object(f) runs one
        // group f for the flying lanes with their object's descriptor
        auto march = [&](auto each_object) __attribute__((always_inline)) {
        for (;;) {
            if (!__any(flying)) break;
            if (__popcll(__ballot(alive && !flying)) >= (unsigned)p.event_batch) break;
            if (!flying) continue;
            each_object([&](const VoxelGrid &gl) __attribute__((always_inline)) {
            const bool lane_pal = BATCH ? gl.layout == kPaletteLane : MODE == kPaletteLane;
            const bool skips = gl.cells != nullptr;
            const int lay = BATCH ? gl.layout : MODE;
            // the material of palette entry c: the object's palette (staged in
            // LDS for a single palette object), or, for a generic object, the
            // table of the values of its uniform cells
            auto pal_material = [&](uint32_t c) __attribute__((always_inline)) -> int {
                return (BATCH || lay == kGeneric) ? (int)dev(gl.pal_id)[c] : (int)s_pal_id[c];
            };
            // c: the voxel's code (generic: its material), or, with run = true,
            // the palette entry of the uniform region the run went through
            auto interact = [&](uint32_t c, double inc, float len, bool run)
                __attribute__((always_inline)) {
                // the point where the optical depth reaches tau* inside step k
                const float si = (float)k * p.step + (float)((ts - tau) / inc * (double)len);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float pin = o[a] + d[a] * tin;
                    o[a] = pin + d[a] * si;
                }
                mat = (lay == kGeneric && !run) ? (int)c : pal_material(c);
                event = 1;
                flying = false;
            };
            // a lane whose step centre lies in a uniform region takes the run of
            // identical steps ahead of it at once: the cube of cells of radius
            // (cellw >> 8) - 1 around the centre's cell.  Count the steps whose
            // centres stay a margin inside it (the centres are monotone along
            // each axis), leave out the last step, and take them in multiples
            // of 4; a hit inside the run is found exactly.
            if (skips && (cellw >> 8) != 0u && k + 1u < nsteps) {
                const uint32_t cell = cellw;
                cellw = 0u;
                const uint32_t cc[3] = {voxel_index(q[0], gl.cmax[0]) >> kCellLog,
                                        voxel_index(q[1], gl.cmax[1]) >> kCellLog,
                                        voxel_index(q[2], gl.cmax[2]) >> kCellLog};
                const int r = (int)(cell >> 8);
                float n = 4194304.0f;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const bool neg = (__float_as_uint(G[a]) >> 31) != 0u;
                    const float bound =
                        neg ? (float)(((int)cc[a] - r + 1) * (1 << kCellLog)) + kSkipMargin
                            : (float)(((int)cc[a] + r) * (1 << kCellLog)) - kSkipMargin;
                    n = fminf(n, fmaxf((bound - q[a]) * ig[a], 0.0f));
                }
                uint32_t cnt = (uint32_t)n;
                const uint32_t avail = nsteps - 1u - k;
                cnt = (cnt < avail ? cnt : avail) & ~3u;
                if (cnt >= kMinSkip) {
                    const uint32_t c = cell & 0xFFu;
                    double inc;
                    if (lane_pal) {
                        inc = *(const double *)((const char *)inc_pal + __umul24(c, bs8));
                    } else {
                        // the per-step increment of the region's (density,
                        // material), as the gathers below would compute it
                        const bool lds_pal = !BATCH && MODE == kPaletteShared;
                        const float rho = lds_pal ? s_pal_rho[c] : dev(gl.pal_rho)[c];
                        const uint32_t id = lds_pal ? (uint32_t)s_pal_id[c]
                                                    : (uint32_t)dev(gl.pal_id)[c];
                        const float mu = rho * mm[id * bs];
                        inc = __builtin_rint((double)mu * step32) * 2.3283064365386963e-10;
                    }
                    const double tn = tau + (double)cnt * inc;
                    if (tn >= ts) {
                        // the first step of the run whose end reaches tau*:
                        // an fp32 estimate, made exact by the fp64 checks
                        const float est = (float)(ts - tau) * __builtin_amdgcn_rcpf((float)inc);
                        uint32_t j = (uint32_t)fminf(fmaxf(ceilf(est) - 1.0f, 0.0f),
                                                     (float)(cnt - 1u));
                        while (j > 0u && tau + (double)j * inc >= ts) --j;
                        while (tau + (double)(j + 1u) * inc < ts) ++j;
                        if (DEBUG) h_steps += j + 1u;
                        if (STATS) {
                            st[kStSteps] += j + 1u;
                            st[kStSkipped] += j + 1u;
                        }
                        tau = tau + (double)j * inc;
                        k += j;
                        interact(c, inc, p.step, true);
                    } else {
                        if (DEBUG) h_steps += cnt;
                        if (STATS) {
                            st[kStSteps] += cnt;
                            st[kStSkipped] += cnt;
                            if (PD) st[kStPdSteps] += pd_flight ? cnt : 0u;
                        }
                        tau = tn;
                        k += cnt;
                        const float kn = (float)k;
#pragma unroll
                        for (int a = 0; a < 3; ++a) q[a] = c0[a] + kn * G[a];
                    }
                }
            }
            if (!flying) return;   // the run held the interaction
            const float kf = (float)k;
            // the anchor after the group and its uniform-cell word (loaded
            // before the group's voxels, so that those are used in the block
            // that loads them)
            float qn[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) qn[a] = c0[a] + (kf + (float)kPrefetch) * G[a];
            cellw = skips ? cell_word(gl, qn) : 0u;
            uint32_t code[kPrefetch];
            float vr[kPrefetch];
            // the group's gathers; with the object's edge copies (and steps of
            // at most a voxel) the coordinates need no clamp, one copy of the
            // loop per case under a branch that is uniform across the wave
            auto gather = [&](auto index) __attribute__((always_inline)) {
#pragma unroll
                for (int u = 0; u < kPrefetch; ++u) {
                    if (u % 4 == 0 && u > 0) {
#pragma unroll
                        for (int a = 0; a < 3; ++a) q[a] = c0[a] + (kf + (float)u) * G[a];
                    }
                    const uint32_t off = brick_offset(gl, index(q[0], gl.cmax[0]),
                                                      index(q[1], gl.cmax[1]),
                                                      index(q[2], gl.cmax[2]));
                    code[u] = dev(gl.vox)[off];
                    vr[u] = 0.0f;
                    if (BATCH ? gl.layout == kGeneric : MODE == kGeneric) vr[u] = dev(gl.vrho)[off];
                    if (u % 4 != 3) {
#pragma unroll
                        for (int a = 0; a < 3; ++a) q[a] = q[a] + G[a];
                    }
                }
            };
            if (gl.unclamped)
                gather([](float c, float) __attribute__((always_inline)) { return saturated_index(c); });
            else
                gather([](float c, float cmax) __attribute__((always_inline)) { return voxel_index(c, cmax); });
#pragma unroll
            for (int a = 0; a < 3; ++a) q[a] = qn[a];
            const uint32_t rem = nsteps - k;   // steps left in this flight
            bool act = true, hit = false;
            double inc_hit = 1.0;
            uint32_t code_hit = 0;
            // a pseudo-particle's chord takes its full steps in the loop and its
            // last (clipped) step after it, so its optical depth is exact
            const uint32_t full = PD && pd_flight ? rem - 1u : 0xFFFFFFFFu;
            double inc_last = 0.0;
            // the steps in order; inc_of(u) is the optical-depth increment of
            // step u.  One copy of the loop per way of finding it, chosen once
            // per group, keeps the per-step code free of layout branches.
            // Steps past the flight's end (u >= rem) are consumed like the
            // others: their centres are clamped into the grid, and a group that
            // takes k to nsteps or beyond ends the flight whatever it found
            // there, so they change nothing but the per-step counts, which the
            // counting variants keep exact.
            auto consume = [&](auto inc_of) __attribute__((always_inline)) {
#pragma unroll
                for (int u = 0; u < kPrefetch; ++u) {
                    const double inc = inc_of(u);
                    const double tn = tau + inc;
                    const bool reach = act && (tn >= ts);
                    if (DEBUG) h_steps += act && (uint32_t)u < rem ? 1u : 0u;
                    if (STATS) st[kStSteps] += act && (uint32_t)u < rem ? 1ull : 0ull;
                    if (STATS && PD)
                        st[kStPdSteps] += pd_flight && act && (uint32_t)u < rem ? 1ull : 0ull;
                    hit = hit || reach;
                    inc_hit = reach ? inc : inc_hit;
                    code_hit = reach ? code[u] : code_hit;
                    if (PD) inc_last = (uint32_t)u == full ? inc : inc_last;
                    const bool adv = act && !reach && (!PD || (uint32_t)u < full);
                    tau = adv ? tn : tau;
                    k += adv ? 1u : 0u;
                    act = adv;
                }
            };
            if (lay == kPaletteLane) {
                // one 24-bit multiply-add for the LDS address
                consume([&](int u) __attribute__((always_inline)) -> double {
                    return *(const double *)((const char *)inc_pal + __umul24(code[u], bs8));
                });
            } else {
                // density and material of the voxel: the gathered density and
                // code (generic layout), replaced by the palette entry's
                consume([&](int u) __attribute__((always_inline)) -> double {
                    float rho = vr[u];
                    uint32_t id = code[u];
                    if (lay == kPaletteShared) {
                        rho = BATCH ? dev(gl.pal_rho)[code[u]] : s_pal_rho[code[u]];
                        id = BATCH ? dev(gl.pal_id)[code[u]] : s_pal_id[code[u]];
                    }
                    const float mu = rho * mm[id * bs];
                    return __builtin_rint((double)mu * step32) * 2.3283064365386963e-10;
                });
            }
            if (PD && pd_flight) {
                if (rem <= (uint32_t)kPrefetch) {
                    // the chord's last step was in this group: add it, clipped
                    double r = (double)last / (double)p.step;
                    r = r > 1.0 ? 1.0 : r;
                    tau = tau + on_grid(inc_last * r);
                    k = nsteps;
                    event = 3;
                    flying = false;
                }
            } else if (k >= nsteps) {
                // the flight ended inside the group (or exactly at its end)
                event = 2;
                flying = false;
            } else if (hit) {
                if (k + 1u == nsteps) {
                    // the last step is shorter: its increment is scaled, and the
                    // photon may leave the object instead
                    double r = (double)last / (double)p.step;
                    r = r > 1.0 ? 1.0 : r;
                    const double inc_l = on_grid(inc_hit * r);
                    if (tau + inc_l >= ts) {
                        interact(code_hit, inc_l, last, false);
                    } else {
                        event = 2;
                        flying = false;
                    }
                } else {
                    interact(code_hit, inc_hit, p.step, false);
                }
            }
            });
        }
        };
        if (!BATCH) {
            march([&](auto f) __attribute__((always_inline)) { f(p.G); });
        } else {
            // no flight starts while marching: when every flying lane is on one
            // object, its descriptor is read once for the whole march
            const unsigned long long fl = __ballot(flying);
            const int g0 = fl ? __builtin_amdgcn_readlane(gi, __ffsll(fl) - 1) : 0;
            if (fl != 0ull && __ballot(flying && gi != g0) == 0ull) {
                VoxelGrid g;
                ConstWord *src = (ConstWord *)(p.grids + g0);
                uint32_t *dst = (uint32_t *)&g;
#pragma unroll
                for (int w = 0; w < (int)(sizeof(VoxelGrid) / 4); ++w) dst[w] = src[w];
                march([&](auto f) __attribute__((always_inline)) {
                    if (flying) f(g);
                });
            } else {
                march([&](auto f) __attribute__((always_inline)) { with_grid(true, f); });
            }
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

// March probe: the voxel gathers of the march and nothing else.  Each lane
// takes rays (the birth directions of photon ids from the launch counter)
// and marches each straight through the object with the transport's step
// centres, clamps, layout and prefetch groups, adding up the codes it
// gathers (sum[0]) and the steps it takes (sum[1]); no optical depth,
// interactions, energies or tallies.  Dead lanes are refilled once
// `event_batch` of them wait.  Its step rate is the
// ceiling of the transport's march on the same object.
template <int MODE>
__global__ void __launch_bounds__(256) march_probe_kernel(const KParams p,
                                                          unsigned long long *sum) {
    const int lane = (int)__lane_id();
    const VoxelGrid &gl = p.G;
    bool alive = false, exhausted = false;
    float c0[3] = {0.0f, 0.0f, 0.0f}, q[3] = {0.0f, 0.0f, 0.0f}, G[3] = {0.0f, 0.0f, 0.0f};
    uint32_t k = 0, nsteps = 0;
    unsigned long long acc = 0, taken = 0;
    for (;;) {
        if (!exhausted && __popcll(__ballot(!alive)) >= (unsigned)p.event_batch) {
            const unsigned long long dead = __ballot(!alive);
            const unsigned nd = (unsigned)__popcll(dead);
            const int leader = __ffsll(dead) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(p.counter, (unsigned long long)nd);
            base = lane_value(base, leader);
            const unsigned long long got =
                base < p.n ? (p.n - base < nd ? p.n - base : nd) : 0ull;
            if (got < nd) exhausted = true;
            if (!alive) {
                const unsigned long long rank =
                    (unsigned long long)__popcll(dead & ((1ull << lane) - 1ull));
                if (rank < got) {
                    PhotonStream rng;
                    rng.reset(p.first + base + rank, p.key0, p.key1);
                    (void)rng.raw();                       // the energy draw
                    float o[3], d[3], tin, tout;
                    cone_direction(p.F, rng, d);
#pragma unroll
                    for (int a = 0; a < 3; ++a) o[a] = p.F.S[a];
                    if (box_entry(gl, o, d, tin, tout)) {
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            const float pin = o[a] + d[a] * tin;
                            G[a] = (d[a] * gl.inv_h) * p.step;
                            c0[a] = (pin - gl.lo[a]) * gl.inv_h + 0.5f * G[a];
                            q[a] = c0[a] + 0.0f * G[a];
                        }
                        nsteps = step_count(tout - tin, p.step);
                        k = 0;
                        alive = nsteps > 0u;
                    }
                }
            }
        }
        if (!__any(alive)) {
            if (exhausted) break;
            continue;
        }
        if (alive) {
            uint32_t code[kPrefetch];
            float vr[kPrefetch];
            const float kf = (float)k;
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) {
                if (u % 4 == 0 && u > 0) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) q[a] = c0[a] + (kf + (float)u) * G[a];
                }
                const uint32_t off = brick_offset(gl, voxel_index(q[0], gl.cmax[0]),
                                                  voxel_index(q[1], gl.cmax[1]),
                                                  voxel_index(q[2], gl.cmax[2]));
                code[u] = gl.vox[off];
                if (MODE == kGeneric) vr[u] = gl.vrho[off];
                if (u % 4 != 3) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) q[a] = q[a] + G[a];
                }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) q[a] = c0[a] + (kf + (float)kPrefetch) * G[a];
            const uint32_t rem = nsteps - k;
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) {
                uint32_t c = code[u];
                if (MODE == kGeneric) c += __float_as_uint(vr[u]) & 1u;
                acc += (uint32_t)u < rem ? c : 0u;
            }
            taken += rem < (uint32_t)kPrefetch ? rem : (uint32_t)kPrefetch;
            k += kPrefetch;
            if (k >= nsteps) alive = false;
        }
    }
    const unsigned long long t = wave_sum(acc), ns = wave_sum(taken);
    if (lane == 0 && t) atomicAdd(sum, t);
    if (lane == 0 && ns) atomicAdd(sum + 1, ns);
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
        float ct = 2.0f, e2 = e_kev;       // a null collision keeps cosine 2
        (void)compton_collision<true>(s, p, material, e_kev, ct, e2);
        cos_out[i] = ct;
        if (e_out) e_out[i] = e2;
    }
}

size_t transport_lds_bytes(const KParams &p, int layout, int block) {
    const int pal = layout == kPaletteLane ? p.G.n_pal : 0;
    return (size_t)(kLdsHeader + p.n_mat * block) * sizeof(float) +
           (size_t)pal * block * sizeof(double);
}

// batches keep a per-lane palette table as large as the largest per-lane palette
size_t batch_lds_bytes(const KParams &p, int max_lane_palette, int block) {
    return (size_t)(kLdsHeader + p.n_mat * block) * sizeof(float) +
           (size_t)max_lane_palette * block * sizeof(double);
}

// the kernel with or without the binding-effect samplers, as p.phys asks
template <int MODE, bool BATCH, bool STATS, bool DEBUG, bool PD>
static void launch_k(const KParams &p, int grid, int block, size_t lds, hipStream_t stream) {
    if (p.phys)
        hipLaunchKernelGGL((transport_kernel<MODE, BATCH, STATS, DEBUG, PD, true>), dim3(grid),
                           dim3(block), lds, stream, p);
    else
        hipLaunchKernelGGL((transport_kernel<MODE, BATCH, STATS, DEBUG, PD, false>), dim3(grid),
                           dim3(block), lds, stream, p);
}

template <int MODE>
static hipError_t launch_mode(const KParams &p, int grid, int block, bool stats, bool debug,
                              hipStream_t stream) {
    const size_t lds = transport_lds_bytes(p, MODE, block);
    const bool pd = p.pd_split > 0;   // point-detector scoring of the scatter image
    if (debug)
        launch_k<MODE, false, false, true, false>(p, grid, block, lds, stream);
    else if (stats && pd)
        launch_k<MODE, false, true, false, true>(p, grid, block, lds, stream);
    else if (pd)
        launch_k<MODE, false, false, false, true>(p, grid, block, lds, stream);
    else if (stats)
        launch_k<MODE, false, true, false, false>(p, grid, block, lds, stream);
    else
        launch_k<MODE, false, false, false, false>(p, grid, block, lds, stream);
    return hipGetLastError();
}

hipError_t launch_transport(const KParams &p, int layout, int grid, int block, bool stats,
                            bool debug, hipStream_t stream) {
    if (layout == kPaletteLane) return launch_mode<kPaletteLane>(p, grid, block, stats, debug, stream);
    if (layout == kPaletteShared)
        return launch_mode<kPaletteShared>(p, grid, block, stats, debug, stream);
    return launch_mode<kGeneric>(p, grid, block, stats, debug, stream);
}

hipError_t launch_batch(const KParams &p, int max_lane_palette, int grid, int block, bool stats,
                        hipStream_t stream) {
    const size_t lds = batch_lds_bytes(p, max_lane_palette, block);
    if (stats)
        launch_k<kPaletteLane, true, true, false, false>(p, grid, block, lds, stream);
    else
        launch_k<kPaletteLane, true, false, false, false>(p, grid, block, lds, stream);
    return hipGetLastError();
}

hipError_t launch_march_probe(const KParams &p, int layout, int grid, int block,
                              unsigned long long *sum, hipStream_t stream) {
    if (layout == kPaletteLane)
        hipLaunchKernelGGL(march_probe_kernel<kPaletteLane>, dim3(grid), dim3(block), 0, stream,
                           p, sum);
    else if (layout == kPaletteShared)
        hipLaunchKernelGGL(march_probe_kernel<kPaletteShared>, dim3(grid), dim3(block), 0,
                           stream, p, sum);
    else
        hipLaunchKernelGGL(march_probe_kernel<kGeneric>, dim3(grid), dim3(block), 0, stream, p,
                           sum);
    return hipGetLastError();
}

// ------------------------------------------------------------------ eq. (7)
// Deterministic primary: the expected primary tally per emitted photon, one
// thread per pixel.  The pixel is integrated over sub x sub sub-pixel rays from
// the source (midpoint rule, d(Omega) = cos(gamma) dA / R^2 over the cone's
// Omega = 2 pi (1 - cos(theta_max))); each ray is marched with the transport's
// step rule (nominal step centres re-anchored every 4 steps, last step clipped)
// and collects rho * length per material in the lane's LDS column (fp64); the
// spectrum sum uses per bin the draw probability times eta(E) (bin_w) and mu
// per unit density per material (bin_mu, [n_bins][n_mat]), both from the host.
template <int MODE>
__global__ void __launch_bounds__(128) primary_kernel(const KParams p, int sub,
                                                      const double *bin_w, const float *bin_mu,
                                                      int n_bins, float *out) {
    extern __shared__ double plds[];
    float *s_pal_rho = (float *)plds;                     // [256]
    uint8_t *s_pal_id = (uint8_t *)(s_pal_rho + 256);     // [256]
    double *lam = plds + 160 + threadIdx.x;               // [n_mat] with stride blockDim
    const int bs = blockDim.x;
    if (MODE != kGeneric) {
        for (int i = threadIdx.x; i < p.G.n_pal; i += bs) {
            s_pal_rho[i] = p.G.pal_rho[i];
            s_pal_id[i] = p.G.pal_id[i];
        }
    }
    __syncthreads();
    const int pix = blockIdx.x * bs + threadIdx.x;
    if (pix >= p.nu * p.nv) return;
    const int iu = pix % p.nu, iv = pix / p.nu;
    const ProjFrame &F = p.F;
    const VoxelGrid &gr = p.G;
    const double da = (double)p.pu * (double)p.pv / ((double)sub * sub);
    double acc = 0.0;
    for (int b = 0; b < sub; ++b)
        for (int a = 0; a < sub; ++a) {
            const double u = -(double)F.hu + ((double)iu + (a + 0.5) / sub) * p.pu;
            const double v = -(double)F.hv + ((double)iv + (b + 0.5) / sub) * p.pv;
            double w[3], r2 = 0.0, ax = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                w[k] = ((double)F.D[k] + u * F.eu[k] + v * F.ev[k]) - (double)F.S[k];
                r2 += w[k] * w[k];
            }
            const double R = sqrt(r2);
            float d[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                d[k] = (float)(w[k] / R);
                ax += w[k] / R * (double)F.ax[k];
            }
            for (int m = 0; m < p.n_mat; ++m) lam[m * bs] = 0.0;
            float tin, tout;
            if (box_entry(gr, F.S, d, tin, tout)) {
                float c0[3], G[3], q[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const float pin = F.S[k] + d[k] * tin;
                    G[k] = (d[k] * gr.inv_h) * p.step;
                    c0[k] = (pin - gr.lo[k]) * gr.inv_h + 0.5f * G[k];
                    q[k] = c0[k];
                }
                const float L = tout - tin;
                for (uint32_t k = 0;; ++k) {
                    const float a0 = (float)k * p.step;
                    if (!(a0 < L)) break;
                    if ((k & 3u) == 0u) {
#pragma unroll
                        for (int t = 0; t < 3; ++t) q[t] = c0[t] + (float)k * G[t];
                    } else {
#pragma unroll
                        for (int t = 0; t < 3; ++t) q[t] = q[t] + G[t];
                    }
                    const uint32_t off = brick_offset(gr, voxel_index(q[0], gr.cmax[0]),
                                                      voxel_index(q[1], gr.cmax[1]),
                                                      voxel_index(q[2], gr.cmax[2]));
                    const uint32_t code = dev(gr.vox)[off];
                    float rho;
                    int id;
                    if (MODE == kGeneric) {
                        rho = dev(gr.vrho)[off];
                        id = (int)code;
                    } else {
                        rho = s_pal_rho[code];
                        id = s_pal_id[code];
                    }
                    const double len =
                        (float)(k + 1u) * p.step < L ? (double)p.step : (double)(L - a0);
                    lam[id * bs] += (double)rho * len;
                }
            }
            double e_sum = 0.0;
            for (int k = 0; k < n_bins; ++k) {
                double tau = 0.0;
                for (int m = 0; m < p.n_mat; ++m)
                    tau += lam[m * bs] * (double)bin_mu[k * p.n_mat + m];
                e_sum += bin_w[k] * exp(-tau);
            }
            acc += e_sum * (ax * da / r2);
        }
    out[pix] = (float)(acc / (6.283185307179586 * (double)F.omc));
}

hipError_t launch_primary(const KParams &p, int sub, const double *bin_w, const float *bin_mu,
                          int n_bins, float *out, hipStream_t stream) {
    const int block = 128;
    const int grid = (p.nu * p.nv + block - 1) / block;
    const size_t lds = 160 * sizeof(double) + (size_t)p.n_mat * block * sizeof(double);
    if (p.G.layout == kGeneric)
        hipLaunchKernelGGL(primary_kernel<kGeneric>, dim3(grid), dim3(block), lds, stream, p, sub,
                           bin_w, bin_mu, n_bins, out);
    else
        hipLaunchKernelGGL(primary_kernel<kPaletteLane>, dim3(grid), dim3(block), lds, stream, p,
                           sub, bin_w, bin_mu, n_bins, out);
    return hipGetLastError();
}

// Angular interpolation (section II-C-3): scatter maps simulated at every
// other angle of a circle, sim[n_sim][n_pix] -> full[2 n_sim][n_pix], the even
// entries copied, the odd ones the mean of their two neighbours (wrapping).
__global__ void interp_angles_kernel(const float *sim, int n_sim, uint64_t n_pix, float *full) {
    const uint64_t n = (uint64_t)n_sim * n_pix;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const uint64_t i = t / n_pix, px = t - i * n_pix;
        const uint64_t j = i + 1 == (uint64_t)n_sim ? 0 : i + 1;
        const float a = sim[t], b = sim[j * n_pix + px];
        full[(2 * i) * n_pix + px] = a;
        full[(2 * i + 1) * n_pix + px] = 0.5f * (a + b);
    }
}

hipError_t launch_interp_angles(const float *sim, int n_sim, uint64_t n_pix, float *full,
                                hipStream_t stream) {
    const uint64_t n = (uint64_t)n_sim * n_pix;
    uint64_t grid = (n + 255) / 256;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(interp_angles_kernel, dim3((unsigned)grid), dim3(256), 0, stream, sim,
                       n_sim, n_pix, full);
    return hipGetLastError();
}

// zero a batch's images and counters: a plain fill kernel, so the batch can
// be captured in a graph without memset nodes
__global__ void clear_kernel(unsigned long long *a, size_t na, unsigned long long *b, size_t nb) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < na; i += stride) a[i] = 0ull;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += stride) b[i] = 0ull;
}

hipError_t launch_clear(unsigned long long *a, size_t na, unsigned long long *b, size_t nb,
                        hipStream_t stream) {
    const size_t n = na > nb ? na : nb;
    const int block = 256;
    size_t grid = (n + block - 1) / block;
    if (grid > 4096) grid = 4096;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL(clear_kernel, dim3((unsigned)grid), dim3(block), 0, stream, a, na, b, nb);
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

template <int MODE, bool BATCH, bool STATS, bool PD>
static int occ_k(int block, size_t lds, bool bind) {
    int nb = 0;
    if (bind)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, transport_kernel<MODE, BATCH, STATS, false, PD, true>, block, lds);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, transport_kernel<MODE, BATCH, STATS, false, PD, false>, block, lds);
    return nb;
}

template <int MODE, bool BATCH>
static int occupancy(int block, size_t lds, bool stats, bool pd, bool bind) {
    if constexpr (!BATCH) {
        if (pd)
            return stats ? occ_k<MODE, false, true, true>(block, lds, bind)
                         : occ_k<MODE, false, false, true>(block, lds, bind);
    }
    return stats ? occ_k<MODE, BATCH, true, false>(block, lds, bind)
                 : occ_k<MODE, BATCH, false, false>(block, lds, bind);
}

int march_probe_blocks_per_cu(int layout, int block) {
    int nb = 0;
    if (layout == kPaletteLane)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, march_probe_kernel<kPaletteLane>,
                                                           block, 0);
    else if (layout == kPaletteShared)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, march_probe_kernel<kPaletteShared>, block, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, march_probe_kernel<kGeneric>,
                                                           block, 0);
    return nb > 0 ? nb : 1;
}

int transport_blocks_per_cu(const KParams &p, int layout, int block, bool stats) {
    const size_t lds = transport_lds_bytes(p, layout, block);
    const bool pd = p.pd_split > 0, bind = p.phys != 0;
    int nb = layout == kPaletteLane ? occupancy<kPaletteLane, false>(block, lds, stats, pd, bind)
             : layout == kPaletteShared
                 ? occupancy<kPaletteShared, false>(block, lds, stats, pd, bind)
                 : occupancy<kGeneric, false>(block, lds, stats, pd, bind);
    return nb > 0 ? nb : 1;
}

int batch_blocks_per_cu(const KParams &p, int max_lane_palette, int block, bool stats) {
    const int nb = occupancy<kPaletteLane, true>(block, batch_lds_bytes(p, max_lane_palette, block),
                                                stats, false, p.phys != 0);
    return nb > 0 ? nb : 1;
}

}  // namespace mcx
