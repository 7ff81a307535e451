// Kernels of the learned scatter denoiser / up-sampler: a 2-D U-Net with
// bf16 weights and activations, fp32 accumulation on the gfx950 matrix cores,
// trained by its own backward kernels.  It stands in for the smoothing and
// interpolation of the paper's correction loop (section II-C-3/4).
//
// Layout: activations NHWC bf16 ([n][y][x][c], channels fastest) addressed
// as (pointer, channel stride ld, channel offset) so concatenated skip
// connections are channel slices of one buffer; 3x3 conv weights bf16
// [Cout][tap][Cin] with tap = 3*(dy+1) + (dx+1).  Channel counts of convolution
// inputs are multiples of 16.
//
// conv3x3_kernel is an implicit GEMM: rows = pixels, columns = output
// channels, reduction k = (tap, input channel).  Each lane's eight k values
// of one MFMA operand are eight consecutive channels, a single 16-byte load
// straight from global memory (L1/L2 serve the reuse), issued a few k-steps
// ahead of the matrix products.  A 32*WM x 32*WN tile is computed with
// v_mfma_f32_32x32x16_bf16 by one wave, or, for layers with few tiles, by 2 or
// 4 waves over interleaved k-steps whose partial sums meet in LDS.  The same
// kernel computes the input gradient of a convolution from its output
// gradient and the flipped, transposed weights.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nn_params.hpp"

namespace mcx {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}

// round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

#ifndef MCX_CONV_DEPTH
#define MCX_CONV_DEPTH 3
#endif
constexpr int kConvDepth = MCX_CONV_DEPTH;   // k-steps of operands in flight
constexpr int kEpStride = 40;   // floats per staged row: the two row groups of a
                                // store fall on disjoint LDS banks

// the wave's LDS writes made visible to all its lanes
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Epilogue of a wave's 32*WM x 32*WN output tile (pixels px0.., channels
// co0..): bias, ReLU, mask, fp32 and bf16 stores, accumulation.  Element r of
// a 32x32 accumulator is row 8*(r/4) + 4*(lane/32) + r%4, column lane%32.
// When the channel count is a multiple of 16 and the rows are 16-byte
// aligned, a slab of 32 channels is turned around in `stage` (32 x kEpStride
// floats of LDS owned by the wave; row = pixel), so that each lane finishes
// 16 consecutive channels of one pixel with 16-byte loads and stores;
// otherwise element by element.
template <int WM, int WN>
__device__ __forceinline__ void conv_epilogue(const ConvArgs &a, f32x16 (&acc)[WM][WN], int px0,
                                              int co0, int npix, float *stage, int lane) {
    const int kh = lane >> 5, lr = lane & 31;
    const bool vec_ok =
        (a.y == nullptr || (((a.ldy | a.yoff) & 7) == 0 && ((uintptr_t)a.y & 15) == 0)) &&
        (a.mask == nullptr || (((a.ldm | a.moff) & 7) == 0 && ((uintptr_t)a.mask & 15) == 0)) &&
        (a.yf == nullptr || ((a.cout & 3) == 0 && ((uintptr_t)a.yf & 15) == 0)) &&
        (a.bias == nullptr || ((uintptr_t)a.bias & 15) == 0);
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            const int cs = co0 + j * 32;
            if (vec_ok && (a.cout & 15) == 0 && cs < a.cout) {
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    stage[(8 * (r >> 2) + 4 * kh + (r & 3)) * kEpStride + lr] = acc[i][j][r];
                wave_sync();
                const int row = lane & 31, half = lane >> 5;
                float v[16];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float4 t = *(const float4 *)(stage + row * kEpStride + half * 16 + 4 * q);
                    v[4 * q] = t.x;
                    v[4 * q + 1] = t.y;
                    v[4 * q + 2] = t.z;
                    v[4 * q + 3] = t.w;
                }
                wave_sync();
                const int p = px0 + i * 32 + row;
                const int co = cs + half * 16;
                if (p >= npix || co >= a.cout) continue;
                if (a.bias) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float4 t = ((const float4 *)(a.bias + co))[q];
                        v[4 * q] += t.x;
                        v[4 * q + 1] += t.y;
                        v[4 * q + 2] += t.z;
                        v[4 * q + 3] += t.w;
                    }
                }
                if (a.relu) {
#pragma unroll
                    for (int e = 0; e < 16; ++e) v[e] = fmaxf(v[e], 0.0f);
                }
                if (a.mask) {
                    const uint4 *mp = (const uint4 *)(a.mask + (size_t)p * a.ldm + a.moff + co);
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const uint4 m = mp[q];
                        const uint32_t mw[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const uint16_t h = (uint16_t)(mw[e >> 1] >> (16 * (e & 1)));
                            if (!(bf16_to_f32(h) > 0.0f)) v[8 * q + e] = 0.0f;
                        }
                    }
                }
                if (a.yf) {
                    float4 *fp = (float4 *)(a.yf + (size_t)p * a.cout + co);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        fp[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
                }
                if (a.y) {
                    uint4 *dp = (uint4 *)(a.y + (size_t)p * a.ldy + a.yoff + co);
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        uint32_t ow[4];
                        uint32_t iw[4] = {0u, 0u, 0u, 0u};
                        if (a.accumulate) {
                            const uint4 t = dp[q];
                            iw[0] = t.x;
                            iw[1] = t.y;
                            iw[2] = t.z;
                            iw[3] = t.w;
                        }
#pragma unroll
                        for (int e2 = 0; e2 < 4; ++e2) {
                            float lo = v[8 * q + 2 * e2], hi = v[8 * q + 2 * e2 + 1];
                            if (a.accumulate) {
                                lo += bf16_to_f32((uint16_t)(iw[e2] & 0xffffu));
                                hi += bf16_to_f32((uint16_t)(iw[e2] >> 16));
                            }
                            ow[e2] = (uint32_t)f32_to_bf16(lo) | ((uint32_t)f32_to_bf16(hi) << 16);
                        }
                        dp[q] = make_uint4(ow[0], ow[1], ow[2], ow[3]);
                    }
                }
                continue;
            }
            const int co = cs + lr;
            if (co >= a.cout) continue;
            const float b = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int p = px0 + i * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
                if (p >= npix) continue;
                float v = acc[i][j][r] + b;
                if (a.relu) v = fmaxf(v, 0.0f);
                if (a.mask && !(bf16_to_f32(a.mask[(size_t)p * a.ldm + a.moff + co]) > 0.0f)) v = 0.0f;
                if (a.yf) a.yf[(size_t)p * a.cout + co] = v;
                if (a.y) {
                    uint16_t *dst = a.y + (size_t)p * a.ldy + a.yoff + co;
                    if (a.accumulate) v += bf16_to_f32(*dst);
                    *dst = f32_to_bf16(v);
                }
            }
        }
}

template <int WM, int WN, int KS>
__global__ void __launch_bounds__(256) conv3x3_kernel(const ConvArgs a) {
    // 4 waves: 4 / KS output tiles of 32*WM pixels x 32*WN channels, each
    // computed by KS waves over interleaved k-steps and summed in LDS in a
    // fixed order (deterministic)
    extern __shared__ float s_part[];
    constexpr int TPB = 4 / KS;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tile = wave / KS, ks = wave - tile * KS;
    const int hw = a.h * a.w_;
    const int npix = a.n * hw;
    const int px0 = (blockIdx.x * TPB + tile) * (32 * WM);
    const int co0 = blockIdx.y * (32 * WN);
    const bool live = px0 < npix;       // no early return: the block meets at a barrier
    const int kh = lane >> 5;           // which 8-channel half of the 16-k slice
    const int lr = lane & 31;

    int pn[WM], py[WM], pxx[WM];
    bool pv[WM];
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        const int p = px0 + i * 32 + lr;
        pv[i] = p < npix;
        const int pp = pv[i] ? p : 0;
        pn[i] = pp / hw;
        const int r = pp - pn[i] * hw;
        py[i] = r / a.w_;
        pxx[i] = r - py[i] * a.w_;
    }
    f32x16 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    // k-step k: tap k / kc, channels 16 * (k % kc) .. +16
    const int kc = a.cin >> 4;
    const int K = 9 * kc;
    const size_t wk = (size_t)9 * a.cin;
    // Loads are issued without branches, so that the compiler can count them
    // in flight: a k-step past the end reloads the last one (its products are
    // skipped), and a tap outside the image reads pixel 0 of the tensor and
    // is masked to zero when used.
    auto load = [&](int k, bf16x8 (&av)[WM], bf16x8 (&bv)[WN], bool (&ok)[WM])
        __attribute__((always_inline)) {
        k = k < K ? k : K - 1;
        const int tap = k / kc;
        const int c0 = (k - tap * kc) << 4;
        const int dy = tap / 3 - 1, dx = tap - 3 * (tap / 3) - 1;
#pragma unroll
        for (int i = 0; i < WM; ++i) {
            const int yy = py[i] + dy, xx = pxx[i] + dx;
            ok[i] = pv[i] && yy >= 0 && yy < a.h && xx >= 0 && xx < a.w_;
            const size_t pix = ok[i] ? (size_t)(pn[i] * a.h + yy) * a.w_ + xx : 0;
            av[i] = *(const bf16x8 *)(a.x + pix * a.ldx + a.xoff + c0 + kh * 8);
        }
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            const int co = co0 + j * 32 + lr;
            bv[j] = *(const bf16x8 *)(a.w + (size_t)co * wk + (size_t)tap * a.cin + c0 + kh * 8);
        }
    };
    if (live && ks < K) {
        // kConvDepth k-steps of operands in flight ahead of the matrix
        // products: a ring of register buffers, each refilled right after its
        // products are issued
        bf16x8 av[kConvDepth][WM], bv[kConvDepth][WN];
        bool ok[kConvDepth][WM];
        const bf16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < kConvDepth; ++s) load(ks + s * KS, av[s], bv[s], ok[s]);
        for (int k = ks; k < K; k += kConvDepth * KS) {
#pragma unroll
            for (int s = 0; s < kConvDepth; ++s) {
                // a step past the end multiplies zeros (no branch: the
                // accumulators stay in the matrix registers)
                const int kk = k + s * KS;
#pragma unroll
                for (int i = 0; i < WM; ++i) {
                    const bf16x8 x = (ok[s][i] && kk < K) ? av[s][i] : zero;
#pragma unroll
                    for (int j = 0; j < WN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, bv[s][j], acc[i][j],
                                                                             0, 0, 0);
                }
                load(kk + kConvDepth * KS, av[s], bv[s], ok[s]);
            }
        }
    }
    if constexpr (KS > 1) {
        // partial tiles of waves ks = 1 .. KS-1, [tile][ks-1][register][lane]
        constexpr int R = WM * WN * 16;
        float *mine = s_part + ((size_t)(tile * (KS - 1) + (ks > 0 ? ks - 1 : 0)) * R) * 64;
        if (ks > 0) {
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r) mine[((i * WN + j) * 16 + r) * 64 + lane] = acc[i][j][r];
        }
        __syncthreads();
        if (ks > 0) return;
        const float *base = s_part + (size_t)tile * (KS - 1) * R * 64;
#pragma unroll 1
        for (int q = 0; q < KS - 1; ++q) {
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        acc[i][j][r] += base[((size_t)q * R + (i * WN + j) * 16 + r) * 64 + lane];
        }
    }
    if (!live) return;
    // this wave's 32 x kEpStride staging tile: in its tile's own (already
    // consumed) partial-sum region, or its own slot
    static_assert(KS == 1 || 32 * kEpStride <= WM * WN * 16 * 64, "staging tile fits a partial");
    float *stage = KS > 1 ? s_part + (size_t)tile * (KS - 1) * (WM * WN * 16 * 64)
                          : s_part + wave * (32 * kEpStride);
    conv_epilogue<WM, WN>(a, acc, px0, co0, npix, stage, lane);
}

// The same convolution for images whose width is a multiple of 64, on layers
// with enough tiles for one wave each (2 x 32 pixels x 32*WN channels): a
// wave's 64 output pixels lie in one image row.  The reduction runs over
// 16-channel chunks; for each chunk every wave stages the three input rows
// around its pixels (66 pixels wide, zeros outside the image) and the block
// stages the nine taps' weights, pixel- and channel-major as in memory, in
// LDS, so each input value is loaded once per chunk instead of once per tap.
// The next chunk's loads are in flight in registers while the products of
// the current one are issued.
constexpr int kLdsInPx = 66;                          // staged pixels per row
constexpr int kLdsInElems = 3 * kLdsInPx * 16;        // one wave's rows, one chunk (bf16)

template <int WN>
constexpr int lds_w_elems() { return 9 * 32 * WN * 16; }   // the block's weights, one chunk

template <int WN>
constexpr size_t conv_lds_bytes() { return (4 * kLdsInElems + lds_w_elems<WN>()) * 2; }

#ifndef MCX_CONV_LDS
#define MCX_CONV_LDS 1
#endif
constexpr bool conv_lds_enabled = MCX_CONV_LDS != 0;
#ifndef MCX_CONV_HALF_TILES
#define MCX_CONV_HALF_TILES 1
#endif
constexpr bool conv_half_tiles = MCX_CONV_HALF_TILES != 0;

template <int WN>
__global__ void __launch_bounds__(256) conv3x3_lds_kernel(const ConvArgs a) {
    constexpr int WM = 2;
    constexpr int kInItems = 3 * kLdsInPx * 2;                  // 16-byte items per wave
    constexpr int kInPer = (kInItems + 63) / 64;
    constexpr int kWItems = 9 * 32 * WN * 2;                    // 16-byte items per block
    constexpr int kWPer = (kWItems + 255) / 256;
    static_assert(32 * kEpStride * 4 <= kLdsInElems * 2, "epilogue staging fits a wave's rows");
    extern __shared__ __align__(16) float s_dyn[];
    uint16_t *lds = (uint16_t *)s_dyn;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kh = lane >> 5, lr = lane & 31;
    const int npix = a.n * a.h * a.w_;
    const int px0 = (blockIdx.x * 4 + wave) * (32 * WM);
    const int co0 = blockIdx.y * (32 * WN);
    const bool live = px0 < npix;       // no early return: the block meets at barriers
    const int row = live ? px0 / a.w_ : 0;   // n * h + y of the wave's pixels
    const int x0 = px0 - row * a.w_;
    const int yy = row % a.h;
    const int kc = a.cin >> 4;
    const size_t wk = (size_t)9 * a.cin;
    uint4 rin[kInPer], rw[kWPer];
    auto load_chunk = [&](int c) __attribute__((always_inline)) {
#pragma unroll
        for (int m = 0; m < kInPer; ++m) {
            const int t = lane + 64 * m;
            const int q = t >> 1, r = q / kLdsInPx, px = q - r * kLdsInPx;
            const int y2 = yy + r - 1, x2 = x0 + px - 1;
            rin[m] = make_uint4(0u, 0u, 0u, 0u);
            if (live && t < kInItems && y2 >= 0 && y2 < a.h && x2 >= 0 && x2 < a.w_)
                rin[m] = *(const uint4 *)(a.x + ((size_t)(row + r - 1) * a.w_ + x2) * a.ldx +
                                          a.xoff + c * 16 + (t & 1) * 8);
        }
#pragma unroll
        for (int m = 0; m < kWPer; ++m) {
            const int u = threadIdx.x + 256 * m;
            const int rest = u >> 1, col = rest % (32 * WN), tap = rest / (32 * WN);
            rw[m] = make_uint4(0u, 0u, 0u, 0u);
            if (u < kWItems)
                rw[m] = *(const uint4 *)(a.w + (size_t)(co0 + col) * wk + (size_t)tap * a.cin +
                                         c * 16 + (u & 1) * 8);
        }
    };
    auto store_chunk = [&]() __attribute__((always_inline)) {
        uint16_t *in = lds + wave * kLdsInElems;
#pragma unroll
        for (int m = 0; m < kInPer; ++m) {
            const int t = lane + 64 * m;
            if (t < kInItems) *(uint4 *)(in + (t >> 1) * 16 + (t & 1) * 8) = rin[m];
        }
        uint16_t *wl = lds + 4 * kLdsInElems;
#pragma unroll
        for (int m = 0; m < kWPer; ++m) {
            const int u = threadIdx.x + 256 * m;
            if (u < kWItems) *(uint4 *)(wl + (u >> 1) * 16 + (u & 1) * 8) = rw[m];
        }
    };
    f32x16 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    load_chunk(0);
    store_chunk();
    __syncthreads();
    for (int c = 0; c < kc; ++c) {
        if (c + 1 < kc) load_chunk(c + 1);
        const uint16_t *in = lds + wave * kLdsInElems;
        const uint16_t *wl = lds + 4 * kLdsInElems;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                bf16x8 av[WM], bv[WN];
#pragma unroll
                for (int i = 0; i < WM; ++i)
                    av[i] = *(const bf16x8 *)(in + (r * kLdsInPx + i * 32 + lr + k) * 16 + kh * 8);
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    bv[j] = *(const bf16x8 *)(wl + ((3 * r + k) * 32 * WN + j * 32 + lr) * 16 +
                                              kh * 8);
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bv[j],
                                                                             acc[i][j], 0, 0, 0);
            }
        __syncthreads();       // every wave is done with this chunk
        if (c + 1 < kc) {
            store_chunk();
            __syncthreads();
        }
    }
    if (!live) return;
    // the epilogue stages in this wave's rows (no longer read)
    conv_epilogue<WM, WN>(a, acc, px0, co0, npix, (float *)(lds + wave * kLdsInElems), lane);
}

// The same staging for layers with few tiles, whose reduction is split over KS
// waves of a block (16-channel chunks c = ks, ks + KS, ...; partial tiles added
// in LDS in a fixed order).  Each wave stages its chunk's input window in its
// own LDS rows; the chunk's weights (nine taps) are loaded into registers
// through L1/L2 at once.  The window is the tile's image rows and one more on
// each side: for widths that are multiples of 64 one row of 66 pixels, for
// widths of 16 or 32 (a 64-pixel tile is 4 or 2 whole rows) the rows at their
// full width plus the zero columns at both ends.
template <int WM, int WN, int KS>
__global__ void __launch_bounds__(256) conv3x3_lds_split_kernel(const ConvArgs a) {
    constexpr int TPB = 4 / KS;
    constexpr int TPX = 32 * WM;                      // pixels per tile
    constexpr int R = WM * WN * 16;                   // floats per lane of a partial tile
    constexpr int kInPer = (3 * (TPX + 2) * 2 + 63) / 64;
    static_assert(3 * (TPX + 2) <= 3 * kLdsInPx, "a window fits a wave's rows");
    static_assert(32 * kEpStride <= R * 64, "epilogue staging fits a partial tile");
    extern __shared__ __align__(16) float s_dyn[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tile = wave / KS, ks = wave - tile * KS;
    const int kh = lane >> 5, lr = lane & 31;
    uint16_t *in = (uint16_t *)s_dyn + wave * kLdsInElems;
    const int npix = a.n * a.h * a.w_;
    const int px0 = (blockIdx.x * TPB + tile) * (32 * WM);
    const int co0 = blockIdx.y * (32 * WN);
    const bool live = px0 < npix;       // no early return: the block meets at barriers
    const bool wide = a.w_ >= TPX;
    const int nr = wide ? 1 : TPX / a.w_;             // image rows of the tile
    const int wn = wide ? TPX + 2 : a.w_ + 2;         // staged pixels per row
    const int row0 = live ? px0 / a.w_ : 0;           // n * h + y of the tile's first row
    const int xs = px0 - row0 * a.w_;                 // its first column (0 for whole rows)
    const int yy0 = row0 % a.h;
    const int items = (nr + 2) * wn * 2;              // 16-byte items of the window
    // staged pixel of this lane's rows for tap (0, 0)
    int aoff[WM];
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        const int j = i * 32 + lr;
        const int ry = wide ? 0 : j / a.w_;
        aoff[i] = ry * wn + (j - ry * (wide ? 0 : a.w_));
    }
    const int kc = a.cin >> 4;
    const size_t wk = (size_t)9 * a.cin;
    f32x16 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    uint4 rin[kInPer];
    auto load_chunk = [&](int c) __attribute__((always_inline)) {
#pragma unroll
        for (int m = 0; m < kInPer; ++m) {
            const int t = lane + 64 * m;
            const int q = t >> 1, r = q / wn, px = q - r * wn;
            const int y2 = yy0 + r - 1, x2 = xs + px - 1;
            rin[m] = make_uint4(0u, 0u, 0u, 0u);
            if (t < items && y2 >= 0 && y2 < a.h && x2 >= 0 && x2 < a.w_)
                rin[m] = *(const uint4 *)(a.x + ((size_t)(row0 + r - 1) * a.w_ + x2) * a.ldx +
                                          a.xoff + c * 16 + (t & 1) * 8);
        }
    };
    if (live && ks < kc) {
        load_chunk(ks);
        for (int c = ks; c < kc; c += KS) {
            // the chunk's nine taps of weights, all in flight at once (one wait
            // per chunk rather than one per tap)
            bf16x8 bw[9][WN];
#pragma unroll
            for (int tap = 0; tap < 9; ++tap)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    bw[tap][j] = *(const bf16x8 *)(a.w + (size_t)(co0 + j * 32 + lr) * wk +
                                                   (size_t)tap * a.cin + c * 16 + kh * 8);
#pragma unroll
            for (int m = 0; m < kInPer; ++m) {
                const int t = lane + 64 * m;
                if (t < items) *(uint4 *)(in + (t >> 1) * 16 + (t & 1) * 8) = rin[m];
            }
            wave_sync();
            if (c + KS < kc) load_chunk(c + KS);   // in flight during the products
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    bf16x8 av[WM];
#pragma unroll
                    for (int i = 0; i < WM; ++i)
                        av[i] = *(const bf16x8 *)(in + (aoff[i] + r * wn + k) * 16 + kh * 8);
#pragma unroll
                    for (int i = 0; i < WM; ++i)
#pragma unroll
                        for (int j = 0; j < WN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                av[i], bw[3 * r + k][j], acc[i][j], 0, 0, 0);
                }
            wave_sync();      // the next chunk overwrites the rows
        }
    }
    // partial tiles of waves ks = 1 .. KS-1 over the (no longer read) rows,
    // [tile][ks-1][register][lane]
    __syncthreads();
    float *mine = s_dyn + ((size_t)(tile * (KS - 1) + (ks > 0 ? ks - 1 : 0)) * R) * 64;
    if (ks > 0) {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) mine[((i * WN + j) * 16 + r) * 64 + lane] = acc[i][j][r];
    }
    __syncthreads();
    if (ks > 0) return;
    const float *base = s_dyn + (size_t)tile * (KS - 1) * R * 64;
#pragma unroll 1
    for (int q = 0; q < KS - 1; ++q) {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    acc[i][j][r] += base[((size_t)q * R + (i * WN + j) * 16 + r) * 64 + lane];
    }
    if (!live) return;
    conv_epilogue<WM, WN>(a, acc, px0, co0, npix, (float *)base, lane);
}

template <int WM, int WN, int KS>
constexpr size_t conv_lds_split_bytes() {
    constexpr size_t rows = 4 * kLdsInElems * 2;
    constexpr size_t parts = (size_t)(4 / KS) * (KS - 1) * WM * WN * 16 * 64 * sizeof(float);
    return rows > parts ? rows : parts;
}

// ---------------------------------------------------------------------------
// weight gradient: dW[co][tap][ci] = sum over pixels of dY[p][co] * X[p + tap][ci].
// One block = 4 waves = a 32(co) x 32(ci) tile of one tap over a pixel range;
// 16-pixel slices of dY and of the shifted X are staged in LDS transposed
// (channel-major) so each lane reads its 8 consecutive pixels in one 16-byte
// LDS load.  Per-split partial tiles are reduced in a fixed order by
// wgrad_group_kernel and wgrad_reduce_kernel, so gradients are deterministic.
__global__ void __launch_bounds__(256) wgrad_kernel(const WgradArgs a) {
    __shared__ uint16_t s_dy[4][32][16 + 8];   // [wave][co][pixel] (+8 pad)
    __shared__ uint16_t s_x[4][32][16 + 8];    // [wave][ci][pixel]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int co0 = blockIdx.x * 32;
    const int ci0 = (blockIdx.y % ((a.cin + 31) / 32)) * 32;
    const int tap = blockIdx.y / ((a.cin + 31) / 32);
    const int split = blockIdx.z;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int hw = a.h * a.w_, npix = a.n * hw;
    const int per = (npix + a.splits - 1) / a.splits;
    const int p_lo = split * per, p_hi = min(npix, p_lo + per);
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    const int kh = lane >> 5, lr = lane & 31;
    // each wave walks 16-pixel slices strided by 4 slices
    for (int p0 = p_lo + wave * 16; p0 < p_hi; p0 += 64) {
        // stage: lane handles pixel p0 + (lane & 15), channels 8*(lane >> 4) .. +8
        {
            const int pl = lane & 15, cq = lane >> 4;   // cq in 0..3: 8-channel groups
            const int p = p0 + pl;
            uint16_t vy[8], vx[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                vy[e] = 0;
                vx[e] = 0;
            }
            if (p < p_hi) {
                const int c = co0 + cq * 8;
                if (c < a.cout) {
                    const uint16_t *src = a.dy + (size_t)p * a.ldy + a.yoff + c;
#pragma unroll
                    for (int e = 0; e < 8; ++e) vy[e] = (c + e < a.cout) ? src[e] : (uint16_t)0;
                }
                const int nn = p / hw, rem = p - nn * hw, yy = rem / a.w_ + dy, xx = rem % a.w_ + dx;
                const int ci = ci0 + cq * 8;
                if (yy >= 0 && yy < a.h && xx >= 0 && xx < a.w_ && ci < a.cin) {
                    const bf16x8 v =
                        *(const bf16x8 *)(a.x + ((size_t)(nn * a.h + yy) * a.w_ + xx) * a.ldx + a.xoff + ci);
#pragma unroll
                    for (int e = 0; e < 8; ++e) vx[e] = (uint16_t)v[e];
                }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                s_dy[wave][cq * 8 + e][pl] = vy[e];
                s_x[wave][cq * 8 + e][pl] = vx[e];
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0);
        bf16x8 av, bv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            av[e] = (short)s_dy[wave][lr][kh * 8 + e];
            bv[e] = (short)s_x[wave][lr][kh * 8 + e];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        __builtin_amdgcn_wave_barrier();
    }
    // reduce the 4 waves' tiles through LDS, then write this split's partial
    __shared__ float s_acc[4][32][33];
#pragma unroll
    for (int r = 0; r < 16; ++r) s_acc[wave][8 * (r >> 2) + 4 * kh + (r & 3)][lr] = acc[r];
    __syncthreads();
    for (int t = threadIdx.x; t < 32 * 32; t += 256) {
        const int row = t >> 5, col = t & 31;
        const float s = ((s_acc[0][row][col] + s_acc[1][row][col]) + s_acc[2][row][col]) +
                        s_acc[3][row][col];
        const int co = co0 + row, ci = ci0 + col;
        if (co < a.cout && ci < a.cin)
            a.partial[(((size_t)split * 9 + tap) * a.cout + co) * a.cin + ci] = s;
    }
}

// dW[co][tap][ci] = sum over splits in order (fp32), optionally + bias grads
// The same weight gradient for images whose width is a multiple of 16, with
// all nine taps of a 32(co) x 32(ci) tile in one block: a wave takes 16-pixel
// slices of one image row, stages the slice of dY and the three input rows
// around it, 18 pixels wide (zeros outside the image), channel-major in its
// own LDS, and issues the nine taps' products from there.  Split ranges are
// whole slices; partial tiles are laid out as wgrad_kernel's.
constexpr int kWgStride = 24;   // bf16 per staged channel row (16-byte aligned rows)

__global__ void __launch_bounds__(256) wgrad9_kernel(const WgradArgs a) {
    __shared__ __align__(16) uint16_t s_dy[4][32][kWgStride];      // [wave][co][pixel]
    __shared__ __align__(16) uint16_t s_x[4][3][32][kWgStride];    // [wave][row][ci][pixel + 1]
    __shared__ float s_acc[4][32][33];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int co0 = blockIdx.x * 32, ci0 = blockIdx.y * 32, split = blockIdx.z;
    const int npix = a.n * a.h * a.w_;
    const int per = (((npix + a.splits - 1) / a.splits) + 15) & ~15;
    const int p_lo = min(npix, split * per), p_hi = min(npix, p_lo + per);
    f32x16 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
    const int kh = lane >> 5, lr = lane & 31;
    auto put8 = [](uint16_t *dst, int stride, uint4 v) __attribute__((always_inline)) {
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) dst[e * stride] = (uint16_t)(w4[e >> 1] >> (16 * (e & 1)));
    };
    for (int p0 = p_lo + wave * 16; p0 < p_hi; p0 += 64) {
        const int row = p0 / a.w_;            // n * h + y of the slice's row
        const int xx0 = p0 - row * a.w_;
        const int yy = row % a.h;
        {
            // dY: pixel p0 + (lane & 15), channels co0 + 8 * (lane >> 4) .. +8
            const int pl = lane & 15, c = co0 + (lane >> 4) * 8;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (c < a.cout) v = *(const uint4 *)(a.dy + (size_t)(p0 + pl) * a.ldy + a.yoff + c);
            put8(&s_dy[wave][c - co0][pl], kWgStride, v);
        }
        // input rows yy - 1 .. yy + 1, pixels xx0 - 1 .. xx0 + 16, 8 channels per item
        for (int t = lane; t < 3 * 18 * 4; t += 64) {
            const int cq = t & 3, q = t >> 2;
            const int r = q / 18, px = q - r * 18;
            const int y2 = yy + r - 1, x2 = xx0 + px - 1, c = ci0 + cq * 8;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (y2 >= 0 && y2 < a.h && x2 >= 0 && x2 < a.w_ && c < a.cin)
                v = *(const uint4 *)(a.x + ((size_t)(row + r - 1) * a.w_ + x2) * a.ldx + a.xoff + c);
            put8(&s_x[wave][r][cq * 8][px], kWgStride, v);
        }
        wave_sync();
        const bf16x8 av = *(const bf16x8 *)&s_dy[wave][lr][kh * 8];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                bf16x8 bv;
#pragma unroll
                for (int e = 0; e < 8; ++e) bv[e] = (short)s_x[wave][r][lr][kh * 8 + k + e];
                acc[3 * r + k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[3 * r + k],
                                                                         0, 0, 0);
            }
        wave_sync();      // the next slice overwrites the staging
    }
    // per tap: the 4 waves' tiles added in LDS in a fixed order, then this
    // split's partial written
#pragma unroll
    for (int t = 0; t < 9; ++t) {
#pragma unroll
        for (int r = 0; r < 16; ++r) s_acc[wave][8 * (r >> 2) + 4 * kh + (r & 3)][lr] = acc[t][r];
        __syncthreads();
        for (int i = threadIdx.x; i < 32 * 32; i += 256) {
            const int rr = i >> 5, col = i & 31;
            const float v = ((s_acc[0][rr][col] + s_acc[1][rr][col]) + s_acc[2][rr][col]) +
                            s_acc[3][rr][col];
            const int co = co0 + rr, ci = ci0 + col;
            if (co < a.cout && ci < a.cin)
                a.partial[(((size_t)split * 9 + t) * a.cout + co) * a.cin + ci] = v;
        }
        __syncthreads();
    }
}

// Sum of the splits' partial tiles in a fixed order, in two levels: groups of
// kWgGroup consecutive splits are summed in parallel (each into its group's
// first slot), then the group sums in order.  partial is [split][tap][co][ci]
// with n = 9*cout*cin elements per split.
constexpr int kWgGroup = 32;

__global__ void wgrad_group_kernel(float *partial, int splits, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k0 = blockIdx.y * kWgGroup, k1 = min(splits, k0 + kWgGroup);
    float s = 0.0f;
#pragma unroll 8
    for (int k = k0; k < k1; ++k) s += partial[(size_t)k * n + i];
    partial[(size_t)k0 * n + i] = s;
}

__global__ void wgrad_reduce_kernel(const float *partial, int splits, int n, float *dw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
#pragma unroll 8
    for (int k = 0; k < splits; k += kWgGroup) s += partial[(size_t)k * n + i];
    dw[i] = s;
}

// [tap][co][ci] -> [co][tap][ci]
__global__ void wgrad_permute_kernel(const float *t, float *dw, int cout, int cin) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = 9 * cout * cin;
    if (i >= n) return;
    const int ci = i % cin, co = (i / cin) % cout, tap = i / (cin * cout);
    dw[((size_t)co * 9 + tap) * cin + ci] = t[i];
}

// bias gradient: db[c] = sum over pixels of dy[p][c], per-block partials then a
// fixed-order sum.  A block sums one pixel range for 64 channels with 256
// threads (4 interleaved pixel streams, four loads in flight per stream), the
// streams added in LDS in a fixed order (deterministic).
__global__ void __launch_bounds__(256) colsum_kernel(const uint16_t *dy, int ldy, int yoff,
                                                     int npix, int c, int chunk, float *partial) {
    __shared__ float s_sum[4][64];
    const int cl = threadIdx.x & 63, sub = threadIdx.x >> 6;
    const int ch = blockIdx.y * 64 + cl;
    const int p0 = blockIdx.x * chunk, p1 = min(npix, p0 + chunk);
    float s = 0.0f;
    if (ch < c) {
        const uint16_t *col = dy + yoff + ch;
        int p = p0 + sub;
        for (; p + 12 < p1; p += 16) {
            const float a0 = bf16_to_f32(col[(size_t)p * ldy]);
            const float a1 = bf16_to_f32(col[(size_t)(p + 4) * ldy]);
            const float a2 = bf16_to_f32(col[(size_t)(p + 8) * ldy]);
            const float a3 = bf16_to_f32(col[(size_t)(p + 12) * ldy]);
            s += ((a0 + a1) + a2) + a3;
        }
        for (; p < p1; p += 4) s += bf16_to_f32(col[(size_t)p * ldy]);
    }
    s_sum[sub][cl] = s;
    __syncthreads();
    if (sub == 0 && ch < c)
        partial[(size_t)blockIdx.x * c + ch] = ((s_sum[0][cl] + s_sum[1][cl]) + s_sum[2][cl]) +
                                               s_sum[3][cl];
}

// the partial sums' rows added per channel, 4 interleaved row streams per
// channel combined in a fixed order
__global__ void __launch_bounds__(256) rowsum_kernel(const float *partial, int rows, int c,
                                                     float *out) {
    __shared__ float s_sum[4][64];
    const int cl = threadIdx.x & 63, sub = threadIdx.x >> 6;
    const int ch = blockIdx.x * 64 + cl;
    float s = 0.0f;
    if (ch < c) {
        int r = sub;
        for (; r + 12 < rows; r += 16) {
            const float a0 = partial[(size_t)r * c + ch];
            const float a1 = partial[(size_t)(r + 4) * c + ch];
            const float a2 = partial[(size_t)(r + 8) * c + ch];
            const float a3 = partial[(size_t)(r + 12) * c + ch];
            s += ((a0 + a1) + a2) + a3;
        }
        for (; r < rows; r += 4) s += partial[(size_t)r * c + ch];
    }
    s_sum[sub][cl] = s;
    __syncthreads();
    if (sub == 0 && ch < c) out[ch] = ((s_sum[0][cl] + s_sum[1][cl]) + s_sum[2][cl]) + s_sum[3][cl];
}

// W'[ci][tap][co] = W[co][8 - tap][ci] (bf16): weights of the input-gradient
// convolution; columns co >= cout and rows ci >= cin are zero padding
__global__ void flip_weights_kernel(const uint16_t *w, uint16_t *wt, int cout, int cin,
                                    int cout_pad, int cin_pad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = cin_pad * 9 * cout_pad;
    if (i >= n) return;
    const int co = i % cout_pad, tap = (i / cout_pad) % 9, ci = i / (9 * cout_pad);
    uint16_t v = 0;
    if (co < cout && ci < cin) v = w[((size_t)co * 9 + (8 - tap)) * cin + ci];
    wt[i] = v;
}

// 2x2 average pooling and its gradient; nearest 2x up-sampling and its gradient
__global__ void pool2_kernel(const uint16_t *x, int ldx, int xoff, uint16_t *y, int ldy, int yoff,
                             int n, int h, int w, int c, int backward, int accumulate) {
    // forward: y[n][h/2][w/2] from x[n][h][w]; backward: x-shaped gradient (here x
    // is dy at the pooled size, y the full-size gradient)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!backward) {
        const int ho = h / 2, wo = w / 2;
        const int64_t total = (int64_t)n * ho * wo * c;
        if (i >= total) return;
        const int ch = (int)(i % c);
        const int64_t q = i / c;
        const int xo = (int)(q % wo), yo = (int)((q / wo) % ho), nn = (int)(q / ((int64_t)wo * ho));
        float s = 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int yy = 2 * yo + (t >> 1), xx = 2 * xo + (t & 1);
            s += bf16_to_f32(x[((size_t)(nn * h + yy) * w + xx) * ldx + xoff + ch]);
        }
        uint16_t *dst = y + ((size_t)(nn * ho + yo) * wo + xo) * ldy + yoff + ch;
        float v = 0.25f * s;
        if (accumulate) v += bf16_to_f32(*dst);
        *dst = f32_to_bf16(v);
    } else {
        const int64_t total = (int64_t)n * h * w * c;
        if (i >= total) return;
        const int ch = (int)(i % c);
        const int64_t q = i / c;
        const int xx = (int)(q % w), yy = (int)((q / w) % h), nn = (int)(q / ((int64_t)w * h));
        const int ho = h / 2, wo = w / 2;
        float v = 0.25f * bf16_to_f32(x[((size_t)(nn * ho + yy / 2) * wo + xx / 2) * ldx + xoff + ch]);
        uint16_t *dst = y + ((size_t)(nn * h + yy) * w + xx) * ldy + yoff + ch;
        if (accumulate) v += bf16_to_f32(*dst);
        *dst = f32_to_bf16(v);
    }
}

__global__ void up2_kernel(const uint16_t *x, int ldx, int xoff, uint16_t *y, int ldy, int yoff,
                           int n, int h, int w, int c, int backward, int accumulate) {
    // forward: y[n][2h][2w] = x[n][h][w]; backward: y[n][h][w] = sum of the 4 children
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!backward) {
        const int64_t total = (int64_t)n * 2 * h * 2 * w * c;
        if (i >= total) return;
        const int ch = (int)(i % c);
        const int64_t q = i / c;
        const int xx = (int)(q % (2 * w)), yy = (int)((q / (2 * w)) % (2 * h)),
                  nn = (int)(q / ((int64_t)4 * w * h));
        float v = bf16_to_f32(x[((size_t)(nn * h + yy / 2) * w + xx / 2) * ldx + xoff + ch]);
        uint16_t *dst = y + ((size_t)(nn * 2 * h + yy) * 2 * w + xx) * ldy + yoff + ch;
        if (accumulate) v += bf16_to_f32(*dst);
        *dst = f32_to_bf16(v);
    } else {
        const int64_t total = (int64_t)n * h * w * c;
        if (i >= total) return;
        const int ch = (int)(i % c);
        const int64_t q = i / c;
        const int xo = (int)(q % w), yo = (int)((q / w) % h), nn = (int)(q / ((int64_t)w * h));
        float s = 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int yy = 2 * yo + (t >> 1), xx = 2 * xo + (t & 1);
            s += bf16_to_f32(x[((size_t)(nn * 2 * h + yy) * 2 * w + xx) * ldx + xoff + ch]);
        }
        uint16_t *dst = y + ((size_t)(nn * h + yo) * w + xo) * ldy + yoff + ch;
        if (accumulate) s += bf16_to_f32(*dst);
        *dst = f32_to_bf16(s);
    }
}

// loss = sum (out - t)^2 / n over fp32 maps (per-block partials, fixed order);
// gradient 2 (out - t) / n * scale written as bf16 into channel `goff` of an
// NHWC buffer with channel stride ldg (other channels untouched)
__global__ void mse_kernel(const float *out, int ldo, const float *t, int64_t n, uint16_t *g,
                           int ldg, int goff, float gscale, float *partial) {
    __shared__ float red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float d = 0.0f;
    if (i < n) {
        d = out[(size_t)i * ldo] - t[i];
        if (g) g[(size_t)i * ldg + goff] = f32_to_bf16(2.0f * d / (float)n * gscale);
    }
    red[threadIdx.x] = d * d;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam on fp32 master weights; writes the bf16 copy the forward pass reads
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n,
                            float lr, float b1, float b2, float eps, float c1, float c2,
                            float gscale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i] * gscale;
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (pb) pb[i] = f32_to_bf16(pi);
}

// g[p][c] = 0 where y[p][c] <= 0: gradient through a ReLU whose output is y
// 8 channels (16 bytes) per thread
__global__ void relu_mask8_kernel(uint16_t *g, int ldg, int goff, const uint16_t *y, int ldy,
                                  int yoff, int npix, int c) {
    const int groups = c >> 3;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * groups) return;
    const int p = i / groups, ch = (i - p * groups) << 3;
    const uint4 yv = *(const uint4 *)(y + (size_t)p * ldy + yoff + ch);
    uint4 *gp = (uint4 *)(g + (size_t)p * ldg + goff + ch);
    const uint4 gv = *gp;
    const uint32_t yw[4] = {yv.x, yv.y, yv.z, yv.w};
    uint32_t gw[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t lo = bf16_to_f32((uint16_t)(yw[k] & 0xffffu)) > 0.0f ? 0x0000ffffu : 0u;
        const uint32_t hi = bf16_to_f32((uint16_t)(yw[k] >> 16)) > 0.0f ? 0xffff0000u : 0u;
        gw[k] &= lo | hi;
    }
    *gp = make_uint4(gw[0], gw[1], gw[2], gw[3]);
}

__global__ void relu_mask_kernel(uint16_t *g, int ldg, int goff, const uint16_t *y, int ldy,
                                 int yoff, int64_t npix, int c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * c) return;
    const int64_t p = i / c;
    const int ch = (int)(i - p * c);
    if (!(bf16_to_f32(y[(size_t)p * ldy + yoff + ch]) > 0.0f)) g[(size_t)p * ldg + goff + ch] = 0;
}

__global__ void cast_bf16_kernel(const float *in, uint16_t *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f32_to_bf16(in[i]);
}

// fp32 planes [n][h][w] -> channel `coff` of an NHWC bf16 buffer (scaled)
__global__ void pack_channel_kernel(const float *in, int64_t npix, float scale, uint16_t *out,
                                    int ld, int coff) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npix) out[(size_t)i * ld + coff] = f32_to_bf16(in[i] * scale);
}

// ---------------------------------------------------------------------------
static unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Split of the reduction over the 4 waves of a block: layers with few output
// tiles (the deep, narrow ones) give each tile 2 or 4 waves so that the chip
// holds at least about two waves per SIMD.
template <int WM, int WN>
static hipError_t conv_launch(const ConvArgs &a, int tiles_co, hipStream_t s) {
    const int npix = a.n * a.h * a.w_;
    const int tiles_px = (npix + 32 * WM - 1) / (32 * WM);
    const long tiles = (long)tiles_px * tiles_co;
    const int K = 9 * (a.cin / 16);
    constexpr size_t R = WM * WN * 16 * 64 * sizeof(float);   // one partial tile
    if (WM == 2 && tiles >= 2048 && a.w_ % 64 == 0 && conv_lds_enabled) {
        const dim3 grid((tiles_px + 3) / 4, tiles_co);
        hipLaunchKernelGGL((conv3x3_lds_kernel<WN>), grid, dim3(256), conv_lds_bytes<WN>(), s, a);
    } else if (tiles >= 2048 || K < 8) {
        const dim3 grid((tiles_px + 3) / 4, tiles_co);
        hipLaunchKernelGGL((conv3x3_kernel<WM, WN, 1>), grid, dim3(256),
                           4 * 32 * kEpStride * sizeof(float), s, a);
    } else if (WM == 2 && conv_lds_enabled &&
               (a.w_ % 64 == 0 || (a.w_ >= 16 && 64 % a.w_ == 0 && a.h % (64 / a.w_) == 0))) {
        // the reduction split over 2 or 4 waves by 16-channel chunks
        if (tiles >= 1024 || a.cin < 64) {
            const dim3 grid((tiles_px + 1) / 2, tiles_co);
            hipLaunchKernelGGL((conv3x3_lds_split_kernel<2, WN, 2>), grid, dim3(256),
                               (conv_lds_split_bytes<2, WN, 2>()), s, a);
        } else {
            if constexpr (WN == 2) {
                if (conv_half_tiles && tiles < 512 && a.cin <= 256) {
                    // the fewest tiles with short reductions: 32-pixel tiles,
                    // twice as many waves (with long reductions the weights,
                    // loaded per tile, cost more than the waves gain)
                    const dim3 grid(2 * tiles_px, tiles_co);
                    hipLaunchKernelGGL((conv3x3_lds_split_kernel<1, WN, 4>), grid, dim3(256),
                                       (conv_lds_split_bytes<1, WN, 4>()), s, a);
                    return hipGetLastError();
                }
            }
            const dim3 grid(tiles_px, tiles_co);
            hipLaunchKernelGGL((conv3x3_lds_split_kernel<2, WN, 4>), grid, dim3(256),
                               (conv_lds_split_bytes<2, WN, 4>()), s, a);
        }
    } else if (tiles >= 1024 || K < 16) {
        const dim3 grid((tiles_px + 1) / 2, tiles_co);
        hipLaunchKernelGGL((conv3x3_kernel<WM, WN, 2>), grid, dim3(256), 2 * R, s, a);
    } else {
        const dim3 grid(tiles_px, tiles_co);
        hipLaunchKernelGGL((conv3x3_kernel<WM, WN, 4>), grid, dim3(256), 3 * R, s, a);
    }
    return hipGetLastError();
}

hipError_t nn_conv3x3(const ConvArgs &a, hipStream_t s) {
    if (a.cout <= 32) return conv_launch<2, 1>(a, (a.cout + 31) / 32, s);
    return conv_launch<2, 2>(a, (a.cout + 63) / 64, s);
}

hipError_t nn_wgrad(const WgradArgs &a, float *tmp, float *dw, hipStream_t s) {
    if (a.w_ % 16 == 0 && (a.ldy | a.yoff) % 8 == 0 && ((uintptr_t)a.dy & 15) == 0) {
        const dim3 grid((a.cout + 31) / 32, (a.cin + 31) / 32, a.splits);
        hipLaunchKernelGGL(wgrad9_kernel, grid, dim3(256), 0, s, a);
    } else {
        const dim3 grid((a.cout + 31) / 32, 9 * ((a.cin + 31) / 32), a.splits);
        hipLaunchKernelGGL(wgrad_kernel, grid, dim3(256), 0, s, a);
    }
    const int n = 9 * a.cout * a.cin;
    if (a.splits > 1)
        hipLaunchKernelGGL(wgrad_group_kernel,
                           dim3(blocks_for(n), (a.splits + kWgGroup - 1) / kWgGroup), dim3(256),
                           0, s, a.partial, a.splits, n);
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(blocks_for(n)), dim3(256), 0, s,
                       (const float *)a.partial, a.splits, n, tmp);
    hipLaunchKernelGGL(wgrad_permute_kernel, dim3(blocks_for(n)), dim3(256), 0, s,
                       (const float *)tmp, dw, a.cout, a.cin);
    return hipGetLastError();
}

hipError_t nn_colsum(const uint16_t *dy, int ldy, int yoff, int npix, int c, float *partial,
                     int rows, float *out, hipStream_t s) {
    const int chunk = (npix + rows - 1) / rows;
    hipLaunchKernelGGL(colsum_kernel, dim3(rows, (c + 63) / 64), dim3(256), 0, s, dy, ldy, yoff,
                       npix, c, chunk, partial);
    hipLaunchKernelGGL(rowsum_kernel, dim3((c + 63) / 64), dim3(256), 0, s, (const float *)partial,
                       rows, c, out);
    return hipGetLastError();
}

hipError_t nn_flip(const uint16_t *w, uint16_t *wt, int cout, int cin, int cout_pad, int cin_pad,
                   hipStream_t s) {
    hipLaunchKernelGGL(flip_weights_kernel, dim3(blocks_for((int64_t)cin_pad * 9 * cout_pad)),
                       dim3(256), 0, s, w, wt, cout, cin, cout_pad, cin_pad);
    return hipGetLastError();
}

// Pooling and up-sampling on 8 channels (16 bytes) per thread: one coarse
// pixel and its 2x2 fine pixels.  gather: the fine values are summed into
// the coarse one (pooling forward, up-sampling backward); else the coarse
// value is copied to the four fine ones (pooling backward, up-sampling
// forward).  quarter: times 0.25 (pooling).  Same arithmetic, in the same
// order, as pool2_kernel / up2_kernel.
__global__ void resample8_kernel(const uint16_t *x, int ldx, int xoff, uint16_t *y, int ldy,
                                 int yoff, int n, int hc, int wc, int c, int gather, int quarter,
                                 int accumulate) {
    const int groups = c >> 3;
    const int total = n * hc * wc * groups;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int g = i % groups, q = i / groups;
    const int xo = q % wc, r = q / wc;
    const int yo = r % hc, nn = r / hc;
    const int ch = g << 3;
    const size_t coarse = (size_t)(nn * hc + yo) * wc + xo;
    auto fine = [&](int t) -> size_t {
        return (size_t)(nn * 2 * hc + 2 * yo + (t >> 1)) * (2 * wc) + 2 * xo + (t & 1);
    };
    auto unpack = [](uint4 u, float (&f)[8]) {
        const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] = bf16_to_f32((uint16_t)(w4[e >> 1] >> (16 * (e & 1))));
    };
    auto pack = [](const float (&f)[8]) {
        uint32_t w4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            w4[k] = (uint32_t)f32_to_bf16(f[2 * k]) | ((uint32_t)f32_to_bf16(f[2 * k + 1]) << 16);
        return make_uint4(w4[0], w4[1], w4[2], w4[3]);
    };
    float v[8];
    if (gather) {
        float s8[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float f[8];
            unpack(*(const uint4 *)(x + fine(t) * ldx + xoff + ch), f);
#pragma unroll
            for (int e = 0; e < 8; ++e) s8[e] += f[e];
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = quarter ? 0.25f * s8[e] : s8[e];
        uint4 *dst = (uint4 *)(y + coarse * ldy + yoff + ch);
        if (accumulate) {
            float f[8];
            unpack(*dst, f);
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] += f[e];
        }
        *dst = pack(v);
    } else {
        float f[8];
        unpack(*(const uint4 *)(x + coarse * ldx + xoff + ch), f);
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = quarter ? 0.25f * f[e] : f[e];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            uint4 *dst = (uint4 *)(y + fine(t) * ldy + yoff + ch);
            float o[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) o[e] = v[e];
            if (accumulate) {
                unpack(*dst, f);
#pragma unroll
                for (int e = 0; e < 8; ++e) o[e] += f[e];
            }
            *dst = pack(o);
        }
    }
}

hipError_t nn_resample(int op, const uint16_t *x, int ldx, int xoff, uint16_t *y, int ldy,
                       int yoff, int n, int h, int w, int c, int backward, int accumulate,
                       hipStream_t s) {
    // 16-byte path: whole 8-channel groups, aligned rows, even sizes for pooling
    const int hc = op == 0 ? h / 2 : h, wc = op == 0 ? w / 2 : w;
    const bool vec = c % 8 == 0 && (ldx | xoff | ldy | yoff) % 8 == 0 &&
                     ((uintptr_t)x & 15) == 0 && ((uintptr_t)y & 15) == 0 &&
                     (op != 0 || (h % 2 == 0 && w % 2 == 0)) &&
                     (int64_t)n * 4 * hc * wc * c < ((int64_t)1 << 31);
    if (vec) {
        const int64_t groups = (int64_t)n * hc * wc * (c / 8);
        const int gather = op == 0 ? !backward : backward;
        hipLaunchKernelGGL(resample8_kernel, dim3(blocks_for(groups)), dim3(256), 0, s, x, ldx,
                           xoff, y, ldy, yoff, n, hc, wc, c, gather, op == 0 ? 1 : 0, accumulate);
        return hipGetLastError();
    }
    int64_t total;
    if (op == 0) total = backward ? (int64_t)n * h * w * c : (int64_t)n * (h / 2) * (w / 2) * c;
    else total = backward ? (int64_t)n * h * w * c : (int64_t)n * 4 * h * w * c;
    if (op == 0)
        hipLaunchKernelGGL(pool2_kernel, dim3(blocks_for(total)), dim3(256), 0, s, x, ldx, xoff, y,
                           ldy, yoff, n, h, w, c, backward, accumulate);
    else
        hipLaunchKernelGGL(up2_kernel, dim3(blocks_for(total)), dim3(256), 0, s, x, ldx, xoff, y,
                           ldy, yoff, n, h, w, c, backward, accumulate);
    return hipGetLastError();
}

hipError_t nn_mse(const float *out, int ldo, const float *t, int64_t n, uint16_t *g, int ldg,
                  int goff, float gscale, float *partial, hipStream_t s) {
    hipLaunchKernelGGL(mse_kernel, dim3(blocks_for(n)), dim3(256), 0, s, out, ldo, t, n, g, ldg,
                       goff, gscale, partial);
    return hipGetLastError();
}

hipError_t nn_adam(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n, float lr,
                   float b1, float b2, float eps, float c1, float c2, float gscale, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, s, p, g, m, v, pb, n, lr,
                       b1, b2, eps, c1, c2, gscale);
    return hipGetLastError();
}

hipError_t nn_relu_mask(uint16_t *g, int ldg, int goff, const uint16_t *y, int ldy, int yoff,
                        int64_t npix, int c, hipStream_t s) {
    if (c % 8 == 0 && (ldg | goff | ldy | yoff) % 8 == 0 && ((uintptr_t)g & 15) == 0 &&
        ((uintptr_t)y & 15) == 0 && npix * c < ((int64_t)1 << 31)) {
        hipLaunchKernelGGL(relu_mask8_kernel, dim3(blocks_for(npix * (c / 8))), dim3(256), 0, s, g,
                           ldg, goff, y, ldy, yoff, (int)npix, c);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(relu_mask_kernel, dim3(blocks_for(npix * c)), dim3(256), 0, s, g, ldg, goff,
                       y, ldy, yoff, npix, c);
    return hipGetLastError();
}

hipError_t nn_cast_bf16(const float *in, uint16_t *out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(cast_bf16_kernel, dim3(blocks_for(n)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t nn_pack_channel(const float *in, int64_t npix, float scale, uint16_t *out, int ld,
                           int coff, hipStream_t s) {
    hipLaunchKernelGGL(pack_channel_kernel, dim3(blocks_for(npix)), dim3(256), 0, s, in, npix,
                       scale, out, ld, coff);
    return hipGetLastError();
}

}  // namespace mcx
