// Argument blocks of the network kernels (unet.hip), shared with the host runtime.
#pragma once

#include <cstdint>

namespace mcx {

struct ConvArgs {
    const uint16_t *x;   // input NHWC
    int ldx, xoff;
    const uint16_t *w;   // [cout_alloc][9][cin]
    const float *bias;   // [cout] or null
    uint16_t *y;         // bf16 output NHWC (or null)
    int ldy, yoff;
    float *yf;           // fp32 output [pixels][cout] (or null)
    const uint16_t *mask;  // output multiplied by (mask > 0) when non-null
    int ldm, moff;
    int n, h, w_, cin, cout;
    int relu;
    int accumulate;      // add to the existing bf16 output
};

struct WgradArgs {
    const uint16_t *x;
    int ldx, xoff;
    const uint16_t *dy;
    int ldy, yoff;
    int n, h, w_, cin, cout;
    int splits;          // pixel ranges
    float *partial;      // [splits][9][cout][cin]
};

}  // namespace mcx
