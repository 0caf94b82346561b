// Device geometry helpers for eq. (1) of the paper, FP32.
#pragma once

#include <hip/hip_runtime.h>

namespace fdkod {

// Detector column of a point relative to a reference point (xc, yc) at one
// angle, a(x, y) - a(xc, yc) with a from eq. (1), written so that no large
// absolute coordinate is formed:
//   a(x, y) = R L / D,  L = y cos - x sin,  D = R + x cos + y sin,
//   a(x, y) - a(xc, yc) = R (dL Dc - Lc dD) / (Dc (Dc + dD)),
// with dL, dD the changes of L, D from (xc, yc) to (x, y).
// dc: Dc, lc: Lc, rdc: 1 / Dc for the reference point.
__device__ __forceinline__ float rel_column(float dx, float dy, float cs, float sn,
                                            float r, float dc, float lc, float rdc) {
    float dl = dy * cs - dx * sn;
    float dd = dx * cs + dy * sn;
    float d = dc + dd;
    return r * (dl * dc - lc * dd) * rdc / d;
}

// Keys' cubic convolution weights (a = -1/2) of the samples at offsets
// -1, 0, 1, 2 from floor(u), for the fraction f of u (the crop's cubic shift).
__device__ __forceinline__ void keys_weights(float f, float (&c)[4]) {
    c[0] = ((-0.5f * f + 1.0f) * f - 0.5f) * f;
    c[1] = (1.5f * f - 2.5f) * f * f + 1.0f;
    c[2] = ((-1.5f * f + 2.0f) * f + 0.5f) * f;
    c[3] = (0.5f * f - 0.5f) * f * f;
}

}  // namespace fdkod
