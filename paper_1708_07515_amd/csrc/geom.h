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

}  // namespace fdkod
