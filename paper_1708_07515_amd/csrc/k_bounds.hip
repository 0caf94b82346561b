// Bounds of every square of the decomposition (Sec. 2.1): eq. (1) at the
// square's centre and at its four vertices, for every angle, FP32.
//
// One workgroup per square.  Per decimated angle m it writes a_c, a_min and
// a_max; a wavefront + workgroup reduction gives the square's extremes of
// a - a_c over the decimated angles, from which the local column grid
// (origin u0 and width W) follows.  Per original angle p it writes a_c(beta_p),
// the centre trajectory that the crop follows.  Batches run the squares of
// all their volumes in one launch (k_bounds_batch).
#include "internal.h"
#include "dtype.h"
#include "geom.h"

namespace fdkod {

__device__ __forceinline__ float pix_pos(float x, float y, float cs, float sn, float r) {
    return r * (y * cs - x * sn) / (r + x * cs + y * sn);
}

__device__ __forceinline__ float wave_min(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// Bounds, grid and crop table of square q (one 256-thread workgroup).
__device__ __forceinline__ void bounds_square(const BoundsArgs& a, int q) {
    __shared__ float red[2][4];
    const SquareDesc sq = a.squares[q];
    const float c = a.cu;
    // vertex offsets from the centre: corner voxel centres of the square
    const float vx[2] = {(float)sq.x0 - c - sq.xc, (float)(sq.x1 - 1) - c - sq.xc};
    const float vy[2] = {(float)sq.y0 - c - sq.yc, (float)(sq.y1 - 1) - c - sq.yc};

    float emin = INFINITY, emax = -INFINITY;
    for (int m = threadIdx.x; m < a.pd; m += blockDim.x) {
        const float2 t = a.trig_m[m];
        const float dc = a.r + sq.xc * t.x + sq.yc * t.y;
        const float lc = sq.yc * t.x - sq.xc * t.y;
        const float rdc = 1.0f / dc;
        const float ac = a.r * lc * rdc;
        float lo = INFINITY, hi = -INFINITY;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float e = rel_column(vx[k & 1], vy[k >> 1], t.x, t.y, a.r, dc, lc, rdc);
            lo = fminf(lo, e);
            hi = fmaxf(hi, e);
        }
        a.geo_m[(size_t)q * a.pd + m] = make_float4(ac, ac + lo, ac + hi, 0.0f);
        emin = fminf(emin, lo);
        emax = fmaxf(emax, hi);
    }
    emin = wave_min(emin);
    emax = wave_max(emax);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red[0][wave] = emin;
        red[1][wave] = emax;
    }
    __syncthreads();
    __shared__ int u0s;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        float lo = red[0][0], hi = red[1][0];
        for (int w = 1; w < nw; ++w) {
            lo = fminf(lo, red[0][w]);
            hi = fmaxf(hi, red[1][w]);
        }
        const int u0 = (int)floorf(lo + c);
        const int w = (int)floorf(hi + c) - u0 + 2;
        a.grid[q] = make_int2(u0, w);
        u0s = u0;
    }
    for (int p = threadIdx.x; p < a.p; p += blockDim.x) {
        const float2 t = a.trig_p[p];
        a.ac_p[(size_t)q * a.p + p] = pix_pos(sq.xc, sq.yc, t.x, t.y, a.r);
    }
    __syncthreads();
    // crop table in schedule order: detector index of local column 0 at the
    // step's projection, split into its integer part and fraction
    const float u0f = (float)u0s;
    for (int t = threadIdx.x; t < a.nsched; t += blockDim.x) {
        const float2 tr = a.trig_p[a.sched[t].p];
        const float o = pix_pos(sq.xc, sq.yc, tr.x, tr.y, a.r) + u0f;
        const float of = floorf(o);
        a.crop[(size_t)q * a.nsched + t] = make_int2((int)of, __float_as_int(o - of));
        if (a.rscale) a.rscale[(size_t)q * a.nsched + t] = a.r / (a.r + sq.xc * tr.x + sq.yc * tr.y);
    }
}

__global__ __launch_bounds__(256) void k_bounds(BoundsArgs a) { bounds_square(a, blockIdx.x); }

// Many volumes: workgroup b is square b - start[v] of volume v.
__global__ __launch_bounds__(256) void k_bounds_batch(BoundsBatchArgs ba) {
    const int b = blockIdx.x;
    const int v = batch_volume(ba.start, ba.nvol, b);
    const BoundsArgs a = const_load(ba.vols + v);
    bounds_square(a, b - const_load(ba.start + v));
}

hipError_t launch_bounds(const BoundsArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_bounds, dim3(a.nsq), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_bounds_batch(const BoundsBatchArgs& a, int workgroups, hipStream_t st) {
    hipLaunchKernelGGL(k_bounds_batch, dim3(workgroups), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace fdkod
