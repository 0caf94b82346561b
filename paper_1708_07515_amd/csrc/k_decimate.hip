// Decomposition of the filtered sinogram (Sec. 2.1; cost eq. (7)): for every
// square q, detector row v and local column j, crop the row part the square
// uses, shift it so the square's centre trajectory becomes one column (linear
// interpolation), and decimate it in angle with the triangle low-pass filter:
//
//   Y_q[m][v][j] = sum_p w[m][p] * Lin(q[p][v][.], a_c(beta_p) + u0_q + j)
//
// One wavefront per task (square, row, group of 64*CH local columns).  The
// wavefront walks the projections once, in the order of a host-built
// schedule; each projection feeds at most two open decimation windows, held
// in two accumulators per column, and a window is written out as soon as its
// last projection has been added.  The shift's fractional part is the same
// for every column of a (square, projection), so each cropped sample costs
// one interpolation and two multiply-adds.  Rows are read with unit stride
// (coalesced); the re-reads of a row by the squares that overlap it hit L2
// because all squares of a row are scheduled together on one XCD.
#include "internal.h"
#include "dtype.h"

namespace fdkod {

template <int CH, int STORE>
__global__ __launch_bounds__(256) void k_decimate(DecimArgs a) {
    using S = Store<STORE>;
    using T = typename S::T;
    // XCD-aware order: consecutive logical blocks share an XCD (and its L2)
    const int nblk = gridDim.x;
    const int chunk = nblk / 8;
    const int b = blockIdx.x;
    const int lblk = (b & 7) * chunk + (b >> 3);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int task = lblk * 4 + wave;
    if (task >= a.ntasks) return;         // no barriers in this kernel

    // task = (v * nsq + q) * tasks_per_sq + g
    const int g = task % a.tasks_per_sq;
    const int vq = task / a.tasks_per_sq;
    const int q = vq % a.nsq;
    const int v = vq / a.nsq;
    const int n = a.n;
    const int2 gd = a.grid[q];
    const int u0 = gd.x, width = gd.y;
    const int jbase = g * 64 * CH + lane;
    if (g * 64 * CH >= width) return;

    const T* filt = (const T*)a.filt;
    T* ws = (T*)a.ws;
    const float* acp = a.ac_p + (size_t)q * a.p;
    const int64_t yoff = a.squares[q].y_off;
    const size_t plane = (size_t)n * width;   // elements per decimated angle

    float acc0[CH], acc1[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        acc0[c] = 0.0f;
        acc1[c] = 0.0f;
    }
    int m = 0;
    for (int t = 0; t < a.nsched; ++t) {
        const DecimStep st = a.sched[t];
        const float o = acp[st.p] + (float)u0;      // index of local column 0
        const float of = floorf(o);
        const float phi = o - of;
        const int k = (int)of;
        const T* row = filt + ((size_t)st.p * n + v) * n;
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int i0 = k + jbase + 64 * c;
            const float x0 = ((unsigned)i0 < (unsigned)n) ? S::load(row, i0) : 0.0f;
            const float x1 = ((unsigned)(i0 + 1) < (unsigned)n) ? S::load(row, i0 + 1) : 0.0f;
            const float val = fmaf(phi, x1 - x0, x0);
            acc0[c] = fmaf(st.w0, val, acc0[c]);
            acc1[c] = fmaf(st.w1, val, acc1[c]);
        }
        if (st.emit) {
            const size_t base = (size_t)yoff + (size_t)m * plane + (size_t)v * width;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int j = jbase + 64 * c;
                if (j < width) S::put(ws, base + j, acc0[c]);
                acc0[c] = acc1[c];
                acc1[c] = 0.0f;
            }
            ++m;
        }
    }
}

template <int CH>
static void launch_ch(const DecimArgs& a, int store, dim3 grid, hipStream_t st) {
    switch (store) {
        case 0: hipLaunchKernelGGL((k_decimate<CH, 0>), grid, dim3(256), 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_decimate<CH, 1>), grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((k_decimate<CH, 2>), grid, dim3(256), 0, st, a); break;
    }
}

hipError_t launch_decimate(const DecimArgs& a, int chunks, int store, hipStream_t st) {
    const int blocks = (a.ntasks + 3) / 4;
    const dim3 grid(((blocks + 7) / 8) * 8);   // a multiple of 8 for the XCD order
    switch (chunks) {
        case 1: launch_ch<1>(a, store, grid, st); break;
        case 2: launch_ch<2>(a, store, grid, st); break;
        case 4: launch_ch<4>(a, store, grid, st); break;
        case 8: launch_ch<8>(a, store, grid, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fdkod
