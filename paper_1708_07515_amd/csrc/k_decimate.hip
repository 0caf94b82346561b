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
//
// Cone-corrected rows (CONE): row v' of square q at angle beta_p is first
// resampled from detector row (v' - c_v) R / D_c(beta_p) + c_v, so each
// cropped sample is a bilinear one: the same column interpolation on the two
// detector rows that bracket the warped row, then a linear one between them.
// The row scale is uniform over the wavefront, so the two rows are two more
// range-checked buffer resources (an empty range for a row outside the
// detector, which reads zero).
#include "internal.h"
#include "dtype.h"

namespace fdkod {

// Read-only tables of the decimation (schedule, crop offsets), read word by
// word through the constant address space so that their lane-uniform loads
// are scalar.
typedef __attribute__((address_space(4))) const int* cword_ptr;
static_assert(sizeof(DecimStep) == 16 && sizeof(int2) == 8, "table layouts");

// Steps whose samples one group loads; two groups are in flight (the next
// group's loads are issued before the current group's arithmetic).
template <int CH>
struct DecimGroup {
    static constexpr int U = CH >= 8 ? 1 : 8 / CH;
};

// One task: square q, detector row v (warped row v' for CONE), column group g
// of 64*CH columns, run by one wavefront (lane = 0..63).
template <int CH, int STORE, bool CONE>
__device__ __forceinline__ void decimate_task(const DecimVol& a, int task, int lane) {
    using S = Store<STORE>;
    using T = typename S::T;
    constexpr int U = DecimGroup<CH>::U;
    constexpr int CC = CONE ? CH : 1;   // second-row samples (CONE only)
    static_assert(kDecimUnroll % U == 0, "the schedule is padded to whole groups");
    // task = (v * nsq + q) * tasks_per_sq + g: the squares of one detector row
    // run together and share its reads in L2.  CONE: task = (q * nv + v) *
    // tasks_per_sq + g, since squares read different detector rows for the
    // same warped row; neighbouring warped rows of one square share theirs.
    const int g = task % a.tasks_per_sq;
    const int vq = task / a.tasks_per_sq;
    const int q = CONE ? vq / a.nv : vq % a.nsq;
    const int v = CONE ? vq % a.nv : vq / a.nsq;   // row within the buffer (detector row v0 + v)
    const int n = a.n;
    const int2 gd = a.grid[q];
    const int u0 = gd.x, width = gd.y;
    const int jbase = g * 64 * CH + lane;
    if (g * 64 * CH >= width) return;
    (void)u0;

    // row v of projection 0 (CONE: row 0, the rows vary with the projection)
    const T* frow = (const T*)uniform_ptr((const T*)a.filt + (CONE ? 0 : (size_t)v * n));
    T* ws = (T*)a.ws;
    const cword_ptr sched = (cword_ptr)a.sched;                       // 4 words per step
    const cword_ptr crop = (cword_ptr)(a.crop + (size_t)q * a.nsched);  // 2 words per step
    const cword_ptr rsc = (cword_ptr)(CONE ? a.rscale + (size_t)q * a.nsched : nullptr);
    const float vrel = (float)v - a.cv;          // v' - c_v (CONE)
    const int64_t yoff = a.squares[q].y_off_row * a.nv;
    const size_t plane = (size_t)a.nv * width;   // elements per decimated angle
    const size_t pstride = (size_t)a.nv * n;     // elements per projection
    constexpr int ES = (int)sizeof(T);
    // per-lane byte offset of each chunk's column within the cropped run
    int lane_off[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) lane_off[c] = (jbase + 64 * c) * ES;

    float acc0[CH], acc1[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        acc0[c] = 0.0f;
        acc1[c] = 0.0f;
    }
    int m = 0;
    // Each detector row is read through a buffer resource spanning exactly
    // that row: the hardware range check returns zero outside [0, N), which is
    // the zero extension of the crop (offsets below the row wrap to huge
    // unsigned values and are out of range too).  Two separately
    // range-checked loads per sample: the empty asm hides that off1 = off0 +
    // ES, so the loads are not merged into one wider load (whose range check
    // would zero both elements at the detector's left edge).
    auto issue = [&](int t, DecimStep (&st)[U], int2 (&cr)[U], float (&fv)[U], float (&x0)[U][CH],
                     float (&x1)[U][CH], float (&y0)[U][CC], float (&y1)[U][CC]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = t + u;
            st[u].p = sched[4 * e];
            st[u].emit = sched[4 * e + 1];
            st[u].w0 = __int_as_float(sched[4 * e + 2]);
            st[u].w1 = __int_as_float(sched[4 * e + 3]);
            cr[u] = make_int2(crop[2 * e], crop[2 * e + 1]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T* pbase = frow + (size_t)st[u].p * pstride;
            int r0 = 0;
            if constexpr (CONE) {
                // warped row -> detector row (v' - c_v) R / D_c + c_v, wave-uniform
                const float rr = fmaf(vrel, __int_as_float(rsc[t + u]), a.cv);
                const float rf = floorf(rr);
                fv[u] = rr - rf;
                r0 = __builtin_amdgcn_readfirstlane((int)rf);
            }
            // CONE: the row's address and extent go through readfirstlane so that
            // the resource is built in scalar registers (a resource the compiler
            // holds in vector registers costs a loop around every load)
            const __amdgpu_buffer_rsrc_t rs =
                CONE ? __builtin_amdgcn_make_buffer_rsrc(
                           uniform_ptr(pbase + (ptrdiff_t)r0 * n), (short)0,
                           __builtin_amdgcn_readfirstlane((unsigned)r0 < (unsigned)n ? n * ES : 0), 0x00020000)
                     : __builtin_amdgcn_make_buffer_rsrc((void*)pbase, (short)0, n * ES, 0x00020000);
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int off0 = cr[u].x * ES + lane_off[c];
                int off1 = off0 + ES;
                asm volatile("" : "+v"(off1));
                x0[u][c] = S::raw(rs, off0);
                x1[u][c] = S::raw(rs, off1);
            }
            if constexpr (CONE) {
                const int r1 = r0 + 1;
                const __amdgpu_buffer_rsrc_t rs1 = __builtin_amdgcn_make_buffer_rsrc(
                    uniform_ptr(pbase + (ptrdiff_t)r1 * n), (short)0,
                    __builtin_amdgcn_readfirstlane((unsigned)r1 < (unsigned)n ? n * ES : 0), 0x00020000);
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int off0 = cr[u].x * ES + lane_off[c];
                    int off1 = off0 + ES;
                    asm volatile("" : "+v"(off1));
                    y0[u][c] = S::raw(rs1, off0);
                    y1[u][c] = S::raw(rs1, off1);
                }
            }
        }
    };
    auto consume = [&](const DecimStep (&st)[U], const int2 (&cr)[U], const float (&fv)[U],
                       const float (&x0)[U][CH], const float (&x1)[U][CH], const float (&y0)[U][CC],
                       const float (&y1)[U][CC]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float phi = __int_as_float(cr[u].y);
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                float val = fmaf(phi, x1[u][c] - x0[u][c], x0[u][c]);
                if constexpr (CONE) {
                    const float hi = fmaf(phi, y1[u][c] - y0[u][c], y0[u][c]);
                    val = fmaf(fv[u], hi - val, val);
                }
                acc0[c] = fmaf(st[u].w0, val, acc0[c]);
                acc1[c] = fmaf(st[u].w1, val, acc1[c]);
            }
            if (st[u].emit) {
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
    };
    // two groups (ping, pong) per iteration; the schedule holds whole groups
    DecimStep sa[U], sb[U];
    int2 ca[U], cb[U];
    float fa[U], fb[U];
    float xa0[U][CH], xa1[U][CH], xb0[U][CH], xb1[U][CH];
    float ya0[U][CC], ya1[U][CC], yb0[U][CC], yb1[U][CC];
    issue(0, sa, ca, fa, xa0, xa1, ya0, ya1);
    for (int t = 0; t < a.nsched; t += 2 * U) {
        const bool b_ok = t + U < a.nsched;
        if (b_ok) issue(t + U, sb, cb, fb, xb0, xb1, yb0, yb1);
        consume(sa, ca, fa, xa0, xa1, ya0, ya1);
        if (t + 2 * U < a.nsched) issue(t + 2 * U, sa, ca, fa, xa0, xa1, ya0, ya1);
        if (b_ok) consume(sb, cb, fb, xb0, xb1, yb0, yb1);
    }
}

template <int CH, int STORE, bool CONE>
__global__ __launch_bounds__(256) void k_decimate(DecimVol a) {
    // XCD-aware order: consecutive logical blocks share an XCD (and its L2)
    const int nblk = gridDim.x;
    const int chunk = nblk / 8;
    const int b = blockIdx.x;
    const int lblk = (b & 7) * chunk + (b >> 3);
    // the wave index is uniform across the wave; say so, so that the task's
    // square, row and buffer resources live in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int task = lblk * 4 + wave;
    if (task >= a.ntasks) return;         // no barriers in this kernel
    decimate_task<CH, STORE, CONE>(a, task, threadIdx.x & 63);
}

// Many volumes in one launch (tasks concatenated volume after volume).  Each
// volume uses its own chunk count (at most CHMAX), so the waves of a small
// volume do not carry idle columns.
template <int CHMAX, int STORE>
__global__ __launch_bounds__(256) void k_decimate_batch(DecimBatchArgs a) {
    const int nblk = gridDim.x;
    const int chunk = nblk / 8;
    const int b = blockIdx.x;
    const int lblk = (b & 7) * chunk + (b >> 3);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int task = lblk * 4 + wave;
    if (task >= a.ntasks) return;
    const int2 bv = uniform_load(a.block_vol + lblk);   // (volume, first task of the volume)
    const DecimVol dv = uniform_load(a.vols + bv.x);    // wave-uniform: scalar registers
    const int t = task - bv.y;
    if (t >= dv.ntasks) return;                         // padding of the volume's range
    const int lane = threadIdx.x & 63;
    if (CHMAX >= 8 && dv.chunks >= 8) decimate_task<(CHMAX >= 8 ? 8 : 1), STORE, false>(dv, t, lane);
    else if (CHMAX >= 4 && dv.chunks >= 4) decimate_task<(CHMAX >= 4 ? 4 : 1), STORE, false>(dv, t, lane);
    else if (CHMAX >= 2 && dv.chunks >= 2) decimate_task<(CHMAX >= 2 ? 2 : 1), STORE, false>(dv, t, lane);
    else decimate_task<1, STORE, false>(dv, t, lane);
}

template <int CH, bool CONE>
static void launch_ch_rows(const DecimVol& a, int store, dim3 grid, hipStream_t st) {
    switch (store) {
        case 0: hipLaunchKernelGGL((k_decimate<CH, 0, CONE>), grid, dim3(256), 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_decimate<CH, 1, CONE>), grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((k_decimate<CH, 2, CONE>), grid, dim3(256), 0, st, a); break;
    }
}

template <int CH>
static void launch_ch(const DecimVol& a, int store, dim3 grid, hipStream_t st) {
    if (a.cone) launch_ch_rows<CH, true>(a, store, grid, st);
    else launch_ch_rows<CH, false>(a, store, grid, st);
}

template <int CH>
static void launch_ch_batch(const DecimBatchArgs& a, int store, dim3 grid, hipStream_t st) {
    switch (store) {
        case 0: hipLaunchKernelGGL((k_decimate_batch<CH, 0>), grid, dim3(256), 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_decimate_batch<CH, 1>), grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((k_decimate_batch<CH, 2>), grid, dim3(256), 0, st, a); break;
    }
}

static dim3 decimate_grid(int ntasks) {
    const int blocks = (ntasks + 3) / 4;
    return dim3(((blocks + 7) / 8) * 8);   // a multiple of 8 for the XCD order
}

hipError_t launch_decimate(const DecimVol& a, int chunks, int store, hipStream_t st) {
    const dim3 grid = decimate_grid(a.ntasks);
    switch (chunks) {
        case 1: launch_ch<1>(a, store, grid, st); break;
        case 2: launch_ch<2>(a, store, grid, st); break;
        case 4: launch_ch<4>(a, store, grid, st); break;
        case 8: launch_ch<8>(a, store, grid, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_decimate_batch(const DecimBatchArgs& a, int chunks, int store, hipStream_t st) {
    const dim3 grid = decimate_grid(a.ntasks);
    switch (chunks) {
        case 1: launch_ch_batch<1>(a, store, grid, st); break;
        case 2: launch_ch_batch<2>(a, store, grid, st); break;
        case 4: launch_ch_batch<4>(a, store, grid, st); break;
        case 8: launch_ch_batch<8>(a, store, grid, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fdkod
