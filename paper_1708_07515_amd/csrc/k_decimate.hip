// Decomposition of the filtered sinogram (Sec. 2.1; cost eq. (7)): for every
// square q, detector row v and local column j, crop the row part the square
// uses, shift it so the square's centre trajectory becomes one column (linear
// interpolation), and decimate it in angle with the triangle low-pass filter:
//
//   Y_q[m][v][j] = sum_p w[m][p] * Lin(q[p][v][.], a_c(beta_p) + u0_q + j)
//
// One wavefront per task (square, one or two rows, group of 64*CH local
// columns).  The wavefront walks the projections once, in the order of a
// host-built schedule; with the triangle each projection feeds at most two
// open decimation windows, held in two accumulators per column, and a window
// is written out as soon as its last projection has been added.  The shift's fractional part is the same
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
//
// Quality knobs: a windowed-sinc decimation keeps `taps` windows open (each
// projection is added to all of them with its own weight; the schedule
// carries the extra weights), and the cubic shift reads four samples per
// cropped value and weights them with Keys' kernel of the step's fraction.
#include "internal.h"
#include "dtype.h"
#include "geom.h"

namespace fdkod {

// Read-only tables of the decimation (schedule, crop offsets, row scales,
// extra window weights), read word by word through the constant address
// space so that their lane-uniform loads are scalar.
typedef __attribute__((address_space(4))) const int* cword_ptr;
static_assert(sizeof(DecimStep) == 16 && sizeof(int2) == 8, "table layouts");

// Shape of one task's inner loop: CH column chunks of 64, NW decimation
// windows open at once (2 for the triangle, `taps` for the windowed sinc), NT
// samples per cropped value along u (2 linear, 4 cubic), NR detector rows per
// cropped value (1, or 2 for cone-corrected rows).  U steps are loaded per
// group and two groups are in flight (the next group's loads are issued
// before the current group's arithmetic), so U shrinks as a step's loads grow.
template <int CH, int NW, int NT, int NR>
struct DecimShape {
    static constexpr int LOADS = NT * NR / 2;          // relative to the linear, plain case
    // at most 4 steps per group: the scalar state of 8 steps (schedule, crop
    // and buffer resources of two groups in flight) spilled and doubled the
    // one-chunk kernel's time
    static constexpr int U0 = CH * LOADS >= 8 ? 1 : 8 / (CH * LOADS);
    static constexpr int U = U0 > 4 ? 4 : U0;
    static constexpr int NX = NW > 2 ? NW - 2 : 1;     // extra weights per step (array size)
};


// One task: square q, detector rows v .. v + RPT - 1 (warped row v' for
// CONE), column group g of 64*CH columns, run by one wavefront (lane =
// 0..63).  With one column chunk and the linear shift of detector rows a
// task takes two rows: they share the step's schedule and crop entries and
// its address arithmetic (1.5x faster for squares narrower than a wave).
template <int CH, int STORE, bool CONE, int NW, bool CUBIC>
__device__ __forceinline__ void decimate_task(const DecimVol& a, int task, int lane) {
    using S = Store<STORE>;
    using T = typename S::T;
    constexpr int NT = CUBIC ? 4 : 2;
    constexpr int RPT = decim_rows_per_task(CONE, CUBIC, CH);   // output rows per task
    constexpr int NR = CONE ? 2 : RPT;                      // detector rows loaded per step
    using Sh = DecimShape<CH, NW, NT, NR>;
    constexpr int U = Sh::U;
    constexpr int NX = Sh::NX;
    static_assert(kDecimUnroll % U == 0, "the schedule is padded to whole groups");
    // task = (vb * nsq + q) * tasks_per_sq + g, rows v = RPT vb ..: the
    // squares of one detector row run together and share its reads in L2.
    // CONE: task = (q * nv + v) * tasks_per_sq + g, since squares read
    // different detector rows for the same warped row; neighbouring warped
    // rows of one square share theirs.
    const int g = task % a.tasks_per_sq;
    const int vq = task / a.tasks_per_sq;
    const int q = CONE ? vq / a.nv : vq % a.nsq;
    const int v = CONE ? vq % a.nv : (vq / a.nsq) * RPT;   // first row within the buffer (detector row v0 + v)
    const bool second = RPT == 2 && v + 1 < a.nv;           // the task's second row exists
    const int n = a.n;
    const int2 gd = a.grid[q];
    const int width = gd.y;
    const int jbase = g * 64 * CH + lane;
    if (g * 64 * CH >= width) return;

    // row v of projection 0 (CONE: row 0, the rows vary with the projection)
    const T* frow = (const T*)uniform_ptr((const T*)a.filt + (CONE ? 0 : (size_t)v * n));
    T* ws = (T*)a.ws;
    const cword_ptr sched = (cword_ptr)a.sched;                       // 4 words per step
    const cword_ptr crop = (cword_ptr)(a.crop + (size_t)q * a.nsched);  // 2 words per step
    const cword_ptr rsc = (cword_ptr)(CONE ? a.rscale + (size_t)q * a.nsched : nullptr);
    const cword_ptr wext = (cword_ptr)(NW > 2 ? a.wext : nullptr);    // NW - 2 words per step
    const float vrel = (float)v - a.cv;          // v' - c_v (CONE)
    const int64_t yoff = a.squares[q].y_off_row * a.nv;
    const size_t plane = (size_t)a.nv * width;   // elements per decimated angle
    const size_t pstride = (size_t)a.nv * n;     // elements per projection
    constexpr int ES = (int)sizeof(T);
    // per-lane byte offset of each chunk's column within the cropped run
    int lane_off[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) lane_off[c] = (jbase + 64 * c) * ES;

    // acc[i][r]: the i-th open window of output row r (acc[0] is written out next)
    float acc[NW][RPT][CH];
#pragma unroll
    for (int i = 0; i < NW; ++i)
#pragma unroll
        for (int r = 0; r < RPT; ++r)
#pragma unroll
            for (int c = 0; c < CH; ++c) acc[i][r][c] = 0.0f;
    int m = 0;

    // Per-group state: the steps, their crop entries, row fractions, extra
    // window weights and the loaded samples x[row][tap][step][chunk].
    struct Group {
        DecimStep st[U];
        int2 cr[U];
        float fv[U];
        float wx[U][NX];
        float x[NR][NT][U][CH];
    };
    // Each detector row is read through a buffer resource spanning exactly
    // that row: the hardware range check returns zero outside [0, N), which is
    // the zero extension of the crop (offsets below the row wrap to huge
    // unsigned values and are out of range too).  Every tap is a separately
    // range-checked load: the empty asm hides that the offsets are ES apart,
    // so the loads are not merged into one wider load (whose range check
    // would zero all its elements at the detector's left edge).
    auto issue = [&](int t, Group& G) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = t + u;
            G.st[u].p = sched[4 * e];
            G.st[u].emit = sched[4 * e + 1];
            G.st[u].w0 = __int_as_float(sched[4 * e + 2]);
            G.st[u].w1 = __int_as_float(sched[4 * e + 3]);
            G.cr[u] = make_int2(crop[2 * e], crop[2 * e + 1]);
            if constexpr (NW > 2) {
#pragma unroll
                for (int i = 0; i < NX; ++i) G.wx[u][i] = __int_as_float(wext[(NW - 2) * e + i]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T* pbase = frow + (size_t)G.st[u].p * pstride;
            int r0 = 0;
            if constexpr (CONE) {
                // warped row -> detector row (v' - c_v) R / D_c + c_v, wave-uniform
                const float rr = fmaf(vrel, __int_as_float(rsc[t + u]), a.cv);
                const float rf = floorf(rr);
                G.fv[u] = rr - rf;
                r0 = __builtin_amdgcn_readfirstlane((int)rf);
            }
#pragma unroll
            for (int rw = 0; rw < NR; ++rw) {
                // CONE: the row's address and extent go through readfirstlane
                // so that the resource is built in scalar registers (a resource
                // the compiler holds in vector registers costs a loop around
                // every load)
                const int rowi = r0 + rw;
                // plain rows: row rw of the task (an absent second row has an
                // empty range and reads zero)
                const __amdgpu_buffer_rsrc_t rs =
                    CONE ? __builtin_amdgcn_make_buffer_rsrc(
                               uniform_ptr(pbase + (ptrdiff_t)rowi * n), (short)0,
                               __builtin_amdgcn_readfirstlane((unsigned)rowi < (unsigned)n ? n * ES : 0),
                               0x00020000)
                         : __builtin_amdgcn_make_buffer_rsrc((void*)(pbase + (size_t)rw * n), (short)0,
                                                             (rw == 0 || second) ? n * ES : 0, 0x00020000);
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int off0 = G.cr[u].x * ES + lane_off[c];
#pragma unroll
                    for (int k = 0; k < NT; ++k) {
                        int off = off0 + (k - (NT == 4 ? 1 : 0)) * ES;
                        if (k > 0) asm volatile("" : "+v"(off));
                        G.x[rw][k][u][c] = S::raw(rs, off);
                    }
                }
            }
        }
    };
    auto consume = [&](const Group& G) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float phi = __int_as_float(G.cr[u].y);
            float cw[4];
            if constexpr (CUBIC) keys_weights(phi, cw);
            float w[NW];
            w[0] = G.st[u].w0;
            w[1] = G.st[u].w1;
#pragma unroll
            for (int i = 2; i < NW; ++i) w[i] = G.wx[u][i - 2];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                float rowv[NR];
#pragma unroll
                for (int rw = 0; rw < NR; ++rw) {
                    if constexpr (CUBIC) {
                        float t = cw[0] * G.x[rw][0][u][c];
                        t = fmaf(cw[1], G.x[rw][1][u][c], t);
                        t = fmaf(cw[2], G.x[rw][2][u][c], t);
                        rowv[rw] = fmaf(cw[3], G.x[rw][3][u][c], t);
                    } else {
                        rowv[rw] = fmaf(phi, G.x[rw][1][u][c] - G.x[rw][0][u][c], G.x[rw][0][u][c]);
                    }
                }
                if constexpr (CONE) {
                    const float val = fmaf(G.fv[u], rowv[1] - rowv[0], rowv[0]);
#pragma unroll
                    for (int i = 0; i < NW; ++i) acc[i][0][c] = fmaf(w[i], val, acc[i][0][c]);
                } else {
#pragma unroll
                    for (int r = 0; r < RPT; ++r)
#pragma unroll
                        for (int i = 0; i < NW; ++i) acc[i][r][c] = fmaf(w[i], rowv[r], acc[i][r][c]);
                }
            }
            if (G.st[u].emit) {
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const size_t base = (size_t)yoff + (size_t)m * plane + (size_t)(v + r) * width;
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        const int j = jbase + 64 * c;
                        if (j < width && (r == 0 || second)) S::put(ws, base + j, acc[0][r][c]);
#pragma unroll
                        for (int i = 0; i + 1 < NW; ++i) acc[i][r][c] = acc[i + 1][r][c];
                        acc[NW - 1][r][c] = 0.0f;
                    }
                }
                ++m;
            }
        }
    };
    // two groups (ping, pong) per iteration; the schedule holds whole groups
    Group ga, gb;
    issue(0, ga);
    for (int t = 0; t < a.nsched; t += 2 * U) {
        const bool b_ok = t + U < a.nsched;
        if (b_ok) issue(t + U, gb);
        consume(ga);
        if (t + 2 * U < a.nsched) issue(t + 2 * U, ga);
        if (b_ok) consume(gb);
    }
}

template <int CH, int STORE, bool CONE, int NW, bool CUBIC>
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
    decimate_task<CH, STORE, CONE, NW, CUBIC>(a, task, threadIdx.x & 63);
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
    if (CHMAX >= 8 && dv.chunks >= 8) decimate_task<(CHMAX >= 8 ? 8 : 1), STORE, false, 2, false>(dv, t, lane);
    else if (CHMAX >= 4 && dv.chunks >= 4) decimate_task<(CHMAX >= 4 ? 4 : 1), STORE, false, 2, false>(dv, t, lane);
    else if (CHMAX >= 2 && dv.chunks >= 2) decimate_task<(CHMAX >= 2 ? 2 : 1), STORE, false, 2, false>(dv, t, lane);
    else decimate_task<1, STORE, false, 2, false>(dv, t, lane);
}

template <int CH, bool CONE, int NW, bool CUBIC>
static void launch_shape(const DecimVol& a, int store, dim3 grid, hipStream_t st) {
    switch (store) {
        case 0: hipLaunchKernelGGL((k_decimate<CH, 0, CONE, NW, CUBIC>), grid, dim3(256), 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_decimate<CH, 1, CONE, NW, CUBIC>), grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((k_decimate<CH, 2, CONE, NW, CUBIC>), grid, dim3(256), 0, st, a); break;
    }
}

template <int CH, int NW>
static void launch_nw(const DecimVol& a, int store, dim3 grid, hipStream_t st) {
    if (a.cone) {
        if (a.cubic) launch_shape<CH, true, NW, true>(a, store, grid, st);
        else launch_shape<CH, true, NW, false>(a, store, grid, st);
    } else {
        if (a.cubic) launch_shape<CH, false, NW, true>(a, store, grid, st);
        else launch_shape<CH, false, NW, false>(a, store, grid, st);
    }
}

// false when no kernel exists for the chunk count and window count
template <int CH>
static bool launch_ch(const DecimVol& a, int store, dim3 grid, hipStream_t st) {
    switch (a.nw) {
        case 2: launch_nw<CH, 2>(a, store, grid, st); return true;
        case 4: if constexpr (CH <= kDecimMaxChunksWide) { launch_nw<CH, 4>(a, store, grid, st); return true; }
                return false;
        case 6: if constexpr (CH <= kDecimMaxChunksWide) { launch_nw<CH, 6>(a, store, grid, st); return true; }
                return false;
        default: return false;
    }
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
    bool ok = false;
    switch (chunks) {
        case 1: ok = launch_ch<1>(a, store, grid, st); break;
        case 2: ok = launch_ch<2>(a, store, grid, st); break;
        case 4: ok = launch_ch<4>(a, store, grid, st); break;
        case 8: ok = launch_ch<8>(a, store, grid, st); break;
        default: break;
    }
    if (!ok) return hipErrorInvalidValue;
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
