// Reconstruction (Sec. 2.2, eq. (6)): cone-weighted bilinear backprojection of
// every square from its decimated sub-sinogram (s > 0), or of the whole slice
// from the filtered projections (s = 0: direct FDK, the same inner loop).
//
//   f(x, y, z) = (pi / P') sum_m U^-2 Bil(Y_q[m], v*, tau)
//   U = depth / R,  tau = a(x, y) - a_c + c_u - u0  (eq. (1), folded back-shift),
//   v* = z R / depth + c_v                            (eq. (9))
//
// Workgroup = 16 x 16 voxels in (x, y) of one square times ZR consecutive
// slices; every thread owns one (x, y) and ZR accumulators in registers.
// Angles are processed in batches of G.  For each angle of a batch the
// footprint of the workgroup's voxel block on the (local) detector is bounded
// with eq. (1) at the block's corners (columns) and eq. (9) at its corner
// depths and end slices (rows) -- the paper's vertex bound applied to the
// block -- and that footprint (at most TH x TW samples, padded by one sample
// on every side) is staged in LDS as quads (Y, dU, dV, dUV) of forward
// differences, so one 128-bit LDS read fetches all four samples of a
// bilinear interpolation, which is then three FMAs.  Per (x, y, angle) a
// thread computes tau, U and the weight once; along z only the row
// coordinate moves, linearly (b = z / U), so an update costs a row index,
// one LDS read and four FMAs.
#include "internal.h"
#include "dtype.h"

namespace fdkod {

// event counters of a checked build (see CheckKind)
static __device__ unsigned g_checks_bp[kCheckKinds];

hipError_t checks_read_backproject(unsigned long long* out, bool reset) {
    unsigned h[kCheckKinds] = {};
    hipError_t e = hipMemcpyFromSymbol(h, HIP_SYMBOL(g_checks_bp), sizeof(h), 0, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    for (int k = 0; k < kCheckKinds; ++k) out[k] += h[k];
    if (reset) {
        const unsigned z[kCheckKinds] = {};
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_checks_bp), z, sizeof(z), 0, hipMemcpyHostToDevice);
    }
    return e;
}

typedef float f4v __attribute__((ext_vector_type(4)));

typedef __attribute__((address_space(3))) const char* lds_cptr;
typedef __attribute__((address_space(3))) const f4v* lds_f4ptr;

// Per-angle footprints and constants are computed for kFpChunk angles at a
// time (one lane per angle) and kept for two such chunks.
constexpr int kFpChunk = 64;

// LDS of one workgroup: G staged footprints and, for two chunks of angles,
// the per-angle constants.
template <int TW, int TH, int G>
struct BpSmem {
    float4 tile[G][TH * (TW + 1)];
    int4 meta[2][kFpChunk];      // c0, r0 (first column / row of the footprint), rows, -
    float4 mgeo[2][kFpChunk];    // cos, sin, Dc, Lc
    float2 mgeo2[2][kFpChunk];   // R / Dc, c_u - u0 - c0
};

// Lane l receives lane l + 1's value (a DPP wave shift; lane 63 receives 0).
__device__ __forceinline__ float from_next_lane(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130 /* wave_shl:1 */, 0xf, 0xf, false));
}

// Backprojection of one 16 x 16 x ZR voxel block (tile tl, slab zt) of one
// volume.  Every thread of the workgroup calls it (it contains barriers).
//
// Angles go in batches of G.  While batch b is accumulated from LDS, the
// detector samples of batch b + 1 are already being loaded into registers
// (their footprints were bounded one batch earlier), so global-memory latency
// overlaps the arithmetic; two barriers per batch separate the LDS phases.
template <int ZR, int TW, int TH, int G, int STORE>
__device__ __forceinline__ void bp_block(const BpVol& v, int zt, const BpTile& tl,
                                         BpSmem<TW, TH, G>& sm) {
    using S = Store<STORE>;
    using T = typename S::T;
    constexpr int TWP = TW + 1;   // LDS row pitch in quads (odd: spreads banks)
    auto& tile = sm.tile;
    const SquareDesc sq = v.squares[tl.sq];
    const int2 gd = v.grid[tl.sq];
    const int u0 = gd.x, width = gd.y;

    const int n = v.n;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int ix1 = min(tl.x0 + 15, sq.x1 - 1);
    const int iy1 = min(tl.y0 + 15, sq.y1 - 1);
    const int i = tl.x0 + tx, j = tl.y0 + ty;
    const bool own = (i <= ix1) && (j <= iy1);
    // offsets from the square centre; threads outside the square use the
    // block's last voxel so every address they form stays in bounds
    const float dx = (float)min(i, ix1) - v.cu - sq.xc;
    const float dy = (float)min(j, iy1) - v.cu - sq.yc;
    const float bx0 = (float)tl.x0 - v.cu - sq.xc, bx1 = (float)ix1 - v.cu - sq.xc;
    const float by0 = (float)tl.y0 - v.cu - sq.yc, by1 = (float)iy1 - v.cu - sq.yc;

    // the run covers ZR slices even past the volume's end (those voxels are
    // computed and discarded), so the staged rows always hold the whole run
    const int l0 = zt * ZR;                       // output slice (volume slice zbase + l0)
    const float z0 = (float)(v.zbase + l0) - v.cz;
    const float zlast = (float)(v.zbase + l0 + ZR - 1) - v.cz;

    const bool direct = v.row_stride_direct != 0;
    const int row_stride = direct ? v.row_stride_direct : width;
    const size_t plane = (size_t)v.nv * row_stride;
    const T* data = (const T*)v.data + (direct ? 0 : sq.y_off_row * v.nv);
    const float kq = v.cu - (float)u0;            // tau = rel + kq

    // staging map: a lane keeps one footprint column and NQ consecutive rows
    // (their quads), for which it loads NQ + 1 rows
    constexpr int NGRP = 256 / TW;
    static_assert(TH % NGRP == 0, "uniform staging trip count");
    constexpr int NQ = TH / NGRP;
    constexpr int NR = NQ + 1;
    const int scol = threadIdx.x % TW;
    const int srow = (threadIdx.x / TW) * NQ;

    // footprints of the block at the kFpChunk angles from m0 (a multiple of
    // kFpChunk), one lane of the first wave per angle: eq. (1) at the block's
    // corners bounds the columns, eq. (9) at its corner depths and end slices
    // the rows; one sample of margin on every side covers the rounding of the
    // reciprocals.  Angle m's constants sit at [(m / kFpChunk) % 2][m % kFpChunk].
    static_assert(kFpChunk % G == 0, "a batch of angles lies within one chunk");
    auto footprint = [&](int m0) {
        const int slot = (m0 / kFpChunk) & 1;
        if (threadIdx.x < kFpChunk && m0 + (int)threadIdx.x < v.pd) {
            const int m = m0 + threadIdx.x;
            const float2 t = v.trig[m];
            const float dc = v.r + sq.xc * t.x + sq.yc * t.y;
            const float lc = sq.yc * t.x - sq.xc * t.y;
            const float rdc = __builtin_amdgcn_rcpf(dc);
            float tlo = INFINITY, thi = -INFINITY, vlo = INFINITY, vhi = -INFINITY;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float cx = (k & 1) ? bx1 : bx0;
                const float cy = (k & 2) ? by1 : by0;
                const float dl = cy * t.x - cx * t.y;
                const float dd = cx * t.x + cy * t.y;
                const float rd = __builtin_amdgcn_rcpf(dc + dd);
                const float tau = v.r * (dl * dc - lc * dd) * rdc * rd + kq;
                tlo = fminf(tlo, tau);
                thi = fmaxf(thi, tau);
                const float iu = (v.cone ? dc : v.r) * rd;   // row offset per unit z
                const float va = z0 * iu + v.cv, vb = zlast * iu + v.cv;
                vlo = fminf(vlo, fminf(va, vb));
                vhi = fmaxf(vhi, fmaxf(va, vb));
            }
            const int c0 = (int)floorf(tlo) - 1;
            const int r0 = (int)floorf(vlo) - 1;
            const int rows = min((int)floorf(vhi) + 3 - r0, TH);
            sm.meta[slot][threadIdx.x] = make_int4(c0, r0, rows, 0);
            sm.mgeo[slot][threadIdx.x] = make_float4(t.x, t.y, dc, lc);
            sm.mgeo2[slot][threadIdx.x] = make_float2(v.r * rdc, kq - (float)c0);
        }
    };
    // detector samples of the footprints of [m0, m0 + G) into registers, as
    // raw bits of the storage type (converted when staged, so no load is
    // waited for early).  One buffer resource spans the angle's plane of the
    // data: rows outside the buffer fall outside it and read zero (a row above
    // the first wraps to a huge unsigned offset), and a column outside
    // [0, width) gets an offset beyond every plane, so its samples read zero
    // too.  A lane's samples are consecutive rows, so each costs one add.
    // Footprints of more than 16 samples per thread are loaded after the
    // arithmetic instead (their registers would cost occupancy).
    constexpr bool kPrefetch = G * NR <= 16;
    constexpr int ES = (int)sizeof(T);
    const uint32_t plane_bytes = (uint32_t)(plane * ES);
    const int rstep_bytes = row_stride * ES;
    uint32_t pre[G][NR];
    auto fetch_one = [&](int m0, int g) {
        {
            const bool gok = m0 + g < v.pd;
            const int4 mt = gok ? sm.meta[((m0 + g) / kFpChunk) & 1][(m0 + g) % kFpChunk] : make_int4(0, 0, 0, 0);
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                uniform_ptr(data + (size_t)(gok ? m0 + g : 0) * plane), (short)0, (int)plane_bytes, 0x00020000);
            const int col = mt.x + scol;
            const int row = mt.y + srow - v.v0;           // row within the buffer
            const int off0 = (unsigned)col < (unsigned)width ? (row * row_stride + col) * ES : (int)0x80000000;
            // (each offset in its own register, never folded into the
            // instruction's constant offset: the range check must see the
            // whole offset of every sample)
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                int off;
                if (r == 0) {
                    off = off0;
                    asm volatile("" : "+v"(off));
                } else {
                    asm volatile("v_add_u32 %0, %1, %2" : "=v"(off) : "s"(r * rstep_bytes), "v"(off0));
                }
                pre[g][r] = S::raw_bits(rs, off);
            }
        }
    };
    // quads (Y, dU, dV, dUV) into LDS: at (r, c), Y = Y[r][c], dU = Y[r][c+1]
    // - Y[r][c], dV = Y[r+1][c] - Y[r][c], dUV = dU[r+1] - dU[r], so that the
    // bilinear sample at (r + fv, c + fu) is Y + fu dU + fv (dV + fu dUV).
    // The last column's quad is never read (the column index is at most
    // TW - 2), so the lane that receives the next group's first sample
    // writes an unused quad; nor is the last row's (the row index is at most
    // TH - 2), whose extra row lies past the tile.  Rows below the
    // footprint's last are written too: they lie inside the tile and are
    // never read.
    auto stage_one = [&](int g) {
        float y[NR], du[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            y[r] = S::from_bits(pre[g][r]);
            du[r] = from_next_lane(y[r]) - y[r];
        }
#pragma unroll
        for (int r = 0; r < NQ; ++r)
            tile[g][(srow + r) * TWP + scol] = make_float4(y[r], du[r], y[r + 1] - y[r], du[r + 1] - du[r]);
    };

    float acc[ZR];
#pragma unroll
    for (int k = 0; k < ZR; ++k) acc[k] = 0.0f;

    auto fetch_stage = [&](int m0) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            fetch_one(m0, g);
            stage_one(g);
        }
    };

    // the first chunk's footprints; the next chunk's are computed while the
    // first batch of a chunk is accumulated (two barriers before their first
    // use, and after the last use of the chunk two before them)
    if (threadIdx.x < 64) footprint(0);
    __syncthreads();
    fetch_stage(0);
    __syncthreads();
#pragma unroll 1
    for (int m0 = 0; m0 < v.pd; m0 += G) {
        const int cs = (m0 / kFpChunk) & 1, ci0 = m0 % kFpChunk;
        const int gcount = min(G, v.pd - m0);
        const bool more = m0 + G < v.pd;
        if (kPrefetch && more) {             // in flight during the arithmetic below
#pragma unroll
            for (int g = 0; g < G; ++g) fetch_one(m0 + G, g);
        }
        if (ci0 == 0 && m0 + kFpChunk < v.pd && threadIdx.x < 64) footprint(m0 + kFpChunk);
#pragma unroll 1
        for (int g = 0; g < gcount; ++g) {
            const float4 mg = sm.mgeo[cs][ci0 + g];
            const float2 mg2 = sm.mgeo2[cs][ci0 + g];
            const int4 mt = sm.meta[cs][ci0 + g];
            const float dl = dy * mg.x - dx * mg.y;
            const float dd = dx * mg.x + dy * mg.y;
            const float d = mg.z + dd;
            const float rd = __builtin_amdgcn_rcpf(d);
            const float tau = (dl * mg.z - mg.w * dd) * mg2.x * rd + mg2.y;
            const float invu = v.r * rd;                 // 1 / U
            float w = v.scale * invu * invu;
            // row offset per unit z: R / D (eq. (9)), or D_c / D on cone-corrected rows
            float vstep = (v.cone ? mg.z : v.r) * rd;
            const float tf = floorf(tau);
            const float fu = tau - tf;
            const int ci = min(max((int)tf, 0), TW - 2);
            FDKOD_CHECK_EVENT(g_checks_bp, kCheckBpCols, own && ((int)tf < 0 || (int)tf > TW - 2));
            float v0 = fmaf(z0, vstep, v.cv - (float)mt.y);
            // the row index is monotone in z: check the run's ends once; a
            // run outside the staged rows (never expected) contributes zero
            const float vend = fmaf((float)(ZR - 1), vstep, v0);
            if (!(v0 >= 0.0f && vend < (float)(mt.z - 1))) {
                FDKOD_CHECK_EVENT(g_checks_bp, kCheckBpRows, own);
                w = 0.0f;
                v0 = 0.5f;
                vstep = 0.0f;
            }
            // 32-bit LDS byte address of the thread's column in this footprint
            uint32_t tga = (uint32_t)(uintptr_t)(lds_cptr)(tile[g] + ci);
            asm volatile("" : "+v"(tga));   // keep it one register: address = mad24(row, pitch, tga)
#pragma unroll
            for (int k = 0; k < ZR; ++k) {
                const float vv = fmaf((float)k, vstep, v0);
                const float fv = __builtin_amdgcn_fractf(vv);
                const uint32_t ri = (uint32_t)(int)vv;
                const lds_f4ptr p = (lds_f4ptr)(uintptr_t)(tga + __umul24(ri, (uint32_t)(TWP * sizeof(float4))));
                const f4v Q = p[0];
                const float top = fmaf(fu, Q.y, Q.x);          // row ri at tau
                const float dv = fmaf(fu, Q.w, Q.z);           // row ri + 1 minus row ri at tau
                acc[k] = fmaf(w, fmaf(fv, dv, top), acc[k]);
                // four slices per group: their accumulators are complete before
                // the next group's reads are issued (without this fence the
                // compiler may issue all ZR reads first and trade occupancy
                // for the registers that holds them)
                if ((k & 3) == 3)
                    asm volatile("" : "+v"(acc[k - 3]), "+v"(acc[k - 2]), "+v"(acc[k - 1]), "+v"(acc[k])
                                 :: "memory");
            }
        }
        __syncthreads();
        if (more) {
            if (kPrefetch) {
#pragma unroll
                for (int g = 0; g < G; ++g) stage_one(g);
            } else {
                fetch_stage(m0 + G);
            }
        }
        __syncthreads();
    }
    if (own) {
        const size_t slice = (size_t)n * n;
        float* out = v.vol + (size_t)l0 * slice + (size_t)j * n + i;
        const int kmax = min(ZR, v.nz - l0);
#pragma unroll
        for (int k = 0; k < ZR; ++k) {
            if (k < kmax) *out = acc[k];
            out += slice;
        }
    }
}

template <int ZR, int TW, int TH, int G, int STORE>
__global__ __launch_bounds__(256) void k_backproject(BpArgs a) {
    __shared__ BpSmem<TW, TH, G> sm;
    // XCD-aware order: each XCD runs a contiguous range of logical blocks
    const int b = blockIdx.x;
    const int lblk = (b & 7) * a.chunk + (b >> 3);
    if (lblk >= a.nlogical) return;               // before any barrier
    const int zt = lblk / a.ntiles;
    const BpTile tl = a.tiles[lblk - zt * a.ntiles];
    bp_block<ZR, TW, TH, G, STORE>(a.v, zt, tl, sm);
}

// Persistent backprojection over the work items of many volumes.  Workgroup
// b runs on XCD b mod 8 (round-robin dispatch) and first takes tickets from
// that XCD's range of items, so the tiles that share footprints (same volume,
// square and slab) meet in one L2; when its range is exhausted it takes
// tickets from the other XCDs' ranges in turn.  Every workgroup leaves after
// all eight ranges are exhausted.  The counters must be zero at launch
// (launch_reset_counter).
template <int ZR, int TW, int TH, int G, int STORE>
__global__ __launch_bounds__(256) void k_backproject_batch(BpBatchArgs a) {
    __shared__ BpSmem<TW, TH, G> sm;
    __shared__ int ticket;
    const int home = blockIdx.x & (kXcds - 1);
    for (int k = 0; k < kXcds; ++k) {
        const int x = (home + k) & (kXcds - 1);
        const int beg = a.xstart[x];
        const int count = a.xstart[x + 1] - beg;
        for (;;) {
            if (threadIdx.x == 0) ticket = (int)atomicAdd(a.counter + x * kCounterStride, 1u);
            __syncthreads();
            const int it = __builtin_amdgcn_readfirstlane(ticket);
            __syncthreads();      // all threads read the ticket before it is replaced
            if (it >= count) break;
            // item and volume parameters are workgroup-uniform: keep them in
            // scalar registers, as the single-volume kernel's arguments are
            const BatchItem bi = uniform_load(a.items + beg + it);
            const BpVol v = uniform_load(a.vols + bi.vol);
            bp_block<ZR, TW, TH, G, STORE>(v, bi.zt, BpTile{bi.sq, bi.x0, bi.y0, 0}, sm);
        }
    }
}

__global__ void k_reset_counter(unsigned* c) {
    if (threadIdx.x < kXcds) c[threadIdx.x * kCounterStride] = 0u;
}

hipError_t launch_reset_counter(unsigned* counter, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter);
    return hipGetLastError();
}

// Variant table: (zrun, TW, TH, G).  G is limited so that the LDS of one
// workgroup stays within 64 KB.
#define FDKOD_BP_VARIANTS(X)  \
    X(64, 32, 96, 1) \
    X(32, 32, 48, 1) X(32, 32, 48, 2) X(32, 32, 48, 4) \
    X(32, 32, 64, 1) X(32, 32, 64, 2) \
    X(32, 64, 48, 1) X(32, 64, 48, 2) \
    X(32, 64, 64, 1) \
    X(16, 32, 48, 1) X(16, 32, 48, 2) X(16, 32, 48, 4) \
    X(16, 32, 64, 1) X(16, 32, 64, 2) \
    X(16, 64, 48, 1) X(16, 64, 48, 2) \
    X(16, 64, 64, 1)

bool backproject_variant_exists(const BpVariant& var) {
#define FDKOD_X(Z, W, H, GG) \
    if (var.zrun == Z && var.tile_w == W && var.tile_h == H && var.g == GG) return true;
    FDKOD_BP_VARIANTS(FDKOD_X)
#undef FDKOD_X
    return false;
}

hipError_t launch_backproject(const BpArgs& a, const BpVariant& var, int store, hipStream_t st) {
    const dim3 grid(8 * a.chunk);
#define FDKOD_X(Z, W, H, GG)                                                                   \
    if (var.zrun == Z && var.tile_w == W && var.tile_h == H && var.g == GG) {                  \
        switch (store) {                                                                       \
            case 0: hipLaunchKernelGGL((k_backproject<Z, W, H, GG, 0>), grid, dim3(256), 0, st, a); break; \
            case 1: hipLaunchKernelGGL((k_backproject<Z, W, H, GG, 1>), grid, dim3(256), 0, st, a); break; \
            default: hipLaunchKernelGGL((k_backproject<Z, W, H, GG, 2>), grid, dim3(256), 0, st, a); break; \
        }                                                                                      \
        return hipGetLastError();                                                              \
    }
    FDKOD_BP_VARIANTS(FDKOD_X)
#undef FDKOD_X
    return hipErrorInvalidValue;
}

hipError_t launch_backproject_batch(const BpBatchArgs& a, const BpVariant& var, int store,
                                    int blocks, hipStream_t st) {
#define FDKOD_X(Z, W, H, GG)                                                                   \
    if (var.zrun == Z && var.tile_w == W && var.tile_h == H && var.g == GG) {                  \
        switch (store) {                                                                       \
            case 0: hipLaunchKernelGGL((k_backproject_batch<Z, W, H, GG, 0>), dim3(blocks), dim3(256), 0, st, a); break; \
            case 1: hipLaunchKernelGGL((k_backproject_batch<Z, W, H, GG, 1>), dim3(blocks), dim3(256), 0, st, a); break; \
            default: hipLaunchKernelGGL((k_backproject_batch<Z, W, H, GG, 2>), dim3(blocks), dim3(256), 0, st, a); break; \
        }                                                                                      \
        return hipGetLastError();                                                              \
    }
    FDKOD_BP_VARIANTS(FDKOD_X)
#undef FDKOD_X
    return hipErrorInvalidValue;
}

int backproject_batch_occupancy(const BpVariant& var, int store) {
    int nb = 0;
#define FDKOD_X(Z, W, H, GG)                                                                   \
    if (var.zrun == Z && var.tile_w == W && var.tile_h == H && var.g == GG) {                  \
        hipError_t e = hipErrorInvalidValue;                                                   \
        switch (store) {                                                                       \
            case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_backproject_batch<Z, W, H, GG, 0>, 256, 0); break; \
            case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_backproject_batch<Z, W, H, GG, 1>, 256, 0); break; \
            default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_backproject_batch<Z, W, H, GG, 2>, 256, 0); break; \
        }                                                                                      \
        return e == hipSuccess ? nb : 0;                                                       \
    }
    FDKOD_BP_VARIANTS(FDKOD_X)
#undef FDKOD_X
    return 0;
}

}  // namespace fdkod
