// Decomposition with the detector rows staged in LDS (Sec. 2.1, cost eq. (7)):
// the paper's own decimation (plain detector rows, linear shift, triangle
// window), the same result as k_decimate, organised so that every sample of a
// filtered row is fetched from memory once per block of squares instead of
// once per square and interpolation tap.
//
// A workgroup owns one detector row v and a 2 x 2 block of neighbouring
// squares (one wavefront per square).  Their crops of row v overlap: at every
// projection they lie within one segment [lo, lo + seg) of the row, lo the
// least crop offset of the four squares.  The workgroup walks the decimation
// schedule a stage of eight (or, for long segments, four) steps
// (projections) at a time: each wave loads a quarter of the next stage's
// segments (zero outside the detector, by the buffer range check) while the
// current stage is computed -- FP32 rows straight into LDS, 16-bit rows into
// registers that are widened and written to LDS after the computation; one
// barrier per stage orders the double buffer.  The step tables (schedule,
// the block's least crop offset, each square's offset from it) are built
// once per plan and read a stage at a time.  A lane owns local columns
// lane + 64 c of its wave's square, reads
// the two samples of each column's linear interpolation from LDS (adjacent
// lanes read adjacent words: no bank conflicts), and adds the interpolated
// value to the two open triangle windows; a window is written when its last
// projection is in (lanes write adjacent columns).
//
// Work per cropped sample: two LDS words read, four VALU operations
// (difference, interpolation, two window updates); the staged segments are
// about 0.5 loads per cropped sample.
#include "internal.h"
#include "dtype.h"

namespace fdkod {

typedef __attribute__((address_space(4))) const int* cword_ptr;
typedef __attribute__((address_space(3))) const float* lds_fptr;

// schedule steps per stage: eight (two per wave), or four for long segments,
// whose double buffer of eight would hold the LDS to five workgroups per CU
// (four steps: 16.7 ms against 19.3 ms at N = 2000, s = 4, 512-sample
// segments; eight where the buffer allows eight workgroups anyway)
template <int SEGC>
constexpr int staged_steps() { return SEGC >= 6 ? 4 : 8; }

// event counters of a checked build (see CheckKind)
static __device__ unsigned g_checks_dec[kCheckKinds];

hipError_t checks_read_decimate(unsigned long long* out, bool reset) {
    unsigned h[kCheckKinds] = {};
    hipError_t e = hipMemcpyFromSymbol(h, HIP_SYMBOL(g_checks_dec), sizeof(h), 0, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    for (int k = 0; k < kCheckKinds; ++k) out[k] += h[k];
    if (reset) {
        const unsigned z[kCheckKinds] = {};
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_checks_dec), z, sizeof(z), 0, hipMemcpyHostToDevice);
    }
    return e;
}
static_assert(kDecimUnroll % 8 == 0 && kDecimUnroll % 4 == 0, "the schedule is padded to whole stages");

// CPT: column chunks of 64 per lane; SEGC: 64-sample chunks of a staged
// segment (seg = 64 SEGC >= the spread of the four crop offsets + 64 CPT + 1).
template <int CPT, int SEGC, int STORE>
__global__ __launch_bounds__(256) void k_decimate_staged(DecimVol a) {
    using S = Store<STORE>;
    using T = typename S::T;
    constexpr int ES = (int)sizeof(T);
    constexpr int SEG = 64 * SEGC;
    constexpr int kStagedSteps = staged_steps<SEGC>();
    constexpr int kSpw = kStagedSteps / 4;             // steps each wave stages
    // FP32 rows go from memory straight into LDS (no registers); 16-bit rows
    // pass through registers, where they are widened to FP32
    constexpr bool kDirect = STORE == 0;
    __shared__ float stage[2][kStagedSteps][SEG];

    // XCD-aware order: consecutive logical workgroups share an XCD (and its
    // L2); they take the blocks of one detector row in turn, so the row's
    // overlapping segments are fetched from HBM about once.
    const int nwg = gridDim.x;
    const int chunk = nwg / 8;
    const int b = blockIdx.x;
    const int lwg = (b & 7) * chunk + (b >> 3);
    const int nblocks = a.bside * a.bside;
    if (lwg >= a.nv * nblocks) return;          // the whole workgroup: no barrier is skipped
    const int v = lwg / nblocks, blk = lwg % nblocks;
    const int bx = blk % a.bside, by = blk / a.bside;
    const int side = 2 * a.bside;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int q = (2 * by + (wave >> 1)) * side + 2 * bx + (wave & 1);
    const int width = a.grid[q].y;

    // per step: the schedule (projection, emit, two window weights), the
    // block's least crop offset, and this square's offset from it and
    // fraction; read word by word through the constant address space (scalar
    // loads), a stage's worth at a time
    const cword_ptr sched = (cword_ptr)a.sched;
    const cword_ptr blo = (cword_ptr)(a.blo + (size_t)blk * a.nsched);
    const cword_ptr sqo = (cword_ptr)(a.sqoff + (size_t)q * a.nsched);

    const T* frow = (const T*)a.filt + (size_t)v * a.n;          // row v of projection 0
    const size_t pstride = (size_t)a.nv * a.n;
    const int nbytes = a.n * ES;

    // staging of a stage's segments: wave w takes steps kSpw w .. kSpw w + kSpw - 1.  Every
    // chunk's offset is its own register: folded into the instruction's
    // constant offset, a lane whose first offset lies left of the row
    // (negative) would read zero for all its chunks.
    float reg[kDirect ? 1 : kSpw][kDirect ? 1 : SEGC];
    // (the step tables are read through pointers to the stage's first step,
    // so each word's address is a constant offset from one scalar base: the
    // per-word 64-bit address arithmetic otherwise costs more scalar
    // instructions than the stage has vector ones)
    auto load_stage = [&](cword_ptr s_st, cword_ptr l_st, int buf) {
        int p[kSpw], lo[kSpw];
#pragma unroll
        for (int h = 0; h < kSpw; ++h) {
            p[h] = s_st[4 * (kSpw * wave + h)];
            lo[h] = l_st[kSpw * wave + h];
        }
#pragma unroll
        for (int h = 0; h < kSpw; ++h) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                uniform_ptr(frow + (size_t)p[h] * pstride), (short)0, nbytes, 0x00020000);
#pragma unroll
            for (int c = 0; c < SEGC; ++c) {
                int off = (lo[h] + lane + 64 * c) * ES;
                asm volatile("" : "+v"(off));
                if constexpr (kDirect) {
                    // lane l's word lands at stage[buf][k][64 c + l]
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        rs, (__attribute__((address_space(3))) void*)&stage[buf][kSpw * wave + h][64 * c], 4, off,
                        0, 0, 0);
                } else {
                    reg[h][c] = S::raw(rs, off);
                }
            }
        }
    };
    auto store_stage = [&](int buf) {
        if constexpr (!kDirect) {
#pragma unroll
            for (int h = 0; h < kSpw; ++h)
#pragma unroll
                for (int c = 0; c < SEGC; ++c) stage[buf][kSpw * wave + h][lane + 64 * c] = reg[h][c];
        } else {
            (void)buf;
            vmem_drain();            // the direct loads have written the LDS
        }
    };

    // the next output window's row: row v of decimated angle m of the square
    const size_t plane = (size_t)a.nv * width;
    T* outp = (T*)a.ws + (size_t)(a.squares[q].y_off_row * a.nv) + (size_t)v * width;
    float acc0[CPT], acc1[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) acc0[c] = acc1[c] = 0.0f;

    cword_ptr s_st = sched, q_st = sqo, l_st = blo;      // the current stage's first step
    load_stage(s_st, l_st, 0);
    store_stage(0);
    __syncthreads();
    const int nstage = a.nsched / kStagedSteps;
    for (int st = 0; st < nstage; ++st) {
        const bool more = st + 1 < nstage;
        if (more) load_stage(s_st + 4 * kStagedSteps, l_st + kStagedSteps, (st + 1) & 1);
        // the stage's step tables, requested together
        int emit[kStagedSteps], off[kStagedSteps];
        float w0[kStagedSteps], w1[kStagedSteps], ph[kStagedSteps];
#pragma unroll
        for (int k = 0; k < kStagedSteps; ++k) {
            emit[k] = s_st[4 * k + 1];
            w0[k] = __int_as_float(s_st[4 * k + 2]);
            w1[k] = __int_as_float(s_st[4 * k + 3]);
            off[k] = q_st[2 * k];
            ph[k] = __int_as_float(q_st[2 * k + 1]);
        }
        s_st += 4 * kStagedSteps;
        q_st += 2 * kStagedSteps;
        l_st += kStagedSteps;
        const float(*buf)[SEG] = stage[st & 1];
#pragma unroll
        for (int k = 0; k < kStagedSteps; ++k) {
            FDKOD_CHECK_EVENT(g_checks_dec, kCheckDecimSegment, lane == 0 && off[k] + 64 * CPT + 1 > SEG);
            // column lane + 64 c interpolates samples x[j] and x[j + 1], both
            // read from LDS (a closed window is written at once: holding it
            // to the next stage, or taking x[j + 1] from the next lane by a
            // DPP shift, measured slower)
            // one address register per step; the chunks' constant offsets
            // (at most 64 (CPT - 1) + 1 words) fold into the LDS reads
            uint32_t ad = (uint32_t)(uintptr_t)(lds_fptr)(buf[k] + off[k]) + 4u * (uint32_t)lane;
            asm volatile("" : "+v"(ad));
            const lds_fptr row = (lds_fptr)(uintptr_t)ad;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const float xa = row[64 * c], xb = row[64 * c + 1];
                const float sv = fmaf(ph[k], xb - xa, xa);
                acc0[c] = fmaf(w0[k], sv, acc0[c]);
                acc1[c] = fmaf(w1[k], sv, acc1[c]);
            }
            if (emit[k]) {
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const int j = lane + 64 * c;
                    if (j < width) S::put(outp, j, acc0[c]);
                    acc0[c] = acc1[c];
                    acc1[c] = 0.0f;
                }
                outp += plane;
            }
        }
        if (more) store_stage((st + 1) & 1);
        __syncthreads();
    }
}

template <int CPT, int SEGC>
static void launch_staged_shape(const DecimVol& a, int store, dim3 grid, hipStream_t st) {
    switch (store) {
        case 0: hipLaunchKernelGGL((k_decimate_staged<CPT, SEGC, 0>), grid, dim3(256), 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_decimate_staged<CPT, SEGC, 1>), grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((k_decimate_staged<CPT, SEGC, 2>), grid, dim3(256), 0, st, a); break;
    }
}

bool staged_shape_exists(int cpt, int segc) {
    switch (cpt) {
        case 1: return segc >= 2 && segc <= 3;
        case 2: return segc >= 3 && segc <= 5;
        case 4: return segc >= 5 && segc <= 9;
        default: return false;
    }
}

hipError_t launch_decimate_staged(const DecimVol& a, int cpt, int segc, int store, hipStream_t st) {
    const int nwg = a.nv * a.bside * a.bside;
    const dim3 grid(((nwg + 7) / 8) * 8);        // a multiple of 8 for the XCD order
    switch (cpt * 16 + segc) {
        case 1 * 16 + 2: launch_staged_shape<1, 2>(a, store, grid, st); break;
        case 1 * 16 + 3: launch_staged_shape<1, 3>(a, store, grid, st); break;
        case 2 * 16 + 3: launch_staged_shape<2, 3>(a, store, grid, st); break;
        case 2 * 16 + 4: launch_staged_shape<2, 4>(a, store, grid, st); break;
        case 2 * 16 + 5: launch_staged_shape<2, 5>(a, store, grid, st); break;
        case 4 * 16 + 5: launch_staged_shape<4, 5>(a, store, grid, st); break;
        case 4 * 16 + 6: launch_staged_shape<4, 6>(a, store, grid, st); break;
        case 4 * 16 + 7: launch_staged_shape<4, 7>(a, store, grid, st); break;
        case 4 * 16 + 8: launch_staged_shape<4, 8>(a, store, grid, st); break;
        case 4 * 16 + 9: launch_staged_shape<4, 9>(a, store, grid, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fdkod
