// Internal declarations shared by the host plan code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace fdkod {

// One square of the decomposition (Sec. 2.1): voxel index ranges, centre
// (vertex mean, voxel coordinates) and where its decimated data starts in a
// workspace: the squares' blocks [P'][rows][W_q] are concatenated, so square
// q starts at y_off_row * rows elements, y_off_row = P' * sum_{q'<q} W_q'.
struct SquareDesc {
    int x0, x1, y0, y1;
    float xc, yc;
    int64_t y_off_row;
};

// One step of the decimation schedule: the extended angle index p_ext
// (the projection read is p_ext mod P), the weights of the projection in the
// two open decimation windows, and whether the older window closes after it.
struct DecimStep {
    int p;        // projection index in [0, P)
    int emit;     // 1: the older window is complete after this step
    float w0;     // weight into the older open window
    float w1;     // weight into the newer open window
};

// Backprojection tile: 16 x 16 voxels in x, y of one square.
struct BpTile {
    int sq;       // square index
    int x0, y0;   // first voxel of the tile (indices)
    int pad;
};

// Arguments of the bounds kernel.
struct BoundsArgs {
    const SquareDesc* squares;
    const float2* trig_p;   // cos, sin of beta_p, [P]
    const float2* trig_m;   // cos, sin of beta'_m, [P']
    float* ac_p;            // [nsq][P]
    float4* geo_m;          // [nsq][P'] a_c, a_min, a_max, 0
    int2* grid;             // [nsq] u0, W
    const DecimStep* sched; // decimation schedule (projection of each step)
    int2* crop;             // [nsq][nsched] floor(a_c + u0), bits of the fraction
    float* rscale;          // [nsq][nsched] R / D_c(beta) (cone-corrected rows), or null
    int n, p, pd, nsq, nsched;
    float r, cu;
};

// Arguments of the ramp filter kernel.
struct FilterArgs {
    const float* proj;      // [rows][n]
    void* out;              // [rows][n] store type
    const float2* resp;     // DFT of the running-sum kernel g, / M, [M]
    const float* gtail;     // g[u - N], u in [0, N)
    const float2* twiddle;  // exp(-2 pi i k / M), [M]
    int n;                  // detector width
    int rows;               // P * nv
    int v0, nv;             // detector rows [v0, v0 + nv) of every projection
    float r;                // R
    float c;                // (N-1)/2
};

// Arguments of the crop + shift + decimate kernel for one volume.
struct DecimVol {
    const void* filt;       // [P][N][N] store type
    void* ws;               // decimated data, store type
    const SquareDesc* squares;
    const int2* grid;       // u0, W per square
    const int2* crop;       // [nsq][nsched] integer shift and fraction per step
    const DecimStep* sched;
    const float* rscale;    // [nsq][nsched] row scale R / D_c(beta) (cone-corrected rows)
    const float* wext;      // [nsched][nw - 2] weights of the open windows 2.. (nw > 2)
    int nsched;
    int nw;                 // decimation windows a projection can feed (2, 4 or 6)
    int cubic;              // 1: Keys' cubic shift along u (four samples), else linear
    int cone;               // 1: rows resampled by rscale about cv before the decimation
    float cv;               // (N-1)/2
    int n, p, pd, nsq;
    int v0, nv;             // detector rows [v0, v0 + nv): filt is [P][nv][N], ws blocks [P'][nv][W_q]
    int tasks_per_sq;       // column groups per square
    int ntasks;             // nsq * ceil(nv / rows per task) * tasks_per_sq
    int chunks;             // 64-column chunks per wave (1, 2, 4 or 8)
    int bside;              // 2^(s-1): 2 x 2 blocks of squares per side (row-staged kernel)
    const int* blo;         // [bside^2][nsched] least crop offset of a block's squares (row-staged)
    const int2* sqoff;      // [nsq][nsched] crop offset - block's least, bits of the fraction (row-staged)
};

// Many volumes' filters or bounds in one launch: volume v owns the
// workgroups [start[v], start[v + 1]) and runs them as its own launch would
// (workgroup b - start[v]); all volumes of a filter launch share the FFT
// length.
struct FilterBatchArgs {
    const FilterArgs* vols;     // [nvol]
    const int* start;           // [nvol + 1]
    int nvol;
};
struct BoundsBatchArgs {
    const BoundsArgs* vols;     // [nvol]
    const int* start;           // [nvol + 1]: the first square of each volume
    int nvol;
};

// Threads per row pair of the radix-16 filter of length 2^logm.
constexpr int filter_threads_per_pair(int logm) {
    return (1 << logm) / 16 < 1 ? 1 : ((1 << logm) / 16 > 256 ? 256 : (1 << logm) / 16);
}

// Many volumes in one launch: volume b owns tasks [start_b, start_b + ntasks_b)
// with start_b a multiple of 4, so a workgroup (4 waves) never spans two
// volumes; block_vol[g] = (volume, start) of workgroup g's volume.
struct DecimBatchArgs {
    const DecimVol* vols;
    const int2* block_vol;  // [ntasks / 4]
    int nvols;
    int ntasks;             // sum of the padded task ranges
};

// Per-volume parameters of the backprojection.
struct BpVol {
    const void* data;       // decimated data (s > 0) or filtered projections (s = 0)
    float* vol;             // [nz][n][n]
    const SquareDesc* squares;
    const int2* grid;       // u0, W per square (direct: 0, N)
    const float2* trig;     // cos, sin of the reconstruction angles, [pd]
    int n, nz, pd;          // nz: slices in the output buffer
    int v0, nv;             // detector rows [v0, v0 + nv) held by data (rows outside read zero)
    int zbase;              // volume slice of output slice 0
    int cone;               // 1: data rows are cone-corrected (row offset z D_c / D)
    int row_stride_direct;  // 0 for per-square layout [m][v][W_q]
    float r, cu, cv, cz;
    float scale;            // pi / P'
};

// Arguments of the backprojection kernel for one volume (grid launch).
struct BpArgs {
    BpVol v;
    const BpTile* tiles;
    int ntiles;             // xy tiles
    int nzt;                // z tiles
    int nlogical;           // ntiles * nzt
    int chunk;              // logical WGs per XCD
};

// One work item of the batched (persistent) backprojection.
struct BatchItem {
    int vol, sq, x0, y0, zt, pad0, pad1, pad2;
};

// Work items are split into one contiguous range per XCD (items
// [xstart[x], xstart[x+1]) with about equal work); each range has its own
// ticket counter, counter[x * kCounterStride], zeroed before each launch.
constexpr int kXcds = 8;
constexpr int kCounterStride = 32;   // 128 bytes between counters

struct BpBatchArgs {
    const BpVol* vols;
    const BatchItem* items;  // per XCD range: larger volumes first, then square, slab, tile
    int nitems;
    int xstart[kXcds + 1];
    unsigned* counter;       // kXcds ticket counters, kCounterStride apart
};

// A backprojection kernel variant: slices per thread, LDS footprint
// (columns x rows), angles staged per barrier.
struct BpVariant {
    int zrun, tile_w, tile_h, g;
};

hipError_t launch_bounds(const BoundsArgs& a, hipStream_t st);
hipError_t launch_bounds_batch(const BoundsBatchArgs& a, int workgroups, hipStream_t st);
hipError_t launch_filter(const FilterArgs& a, int logm, int store, hipStream_t st);
// workgroups of one volume's filter launch
int filter_workgroups(const FilterArgs& a, int logm);
hipError_t launch_filter_batch(const FilterBatchArgs& a, int logm, int store, int workgroups, hipStream_t st);
hipError_t launch_decimate(const DecimVol& a, int chunks, int store, hipStream_t st);
// row-staged decimation (plain rows, triangle, linear shift): cpt 64-column
// chunks per lane, segc 64-sample chunks per staged row segment
bool staged_shape_exists(int cpt, int segc);
hipError_t launch_decimate_staged(const DecimVol& a, int cpt, int segc, int store, hipStream_t st);
hipError_t launch_decimate_batch(const DecimBatchArgs& a, int chunks, int store, hipStream_t st);
hipError_t launch_backproject(const BpArgs& a, const BpVariant& var, int store, hipStream_t st);
hipError_t launch_backproject_batch(const BpBatchArgs& a, const BpVariant& var, int store,
                                    int blocks, hipStream_t st);
// workgroups of the batched kernel that fit on one CU (0 if the variant is unknown)
int backproject_batch_occupancy(const BpVariant& var, int store);
bool backproject_variant_exists(const BpVariant& var);
hipError_t launch_reset_counter(unsigned* counter, hipStream_t st);

// Learned decimation (conv net over angle x column added to the triangle
// decimation): 817 BF16 parameters W1 [16][5][5], b1 [16], W2 [16][5][5], b2.
constexpr int kLearnedParams = 817;
constexpr int kLearnedMaxWidth = 252;   // widest square (local columns) it takes
constexpr int kLearnedBwdGrid = 1024;   // workgroups of the backward pass (most)

struct LearnedArgs {
    const void* filt;        // [P][N][N] store type
    void* ws;                // decimated data, store type (forward adds R)
    const float* dws;        // dL/dY, FP32, workspace layout (backward)
    const SquareDesc* squares;
    const int2* grid;        // u0, W per square
    const float* ac_p;       // [nsq][P] a_c(beta_p)
    const uint16_t* w;       // BF16 parameters
    float* grad;             // [817] FP32 (backward, overwritten)
    float* partials;         // [kLearnedBwdGrid][817] per-workgroup partial gradients (backward)
    int n, p, pd, nsq;
    int nv;                  // detector rows held by filt / ws / dws (a band of them: N in the whole-volume calls)
    int d;                   // angle dilation max(1, D / 4)
    int ntasks;              // nsq * nv
    int cubic;               // S by Keys' cubic convolution (the plan's cubic shift), else linear
};

// Transpose of the per-square backprojection (training).
// the adjoint's fixed-point scale: qscale = 2^e with bound * max |resid| *
// qscale < 2^61 (qscale = 0 when resid holds a value that is not finite)
struct AdjScale {
    double qscale;
    unsigned rmax;           // bits of max |resid| (non-negative floats order as integers)
    unsigned pad;
};

struct AdjArgs {
    const float* resid;      // [nz][n][n]
    float* dws;              // FP32, workspace layout, overwritten
    const SquareDesc* squares;
    const int2* grid;
    const float2* trig;      // cos, sin of beta'_m, [pd]
    const BpTile* tiles;     // 16 x 16 (x, y) tiles of the squares
    int ntiles;
    int n, nz, pd;           // nz: slices of resid (a slab of them: N_z in the whole-volume call)
    int v0, nv;              // detector rows [v0, v0 + nv) held by dws
    int zbase;               // volume slice of resid's slice 0
    float r, cu, cv, cz;
    float scale;             // pi / P'
    int64_t ws_elems;
    // fixed-point accumulation: every contribution is rounded to an integer
    // multiple of 1 / qscale and summed in int64 (exact, so the result does
    // not depend on the order of the atomics)
    unsigned long long* dq;  // [ws_elems] int64 sums, two's complement
    AdjScale* qs;            // the call's scale (device)
    double bound;            // an upper bound of sum |weight| over the voxels, per unit of max |resid|
    int64_t nvox;            // voxels of resid
};

struct AdamArgs {
    float* master;           // FP32 parameters
    float* m1;
    float* m2;
    const float* grad;
    uint16_t* w_bf16;        // BF16 copy used by the kernels
    int count, step;
    float lr, beta1, beta2, eps, weight_decay;
};

// dfac: the decimation factor D (selects the row-reusing form when D | P, D >= 4)
hipError_t launch_learned_fwd(const LearnedArgs& a, int max_width, int dfac, int store, hipStream_t st);
hipError_t launch_learned_bwd(const LearnedArgs& a, int store, hipStream_t st);
hipError_t launch_bp_adjoint(const AdjArgs& a, hipStream_t st);
hipError_t launch_residual(const float* f, const float* ref, float* r, double* loss, int64_t count, float weight,
                           hipStream_t st);
hipError_t launch_adamw(const AdamArgs& a, hipStream_t st);

// Checked builds (-DFDKOD_CHECKS).  Some kernel paths exist only to stay in
// bounds when the host's planning has gone wrong (a backprojection z run
// outside the staged detector rows contributes zero, a column outside the
// staged footprint is clamped, a decimation read beyond the staged segment);
// a checked build counts each such event in a device counter per kind, so
// tests can require that none occurs.  Unchecked builds compile the counting
// away.
enum CheckKind { kCheckBpRows = 0, kCheckBpCols = 1, kCheckDecimSegment = 2, kCheckKinds = 4 };
#ifdef FDKOD_CHECKS
#define FDKOD_CHECK_EVENT(counters, kind, cond)            \
    do {                                                   \
        if (cond) atomicAdd(&(counters)[(kind)], 1u);      \
    } while (0)
#else
#define FDKOD_CHECK_EVENT(counters, kind, cond) \
    do {                                        \
    } while (0)
#endif
// Each kernel file that counts keeps its own counters on the device; these
// read (and optionally clear) them on the current device, adding to out.
hipError_t checks_read_backproject(unsigned long long* out, bool reset);
hipError_t checks_read_decimate(unsigned long long* out, bool reset);

// Limits the host checks before choosing a backprojection variant.
constexpr int kTileXY = 16;      // voxels per tile side in x and y
constexpr int kDecimUnroll = 8;  // the decimation schedule is padded to a multiple of this
constexpr int kDecimMaxChunksWide = 4;  // column chunks per task when more than 2 windows are open
// detector rows per decimation task: two for one column chunk with the
// linear shift of detector rows (squares narrower than a wavefront: the two
// rows share the step's tables and fill more of the wave's work), else one
__host__ __device__ constexpr int decim_rows_per_task(bool cone, bool cubic, int chunks) {
    return !cone && !cubic && chunks == 1 ? 2 : 1;
}

}  // namespace fdkod
