// Host-side plan state shared by the single-plan and the batch entry points.
#pragma once

#include <string>
#include <vector>

#include "fdkod.h"
#include "internal.h"

struct fdkod_plan_s {
    fdkod_params prm{};
    int device = 0;
    int n = 0, nz = 0, p = 0, s = 0, k = 0, d = 1, pd = 0, nsq = 1, store = 0;
    int logm = 0;
    int cone = 0;           // cone-corrected rows (FDKOD_ROWS_CONE with s > 0)
    int nw = 2;             // windows a projection can feed: the decimation window's taps
    int sinc = 0;           // windowed-sinc decimation (FDKOD_DECIM_SINC)
    int cubic = 0;          // cubic shift (FDKOD_INTERP_CUBIC)
    double r = 0;
    std::vector<fdkod::SquareDesc> sq;
    std::vector<int2> grid;
    int wmax = 0;
    // decomposition kernel shape: 64-column chunks per wavefront of k_decimate,
    // or 0 for the row-staged kernel (whose shape is staged_cpt, staged_segc;
    // staged_cpt = 0 when it does not apply to the plan)
    int dec_chunks = 1;
    int staged_cpt = 0, staged_segc = 0;
    // backprojection kernel shape
    fdkod::BpVariant bpv{32, 32, 48, 1};
    bool bp_ok = false;     // some variant's LDS footprint holds a block's footprint
    int ntiles = 0;
    int64_t ws_row_elems = 0;  // workspace elements per detector row: P' * sum_q W_q
    int64_t ws_elems = 0;      // ws_row_elems * N
    float tuned_bp_ms = 0.0f, tuned_dec_ms = 0.0f;
    // device tables
    fdkod::SquareDesc* d_sq = nullptr;
    float2* d_trig_p = nullptr;
    float2* d_trig_m = nullptr;
    float* d_ac_p = nullptr;
    int2* d_crop = nullptr;
    int* d_blo = nullptr;       // row-staged decimation: [blocks][nsched] least crop offset of a 2 x 2 block
    int2* d_sqoff = nullptr;    // row-staged decimation: [nsq][nsched] offset from it, fraction bits
    float* d_lpartials = nullptr;  // learned backward: per-workgroup partial gradients (learned plans only)
    // the adjoint's scale and int64 sums (allocated by the first adjoint call,
    // grown when a later call needs more; freed with the plan)
    void* d_adj = nullptr;
    int64_t adj_cap = 0;        // int64 elements after the 256-byte scale block
    float* d_rscale = nullptr;  // [nsq][nsched] R / D_c (cone-corrected rows only)
    float* d_wext = nullptr;    // [nsched][nw - 2] weights of windows 2.. (nw > 2 only)
    float4* d_geo_m = nullptr;
    int2* d_grid = nullptr;
    int2* d_grid_direct = nullptr;
    fdkod::DecimStep* d_sched = nullptr;
    int nsched = 0;
    float2* d_resp = nullptr;
    float* d_gtail = nullptr;
    float2* d_tw = nullptr;
    fdkod::BpTile* d_tiles = nullptr;
    std::vector<void*> allocs;
};

namespace fdkod {

fdkod_status fail(fdkod_status st, const std::string& msg);
fdkod_status hip_fail(hipError_t e, const char* what);
// hipMalloc through the fault-injection switch (FDKOD_FAULT=nomem)
fdkod_status dev_alloc(std::vector<void*>& owner, void** ptr, size_t bytes);

// minimal LDS footprint (columns, rows) of a 16 x 16 x zrun block for a plan's
// geometry; false when no tile holds it.  cone_side > 0: cone-corrected rows
// of squares at most cone_side voxels wide.
bool bp_tiles_for(int n, int nz, double r, int zrun, int cone_side, int* tw, int* th);
// largest column-chunk count the plan's decimation kernels exist for
inline int max_chunks(const fdkod_plan_s* pl) { return pl->nw > 2 ? kDecimMaxChunksWide : 8; }
// square side bound for bp_tiles_for (0 unless the plan's rows are cone-corrected)
inline int cone_side(const fdkod_plan_s* pl) { return pl->cone ? (pl->n + (1 << pl->s) - 1) >> pl->s : 0; }
// a backprojection variant exists and its LDS footprint holds the plan's
bool variant_holds(const fdkod_plan_s* pl, const BpVariant& v);
// tasks per square of the decimation for a chunk count
inline int dec_tasks_per_sq(int wmax, int chunks) { return (wmax + 64 * chunks - 1) / (64 * chunks); }
// z slabs of the backprojection for a variant
inline int bp_zslabs(int nz, int zrun) { return (nz + zrun - 1) / zrun; }

// argument blocks for one plan (data pointers supplied by the caller); the
// _band forms cover detector rows [v0, v0 + nv) and output slices
// [zbase, zbase + nzs)
DecimVol decim_args(const fdkod_plan_s* pl, const void* filt, void* ws, int chunks);
DecimVol decim_args_band(const fdkod_plan_s* pl, const void* filt, void* ws, int chunks, int v0, int nv);
BpVol bp_vol(const fdkod_plan_s* pl, const void* filt, const void* ws, float* vol);
BpVol bp_vol_band(const fdkod_plan_s* pl, const void* filt, const void* ws, float* vol, int v0, int nv,
                  int zbase, int nzs);
FilterArgs filter_args(const fdkod_plan_s* pl, const float* proj, void* filt, int v0, int nv);
// arguments of the bounds kernel for a plan
BoundsArgs bounds_args(const fdkod_plan_s* pl);
// bands of detector rows and slabs of slices (eq. (9)): the rows a slab
// samples, and argument checks of the band calls
void band_for(const fdkod_plan_s* pl, int z0, int nzs, int* v0, int* nv);
fdkod_status check_rows_are_detector_rows(const fdkod_plan_s* pl);
fdkod_status check_band(const fdkod_plan_s* pl, int v0, int nv);
fdkod_status check_slab(const fdkod_plan_s* pl, int v0, int nv, int z0, int nzs);
// the plan's decimation kernel on detector rows [v0, v0 + nv) (filt and ws
// hold those rows)
fdkod_status enqueue_decimate(const fdkod_plan_s* pl, const void* filt, void* ws, int v0, int nv,
                              hipStream_t st);

}  // namespace fdkod

#define HIP_TRY(expr, what)                                     \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return fdkod::hip_fail(e_, what); \
    } while (0)
