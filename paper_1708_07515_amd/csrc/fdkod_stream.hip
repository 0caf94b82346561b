// Low-memory reconstruction by slabs (C ABI in include/fdkod.h).  Eq. (9)
// bounds the detector rows that a slab of slices uses, so the filter, the
// decomposition and the reconstruction of a slab run on a band of rows of
// every projection; the streaming driver moves the bands from host memory
// through two device buffers while the previous band is being processed.
#include <algorithm>
#include <cmath>

#include "dtype.h"
#include "plan.h"

using namespace fdkod;

namespace fdkod {

// Detector rows [v0, v0 + nv) that the voxels of slices [z0, z0 + nzs) sample
// at any angle: b = z R / depth (eq. (9)) over depth in [R - c sqrt2, R + c sqrt2]
// and the slab's extreme z, the two rows of the bilinear sample, one row of
// margin on each side, widened to even row boundaries (the filter transforms
// rows in pairs 2k, 2k + 1) and clipped to the detector.
void band_for(const fdkod_plan_s* pl, int z0, int nzs, int* v0, int* nv) {
    const double c = (pl->n - 1) / 2.0, cz = (pl->nz - 1) / 2.0;
    const double dmin = pl->r - c * std::sqrt(2.0), dmax = pl->r + c * std::sqrt(2.0);
    const double zl = z0 - cz, zh = z0 + nzs - 1 - cz;
    const double b[4] = {zl * pl->r / dmin, zl * pl->r / dmax, zh * pl->r / dmin, zh * pl->r / dmax};
    const double bmin = *std::min_element(b, b + 4), bmax = *std::max_element(b, b + 4);
    const int lo = std::max(0, (int)std::floor(c + bmin) - 1) & ~1;
    const int hi = std::min(pl->n, ((int)std::floor(c + bmax) + 3 + 1) & ~1);
    *v0 = lo;
    *nv = std::max(0, hi - lo);
}

// cone-corrected rows are not detector rows: a band of them would need the
// whole detector height, so the slab mode covers the triangle decimation only
fdkod_status check_rows_are_detector_rows(const fdkod_plan_s* pl) {
    if (pl->cone) return fail(FDKOD_E_UNSUPPORTED, "the slab mode needs the triangle decimation");
    return FDKOD_OK;
}

fdkod_status check_band(const fdkod_plan_s* pl, int v0, int nv) {
    if (v0 < 0 || nv < 1 || v0 + nv > pl->n) return fail(FDKOD_E_ARG, "band rows outside the detector");
    return FDKOD_OK;
}

fdkod_status check_slab(const fdkod_plan_s* pl, int v0, int nv, int z0, int nzs) {
    if (z0 < 0 || nzs < 1 || z0 + nzs > pl->nz) return fail(FDKOD_E_ARG, "slab slices outside the volume");
    int need0 = 0, neednv = 0;
    band_for(pl, z0, nzs, &need0, &neednv);
    if (v0 > need0 || v0 + nv < need0 + neednv)
        return fail(FDKOD_E_ARG, "the band does not hold every row the slab samples (see fdkod_band_rows)");
    return FDKOD_OK;
}

}  // namespace fdkod

namespace {

struct StreamLayout {
    int slab = 0, maxnv = 0;
    int64_t proj = 0, filt = 0, ws = 0, vol = 0;   // bytes of one buffer
    int64_t off_proj[2] = {0, 0}, off_filt = 0, off_ws = 0, off_vol[2] = {0, 0}, total = 0;
};

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

StreamLayout stream_layout(const fdkod_plan_s* pl, int nzs) {
    StreamLayout L;
    // slabs start at multiples of the z run, so the band results equal the
    // whole-volume results bit for bit
    const int zr = pl->bpv.zrun;
    L.slab = std::max(zr, (nzs + zr - 1) / zr * zr);
    for (int z0 = 0; z0 < pl->nz; z0 += L.slab) {
        int v0 = 0, nv = 0;
        band_for(pl, z0, std::min(L.slab, pl->nz - z0), &v0, &nv);
        L.maxnv = std::max(L.maxnv, nv);
    }
    const int64_t es = store_bytes(pl->store);
    L.proj = (int64_t)pl->p * L.maxnv * pl->n * 4;
    L.filt = (int64_t)pl->p * L.maxnv * pl->n * es;
    L.ws = pl->s > 0 ? pl->ws_row_elems * L.maxnv * es : 0;
    L.vol = (int64_t)std::min(L.slab, pl->nz) * pl->n * pl->n * 4;
    int64_t off = 0;
    for (int b = 0; b < 2; ++b) {
        L.off_proj[b] = off;
        off = align256(off + L.proj);
    }
    L.off_filt = off;
    off = align256(off + L.filt);
    L.off_ws = off;
    off = align256(off + L.ws);
    for (int b = 0; b < 2; ++b) {
        L.off_vol[b] = off;
        off = align256(off + L.vol);
    }
    L.total = off;
    return L;
}

fdkod_status launch_slab(const fdkod_plan_s* pl, const void* filt, const void* ws, int v0, int nv, int z0,
                         int nzs, float* vol, hipStream_t st) {
    BpArgs a;
    a.v = bp_vol_band(pl, filt, ws, vol, v0, nv, z0, nzs);
    a.tiles = pl->d_tiles;
    a.ntiles = pl->ntiles;
    a.nzt = bp_zslabs(nzs, pl->bpv.zrun);
    a.nlogical = a.ntiles * a.nzt;
    a.chunk = (a.nlogical + 7) / 8;
    HIP_TRY(launch_backproject(a, pl->bpv, pl->store, st), "backprojection kernel launch");
    return FDKOD_OK;
}

}  // namespace

extern "C" {

fdkod_status fdkod_band_rows(fdkod_plan_t pl, int32_t z0, int32_t nzs, int32_t* v0, int32_t* nrows) {
    if (!pl || !v0 || !nrows) return fail(FDKOD_E_ARG, "NULL argument");
    if (z0 < 0 || nzs < 1 || z0 + nzs > pl->nz) return fail(FDKOD_E_ARG, "slab slices outside the volume");
    if (check_rows_are_detector_rows(pl) != FDKOD_OK) return FDKOD_E_UNSUPPORTED;
    int a = 0, b = 0;
    band_for(pl, z0, nzs, &a, &b);
    *v0 = a;
    *nrows = b;
    return FDKOD_OK;
}

fdkod_status fdkod_filter_band(fdkod_plan_t pl, const float* proj_band, int32_t v0, int32_t nrows,
                               void* filt_band, fdkod_stream_t stream) {
    if (!pl || !proj_band || !filt_band) return fail(FDKOD_E_ARG, "NULL argument");
    fdkod_status st = check_band(pl, v0, nrows);
    if (st != FDKOD_OK) return st;
    const FilterArgs a = filter_args(pl, proj_band, filt_band, v0, nrows);
    HIP_TRY(launch_filter(a, pl->logm, pl->store, (hipStream_t)stream), "filter kernel launch");
    return FDKOD_OK;
}

fdkod_status fdkod_decompose_band(fdkod_plan_t pl, const void* filt_band, int32_t v0, int32_t nrows,
                                  void* ws_band, fdkod_stream_t stream) {
    if (!pl || !filt_band) return fail(FDKOD_E_ARG, "NULL argument");
    fdkod_status st = check_band(pl, v0, nrows);
    if (st != FDKOD_OK) return st;
    if ((st = check_rows_are_detector_rows(pl)) != FDKOD_OK) return st;
    if (pl->s == 0) return FDKOD_OK;
    if (!ws_band) return fail(FDKOD_E_ARG, "workspace is NULL");
    return enqueue_decimate(pl, filt_band, ws_band, v0, nrows, (hipStream_t)stream);
}

fdkod_status fdkod_reconstruct_slab(fdkod_plan_t pl, const void* filt_band, const void* ws_band, int32_t v0,
                                    int32_t nrows, int32_t z0, int32_t nzs, float* vol_slab,
                                    fdkod_stream_t stream) {
    if (!pl || !vol_slab) return fail(FDKOD_E_ARG, "NULL argument");
    if (pl->s == 0 && !filt_band) return fail(FDKOD_E_ARG, "filtered band is NULL");
    if (pl->s > 0 && !ws_band) return fail(FDKOD_E_ARG, "workspace band is NULL");
    if (!pl->bp_ok)
        return fail(FDKOD_E_UNSUPPORTED, "R too small: a block's detector footprint exceeds the LDS tiles");
    fdkod_status st = check_band(pl, v0, nrows);
    if (st != FDKOD_OK) return st;
    if ((st = check_rows_are_detector_rows(pl)) != FDKOD_OK) return st;
    if ((st = check_slab(pl, v0, nrows, z0, nzs)) != FDKOD_OK) return st;
    return launch_slab(pl, filt_band, ws_band, v0, nrows, z0, nzs, vol_slab, (hipStream_t)stream);
}

fdkod_status fdkod_streamed_bytes(fdkod_plan_t pl, int32_t nzs, int64_t* bytes) {
    if (!pl || !bytes) return fail(FDKOD_E_ARG, "NULL argument");
    if (nzs < 1) return fail(FDKOD_E_ARG, "slab must hold at least one slice");
    *bytes = stream_layout(pl, nzs).total;
    return FDKOD_OK;
}

fdkod_status fdkod_reconstruct_streamed(fdkod_plan_t pl, const float* host_proj, float* host_vol, int32_t nzs,
                                        void* work, int64_t work_bytes, fdkod_stream_t stream,
                                        fdkod_stream_t copy_stream) {
    if (!pl || !host_proj || !host_vol || !work) return fail(FDKOD_E_ARG, "NULL argument");
    if (nzs < 1) return fail(FDKOD_E_ARG, "slab must hold at least one slice");
    if (check_rows_are_detector_rows(pl) != FDKOD_OK) return FDKOD_E_UNSUPPORTED;
    if (!pl->bp_ok)
        return fail(FDKOD_E_UNSUPPORTED, "R too small: a block's detector footprint exceeds the LDS tiles");
    const StreamLayout L = stream_layout(pl, nzs);
    if (work_bytes < L.total) return fail(FDKOD_E_ARG, "work buffer smaller than fdkod_streamed_bytes");
    int prev = 0;
    HIP_TRY(hipGetDevice(&prev), "hipGetDevice");
    HIP_TRY(hipSetDevice(pl->device), "hipSetDevice");
    hipStream_t cs = (hipStream_t)stream;
    hipStream_t ms = copy_stream ? (hipStream_t)copy_stream : cs;
    char* base = (char*)work;
    float* proj[2] = {(float*)(base + L.off_proj[0]), (float*)(base + L.off_proj[1])};
    void* filt = base + L.off_filt;
    void* ws = pl->s > 0 ? (void*)(base + L.off_ws) : nullptr;
    float* vol[2] = {(float*)(base + L.off_vol[0]), (float*)(base + L.off_vol[1])};
    const int nslab = (pl->nz + L.slab - 1) / L.slab;
    const size_t row_bytes = (size_t)pl->n * 4;
    const size_t proj_pitch = (size_t)pl->n * pl->n * 4;

    // events: band b copied in, band b consumed by the filter, slab b written,
    // slab b copied out
    hipEvent_t ev[8] = {};
    fdkod_status r = FDKOD_OK;
    for (int i = 0; i < 8 && r == FDKOD_OK; ++i) {
        hipError_t e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
        if (e != hipSuccess) r = hip_fail(e, "hipEventCreate");
    }
    hipEvent_t* copied = ev;
    hipEvent_t* consumed = ev + 2;
    hipEvent_t* written = ev + 4;
    hipEvent_t* drained = ev + 6;
    bool used_proj[2] = {false, false}, used_vol[2] = {false, false};
    auto copy_in = [&](int k) -> fdkod_status {
        const int b = k & 1;
        const int z0 = k * L.slab, nz = std::min(L.slab, pl->nz - z0);
        int v0 = 0, nv = 0;
        band_for(pl, z0, nz, &v0, &nv);
        if (used_proj[b]) HIP_TRY(hipStreamWaitEvent(ms, consumed[b], 0), "hipStreamWaitEvent");
        // rows [v0, v0 + nv) of every projection: one strided copy
        HIP_TRY(hipMemcpy2DAsync(proj[b], (size_t)nv * row_bytes, (const char*)host_proj + (size_t)v0 * row_bytes,
                                 proj_pitch, (size_t)nv * row_bytes, pl->p, hipMemcpyHostToDevice, ms),
                "hipMemcpy2DAsync band");
        HIP_TRY(hipEventRecord(copied[b], ms), "hipEventRecord");
        used_proj[b] = true;
        return FDKOD_OK;
    };
    if (r == FDKOD_OK) r = copy_in(0);
    for (int k = 0; k < nslab && r == FDKOD_OK; ++k) {
        const int b = k & 1;
        const int z0 = k * L.slab, nz = std::min(L.slab, pl->nz - z0);
        int v0 = 0, nv = 0;
        band_for(pl, z0, nz, &v0, &nv);
        if (k + 1 < nslab && (r = copy_in(k + 1)) != FDKOD_OK) break;
        auto step = [&]() -> fdkod_status {
            HIP_TRY(hipStreamWaitEvent(cs, copied[b], 0), "hipStreamWaitEvent");
            fdkod_status s2 = fdkod_filter_band(pl, proj[b], v0, nv, filt, cs);
            if (s2 != FDKOD_OK) return s2;
            HIP_TRY(hipEventRecord(consumed[b], cs), "hipEventRecord");
            if ((s2 = fdkod_decompose_band(pl, filt, v0, nv, ws, cs)) != FDKOD_OK) return s2;
            if (used_vol[b]) HIP_TRY(hipStreamWaitEvent(cs, drained[b], 0), "hipStreamWaitEvent");
            if ((s2 = launch_slab(pl, filt, ws, v0, nv, z0, nz, vol[b], cs)) != FDKOD_OK) return s2;
            HIP_TRY(hipEventRecord(written[b], cs), "hipEventRecord");
            HIP_TRY(hipStreamWaitEvent(ms, written[b], 0), "hipStreamWaitEvent");
            HIP_TRY(hipMemcpyAsync(host_vol + (size_t)z0 * pl->n * pl->n, vol[b], (size_t)nz * pl->n * pl->n * 4,
                                   hipMemcpyDeviceToHost, ms),
                    "hipMemcpyAsync slab");
            HIP_TRY(hipEventRecord(drained[b], ms), "hipEventRecord");
            used_vol[b] = true;
            return FDKOD_OK;
        };
        r = step();
    }
    // drain both streams whatever happened, then release the events
    const hipError_t e1 = hipStreamSynchronize(cs);
    const hipError_t e2 = ms != cs ? hipStreamSynchronize(ms) : hipSuccess;
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    (void)hipSetDevice(prev);
    if (r != FDKOD_OK) return r;
    if (e1 != hipSuccess) return hip_fail(e1, "hipStreamSynchronize");
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamSynchronize");
    return FDKOD_OK;
}

}  // extern "C"
