// Batches of uneven volumes (C ABI in include/fdkod.h): every volume keeps its
// own plan (squares, bounds, schedule); the bounds of all volumes run as one
// launch, the filters as one launch per FFT length (volumes that fill the GPU
// alone keep their own), the decimation as one grouped launch and the
// backprojection as one persistent launch that takes (volume, square, tile,
// slab) items from a ticket queue, largest first.
// The launch sequence is capture-safe and can be replayed as a hipGraph.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <utility>
#include <vector>

#include "fdkod.h"
#include "internal.h"
#include "plan.h"

using namespace fdkod;

struct fdkod_batch_s {
    int device = 0, count = 0, store = 0;
    std::vector<fdkod_plan_t> plans;
    BpVariant bpv{32, 32, 48, 1};
    int dec_chunks = 1;
    int bp_blocks = 0;
    int nitems = 0;
    int xstart[kXcds + 1] = {};
    int64_t updates_eq = 0;
    // device tables
    BatchItem* d_items = nullptr;
    int items_cap = 0;
    BpVol* d_vols = nullptr;
    DecimVol* d_dvols = nullptr;
    int2* d_block_vol = nullptr;
    int block_vol_cap = 0;
    unsigned* d_counter = nullptr;
    // bounds of every volume in one launch, filters in one launch per FFT
    // length (volumes grouped by length; per-volume arguments and workgroup
    // ranges, written when the buffers are bound)
    struct FilterGroup {
        int logm, nvol, workgroups;
        const FilterArgs* args;
        const int* start;
    };
    std::vector<FilterGroup> fgroups;
    std::vector<std::pair<FilterArgs, int>> fown;   // (arguments, log2 M) of volumes with a launch of their own
    FilterArgs* d_fargs = nullptr;
    int* d_fstart = nullptr;
    BoundsArgs* d_bargs = nullptr;
    int* d_bstart = nullptr;
    int bounds_wg = 0;
    std::vector<void*> allocs;
    // bound buffers
    bool bound = false;
    std::vector<const float*> proj;
    std::vector<void*> filt, ws;
    std::vector<float*> vol;
    int ndec = 0, dec_ntasks = 0;
    // captured launch sequence
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void drop_graph(fdkod_batch_t b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

void release_batch(fdkod_batch_t b) {
    if (!b) return;
    drop_graph(b);
    int prev = 0;
    if (hipGetDevice(&prev) == hipSuccess) {
        (void)hipSetDevice(b->device);
        for (void* p : b->allocs) (void)hipFree(p);
        (void)hipSetDevice(prev);
    }
    for (fdkod_plan_t p : b->plans) fdkod_plan_destroy(p);
    delete b;
}

// A variant usable by every volume of the batch.
bool holds_all(const fdkod_batch_t b, const BpVariant& v) {
    for (fdkod_plan_t p : b->plans)
        if (!variant_holds(p, v)) return false;
    return true;
}

// Work items of the persistent backprojection for the current z run: volumes
// by decreasing work, each volume's items by square, slab and tile (tiles
// that share footprints are adjacent), then cut into one range per XCD of
// about equal work (tile voxels x slab depth x decimated angles).
fdkod_status build_items(fdkod_batch_t b) {
    std::vector<int> order(b->count);
    std::iota(order.begin(), order.end(), 0);
    auto vol_work = [&](int vb) {
        const fdkod_plan_s* pl = b->plans[vb];
        return (int64_t)pl->n * pl->n * pl->nz * pl->pd;
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return vol_work(x) > vol_work(y); });
    std::vector<BatchItem> items;
    std::vector<int64_t> work;
    for (int vb : order) {
        const fdkod_plan_s* pl = b->plans[vb];
        const int nzt = bp_zslabs(pl->nz, b->bpv.zrun);
        for (int q = 0; q < pl->nsq; ++q) {
            const SquareDesc& d = pl->sq[q];
            for (int zt = 0; zt < nzt; ++zt) {
                const int zc = std::min(b->bpv.zrun, pl->nz - zt * b->bpv.zrun);
                for (int y = d.y0; y < d.y1; y += kTileXY)
                    for (int x = d.x0; x < d.x1; x += kTileXY) {
                        const int64_t vox = (int64_t)std::min(kTileXY, d.x1 - x) * std::min(kTileXY, d.y1 - y);
                        items.push_back(BatchItem{vb, q, x, y, zt, 0, 0, 0});
                        work.push_back(vox * zc * pl->pd);
                    }
            }
        }
        if ((int64_t)items.size() > (int64_t)1 << 30) return fail(FDKOD_E_UNSUPPORTED, "too many work items");
    }
    const int64_t total = std::accumulate(work.begin(), work.end(), (int64_t)0);
    b->xstart[0] = 0;
    int64_t acc = 0;
    size_t i = 0;
    for (int x = 1; x < kXcds; ++x) {
        const int64_t target = total * x / kXcds;
        while (i < items.size() && acc + work[i] <= target) acc += work[i++];
        b->xstart[x] = (int)i;
    }
    b->xstart[kXcds] = (int)items.size();
    if ((int)items.size() > b->items_cap) {
        fdkod_status st = dev_alloc(b->allocs, (void**)&b->d_items, sizeof(BatchItem) * items.size());
        if (st != FDKOD_OK) return st;
        b->items_cap = (int)items.size();
    }
    HIP_TRY(hipMemcpy(b->d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice),
            "hipMemcpy items");
    b->nitems = (int)items.size();
    const int occ = backproject_batch_occupancy(b->bpv, b->store);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, b->device), "hipGetDeviceProperties");
    b->bp_blocks = std::max(1, occ) * prop.multiProcessorCount;
    b->bp_blocks = (b->bp_blocks + kXcds - 1) / kXcds * kXcds;
    return FDKOD_OK;
}

// Per-volume argument tables for the bound buffers and the current chunking.
fdkod_status upload_tables(fdkod_batch_t b) {
    std::vector<BpVol> vols(b->count);
    std::vector<DecimVol> dvols;
    std::vector<int2> block_vol;
    int start = 0;
    for (int vb = 0; vb < b->count; ++vb) {
        const fdkod_plan_s* pl = b->plans[vb];
        vols[vb] = bp_vol(pl, b->filt[vb], b->ws[vb], b->vol[vb]);
        if (pl->s > 0) {
            // the batch's chunk count is an upper bound: narrow volumes use fewer
            int c = 1;
            while (c < b->dec_chunks && 64 * c < pl->wmax) c <<= 1;
            dvols.push_back(decim_args(pl, b->filt[vb], b->ws[vb], c));
            const int nblk = (dvols.back().ntasks + 3) / 4;     // padded to whole workgroups
            for (int g = 0; g < nblk; ++g) block_vol.push_back(make_int2((int)dvols.size() - 1, start));
            start += 4 * nblk;
        }
    }
    b->ndec = (int)dvols.size();
    b->dec_ntasks = start;
    HIP_TRY(hipMemcpy(b->d_vols, vols.data(), sizeof(BpVol) * vols.size(), hipMemcpyHostToDevice),
            "hipMemcpy volumes");
    if (!dvols.empty()) {
        HIP_TRY(hipMemcpy(b->d_dvols, dvols.data(), sizeof(DecimVol) * dvols.size(), hipMemcpyHostToDevice),
                "hipMemcpy decimation volumes");
        if ((int)block_vol.size() > b->block_vol_cap) {
            fdkod_status st = dev_alloc(b->allocs, (void**)&b->d_block_vol, sizeof(int2) * block_vol.size());
            if (st != FDKOD_OK) return st;
            b->block_vol_cap = (int)block_vol.size();
        }
        HIP_TRY(hipMemcpy(b->d_block_vol, block_vol.data(), sizeof(int2) * block_vol.size(), hipMemcpyHostToDevice),
                "hipMemcpy workgroup table");
    }
    return FDKOD_OK;
}

// A volume whose filter alone has this many workgroups fills the GPU and
// keeps a launch of its own (the grouped kernels of the larger lengths spill
// registers to scratch; the single-volume ones do not).
constexpr int kFilterOwnLaunch = 8192;

// The bounds and filter tables of the bound buffers (sizes depend only on
// the volumes: allocated at the first binding).
fdkod_status upload_front_tables(fdkod_batch_t b) {
    const int n = b->count;
    fdkod_status st;
    if (!b->d_fargs) {
        if ((st = dev_alloc(b->allocs, (void**)&b->d_fargs, sizeof(FilterArgs) * n)) != FDKOD_OK) return st;
        if ((st = dev_alloc(b->allocs, (void**)&b->d_fstart, sizeof(int) * 2 * n)) != FDKOD_OK) return st;
        if ((st = dev_alloc(b->allocs, (void**)&b->d_bargs, sizeof(BoundsArgs) * n)) != FDKOD_OK) return st;
        if ((st = dev_alloc(b->allocs, (void**)&b->d_bstart, sizeof(int) * (n + 1))) != FDKOD_OK) return st;
    }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->plans[x]->logm < b->plans[y]->logm; });
    std::vector<FilterArgs> fargs;
    std::vector<int> fstart;
    b->fgroups.clear();
    b->fown.clear();
    for (int i = 0; i < n;) {
        const int logm = b->plans[order[i]]->logm;
        fdkod_batch_s::FilterGroup g{logm, 0, 0, b->d_fargs + fargs.size(), b->d_fstart + fstart.size()};
        int wg = 0;
        for (; i < n && b->plans[order[i]]->logm == logm; ++i) {
            const int v = order[i];
            const FilterArgs fa = filter_args(b->plans[v], b->proj[v], b->filt[v], 0, b->plans[v]->n);
            if (filter_workgroups(fa, logm) >= kFilterOwnLaunch) {
                b->fown.emplace_back(fa, logm);
                continue;
            }
            fargs.push_back(fa);
            fstart.push_back(wg);
            wg += filter_workgroups(fa, logm);
            ++g.nvol;
        }
        if (g.nvol == 0) continue;
        fstart.push_back(wg);
        g.workgroups = wg;
        b->fgroups.push_back(g);
    }
    std::vector<BoundsArgs> bargs(n);
    std::vector<int> bstart(n + 1, 0);
    for (int v = 0; v < n; ++v) {
        bargs[v] = bounds_args(b->plans[v]);
        bstart[v + 1] = bstart[v] + b->plans[v]->nsq;
    }
    b->bounds_wg = bstart[n];
    if (!fargs.empty()) {
        HIP_TRY(hipMemcpy(b->d_fargs, fargs.data(), sizeof(FilterArgs) * fargs.size(), hipMemcpyHostToDevice),
                "hipMemcpy filter arguments");
        HIP_TRY(hipMemcpy(b->d_fstart, fstart.data(), sizeof(int) * fstart.size(), hipMemcpyHostToDevice),
                "hipMemcpy filter ranges");
    }
    HIP_TRY(hipMemcpy(b->d_bargs, bargs.data(), sizeof(BoundsArgs) * n, hipMemcpyHostToDevice),
            "hipMemcpy bounds arguments");
    HIP_TRY(hipMemcpy(b->d_bstart, bstart.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice),
            "hipMemcpy bounds ranges");
    return FDKOD_OK;
}

fdkod_status run_filters(fdkod_batch_t b, hipStream_t st) {
    for (const auto& g : b->fgroups)
        HIP_TRY(launch_filter_batch(FilterBatchArgs{g.args, g.start, g.nvol}, g.logm, b->store, g.workgroups, st),
                "batched filter launch");
    for (const auto& f : b->fown)
        HIP_TRY(launch_filter(f.first, f.second, b->store, st), "filter kernel launch");
    return FDKOD_OK;
}

fdkod_status run_bounds(fdkod_batch_t b, hipStream_t st) {
    HIP_TRY(launch_bounds_batch(BoundsBatchArgs{b->d_bargs, b->d_bstart, b->count}, b->bounds_wg, st),
            "batched bounds launch");
    return FDKOD_OK;
}

fdkod_status run_decimate(fdkod_batch_t b, hipStream_t st) {
    if (b->ndec == 0) return FDKOD_OK;
    DecimBatchArgs a{b->d_dvols, b->d_block_vol, b->ndec, b->dec_ntasks};
    HIP_TRY(launch_decimate_batch(a, b->dec_chunks, b->store, st), "batched decimation launch");
    return FDKOD_OK;
}

fdkod_status run_backproject(fdkod_batch_t b, hipStream_t st) {
    HIP_TRY(launch_reset_counter(b->d_counter, st), "counter reset launch");
    BpBatchArgs a;
    a.vols = b->d_vols;
    a.items = b->d_items;
    a.nitems = b->nitems;
    for (int x = 0; x <= kXcds; ++x) a.xstart[x] = b->xstart[x];
    a.counter = b->d_counter;
    HIP_TRY(launch_backproject_batch(a, b->bpv, b->store, b->bp_blocks, st), "persistent backprojection launch");
    return FDKOD_OK;
}

template <class F>
fdkod_status time_ms(hipStream_t st, int reps, F fn, float* ms) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
    fdkod_status r = fn();
    if (r == FDKOD_OK) {
        (void)hipEventRecord(e0, st);
        for (int i = 0; i < reps && r == FDKOD_OK; ++i) r = fn();
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float t = 0.0f;
        (void)hipEventElapsedTime(&t, e0, e1);
        *ms = t / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return r;
}

}  // namespace

extern "C" {

fdkod_status fdkod_batch_create(const fdkod_params* prms, int32_t count, int device, fdkod_batch_t* out) {
    if (!out) return fail(FDKOD_E_ARG, "out is NULL");
    *out = nullptr;
    if (!prms || count < 1 || count > 4096) return fail(FDKOD_E_ARG, "count must be in [1, 4096]");
    for (int i = 0; i < count; ++i) {
        fdkod_status st = fdkod_validate(&prms[i]);
        if (st != FDKOD_OK) return st;
        if (prms[i].store != prms[0].store) return fail(FDKOD_E_ARG, "all volumes of a batch share the store type");
        if (prms[i].s > 0 && (prms[i].decim != FDKOD_DECIM_TRIANGLE || prms[i].rows != FDKOD_ROWS_DETECTOR ||
                              prms[i].interp != FDKOD_INTERP_LINEAR))
            return fail(FDKOD_E_UNSUPPORTED, "batches use the triangle decimation on detector rows, linear shift");
    }
    fdkod_batch_t b = new fdkod_batch_s();
    b->device = device;
    b->count = count;
    b->store = prms[0].store;
    for (int i = 0; i < count; ++i) {
        fdkod_plan_t p = nullptr;
        fdkod_status st = fdkod_plan_create(&prms[i], device, &p);
        if (st != FDKOD_OK) {
            release_batch(b);
            return st;
        }
        b->plans.push_back(p);
        b->updates_eq += (int64_t)p->n * p->n * p->nz * p->p;
    }
    int prev = 0;
    HIP_TRY(hipGetDevice(&prev), "hipGetDevice");
    HIP_TRY(hipSetDevice(device), "hipSetDevice");
    auto bail = [&](fdkod_status code) {
        release_batch(b);
        (void)hipSetDevice(prev);
        return code;
    };
    // common kernel shapes: the longest z run every volume supports, the
    // largest footprint among the volumes, chunks for the widest square
    bool ok = false;
    for (int zr : {32, 16}) {
        int tw = 0, th = 0;
        bool all = true;
        for (fdkod_plan_t p : b->plans) {
            int w = 0, h = 0;
            if (!bp_tiles_for(p->n, p->nz, p->r, zr, 0, &w, &h)) {
                all = false;
                break;
            }
            tw = std::max(tw, w);
            th = std::max(th, h);
        }
        if (!all) continue;
        b->bpv = BpVariant{zr, tw, th, 1};
        ok = holds_all(b, b->bpv);
        if (ok) break;
    }
    if (!ok) return bail(fail(FDKOD_E_UNSUPPORTED, "no backprojection variant holds every volume"));
    int wmax = 0;
    for (fdkod_plan_t p : b->plans)
        if (p->s > 0) wmax = std::max(wmax, p->wmax);
    b->dec_chunks = 1;
    while (b->dec_chunks < 8 && 64 * b->dec_chunks < wmax) b->dec_chunks <<= 1;

    fdkod_status st;
    if ((st = dev_alloc(b->allocs, (void**)&b->d_vols, sizeof(BpVol) * count)) != FDKOD_OK) return bail(st);
    if ((st = dev_alloc(b->allocs, (void**)&b->d_dvols, sizeof(DecimVol) * count)) != FDKOD_OK) return bail(st);
    if ((st = dev_alloc(b->allocs, (void**)&b->d_counter, sizeof(unsigned) * kXcds * kCounterStride)) != FDKOD_OK)
        return bail(st);
    if ((st = build_items(b)) != FDKOD_OK) return bail(st);
    (void)hipSetDevice(prev);
    *out = b;
    return FDKOD_OK;
}

fdkod_status fdkod_batch_destroy(fdkod_batch_t batch) {
    release_batch(batch);
    return FDKOD_OK;
}

fdkod_status fdkod_batch_plan(fdkod_batch_t b, int32_t index, fdkod_plan_t* out) {
    if (!b || !out || index < 0 || index >= b->count) return fail(FDKOD_E_ARG, "bad batch index");
    *out = b->plans[index];
    return FDKOD_OK;
}

fdkod_status fdkod_batch_bind(fdkod_batch_t b, const float* const* proj, void* const* filt,
                              void* const* ws, float* const* vol) {
    if (!b || !proj || !filt || !ws || !vol) return fail(FDKOD_E_ARG, "NULL argument");
    for (int i = 0; i < b->count; ++i)
        if (!proj[i] || !filt[i] || !vol[i] || (b->plans[i]->s > 0 && !ws[i]))
            return fail(FDKOD_E_ARG, "NULL buffer in batch binding");
    b->proj.assign(proj, proj + b->count);
    b->filt.assign(filt, filt + b->count);
    b->ws.assign(ws, ws + b->count);
    b->vol.assign(vol, vol + b->count);
    drop_graph(b);
    fdkod_status st = upload_tables(b);
    if (st == FDKOD_OK) st = upload_front_tables(b);
    b->bound = st == FDKOD_OK;
    return st;
}

fdkod_status fdkod_batch_run(fdkod_batch_t b, fdkod_stream_t stream) {
    if (!b) return fail(FDKOD_E_ARG, "batch is NULL");
    if (!b->bound) return fail(FDKOD_E_STATE, "batch buffers are not bound");
    hipStream_t st = (hipStream_t)stream;
    fdkod_status r;
    if ((r = run_bounds(b, st)) != FDKOD_OK) return r;
    if ((r = run_filters(b, st)) != FDKOD_OK) return r;
    if ((r = run_decimate(b, st)) != FDKOD_OK) return r;
    return run_backproject(b, st);
}

fdkod_status fdkod_batch_capture(fdkod_batch_t b, fdkod_stream_t stream) {
    if (!b) return fail(FDKOD_E_ARG, "batch is NULL");
    if (!stream) return fail(FDKOD_E_ARG, "graph capture needs a non-null stream");
    if (!b->bound) return fail(FDKOD_E_STATE, "batch buffers are not bound");
    drop_graph(b);
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    const fdkod_status r = fdkod_batch_run(b, stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (r != FDKOD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    return FDKOD_OK;
}

fdkod_status fdkod_batch_replay(fdkod_batch_t b, fdkod_stream_t stream) {
    if (!b) return fail(FDKOD_E_ARG, "batch is NULL");
    if (!b->exec) return fail(FDKOD_E_STATE, "no captured graph (call fdkod_batch_capture)");
    HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)stream), "hipGraphLaunch");
    return FDKOD_OK;
}

fdkod_status fdkod_batch_tune(fdkod_batch_t b, fdkod_stream_t stream, fdkod_tuning* out) {
    if (!b) return fail(FDKOD_E_ARG, "batch is NULL");
    if (!b->bound) return fail(FDKOD_E_STATE, "batch buffers are not bound");
    hipStream_t st = (hipStream_t)stream;
    drop_graph(b);
    fdkod_status r;
    if ((r = run_filters(b, st)) != FDKOD_OK) return r;
    float dec_best = 0.0f;
    if (b->ndec > 0) {
        float best = 1e30f;
        int bestc = b->dec_chunks;
        for (int c : {1, 2, 4, 8}) {
            b->dec_chunks = c;
            if ((r = upload_tables(b)) != FDKOD_OK) return r;
            float ms = 0.0f;
            if ((r = time_ms(st, 3, [&] { return run_decimate(b, st); }, &ms)) != FDKOD_OK) return r;
            if (ms < best) {
                best = ms;
                bestc = c;
            }
        }
        b->dec_chunks = bestc;
        dec_best = best;
        if ((r = upload_tables(b)) != FDKOD_OK) return r;
        if ((r = run_decimate(b, st)) != FDKOD_OK) return r;
    }
    float best = 1e30f;
    BpVariant bestv = b->bpv;
    for (int zr : {64, 32, 16})
        for (int tw : {32, 64})
            for (int th : {48, 64, 96})
                for (int g : {1, 2, 4}) {
                    const BpVariant v{zr, tw, th, g};
                    if (!holds_all(b, v)) continue;
                    b->bpv = v;
                    if ((r = build_items(b)) != FDKOD_OK) return r;
                    float ms = 0.0f;
                    if ((r = time_ms(st, 3, [&] { return run_backproject(b, st); }, &ms)) != FDKOD_OK) return r;
                    if (ms < best) {
                        best = ms;
                        bestv = v;
                    }
                }
    b->bpv = bestv;
    if ((r = build_items(b)) != FDKOD_OK) return r;
    if (out) {
        out->z_run = b->bpv.zrun;
        out->tile_w = b->bpv.tile_w;
        out->tile_h = b->bpv.tile_h;
        out->angles_per_stage = b->bpv.g;
        out->decim_chunks = b->dec_chunks;
        out->bp_ms = best;
        out->decim_ms = dec_best;
    }
    return FDKOD_OK;
}

fdkod_status fdkod_batch_info(fdkod_batch_t b, int64_t* items, int32_t* blocks, int64_t* updates_eq) {
    if (!b) return fail(FDKOD_E_ARG, "batch is NULL");
    if (items) *items = b->nitems;
    if (blocks) *blocks = b->bp_blocks;
    if (updates_eq) *updates_eq = b->updates_eq;
    return FDKOD_OK;
}

}  // extern "C"
