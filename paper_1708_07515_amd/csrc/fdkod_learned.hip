// Host entry points of the learned decimation filter and its training step
// (forward correction, weight gradient, transpose of the backprojection,
// squared-error residual, AdamW).  Every call is asynchronous on the given
// stream and allocates nothing.
#include <cmath>

#include "plan.h"

using namespace fdkod;

namespace {

fdkod_status learned_check(const fdkod_plan_s* pl) {
    if (pl->s == 0) return fail(FDKOD_E_UNSUPPORTED, "the learned decimation needs s > 0");
    if (pl->cone)
        return fail(FDKOD_E_UNSUPPORTED, "the learned decimation corrects a decimation of detector rows");
    if (pl->wmax > kLearnedMaxWidth)
        return fail(FDKOD_E_UNSUPPORTED, "a square is wider than 252 local columns");
    return FDKOD_OK;
}

LearnedArgs learned_args(const fdkod_plan_s* pl, const void* filt, void* ws, const float* dws,
                         const uint16_t* w, float* grad, int nv) {
    LearnedArgs a;
    a.filt = filt;
    a.ws = ws;
    a.dws = dws;
    a.squares = pl->d_sq;
    a.grid = pl->d_grid;
    a.ac_p = pl->d_ac_p;
    a.w = w;
    a.grad = grad;
    a.partials = pl->d_lpartials;
    a.n = pl->n;
    a.p = pl->p;
    a.pd = pl->pd;
    a.nsq = pl->nsq;
    a.d = pl->d / 4 > 1 ? pl->d / 4 : 1;
    a.nv = nv;
    a.ntasks = pl->nsq * nv;
    a.cubic = pl->cubic;
    return a;
}

AdjArgs adjoint_args(const fdkod_plan_s* pl, const float* resid, float* dws, int v0, int nv, int zbase,
                     int nzs) {
    AdjArgs a;
    a.resid = resid;
    a.dws = dws;
    a.squares = pl->d_sq;
    a.grid = pl->d_grid;
    a.trig = pl->d_trig_m;
    a.tiles = pl->d_tiles;
    a.ntiles = pl->ntiles;
    a.n = pl->n;
    a.nz = nzs;
    a.pd = pl->pd;
    a.v0 = v0;
    a.nv = nv;
    a.zbase = zbase;
    a.r = (float)pl->r;
    a.cu = (float)((pl->n - 1) / 2.0);
    a.cv = a.cu;
    a.cz = (float)((pl->nz - 1) / 2.0);
    a.scale = (float)(M_PI / pl->pd);
    a.ws_elems = pl->ws_row_elems * nv;
    a.nvox = (int64_t)nzs * pl->n * pl->n;
    // a voxel's weight (pi / P') U^-2 is largest at the least source
    // distance along the central ray, R - (N - 1) / sqrt(2); its four
    // bilinear shares sum to it.  Twice the product bounds every partial sum
    // of |contributions| per unit of max |resid|.
    const double umax = pl->r / (pl->r - (pl->n - 1) / std::sqrt(2.0));
    a.bound = 2.0 * (M_PI / pl->pd) * umax * umax * (double)a.nvox;
    a.qs = (AdjScale*)pl->d_adj;
    a.dq = (unsigned long long*)((char*)pl->d_adj + 256);
    return a;
}

// the adjoint's scale block and int64 sums for elems workspace elements
fdkod_status adjoint_buffer(fdkod_plan_s* pl, int64_t elems) {
    if (pl->d_adj && pl->adj_cap >= elems) return FDKOD_OK;
    int prev = 0;
    HIP_TRY(hipGetDevice(&prev), "hipGetDevice");
    HIP_TRY(hipSetDevice(pl->device), "hipSetDevice");
    if (pl->d_adj) {
        (void)hipFree(pl->d_adj);          // waits for the work that used it
        pl->d_adj = nullptr;
        pl->adj_cap = 0;
    }
    std::vector<void*> tmp;
    const fdkod_status st = dev_alloc(tmp, &pl->d_adj, 256 + sizeof(int64_t) * (size_t)elems);
    (void)hipSetDevice(prev);
    if (st != FDKOD_OK) {
        pl->d_adj = nullptr;
        return st;
    }
    pl->adj_cap = elems;
    return FDKOD_OK;
}

fdkod_status adjoint_check(const fdkod_plan_s* pl) {
    if (pl->s == 0) return fail(FDKOD_E_UNSUPPORTED, "the adjoint is defined for s > 0");
    if (pl->cone)
        return fail(FDKOD_E_UNSUPPORTED, "the adjoint samples detector rows, not cone-corrected rows");
    return FDKOD_OK;
}

}  // namespace

extern "C" {

fdkod_status fdkod_learned_decompose(fdkod_plan_t pl, const void* filt, void* ws, const uint16_t* weights,
                                     fdkod_stream_t stream) {
    if (!pl || !filt || !ws || !weights) return fail(FDKOD_E_ARG, "NULL argument");
    fdkod_status st = learned_check(pl);
    if (st != FDKOD_OK) return st;
    if ((st = fdkod_decompose(pl, filt, ws, stream)) != FDKOD_OK) return st;
    const LearnedArgs a = learned_args(pl, filt, ws, nullptr, weights, nullptr, pl->n);
    HIP_TRY(launch_learned_fwd(a, pl->wmax, pl->d, pl->store, (hipStream_t)stream),
            "learned decimation kernel launch");
    return FDKOD_OK;
}

fdkod_status fdkod_learned_decompose_band(fdkod_plan_t pl, const void* filt_band, int32_t v0, int32_t nrows,
                                          void* ws_band, const uint16_t* weights, fdkod_stream_t stream) {
    if (!pl || !filt_band || !ws_band || !weights) return fail(FDKOD_E_ARG, "NULL argument");
    fdkod_status st = learned_check(pl);
    if (st != FDKOD_OK) return st;
    if ((st = check_band(pl, v0, nrows)) != FDKOD_OK) return st;
    if ((st = fdkod_decompose_band(pl, filt_band, v0, nrows, ws_band, stream)) != FDKOD_OK) return st;
    const LearnedArgs a = learned_args(pl, filt_band, ws_band, nullptr, weights, nullptr, nrows);
    HIP_TRY(launch_learned_fwd(a, pl->wmax, pl->d, pl->store, (hipStream_t)stream),
            "learned decimation kernel launch");
    return FDKOD_OK;
}

fdkod_status fdkod_learned_backward(fdkod_plan_t pl, const void* filt, const float* dws,
                                    const uint16_t* weights, float* grad, fdkod_stream_t stream) {
    if (!pl || !filt || !dws || !weights || !grad) return fail(FDKOD_E_ARG, "NULL argument");
    fdkod_status st = learned_check(pl);
    if (st != FDKOD_OK) return st;
    const LearnedArgs a = learned_args(pl, filt, nullptr, dws, weights, grad, pl->n);
    HIP_TRY(launch_learned_bwd(a, pl->store, (hipStream_t)stream), "learned gradient kernel launch");
    return FDKOD_OK;
}

fdkod_status fdkod_learned_backward_band(fdkod_plan_t pl, const void* filt_band, int32_t v0, int32_t nrows,
                                         const float* dws_band, const uint16_t* weights, float* grad,
                                         fdkod_stream_t stream) {
    if (!pl || !filt_band || !dws_band || !weights || !grad) return fail(FDKOD_E_ARG, "NULL argument");
    fdkod_status st = learned_check(pl);
    if (st != FDKOD_OK) return st;
    if ((st = check_band(pl, v0, nrows)) != FDKOD_OK) return st;
    const LearnedArgs a = learned_args(pl, filt_band, nullptr, dws_band, weights, grad, nrows);
    HIP_TRY(launch_learned_bwd(a, pl->store, (hipStream_t)stream), "learned gradient kernel launch");
    return FDKOD_OK;
}

fdkod_status fdkod_reconstruct_adjoint(fdkod_plan_t pl, const float* resid, float* dws,
                                       fdkod_stream_t stream) {
    if (!pl || !resid || !dws) return fail(FDKOD_E_ARG, "NULL argument");
    fdkod_status st = adjoint_check(pl);
    if (st != FDKOD_OK) return st;
    if ((st = adjoint_buffer(pl, pl->ws_row_elems * pl->n)) != FDKOD_OK) return st;
    const AdjArgs a = adjoint_args(pl, resid, dws, 0, pl->n, 0, pl->nz);
    HIP_TRY(launch_bp_adjoint(a, (hipStream_t)stream), "adjoint kernel launch");
    return FDKOD_OK;
}

fdkod_status fdkod_reconstruct_adjoint_slab(fdkod_plan_t pl, const float* resid_slab, int32_t v0, int32_t nrows,
                                            int32_t z0, int32_t nzs, float* dws_band, fdkod_stream_t stream) {
    if (!pl || !resid_slab || !dws_band) return fail(FDKOD_E_ARG, "NULL argument");
    fdkod_status st = adjoint_check(pl);
    if (st != FDKOD_OK) return st;
    if ((st = check_band(pl, v0, nrows)) != FDKOD_OK) return st;
    if ((st = check_slab(pl, v0, nrows, z0, nzs)) != FDKOD_OK) return st;
    if ((st = adjoint_buffer(pl, pl->ws_row_elems * nrows)) != FDKOD_OK) return st;
    const AdjArgs a = adjoint_args(pl, resid_slab, dws_band, v0, nrows, z0, nzs);
    HIP_TRY(launch_bp_adjoint(a, (hipStream_t)stream), "adjoint kernel launch");
    return FDKOD_OK;
}

fdkod_status fdkod_sq_residual(const float* f, const float* ref, float* resid, double* loss, int64_t count,
                               fdkod_stream_t stream) {
    if (!f || !ref || !resid || !loss) return fail(FDKOD_E_ARG, "NULL argument");
    if (count < 0) return fail(FDKOD_E_ARG, "negative count");
    HIP_TRY(launch_residual(f, ref, resid, loss, count, 1.0f, (hipStream_t)stream), "residual kernel launch");
    return FDKOD_OK;
}

fdkod_status fdkod_sq_residual_weighted(const float* f, const float* ref, float* resid, double* loss, int64_t count,
                                        float weight, fdkod_stream_t stream) {
    if (!f || !ref || !resid || !loss) return fail(FDKOD_E_ARG, "NULL argument");
    if (count < 0 || !(weight >= 0.0f)) return fail(FDKOD_E_ARG, "negative count or weight");
    HIP_TRY(launch_residual(f, ref, resid, loss, count, weight, (hipStream_t)stream), "residual kernel launch");
    return FDKOD_OK;
}

fdkod_status fdkod_adamw_step(float* master, float* m1, float* m2, const float* grad, uint16_t* w_bf16,
                              int32_t count, int32_t step, float lr, float beta1, float beta2, float eps,
                              float weight_decay, fdkod_stream_t stream) {
    if (!master || !m1 || !m2 || !grad || !w_bf16) return fail(FDKOD_E_ARG, "NULL argument");
    if (count <= 0 || step <= 0) return fail(FDKOD_E_ARG, "count and step must be positive");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && lr >= 0.0f))
        return fail(FDKOD_E_ARG, "invalid AdamW hyper-parameters");
    AdamArgs a;
    a.master = master;
    a.m1 = m1;
    a.m2 = m2;
    a.grad = grad;
    a.w_bf16 = w_bf16;
    a.count = count;
    a.step = step;
    a.lr = lr;
    a.beta1 = beta1;
    a.beta2 = beta2;
    a.eps = eps;
    a.weight_decay = weight_decay;
    HIP_TRY(launch_adamw(a, (hipStream_t)stream), "AdamW kernel launch");
    return FDKOD_OK;
}

}  // extern "C"
