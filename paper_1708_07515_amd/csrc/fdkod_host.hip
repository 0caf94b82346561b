// Host side of the C ABI declared in include/fdkod.h: parameter validation,
// plan tables (built in FP64, stored in FP32), workspace layout, kernel
// variant choice, the autotuner and launch sequencing for one plan.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "fdkod.h"
#include "internal.h"
#include "dtype.h"
#include "plan.h"

using namespace fdkod;

namespace fdkod {

thread_local std::string g_last_error;

fdkod_status fail(fdkod_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

fdkod_status hip_fail(hipError_t e, const char* what) {
    return fail(FDKOD_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

fdkod_status dev_alloc(std::vector<void*>& owner, void** ptr, size_t bytes) {
    if (std::getenv("FDKOD_FAULT") && std::strcmp(std::getenv("FDKOD_FAULT"), "nomem") == 0)
        return fail(FDKOD_E_NOMEM, "allocation refused (FDKOD_FAULT=nomem)");
    hipError_t e = hipMalloc(ptr, bytes ? bytes : 1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FDKOD_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    owner.push_back(*ptr);
    return FDKOD_OK;
}

}  // namespace fdkod

namespace {

int64_t floordiv(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

int64_t ceildiv(int64_t a, int64_t b) { return -floordiv(-a, b); }

// Windows a projection can feed: the decimation window's length in decimated
// steps (2 for the triangle; the windowed sinc's taps, 4 by default).
int window_taps(const fdkod_params& q) {
    if (q.decim == FDKOD_DECIM_SINC) return q.taps ? q.taps : 4;
    return 2;
}

// Near-equal contiguous blocks of [0, n), larger blocks first.
std::vector<std::pair<int, int>> blocks(int n, int parts) {
    std::vector<std::pair<int, int>> out;
    int base = n / parts, extra = n % parts, start = 0;
    for (int k = 0; k < parts; ++k) {
        int size = base + (k < extra ? 1 : 0);
        out.emplace_back(start, start + size);
        start += size;
    }
    return out;
}

// Decimation schedule: a single walk over the extended projection index
// p_ext = lo(0) .. P - 1 that feeds the triangle windows of the decimated
// angles in order.  Window m holds the p_ext with |p_ext P' - m P| < P and
// weights (P - |p_ext P' - m P|) / sum; integers keep the support exact.
// Weights of the decimation windows in walk order.  Window m covers the
// (unwrapped) projections pe with |pe P' - m P| < (taps / 2) P, i.e. within
// taps / 2 decimated steps of beta'_m; the walk runs from window 0's first
// projection to window P'-1's last, and at every projection the windows
// cur .. cur + taps - 1 are the only ones open (window cur + taps opens after
// window cur closes).  Step weights for windows cur and cur + 1 go in the
// step itself, those of windows cur + 2 .. into `wext` (taps - 2 per step).
// Triangle: P - |pe P' - m P| (integers, exact); windowed sinc:
// sinc(t) (1 + cos(2 pi t / taps)) / 2 with t = |pe P' - m P| / P.  Both are
// normalised per window in FP64.
struct Schedule {
    std::vector<DecimStep> steps;
    std::vector<float> wext;
};

Schedule build_schedule(int P, int pd, int taps, bool sinc) {
    const int64_t h = taps / 2;
    auto lo = [&](int64_t m) { return floordiv(m * P - h * P, pd) + 1; };
    auto hi = [&](int64_t m) { return ceildiv(m * P + h * P, pd) - 1; };
    auto weight = [&](int64_t m, int64_t pe) -> double {
        const int64_t e = std::llabs(pe * pd - m * P);
        if (!sinc) return (double)((int64_t)P - e);
        const double t = (double)e / (double)P;
        const double sc = e == 0 ? 1.0 : std::sin(M_PI * t) / (M_PI * t);
        return sc * 0.5 * (1.0 + std::cos(2.0 * M_PI * t / (double)taps));
    };
    std::vector<double> sum(pd, 0.0);
    for (int m = 0; m < pd; ++m)
        for (int64_t pe = lo(m); pe <= hi(m); ++pe) sum[m] += weight(m, pe);
    auto w_of = [&](int64_t m, int64_t pe) -> float {
        return (m < pd && pe >= lo(m) && pe <= hi(m)) ? (float)(weight(m, pe) / sum[m]) : 0.0f;
    };
    Schedule out;
    int cur = 0;
    for (int64_t pe = lo(0); pe <= hi(pd - 1); ++pe) {
        DecimStep st;
        st.p = (int)(((pe % P) + P) % P);
        st.w0 = w_of(cur, pe);
        st.w1 = w_of(cur + 1, pe);
        for (int i = 2; i < taps; ++i) out.wext.push_back(w_of(cur + i, pe));
        st.emit = (pe == hi(cur)) ? 1 : 0;
        out.steps.push_back(st);
        if (st.emit) ++cur;
    }
    return out;
}

}  // namespace

namespace {

template <class T>
fdkod_status upload(fdkod_plan_t pl, T** dptr, const std::vector<T>& h) {
    fdkod_status st = dev_alloc(pl->allocs, (void**)dptr, h.size() * sizeof(T));
    if (st != FDKOD_OK) return st;
    if (!h.empty()) HIP_TRY(hipMemcpy(*dptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice),
                            "hipMemcpy");
    return FDKOD_OK;
}

void release(fdkod_plan_t pl) {
    if (!pl) return;
    int prev = 0;
    if (hipGetDevice(&prev) == hipSuccess) {
        (void)hipSetDevice(pl->device);
        for (void* p : pl->allocs) (void)hipFree(p);
        if (pl->d_adj) (void)hipFree(pl->d_adj);
        (void)hipSetDevice(prev);
    }
    delete pl;
}

std::vector<float2> trig_table(int count) {
    std::vector<float2> t(count);
    for (int i = 0; i < count; ++i) {
        double b = 2.0 * M_PI * (double)i / (double)count;
        t[i] = make_float2((float)std::cos(b), (float)std::sin(b));
    }
    return t;
}

// In-place radix-2 FFT in FP64 (host tables only), sign -1.
void fft64(std::vector<double>& re, std::vector<double>& im) {
    const size_t m = re.size();
    for (size_t i = 1, j = 0; i < m; ++i) {
        size_t bit = m >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            std::swap(re[i], re[j]);
            std::swap(im[i], im[j]);
        }
    }
    for (size_t len = 2; len <= m; len <<= 1) {
        const double ang = -2.0 * M_PI / (double)len;
        for (size_t i = 0; i < m; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const double wr = std::cos(ang * k), wi = std::sin(ang * k);
                const size_t a = i + k, b = i + k + len / 2;
                const double xr = re[b] * wr - im[b] * wi, xi = re[b] * wi + im[b] * wr;
                re[b] = re[a] - xr;
                im[b] = im[a] - xi;
                re[a] += xr;
                im[a] += xi;
            }
    }
}

// Running sum of the Ram-Lak kernel, g[n] = sum_{k <= n} h[k], FP64, for
// n in [-lim, lim].  With T(m) = sum_{k >= m, k odd} 1/k^2:
// g[n] = T(n+1)/pi^2 for n >= 0 and g[n] = -T(-n)/pi^2 for n < 0
// (the kernel sums to zero, h is even, h[0] = 1/4, h[odd k] = -1/(pi^2 k^2)).
std::vector<double> ramlak_running_sum(int lim) {
    const int64_t kmax = ((int64_t)1 << 22) + 1;     // odd
    // tail sum_{j >= 0} 1/(K + 2j)^2 by Euler-Maclaurin, error O(K^-5)
    const double kk = (double)kmax;
    double tail = 1.0 / (2.0 * kk) + 1.0 / (2.0 * kk * kk) + 1.0 / (3.0 * kk * kk * kk);
    std::vector<double> t(lim + 2, 0.0);             // t[m] = T(m), m in [1, lim + 1]
    double acc = tail;
    for (int64_t k = kmax - 2; k >= 1; k -= 2) {
        acc += 1.0 / ((double)k * (double)k);
        if (k <= lim + 1) t[k] = acc;
        if (k + 1 <= lim + 1) t[k + 1] = acc - 1.0 / ((double)k * (double)k);
    }
    std::vector<double> g(2 * lim + 1);
    for (int n = -lim; n <= lim; ++n)
        g[n + lim] = n >= 0 ? t[n + 1] / (M_PI * M_PI) : -t[-n] / (M_PI * M_PI);
    return g;
}

// Filter tables: the DFT of the circularly wrapped running-sum kernel g
// divided by M, the tail g[u - N] for the last difference, and the FFT
// twiddles exp(-2 pi i k / M).
void ramp_tables(int n, int m, std::vector<float2>& resp, std::vector<float>& gtail,
                 std::vector<float2>& tw) {
    const std::vector<double> g = ramlak_running_sum(m);
    auto gat = [&](int lag) { return g[lag + m]; };
    std::vector<double> re(m), im(m, 0.0);
    for (int t = 0; t < m; ++t) re[t] = gat(t <= m / 2 ? t : t - m);
    fft64(re, im);
    resp.resize(m);
    tw.resize(m);
    for (int k = 0; k < m; ++k) {
        resp[k] = make_float2((float)(re[k] / m), (float)(im[k] / m));
        tw[k] = make_float2((float)std::cos(2.0 * M_PI * k / m), (float)-std::sin(2.0 * M_PI * k / m));
    }
    gtail.resize(n);
    for (int u = 0; u < n; ++u) gtail[u] = (float)gat(u - n);
}


}  // namespace

namespace fdkod {

// Choose the backprojection LDS footprint (TW x TH samples) that holds the
// footprint of a 16 x 16 x zrun voxel block at any angle, from the slice's
// smallest depth Dmin = R - (N-1)/sqrt(2).
bool bp_tiles_for(int n, int nz, double r, int zrun, int cone_side, int* tw, int* th) {
    const double c = (n - 1) / 2.0;
    const double dmin = r - c * std::sqrt(2.0);
    const double mag = r / dmin;
    const double lat = c * std::sqrt(2.0) / dmin;
    const double diag = (kTileXY - 1) * std::sqrt(2.0);
    const double span_c = diag * mag * std::sqrt(1.0 + lat * lat);
    const double zmax = (nz - 1) / 2.0 + zrun;     // runs may extend past the last slice
    // rows per slice: R / D (eq. (9)); on cone-corrected rows D_c / D, where
    // D_c <= D + h with h the square's half diagonal
    const double hd = cone_side * std::sqrt(0.5);
    const double rows_per_z = cone_side ? (dmin + hd) / dmin : mag;
    const double numer = cone_side ? dmin + hd : r;   // bounds R (or D_c) where D = dmin
    const double span_r = (zrun - 1) * rows_per_z + zmax * numer * diag / (dmin * dmin);
    const int need_c = (int)std::ceil(span_c + 1e-6) + 4;
    const int need_r = (int)std::ceil(span_r + 1e-6) + 4;
    *tw = need_c <= 32 ? 32 : (need_c <= 64 ? 64 : 0);
    *th = need_r <= 48 ? 48 : (need_r <= 64 ? 64 : (need_r <= 96 ? 96 : 0));
    return *tw && *th;
}


DecimVol decim_args(const fdkod_plan_s* pl, const void* filt, void* ws, int chunks) {
    return decim_args_band(pl, filt, ws, chunks, 0, pl->n);
}

DecimVol decim_args_band(const fdkod_plan_s* pl, const void* filt, void* ws, int chunks, int v0, int nv) {
    DecimVol a;
    a.filt = filt;
    a.ws = ws;
    a.squares = pl->d_sq;
    a.grid = pl->d_grid;
    a.crop = pl->d_crop;
    a.sched = pl->d_sched;
    a.rscale = pl->d_rscale;
    a.wext = pl->d_wext;
    a.nsched = pl->nsched;
    a.nw = pl->nw;
    a.cubic = pl->cubic;
    a.cone = pl->cone;
    a.cv = (float)((pl->n - 1) / 2.0);
    a.n = pl->n;
    a.p = pl->p;
    a.pd = pl->pd;
    a.nsq = pl->nsq;
    a.v0 = v0;
    a.nv = nv;
    const int ch = chunks > 0 ? chunks : 1;
    a.tasks_per_sq = dec_tasks_per_sq(pl->wmax, ch);
    const int rpt = decim_rows_per_task(pl->cone != 0, pl->cubic != 0, ch);
    a.ntasks = pl->nsq * ((nv + rpt - 1) / rpt) * a.tasks_per_sq;
    a.chunks = ch;
    a.bside = pl->s > 0 ? 1 << (pl->s - 1) : 0;
    a.blo = pl->d_blo;
    a.sqoff = pl->d_sqoff;
    return a;
}

fdkod_status enqueue_decimate(const fdkod_plan_s* pl, const void* filt, void* ws, int v0, int nv,
                              hipStream_t st) {
    const DecimVol a = decim_args_band(pl, filt, ws, pl->dec_chunks, v0, nv);
    if (pl->dec_chunks == 0) {
        HIP_TRY(launch_decimate_staged(a, pl->staged_cpt, pl->staged_segc, pl->store, st),
                "row-staged decimation kernel launch");
    } else {
        HIP_TRY(launch_decimate(a, pl->dec_chunks, pl->store, st), "decimate kernel launch");
    }
    return FDKOD_OK;
}

BoundsArgs bounds_args(const fdkod_plan_s* pl) {
    BoundsArgs a;
    a.squares = pl->d_sq;
    a.trig_p = pl->d_trig_p;
    a.trig_m = pl->d_trig_m;
    a.ac_p = pl->d_ac_p;
    a.geo_m = pl->d_geo_m;
    a.grid = pl->d_grid;
    a.sched = pl->d_sched;
    a.crop = pl->d_crop;
    a.rscale = pl->d_rscale;
    a.n = pl->n;
    a.p = pl->p;
    a.pd = pl->pd;
    a.nsq = pl->nsq;
    a.nsched = pl->nsched;
    a.r = (float)pl->r;
    a.cu = (float)((pl->n - 1) / 2.0);
    return a;
}

FilterArgs filter_args(const fdkod_plan_s* pl, const float* proj, void* filt, int v0, int nv) {
    FilterArgs a;
    a.proj = proj;
    a.out = filt;
    a.resp = pl->d_resp;
    a.gtail = pl->d_gtail;
    a.twiddle = pl->d_tw;
    a.n = pl->n;
    a.rows = pl->p * nv;
    a.v0 = v0;
    a.nv = nv;
    a.r = (float)pl->r;
    a.c = (float)((pl->n - 1) / 2.0);
    return a;
}

// A variant is usable for a plan when it exists and its LDS footprint holds
// the plan's block footprint for its z run.
bool variant_holds(const fdkod_plan_s* pl, const BpVariant& v) {
    if (!backproject_variant_exists(v)) return false;
    int tw = 0, th = 0;
    if (!bp_tiles_for(pl->n, pl->nz, pl->r, v.zrun, cone_side(pl), &tw, &th)) return false;
    return v.tile_w >= tw && v.tile_h >= th;
}

BpVol bp_vol(const fdkod_plan_s* pl, const void* filt, const void* ws, float* vol) {
    return bp_vol_band(pl, filt, ws, vol, 0, pl->n, 0, pl->nz);
}

BpVol bp_vol_band(const fdkod_plan_s* pl, const void* filt, const void* ws, float* vol, int v0, int nv,
                  int zbase, int nzs) {
    const bool direct = pl->s == 0;
    BpVol v;
    v.data = direct ? filt : ws;
    v.vol = vol;
    v.squares = pl->d_sq;
    v.grid = direct ? pl->d_grid_direct : pl->d_grid;
    v.trig = pl->d_trig_m;
    v.n = pl->n;
    v.nz = nzs;
    v.pd = pl->pd;
    v.v0 = v0;
    v.nv = nv;
    v.zbase = zbase;
    v.cone = pl->cone;
    v.row_stride_direct = direct ? pl->n : 0;
    v.r = (float)pl->r;
    v.cu = (float)((pl->n - 1) / 2.0);
    v.cv = v.cu;
    v.cz = (float)((pl->nz - 1) / 2.0);
    v.scale = (float)(M_PI / pl->pd);
    return v;
}

}  // namespace fdkod

namespace {

// Shape of the row-staged decimation for a plan, or none (staged_cpt = 0):
// it takes the paper's plain decimation (detector rows, triangle, linear
// shift) with s >= 1 and squares at most 256 columns wide.  A staged segment
// must hold, at every schedule step, every local column of the four squares
// of a 2 x 2 block from the least of their crop offsets: the spread of the
// offsets (read back from the bounds kernel's crop table) plus 64 cpt
// columns and the interpolation's second sample.
fdkod_status staged_shape(fdkod_plan_s* pl) {
    pl->staged_cpt = pl->staged_segc = 0;
    if (pl->s < 1 || pl->cone || pl->sinc || pl->cubic) return FDKOD_OK;
    int cpt = 1;
    while (cpt < 4 && 64 * cpt < pl->wmax) cpt <<= 1;
    if (64 * cpt < pl->wmax) return FDKOD_OK;
    std::vector<int2> crop((size_t)pl->nsq * pl->nsched);
    HIP_TRY(hipMemcpy(crop.data(), pl->d_crop, sizeof(int2) * crop.size(), hipMemcpyDeviceToHost),
            "hipMemcpy crop table");
    const int side = 1 << pl->s, bside = side / 2;
    std::vector<int> blo((size_t)bside * bside * pl->nsched);
    std::vector<int2> sqoff(crop.size());
    int spread = 0;
    for (int by = 0; by < bside; ++by)
        for (int bx = 0; bx < bside; ++bx) {
            const int q0 = (2 * by) * side + 2 * bx;
            const int qs[4] = {q0, q0 + 1, q0 + side, q0 + side + 1};
            for (int e = 0; e < pl->nsched; ++e) {
                int lo = crop[(size_t)qs[0] * pl->nsched + e].x, hi = lo;
                for (int i = 1; i < 4; ++i) {
                    const int o = crop[(size_t)qs[i] * pl->nsched + e].x;
                    lo = std::min(lo, o);
                    hi = std::max(hi, o);
                }
                spread = std::max(spread, hi - lo);
                blo[(size_t)(by * bside + bx) * pl->nsched + e] = lo;
                for (int i = 0; i < 4; ++i) {
                    const int2 c = crop[(size_t)qs[i] * pl->nsched + e];
                    sqoff[(size_t)qs[i] * pl->nsched + e] = make_int2(c.x - lo, c.y);
                }
            }
        }
    const int segc = (spread + 64 * cpt + 1 + 63) / 64;
    if (!staged_shape_exists(cpt, segc)) return FDKOD_OK;
    fdkod_status st = upload(pl, &pl->d_blo, blo);
    if (st == FDKOD_OK) st = upload(pl, &pl->d_sqoff, sqoff);
    if (st != FDKOD_OK) return st;
    pl->staged_cpt = cpt;
    pl->staged_segc = segc;
    return FDKOD_OK;
}

std::string tune_key(const fdkod_plan_s* pl) {
    std::ostringstream k;
    k << "gfx950 n=" << pl->n << " nz=" << pl->nz << " p=" << pl->p << " r=" << pl->r
      << " s=" << pl->s << " k=" << pl->k << " store=" << pl->store;
    if (pl->cone) k << " rows=cone";
    if (pl->sinc) k << " decim=sinc" << pl->nw;
    if (pl->cubic) k << " interp=cubic";
    return k.str();
}

// Last entry of the tuning cache file for this plan, if any.
bool tune_cache_lookup(const fdkod_plan_s* pl, BpVariant* v, int* chunks) {
    const char* path = std::getenv("FDKOD_TUNE_CACHE");
    if (!path || !*path) return false;
    std::ifstream f(path);
    if (!f) return false;
    const std::string key = tune_key(pl) + " :";
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        if (line.compare(0, key.size(), key) != 0) continue;
        std::istringstream in(line.substr(key.size()));
        BpVariant t{};
        int c = 0;
        if (in >> t.zrun >> t.tile_w >> t.tile_h >> t.g >> c) {
            *v = t;
            *chunks = c;
            found = true;
        }
    }
    return found;
}

void tune_cache_store(const fdkod_plan_s* pl) {
    const char* path = std::getenv("FDKOD_TUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream f(path, std::ios::app);
    if (!f) return;
    f << tune_key(pl) << " : " << pl->bpv.zrun << " " << pl->bpv.tile_w << " " << pl->bpv.tile_h
      << " " << pl->bpv.g << " " << pl->dec_chunks << "\n";
}

// Time `fn` on `st`: one warm-up, then the mean of `reps` runs (ms).
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

const char* fdkod_status_str(fdkod_status st) {
    switch (st) {
        case FDKOD_OK: return "ok";
        case FDKOD_E_ARG: return "invalid argument";
        case FDKOD_E_GEOMETRY: return "invalid geometry";
        case FDKOD_E_UNSUPPORTED: return "unsupported";
        case FDKOD_E_NOMEM: return "out of memory";
        case FDKOD_E_HIP: return "HIP runtime error";
        case FDKOD_E_STATE: return "invalid state";
    }
    return "unknown status";
}

const char* fdkod_last_error(void) { return fdkod::g_last_error.c_str(); }

int32_t fdkod_version(void) { return 100; }

fdkod_status fdkod_cost_counts(const fdkod_params* prm, int64_t* cropped, int64_t* updates) {
    fdkod_status st = fdkod_validate(prm);
    if (st != FDKOD_OK) return st;
    if (!cropped || !updates) return fail(FDKOD_E_ARG, "NULL argument");
    const int n = prm->n, nz = prm->nz ? prm->nz : prm->n, s = prm->s;
    const int d = 1 << (prm->s - prm->skip);
    const int pd = (int)ceildiv(prm->p, d);
    *updates = (int64_t)n * n * nz * (s == 0 ? prm->p : pd);
    *cropped = 0;
    if (s == 0) return FDKOD_OK;
    // the local grid of every square as the bounds kernel forms it, in FP64:
    // eq. (1) at the vertices relative to the centre trajectory, extremes over
    // the decimated angles
    const double c = (n - 1) / 2.0, r = prm->r;
    const auto bl = blocks(n, 1 << s);
    int64_t sum_w = 0;
    for (auto& by : bl)
        for (auto& bx : bl) {
            const double xc = 0.5 * ((bx.first - c) + (bx.second - 1 - c));
            const double yc = 0.5 * ((by.first - c) + (by.second - 1 - c));
            const double vx[2] = {bx.first - c, bx.second - 1 - c}, vy[2] = {by.first - c, by.second - 1 - c};
            double emin = 1e300, emax = -1e300;
            for (int m = 0; m < pd; ++m) {
                const double b = 2.0 * M_PI * m / pd, cs = std::cos(b), sn = std::sin(b);
                const double ac = r * (yc * cs - xc * sn) / (r + xc * cs + yc * sn);
                for (int k = 0; k < 4; ++k) {
                    const double x = vx[k & 1], y = vy[k >> 1];
                    const double e = r * (y * cs - x * sn) / (r + x * cs + y * sn) - ac;
                    emin = std::min(emin, e);
                    emax = std::max(emax, e);
                }
            }
            const int u0 = (int)std::floor(emin + c);
            sum_w += (int64_t)((int)std::floor(emax + c) - u0 + 2);
        }
    *cropped = sum_w * prm->p * n;
    return FDKOD_OK;
}

fdkod_status fdkod_choose_s(const fdkod_params* prm, int32_t s_max, double c1_ms, double c2_ms, int32_t* s_out,
                            double* ms_out) {
    if (!prm || !s_out) return fail(FDKOD_E_ARG, "NULL argument");
    if (!(c1_ms > 0.0) || !(c2_ms >= 0.0) || s_max < 0) return fail(FDKOD_E_ARG, "invalid cost constants or s_max");
    double best = 1e300;
    int best_s = -1;
    for (int s = 0; s <= s_max && (1 << s) <= prm->n; ++s) {
        fdkod_params q = *prm;
        q.s = s;
        q.skip = std::min(prm->skip, s);
        if (fdkod_validate(&q) != FDKOD_OK) continue;
        int64_t cropped = 0, updates = 0;
        fdkod_status st = fdkod_cost_counts(&q, &cropped, &updates);
        if (st != FDKOD_OK) return st;
        const double t = c1_ms * (double)updates + c2_ms * (double)cropped;
        if (t < best) {
            best = t;
            best_s = s;
        }
    }
    if (best_s < 0) return fail(FDKOD_E_GEOMETRY, "no valid s for these parameters");
    *s_out = best_s;
    if (ms_out) *ms_out = best;
    g_last_error.clear();
    return FDKOD_OK;
}

fdkod_status fdkod_check_counts(int64_t* counts, int32_t n, int32_t reset) {
    if (!counts || n < 1 || n > kCheckKinds) return fail(FDKOD_E_ARG, "counts must hold 1..4 values");
#ifdef FDKOD_CHECKS
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    unsigned long long sum[kCheckKinds] = {};
    HIP_TRY(checks_read_backproject(sum, reset != 0), "reading the backprojection's check counters");
    HIP_TRY(checks_read_decimate(sum, reset != 0), "reading the decimation's check counters");
    for (int k = 0; k < n; ++k) counts[k] = (int64_t)sum[k];
    return FDKOD_OK;
#else
    (void)reset;
    for (int k = 0; k < n; ++k) counts[k] = 0;
    return fail(FDKOD_E_UNSUPPORTED, "not a checked build (FDKOD_CHECKS undefined)");
#endif
}

fdkod_status fdkod_validate(const fdkod_params* prm) {
    if (!prm) return fail(FDKOD_E_ARG, "params is NULL");
    const fdkod_params& q = *prm;
    if (q.n < 2 || q.n > 4096) return fail(FDKOD_E_ARG, "n must be in [2, 4096]");
    if (q.nz < 0 || q.nz > 65536) return fail(FDKOD_E_ARG, "nz must be in [0, 65536]");
    if (q.p < 1 || q.p > 65536) return fail(FDKOD_E_ARG, "p must be in [1, 65536]");
    if (q.store < FDKOD_F32 || q.store > FDKOD_BF16) return fail(FDKOD_E_ARG, "unknown store type");
    if (q.decim != FDKOD_DECIM_TRIANGLE && q.decim != FDKOD_DECIM_SINC)
        return fail(FDKOD_E_ARG, "unknown decimation window");
    if (q.decim == FDKOD_DECIM_TRIANGLE && q.taps != 0 && q.taps != 2)
        return fail(FDKOD_E_ARG, "the triangle window has 2 taps");
    if (q.decim == FDKOD_DECIM_SINC && !(q.taps == 0 || q.taps == 2 || q.taps == 4 || q.taps == 6))
        return fail(FDKOD_E_ARG, "windowed-sinc taps must be 2, 4 or 6");
    if (q.rows != FDKOD_ROWS_DETECTOR && q.rows != FDKOD_ROWS_CONE) return fail(FDKOD_E_ARG, "unknown rows");
    if (q.interp != FDKOD_INTERP_LINEAR && q.interp != FDKOD_INTERP_CUBIC)
        return fail(FDKOD_E_ARG, "unknown interpolation");
    if (!std::isfinite(q.r)) return fail(FDKOD_E_GEOMETRY, "R is not finite");
    if (q.s < 0 || q.s > 12) return fail(FDKOD_E_GEOMETRY, "s must be in [0, 12]");
    if ((1 << q.s) > q.n) return fail(FDKOD_E_GEOMETRY, "2^s exceeds N");
    if (q.skip < 0 || q.skip > q.s) return fail(FDKOD_E_GEOMETRY, "skip must be in [0, s]");
    if (!(q.r > (q.n - 1) / std::sqrt(2.0)))
        return fail(FDKOD_E_GEOMETRY, "R must exceed (N-1)/sqrt(2) (eq. (1) denominator)");
    const int d = 1 << (q.s - q.skip);
    if (d > 1 && q.p < 2 * d) return fail(FDKOD_E_GEOMETRY, "decimation needs P >= 2 D");
    if (d > 1 && q.p < window_taps(q) * d)
        return fail(FDKOD_E_GEOMETRY, "the windowed sinc needs P >= taps * D");
    return FDKOD_OK;
}

fdkod_status fdkod_plan_create(const fdkod_params* prm, int device, fdkod_plan_t* out) {
    if (!out) return fail(FDKOD_E_ARG, "out is NULL");
    *out = nullptr;
    fdkod_status st = fdkod_validate(prm);
    if (st != FDKOD_OK) return st;

    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(FDKOD_E_ARG, "device out of range");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(FDKOD_E_UNSUPPORTED, std::string("device is ") + prop.gcnArchName + ", not gfx950");
    int prev = 0;
    HIP_TRY(hipGetDevice(&prev), "hipGetDevice");
    HIP_TRY(hipSetDevice(device), "hipSetDevice");

    fdkod_plan_t pl = new fdkod_plan_s();
    pl->prm = *prm;
    pl->device = device;
    pl->n = prm->n;
    pl->nz = prm->nz ? prm->nz : prm->n;
    pl->p = prm->p;
    pl->r = prm->r;
    pl->s = prm->s;
    pl->k = prm->skip;
    pl->d = 1 << (prm->s - prm->skip);
    pl->pd = (int)ceildiv(pl->p, pl->d);
    pl->nsq = 1 << (2 * pl->s);
    pl->store = prm->store;
    pl->cone = prm->rows == FDKOD_ROWS_CONE && prm->s > 0;
    pl->sinc = prm->decim == FDKOD_DECIM_SINC;
    pl->nw = window_taps(*prm);
    pl->cubic = prm->interp == FDKOD_INTERP_CUBIC;
    {
        // the FFT length: the least power of two (at least 8) holding the
        // linear convolution, so N <= M / 2, which the filter kernel's pruned
        // first and last stages rely on
        int m = 8;
        while (m < 2 * pl->n - 1) m <<= 1;
        pl->logm = 0;
        while ((1 << pl->logm) < m) ++pl->logm;
    }

    auto bail = [&](fdkod_status code) {
        release(pl);
        (void)hipSetDevice(prev);
        return code;
    };

    // squares (Sec. 2.1): vertex-mean centres in voxel coordinates
    const double c = (pl->n - 1) / 2.0;
    const auto bl = blocks(pl->n, 1 << pl->s);
    for (auto& by : bl)
        for (auto& bx : bl) {
            SquareDesc d{};
            d.x0 = bx.first; d.x1 = bx.second; d.y0 = by.first; d.y1 = by.second;
            d.xc = (float)(0.5 * ((bx.first - c) + (bx.second - 1 - c)));
            d.yc = (float)(0.5 * ((by.first - c) + (by.second - 1 - c)));
            d.y_off_row = 0;
            pl->sq.push_back(d);
        }

    // tables
    const std::vector<float2> trig_p = trig_table(pl->p);
    const std::vector<float2> trig_m = trig_table(pl->pd);
    std::vector<float2> resp, tw;
    std::vector<float> gtail;
    ramp_tables(pl->n, 1 << pl->logm, resp, gtail, tw);
    Schedule schedule = build_schedule(pl->p, pl->pd, pl->nw, pl->sinc != 0);
    std::vector<DecimStep>& sched = schedule.steps;
    while (sched.size() % kDecimUnroll) {
        sched.push_back(DecimStep{0, 0, 0.0f, 0.0f});
        for (int i = 2; i < pl->nw; ++i) schedule.wext.push_back(0.0f);
    }
    pl->nsched = (int)sched.size();
    {
        int emits = 0;
        for (const DecimStep& st_ : sched) emits += st_.emit;
        if (emits != pl->pd) return bail(fail(FDKOD_E_GEOMETRY, "decimation schedule does not close every window"));
    }

    if ((st = upload(pl, &pl->d_sq, pl->sq)) != FDKOD_OK) return bail(st);
    if ((st = upload(pl, &pl->d_trig_p, trig_p)) != FDKOD_OK) return bail(st);
    if ((st = upload(pl, &pl->d_trig_m, trig_m)) != FDKOD_OK) return bail(st);
    if ((st = upload(pl, &pl->d_resp, resp)) != FDKOD_OK) return bail(st);
    if ((st = upload(pl, &pl->d_gtail, gtail)) != FDKOD_OK) return bail(st);
    if ((st = upload(pl, &pl->d_tw, tw)) != FDKOD_OK) return bail(st);
    if ((st = upload(pl, &pl->d_sched, sched)) != FDKOD_OK) return bail(st);
    if (pl->nw > 2 && (st = upload(pl, &pl->d_wext, schedule.wext)) != FDKOD_OK) return bail(st);
    if ((st = upload(pl, &pl->d_grid_direct, std::vector<int2>{make_int2(0, pl->n)})) != FDKOD_OK)
        return bail(st);
    if ((st = dev_alloc(pl->allocs, (void**)&pl->d_ac_p, sizeof(float) * (size_t)pl->nsq * pl->p)) != FDKOD_OK)
        return bail(st);
    if ((st = dev_alloc(pl->allocs, (void**)&pl->d_geo_m, sizeof(float4) * (size_t)pl->nsq * pl->pd)) != FDKOD_OK)
        return bail(st);
    if ((st = dev_alloc(pl->allocs, (void**)&pl->d_crop, sizeof(int2) * (size_t)pl->nsq * pl->nsched)) != FDKOD_OK)
        return bail(st);
    if ((st = dev_alloc(pl->allocs, (void**)&pl->d_grid, sizeof(int2) * (size_t)pl->nsq)) != FDKOD_OK)
        return bail(st);
    if (pl->cone &&
        (st = dev_alloc(pl->allocs, (void**)&pl->d_rscale, sizeof(float) * (size_t)pl->nsq * pl->nsched)) != FDKOD_OK)
        return bail(st);

    // bounds kernel, then one synchronisation to lay out the workspace
    if ((st = fdkod_bounds(pl, nullptr)) != FDKOD_OK) return bail(st);
    {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return bail(hip_fail(e, "bounds kernel"));
    }
    pl->grid.resize(pl->nsq);
    {
        hipError_t e = hipMemcpy(pl->grid.data(), pl->d_grid, sizeof(int2) * pl->nsq, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return bail(hip_fail(e, "hipMemcpy grid"));
    }
    int64_t off = 0;
    pl->wmax = 0;
    for (int q = 0; q < pl->nsq; ++q) {
        const int w = pl->grid[q].y;
        if (w < 2 || w > 4 * pl->n + 8) return bail(fail(FDKOD_E_HIP, "bounds kernel produced an invalid width"));
        pl->wmax = std::max(pl->wmax, w);
        pl->sq[q].y_off_row = off;
        off += (int64_t)w * pl->pd;
    }
    pl->ws_row_elems = pl->s > 0 ? off : 0;
    pl->ws_elems = pl->ws_row_elems * pl->n;
    {
        hipError_t e = hipMemcpy(pl->d_sq, pl->sq.data(), sizeof(SquareDesc) * pl->nsq, hipMemcpyHostToDevice);
        if (e != hipSuccess) return bail(hip_fail(e, "hipMemcpy squares"));
    }

    // default kernel shapes: the row-staged decimation where it applies (the
    // paper's plain decimation), else 64 * chunks local columns per
    // decimation wavefront (the smallest power of two covering the widest
    // square, at most 8); the longest z run whose block footprint fits an LDS
    // tile, one angle per stage
    if ((st = staged_shape(pl)) != FDKOD_OK) return bail(st);
    int ch = 1;
    while (ch < max_chunks(pl) && 64 * ch < pl->wmax) ch <<= 1;
    pl->dec_chunks = pl->staged_cpt ? 0 : ch;
    pl->bp_ok = false;
    for (int zr : {32, 16, 64}) {
        int tw = 0, th = 0;
        // one angle per stage: the smallest LDS footprint, the highest occupancy
        if (bp_tiles_for(pl->n, pl->nz, pl->r, zr, cone_side(pl), &tw, &th) &&
            backproject_variant_exists(BpVariant{zr, tw, th, 1})) {
            pl->bpv = BpVariant{zr, tw, th, 1};
            pl->bp_ok = true;
            break;
        }
    }
    {
        BpVariant cv{};
        int cc = 0;
        if (pl->bp_ok && tune_cache_lookup(pl, &cv, &cc) && variant_holds(pl, cv) &&
            ((cc == 0 && pl->staged_cpt) || cc == 1 || cc == 2 || cc == 4 || cc == 8) && cc <= max_chunks(pl)) {
            pl->bpv = cv;
            pl->dec_chunks = cc;
        }
    }
    std::vector<BpTile> tiles;
    for (int q = 0; q < pl->nsq; ++q) {
        const SquareDesc& d = pl->sq[q];
        for (int y = d.y0; y < d.y1; y += kTileXY)
            for (int x = d.x0; x < d.x1; x += kTileXY) tiles.push_back(BpTile{q, x, y, 0});
    }
    pl->ntiles = (int)tiles.size();
    if ((int64_t)pl->ntiles * bp_zslabs(pl->nz, 16) > (int64_t)1 << 30)
        return bail(fail(FDKOD_E_UNSUPPORTED, "volume too large for one launch"));
    if ((st = upload(pl, &pl->d_tiles, tiles)) != FDKOD_OK) return bail(st);
    // the learned filter's backward pass sums its workgroups' partial
    // gradients in a fixed order (a plan the filter applies to only)
    if (pl->s > 0 && !pl->cone && pl->wmax <= kLearnedMaxWidth &&
        (st = dev_alloc(pl->allocs, (void**)&pl->d_lpartials,
                        sizeof(float) * (size_t)kLearnedBwdGrid * kLearnedParams)) != FDKOD_OK)
        return bail(st);

    (void)hipSetDevice(prev);
    *out = pl;
    return FDKOD_OK;
}

fdkod_status fdkod_plan_destroy(fdkod_plan_t plan) {
    release(plan);
    return FDKOD_OK;
}

fdkod_status fdkod_plan_info(fdkod_plan_t pl, fdkod_info* info) {
    if (!pl || !info) return fail(FDKOD_E_ARG, "NULL argument");
    info->squares = pl->nsq;
    info->p_dec = pl->pd;
    info->d = pl->d;
    info->fft_len = 1 << pl->logm;
    info->max_width = pl->wmax;
    info->z_run = pl->bpv.zrun;
    info->filtered_bytes = (int64_t)pl->p * pl->n * pl->n * store_bytes(pl->store);
    info->workspace_bytes = pl->ws_elems * store_bytes(pl->store);
    info->volume_bytes = (int64_t)pl->nz * pl->n * pl->n * 4;
    info->updates = (int64_t)pl->n * pl->n * pl->nz * pl->pd;
    return FDKOD_OK;
}

fdkod_status fdkod_bounds(fdkod_plan_t pl, fdkod_stream_t stream) {
    if (!pl) return fail(FDKOD_E_ARG, "plan is NULL");
    HIP_TRY(launch_bounds(bounds_args(pl), (hipStream_t)stream), "bounds kernel launch");
    return FDKOD_OK;
}

fdkod_status fdkod_filter(fdkod_plan_t pl, const float* proj, void* filt, fdkod_stream_t stream) {
    if (!pl || !proj || !filt) return fail(FDKOD_E_ARG, "NULL argument");
    const FilterArgs a = filter_args(pl, proj, filt, 0, pl->n);
    HIP_TRY(launch_filter(a, pl->logm, pl->store, (hipStream_t)stream), "filter kernel launch");
    return FDKOD_OK;
}

fdkod_status fdkod_decompose(fdkod_plan_t pl, const void* filt, void* ws, fdkod_stream_t stream) {
    if (!pl || !filt) return fail(FDKOD_E_ARG, "NULL argument");
    if (pl->s == 0) return FDKOD_OK;
    if (!ws) return fail(FDKOD_E_ARG, "workspace is NULL");
    return enqueue_decimate(pl, filt, ws, 0, pl->n, (hipStream_t)stream);
}

fdkod_status fdkod_reconstruct(fdkod_plan_t pl, const void* filt, const void* ws, float* vol,
                               fdkod_stream_t stream) {
    if (!pl || !vol) return fail(FDKOD_E_ARG, "NULL argument");
    const bool direct = pl->s == 0;
    if (direct && !filt) return fail(FDKOD_E_ARG, "filtered projections are NULL");
    if (!direct && !ws) return fail(FDKOD_E_ARG, "workspace is NULL");
    if (!pl->bp_ok)
        return fail(FDKOD_E_UNSUPPORTED, "R too small: a block's detector footprint exceeds 64 x 64");
    BpArgs a;
    a.v = bp_vol(pl, filt, ws, vol);
    a.tiles = pl->d_tiles;
    a.ntiles = pl->ntiles;
    a.nzt = bp_zslabs(pl->nz, pl->bpv.zrun);
    a.nlogical = a.ntiles * a.nzt;
    a.chunk = (a.nlogical + 7) / 8;
    HIP_TRY(launch_backproject(a, pl->bpv, pl->store, (hipStream_t)stream), "backprojection kernel launch");
    return FDKOD_OK;
}

fdkod_status fdkod_backproject(fdkod_plan_t pl, const void* filt, float* vol, void* ws,
                               fdkod_stream_t stream) {
    fdkod_status st = fdkod_decompose(pl, filt, ws, stream);
    if (st != FDKOD_OK) return st;
    return fdkod_reconstruct(pl, filt, ws, vol, stream);
}

fdkod_status fdkod_get_bounds(fdkod_plan_t pl, float* ac_p, float* ac_m, float* amin_m, float* amax_m,
                              int32_t* u0, int32_t* width, int32_t* rect) {
    if (!pl) return fail(FDKOD_E_ARG, "plan is NULL");
    int prev = 0;
    HIP_TRY(hipGetDevice(&prev), "hipGetDevice");
    HIP_TRY(hipSetDevice(pl->device), "hipSetDevice");
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (ac_p)
        HIP_TRY(hipMemcpy(ac_p, pl->d_ac_p, sizeof(float) * (size_t)pl->nsq * pl->p, hipMemcpyDeviceToHost),
                "hipMemcpy ac_p");
    if (ac_m || amin_m || amax_m) {
        std::vector<float4> geo((size_t)pl->nsq * pl->pd);
        HIP_TRY(hipMemcpy(geo.data(), pl->d_geo_m, sizeof(float4) * geo.size(), hipMemcpyDeviceToHost),
                "hipMemcpy geo");
        for (size_t i = 0; i < geo.size(); ++i) {
            if (ac_m) ac_m[i] = geo[i].x;
            if (amin_m) amin_m[i] = geo[i].y;
            if (amax_m) amax_m[i] = geo[i].z;
        }
    }
    std::vector<int2> g(pl->nsq);
    HIP_TRY(hipMemcpy(g.data(), pl->d_grid, sizeof(int2) * pl->nsq, hipMemcpyDeviceToHost), "hipMemcpy grid");
    for (int q = 0; q < pl->nsq; ++q) {
        if (u0) u0[q] = g[q].x;
        if (width) width[q] = g[q].y;
        if (rect) {
            rect[4 * q + 0] = pl->sq[q].x0;
            rect[4 * q + 1] = pl->sq[q].x1;
            rect[4 * q + 2] = pl->sq[q].y0;
            rect[4 * q + 3] = pl->sq[q].y1;
        }
    }
    (void)hipSetDevice(prev);
    return FDKOD_OK;
}

fdkod_status fdkod_get_tuning(fdkod_plan_t pl, fdkod_tuning* out) {
    if (!pl || !out) return fail(FDKOD_E_ARG, "NULL argument");
    out->z_run = pl->bpv.zrun;
    out->tile_w = pl->bpv.tile_w;
    out->tile_h = pl->bpv.tile_h;
    out->angles_per_stage = pl->bpv.g;
    out->decim_chunks = pl->dec_chunks;
    out->bp_ms = pl->tuned_bp_ms;
    out->decim_ms = pl->tuned_dec_ms;
    return FDKOD_OK;
}

fdkod_status fdkod_set_tuning(fdkod_plan_t pl, const fdkod_tuning* t) {
    if (!pl || !t) return fail(FDKOD_E_ARG, "NULL argument");
    const BpVariant v{t->z_run, t->tile_w, t->tile_h, t->angles_per_stage};
    if (!variant_holds(pl, v))
        return fail(FDKOD_E_UNSUPPORTED, "backprojection variant missing or too small for this geometry");
    const int c = t->decim_chunks;
    if (c == 0 && !pl->staged_cpt)
        return fail(FDKOD_E_UNSUPPORTED, "the row-staged decimation does not apply to this plan");
    if (!(c == 0 || c == 1 || c == 2 || c == 4 || c == 8))
        return fail(FDKOD_E_UNSUPPORTED, "decim_chunks must be 0, 1, 2, 4 or 8");
    if (c > max_chunks(pl))
        return fail(FDKOD_E_UNSUPPORTED, "decim_chunks above 4 with more than two decimation windows");
    pl->bpv = v;
    pl->dec_chunks = c;
    pl->tuned_bp_ms = t->bp_ms;
    pl->tuned_dec_ms = t->decim_ms;
    return FDKOD_OK;
}

fdkod_status fdkod_tune(fdkod_plan_t pl, const void* filt, void* ws, float* vol,
                        fdkod_stream_t stream, fdkod_tuning* out) {
    if (!pl || !filt || !vol || (pl->s > 0 && !ws)) return fail(FDKOD_E_ARG, "NULL argument");
    if (!pl->bp_ok) return fail(FDKOD_E_UNSUPPORTED, "no backprojection variant holds this geometry");
    hipStream_t st = (hipStream_t)stream;
    fdkod_status r = FDKOD_OK;
    // decimation chunking (its output feeds the backprojection timings)
    if (pl->s > 0) {
        float best = 1e30f;
        int bestc = pl->dec_chunks;
        for (int c : {0, 1, 2, 4, 8}) {
            if (c > max_chunks(pl) || (c == 0 && !pl->staged_cpt)) continue;
            pl->dec_chunks = c;
            float ms = 0.0f;
            r = time_ms(st, 3, [&] { return fdkod_decompose(pl, filt, ws, stream); }, &ms);
            if (r != FDKOD_OK) return r;
            if (ms < best) {
                best = ms;
                bestc = c;
            }
        }
        pl->dec_chunks = bestc;
        pl->tuned_dec_ms = best;
        if ((r = fdkod_decompose(pl, filt, ws, stream)) != FDKOD_OK) return r;
    }
    float best = 1e30f;
    BpVariant bestv = pl->bpv;
    for (int zr : {64, 32, 16})
        for (int tw : {32, 64})
            for (int th : {48, 64, 96})
                for (int g : {1, 2, 4}) {
                    const BpVariant v{zr, tw, th, g};
                    if (!variant_holds(pl, v)) continue;
                    pl->bpv = v;
                    float ms = 0.0f;
                    r = time_ms(st, 3, [&] { return fdkod_reconstruct(pl, filt, ws, vol, stream); }, &ms);
                    if (r != FDKOD_OK) return r;
                    if (ms < best) {
                        best = ms;
                        bestv = v;
                    }
                }
    pl->bpv = bestv;
    pl->tuned_bp_ms = best;
    tune_cache_store(pl);
    return out ? fdkod_get_tuning(pl, out) : FDKOD_OK;
}

}  // extern "C"
