// fdkod_backproject_noalloc: decomposition and reconstruction with the
// decimated sub-sinograms kept in a fixed device array of the library instead
// of a caller workspace, for callers that cannot allocate device memory.
//
// The array `scratch` is a file-scope device variable: every GPU the library
// runs on holds one copy of kNoallocScratchBytes bytes from the time the
// library's code is loaded on it until the process ends.  Its device address
// is looked up once per device with hipGetSymbolAddress (the array's name in
// host code is only a host-side handle, never a device address) and passed to
// the decimation and backprojection kernels as their workspace pointer.  The
// decimation writes every element the backprojection reads, so nothing has to
// start at zero; calls that overlap on one GPU share the array and race.
#include <mutex>

#include "plan.h"
#include "dtype.h"

using namespace fdkod;

constexpr size_t kNoallocScratchBytes = FDKOD_NOALLOC_SCRATCH_BYTES;   // 256 MiB per GPU
static_assert(kNoallocScratchBytes == size_t(256) << 20, "the limit the header states");

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (looked up on first use, with
// that device current; the caller's current device is restored).
fdkod_status scratch_on(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return fail(FDKOD_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int prev = 0;
        HIP_TRY(hipGetDevice(&prev), "hipGetDevice");
        HIP_TRY(hipSetDevice(device), "hipSetDevice");
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        (void)hipSetDevice(prev);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(FDKOD_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return FDKOD_OK;
}

}  // namespace

extern "C" {

fdkod_status fdkod_backproject_noalloc(fdkod_plan_t pl, const void* filt, float* vol, fdkod_stream_t stream) {
    if (!pl || !filt || !vol) return fail(FDKOD_E_ARG, "NULL argument");
    if (pl->s == 0) return fdkod_reconstruct(pl, filt, nullptr, vol, stream);
    const int64_t need = pl->ws_elems * store_bytes(pl->store);
    if (need > (int64_t)kNoallocScratchBytes)
        return fail(FDKOD_E_UNSUPPORTED,
                    "the decimated sub-sinograms need " + std::to_string(need) +
                        " bytes, more than the " + std::to_string(kNoallocScratchBytes) +
                        "-byte array of fdkod_backproject_noalloc");
    void* ws = nullptr;
    fdkod_status st = scratch_on(pl->device, &ws);
    if (st != FDKOD_OK) return st;
    if ((st = fdkod_decompose(pl, filt, ws, stream)) != FDKOD_OK) return st;
    return fdkod_reconstruct(pl, filt, ws, vol, stream);
}

}  // extern "C"
