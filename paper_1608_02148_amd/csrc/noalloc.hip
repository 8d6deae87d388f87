// rsvd_run for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation): the
// workspace is a fixed array in device memory that the library owns, so the
// caller passes only A and the outputs.
//
// The array is a file-scope __device__ object: each device the library runs
// on holds one copy (RSVD_NOALLOC_SCRATCH_BYTES) from the first call on that
// device until the process ends.  Host code never uses the array's name as a
// device address: the address of the current device's copy is looked up once
// per device (hipGetSymbolAddress, with that device current) and kept.
// Every call on a device shares that copy; the solve clears what has to start
// at zero (its status words) with a kernel, so no state leaks from one call
// to the next, but calls that overlap on one device (on different streams or
// from different threads) race on it.
#include <mutex>

#include "plan.hpp"

using namespace rsvd;

namespace {

__device__ __align__(256) unsigned char scratch[RSVD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the scratch array (null on error,
// with *err set).
void* scratch_for(int dev, hipError_t* err) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return g_scratch_ptr[dev];
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
        const hipError_t e2 = hipSetDevice(cur);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess || !p) {
        *err = (e != hipSuccess) ? e : hipErrorInvalidSymbol;
        return nullptr;
    }
    g_scratch_ptr[dev] = p;
    return p;
}

}  // namespace

extern "C" int rsvd_run_noalloc(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A,
                                int64_t lda, int32_t k, const rsvd_params* params, void* U, int64_t ldu,
                                double* S, void* V, int64_t ldv, rsvd_info* info) {
    if (!handle) return RSVD_ERR_INVALID;
    const int v = validate(dtype, m, n, k, params);
    if (v != RSVD_OK) return v;
    const Plan P = make_plan(dtype, m, n, k, params, handle->dev.num_cu, false, handle->variants);
    if (P.bytes > RSVD_NOALLOC_SCRATCH_BYTES) return RSVD_ERR_UNSUPPORTED;
    const int dev = handle->dev.device;
    if (dev < 0 || dev >= kMaxDevices) return RSVD_ERR_UNSUPPORTED;
    hipError_t e = hipSuccess;
    void* work = scratch_for(dev, &e);
    if (!work) return hip_status(handle, e);
    // the optional event timing creates events on first use; not here
    const bool prof = handle->profiling;
    handle->profiling = false;
    const int st = rsvd_run(handle, dtype, m, n, A, lda, k, params, U, ldu, S, V, ldv, work,
                            RSVD_NOALLOC_SCRATCH_BYTES, info);
    handle->profiling = prof;
    return st;
}
