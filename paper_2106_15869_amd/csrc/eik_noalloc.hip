// eik_solve_noalloc: eik_solve for callers that cannot allocate memory.
//
// The solve's workspace (labels, work lists, scheduling state, control block
// and statistics) lives in `scratch`, a file-scope device array of
// kScratchBytes that the HIP runtime creates on each GPU when the library's
// code object is loaded there and keeps until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host it is only
// a stand-in for the symbol): the first call on a device looks up the array's
// device address with hipGetSymbolAddress, with that device current, and
// keeps it per device.  A call then runs eik_solve's checks and schedule on
// that address and reads its results back through pageable host memory, so
// it calls no allocating routine (no hipMalloc / hipFree / hipHostMalloc, no
// event creation).
//
// Every call on a device shares its array, which keeps the last call's
// contents; a solve initialises all of the state it reads (control block,
// statistics, labels, list counters, stamps, masks, keys) before use.  Calls
// that overlap on one device (other host threads, other streams) race on the
// array and must be serialised by the caller.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/eik.h"
#include "eik_host.hpp"
#include "eik_internal.hpp"

#define EIK_API extern "C" __attribute__((visibility("default")))

namespace eik {
namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, once looked up

// Device address of the current device's scratch array.
eik_status scratch_address(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(EIK_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255u))
            return fail(EIK_ERR_DEVICE, "scratch array has no usable device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return EIK_OK;
}

}  // namespace
}  // namespace eik

using namespace eik;

EIK_API eik_status eik_solve_noalloc(const void* F, int32_t ndim, const int64_t* dims, double h,
                                     const int64_t* sources, int64_t n_sources, double eps, void* phi_out,
                                     const eik_options* opt) {
    g_last_error.clear();
    eik_options o;
    eik_default_options(&o);
    if (opt) o = *opt;
    if (o.workspace || o.workspace_bytes)
        return fail(EIK_ERR_INVALID_ARGUMENT, "eik_solve_noalloc uses its static scratch: workspace must be NULL");
    if (o.flags & EIK_FLAG_ASYNC)
        return fail(EIK_ERR_UNSUPPORTED,
                    "eik_solve_noalloc is synchronous (an asynchronous outcome is read from a caller workspace)");
    if (o.flags & EIK_FLAG_PROFILE)
        return fail(EIK_ERR_UNSUPPORTED, "EIK_FLAG_PROFILE creates HIP events; use eik_solve");
    eik_status rc = validate_solve(F, ndim, dims, h, sources, n_sources, eps, phi_out, o);
    if (rc) return rc;
    const size_t need = eik_workspace_size(ndim, dims, &o);
    if (need == 0) return fail(EIK_ERR_INVALID_ARGUMENT, "invalid shape or options");
    if (need > kScratchBytes)
        return fail(EIK_ERR_OUT_OF_MEMORY, "the problem needs " + std::to_string(need) +
                                               " bytes of workspace; the static scratch holds " +
                                               std::to_string(kScratchBytes));
    void* p = nullptr;
    if ((rc = scratch_address(&p))) return rc;
    o.workspace = p;
    o.workspace_bytes = kScratchBytes;
    return solve_entry(F, ndim, dims, h, sources, n_sources, eps, phi_out, o, kFlagPageable);
}
