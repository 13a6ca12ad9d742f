// Host-side helpers shared by the C ABI driver files: error reporting, the
// chunked device-resident loop and pinned read-back slots.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/eik.h"
#include "eik_internal.hpp"

namespace eik {

extern thread_local std::string g_last_error;

inline eik_status fail(eik_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(EIK_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Pinned host words for counter read-back (one set per host thread).
struct HostSlots {
    static constexpr int kWords = 8192;  // two slots of segment lengths
    int* words = nullptr;
    Ctl* ctl = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool ok = false;
    HostSlots() {
        if (hipHostMalloc(reinterpret_cast<void**>(&words), kWords * sizeof(int)) != hipSuccess) return;
        if (hipHostMalloc(reinterpret_cast<void**>(&ctl), sizeof(Ctl)) != hipSuccess) return;
        if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess) return;
        if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) return;
        ok = true;
    }
};

inline HostSlots& host_slots() {
    static thread_local HostSlots hs;  // lives until the thread ends
    return hs;
}

// Run `step(t)` for t = 0, 1, ... until the list a step would consume is
// empty.  counts(t) points at the `nseg` segment lengths of that list; their
// sum is read back after every chunk while the next chunk is already queued,
// so the device never idles on the host.  Returns EIK_OK, or
// EIK_ERR_NO_CONVERGENCE after max_iters steps; *steps receives the number of
// steps enqueued.
template <typename StepFn, typename CountsFn>
inline eik_status run_loop(StepFn step, CountsFn counts, int nseg, int64_t max_iters, bool async,
                           hipStream_t s, int64_t* steps) {
    if (async) {
        for (int64_t t = 0; t < max_iters; ++t) HIP_TRY(step(t));
        *steps = max_iters;
        return EIK_OK;
    }
    HostSlots& hs = host_slots();
    if (!hs.ok) return fail(EIK_ERR_DEVICE, "pinned host buffer allocation failed");
    if (nseg > HostSlots::kWords / 2) return fail(EIK_ERR_UNSUPPORTED, "too many list segments");
    const int64_t chunk = 16;  // even: list parity repeats
    auto total = [&](int slot) {
        long long sum = 0;
        const int* w = hs.words + slot * (HostSlots::kWords / 2);
        for (int k = 0; k < nseg; ++k) sum += w[k];
        return sum;
    };
    int64_t t = 0;
    int pending = -1, slot = 0;
    for (;;) {
        const int64_t end = std::min(max_iters, t + chunk);
        for (; t < end; ++t) HIP_TRY(step(t));
        HIP_TRY(hipMemcpyAsync(hs.words + slot * (HostSlots::kWords / 2), counts(t), nseg * sizeof(int),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(hs.ev[slot], s));
        if (pending >= 0) {
            HIP_TRY(hipEventSynchronize(hs.ev[pending]));
            if (total(pending) == 0) break;  // the chunk just enqueued is empty work
        }
        if (t >= max_iters) {
            HIP_TRY(hipEventSynchronize(hs.ev[slot]));
            if (total(slot) == 0) break;
            *steps = t;
            return fail(EIK_ERR_NO_CONVERGENCE, "iteration cap reached");
        }
        pending = slot;
        slot ^= 1;
    }
    *steps = t;
    return EIK_OK;
}

}  // namespace eik
