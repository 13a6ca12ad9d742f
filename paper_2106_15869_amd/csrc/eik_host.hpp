// Host-side helpers shared by the C ABI driver files: error reporting, the
// chunked device-resident loop and pinned read-back slots.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

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

// Every argument check of eik_solve (no device work; sets the last error).
eik_status validate_solve(const void* F, int32_t ndim, const int64_t* dims, double h, const int64_t* sources,
                          int64_t n_sources, double eps, const void* phi_out, const eik_options& o);

// eik_solve's checks, workspace and schedule on options with the defaults
// filled in; `internal` option bits (kFlagPageable) are added after the
// checks, which reject them from callers.
eik_status solve_entry(const void* F, int32_t ndim, const int64_t* dims, double h, const int64_t* sources,
                       int64_t n_sources, double eps, void* phi_out, const eik_options& o, uint32_t internal);

// Pinned host words for counter read-back (one set per host thread).
struct HostSlots {
    static constexpr int kWords = 8192;  // two slots of segment lengths
    int* words = nullptr;
    Ctl* ctl = nullptr;
    unsigned long long* blk = nullptr;   // per-workgroup statistics read-back
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool ok = false;
    HostSlots() {
        if (hipHostMalloc(reinterpret_cast<void**>(&words), kWords * sizeof(int)) != hipSuccess) return;
        if (hipHostMalloc(reinterpret_cast<void**>(&ctl), sizeof(Ctl)) != hipSuccess) return;
        if (hipHostMalloc(reinterpret_cast<void**>(&blk), sizeof(unsigned long long) * kStatFields *
                                                              kMaxStatBlocks) != hipSuccess)
            return;
        if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess) return;
        if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) return;
        ok = true;
    }
};

inline HostSlots& host_slots() {
    static thread_local HostSlots hs;  // lives until the thread ends
    return hs;
}

// Optional per-launch device timing (EIK_FLAG_PROFILE): events bracket each
// launch on the solve's stream; elapsed times are summed per kernel kind after
// the final synchronisation.
struct Profiler {
    bool on = false;
    hipStream_t s = nullptr;
    std::vector<hipEvent_t>* pool = nullptr;
    std::vector<int> kinds;
    size_t used = 0;
    hipError_t begin(int kind) {
        if (!on) return hipSuccess;
        hipError_t e = grow();
        if (e != hipSuccess) return e;
        kinds.push_back(kind);
        return hipEventRecord((*pool)[used++], s);
    }
    hipError_t end() {
        if (!on) return hipSuccess;
        hipError_t e = grow();
        if (e != hipSuccess) return e;
        return hipEventRecord((*pool)[used++], s);
    }
    // after the stream has been synchronised
    hipError_t collect(eik_stats* st) {
        if (!on || !st) return hipSuccess;
        for (int k = 0; k < EIK_KERNEL_KINDS; ++k) {
            st->kernel_ms[k] = 0.0;
            st->kernel_launches[k] = 0;
        }
        for (size_t j = 0; j + 1 < used; j += 2) {
            float ms = 0.f;
            hipError_t e = hipEventElapsedTime(&ms, (*pool)[j], (*pool)[j + 1]);
            if (e != hipSuccess) return e;
            st->kernel_ms[kinds[j / 2]] += ms;
            st->kernel_launches[kinds[j / 2]] += 1;
        }
        return hipSuccess;
    }
    static std::vector<hipEvent_t>& thread_pool() {
        static thread_local std::vector<hipEvent_t> p;
        return p;
    }
    void start(bool enable, hipStream_t stream) {
        on = enable;
        s = stream;
        pool = &thread_pool();
        used = 0;
        kinds.clear();
    }

   private:
    hipError_t grow() {
        if (used < pool->size()) return hipSuccess;
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        pool->push_back(e);
        return hipSuccess;
    }
};

// Launch `fn` bracketed by profiler events of kind `kind`.
template <typename Fn>
inline hipError_t timed(Profiler& p, int kind, Fn fn) {
    hipError_t e = p.begin(kind);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    return p.end();
}

// Sum the per-workgroup statistics columns (after the stream was synchronised
// and `blk` copied to hs.blk).
inline unsigned long long blk_sum(const unsigned long long* blk, int field, int nblocks) {
    unsigned long long v = 0;
    for (int b = 0; b < nblocks; ++b) v += blk[field * nblocks + b];
    return v;
}

// Run `step(t)` for t = 0, 1, ... until the list a step would consume is
// empty.  counts(t) points at the `nseg` segment lengths of that list; their
// sum is read back after every chunk while the next chunk is already queued,
// so the device never idles on the host.  Returns EIK_OK, or
// EIK_ERR_NO_CONVERGENCE after max_iters steps; *steps receives the number of
// steps enqueued.  Asynchronously (no host round trip) exactly max_iters
// steps are enqueued, launches after convergence finding empty lists, and a
// last kernel records in ctl->open_lists whether work was left over (read
// back later by eik_async_status).
// With `pageable` the lengths are copied into a stack buffer after each
// chunk and the host waits for them before enqueuing the next chunk (no
// pinned memory, no events; the device idles while the host enqueues).
template <typename StepFn, typename CountsFn>
inline eik_status run_loop(StepFn step, CountsFn counts, int nseg, int64_t max_iters, bool async,
                           hipStream_t s, int64_t* steps, Ctl* ctl, bool pageable = false) {
    if (async) {
        for (int64_t t = 0; t < max_iters; ++t) HIP_TRY(step(t));
        HIP_TRY(launch_loop_status(ctl, counts(max_iters), nseg, s));
        *steps = max_iters;
        return EIK_OK;
    }
    if (nseg > HostSlots::kWords / 2) return fail(EIK_ERR_UNSUPPORTED, "too many list segments");
    if (pageable) {
        int words[HostSlots::kWords / 2];
        int64_t t = 0;
        for (;;) {
            const int64_t end = std::min(max_iters, t + 16);
            for (; t < end; ++t) HIP_TRY(step(t));
            HIP_TRY(hipMemcpyAsync(words, counts(t), nseg * sizeof(int), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            long long sum = 0;
            for (int k = 0; k < nseg; ++k) sum += words[k];
            if (sum == 0) break;
            if (t >= max_iters) {
                *steps = t;
                return fail(EIK_ERR_NO_CONVERGENCE, "iteration cap reached");
            }
        }
        *steps = t;
        return EIK_OK;
    }
    HostSlots& hs = host_slots();
    if (!hs.ok) return fail(EIK_ERR_DEVICE, "pinned host buffer allocation failed");
    const int64_t chunk = 8;  // even: list parity repeats
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

// The control block and the statistics totals of a synchronous call, after
// its last kernel: through the per-thread pinned slots, or (pageable) by
// summing the statistics on the device and copying the totals into *r.
struct Results {
    Ctl ctl;
    unsigned long long sum[kStatFields];
};

inline eik_status read_results(const Ctl* dctl, unsigned long long* blkstat, int nblocks, bool pageable,
                               hipStream_t s, Results& r) {
    if (pageable) {
        HIP_TRY(launch_sum_stats(blkstat, nblocks, s));
        HIP_TRY(hipMemcpyAsync(&r.ctl, dctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(r.sum, blkstat, sizeof(r.sum), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return EIK_OK;
    }
    HostSlots& hs = host_slots();
    if (!hs.ok) return fail(EIK_ERR_DEVICE, "pinned host buffer allocation failed");
    HIP_TRY(hipMemcpyAsync(hs.ctl, dctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hs.blk, blkstat, sizeof(unsigned long long) * kStatFields * nblocks,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    r.ctl = *hs.ctl;
    for (int f = 0; f < kStatFields; ++f) r.sum[f] = blk_sum(hs.blk, f, nblocks);
    return EIK_OK;
}

}  // namespace eik
