// eik_tune: per-problem choice of the tile variant's schedule -- tile shape
// and inner-iteration cap, then the ordered remedy's per-launch minimum and
// the persistent workgroups per launch -- by timing candidates with HIP events
// on the caller's stream.  Choices are cached per (ndim, dtype, log2 N,
// per-axis spacing or not, remedy schedule flags) for the process.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/eik.h"
#include "eik_host.hpp"

#define EIK_API extern "C" __attribute__((visibility("default")))

namespace eik {
namespace {

struct Choice {
    int32_t tile[3];
    int32_t inner;
    int32_t order_min = 0;   // 0: default
    int32_t workgroups = 0;  // 0: default
};

std::mutex g_tune_mu;
using TuneKey = std::tuple<int, int, int, int, unsigned>;
std::map<TuneKey, Choice>& tune_cache() {
    static std::map<TuneKey, Choice> m;
    return m;
}

// Flags that change what a tile solve does (and so which shape is fastest);
// with these the remedy is not ordered, so its per-launch minimum is not searched.
constexpr uint32_t kScheduleFlags = EIK_FLAG_SKIP_REMEDY | EIK_FLAG_FIFO_REMEDY;
// Flags a cached choice belongs to.
constexpr uint32_t kCacheFlags = kScheduleFlags | EIK_FLAG_NO_EARLY_REMEDY;

// A zero tile is the library default: in 2D that runs the update step on
// 32 x 32 tiles and detection/remedy on 16 x 16, a pairing no explicit shape
// gives.  Per-axis spacing (Eq 5) is supported on the default shapes only
// (16 x 16 in 2D, 8^3 in 3D), so only those are timed then; the zero tile is
// then the same configuration as the explicit default and is left out.
std::vector<Choice> candidates(int nd, bool aniso) {
    std::vector<Choice> all;
    if (nd == 2)
        all = {{{0, 0, 0}, 0}, {{1, 16, 16}, 0}, {{1, 16, 16}, 48}, {{1, 32, 32}, 0},
               {{1, 16, 64}, 0}, {{1, 8, 32}, 0}, {{1, 64, 64}, 0}};
    else
        all = {{{8, 8, 8}, 0}, {{8, 8, 8}, 16}, {{4, 8, 8}, 0}, {{4, 4, 16}, 0}, {{8, 8, 16}, 0}};
    if (!aniso) return all;
    std::vector<Choice> out;
    for (const Choice& c : all) {
        const bool zero = c.tile[0] == 0 && c.tile[1] == 0 && c.tile[2] == 0;
        const bool def = nd == 2 ? (c.tile[1] == 16 && c.tile[2] == 16)
                                 : (c.tile[0] == 8 && c.tile[1] == 8 && c.tile[2] == 8);
        if (def && !zero) out.push_back(c);
    }
    return out;
}

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

struct Scratch {
    void* p = nullptr;
    hipStream_t s = nullptr;
    ~Scratch() {
        if (p) (void)hipFreeAsync(p, s);
    }
};

}  // namespace
}  // namespace eik

using namespace eik;

EIK_API eik_status eik_tune(const void* F, int32_t ndim, const int64_t* dims, double h, const int64_t* sources,
                            int64_t n_sources, double eps, void* phi_scratch, eik_options* opt,
                            eik_tune_entry* report, int32_t report_cap, int32_t* n_report) {
    g_last_error.clear();
    if (n_report) *n_report = 0;
    if (!opt) return fail(EIK_ERR_INVALID_ARGUMENT, "opt is NULL (it receives the choice)");
    if (!phi_scratch) return fail(EIK_ERR_INVALID_ARGUMENT, "phi_scratch is NULL");
    if (opt->flags & (EIK_FLAG_ASYNC | EIK_FLAG_PROFILE))
        return fail(EIK_ERR_INVALID_ARGUMENT, "eik_tune runs synchronous, unprofiled solves");
    {
        // the candidates' solves check the arguments again; checking here
        // first means a cached choice is never returned for a call that a
        // solve would reject
        eik_options v = *opt;
        v.variant = EIK_VARIANT_TILE;
        std::memset(v.tile, 0, sizeof(v.tile));
        v.inner_iters = 0;
        const eik_status rc = validate_solve(F, ndim, dims, h, sources, n_sources, eps, phi_scratch, v);
        if (rc != EIK_OK) return rc;
    }
    int64_t n = 1;
    for (int k = 0; k < ndim; ++k) n *= dims[k];
    bool aniso = false;
    for (int k = 0; k < 3; ++k) aniso |= opt->spacing[k] != 0.0;
    const TuneKey key = std::make_tuple(static_cast<int>(ndim), static_cast<int>(opt->dtype),
                                        static_cast<int>(std::floor(std::log2(static_cast<double>(n)))),
                                        static_cast<int>(aniso), opt->flags & kCacheFlags);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = tune_cache().find(key);
        if (it != tune_cache().end()) {
            opt->variant = EIK_VARIANT_TILE;
            std::memcpy(opt->tile, it->second.tile, sizeof(opt->tile));
            opt->inner_iters = it->second.inner;
            opt->order_min = it->second.order_min;
            opt->workgroups = it->second.workgroups;
            return EIK_OK;
        }
    }
    eik_options base = *opt;
    base.variant = EIK_VARIANT_TILE;
    base.stats = nullptr;
    base.order_min = 0;
    base.workgroups = 0;
    const std::vector<Choice> cand = candidates(ndim, aniso);
    size_t need = 0;
    for (const Choice& c : cand) {
        eik_options q = base;
        std::memcpy(q.tile, c.tile, sizeof(q.tile));
        q.workspace = nullptr;
        need = std::max(need, eik_workspace_size(ndim, dims, &q));
    }
    if (need == 0) return fail(EIK_ERR_INVALID_ARGUMENT, "invalid shape or options");
    hipStream_t s = static_cast<hipStream_t>(base.stream);
    Scratch scratch;
    if (!base.workspace || base.workspace_bytes < need) {
        if (hipMallocAsync(&scratch.p, need, s) != hipSuccess)
            return fail(EIK_ERR_OUT_OF_MEMORY, "workspace allocation failed");
        scratch.s = s;
        base.workspace = scratch.p;
        base.workspace_bytes = need;
    }
    Events ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    double best = 0.0;
    Choice pick = cand[0];
    int32_t written = 0;
    // warm-up solve, then the best of two timed ones; the fastest so far is kept
    auto trial = [&](const Choice& c) -> eik_status {
        eik_options q = base;
        std::memcpy(q.tile, c.tile, sizeof(q.tile));
        q.inner_iters = c.inner;
        q.order_min = c.order_min;
        q.workgroups = c.workgroups;
        eik_status rc = eik_solve(F, ndim, dims, h, sources, n_sources, eps, phi_scratch, &q);
        if (rc != EIK_OK) return rc;
        double ms_best = 0.0;
        for (int rep = 0; rep < 2; ++rep) {
            HIP_TRY(hipEventRecord(ev.a, s));
            rc = eik_solve(F, ndim, dims, h, sources, n_sources, eps, phi_scratch, &q);
            if (rc != EIK_OK) return rc;
            HIP_TRY(hipEventRecord(ev.b, s));
            HIP_TRY(hipEventSynchronize(ev.b));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
            if (rep == 0 || ms < ms_best) ms_best = ms;
        }
        if (report && written < report_cap) {
            eik_tune_entry& e = report[written++];
            std::memcpy(e.tile, c.tile, sizeof(e.tile));
            e.inner_iters = c.inner;
            e.ms = ms_best;
            e.order_min = c.order_min;
            e.workgroups = c.workgroups;
        }
        if (best == 0.0 || ms_best < best) {
            best = ms_best;
            pick = c;
        }
        return EIK_OK;
    };
    for (const Choice& c : cand) {
        const eik_status rc = trial(c);
        if (rc != EIK_OK) return rc;
    }
    // launch parameters for the chosen shape: the ordered remedy's per-launch
    // minimum (when the remedy runs ordered), then the workgroups per launch
    const Choice shape = pick;
    if (!(base.flags & kScheduleFlags)) {
        const int om = order_min_of(ndim, 0);
        for (int v : {om / 2, 2 * om}) {
            Choice c = shape;
            c.order_min = v;
            const eik_status rc = trial(c);
            if (rc != EIK_OK) return rc;
        }
    }
    const Choice launch = pick;
    for (int v : {1024, 1536, 2048}) {
        if (v == workgroups_of(ndim, 0)) continue;  // timed already
        Choice c = launch;
        c.workgroups = v;
        const eik_status rc = trial(c);
        if (rc != EIK_OK) return rc;
    }
    if (n_report) *n_report = written;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache()[key] = pick;
    }
    opt->variant = EIK_VARIANT_TILE;
    std::memcpy(opt->tile, pick.tile, sizeof(opt->tile));
    opt->inner_iters = pick.inner;
    opt->order_min = pick.order_min;
    opt->workgroups = pick.workgroups;
    return EIK_OK;
}
