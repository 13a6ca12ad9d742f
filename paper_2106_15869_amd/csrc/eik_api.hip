// C ABI of libeik.so: argument validation, workspace carving and the host
// driver that enqueues Algorithm 2's loops without a host round trip per
// iteration.  The loops are enqueued in chunks; the list length after a chunk
// is copied to pinned host memory and inspected while the next chunk already
// runs, so the device never waits for the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/eik.h"
#include "eik_internal.hpp"
#include "eik_host.hpp"
#include "eik_tile.hpp"

#define EIK_API extern "C" __attribute__((visibility("default")))

namespace eik {

thread_local std::string g_last_error;

struct Problem {
    GridDims g;
    int64_t n;
};

static eik_status check_shape(int32_t ndim, const int64_t* dims, Problem& P) {
    if (ndim != 2 && ndim != 3) return fail(EIK_ERR_INVALID_ARGUMENT, "ndim must be 2 or 3");
    if (!dims) return fail(EIK_ERR_INVALID_ARGUMENT, "dims is NULL");
    int64_t n = 1;
    for (int k = 0; k < ndim; ++k) {
        if (dims[k] < 1) return fail(EIK_ERR_INVALID_ARGUMENT, "every dim must be >= 1");
        if (dims[k] > (int64_t(1) << 31)) return fail(EIK_ERR_INVALID_ARGUMENT, "dim too large");
        n *= dims[k];
        if (n >= (int64_t(1) << 31)) return fail(EIK_ERR_INVALID_ARGUMENT, "grid must have < 2^31 nodes");
    }
    P.n = n;
    P.g.nd = ndim;
    P.g.n = static_cast<int>(n);
    if (ndim == 2) {
        P.g.nz = 1;
        P.g.ny = static_cast<int>(dims[0]);
        P.g.nx = static_cast<int>(dims[1]);
    } else {
        P.g.nz = static_cast<int>(dims[0]);
        P.g.ny = static_cast<int>(dims[1]);
        P.g.nx = static_cast<int>(dims[2]);
    }
    return EIK_OK;
}

static eik_options resolve(const eik_options* opt) {
    eik_options o;
    eik_default_options(&o);
    if (opt) o = *opt;
    return o;
}

// The option enums come from C callers, for whom any int is a value: they
// are read as integers until checked (loading an out-of-range value as the
// enum type is undefined in C++).
template <typename E>
static int raw_enum(const E& e) {
    static_assert(sizeof(E) == sizeof(int), "C enums are int-sized here");
    int v;
    std::memcpy(&v, &e, sizeof v);
    return v;
}

static bool known_dtype(const eik_options& o) {
    const int d = raw_enum(o.dtype);
    return d == EIK_FLOAT32 || d == EIK_FLOAT64;
}

static eik_status check_options(const eik_options& o) {
    if (!known_dtype(o)) return fail(EIK_ERR_INVALID_ARGUMENT, "unknown dtype");
    const int v = raw_enum(o.variant);
    if (v != EIK_VARIANT_NODE_LIST && v != EIK_VARIANT_TILE && v != EIK_VARIANT_FIM)
        return fail(EIK_ERR_INVALID_ARGUMENT, "unknown variant");
    if (o.variant == EIK_VARIANT_FIM && (o.flags & EIK_FLAG_SKIP_REMEDY))
        return fail(EIK_ERR_INVALID_ARGUMENT, "EIK_VARIANT_FIM has no remedy step to skip");
    if (o.max_iters < 0) return fail(EIK_ERR_INVALID_ARGUMENT, "max_iters must be >= 0");
    if (o.inner_iters < 0) return fail(EIK_ERR_INVALID_ARGUMENT, "inner_iters must be >= 0");
    if (o.flags & ~63u) return fail(EIK_ERR_INVALID_ARGUMENT, "unknown flag bits");
    if ((o.flags & EIK_FLAG_FIFO_REMEDY) && o.variant != EIK_VARIANT_TILE)
        return fail(EIK_ERR_INVALID_ARGUMENT, "EIK_FLAG_FIFO_REMEDY needs the tile variant");
    if ((o.flags & EIK_FLAG_ASYNC) && (o.flags & EIK_FLAG_PROFILE))
        return fail(EIK_ERR_INVALID_ARGUMENT, "EIK_FLAG_PROFILE needs a synchronous call");
    if ((o.flags & EIK_FLAG_DETERMINISTIC) && o.variant != EIK_VARIANT_NODE_LIST)
        return fail(EIK_ERR_INVALID_ARGUMENT, "EIK_FLAG_DETERMINISTIC needs the node-list variant");
    if ((o.flags & EIK_FLAG_ASYNC) && (!o.workspace || o.max_iters == 0))
        return fail(EIK_ERR_INVALID_ARGUMENT,
                    "EIK_FLAG_ASYNC needs a caller workspace and an explicit max_iters");
    if (o.workspace && (reinterpret_cast<uintptr_t>(o.workspace) & 255u))
        return fail(EIK_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
    for (int k = 0; k < 3; ++k)
        if (o.tile[k] < 0) return fail(EIK_ERR_INVALID_ARGUMENT, "tile extents must be >= 0");
    if (o.order_min < 0) return fail(EIK_ERR_INVALID_ARGUMENT, "order_min must be >= 0");
    if (o.workgroups < 0 || o.workgroups > kMaxStatBlocks || o.workgroups % kWorkgroupStep)
        return fail(EIK_ERR_INVALID_ARGUMENT, "workgroups must be 0 or a multiple of 8 up to 2048");
    return EIK_OK;
}

// Per-axis spacing of opt (all zero: isotropic h).  Fails unless the first
// ndim entries are all finite and > 0 (or all zero) and the rest zero.
static eik_status check_spacing(const eik_options& o, int ndim, bool& aniso) {
    aniso = false;
    for (int k = 0; k < 3; ++k) aniso |= o.spacing[k] != 0.0;
    if (!aniso) return EIK_OK;
    for (int k = 0; k < 3; ++k) {
        const double v = o.spacing[k];
        if (k < ndim ? !(v > 0.0 && std::isfinite(v)) : v != 0.0)
            return fail(EIK_ERR_INVALID_ARGUMENT, "spacing needs ndim finite positive entries (dims order), the rest 0");
    }
    return EIK_OK;
}

template <typename T>
static Spacing<T> make_spacing(double h, const eik_options& o, bool aniso) {
    Spacing<T> sp{};
    sp.h = static_cast<T>(h);
    sp.aniso = aniso ? 1 : 0;
    for (int k = 0; k < 3; ++k) sp.d[k] = static_cast<T>(o.spacing[k]);
    return sp;
}

// ---------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------
struct NodeWs {
    Ctl* ctl;
    unsigned long long* blkstat;
    uint8_t* lab;
    uint32_t* stamp;
    SegList seg[3];  // two alternating lists; the third is FIM's converged list
    void* vals;
    size_t bytes;
};

// A segment holds what one workgroup can append from its slice of at most
// ceil(N / G) entries, each producing at most 7 items (itself and 6
// neighbours), plus room for source seeding.
static int node_seg_cap(int64_t n) {
    return static_cast<int>(7 * ((n + kNodeSegs - 1) / kNodeSegs) + 512);
}

static NodeWs node_layout(char* base, int64_t n, size_t esz, bool det, bool fim) {
    NodeWs w{};
    size_t off = 0;
    auto take = [&](size_t b) {
        char* p = base ? base + off : nullptr;
        off = align_up(off + b, 256);
        return p;
    };
    const int cap = node_seg_cap(n);
    w.ctl = reinterpret_cast<Ctl*>(take(sizeof(Ctl)));
    w.blkstat = reinterpret_cast<unsigned long long*>(take(8 * static_cast<size_t>(kStatFields) * kNodeSegs));
    w.lab = reinterpret_cast<uint8_t*>(take(static_cast<size_t>(n)));
    w.stamp = reinterpret_cast<uint32_t*>(take(4 * static_cast<size_t>(n)));
    for (int k = 0; k < (fim ? 3 : 2); ++k) {
        w.seg[k].cap = cap;
        w.seg[k].count = reinterpret_cast<int*>(take(4 * static_cast<size_t>(kNodeSegs)));
        w.seg[k].data = reinterpret_cast<int*>(take(4 * static_cast<size_t>(cap) * kNodeSegs));
    }
    w.vals = det ? take(esz * static_cast<size_t>(n)) : nullptr;
    w.bytes = off;
    return w;
}

static size_t elem_size(eik_dtype d) { return d == EIK_FLOAT64 ? 8 : 4; }

// A single grid as a batch of one instance (sources may be empty for size
// queries).
static Batch single_batch(const Problem& P, const eik_options& o, TileCfg c,
                          const std::vector<std::pair<int, double>>& src, double h) {
    Batch b;
    b.nd = P.g.nd;
    b.cfg = c;
    bool aniso = false;
    for (int k = 0; k < 3; ++k) aniso |= o.spacing[k] != 0.0;
    batch_add(b, P.g.nx, P.g.ny, P.g.nz, h, aniso ? o.spacing : nullptr);
    b.src = src;
    b.src_inst.assign(src.size(), 0);
    return b;
}

static size_t workspace_bytes(const Problem& P, const eik_options& o) {
    if (o.variant == EIK_VARIANT_TILE)
        return tile_workspace_bytes(single_batch(P, o, pick_tile(P.g.nd, o), {}, 1.0), elem_size(o.dtype));
    return node_layout(nullptr, P.n, elem_size(o.dtype), (o.flags & EIK_FLAG_DETERMINISTIC) != 0,
                       o.variant == EIK_VARIANT_FIM).bytes;
}

// Scratch owned by the library when the caller passes no workspace.
struct OwnedWs {
    void* p = nullptr;
    hipStream_t s = nullptr;
    ~OwnedWs() {
        if (p) (void)hipFreeAsync(p, s);
    }
};

std::vector<std::pair<int, double>> dedupe_sources(const int64_t* src, const double* val, int64_t ns) {
    std::vector<std::pair<int, double>> v;
    v.reserve(static_cast<size_t>(ns));
    for (int64_t k = 0; k < ns; ++k) v.emplace_back(static_cast<int>(src[k]), val ? val[k] : 0.0);
    std::sort(v.begin(), v.end());
    std::vector<std::pair<int, double>> out;
    for (auto& e : v)
        if (out.empty() || out.back().first != e.first) out.push_back(e);
    return out;  // sorted by (index, value): the first of each index has the minimum value
}

eik_status check_sources(const Problem& P, const int64_t* sources, int64_t n_sources,
                         const double* values) {
    if (n_sources < 1) return fail(EIK_ERR_INVALID_ARGUMENT, "need at least one source");
    if (!sources) return fail(EIK_ERR_INVALID_ARGUMENT, "sources is NULL");
    for (int64_t k = 0; k < n_sources; ++k) {
        if (sources[k] < 0 || sources[k] >= P.n)
            return fail(EIK_ERR_INVALID_ARGUMENT, "source index out of range");
        if (values && !std::isfinite(values[k]))
            return fail(EIK_ERR_INVALID_ARGUMENT, "source values must be finite");
    }
    return EIK_OK;
}

template <typename T>
static eik_status solve_nodelist(const Problem& P, const T* F, const Spacing<T>& hT, double eps,
                                 const std::vector<std::pair<int, double>>& src, T* phi,
                                 const eik_options& o, char* ws, hipStream_t s, eik_stats* st) {
    const bool det = (o.flags & EIK_FLAG_DETERMINISTIC) != 0;
    const bool async = (o.flags & EIK_FLAG_ASYNC) != 0;
    const bool fim = o.variant == EIK_VARIANT_FIM;
    const bool pageable = (o.flags & kFlagPageable) != 0;
    NodeWs w = node_layout(ws, P.n, sizeof(T), det, fim);
    const int64_t cap = o.max_iters > 0 ? o.max_iters : 4 * P.n + 64;
    int64_t launched = 0;

    Profiler prof;
    prof.start((o.flags & EIK_FLAG_PROFILE) != 0, s);
    const size_t blk_bytes = 8 * static_cast<size_t>(kStatFields) * kNodeSegs;
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_ctl_init(w.ctl, s); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_zero_words(w.blkstat, blk_bytes, s); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_init<T>(F, phi, w.lab, w.stamp, P.g.n, w.ctl, s); }));
    launched += 3;
    // STEP 1: fixed boundary values, then their FAR neighbours become active
    std::vector<SrcBatch<T>> batches;
    for (size_t k = 0; k < src.size(); k += kMaxSrcBatch) {
        SrcBatch<T> b{};
        b.count = static_cast<int>(std::min<size_t>(kMaxSrcBatch, src.size() - k));
        for (int j = 0; j < b.count; ++j) {
            b.idx[j] = src[k + j].first;
            b.val[j] = static_cast<T>(src[k + j].second);
        }
        batches.push_back(b);
    }
    for (auto& b : batches)
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_seed<T>(phi, w.lab, b, s); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_seg_clear(w.seg[0].count, kNodeSegs, s); }));
    for (size_t j = 0; j < batches.size(); ++j)
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
            return launch_seed_active<T>(P.g, F, w.lab, batches[j], w.seg[0], static_cast<int>(j % kNodeSegs), s);
        }));
    launched += 1 + 2 * static_cast<int64_t>(batches.size());

    const T eT = static_cast<T>(eps);
    auto iter_args = [&](int64_t t, bool first) {
        NodeIter<T> a{};
        a.F = F;
        a.phi = phi;
        a.lab = w.lab;
        a.stamp = w.stamp;
        a.vals = static_cast<T*>(w.vals);
        a.cur = w.seg[t & 1];
        a.next = w.seg[(t + 1) & 1];
        a.conv = w.seg[2];
        a.ctl = w.ctl;
        a.blkstat = w.blkstat;
        a.tag_slot = static_cast<int>(t & 1);
        a.first = first ? 1 : 0;
        return a;
    };
    auto counts = [&](int64_t t) { return w.seg[t & 1].count; };
    const int per_iter = det ? 2 : 1;

    // STEP 2 (FIM: its update with the neighbour check, two launches per iteration)
    int64_t n2 = 0, n3 = 0;
    eik_status rc = run_loop(
        [&](int64_t t) {
            return timed(prof, EIK_KERNEL_UPDATE, [&] {
                return fim ? launch_fim<T>(P.g, iter_args(t, t == 0), hT, eT, s)
                           : launch_step2<T>(P.g, iter_args(t, t == 0), hT, eT, det, s);
            });
        },
        counts, kNodeSegs, cap, async, s, &n2, w.ctl, pageable);
    launched += (fim ? 2 : per_iter) * n2;
    if (rc == EIK_OK && !fim && !(o.flags & EIK_FLAG_SKIP_REMEDY)) {
        // STEP 3a: whole-grid check into list 0
        HIP_TRY(timed(prof, EIK_KERNEL_DETECT,
                      [&] { return launch_detect<T>(P.g, F, phi, w.lab, hT, eT, w.seg[0], s); }));
        launched += 1;
        // STEP 3b: remedy loop
        rc = run_loop(
            [&](int64_t t) {
                return timed(prof, EIK_KERNEL_REMEDY,
                             [&] { return launch_remedy<T>(P.g, iter_args(t, t == 0), hT, eT, det, s); });
            },
            counts, kNodeSegs, cap, async, s, &n3, w.ctl, pageable);
        launched += per_iter * n3;
    }
    if (async) return rc;
    Results res;
    const eik_status rr = read_results(w.ctl, w.blkstat, kNodeSegs, pageable, s, res);
    if (rr != EIK_OK) return rr;
    if (res.ctl.err & 1) return fail(EIK_ERR_INVALID_ARGUMENT, "F has negative or non-finite values");
    if (st) {
        *st = eik_stats{};
        st->step2_iters = static_cast<int64_t>(res.ctl.iters2);
        st->step3_iters = static_cast<int64_t>(res.ctl.iters3);
        st->evals_step2 = static_cast<int64_t>(res.ctl.evals2);
        st->evals_detect = (fim || (o.flags & EIK_FLAG_SKIP_REMEDY)) ? 0 : P.n - static_cast<int64_t>(src.size());
        st->evals_check = static_cast<int64_t>(res.sum[SF_CHECK]);
        st->evals_remedy = static_cast<int64_t>(res.ctl.evals_rem);
        st->remedy_initial = static_cast<int64_t>(res.ctl.remedy_init);
        st->max_active = static_cast<int64_t>(res.ctl.max_active);
        st->launches = launched;
        st->written_step2 = static_cast<int64_t>(res.sum[SF_WRITTEN2]);
        st->written_step3 = static_cast<int64_t>(res.sum[SF_WRITTEN3]);
        HIP_TRY(prof.collect(st));
    }
    return rc;
}

}  // namespace eik

using namespace eik;

EIK_API void eik_default_options(eik_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->dtype = EIK_FLOAT32;
    opt->variant = EIK_VARIANT_TILE;
}

EIK_API size_t eik_workspace_size(int32_t ndim, const int64_t* dims, const eik_options* opt) {
    Problem P;
    if (check_shape(ndim, dims, P) != EIK_OK) return 0;
    eik_options o = resolve(opt);
    if (check_options(o) != EIK_OK) {
        // ASYNC without a workspace is still a valid size query
        eik_options q = o;
        q.flags &= ~static_cast<uint32_t>(EIK_FLAG_ASYNC);
        q.workspace = nullptr;
        if (check_options(q) != EIK_OK) return 0;
    }
    return workspace_bytes(P, o);
}

namespace eik {

// Every check eik_solve makes before device work (host only).
static eik_status check_solve(const void* F, int32_t ndim, const int64_t* dims, double h, const int64_t* sources,
                              int64_t n_sources, double eps, const void* phi_out, const eik_options& o,
                              Problem& P, bool& aniso) {
    eik_status rc = check_shape(ndim, dims, P);
    if (rc) return rc;
    if ((rc = check_options(o))) return rc;
    if (!F || !phi_out) return fail(EIK_ERR_INVALID_ARGUMENT, "F and phi_out must be non-NULL");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(EIK_ERR_INVALID_ARGUMENT, "h must be finite and > 0");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(EIK_ERR_INVALID_ARGUMENT, "eps must be finite and >= 0");
    if ((rc = check_sources(P, sources, n_sources, o.source_values))) return rc;
    if (F == phi_out) return fail(EIK_ERR_INVALID_ARGUMENT, "phi_out must not alias F");
    return check_spacing(o, ndim, aniso);
}

eik_status validate_solve(const void* F, int32_t ndim, const int64_t* dims, double h, const int64_t* sources,
                          int64_t n_sources, double eps, const void* phi_out, const eik_options& o) {
    Problem P;
    bool aniso = false;
    return check_solve(F, ndim, dims, h, sources, n_sources, eps, phi_out, o, P, aniso);
}

}  // namespace eik

namespace eik {

eik_status solve_entry(const void* F, int32_t ndim, const int64_t* dims, double h, const int64_t* sources,
                       int64_t n_sources, double eps, void* phi_out, const eik_options& checked,
                       uint32_t internal) {
    Problem P;
    eik_options o = checked;
    bool aniso = false;
    eik_status rc = check_solve(F, ndim, dims, h, sources, n_sources, eps, phi_out, o, P, aniso);
    if (rc) return rc;
    o.flags |= internal;

    const size_t need = workspace_bytes(P, o);
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    OwnedWs owned;
    char* ws = static_cast<char*>(o.workspace);
    if (ws) {
        if (o.workspace_bytes < need) return fail(EIK_ERR_OUT_OF_MEMORY, "workspace too small");
    } else {
        if (hipMallocAsync(&owned.p, need, s) != hipSuccess)
            return fail(EIK_ERR_OUT_OF_MEMORY, "workspace allocation failed");
        owned.s = s;
        ws = static_cast<char*>(owned.p);
    }
    auto src = dedupe_sources(sources, o.source_values, n_sources);
    if (o.variant == EIK_VARIANT_TILE) {
        const Batch b = single_batch(P, o, pick_tile(P.g.nd, o), src, h);
        if (o.dtype == EIK_FLOAT64)
            return solve_tile<double>(b, static_cast<const double*>(F), eps, static_cast<double*>(phi_out), o, ws,
                                      s, o.stats);
        return solve_tile<float>(b, static_cast<const float*>(F), eps, static_cast<float*>(phi_out), o, ws, s,
                                 o.stats);
    }
    if (o.dtype == EIK_FLOAT64)
        return solve_nodelist<double>(P, static_cast<const double*>(F), make_spacing<double>(h, o, aniso), eps, src,
                                      static_cast<double*>(phi_out), o, ws, s, o.stats);
    return solve_nodelist<float>(P, static_cast<const float*>(F), make_spacing<float>(h, o, aniso), eps, src,
                                 static_cast<float*>(phi_out), o, ws, s, o.stats);
}

}  // namespace eik

EIK_API eik_status eik_solve(const void* F, int32_t ndim, const int64_t* dims, double h,
                             const int64_t* sources, int64_t n_sources, double eps, void* phi_out,
                             const eik_options* opt) {
    g_last_error.clear();
    return solve_entry(F, ndim, dims, h, sources, n_sources, eps, phi_out, resolve(opt), 0u);
}

EIK_API eik_status eik_apply_local(const void* F, const void* phi, int32_t ndim,
                                   const int64_t* dims, double h, void* out,
                                   const eik_options* opt) {
    g_last_error.clear();
    Problem P;
    eik_status rc = check_shape(ndim, dims, P);
    if (rc) return rc;
    eik_options o = resolve(opt);
    if ((rc = check_options(o))) return rc;
    if (!F || !phi || !out) return fail(EIK_ERR_INVALID_ARGUMENT, "null array argument");
    if (out == phi || out == F) return fail(EIK_ERR_INVALID_ARGUMENT, "out must not alias the inputs");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(EIK_ERR_INVALID_ARGUMENT, "h must be finite and > 0");
    bool aniso = false;
    if ((rc = check_spacing(o, ndim, aniso))) return rc;
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    if (o.dtype == EIK_FLOAT64)
        HIP_TRY(launch_apply_local<double>(P.g, static_cast<const double*>(F),
                                           static_cast<const double*>(phi), make_spacing<double>(h, o, aniso),
                                           static_cast<double*>(out), s));
    else
        HIP_TRY(launch_apply_local<float>(P.g, static_cast<const float*>(F),
                                          static_cast<const float*>(phi), make_spacing<float>(h, o, aniso),
                                          static_cast<float*>(out), s));
    if (!(o.flags & EIK_FLAG_ASYNC)) HIP_TRY(hipStreamSynchronize(s));
    return EIK_OK;
}

EIK_API size_t eik_adjoint_workspace_size(int32_t ndim, const int64_t* dims, const eik_options* opt) {
    Problem P;
    if (check_shape(ndim, dims, P) != EIK_OK) return 0;
    eik_options o = resolve(opt);
    if (!known_dtype(o)) return 0;
    return adjoint_workspace_bytes(single_batch(P, o, pick_tile(P.g.nd, o), {}, 1.0), elem_size(o.dtype));
}

EIK_API eik_status eik_adjoint(const void* F, const void* phi, int32_t ndim, const int64_t* dims,
                               double h, const int64_t* sources, int64_t n_sources,
                               const void* dL_dphi, void* dL_dF_out, const eik_options* opt) {
    g_last_error.clear();
    Problem P;
    eik_status rc = check_shape(ndim, dims, P);
    if (rc) return rc;
    eik_options o = resolve(opt);
    if ((rc = check_options(o))) return rc;
    if (!F || !phi || !dL_dphi || !dL_dF_out) return fail(EIK_ERR_INVALID_ARGUMENT, "null array argument");
    if (dL_dF_out == F || dL_dF_out == phi || dL_dF_out == dL_dphi)
        return fail(EIK_ERR_INVALID_ARGUMENT, "dL_dF_out must not alias the inputs");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(EIK_ERR_INVALID_ARGUMENT, "h must be finite and > 0");
    if ((rc = check_sources(P, sources, n_sources, nullptr))) return rc;
    bool aniso = false;
    if ((rc = check_spacing(o, ndim, aniso))) return rc;
    auto src = dedupe_sources(sources, nullptr, n_sources);
    const Batch b = single_batch(P, o, pick_tile(P.g.nd, o), src, h);
    const size_t need = adjoint_workspace_bytes(b, elem_size(o.dtype));
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    OwnedWs owned;
    char* ws = static_cast<char*>(o.workspace);
    if (ws) {
        if (o.workspace_bytes < need) return fail(EIK_ERR_OUT_OF_MEMORY, "workspace too small");
    } else {
        if (hipMallocAsync(&owned.p, need, s) != hipSuccess)
            return fail(EIK_ERR_OUT_OF_MEMORY, "workspace allocation failed");
        owned.s = s;
        ws = static_cast<char*>(owned.p);
    }
    if (o.dtype == EIK_FLOAT64)
        return adjoint_solve<double>(b, static_cast<const double*>(F), static_cast<const double*>(phi),
                                     static_cast<const double*>(dL_dphi), static_cast<double*>(dL_dF_out), o, ws,
                                     s, o.stats);
    return adjoint_solve<float>(b, static_cast<const float*>(F), static_cast<const float*>(phi),
                                static_cast<const float*>(dL_dphi), static_cast<float*>(dL_dF_out), o, ws, s,
                                o.stats);
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
namespace eik {

// Validate the instance descriptions and sources and build the batch (with
// empty sources when `sources` is NULL: workspace queries).
static eik_status make_batch(int32_t ndim, const eik_instance* inst, int32_t n_inst, const int64_t* sources,
                             const double* values, const eik_options& o, Batch& b) {
    if (ndim != 2 && ndim != 3) return fail(EIK_ERR_INVALID_ARGUMENT, "ndim must be 2 or 3");
    if (!inst || n_inst < 1) return fail(EIK_ERR_INVALID_ARGUMENT, "need at least one instance");
    b = Batch{};
    b.nd = ndim;
    b.cfg = pick_tile(ndim, o);
    std::vector<std::pair<int, int64_t>> ranges;
    int64_t nsrc = 0;
    for (int32_t k = 0; k < n_inst; ++k) {
        const eik_instance& e = inst[k];
        int64_t d[3] = {1, 1, 1};
        for (int j = 0; j < ndim; ++j) {
            if (e.dims[j] < 1) return fail(EIK_ERR_INVALID_ARGUMENT, "every dim must be >= 1");
            d[3 - ndim + j] = e.dims[j];
        }
        if (!(e.h > 0.0) || !std::isfinite(e.h)) return fail(EIK_ERR_INVALID_ARGUMENT, "h must be finite and > 0");
        if (e.n_sources < 1) return fail(EIK_ERR_INVALID_ARGUMENT, "every instance needs a source");
        const int64_t n = d[0] * d[1] * d[2];
        if (d[0] >= (int64_t(1) << 31) || d[1] >= (int64_t(1) << 31) || d[2] >= (int64_t(1) << 31) ||
            b.n + n >= (int64_t(1) << 31))
            return fail(EIK_ERR_INVALID_ARGUMENT, "a batch must have < 2^31 nodes");
        batch_add(b, static_cast<int>(d[2]), static_cast<int>(d[1]), static_cast<int>(d[0]), e.h, nullptr);
        nsrc += e.n_sources;
    }
    if (!sources) return EIK_OK;
    std::vector<int64_t> glob(static_cast<size_t>(nsrc));
    std::vector<int> owner(static_cast<size_t>(nsrc));
    int64_t q = 0;
    for (int32_t k = 0; k < n_inst; ++k) {
        const HostInst& h = b.inst[static_cast<size_t>(k)];
        const int64_t n = static_cast<int64_t>(h.nx) * h.ny * h.nz;
        for (int64_t j = 0; j < inst[k].n_sources; ++j, ++q) {
            if (sources[q] < 0 || sources[q] >= n) return fail(EIK_ERR_INVALID_ARGUMENT, "source index out of range");
            if (values && !std::isfinite(values[q])) return fail(EIK_ERR_INVALID_ARGUMENT, "source values must be finite");
            glob[static_cast<size_t>(q)] = h.node_base + sources[q];
            owner[static_cast<size_t>(q)] = k;
        }
    }
    b.src = dedupe_sources(glob.data(), values, nsrc);
    // instances own disjoint index ranges: recover each source's owner
    b.src_inst.resize(b.src.size());
    for (size_t j = 0; j < b.src.size(); ++j) {
        int lo = 0, hi = n_inst;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (b.inst[static_cast<size_t>(mid)].node_base <= b.src[j].first) lo = mid; else hi = mid;
        }
        b.src_inst[j] = lo;
    }
    return EIK_OK;
}

static eik_status batch_options(const eik_options& o) {
    eik_status rc = check_options(o);
    if (rc) return rc;
    if (o.spacing[0] != 0.0 || o.spacing[1] != 0.0 || o.spacing[2] != 0.0)
        return fail(EIK_ERR_UNSUPPORTED, "batched solves take one isotropic spacing per instance");
    if (o.variant != EIK_VARIANT_TILE)
        return fail(EIK_ERR_UNSUPPORTED, "batched solves use the tile variant");
    return EIK_OK;
}

}  // namespace eik

EIK_API size_t eik_batch_workspace_size(int32_t ndim, const eik_instance* inst, int32_t n_inst,
                                        const eik_options* opt) {
    eik_options o = resolve(opt);
    o.flags &= ~static_cast<uint32_t>(EIK_FLAG_ASYNC);
    o.workspace = nullptr;
    Batch b;
    if (batch_options(o) != EIK_OK || make_batch(ndim, inst, n_inst, nullptr, nullptr, o, b) != EIK_OK) return 0;
    return tile_workspace_bytes(b, elem_size(o.dtype));
}

EIK_API eik_status eik_solve_batch(const void* F, int32_t ndim, const eik_instance* inst, int32_t n_inst,
                                   const int64_t* sources, double eps, void* phi_out, const eik_options* opt) {
    g_last_error.clear();
    eik_options o = resolve(opt);
    eik_status rc = batch_options(o);
    if (rc) return rc;
    if (!F || !phi_out) return fail(EIK_ERR_INVALID_ARGUMENT, "F and phi_out must be non-NULL");
    if (F == phi_out) return fail(EIK_ERR_INVALID_ARGUMENT, "phi_out must not alias F");
    if (!sources) return fail(EIK_ERR_INVALID_ARGUMENT, "sources is NULL");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(EIK_ERR_INVALID_ARGUMENT, "eps must be finite and >= 0");
    Batch b;
    if ((rc = make_batch(ndim, inst, n_inst, sources, o.source_values, o, b))) return rc;
    const size_t need = tile_workspace_bytes(b, elem_size(o.dtype));
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    OwnedWs owned;
    char* ws = static_cast<char*>(o.workspace);
    if (ws) {
        if (o.workspace_bytes < need) return fail(EIK_ERR_OUT_OF_MEMORY, "workspace too small");
    } else {
        if (hipMallocAsync(&owned.p, need, s) != hipSuccess)
            return fail(EIK_ERR_OUT_OF_MEMORY, "workspace allocation failed");
        owned.s = s;
        ws = static_cast<char*>(owned.p);
    }
    if (o.dtype == EIK_FLOAT64)
        return solve_tile<double>(b, static_cast<const double*>(F), eps, static_cast<double*>(phi_out), o, ws, s,
                                  o.stats);
    return solve_tile<float>(b, static_cast<const float*>(F), eps, static_cast<float*>(phi_out), o, ws, s, o.stats);
}

EIK_API size_t eik_adjoint_batch_workspace_size(int32_t ndim, const eik_instance* inst, int32_t n_inst,
                                                const eik_options* opt) {
    eik_options o = resolve(opt);
    if (!known_dtype(o)) return 0;
    Batch b;
    if (make_batch(ndim, inst, n_inst, nullptr, nullptr, o, b) != EIK_OK) return 0;
    return adjoint_workspace_bytes(b, elem_size(o.dtype));
}

EIK_API eik_status eik_adjoint_batch(const void* F, const void* phi, int32_t ndim, const eik_instance* inst,
                                     int32_t n_inst, const int64_t* sources, const void* dL_dphi,
                                     void* dL_dF_out, const eik_options* opt) {
    g_last_error.clear();
    eik_options o = resolve(opt);
    eik_status rc = check_options(o);
    if (rc) return rc;
    if (o.spacing[0] != 0.0 || o.spacing[1] != 0.0 || o.spacing[2] != 0.0)
        return fail(EIK_ERR_UNSUPPORTED, "batched solves take one isotropic spacing per instance");
    if (!F || !phi || !dL_dphi || !dL_dF_out) return fail(EIK_ERR_INVALID_ARGUMENT, "null array argument");
    if (dL_dF_out == F || dL_dF_out == phi || dL_dF_out == dL_dphi)
        return fail(EIK_ERR_INVALID_ARGUMENT, "dL_dF_out must not alias the inputs");
    if (!sources) return fail(EIK_ERR_INVALID_ARGUMENT, "sources is NULL");
    Batch b;
    if ((rc = make_batch(ndim, inst, n_inst, sources, nullptr, o, b))) return rc;
    const size_t need = adjoint_workspace_bytes(b, elem_size(o.dtype));
    hipStream_t s = static_cast<hipStream_t>(o.stream);
    OwnedWs owned;
    char* ws = static_cast<char*>(o.workspace);
    if (ws) {
        if (o.workspace_bytes < need) return fail(EIK_ERR_OUT_OF_MEMORY, "workspace too small");
    } else {
        if (hipMallocAsync(&owned.p, need, s) != hipSuccess)
            return fail(EIK_ERR_OUT_OF_MEMORY, "workspace allocation failed");
        owned.s = s;
        ws = static_cast<char*>(owned.p);
    }
    if (o.dtype == EIK_FLOAT64)
        return adjoint_solve<double>(b, static_cast<const double*>(F), static_cast<const double*>(phi),
                                     static_cast<const double*>(dL_dphi), static_cast<double*>(dL_dF_out), o, ws,
                                     s, o.stats);
    return adjoint_solve<float>(b, static_cast<const float*>(F), static_cast<const float*>(phi),
                                static_cast<const float*>(dL_dphi), static_cast<float*>(dL_dF_out), o, ws, s,
                                o.stats);
}

EIK_API eik_status eik_async_status(const void* workspace, void* stream) {
    g_last_error.clear();
    if (!workspace) return fail(EIK_ERR_INVALID_ARGUMENT, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) & 255u)
        return fail(EIK_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
    // every workspace layout starts with the control block
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ctl c;
    HIP_TRY(hipMemcpyAsync(&c, workspace, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c.err & 1) return fail(EIK_ERR_INVALID_ARGUMENT, "F has negative or non-finite values");
    if (c.open_lists) return fail(EIK_ERR_NO_CONVERGENCE, "a loop used up its launch budget with work left");
    return EIK_OK;
}

EIK_API const char* eik_status_string(eik_status s) {
    switch (raw_enum(s)) {
        case EIK_OK: return "EIK_OK";
        case EIK_ERR_INVALID_ARGUMENT: return "EIK_ERR_INVALID_ARGUMENT";
        case EIK_ERR_NO_CONVERGENCE: return "EIK_ERR_NO_CONVERGENCE";
        case EIK_ERR_OUT_OF_MEMORY: return "EIK_ERR_OUT_OF_MEMORY";
        case EIK_ERR_DEVICE: return "EIK_ERR_DEVICE";
        case EIK_ERR_UNSUPPORTED: return "EIK_ERR_UNSUPPORTED";
    }
    return "EIK_UNKNOWN_STATUS";
}

EIK_API const char* eik_last_error(void) { return g_last_error.c_str(); }

EIK_API int32_t eik_abi_version(void) { return EIK_ABI_VERSION; }
