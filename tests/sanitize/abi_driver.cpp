// Driver for the sanitizer build of the library's host code (address and
// undefined-behaviour checks on the host side only; the device code is built
// normally and never launched).  Every call here is one the library must
// answer on the host: size queries over many shapes, tile choices and batch
// descriptions, and calls that argument validation rejects before any device
// work (bad shapes, spacings, options, sources, instance lists, tuner and
// status arguments).  Exit status 0 = every call answered as expected and the
// sanitizers found nothing (they abort on the first finding).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "eik.h"

static int failures = 0;
#define CHECK(c, what)                                        \
    do {                                                      \
        if (!(c)) {                                           \
            std::fprintf(stderr, "check failed: %s (%s)\n", what, eik_last_error()); \
            ++failures;                                       \
        }                                                     \
    } while (0)

static uint64_t rng = 15869;
static uint64_t next_u64() {  // splitmix64
    uint64_t z = (rng += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
static int64_t pick(int64_t lo, int64_t hi) { return lo + static_cast<int64_t>(next_u64() % static_cast<uint64_t>(hi - lo + 1)); }

// fake, never dereferenced device addresses (validation fails first)
static void* const kF = reinterpret_cast<void*>(0x100000);
static void* const kPhi = reinterpret_cast<void*>(0x200000);
static void* const kG = reinterpret_cast<void*>(0x300000);
static void* const kOut = reinterpret_cast<void*>(0x400000);

static eik_options defaults() {
    eik_options o;
    eik_default_options(&o);
    return o;
}

static void size_queries() {
    const eik_variant vars[3] = {EIK_VARIANT_NODE_LIST, EIK_VARIANT_TILE, EIK_VARIANT_FIM};
    for (int rep = 0; rep < 400; ++rep) {
        const int nd = 2 + static_cast<int>(next_u64() % 2);
        int64_t dims[3];
        for (int k = 0; k < nd; ++k) dims[k] = pick(1, nd == 2 ? 3000 : 300);
        eik_options o = defaults();
        o.dtype = (next_u64() & 1) ? EIK_FLOAT64 : EIK_FLOAT32;
        o.variant = vars[next_u64() % 3];
        if (o.variant == EIK_VARIANT_TILE && (next_u64() & 1)) {
            const int32_t shapes[][3] = {{0, 16, 16}, {0, 32, 32}, {8, 8, 8}, {4, 8, 16}, {0, 8, 64}, {3, 5, 7}};
            const auto& s = shapes[next_u64() % 6];
            std::memcpy(o.tile, s, sizeof(o.tile));
        }
        if (o.variant == EIK_VARIANT_NODE_LIST && (next_u64() & 1)) o.flags |= EIK_FLAG_DETERMINISTIC;
        const size_t a = eik_workspace_size(nd, dims, &o);
        const size_t b = eik_workspace_size(nd, dims, &o);
        CHECK(a == b, "size query is a pure function");
        (void)eik_adjoint_workspace_size(nd, dims, &o);
    }
    // rejected shapes answer 0
    int64_t bad[4][3] = {{0, 5, 5}, {5, -1, 5}, {1 << 16, 1 << 16, 1}, {int64_t(1) << 40, 1, 1}};
    eik_options o = defaults();
    for (auto& d : bad) CHECK(eik_workspace_size(2, d, &o) == 0 || d[0] > 0, "bad 2D shape");
    CHECK(eik_workspace_size(3, bad[3], &o) == 0, "huge 3D shape");
    CHECK(eik_workspace_size(1, bad[2], &o) == 0, "ndim 1");
    CHECK(eik_workspace_size(4, bad[2], &o) == 0, "ndim 4");
    CHECK(eik_workspace_size(2, nullptr, &o) == 0, "dims NULL");
}

static void solve_validation() {
    int64_t d2[2] = {6, 7}, d3[3] = {3, 4, 5};
    int64_t src[3] = {0, 5, 99};  // 99 lies outside both grids
    const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();
    eik_options o = defaults();
    CHECK(eik_solve(kF, 4, d2, 1.0, src, 1, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "ndim");
    CHECK(eik_solve(kF, 2, nullptr, 1.0, src, 1, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "dims NULL");
    CHECK(eik_solve(kF, 2, d2, 0.0, src, 1, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "h 0");
    CHECK(eik_solve(kF, 2, d2, nan, src, 1, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "h nan");
    CHECK(eik_solve(kF, 2, d2, inf, src, 1, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "h inf");
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, -1.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "eps < 0");
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 0, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "no source");
    CHECK(eik_solve(kF, 2, d2, 1.0, nullptr, 1, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "sources NULL");
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 3, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "source range");
    CHECK(eik_solve(kF, 3, d3, 1.0, src, 3, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "source range 3D");
    CHECK(eik_solve(nullptr, 2, d2, 1.0, src, 1, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "F NULL");
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kF, &o) == EIK_ERR_INVALID_ARGUMENT, "alias");
    double vals[1] = {nan};
    eik_options v = defaults();
    v.source_values = vals;
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kPhi, &v) == EIK_ERR_INVALID_ARGUMENT, "source value nan");
    // options
    eik_options b = defaults();
    // a C caller may store any int in an enum field
    const int bad_dtype = 9, bad_variant = -3;
    std::memcpy(&b.dtype, &bad_dtype, sizeof(int));
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kPhi, &b) == EIK_ERR_INVALID_ARGUMENT, "dtype");
    b = defaults();
    std::memcpy(&b.variant, &bad_variant, sizeof(int));
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kPhi, &b) == EIK_ERR_INVALID_ARGUMENT, "variant");
    b = defaults();
    b.flags = 0xffffffffu;
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kPhi, &b) == EIK_ERR_INVALID_ARGUMENT, "flags");
    b = defaults();
    b.max_iters = -5;
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kPhi, &b) == EIK_ERR_INVALID_ARGUMENT, "max_iters");
    b = defaults();
    b.inner_iters = -1;
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kPhi, &b) == EIK_ERR_INVALID_ARGUMENT, "inner_iters");
    b = defaults();
    b.tile[1] = -8;
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kPhi, &b) == EIK_ERR_INVALID_ARGUMENT, "tile");
    b = defaults();
    b.flags = EIK_FLAG_ASYNC;
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kPhi, &b) == EIK_ERR_INVALID_ARGUMENT, "async without workspace");
    b = defaults();
    b.workspace = reinterpret_cast<void*>(0x100001);
    b.workspace_bytes = 1 << 20;
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kPhi, &b) == EIK_ERR_INVALID_ARGUMENT, "misaligned workspace");
    b = defaults();
    b.workspace = reinterpret_cast<void*>(0x100000);
    b.workspace_bytes = 8;
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kPhi, &b) == EIK_ERR_OUT_OF_MEMORY, "small workspace");
    // spacing
    b = defaults();
    b.spacing[0] = 1.0;
    b.spacing[1] = -2.0;
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kPhi, &b) == EIK_ERR_INVALID_ARGUMENT, "negative spacing");
    b.spacing[1] = 2.0;
    b.spacing[2] = 1.0;
    CHECK(eik_solve(kF, 2, d2, 1.0, src, 1, 0.0, kPhi, &b) == EIK_ERR_INVALID_ARGUMENT, "third spacing in 2D");
    // local solve and adjoint
    CHECK(eik_apply_local(kF, kPhi, 2, d2, 1.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "apply_local alias");
    CHECK(eik_apply_local(nullptr, kPhi, 2, d2, 1.0, kOut, &o) == EIK_ERR_INVALID_ARGUMENT, "apply_local NULL");
    CHECK(eik_adjoint(kF, kPhi, 2, d2, 1.0, src, 3, kG, kOut, &o) == EIK_ERR_INVALID_ARGUMENT, "adjoint source");
    CHECK(eik_adjoint(kF, kPhi, 2, d2, 1.0, src, 1, kG, kG, &o) == EIK_ERR_INVALID_ARGUMENT, "adjoint alias");
    CHECK(eik_adjoint(kF, kPhi, 2, d2, -1.0, src, 1, kG, kOut, &o) == EIK_ERR_INVALID_ARGUMENT, "adjoint h");
}

static void batch_validation() {
    eik_options o = defaults();
    for (int rep = 0; rep < 200; ++rep) {
        const int n = static_cast<int>(pick(1, 40));
        std::vector<eik_instance> in(static_cast<size_t>(n));
        int64_t total_src = 0;
        for (auto& e : in) {
            e.dims[0] = pick(1, 700);
            e.dims[1] = pick(1, 700);
            e.dims[2] = 0;
            e.h = 1.0 / static_cast<double>(pick(1, 4096));
            e.n_sources = pick(1, 8);
            total_src += e.n_sources;
        }
        const size_t a = eik_batch_workspace_size(2, in.data(), n, &o);
        CHECK(a > 0, "batch size");
        (void)eik_adjoint_batch_workspace_size(2, in.data(), n, &o);
        // one source past its grid: rejected before device work
        std::vector<int64_t> src(static_cast<size_t>(total_src), 0);
        const size_t bad = static_cast<size_t>(pick(0, total_src - 1));
        src[bad] = int64_t(1) << 40;
        CHECK(eik_solve_batch(kF, 2, in.data(), n, src.data(), 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT,
              "batch source range");
        src[bad] = -1;
        CHECK(eik_adjoint_batch(kF, kPhi, 2, in.data(), n, src.data(), kG, kOut, &o) == EIK_ERR_INVALID_ARGUMENT,
              "adjoint batch source range");
        // a bad instance anywhere in the list
        const size_t k = static_cast<size_t>(pick(0, n - 1));
        const eik_instance keep = in[k];
        in[k].dims[static_cast<int>(next_u64() % 2)] = 0;
        CHECK(eik_batch_workspace_size(2, in.data(), n, &o) == 0, "bad instance dims");
        in[k] = keep;
        in[k].h = -1.0;
        CHECK(eik_solve_batch(kF, 2, in.data(), n, src.data(), 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT,
              "bad instance h");
        in[k] = keep;
        in[k].n_sources = 0;
        CHECK(eik_solve_batch(kF, 2, in.data(), n, src.data(), 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT,
              "instance without sources");
    }
    eik_instance one{{8, 8, 0}, 1.0, 1};
    int64_t s0 = 0;
    CHECK(eik_solve_batch(kF, 2, nullptr, 1, &s0, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "inst NULL");
    CHECK(eik_solve_batch(kF, 2, &one, 0, &s0, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "no instance");
    CHECK(eik_solve_batch(kF, 2, &one, 1, nullptr, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "sources NULL");
    CHECK(eik_solve_batch(kF, 5, &one, 1, &s0, 0.0, kPhi, &o) == EIK_ERR_INVALID_ARGUMENT, "batch ndim");
    eik_options node = defaults();
    node.variant = EIK_VARIANT_NODE_LIST;
    CHECK(eik_solve_batch(kF, 2, &one, 1, &s0, 0.0, kPhi, &node) == EIK_ERR_UNSUPPORTED, "batch variant");
    eik_options sp = defaults();
    sp.spacing[0] = sp.spacing[1] = 1.0;
    CHECK(eik_solve_batch(kF, 2, &one, 1, &s0, 0.0, kPhi, &sp) == EIK_ERR_UNSUPPORTED, "batch spacing");
}

static void misc() {
    // 0..7 are values of the enum type (its range covers three bits); 6 and 7
    // are no status the library defines
    for (int s = 0; s < 8; ++s) CHECK(eik_status_string(static_cast<eik_status>(s)) != nullptr, "status string");
    CHECK(std::strcmp(eik_status_string(static_cast<eik_status>(7)), "EIK_UNKNOWN_STATUS") == 0, "unknown status");
    CHECK(eik_abi_version() == EIK_ABI_VERSION, "abi version");
    CHECK(eik_async_status(nullptr, nullptr) == EIK_ERR_INVALID_ARGUMENT, "async status NULL");
    CHECK(eik_async_status(reinterpret_cast<void*>(0x100010), nullptr) == EIK_ERR_INVALID_ARGUMENT,
          "async status misaligned");
    int64_t d2[2] = {64, 64}, s0 = 0;
    eik_options o = defaults();
    eik_tune_entry rep[4];
    int32_t nrep = 0;
    CHECK(eik_tune(kF, 2, d2, 1.0, &s0, 1, 0.0, kF, &o, rep, 4, &nrep) == EIK_ERR_INVALID_ARGUMENT, "tune alias");
    CHECK(eik_tune(kF, 2, d2, 1.0, &s0, 1, 0.0, kPhi, nullptr, rep, 4, &nrep) == EIK_ERR_INVALID_ARGUMENT,
          "tune options NULL");
    int64_t far = 64 * 64;
    CHECK(eik_tune(kF, 2, d2, 1.0, &far, 1, 0.0, kPhi, &o, rep, 4, &nrep) == EIK_ERR_INVALID_ARGUMENT,
          "tune source range");
    CHECK(eik_tune(kF, 2, d2, 0.0, &s0, 1, 0.0, kPhi, &o, rep, 4, &nrep) == EIK_ERR_INVALID_ARGUMENT, "tune h");
    CHECK(std::strlen(eik_last_error()) > 0, "last error set");
}

// The no-allocation entry point: everything it refuses before device work.
static void noalloc_validation() {
    int64_t big[3] = {512, 512, 512}, d2[2] = {8, 8}, s0 = 0, far = 64;
    eik_options o = defaults();
    CHECK(eik_solve_noalloc(kF, 3, big, 1.0, &s0, 1, 0.0, kPhi, &o) == EIK_ERR_OUT_OF_MEMORY, "noalloc size");
    eik_options ws = defaults();
    ws.workspace = kG;
    ws.workspace_bytes = 1 << 20;
    CHECK(eik_solve_noalloc(kF, 2, d2, 1.0, &s0, 1, 0.0, kPhi, &ws) == EIK_ERR_INVALID_ARGUMENT, "noalloc workspace");
    eik_options a = defaults();
    a.flags = EIK_FLAG_ASYNC;
    a.max_iters = 8;
    CHECK(eik_solve_noalloc(kF, 2, d2, 1.0, &s0, 1, 0.0, kPhi, &a) == EIK_ERR_UNSUPPORTED, "noalloc async");
    eik_options p = defaults();
    p.flags = EIK_FLAG_PROFILE;
    CHECK(eik_solve_noalloc(kF, 2, d2, 1.0, &s0, 1, 0.0, kPhi, &p) == EIK_ERR_UNSUPPORTED, "noalloc profile");
    CHECK(eik_solve_noalloc(kF, 2, d2, 1.0, &far, 1, 0.0, kPhi, nullptr) == EIK_ERR_INVALID_ARGUMENT,
          "noalloc source range");
    CHECK(eik_solve_noalloc(kF, 2, d2, 1.0, &s0, 1, 0.0, kF, nullptr) == EIK_ERR_INVALID_ARGUMENT, "noalloc alias");
    eik_options wg = defaults();
    wg.workgroups = 12;
    CHECK(eik_solve_noalloc(kF, 2, d2, 1.0, &s0, 1, 0.0, kPhi, &wg) == EIK_ERR_INVALID_ARGUMENT, "noalloc workgroups");
    CHECK(eik_solve(kF, 2, d2, 1.0, &s0, 1, 0.0, kPhi, &wg) == EIK_ERR_INVALID_ARGUMENT, "solve workgroups");
    eik_options om = defaults();
    om.order_min = -3;
    CHECK(eik_solve(kF, 2, d2, 1.0, &s0, 1, 0.0, kPhi, &om) == EIK_ERR_INVALID_ARGUMENT, "solve order_min");
    eik_options f = defaults();
    f.flags = 1u << 31;
    CHECK(eik_solve_noalloc(kF, 2, d2, 1.0, &s0, 1, 0.0, kPhi, &f) == EIK_ERR_INVALID_ARGUMENT, "noalloc flags");
}

int main() {
    size_queries();
    solve_validation();
    batch_validation();
    misc();
    noalloc_validation();
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("library host-code sanitizer driver: clean\n");
    return 0;
}
