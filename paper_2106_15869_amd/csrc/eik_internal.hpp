// Host/device shared definitions of the eikonal library: control block,
// kernel argument packs and the launchers the C ABI driver calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace eik {

struct Grid;

// Grid spacing: isotropic h, or per-axis spacing d[k] (dims order: z, y, x in
// 3D; y, x in 2D) when aniso is set.
template <typename T>
struct Spacing {
    T h;
    T d[3];
    int aniso;
};

// Device control block (lives in the workspace).
struct Ctl {
    int cnt[4];       // spare counters
    int err;          // bit 0: F negative or not finite
    int tag[2];       // remedy stamp tags, alternating by iteration parity
    int open_lists;   // asynchronous calls: nonzero when a loop used up its
                      // launch budget with work still listed (k_loop_status)
    unsigned long long iters2, iters3, evals2, evals_det, evals_rem, remedy_init, max_active;
    unsigned long long visits2, visits3, inner2, inner3;
};

// Per-workgroup statistics: column b of a [kStatFields][G] array is written
// only by workgroup b of each launch (plain read-modify-write, launches are
// ordered on the stream), so no launch serialises on a shared counter; the
// host sums the columns after the solve.
enum StatField {
    SF_EVALS2 = 0, SF_EVALS3, SF_VISITS2, SF_VISITS3, SF_INNER2, SF_INNER3, SF_WRITTEN2, SF_WRITTEN3,
    SF_CHECK,  // FIM: neighbour-check evaluations
    kStatFields
};
constexpr int kMaxStatBlocks = 2048;

// Persistent workgroups of a tile launch: a multiple of kWorkgroupStep (the
// sub-lists of a tile list) up to kMaxStatBlocks; by default six resident
// per CU on 256 CUs in 3D, 2048 in 2D (eik_options.workgroups).
constexpr int kWorkgroupStep = 8;
inline int default_workgroups(int nd) { return nd == 3 ? 1536 : 2048; }
// The persistent workgroups a call uses (eik_options.workgroups, 0: default).
inline int workgroups_of(int nd, int32_t opt) { return opt > 0 ? opt : default_workgroups(nd); }

// Ordered remedy: a launch takes at least this many of the queued tiles with
// the lowest order keys.  In 3D 1024; a 2D front is a curve and keeps fewer
// tiles final at a time, 512 (measured: maze 256^3 best at 1024, layered
// 192^3 5 % faster at 512, 2D lognormal 4096^2 and the paper's Example 5 at
// 4000^2 3-4 % faster at 512 than at 1024; eik_tune times both).
inline int order_min(int nd) { return nd == 2 ? 512 : 1024; }
// The per-launch minimum a call uses (eik_options.order_min, 0: default).
inline int order_min_of(int nd, int32_t opt) { return opt > 0 ? opt : order_min(nd); }

// Internal option bit, added after the caller's options are checked (callers
// cannot set it): a synchronous call reads its list lengths and results back
// through pageable host memory instead of the per-thread pinned slots and
// events, so that it allocates nothing (the no-allocation entry point).
constexpr uint32_t kFlagPageable = 1u << 31;

constexpr int kMaxSrcBatch = 64;

template <typename T>
struct SrcBatch {
    int count;
    int idx[kMaxSrcBatch];    // flat index in the batch-wide arrays
    int inst[kMaxSrcBatch];   // instance of the source (batched tile solves)
    T val[kMaxSrcBatch];
};

// Segmented list (see eik_seglist.hpp): G regions of cap entries + G lengths.
struct SegList {
    int* data;
    int* count;
    int cap;
};

// Workgroups per list launch of the node-list variant (one segment each).
constexpr int kNodeSegs = 512;

// Pointers a node-list iteration needs; the host loop alternates the two lists
// by iteration parity.
template <typename T>
struct NodeIter {
    const T* F;
    T* phi;
    uint8_t* lab;
    uint32_t* stamp;
    T* vals;           // per-entry values (synchronous-read mode)
    SegList cur;
    SegList next;
    SegList conv;      // FIM: nodes that converged in this iteration
    Ctl* ctl;
    unsigned long long* blkstat;  // [kStatFields][kNodeSegs]
    int tag_slot;      // parity of this iteration (remedy stamp tag slot)
    int first;         // first iteration of its loop
};

struct GridDims {
    int nd;
    int nx, ny, nz;
    int n;
};

// One grid of a batch (a single solve is a batch of one): its extents, its
// tile grid and where its nodes and tiles start in the batch-wide arrays.
template <typename T>
struct Inst {
    int nx, ny, nz;
    int ntx, nty, ntz;
    int node_base;   // flat index of the grid's first node in F / phi / labels
    int tile_base;   // id of its first tile
    T h;
    T d[3];          // per-axis spacing (dims order) when aniso
    int aniso;
};

// Batch-wide tile geometry handed to every tile kernel.
template <typename T>
struct BatchGeom {
    Inst<T> one;              // the instance when ninst == 1
    const Inst<T>* table;     // device, ninst entries (used when ninst > 1)
    const int* tile_inst;     // device, instance of every tile (ninst > 1)
    int ninst;
    int ntiles;               // over all instances
};

// Instance holding tile t (t must be uniform across the wave).  A table entry
// is read word by word into scalar registers; the two cases stay separate
// (a shared load through a merged pointer would go through the generic
// address space and put a memory round trip in front of every tile visit).
template <typename T>
__device__ __forceinline__ Inst<T> inst_of(const BatchGeom<T>& g, int t) {
    if (g.ninst == 1) return g.one;
    const int k = __builtin_amdgcn_readfirstlane(g.tile_inst[__builtin_amdgcn_readfirstlane(t)]);
    constexpr int W = sizeof(Inst<T>) / 4;
    static_assert(sizeof(Inst<T>) % 4 == 0, "Inst is read in 32-bit words");
    const uint32_t* src = reinterpret_cast<const uint32_t*>(g.table + k);
    Inst<T> r;
    uint32_t* dst = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
    for (int i = 0; i < W; ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return r;
}

// ---- launchers implemented in eik_nodelist.hip (T = float/double, ND = 2/3)
template <typename T>
hipError_t launch_init(const T* F, T* phi, uint8_t* lab, uint32_t* stamp, int n, Ctl* ctl,
                       hipStream_t s);
template <typename T>
hipError_t launch_seed(T* phi, uint8_t* lab, const SrcBatch<T>& b, hipStream_t s);
template <typename T>
hipError_t launch_seed_active(const GridDims& g, const T* F, uint8_t* lab, const SrcBatch<T>& b,
                              const SegList& out, int seg, hipStream_t s);
template <typename T>
hipError_t launch_step2(const GridDims& g, const NodeIter<T>& it, const Spacing<T>& h, T eps, bool det, hipStream_t s);
template <typename T>
hipError_t launch_detect(const GridDims& g, const T* F, const T* phi, const uint8_t* lab, const Spacing<T>& h, T eps,
                         const SegList& out, hipStream_t s);
template <typename T>
hipError_t launch_remedy(const GridDims& g, const NodeIter<T>& it, const Spacing<T>& h, T eps, bool det, hipStream_t s);
hipError_t launch_seg_clear(int* count, int nseg, hipStream_t s);
hipError_t launch_zero_words(void* p, size_t bytes, hipStream_t s);
hipError_t launch_fill_words(void* p, size_t n, uint32_t v, hipStream_t s);  // n 32-bit words
template <typename T>
hipError_t launch_apply_local(const GridDims& g, const T* F, const T* phi, const Spacing<T>& h, T* out,
                              hipStream_t s);
template <typename T>
hipError_t launch_fim(const GridDims& g, const NodeIter<T>& it, const Spacing<T>& h, T eps, hipStream_t s);
hipError_t launch_reset_counters(Ctl* ctl, hipStream_t s);
hipError_t launch_ctl_init(Ctl* ctl, hipStream_t s);
// After the last budgeted launch of an asynchronous loop: sums the `nseg`
// length words of the list the next launch would drain and records in
// ctl->open_lists whether it is non-empty.
hipError_t launch_loop_status(Ctl* ctl, const int* counts, int nseg, hipStream_t s);
// Sums each statistics field of a [kStatFields][nblocks] array into its
// first kStatFields words.
hipError_t launch_sum_stats(unsigned long long* blkstat, int nblocks, hipStream_t s);

}  // namespace eik
