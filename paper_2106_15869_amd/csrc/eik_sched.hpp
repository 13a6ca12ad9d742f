// Tile scheduling shared by the forward tile kernels and the adjoint: tile
// lists of kSub sub-lists drained by persistent workgroups through fetch
// counters, per-list tile stamps, dirty-face masks by launch parity, order
// keys with their histograms (ordered scheduling) and the split kernel that
// picks a launch's tiles, plus the in-tile geometry and LDS list helpers.
#pragma once

#include <stdint.h>

#include "eik_device.hpp"
#include "eik_internal.hpp"

namespace eik {
namespace {

// Persistent workgroups of a tile launch (eik_options.workgroups, a multiple
// of kSub); group k = blockIdx % kSub drains sub-list k of the launch's tile
// list.  GT is the most a launch takes.
constexpr int GT = kMaxStatBlocks;
constexpr int kSub = kWorkgroupStep;  // sub-lists per tile list
static_assert(GT % kSub == 0, "each sub-list has the same number of workgroups");
constexpr int kPad = 32;      // ints between counters (separate cache lines)
// Dirty-face mask bit meaning "recheck every node of the tile".
constexpr uint32_t kAllFaces = 64u;
// Ordered remedy: per-tile order keys (monotone 32-bit images of the
// smallest value that made the tile pending), a histogram of them over kBins
// bins (the top key bits: sign, exponent and the leading mantissa bits), and
// the number of lowest-key tiles a launch processes at least (order_min in
// eik_internal.hpp).
constexpr int kBins = 8192;
constexpr int kBinShift = 32 - 13;  // kBins = 2^13

constexpr uint32_t kNoKey = 0xffffffffu;


// A tile list: kSub sub-lists of `cap` tile ids.  count[k * kPad] is the
// length of sub-list k (appended with atomicAdd by producers), fetch[k * kPad]
// the next entry a consumer of sub-list k takes (atomicAdd by consumers).
// A work list (ordered scheduling) also holds, entry by entry, the tile's
// order key and dirty faces, so that a consumer reads them together with the
// tile id instead of after it.
struct TList {
    int* data;
    int* count;
    int* fetch;
    int cap;
    uint32_t* key = nullptr;
    uint32_t* mask = nullptr;
};

// Scheduling state of a tile launch (shared by the forward kernels and the
// adjoint): the list it drains and the one it fills, tile stamps, dirty-face
// masks, order keys and histograms, the ordered work list, the control block.
struct Sched {
    uint32_t* tstamp;
    // Per tile dirty faces (bit d) or kAllFaces, double-buffered by launch
    // parity: a launch reads and clears `mask_cur` of the tiles it visits and
    // sets bits only in `mask_next`, which the next launch reads.  A bit set
    // during a launch is therefore never consumed by a visit that may have
    // staged the neighbour's values before the change that set it.
    uint32_t* mask_cur;
    uint32_t* mask_next;
    // ordered scheduling: keys by launch parity, histograms rotating like the
    // list counters
    uint32_t* key_cur;
    uint32_t* key_next;
    unsigned* hist_cur;
    unsigned* hist_next;
    int ordered;
    int order_min;           // ordered: lowest-key tiles a launch takes at least
    TList work;              // ordered: the tiles of this launch, split off by k_tile_split
    int* work_zero_count;    // counters of the other work list: cleared by the consuming launch
    int* work_zero_fetch;
    TList cur;
    TList next;
    int* zero_count;   // counters of the list two launches ahead: cleared by this launch
    int* zero_fetch;
    Ctl* ctl;
    unsigned long long* blkstat;  // [kStatFields][kMaxStatBlocks], column blockIdx % kMaxStatBlocks
    int tag_slot;
    int phase;  // 0 update step, 1 remedy (or adjoint) loop
    int first;  // first launch of its loop
};

__device__ __forceinline__ bool claim_tile(uint32_t* tstamp, int t, uint32_t tag) {
    return atomicMax(tstamp + t, tag) < tag;
}

template <int ND, int TX, int TY, int TZ>
struct Shape {
    static constexpr int LX = TX + 2;
    static constexpr int LY = TY + 2;
    static constexpr int LZ = ND == 3 ? TZ + 2 : 1;
    static constexpr int NT = TX * TY * (ND == 3 ? TZ : 1);
    static constexpr int NL = LX * LY * LZ;
    static constexpr int NPT = (NT + kBlock - 1) / kBlock;
    static constexpr int SY = LX;
    static constexpr int SZ = LX * LY;
};

template <int ND, int TX, int TY, int TZ>
__device__ __forceinline__ int lds_offset(int d) {
    using S = Shape<ND, TX, TY, TZ>;
    switch (d) {
        case 0: return -1;
        case 1: return 1;
        case 2: return -S::SY;
        case 3: return S::SY;
        case 4: return -S::SZ;
        default: return S::SZ;
    }
}

template <typename T>
__device__ __forceinline__ int neighbour_tile(const Inst<T>& g, int t, int d) {
    switch (d) {
        case 0: return t - 1;
        case 1: return t + 1;
        case 2: return t - g.ntx;
        case 3: return t + g.ntx;
        case 4: return t - g.ntx * g.nty;
        default: return t + g.ntx * g.nty;
    }
}

// Tag chain: launch with slot p reads tag[p] and stores tag[p] + 1 into
// tag[p ^ 1]; tiles it schedules are claimed with tag[p] + 1.
__device__ __forceinline__ uint32_t launch_tag(const Sched& a) {
    const uint32_t tag = static_cast<uint32_t>(a.ctl->tag[a.tag_slot]);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->tag[a.tag_slot ^ 1] = static_cast<int>(tag + 1);
    return tag + 1;
}

__device__ __forceinline__ void launch_stats(const Sched& a, int n) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned long long un = static_cast<unsigned long long>(n);
        if (n > 0) {
            if (a.phase == 0) {
                a.ctl->iters2 += 1;
                if (un > a.ctl->max_active) a.ctl->max_active = un;
            } else {
                a.ctl->iters3 += 1;
            }
        }
        if (a.first) a.ctl->remedy_init = un;
    }
}

// Claim tile t for the next list and append it to sub-list t % kSub.
__device__ __forceinline__ bool push_tile(const TList& out, uint32_t* tstamp, int t, uint32_t tag) {
    if (!claim_tile(tstamp, t, tag)) return false;
    const int k = t & (kSub - 1);
    const int pos = atomicAdd(out.count + k * kPad, 1);
    out.data[static_cast<size_t>(k) * out.cap + pos] = t;
    return true;
}

// Order key of a value: unsigned integers compare like the (float) values.
template <typename T>
__device__ __forceinline__ uint32_t order_key(T v) {
    const uint32_t b = __float_as_uint(static_cast<float>(v));
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ int key_bin(uint32_t key) { return static_cast<int>(key >> kBinShift); }

// Append tile t to sub-list t % kSub of `out` (the caller has made sure it
// is not there yet).
__device__ __forceinline__ void append_tile(const TList& out, int t) {
    const int k = t & (kSub - 1);
    const int pos = atomicAdd(out.count + k * kPad, 1);
    out.data[static_cast<size_t>(k) * out.cap + pos] = t;
}

// push_tile with an order key.  In ordered mode the tile's key in the next
// list drops to `key` if lower, and the key array also tells membership: the
// keys of a list start at kNoKey (a tile leaving a list has its key reset,
// a tile carried over to the next list takes its key there), so the push
// that sees kNoKey is the first of t into the next list and appends it.  The
// next list's histogram counts every listed tile in the bin of its current
// key: the first push counts it, a push that lowers the key into a lower bin
// moves the count; the chain of lowering pushes is ordered by atomicMin, so
// the histogram is exact once the launch ends.  Without ordering the tile
// stamp deduplicates (push_tile).
__device__ __forceinline__ void push_keyed(const Sched& a, int t, uint32_t tag, uint32_t key) {
    if (!a.ordered) {
        push_tile(a.next, a.tstamp, t, tag);
        return;
    }
    const uint32_t old = atomicMin(a.key_next + t, key);
    const int nb = key_bin(key);
    if (old == kNoKey) {
        append_tile(a.next, t);
        atomicAdd(a.hist_next + nb, 1u);
    } else if (nb < key_bin(old)) {
        atomicSub(a.hist_next + key_bin(old), 1u);
        atomicAdd(a.hist_next + nb, 1u);
    }
}

// Ordered remedy: the largest histogram bin whose tiles this launch
// processes -- the first bin where the running count reaches
// min(list length, order_min).  Block-wide.
__device__ __forceinline__ int order_threshold(const Sched& a, int n, int* s_thr) {
    constexpr int PER = kBins / kBlock;
    __shared__ int s_wave[kBlock / 64];
    const unsigned* h = a.hist_cur + threadIdx.x * PER;
    int sum = 0;
    for (int j = 0; j < PER; ++j) sum += static_cast<int>(h[j]);
    const int incl = wave_incl_scan(sum);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) s_wave[w] = incl;
    if (threadIdx.x == 0) *s_thr = kBins - 1;
    __syncthreads();
    int run = incl - sum;
    for (int q = 0; q < w; ++q) run += s_wave[q];
    const int need = min(n, a.order_min);
    if (run < need && run + sum >= need) {  // exactly one thread holds the crossing bin
        for (int j = 0; j < PER; ++j) {
            run += static_cast<int>(h[j]);
            if (run >= need) {
                *s_thr = threadIdx.x * PER + j;
                break;
            }
        }
    }
    __syncthreads();
    return *s_thr;
}

// Clear the counters of the list two launches ahead (nobody reads or writes
// them during this launch) and return the total length of the current list.
// With s_wlen (a consumer of the ordered work list) the work list's lengths
// are read in the same round and the other work list's counters cleared.
__device__ __forceinline__ int list_open(const Sched& a, int* s_len, int* s_wlen = nullptr) {
    if (blockIdx.x == 0 && threadIdx.x < kSub) {
        a.zero_count[threadIdx.x * kPad] = 0;
        a.zero_fetch[threadIdx.x * kPad] = 0;
        if (s_wlen && a.ordered) {
            a.work_zero_count[threadIdx.x * kPad] = 0;
            a.work_zero_fetch[threadIdx.x * kPad] = 0;
        }
    }
    if (threadIdx.x < kSub) {
        s_len[threadIdx.x] = a.cur.count[threadIdx.x * kPad];
        if (s_wlen && a.ordered) s_wlen[threadIdx.x] = a.work.count[threadIdx.x * kPad];
    }
    __syncthreads();
    int n = 0;
#pragma unroll
    for (int k = 0; k < kSub; ++k) n += s_len[k];
    return n;
}

// Ordered mode with a current list of n tiles: whether the launch drains the
// current list itself (k_tile_split moved nothing to the work list).
__device__ __forceinline__ bool list_direct(const Sched& a, int n) { return a.ordered && n <= a.order_min; }

// Index of the next entry of sub-list k (of `len` entries) a workgroup takes
// (grids of a multiple of kSub workgroups).  Its first entry is fixed,
// blockIdx / kSub: the gridDim / kSub workgroups of group k cover the first
// gridDim / kSub entries without an atomic (a launch's opening fetches would
// otherwise queue on the group's counter).  Later entries come from the
// fetch counter, offset past them -- unless the fixed entries already cover
// the sub-list, when a workgroup is done after its first visit.
__device__ __forceinline__ int fetch_index(const TList& L, int k, int len, bool first) {
    const int fixed = static_cast<int>(gridDim.x) / kSub;
    if (first) return static_cast<int>(blockIdx.x) / kSub;
    if (len <= fixed) return len;
    return fixed + atomicAdd(L.fetch + k * kPad, 1);
}

// A workgroup's first entry has a fixed index (fetch_index), so lane 0 can
// load it before the list lengths are known, in the same memory round: from
// the current list and, ordered, from the work list with its key and dirty
// faces (an entry at or past its sub-list's length is not used).  The
// adjoint's tile kernel does (adjoint 2D lognormal 4096^2 25.4 -> 25.1 ms);
// in the forward kernels the values held through the first visit made the
// remedy and the 2D update step slower.
struct FirstEntry {
    int cur = -1;
    int work = -1;
    uint32_t key = kNoKey;
    uint32_t mask = 0u;
};
__device__ __forceinline__ FirstEntry first_entry(const Sched& a, bool with_work) {
    FirstEntry f;
    if (threadIdx.x == 0) {
        const int k = blockIdx.x & (kSub - 1);
        const int e = static_cast<int>(blockIdx.x) / kSub;
        if (e < a.cur.cap) f.cur = a.cur.data[static_cast<size_t>(k) * a.cur.cap + e];
        if (with_work && a.ordered && e < a.work.cap) {
            const size_t idx = static_cast<size_t>(k) * a.work.cap + e;
            f.work = a.work.data[idx];
            f.key = a.work.key[idx];
            f.mask = a.work.mask[idx];
        }
    }
    return f;
}

// Next entry of sub-list k for this workgroup (-1 when drained).  Lane 0
// fetches; the value is broadcast through LDS.
__device__ __forceinline__ int list_fetch(const TList& L, int k, int len, int* s_slot, bool first) {
    if (threadIdx.x == 0) {
        const int e = fetch_index(L, k, len, first);
        *s_slot = e < len ? L.data[static_cast<size_t>(k) * L.cap + e] : -1;
    }
    __syncthreads();
    const int t = *s_slot;
    __syncthreads();
    return t;
}

__device__ __forceinline__ void stat_add(unsigned long long* blkstat, int field, unsigned long long v) {
    if (v) atomicAdd(blkstat + field * kMaxStatBlocks + (blockIdx.x & (kMaxStatBlocks - 1)), v);
}

// ---------------------------------------------------------------------------
// In-tile work lists
// ---------------------------------------------------------------------------
// Nodes of a tile are numbered n = (z * TY + y) * TX + x.  The inner
// iterations of a visit work on an LDS list of node ids instead of sweeping
// all nodes: iteration it drains list it & 1 (length cnt[it % 3]) and appends
// to list (it + 1) & 1; a per-list flag array keeps entries unique.  Only as
// many waves as the list needs evaluate the local solver.
template <int ND, int TX, int TY, int TZ>
__device__ __forceinline__ void node_loc(int n, int& x, int& y, int& z, int& L) {
    using S = Shape<ND, TX, TY, TZ>;
    x = n % TX;
    y = (n / TX) % TY;
    z = ND == 3 ? n / (TX * TY) : 0;
    L = ND == 3 ? ((z + 1) * S::LY + (y + 1)) * S::LX + (x + 1) : (y + 1) * S::LX + (x + 1);
}

template <int TX, int TY>
__device__ __forceinline__ int node_step(int d) {
    switch (d) {
        case 0: return -1;
        case 1: return 1;
        case 2: return -TX;
        case 3: return TX;
        case 4: return -TX * TY;
        default: return TX * TY;
    }
}

// bit d: the node lies on the tile face in direction d
template <int ND, int TX, int TY, int TZ>
__device__ __forceinline__ int edge_bits(int x, int y, int z) {
    int e = (x == 0 ? 1 : 0) | (x == TX - 1 ? 2 : 0) | (y == 0 ? 4 : 0) | (y == TY - 1 ? 8 : 0);
    if (ND == 3) e |= (z == 0 ? 16 : 0) | (z == TZ - 1 ? 32 : 0);
    return e;
}

// bit d: the grid continues past the tile face in direction d
template <int ND, int TX, int TY, int TZ, typename T>
__device__ __forceinline__ int open_bits(const Inst<T>& g, int x0, int y0, int z0) {
    int f = (x0 > 0 ? 1 : 0) | (x0 + TX < g.nx ? 2 : 0) | (y0 > 0 ? 4 : 0) | (y0 + TY < g.ny ? 8 : 0);
    if (ND == 3) f |= (z0 > 0 ? 16 : 0) | (z0 + TZ < g.nz ? 32 : 0);
    return f;
}

template <int NT>
struct TileLists {
    uint32_t flag[2][NT];
    uint16_t list[2][NT];
    uint8_t dirty[NT];  // remedy: node value changed during this visit
    int cnt[3];
};

// Append node q to the next list once (returns whether it was added).
template <int NT>
__device__ __forceinline__ bool list_add(TileLists<NT>& tl, int nb, int* ncnt, int q) {
    if (atomicExch(&tl.flag[nb][q], 1u) != 0u) return false;
    tl.list[nb][atomicAdd(ncnt, 1)] = static_cast<uint16_t>(q);
    return true;
}

// Ordered remedy: before each remedy launch, one lane per entry of the
// current list sends the tile either to the work list of the launch (its key
// is within the threshold of order_threshold) or on to the next list with its
// key and dirty faces.
__global__ __launch_bounds__(kBlock) void k_tile_split(Sched a) {
    __shared__ int s_len[kSub];
    __shared__ int s_thr;
    // Block b takes sub-list k = b % kSub, chunks b / kSub, b / kSub + G, ...
    // of kBlock entries (G = gridDim.x / kSub; gridDim.x is a multiple of
    // kSub), so its first entry is known before the list lengths and is
    // loaded with them (an entry past the sub-list's length is not used).
    const int k = blockIdx.x & (kSub - 1);
    const int c0 = blockIdx.x / kSub;
    const int i0 = c0 * kBlock + threadIdx.x;
    const int t_first = i0 < a.cur.cap ? a.cur.data[static_cast<size_t>(k) * a.cur.cap + i0] : -1;
    if (threadIdx.x < kSub) s_len[threadIdx.x] = a.cur.count[threadIdx.x * kPad];
    __syncthreads();
    int n = 0;
#pragma unroll
    for (int q = 0; q < kSub; ++q) n += s_len[q];
    const int len = s_len[k];
    // an empty list stays empty (nothing is processed that could queue tiles)
    if (n == 0) return;
    // A list no longer than order_min goes to the launch whole: the consumer
    // then drains the current list itself (list_direct) and only the next
    // list's histogram has to start at zero.
    if (n <= a.order_min) {
        if (blockIdx.x == 0)
            for (int j = threadIdx.x; j < kBins; j += kBlock) a.hist_next[j] = 0u;
        return;
    }
    // blocks past their sub-list's end have nothing to do (the first kSub
    // blocks stay: they write the next list's histogram)
    if (blockIdx.x >= kSub && c0 * kBlock >= len) return;
    // the first entry's key and dirty faces: loaded before the threshold so
    // that both memory rounds are in flight together
    const int t0 = i0 < len ? t_first : -1;
    const uint32_t key0 = t0 >= 0 ? a.key_cur[t0] : kNoKey;
    const uint32_t mk0 = t0 >= 0 ? a.mask_cur[t0] : 0u;
    const int thr = order_threshold(a, n, &s_thr);
    // The deferred tiles are the listed tiles with key bins above thr, and
    // the current histogram counts the listed tiles by key bin, so the next
    // list's histogram starts as its part above thr (the launch that adds to
    // it runs after this one).  The first kSub blocks share the bins.
    if (blockIdx.x < kSub)
        for (int j = blockIdx.x * kBlock + threadIdx.x; j < kBins; j += kSub * kBlock)
            a.hist_next[j] = j > thr ? a.hist_cur[j] : 0u;
    // appends are counted per sub-list in LDS and reserved with one global
    // atomic per (list, sub-list) and block: thousands of waves hitting the
    // same list counters would otherwise queue behind each other
    __shared__ int s_cnt[2 * kSub];
    __shared__ int s_base[2 * kSub];
    const int chunks = static_cast<int>(gridDim.x) / kSub;
    for (int c = c0; c * kBlock < len; c += chunks) {
        const int i = c * kBlock + threadIdx.x;
        int t = t0;
        uint32_t key = key0, mk = mk0;
        if (c != c0) {
            t = i < len ? a.cur.data[static_cast<size_t>(k) * a.cur.cap + i] : -1;
            key = t >= 0 ? a.key_cur[t] : kNoKey;
            mk = t >= 0 ? a.mask_cur[t] : 0u;
        }
        const bool now = t >= 0 && key_bin(key) <= thr;
        const bool defer = t >= 0 && !now;
        if (t >= 0) {
            // the tile leaves the current list: its key and dirty faces go with
            // it (into the work entry, or on to the next list)
            a.key_cur[t] = kNoKey;
            a.mask_cur[t] = 0u;
        }
        if (defer) {
            // A tile appears once in the current list and the launch that
            // queues tiles for the next list runs after this one, so the
            // deferred tile's key and dirty faces carry over with plain stores
            // (its key tells that launch the tile is queued already).
            a.mask_next[t] = mk;
            a.key_next[t] = key;
        }
        for (int j = threadIdx.x; j < 2 * kSub; j += kBlock) s_cnt[j] = 0;
        __syncthreads();
        const int slot = (now ? 0 : kSub) + (t & (kSub - 1));
        const int pos = (now || defer) ? atomicAdd(&s_cnt[slot], 1) : 0;
        __syncthreads();
        for (int j = threadIdx.x; j < 2 * kSub; j += kBlock) {
            const TList& L = j < kSub ? a.work : a.next;
            s_base[j] = s_cnt[j] ? atomicAdd(L.count + (j & (kSub - 1)) * kPad, s_cnt[j]) : 0;
        }
        __syncthreads();
        if (now || defer) {
            const TList& L = now ? a.work : a.next;
            const size_t idx = static_cast<size_t>(t & (kSub - 1)) * L.cap + s_base[slot] + pos;
            L.data[idx] = t;
            if (now) {
                a.work.key[idx] = key;
                a.work.mask[idx] = mk;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host side: workspace of the scheduling state and the per-launch arguments
// ---------------------------------------------------------------------------
constexpr size_t kCounterBytes = (3 * 2 * kSub * kPad + 3 * kBins) * sizeof(int);

// Grid of k_tile_split: kSub blocks per chunk of kBlock entries of the
// longest sub-list a list of ntiles tiles can hold (a tile is listed once,
// in sub-list t % kSub), at most 128 chunks (blocks loop over the rest).
inline int split_blocks_of(int64_t ntiles) {
    const int64_t per_sub = (ntiles + kSub - 1) / kSub;
    const int64_t chunks = (per_sub + kBlock - 1) / kBlock;
    return kSub * static_cast<int>(chunks < 1 ? 1 : chunks > 128 ? 128 : chunks);
}
constexpr size_t kWorkCounterBytes = 2 * 2 * kSub * kPad * sizeof(int);

struct SchedWs {
    uint32_t* tstamp;
    uint32_t* tmask;    // two arrays of ntiles dirty-face masks (by launch parity), after tstamp
    int* data[2];       // two list buffers (alternating)
    int* counters;      // 3 rotating sets of {count[kSub*kPad], fetch[kSub*kPad]}, then
                        // 3 rotating order-key histograms of kBins counts
    uint32_t* keys;     // two arrays of ntiles order keys (by launch parity)
    int* work[2];       // ordered: work lists (by launch parity): ids, keys, masks ...
    int* work_counters; // ... and their {count, fetch} sets
    int cap;            // entries per sub-list: a sub-list can receive every tile once
    int ntiles;
    int* count_of(int set) const { return counters + set * 2 * kSub * kPad; }
    int* fetch_of(int set) const { return counters + set * 2 * kSub * kPad + kSub * kPad; }
    unsigned* hist_of(int set) const {
        return reinterpret_cast<unsigned*>(counters + 3 * 2 * kSub * kPad) + set * kBins;
    }
    // list t: buffer t % 2, counter set t % 3
    TList list_of(int64_t t) const {
        TList L;
        L.data = data[t & 1];
        L.count = count_of(static_cast<int>(t % 3));
        L.fetch = fetch_of(static_cast<int>(t % 3));
        L.cap = cap;
        return L;
    }
    TList work_of(int64_t t) const {
        TList L;
        L.data = work[t & 1];
        L.count = work_counters + (t & 1) * 2 * kSub * kPad;
        L.fetch = L.count + kSub * kPad;
        L.cap = cap;
        L.key = reinterpret_cast<uint32_t*>(L.data + static_cast<size_t>(cap) * kSub);
        L.mask = L.key + static_cast<size_t>(cap) * kSub;
        return L;
    }
};

// `take(bytes)` hands out aligned workspace regions in order.
template <typename Take>
SchedWs sched_layout(Take&& take, int64_t ntiles) {
    SchedWs w{};
    w.cap = static_cast<int>(ntiles + 64);
    w.ntiles = static_cast<int>(ntiles);
    w.tstamp = reinterpret_cast<uint32_t*>(take(4 * static_cast<size_t>(ntiles)));
    w.tmask = reinterpret_cast<uint32_t*>(take(8 * static_cast<size_t>(ntiles)));
    w.counters = reinterpret_cast<int*>(take(kCounterBytes));
    w.keys = reinterpret_cast<uint32_t*>(take(8 * static_cast<size_t>(ntiles)));
    for (int k = 0; k < 2; ++k) w.work[k] = reinterpret_cast<int*>(take(12 * static_cast<size_t>(w.cap) * kSub));
    w.work_counters = reinterpret_cast<int*>(take(kWorkCounterBytes));
    for (int k = 0; k < 2; ++k) w.data[k] = reinterpret_cast<int*>(take(4 * static_cast<size_t>(w.cap) * kSub));
    return w;
}

// Scheduling state of an unordered (first-in first-out) tile loop only:
// stamps, dirty-face masks, counters and the two list buffers, each sub-list
// sized for the tiles of its residue class (no keys, no work lists).
template <typename Take>
SchedWs early_layout(Take&& take, int64_t ntiles) {
    SchedWs w{};
    w.cap = static_cast<int>(ntiles / kSub + 64);
    w.ntiles = static_cast<int>(ntiles);
    w.tstamp = reinterpret_cast<uint32_t*>(take(4 * static_cast<size_t>(ntiles)));
    w.tmask = reinterpret_cast<uint32_t*>(take(8 * static_cast<size_t>(ntiles)));
    w.counters = reinterpret_cast<int*>(take(kCounterBytes));
    for (int k = 0; k < 2; ++k) w.data[k] = reinterpret_cast<int*>(take(4 * static_cast<size_t>(w.cap) * kSub));
    return w;
}

// Launch t of a loop drains list t and fills list t + 1 (the counter set of
// list t + 2 is cleared by launch t); tag_slot is the parity in the device
// tag chain.
inline void sched_fill(Sched& a, const SchedWs& w, int64_t t, bool ordered, int omin, int tag_slot, int phase,
                       Ctl* ctl, unsigned long long* blkstat) {
    const size_t nt = static_cast<size_t>(w.ntiles);
    a.tstamp = w.tstamp;
    a.mask_cur = w.tmask + static_cast<size_t>(t & 1) * nt;
    a.mask_next = w.tmask + static_cast<size_t>((t + 1) & 1) * nt;
    a.key_cur = w.keys + static_cast<size_t>(t & 1) * nt;
    a.key_next = w.keys + static_cast<size_t>((t + 1) & 1) * nt;
    a.hist_cur = w.hist_of(static_cast<int>(t % 3));
    a.hist_next = w.hist_of(static_cast<int>((t + 1) % 3));
    a.ordered = ordered ? 1 : 0;
    a.order_min = omin;
    a.work = w.work_of(t);
    a.work_zero_count = w.work_of(t + 1).count;
    a.work_zero_fetch = w.work_of(t + 1).fetch;
    a.cur = w.list_of(t);
    a.next = w.list_of(t + 1);
    a.zero_count = w.count_of(static_cast<int>((t + 2) % 3));
    a.zero_fetch = w.fetch_of(static_cast<int>((t + 2) % 3));
    a.ctl = ctl;
    a.blkstat = blkstat;
    a.tag_slot = tag_slot;
    a.phase = phase;
    a.first = (phase == 1 && t == 0) ? 1 : 0;
}

// Before a solve, for an early_layout state: stamps, masks and counters zero.
inline hipError_t early_clear(const SchedWs& w, hipStream_t s) {
    hipError_t e = launch_zero_words(w.tstamp, 4 * (static_cast<size_t>(w.tmask - w.tstamp) + 2 * static_cast<size_t>(w.ntiles)), s);
    if (e == hipSuccess) e = launch_zero_words(w.counters, kCounterBytes, s);
    return e;
}

// Before a solve: stamps and masks zero, list counters and histograms zero,
// order keys "none", work counters zero.
inline hipError_t sched_clear(const SchedWs& w, hipStream_t s) {
    hipError_t e = launch_zero_words(w.tstamp, 4 * (static_cast<size_t>(w.tmask - w.tstamp) + 2 * static_cast<size_t>(w.ntiles)), s);
    if (e == hipSuccess) e = launch_zero_words(w.counters, kCounterBytes, s);
    if (e == hipSuccess) e = launch_fill_words(w.keys, 2 * static_cast<size_t>(w.ntiles), kNoKey, s);
    if (e == hipSuccess) e = launch_zero_words(w.work_counters, kWorkCounterBytes, s);
    return e;
}

}  // namespace
}  // namespace eik
