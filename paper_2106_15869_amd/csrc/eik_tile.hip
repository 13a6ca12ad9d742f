// Tile-activated IFIM for gfx950.
//
// The grid is cut into tiles of TZ x TY x TX nodes.  A launch processes a list
// of tiles, one workgroup (256 lanes, four wave64) per tile at a time.  Each
// workgroup stages the tile's values and labels plus a one-cell halo in LDS,
// then runs the node rules of Algorithm 2 for several inner iterations
// without touching HBM, and writes back what changed.
//
//   update step (STEP 2): FAR nodes with F > 0 next to a converged or fixed
//     node become active; active nodes take phi~ = G_i(phi); a node whose
//     value no longer moves (phi - phi~ <= eps) converges and activates its FAR
//     neighbours -- no convergence check of those neighbours (Section 3.3).
//     A node converging on a tile face schedules the tile across that face; a
//     tile that still holds active nodes schedules itself.
//   remedy detection (STEP 3, first part): one dense pass over all tiles;
//     a tile with any node whose phi~ < phi - eps enters the remedy list.
//   remedy loop (STEP 3): the remedy rule of Section 3.1.2 restricted to the
//     tile: recompute the flagged nodes, take the drops, flag the changed
//     nodes and their in-tile neighbours for the next inner iteration, until
//     no flagged node changes.  A tile enters with all nodes flagged (first
//     visit) or with the nodes on the faces whose neighbour tile changed; a
//     change on a tile face marks that face dirty in the tile across it and
//     schedules it.
// Within an inner iteration all phi~ are computed before any is applied (two
// LDS phases), so a tile's iterations are synchronous; tiles of one launch see
// each other's values only through the halo staged at the start.  Tile lists
// are segmented per workgroup (eik_seglist.hpp).
#include <utility>
#include <vector>

#include "eik_device.hpp"
#include "eik_host.hpp"
#include "eik_seglist.hpp"
#include "eik_batch.hpp"
#include "eik_tile.hpp"

namespace eik {

namespace {

// LDS label byte: bits 0-1 state, bit 2 passable (F > 0), bit 3 outside grid.
constexpr uint8_t kPass = 4u, kOut = 8u;
// Workgroups per tile launch (one list segment each).
// Persistent workgroups per tile launch; group k = blockIdx % kSub drains
// sub-list k of the launch's tile list.
constexpr int GT = 2048;
constexpr int kSub = 8;       // sub-lists per tile list
constexpr int kPad = 32;      // ints between counters (separate cache lines)
// Dirty-face mask bit meaning "recheck every node of the tile".
constexpr uint32_t kAllFaces = 64u;
// Ordered remedy: per-tile order keys (monotone 32-bit images of the
// smallest value that made the tile pending), a histogram of them over kBins
// bins (the top key bits: sign, exponent and the leading mantissa bits), and
// the number of lowest-key tiles a launch processes at least.
constexpr int kBins = 8192;
constexpr int kBinShift = 32 - 13;  // kBins = 2^13
constexpr int kOrderMin = 1024;
constexpr uint32_t kNoKey = 0xffffffffu;


// A tile list: kSub sub-lists of `cap` tile ids.  count[k * kPad] is the
// length of sub-list k (appended with atomicAdd by producers), fetch[k * kPad]
// the next entry a consumer of sub-list k takes (atomicAdd by consumers).
struct TList {
    int* data;
    int* count;
    int* fetch;
    int cap;
};

template <typename T>
struct TileIter {
    const T* F;
    T* phi;
    uint8_t* lab;
    uint32_t* tstamp;
    // Per tile dirty faces (bit d) or kAllFaces, double-buffered by launch
    // parity: a launch reads and clears `mask_cur` of the tiles it visits and
    // sets bits only in `mask_next`, which the next launch reads.  A bit set
    // during a launch is therefore never consumed by a visit that may have
    // staged the neighbour's values before the change that set it.
    uint32_t* mask_cur;
    uint32_t* mask_next;
    // ordered remedy (the default; EIK_FLAG_FIFO_REMEDY turns it off): keys by
    // launch parity, histograms rotating like the list counters
    uint32_t* key_cur;
    uint32_t* key_next;
    unsigned* hist_cur;
    unsigned* hist_next;
    unsigned* hist_zero;
    int ordered;
    TList work;              // ordered: the tiles of this launch, split off by k_tile_split
    int* work_zero_count;    // counters of the other work list: cleared by the remedy launch
    int* work_zero_fetch;
    TList cur;
    TList next;
    int* zero_count;   // counters of the list two launches ahead: cleared by this launch
    int* zero_fetch;
    Ctl* ctl;
    unsigned long long* blkstat;  // [kStatFields][kMaxStatBlocks], column blockIdx % kMaxStatBlocks
    int tag_slot;
    int phase;  // 0 update step, 1 remedy loop
    int first;  // first launch of the remedy loop
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

// Per-node value kept in LDS for the local solve: H = h / F (+inf on a
// barrier), or with per-axis spacing the speed F itself (0 on a barrier).
template <typename T, bool AN>
__device__ __forceinline__ T cell_value(const Inst<T>& g, T f) {
    if (AN) return f > T(0) ? f : T(0);
    return cell_H(g.h, f);
}
template <typename T, bool AN>
__device__ __forceinline__ T dead_value() {
    return AN ? T(0) : pos_inf<T>();
}
// whether the node can take a finite value (not a barrier, inside the grid)
template <typename T, bool AN>
__device__ __forceinline__ bool cell_live(T v) {
    return AN ? v > T(0) : v < pos_inf<T>();
}

// Per-lane description of the nodes a lane owns in the current tile.
template <typename T, int NPT>
struct Owned {
    int G[NPT];      // global index
    int L[NPT];      // LDS index (with halo)
    int face[NPT];   // bit d set: node on the tile face in direction d (-x,+x,-y,+y,-z,+z)
                     // and the grid continues across it
    int edge[NPT];   // bit d set: node on the tile face in direction d
    T H[NPT];
    bool ok[NPT];
};

// Stage the tile and its halo: values (+inf outside) and labels (kOut outside).
// All global loads of a lane are issued before its first LDS store.
template <typename T, int ND, int TX, int TY, int TZ>
__device__ __forceinline__ void stage(const Inst<T>& g, int x0, int y0, int z0, const T* phi,
                                      const uint8_t* lab, T* sphi, uint8_t* sl) {
    using S = Shape<ND, TX, TY, TZ>;
    constexpr int NIT = (S::NL + kBlock - 1) / kBlock;
    const T inf = pos_inf<T>();
    T v[NIT];
    uint8_t l[NIT];
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
        const int q = threadIdx.x + j * kBlock;
        const int lx = q % S::LX;
        const int ly = (q / S::LX) % S::LY;
        const int lz = q / (S::LX * S::LY);
        const int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = ND == 3 ? z0 + lz - 1 : 0;
        const bool in = q < S::NL && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz;
        const int G = g.node_base + (gz * g.ny + gy) * g.nx + gx;
        v[j] = in ? phi[G] : inf;
        l[j] = in ? lab[G] : kOut;
    }
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
        const int q = threadIdx.x + j * kBlock;
        if (q < S::NL) {
            sphi[q] = v[j];
            sl[q] = l[j];
        }
    }
}

template <typename T, int ND, int TX, int TY, int TZ, bool AN>
__device__ __forceinline__ void own_nodes(const Inst<T>& g, int x0, int y0, int z0, const T* F,
                                          Owned<T, Shape<ND, TX, TY, TZ>::NPT>& o) {
    using S = Shape<ND, TX, TY, TZ>;
#pragma unroll
    for (int r = 0; r < S::NPT; ++r) {
        const int n = threadIdx.x + r * kBlock;
        const int x = n % TX, y = (n / TX) % TY, z = ND == 3 ? n / (TX * TY) : 0;
        const int gx = x0 + x, gy = y0 + y, gz = z0 + z;
        o.ok[r] = n < S::NT && gx < g.nx && gy < g.ny && gz < g.nz;
        o.G[r] = g.node_base + (gz * g.ny + gy) * g.nx + gx;
        o.L[r] = ND == 3 ? ((z + 1) * S::LY + (y + 1)) * S::LX + (x + 1) : (y + 1) * S::LX + (x + 1);
        int e = 0;
        if (x == 0) e |= 1;
        if (x == TX - 1) e |= 2;
        if (y == 0) e |= 4;
        if (y == TY - 1) e |= 8;
        if (ND == 3) {
            if (z == 0) e |= 16;
            if (z == TZ - 1) e |= 32;
        }
        o.edge[r] = e;
        int f = 0;
        if (x == 0 && gx > 0) f |= 1;
        if (x == TX - 1 && gx + 1 < g.nx) f |= 2;
        if (y == 0 && gy > 0) f |= 4;
        if (y == TY - 1 && gy + 1 < g.ny) f |= 8;
        if (ND == 3) {
            if (z == 0 && gz > 0) f |= 16;
            if (z == TZ - 1 && gz + 1 < g.nz) f |= 32;
        }
        o.face[r] = f;
        o.H[r] = dead_value<T, AN>();
        if (o.ok[r]) o.H[r] = cell_value<T, AN>(g, F[o.G[r]]);
    }
}

// G_i from the LDS tile (halo holds +inf outside the grid).
// v is the node's H = h / F (isotropic) or its speed F (AN: per-axis spacing,
// H_k = spacing_k / F); see cell_value.
template <typename T, int ND, int TX, int TY, int TZ, bool AN>
__device__ __forceinline__ T eval_lds(const T* sphi, int L, T v, const Inst<T>& g) {
    using S = Shape<ND, TX, TY, TZ>;
    const T inf = pos_inf<T>();
    const T ax = tmin(sphi[L - 1], sphi[L + 1]);
    const T ay = tmin(sphi[L - S::SY], sphi[L + S::SY]);
    if (AN) {
        if (!(v > T(0))) return inf;
        if (ND == 2) return godunov_aniso<T, 2>(ay, ax, inf, g.d[0] / v, g.d[1] / v, inf);
        const T az = tmin(sphi[L - S::SZ], sphi[L + S::SZ]);
        return godunov_aniso<T, 3>(az, ay, ax, g.d[0] / v, g.d[1] / v, g.d[2] / v);
    }
    if (ND == 2) return godunov<T, 2>(ay, ax, inf, v);
    const T az = tmin(sphi[L - S::SZ], sphi[L + S::SZ]);
    return godunov<T, 3>(az, ay, ax, v);
}


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
template <typename T>
__device__ __forceinline__ uint32_t launch_tag(const TileIter<T>& a) {
    const uint32_t tag = static_cast<uint32_t>(a.ctl->tag[a.tag_slot]);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->tag[a.tag_slot ^ 1] = static_cast<int>(tag + 1);
    return tag + 1;
}

template <typename T>
__device__ __forceinline__ void launch_stats(const TileIter<T>& a, int n) {
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

// push_tile for the remedy: in ordered mode also lower the tile's key and
// count the claim in the next list's histogram.
template <typename T>
__device__ __forceinline__ void push_keyed(const TileIter<T>& a, int t, uint32_t tag, uint32_t key) {
    if (a.ordered) atomicMin(a.key_next + t, key);
    if (push_tile(a.next, a.tstamp, t, tag) && a.ordered) atomicAdd(a.hist_next + key_bin(key), 1u);
}

// Ordered remedy: the largest histogram bin whose tiles this launch
// processes -- the first bin where the running count reaches
// min(list length, kOrderMin).  Block-wide; block 0 also clears the
// histogram of the list two launches ahead.
template <typename T>
__device__ __forceinline__ int order_threshold(const TileIter<T>& a, int n, int* s_thr) {
    constexpr int PER = kBins / kBlock;
    __shared__ int s_wave[kBlock / 64];
    if (blockIdx.x == 0)
        for (int j = threadIdx.x; j < kBins; j += kBlock) a.hist_zero[j] = 0u;
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
    const int need = min(n, kOrderMin);
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
template <typename T>
__device__ __forceinline__ int list_open(const TileIter<T>& a, int* s_len) {
    if (blockIdx.x == 0 && threadIdx.x < kSub) {
        a.zero_count[threadIdx.x * kPad] = 0;
        a.zero_fetch[threadIdx.x * kPad] = 0;
    }
    if (threadIdx.x < kSub) s_len[threadIdx.x] = a.cur.count[threadIdx.x * kPad];
    __syncthreads();
    int n = 0;
#pragma unroll
    for (int k = 0; k < kSub; ++k) n += s_len[k];
    return n;
}

// Next entry of sub-list k for this workgroup (-1 when drained).  Lane 0
// fetches; the value is broadcast through LDS.
__device__ __forceinline__ int list_fetch(const TList& L, int k, int len, int* s_slot) {
    if (threadIdx.x == 0) {
        const int e = atomicAdd(L.fetch + k * kPad, 1);
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

// ---------------------------------------------------------------------------
// STEP 2 on tiles
// ---------------------------------------------------------------------------
template <typename T, int ND, int TX, int TY, int TZ, bool AN>
__global__ __launch_bounds__(kBlock) void k_tile_update(TileIter<T> a, BatchGeom<T> bg, T eps, int inner) {
    using S = Shape<ND, TX, TY, TZ>;
    __shared__ T sphi[S::NL];
    __shared__ uint8_t sl[S::NL];
    __shared__ T sH[S::NT];
    __shared__ TileLists<S::NT> tl;
    __shared__ int s_len[kSub];
    __shared__ int s_slot;
    __shared__ int s_face;
    __shared__ int s_evals;
    __shared__ int s_written;
    const T inf = pos_inf<T>();
    const uint32_t ntag = launch_tag(a);
    const int n = list_open(a, s_len);
    launch_stats(a, n);
    // workgroups of group k take entries of sub-list k one at a time
    const int k = blockIdx.x & (kSub - 1);
    const int len = s_len[k];
    unsigned long long evals = 0, inner_sum = 0, written = 0, visits = 0;
    for (;;) {
        const int t = list_fetch(a.cur, k, len, &s_slot);
        if (t < 0) break;
        ++visits;
        const Inst<T> g = inst_of(bg, t);
        const int lt = t - g.tile_base;
        const int tx = lt % g.ntx, ty = (lt / g.ntx) % g.nty, tz = lt / (g.ntx * g.nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * (ND == 3 ? TZ : 1);
        const int open = open_bits<ND, TX, TY, TZ>(g, x0, y0, z0);
        stage<T, ND, TX, TY, TZ>(g, x0, y0, z0, a.phi, a.lab, sphi, sl);
        bool ok[S::NPT];
        int G[S::NPT], L[S::NPT];
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) {
            const int nn = threadIdx.x + r * kBlock;
            int x, y, z;
            node_loc<ND, TX, TY, TZ>(nn, x, y, z, L[r]);
            ok[r] = nn < S::NT && x0 + x < g.nx && y0 + y < g.ny && z0 + z < g.nz;
            G[r] = g.node_base + ((z0 + z) * g.ny + (y0 + y)) * g.nx + (x0 + x);
            if (nn < S::NT) {
                sH[nn] = ok[r] ? cell_value<T, AN>(g, a.F[G[r]]) : dead_value<T, AN>();
                tl.flag[0][nn] = 0u;
                tl.flag[1][nn] = 0u;
            }
        }
        if (threadIdx.x == 0) {
            s_face = 0;
            s_evals = 0;
            s_written = 0;
            tl.cnt[0] = tl.cnt[1] = tl.cnt[2] = 0;
        }
        __syncthreads();
        uint8_t lab0[S::NPT];
        T phi0[S::NPT];
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) {
            lab0[r] = ok[r] ? sl[L[r]] : uint8_t(0);
            phi0[r] = ok[r] ? sphi[L[r]] : inf;
            if (ok[r] && cell_live<T, AN>(sH[threadIdx.x + r * kBlock])) sl[L[r]] = lab0[r] | kPass;
        }
        __syncthreads();
        // initial active list: active nodes, and FAR nodes next to a converged
        // or fixed node (their activation was requested by a neighbour)
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) {
            if (!ok[r]) continue;
            const uint8_t me = sl[L[r]];
            bool act = (me & 3u) == L_ACTIVE;
            if ((me & 3u) == L_FAR && (me & kPass)) {
#pragma unroll
                for (int d = 0; d < 2 * ND; ++d) {
                    const uint8_t nb = sl[L[r] + lds_offset<ND, TX, TY, TZ>(d)];
                    const uint32_t st = nb & 3u;
                    act |= !(nb & kOut) && (st == L_CONV || st == L_FIXED);
                }
                if (act) sl[L[r]] = (me & ~3u) | L_ACTIVE;
            }
            if (act) tl.list[0][atomicAdd(&tl.cnt[0], 1)] = static_cast<uint16_t>(threadIdx.x + r * kBlock);
        }
        __syncthreads();
        // Inner iterations on the LDS active list, values updated in place:
        // one barrier each.  Reads racing with updates see either value, both
        // upper bounds of the solution.
        bool any_active = false;
        int my_evals = 0, fm = 0;
        int it = 0;
        for (;; ++it) {
            const int ncur = tl.cnt[it % 3];
            if (ncur == 0) break;
            if (it == inner) {
                any_active = true;  // cap reached: the listed nodes stay active
                break;
            }
            const int cb = it & 1, nb = cb ^ 1;
            int* ncnt = &tl.cnt[(it + 1) % 3];
            if (threadIdx.x == 0) tl.cnt[(it + 2) % 3] = 0;
            for (int i = threadIdx.x; i < ncur; i += kBlock) {
                const int q = tl.list[cb][i];
                tl.flag[cb][q] = 0u;
                int x, y, z, Lq;
                node_loc<ND, TX, TY, TZ>(q, x, y, z, Lq);
                ++my_evals;
                const T pt = eval_lds<T, ND, TX, TY, TZ, AN>(sphi, Lq, sH[q], g);
                const T cur = sphi[Lq];
                if (pt < inf && cur - pt <= eps) {
                    // converged: joins Source; FAR neighbours become active
                    sl[Lq] = (sl[Lq] & ~3u) | L_CONV;
                    const int edge = edge_bits<ND, TX, TY, TZ>(x, y, z);
#pragma unroll
                    for (int d = 0; d < 2 * ND; ++d) {
                        const int Ln = Lq + lds_offset<ND, TX, TY, TZ>(d);
                        const uint8_t lb = sl[Ln];
                        if (edge & (1 << d)) {
                            if ((open & (1 << d)) && (lb & 3u) == L_FAR) fm |= 1 << d;
                        } else if (!(lb & kOut) && (lb & 3u) == L_FAR && (lb & kPass)) {
                            if (list_add(tl, nb, ncnt, q + node_step<TX, TY>(d))) sl[Ln] = (lb & ~3u) | L_ACTIVE;
                        }
                    }
                } else if (!(pt < inf)) {
                    sl[Lq] = (sl[Lq] & ~3u) | L_FAR;
                } else {
                    if (pt < cur) sphi[Lq] = pt;
                    list_add(tl, nb, ncnt, q);
                }
            }
            __syncthreads();
        }
        if (fm) atomicOr(&s_face, fm);
        // write back what changed
        int my_written = 0;
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) {
            if (!ok[r]) continue;
            const uint8_t st = sl[L[r]] & 3u;
            if (st != (lab0[r] & 3u)) a.lab[G[r]] = st;
            const T v = sphi[L[r]];
            if (v != phi0[r]) {
                a.phi[G[r]] = v;
                ++my_written;
            }
        }
        if (my_evals) atomicAdd(&s_evals, my_evals);
        if (my_written) atomicAdd(&s_written, my_written);
        __syncthreads();
        // scheduling: lane d < 2*ND handles face d, lane 6 the tile itself,
        // so the device atomics of one visit are in flight together
        if (threadIdx.x < 7) {
            const int d = threadIdx.x;
            const int fmask = s_face;
            if (d == 6) {
                if (any_active) push_tile(a.next, a.tstamp, t, ntag);
            } else if (d < 2 * ND && (fmask & (1 << d))) {
                push_tile(a.next, a.tstamp, neighbour_tile(g, t, d), ntag);
            }
        }
        if (threadIdx.x == 0) {
            evals += static_cast<unsigned long long>(s_evals);
            inner_sum += static_cast<unsigned long long>(it);
            written += static_cast<unsigned long long>(s_written);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && visits) {
        stat_add(a.blkstat, SF_EVALS2, evals);
        stat_add(a.blkstat, SF_VISITS2, visits);
        stat_add(a.blkstat, SF_INNER2, inner_sum);
        stat_add(a.blkstat, SF_WRITTEN2, written);
    }
}

// ---------------------------------------------------------------------------
// STEP 3: whole-grid detection, one workgroup per tile
// ---------------------------------------------------------------------------
template <typename T, int ND, int TX, int TY, int TZ, bool AN>
__global__ __launch_bounds__(kBlock) void k_tile_detect(TileIter<T> a, BatchGeom<T> bg, T eps) {
    using S = Shape<ND, TX, TY, TZ>;
    __shared__ T sphi[S::NL];
    __shared__ uint8_t sl[S::NL];
    __shared__ uint32_t s_key;
    const uint32_t ntag = launch_tag(a);
    for (int t = blockIdx.x; t < bg.ntiles; t += gridDim.x) {
        const Inst<T> g = inst_of(bg, t);
        const int lt = t - g.tile_base;
        const int tx = lt % g.ntx, ty = (lt / g.ntx) % g.nty, tz = lt / (g.ntx * g.nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * (ND == 3 ? TZ : 1);
        if (threadIdx.x == 0) s_key = kNoKey;  // ordered below the staging barrier
        stage<T, ND, TX, TY, TZ>(g, x0, y0, z0, a.phi, a.lab, sphi, sl);
        Owned<T, S::NPT> o;
        own_nodes<T, ND, TX, TY, TZ, AN>(g, x0, y0, z0, a.F, o);
        __syncthreads();
        bool flag = false;
        T low = pos_inf<T>();
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) {
            if (!o.ok[r] || (sl[o.L[r]] & 3u) == L_FIXED) continue;
            const T pt = eval_lds<T, ND, TX, TY, TZ, AN>(sphi, o.L[r], o.H[r], g);
            if (pt < sphi[o.L[r]] - eps) {
                flag = true;
                low = tmin(low, pt);
            }
        }
        if (a.ordered && flag) atomicMin(&s_key, order_key(low));
        if (__syncthreads_or(flag) && threadIdx.x == 0) {
            a.mask_next[t] = kAllFaces;  // one writer: the workgroup of tile t
            if (a.ordered) a.key_next[t] = s_key;
            push_keyed(a, t, ntag, s_key);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// STEP 3: remedy loop on tiles
// ---------------------------------------------------------------------------
// The remedy rule restricted to the tile, on an LDS remedy list: a listed
// node that drops takes the new value; its in-tile neighbours are listed for
// the next iteration when the new value lies below theirs (otherwise their
// update cannot change: the node is not upwind of them), and a face neighbour
// below the halo value marks that face dirty in the tile across it.
// Occupancy matters more than a few spilled registers here: the inner
// iterations are latency-bound, and more resident workgroups hide it (float
// tiles of up to 512 nodes: eight waves per SIMD measured fastest).
template <typename T, int ND, int TX, int TY, int TZ, bool AN>
__global__ __launch_bounds__(kBlock, (sizeof(T) == 4 && Shape<ND, TX, TY, TZ>::NPT <= 2) ? 8 : 1) void k_tile_remedy(
    TileIter<T> a, BatchGeom<T> bg, T eps, int inner) {
    using S = Shape<ND, TX, TY, TZ>;
    __shared__ T sphi[S::NL];
    __shared__ uint8_t sl[S::NL];
    __shared__ T sH[S::NT];
    __shared__ TileLists<S::NT> tl;
    __shared__ int s_len[kSub];
    __shared__ int s_slot;
    __shared__ int s_face;
    __shared__ int s_evals;
    __shared__ int s_written;
    __shared__ uint32_t s_mask;
    __shared__ uint32_t s_key, s_kmin;
    const T inf = pos_inf<T>();
    const uint32_t ntag = launch_tag(a);
    const int n = list_open(a, s_len);
    launch_stats(a, n);
    // ordered mode: k_tile_split has moved this launch's tiles into the work
    // list (the rest went on to the next list)
    const TList src = a.ordered ? a.work : a.cur;
    if (a.ordered) {
        __syncthreads();  // s_len of the current list has been read
        if (threadIdx.x < kSub) s_len[threadIdx.x] = a.work.count[threadIdx.x * kPad];
        if (blockIdx.x == 0 && threadIdx.x < kSub) {
            a.work_zero_count[threadIdx.x * kPad] = 0;
            a.work_zero_fetch[threadIdx.x * kPad] = 0;
        }
        __syncthreads();
    }
    const int k = blockIdx.x & (kSub - 1);
    const int len = s_len[k];
    unsigned long long evals = 0, inner_sum = 0, written = 0, visits = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            const int e = atomicAdd(src.fetch + k * kPad, 1);
            const int tt = e < len ? src.data[static_cast<size_t>(k) * src.cap + e] : -1;
            if (tt >= 0 && a.ordered) {
                s_key = a.key_cur[tt];
                a.key_cur[tt] = kNoKey;
            }
            s_slot = tt;
        }
        __syncthreads();
        const int t = s_slot;
        __syncthreads();
        if (t < 0) break;
        ++visits;
        const Inst<T> g = inst_of(bg, t);
        const int lt = t - g.tile_base;
        const int tx = lt % g.ntx, ty = (lt / g.ntx) % g.nty, tz = lt / (g.ntx * g.nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * (ND == 3 ? TZ : 1);
        const int open = open_bits<ND, TX, TY, TZ>(g, x0, y0, z0);
        uint32_t mask_in = 0;
        if (threadIdx.x == 0) {
            // written by the previous launch; no writer during this one
            mask_in = a.mask_cur[t];
            a.mask_cur[t] = 0u;
            s_kmin = kNoKey;
        }
        stage<T, ND, TX, TY, TZ>(g, x0, y0, z0, a.phi, a.lab, sphi, sl);
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) {
            const int nn = threadIdx.x + r * kBlock;
            if (nn < S::NT) {
                int x, y, z, L;
                node_loc<ND, TX, TY, TZ>(nn, x, y, z, L);
                const bool ok = x0 + x < g.nx && y0 + y < g.ny && z0 + z < g.nz;
                const int G = g.node_base + ((z0 + z) * g.ny + (y0 + y)) * g.nx + (x0 + x);
                sH[nn] = ok ? cell_value<T, AN>(g, a.F[G]) : dead_value<T, AN>();
                tl.flag[0][nn] = 0u;
                tl.flag[1][nn] = 0u;
                tl.dirty[nn] = 0;
            }
        }
        if (threadIdx.x == 0) {
            s_face = 0;
            s_evals = 0;
            s_written = 0;
            s_mask = mask_in;
            tl.cnt[0] = tl.cnt[1] = tl.cnt[2] = 0;
        }
        __syncthreads();
        // initial remedy list: every non-source node on a first visit, else the
        // nodes on the faces whose neighbour tile changed (barrier cells and
        // nodes outside the grid have H = +inf and never change)
        const uint32_t m = s_mask;
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) {
            const int nn = threadIdx.x + r * kBlock;
            if (nn >= S::NT) continue;
            int x, y, z, L;
            node_loc<ND, TX, TY, TZ>(nn, x, y, z, L);
            const int E = edge_bits<ND, TX, TY, TZ>(x, y, z) & open;
            const bool live = cell_live<T, AN>(sH[nn]) && (sl[L] & 3u) != L_FIXED;
            if (live && ((m & kAllFaces) || (E & static_cast<int>(m))))
                tl.list[0][atomicAdd(&tl.cnt[0], 1)] = static_cast<uint16_t>(nn);
        }
        __syncthreads();
        bool pending = false;
        int my_evals = 0, fm = 0;
        T kmin = inf;  // smallest value that crossed a face (order key of the pushes)
        int it = 0;
        for (;; ++it) {
            const int ncur = tl.cnt[it % 3];
            if (ncur == 0) break;
            if (it == inner) {
                pending = true;
                break;
            }
            const int cb = it & 1, nb = cb ^ 1;
            int* ncnt = &tl.cnt[(it + 1) % 3];
            if (threadIdx.x == 0) tl.cnt[(it + 2) % 3] = 0;
            for (int i = threadIdx.x; i < ncur; i += kBlock) {
                const int q = tl.list[cb][i];
                tl.flag[cb][q] = 0u;
                int x, y, z, Lq;
                node_loc<ND, TX, TY, TZ>(q, x, y, z, Lq);
                ++my_evals;
                const T pt = eval_lds<T, ND, TX, TY, TZ, AN>(sphi, Lq, sH[q], g);
                if (pt < sphi[Lq] - eps) {
                    sphi[Lq] = pt;
                    tl.dirty[q] = 1;
                    const int edge = edge_bits<ND, TX, TY, TZ>(x, y, z);
#pragma unroll
                    for (int d = 0; d < 2 * ND; ++d) {
                        const int Ln = Lq + lds_offset<ND, TX, TY, TZ>(d);
                        if (!(pt < sphi[Ln])) continue;  // not upwind of that neighbour
                        if (edge & (1 << d)) {
                            if (open & (1 << d)) {
                                fm |= 1 << d;
                                kmin = tmin(kmin, pt);
                            }
                        } else {
                            const uint8_t lb = sl[Ln];
                            if (!(lb & kOut) && (lb & 3u) != L_FIXED) list_add(tl, nb, ncnt, q + node_step<TX, TY>(d));
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (fm) atomicOr(&s_face, fm);
        if (my_evals) atomicAdd(&s_evals, my_evals);
        if (a.ordered && kmin < inf) atomicMin(&s_kmin, order_key(kmin));
        __syncthreads();
        // scheduling, one lane per target tile (see the update kernel); the
        // targets are read by the next launch, so these atomics may overlap
        // the write-back below
        if (threadIdx.x < 7) {
            const int d = threadIdx.x;
            const int fmask = s_face;
            const uint32_t key = s_kmin;
            if (d == 6) {
                if (pending) {
                    atomicOr(a.mask_next + t, kAllFaces);
                    push_keyed(a, t, ntag, min(key, s_key));
                }
            } else if (d < 2 * ND && (fmask & (1 << d))) {
                const int tn = neighbour_tile(g, t, d);
                atomicOr(a.mask_next + tn, 1u << (d ^ 1));  // the face of tn shared with t
                push_keyed(a, tn, ntag, key);
            }
        }
        int my_written = 0;
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) {
            const int nn = threadIdx.x + r * kBlock;
            if (nn >= S::NT || !tl.dirty[nn]) continue;
            int x, y, z, L;
            node_loc<ND, TX, TY, TZ>(nn, x, y, z, L);
            a.phi[g.node_base + ((z0 + z) * g.ny + (y0 + y)) * g.nx + (x0 + x)] = sphi[L];
            ++my_written;
        }
        if (my_written) atomicAdd(&s_written, my_written);
        __syncthreads();
        if (threadIdx.x == 0) {
            evals += static_cast<unsigned long long>(s_evals);
            inner_sum += static_cast<unsigned long long>(it);
            written += static_cast<unsigned long long>(s_written);
        }
    }
    if (threadIdx.x == 0 && visits) {
        stat_add(a.blkstat, SF_EVALS3, evals);
        stat_add(a.blkstat, SF_VISITS3, visits);
        stat_add(a.blkstat, SF_INNER3, inner_sum);
        stat_add(a.blkstat, SF_WRITTEN3, written);
    }
}

// Ordered remedy: before each remedy launch, one lane per entry of the
// current list sends the tile either to the work list of the launch (its key
// is within the threshold of order_threshold) or on to the next list with its
// key and dirty faces.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_split(TileIter<T> a) {
    __shared__ int s_len[kSub];
    __shared__ int s_thr;
    const uint32_t ntag = launch_tag(a);
    if (threadIdx.x < kSub) s_len[threadIdx.x] = a.cur.count[threadIdx.x * kPad];
    __syncthreads();
    int n = 0;
#pragma unroll
    for (int k = 0; k < kSub; ++k) n += s_len[k];
    if (n == 0) return;
    const int thr = order_threshold(a, n, &s_thr);
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < n; e += gridDim.x * kBlock) {
        int k = 0, i = e;
        while (i >= s_len[k]) i -= s_len[k++];
        const int t = a.cur.data[static_cast<size_t>(k) * a.cur.cap + i];
        const uint32_t key = a.key_cur[t];
        if (key_bin(key) <= thr) {
            const int w = t & (kSub - 1);
            a.work.data[static_cast<size_t>(w) * a.work.cap + atomicAdd(a.work.count + w * kPad, 1)] = t;
        } else {
            a.key_cur[t] = kNoKey;
            const uint32_t mk = a.mask_cur[t];
            a.mask_cur[t] = 0u;
            if (mk) atomicOr(a.mask_next + t, mk);
            push_keyed(a, t, ntag, key);
        }
    }
}

// ---------------------------------------------------------------------------
// STEP 1 helpers
// ---------------------------------------------------------------------------

// Initial tile list: tiles holding a grid neighbour of a source (claimed with
// tag 1).
template <typename T>
__global__ void k_seed_tiles(BatchGeom<T> bg, int nd, int tx_, int ty_, int tz_, SrcBatch<T> b,
                             uint32_t* tstamp, TList out) {
    const int k = threadIdx.x;
    if (k >= b.count) return;
    const Inst<T> g = bg.ninst == 1 ? bg.one : bg.table[b.inst[k]];
    const int i = b.idx[k] - g.node_base;
    const int x = i % g.nx, y = (i / g.nx) % g.ny, z = i / (g.nx * g.ny);
    const int dx[6] = {-1, 1, 0, 0, 0, 0}, dy[6] = {0, 0, -1, 1, 0, 0}, dz[6] = {0, 0, 0, 0, -1, 1};
    for (int d = 0; d < 2 * nd; ++d) {
        const int X = x + dx[d], Y = y + dy[d], Z = z + dz[d];
        if (X < 0 || X >= g.nx || Y < 0 || Y >= g.ny || Z < 0 || Z >= g.nz) continue;
        push_tile(out, tstamp, g.tile_base + ((Z / tz_) * g.nty + (Y / ty_)) * g.ntx + (X / tx_), 1u);
    }
}

// Initial tile list holding every tile (used when there are many sources):
// tile t is entry t / kSub of sub-list t % kSub.
__global__ void k_seed_all_tiles(int ntiles, uint32_t* tstamp, TList out) {
    for (int t = blockIdx.x * kBlock + threadIdx.x; t < ntiles; t += gridDim.x * kBlock) {
        tstamp[t] = 1u;
        out.data[static_cast<size_t>(t & (kSub - 1)) * out.cap + (t / kSub)] = t;
    }
    if (blockIdx.x == 0 && threadIdx.x < kSub)
        out.count[threadIdx.x * kPad] = (ntiles - static_cast<int>(threadIdx.x) + kSub - 1) / kSub;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct TileWs {
    Ctl* ctl;
    unsigned long long* blkstat;
    uint8_t* lab;
    uint32_t* tstamp;
    uint32_t* tmask;    // two arrays of ntiles dirty-face masks (by launch parity)
    int* data[2];       // two list buffers (alternating)
    int* counters;      // 3 rotating sets of {count[kSub*kPad], fetch[kSub*kPad]}, then
                        // 3 rotating order-key histograms of kBins counts
    uint32_t* keys;     // two arrays of ntiles order keys (by launch parity)
    int* work[2];       // ordered remedy: work lists (by launch parity) ...
    int* work_counters; // ... and their {count, fetch} sets
    void* table;        // instance table (batches of more than one instance)
    int* tile_inst;     // instance of every tile (idem)
    int cap;
    size_t bytes;
    int* count_of(int set) const { return counters + set * 2 * kSub * kPad; }
    int* fetch_of(int set) const { return counters + set * 2 * kSub * kPad + kSub * kPad; }
    unsigned* hist_of(int set) const {
        return reinterpret_cast<unsigned*>(counters + 3 * 2 * kSub * kPad) + set * kBins;
    }
};

constexpr size_t kCounterBytes = (3 * 2 * kSub * kPad + 3 * kBins) * sizeof(int);
constexpr size_t kWorkCounterBytes = 2 * 2 * kSub * kPad * sizeof(int);

// A sub-list can receive every tile (tiles are deduplicated per list).
TileWs tile_layout(char* base, int64_t n, int64_t ntiles, size_t ninst, size_t inst_bytes) {
    TileWs w{};
    size_t off = 0;
    auto take = [&](size_t b) {
        char* p = base ? base + off : nullptr;
        off = align_up(off + b, 256);
        return p;
    };
    w.cap = static_cast<int>(ntiles + 64);
    w.ctl = reinterpret_cast<Ctl*>(take(sizeof(Ctl)));
    w.blkstat = reinterpret_cast<unsigned long long*>(take(8 * static_cast<size_t>(kStatFields) * kMaxStatBlocks));
    w.lab = reinterpret_cast<uint8_t*>(take(static_cast<size_t>(n)));
    w.tstamp = reinterpret_cast<uint32_t*>(take(4 * static_cast<size_t>(ntiles)));
    w.tmask = reinterpret_cast<uint32_t*>(take(8 * static_cast<size_t>(ntiles)));
    w.counters = reinterpret_cast<int*>(take(kCounterBytes));
    w.keys = reinterpret_cast<uint32_t*>(take(8 * static_cast<size_t>(ntiles)));
    for (int k = 0; k < 2; ++k) w.work[k] = reinterpret_cast<int*>(take(4 * static_cast<size_t>(w.cap) * kSub));
    w.work_counters = reinterpret_cast<int*>(take(kWorkCounterBytes));
    for (int k = 0; k < 2; ++k) w.data[k] = reinterpret_cast<int*>(take(4 * static_cast<size_t>(w.cap) * kSub));
    if (ninst > 1) {
        w.table = take(inst_bytes * ninst);
        w.tile_inst = reinterpret_cast<int*>(take(4 * static_cast<size_t>(ntiles)));
    }
    w.bytes = off;
    return w;
}

template <typename T, int ND, int TX, int TY, int TZ, bool AN>
struct TileKernels {
    static hipError_t update(const TileIter<T>& a, const BatchGeom<T>& g, T eps, int inner, hipStream_t s) {
        hipLaunchKernelGGL((k_tile_update<T, ND, TX, TY, TZ, AN>), dim3(GT), dim3(kBlock), 0, s, a, g, eps, inner);
        return hipGetLastError();
    }
    static hipError_t detect(const TileIter<T>& a, const BatchGeom<T>& g, T eps, hipStream_t s) {
        hipLaunchKernelGGL((k_tile_detect<T, ND, TX, TY, TZ, AN>), dim3(GT), dim3(kBlock), 0, s, a, g, eps);
        return hipGetLastError();
    }
    static hipError_t remedy(const TileIter<T>& a, const BatchGeom<T>& g, T eps, int inner, hipStream_t s) {
        hipLaunchKernelGGL((k_tile_remedy<T, ND, TX, TY, TZ, AN>), dim3(GT), dim3(kBlock), 0, s, a, g, eps, inner);
        return hipGetLastError();
    }
};

template <typename T>
struct TileOps {
    hipError_t (*update)(const TileIter<T>&, const BatchGeom<T>&, T, int, hipStream_t) = nullptr;
    hipError_t (*detect)(const TileIter<T>&, const BatchGeom<T>&, T, hipStream_t) = nullptr;
    hipError_t (*remedy)(const TileIter<T>&, const BatchGeom<T>&, T, int, hipStream_t) = nullptr;
};

template <typename T, int ND, int TX, int TY, int TZ, bool AN = false>
TileOps<T> ops_of() {
    TileOps<T> k;
    k.update = &TileKernels<T, ND, TX, TY, TZ, AN>::update;
    k.detect = &TileKernels<T, ND, TX, TY, TZ, AN>::detect;
    k.remedy = &TileKernels<T, ND, TX, TY, TZ, AN>::remedy;
    return k;
}

// Supported tile shapes (z, y, x); per-axis spacing only with the default
// shapes (32 x 32 in 2D, 8^3 in 3D).
template <typename T>
bool select_ops(int nd, const TileCfg& c, bool aniso, TileOps<T>& k) {
    if (aniso) {
        if (nd == 2 && c.ty == 32 && c.tx == 32) return k = ops_of<T, 2, 32, 32, 1, true>(), true;
        if (nd == 3 && c.tz == 8 && c.ty == 8 && c.tx == 8) return k = ops_of<T, 3, 8, 8, 8, true>(), true;
        return false;
    }
    if (nd == 2) {
        if (c.ty == 16 && c.tx == 16) return k = ops_of<T, 2, 16, 16, 1>(), true;
        if (c.ty == 32 && c.tx == 32) return k = ops_of<T, 2, 32, 32, 1>(), true;
        if (c.ty == 16 && c.tx == 64) return k = ops_of<T, 2, 64, 16, 1>(), true;
        if (c.ty == 8 && c.tx == 32) return k = ops_of<T, 2, 32, 8, 1>(), true;
        if (c.ty == 64 && c.tx == 64) return k = ops_of<T, 2, 64, 64, 1>(), true;
        return false;
    }
    if (c.tz == 8 && c.ty == 8 && c.tx == 8) return k = ops_of<T, 3, 8, 8, 8>(), true;
    if (c.tz == 4 && c.ty == 8 && c.tx == 8) return k = ops_of<T, 3, 8, 8, 4>(), true;
    if (c.tz == 4 && c.ty == 4 && c.tx == 16) return k = ops_of<T, 3, 16, 4, 4>(), true;
    if (c.tz == 8 && c.ty == 8 && c.tx == 16) return k = ops_of<T, 3, 16, 8, 8>(), true;
    if (c.tz == 16 && c.ty == 16 && c.tx == 16) return k = ops_of<T, 3, 16, 16, 16>(), true;
    return false;
}

}  // namespace

TileCfg pick_tile(int nd, const eik_options& o) {
    TileCfg c{o.tile[2], o.tile[1], o.tile[0]};
    if (nd == 2) {
        c.tz = 1;
        if (c.tx == 0 || c.ty == 0) c = TileCfg{32, 32, 1};
    } else if (c.tx == 0 || c.ty == 0 || c.tz == 0) {
        c = TileCfg{8, 8, 8};
    }
    return c;
}

void batch_add(Batch& b, int nx, int ny, int nz, double h, const double* d) {
    HostInst e{};
    e.nx = nx;
    e.ny = ny;
    e.nz = nz;
    e.ntx = (nx + b.cfg.tx - 1) / b.cfg.tx;
    e.nty = (ny + b.cfg.ty - 1) / b.cfg.ty;
    e.ntz = (nz + b.cfg.tz - 1) / b.cfg.tz;
    e.node_base = static_cast<int>(b.n);
    e.tile_base = static_cast<int>(b.ntiles);
    e.h = h;
    e.aniso = d ? 1 : 0;
    for (int k = 0; k < 3; ++k) e.d[k] = d ? d[k] : 0.0;
    b.inst.push_back(e);
    b.n += static_cast<int64_t>(nx) * ny * nz;
    b.ntiles += static_cast<int64_t>(e.ntx) * e.nty * e.ntz;
}

Batch with_tiles(const Batch& b, const TileCfg& c) {
    Batch r;
    r.nd = b.nd;
    r.cfg = c;
    for (const HostInst& e : b.inst) batch_add(r, e.nx, e.ny, e.nz, e.h, e.aniso ? e.d : nullptr);
    r.src = b.src;
    r.src_inst = b.src_inst;
    return r;
}

size_t tile_workspace_bytes(const Batch& b, size_t esz) {
    const size_t ib = esz == 8 ? sizeof(Inst<double>) : sizeof(Inst<float>);
    return tile_layout(nullptr, b.n, b.ntiles, b.inst.size(), ib).bytes;
}

template <typename T>
eik_status solve_tile(const Batch& b, const T* F, double eps, T* phi, const eik_options& o, char* ws,
                      hipStream_t s, eik_stats* st) {
    const bool async = (o.flags & EIK_FLAG_ASYNC) != 0;
    const TileCfg c = b.cfg;
    TileOps<T> k;
    if (!select_ops<T>(b.nd, c, b.inst[0].aniso != 0, k))
        return fail(EIK_ERR_INVALID_ARGUMENT, b.inst[0].aniso ? "per-axis spacing needs the default tile shape"
                                                              : "unsupported tile shape");
    TileWs w = tile_layout(ws, b.n, b.ntiles, b.inst.size(), sizeof(Inst<T>));
    const int64_t cap = o.max_iters > 0 ? o.max_iters : 4 * b.n + 64;
    const int inner = o.inner_iters > 0 ? o.inner_iters : 4 * (c.tx + c.ty + c.tz);
    const int ntiles = static_cast<int>(b.ntiles);
    int64_t launched = 0;

    Profiler prof;
    prof.start((o.flags & EIK_FLAG_PROFILE) != 0, s);
    const size_t blk_bytes = 8 * static_cast<size_t>(kStatFields) * kMaxStatBlocks;
    BatchGeom<T> geom;
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return upload_batch_geom<T>(b, w.table, w.tile_inst, s, geom, launched); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_ctl_init(w.ctl, s); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_zero_words(w.blkstat, blk_bytes, s); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_init<T>(F, phi, w.lab, nullptr, static_cast<int>(b.n), w.ctl, s); }));
    // tile stamps and dirty-face masks are adjacent: clear both
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
        return launch_zero_words(w.tstamp, 4 * (static_cast<size_t>(w.tmask - w.tstamp) + 2 * static_cast<size_t>(ntiles)), s);
    }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_zero_words(w.counters, kCounterBytes, s); }));
    launched += 5;
    const bool ordered = (o.flags & EIK_FLAG_FIFO_REMEDY) == 0;
    if (ordered) {
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_fill_words(w.keys, 2 * static_cast<size_t>(ntiles), kNoKey, s); }));
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_zero_words(w.work_counters, kWorkCounterBytes, s); }));
        launched += 2;
    }
    std::vector<SrcBatch<T>> batches;
    for (size_t q = 0; q < b.src.size(); q += kMaxSrcBatch) {
        SrcBatch<T> sb{};
        sb.count = static_cast<int>(std::min<size_t>(kMaxSrcBatch, b.src.size() - q));
        for (int j = 0; j < sb.count; ++j) {
            sb.idx[j] = b.src[q + j].first;
            sb.inst[j] = b.src_inst[q + j];
            sb.val[j] = static_cast<T>(b.src[q + j].second);
        }
        batches.push_back(sb);
    }
    for (auto& sb : batches)
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_seed<T>(phi, w.lab, sb, s); }));
    launched += static_cast<int64_t>(batches.size());
    auto list_of = [&](int64_t t) {
        TList L;
        L.data = w.data[t & 1];
        L.count = w.count_of(static_cast<int>(t % 3));
        L.fetch = w.fetch_of(static_cast<int>(t % 3));
        L.cap = w.cap;
        return L;
    };
    if (batches.size() <= 8) {
        // tiles next to the sources
        for (auto& sb : batches)
            HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
                hipLaunchKernelGGL(k_seed_tiles<T>, dim3(1), dim3(kMaxSrcBatch), 0, s, geom, b.nd, c.tx, c.ty, c.tz,
                                   sb, w.tstamp, list_of(0));
                return hipGetLastError();
            }));
        launched += static_cast<int64_t>(batches.size());
    } else {
        // many sources: start from every tile; tiles with nothing to do drop out
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
            hipLaunchKernelGGL(k_seed_all_tiles, dim3(std::min((ntiles + kBlock - 1) / kBlock, 1024)), dim3(kBlock),
                               0, s, ntiles, w.tstamp, list_of(0));
            return hipGetLastError();
        }));
        launched += 1;
    }

    const T eT = static_cast<T>(eps);
    int64_t gl = 0;  // launches in the tag chain so far (selects the tag slot)
    // launch t drains list t and fills list t + 1; lists alternate two buffers
    // and three counter sets (the set of list t + 2 is cleared by launch t)
    auto iter_args = [&](int64_t t, int phase) {
        TileIter<T> a{};
        a.F = F;
        a.phi = phi;
        a.lab = w.lab;
        a.tstamp = w.tstamp;
        a.mask_cur = w.tmask + static_cast<size_t>(t & 1) * ntiles;
        a.mask_next = w.tmask + static_cast<size_t>((t + 1) & 1) * ntiles;
        a.key_cur = w.keys + static_cast<size_t>(t & 1) * ntiles;
        a.key_next = w.keys + static_cast<size_t>((t + 1) & 1) * ntiles;
        a.hist_cur = w.hist_of(static_cast<int>(t % 3));
        a.hist_next = w.hist_of(static_cast<int>((t + 1) % 3));
        a.hist_zero = w.hist_of(static_cast<int>((t + 2) % 3));
        a.ordered = (ordered && phase == 1) ? 1 : 0;
        auto work_of = [&](int64_t u) {
            TList L;
            L.data = w.work[u & 1];
            L.count = w.work_counters + (u & 1) * 2 * kSub * kPad;
            L.fetch = L.count + kSub * kPad;
            L.cap = w.cap;
            return L;
        };
        a.work = work_of(t);
        a.work_zero_count = work_of(t + 1).count;
        a.work_zero_fetch = work_of(t + 1).fetch;
        a.cur = list_of(t);
        a.next = list_of(t + 1);
        a.zero_count = w.count_of(static_cast<int>((t + 2) % 3));
        a.zero_fetch = w.fetch_of(static_cast<int>((t + 2) % 3));
        a.ctl = w.ctl;
        a.blkstat = w.blkstat;
        a.tag_slot = static_cast<int>((gl + t) & 1);
        a.phase = phase;
        a.first = (phase == 1 && t == 0) ? 1 : 0;
        return a;
    };
    auto counts = [&](int64_t t) { return w.count_of(static_cast<int>(t % 3)); };

    int64_t n2 = 0;
    eik_status rc = run_loop(
        [&](int64_t t) {
            return timed(prof, EIK_KERNEL_UPDATE, [&] { return k.update(iter_args(t, 0), geom, eT, inner, s); });
        },
        counts, kSub * kPad, cap, async, s, &n2);
    gl += n2;
    launched += n2;
    if (rc == EIK_OK && !(o.flags & EIK_FLAG_SKIP_REMEDY)) {
        // detection fills list 0 of the remedy loop
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_zero_words(w.counters, kCounterBytes, s); }));
        TileIter<T> d = iter_args(0, 1);  // only `next` (list 0), its masks and the tag are used
        d.next = list_of(0);
        d.mask_next = w.tmask;  // read by remedy launch 0
        d.key_next = w.keys;
        d.hist_next = w.hist_of(0);
        d.first = 0;
        d.tag_slot = static_cast<int>(gl & 1);
        HIP_TRY(timed(prof, EIK_KERNEL_DETECT, [&] { return k.detect(d, geom, eT, s); }));
        gl += 1;
        launched += 2;
        int64_t n3 = 0;
        const int split_blocks = static_cast<int>(std::min<int64_t>((b.ntiles + kBlock - 1) / kBlock, 1024));
        rc = run_loop(
            [&](int64_t t) {
                const TileIter<T> a = iter_args(t, 1);
                if (ordered) {
                    const hipError_t e = timed(prof, EIK_KERNEL_OTHER, [&] {
                        hipLaunchKernelGGL(k_tile_split<T>, dim3(split_blocks), dim3(kBlock), 0, s, a);
                        return hipGetLastError();
                    });
                    if (e != hipSuccess) return e;
                }
                return timed(prof, EIK_KERNEL_REMEDY, [&] { return k.remedy(a, geom, eT, inner, s); });
            },
            counts, kSub * kPad, cap, async, s, &n3);
        launched += (ordered ? 2 : 1) * n3;
    }
    if (async) return rc;
    HostSlots& hs = host_slots();
    HIP_TRY(hipMemcpyAsync(hs.ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hs.blk, w.blkstat, blk_bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hs.ctl->err & 1) return fail(EIK_ERR_INVALID_ARGUMENT, "F has negative or non-finite values");
    if (st) {
        *st = eik_stats{};
        st->step2_iters = static_cast<int64_t>(hs.ctl->iters2);
        st->step3_iters = static_cast<int64_t>(hs.ctl->iters3);
        st->evals_step2 = static_cast<int64_t>(blk_sum(hs.blk, SF_EVALS2, kMaxStatBlocks));
        st->evals_detect = (o.flags & EIK_FLAG_SKIP_REMEDY) ? 0 : b.n - static_cast<int64_t>(b.src.size());
        st->evals_remedy = static_cast<int64_t>(blk_sum(hs.blk, SF_EVALS3, kMaxStatBlocks));
        st->remedy_initial = static_cast<int64_t>(hs.ctl->remedy_init);
        st->max_active = static_cast<int64_t>(hs.ctl->max_active);
        st->launches = launched;
        st->tile_visits_step2 = static_cast<int64_t>(blk_sum(hs.blk, SF_VISITS2, kMaxStatBlocks));
        st->tile_visits_step3 = static_cast<int64_t>(blk_sum(hs.blk, SF_VISITS3, kMaxStatBlocks));
        st->inner_step2 = static_cast<int64_t>(blk_sum(hs.blk, SF_INNER2, kMaxStatBlocks));
        st->inner_step3 = static_cast<int64_t>(blk_sum(hs.blk, SF_INNER3, kMaxStatBlocks));
        st->written_step2 = static_cast<int64_t>(blk_sum(hs.blk, SF_WRITTEN2, kMaxStatBlocks));
        st->written_step3 = static_cast<int64_t>(blk_sum(hs.blk, SF_WRITTEN3, kMaxStatBlocks));
        HIP_TRY(prof.collect(st));
    }
    return rc;
}

template eik_status solve_tile<float>(const Batch&, const float*, double, float*, const eik_options&, char*,
                                      hipStream_t, eik_stats*);
template eik_status solve_tile<double>(const Batch&, const double*, double, double*, const eik_options&, char*,
                                       hipStream_t, eik_stats*);

}  // namespace eik
