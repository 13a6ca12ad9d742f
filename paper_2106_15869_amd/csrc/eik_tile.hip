// Tile-activated IFIM for gfx950.
//
// The grid is cut into tiles of TZ x TY x TX nodes.  A launch drains a list
// of tiles with persistent workgroups (256 lanes, four wave64), one tile
// visit at a time.  A visit stages the tile's values, labels and speeds plus
// a one-cell halo in LDS (one round of global loads), runs the node rules of
// Algorithm 2 for several inner iterations on an LDS list of nodes without
// touching HBM, writes back what changed and schedules the tiles that have
// to be visited next (eik_sched.hpp: sub-list queues, stamps, order keys).
//
//   update step (STEP 2): FAR nodes with F > 0 next to a converged or fixed
//     node become active; active nodes take phi~ = G_i(phi); a node whose
//     value no longer moves (phi - phi~ <= eps) converges and activates its FAR
//     neighbours -- no convergence check of those neighbours (Section 3.3).
//     A node converging on a tile face schedules the tile across that face; a
//     tile that still holds active nodes schedules itself.  In 3D the
//     workgroups that find no update tile in a launch run early remedy
//     visits (below) on tiles whose update work is done.
//   remedy detection (STEP 3, first part): one dense pass over all tiles;
//     a tile with any node whose phi~ < phi - eps enters the remedy list.
//   remedy loop (STEP 3): the remedy rule of Section 3.1.2 restricted to the
//     tile: recompute the listed nodes, take the drops, list the in-tile
//     neighbours below which a dropped value now lies for the next inner
//     iteration, until the list is empty.  A tile enters with all nodes
//     listed (first visit) or with the nodes on the faces whose neighbour tile
//     changed; a drop on a tile face marks that face dirty in the tile across
//     it and schedules it with the dropped value as its order key.  By
//     default (ordered remedy) k_tile_split hands each launch only the
//     lowest-key tiles of the list.
// Values are updated in place within an inner iteration (a read racing with
// an update sees either value, both upper bounds of the solution); tiles of
// one launch see each other's values only through the halo staged at the
// start of a visit.
#include <utility>
#include <vector>

#include "eik_device.hpp"
#include "eik_host.hpp"
#include "eik_seglist.hpp"
#include "eik_batch.hpp"
#include "eik_sched.hpp"
#include "eik_tile.hpp"

namespace eik {

namespace {

// LDS label byte: bits 0-1 state, bit 2 passable (F > 0), bit 3 outside grid.
constexpr uint8_t kPass = 4u, kOut = 8u;

template <typename T>
struct TileIter : Sched {
    const T* F;
    T* phi;
    uint8_t* lab;
    const T* cells;  // tile-major cell values (k_build_cells), read by detection and the remedy
    // early remedy visits during the update step (3D): per tile whether its
    // last update visit left no active node, and the update visits finished
    // in this launch and in the next one (cleared by this one)
    uint8_t* done;
    int* fin;
    int* fin_clear;
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
// The tile-major cell array marks a fixed (source) node with -1, a value no
// cell_value takes.
template <typename T>
__device__ __forceinline__ T fixed_cell() {
    return T(-1);
}
// whether a cell-array entry belongs to a node the remedy may change
template <typename T, bool AN>
__device__ __forceinline__ bool cell_free(T v) {
    return cell_live<T, AN>(v) && !(v < T(0));
}

// Global index of in-tile node n (clamped into the grid, so that it can be
// loaded unconditionally) and whether the node lies in the grid.
template <typename T, int ND, int TX, int TY, int TZ>
__device__ __forceinline__ int owned_index(const Inst<T>& g, int x0, int y0, int z0, int n, bool& ok) {
    using S = Shape<ND, TX, TY, TZ>;
    const int x = n % TX, y = (n / TX) % TY, z = ND == 3 ? n / (TX * TY) : 0;
    const int gx = x0 + x, gy = y0 + y, gz = z0 + z;
    ok = n < S::NT && gx < g.nx && gy < g.ny && gz < g.nz;
    return g.node_base + (min(gz, g.nz - 1) * g.ny + min(gy, g.ny - 1)) * g.nx + min(gx, g.nx - 1);
}

// F of the nodes a lane owns (n = threadIdx.x + r * kBlock), loaded before
// the staging so that both are in flight together.
template <typename T, int ND, int TX, int TY, int TZ>
__device__ __forceinline__ void load_owned_F(const Inst<T>& g, int x0, int y0, int z0, const T* F,
                                             T (&f)[Shape<ND, TX, TY, TZ>::NPT]) {
    using S = Shape<ND, TX, TY, TZ>;
#pragma unroll
    for (int r = 0; r < S::NPT; ++r) {
        bool ok;
        f[r] = F[owned_index<T, ND, TX, TY, TZ>(g, x0, y0, z0, threadIdx.x + r * kBlock, ok)];
    }
}

// Stage the tile and its halo: values (+inf outside) and labels (kOut outside).
// Addresses are clamped into the grid, so every global load of a lane is
// issued unconditionally, before its first LDS store (one memory round trip).
// Without HALO_LABELS only the tile's own labels are loaded (the halo's are
// set to 0, or kOut outside the grid): the detection pass and the remedy read
// labels of in-tile nodes only, and a halo row of labels is a cache line for
// ten bytes.
// With LABELS false no labels are loaded or stored (sl may be null).
template <typename T, int ND, int TX, int TY, int TZ, bool HALO_LABELS = true, bool LABELS = true>
__device__ __forceinline__ void stage(const Inst<T>& g, int x0, int y0, int z0, const T* phi,
                                      const uint8_t* lab, T* sphi, uint8_t* sl) {
    using S = Shape<ND, TX, TY, TZ>;
    constexpr int NIT = (S::NL + kBlock - 1) / kBlock;
    const T inf = pos_inf<T>();
    T v[NIT];
    uint8_t l[NIT];
    bool in[NIT];
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
        const int q = min(static_cast<int>(threadIdx.x) + j * kBlock, S::NL - 1);
        const int lx = q % S::LX;
        const int ly = (q / S::LX) % S::LY;
        const int lz = q / (S::LX * S::LY);
        const int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = ND == 3 ? z0 + lz - 1 : 0;
        in[j] = gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz;
        const int cx = min(max(gx, 0), g.nx - 1), cy = min(max(gy, 0), g.ny - 1), cz = min(max(gz, 0), g.nz - 1);
        const int G = g.node_base + (cz * g.ny + cy) * g.nx + cx;
        v[j] = phi[G];
        const bool inner = lx >= 1 && lx <= TX && ly >= 1 && ly <= TY && (ND == 2 || (lz >= 1 && lz <= TZ));
        l[j] = LABELS && (HALO_LABELS || inner) ? lab[G] : uint8_t(0);
    }
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
        const int q = threadIdx.x + j * kBlock;
        if (q < S::NL) {
            sphi[q] = in[j] ? v[j] : inf;
            if (LABELS) sl[q] = in[j] ? l[j] : static_cast<uint8_t>(kOut);
        }
    }
}

// The neighbour values of LDS node L in direction order (-x, +x, -y, +y, -z, +z).
template <typename T, int ND, int TX, int TY, int TZ>
__device__ __forceinline__ void load_nb(const T* sphi, int L, T (&nb)[2 * ND]) {
#pragma unroll
    for (int d = 0; d < 2 * ND; ++d) nb[d] = sphi[L + lds_offset<ND, TX, TY, TZ>(d)];
}

// G_i from the neighbour values (+inf outside the grid).
// v is the node's H = h / F (isotropic) or its speed F (AN: per-axis spacing,
// H_k = spacing_k / F); see cell_value.
template <typename T, int ND, bool AN>
__device__ __forceinline__ T eval_nb(const T (&nb)[2 * ND], T v, const Inst<T>& g) {
    const T inf = pos_inf<T>();
    const T ax = tmin(nb[0], nb[1]);
    const T ay = tmin(nb[2], nb[3]);
    if (AN) {
        if (!(v > T(0))) return inf;
        if (ND == 2) return godunov_aniso<T, 2>(ay, ax, inf, g.d[0] / v, g.d[1] / v, inf);
        const T az = tmin(nb[4], nb[5]);
        return godunov_aniso<T, 3>(az, ay, ax, g.d[0] / v, g.d[1] / v, g.d[2] / v);
    }
    if (ND == 2) return godunov<T, 2>(ay, ax, inf, v);
    const T az = tmin(nb[4], nb[5]);
    return godunov<T, 3>(az, ay, ax, v);
}

// G_i from the LDS tile (halo holds +inf outside the grid).
template <typename T, int ND, int TX, int TY, int TZ, bool AN>
__device__ __forceinline__ T eval_lds(const T* sphi, int L, T v, const Inst<T>& g) {
    T nb[2 * ND];
    load_nb<T, ND, TX, TY, TZ>(sphi, L, nb);
    return eval_nb<T, ND, AN>(nb, v, g);
}




// ---------------------------------------------------------------------------
// A remedy visit (shared by the remedy launches and, in 3D, the early remedy
// visits of the update step)
// ---------------------------------------------------------------------------
// LDS of a remedy visit.
template <typename T, int NT>
struct RemedyLds {
    T* sphi;           // values with the one-cell halo
    T* sH;             // the tile's cell values
    TileLists<NT>* tl;
    uint32_t* mask;    // dirty faces the visit starts from
    int* face;         // faces a drop crossed
    int* evals;        // local-solver evaluations
    uint32_t* kmin;    // ordered: key of the smallest value that crossed a face (the caller sets kNoKey)
    int* stop;         // POLL: lane 0's stop answer
    int* written;      // values written back, or null (not counted)
};

// The remedy rule on tile t at (x0, y0, z0): stage its values with the halo
// and its cell values, list the free nodes to recheck (all of them for
// kAllFaces in the dirty faces, else those on the dirty faces), and iterate
// until the list is empty, `inner` iterations ran or (POLL) poll() reached
// stop_at (pending: nodes were still listed).  Lane 0 issues poll() every
// other iteration and reads its value one iteration later, so the load's
// latency hides behind an iteration instead of holding the workgroup.
// The dirty faces are *s.mask, or lane 0's mask_in when set_mask.  Leaves the
// new values in sphi with tl->dirty set for the changed nodes, and the
// crossed faces, evaluations and (ordered) the crossing key in LDS.  Returns
// the iterations run.
template <typename T, int ND, int TX, int TY, int TZ, bool AN, bool POLL, typename Poll>
__device__ __forceinline__ int remedy_visit(const T* cells, const T* phi, const Inst<T>& g, int t, int x0, int y0,
                                            int z0, int open, T eps, int inner, bool ordered, uint32_t mask_in,
                                            bool set_mask, const RemedyLds<T, Shape<ND, TX, TY, TZ>::NT>& s,
                                            bool& pending, Poll poll, int stop_at) {
    using S = Shape<ND, TX, TY, TZ>;
    const T inf = pos_inf<T>();
    TileLists<S::NT>& tl = *s.tl;
    T* sphi = s.sphi;
    T hv[S::NPT];
#pragma unroll
    for (int r = 0; r < S::NPT; ++r) {
        const int nn = min(static_cast<int>(threadIdx.x) + r * kBlock, S::NT - 1);
        hv[r] = cells[static_cast<size_t>(t) * S::NT + nn];
    }
    stage<T, ND, TX, TY, TZ, false, false>(g, x0, y0, z0, phi, nullptr, sphi, nullptr);
#pragma unroll
    for (int r = 0; r < S::NPT; ++r) {
        const int nn = threadIdx.x + r * kBlock;
        if (nn < S::NT) {
            s.sH[nn] = hv[r];
            tl.flag[0][nn] = 0u;
            tl.flag[1][nn] = 0u;
            tl.dirty[nn] = 0;
        }
    }
    if (threadIdx.x == 0) {
        *s.face = 0;
        *s.evals = 0;
        if (s.written) *s.written = 0;
        if (POLL) *s.stop = 0;
        if (set_mask) *s.mask = mask_in;
        tl.cnt[0] = tl.cnt[1] = tl.cnt[2] = 0;
    }
    __syncthreads();
    // initial remedy list: every non-source node on a first visit, else the
    // nodes on the faces whose neighbour tile changed (barrier cells and
    // nodes outside the grid have H = +inf and never change)
    const uint32_t m = *s.mask;
#pragma unroll
    for (int r = 0; r < S::NPT; ++r) {
        const int nn = threadIdx.x + r * kBlock;
        if (nn >= S::NT) continue;
        int x, y, z, L;
        node_loc<ND, TX, TY, TZ>(nn, x, y, z, L);
        const int E = edge_bits<ND, TX, TY, TZ>(x, y, z) & open;
        if (cell_free<T, AN>(s.sH[nn]) && ((m & kAllFaces) || (E & static_cast<int>(m))))
            tl.list[0][atomicAdd(&tl.cnt[0], 1)] = static_cast<uint16_t>(nn);
    }
    __syncthreads();
    pending = false;
    int my_evals = 0, fm = 0;
    T kmin = inf;  // smallest value that crossed a face (order key of the pushes)
    int polled = 0;  // lane 0 (POLL): the value of the last poll()
    int it = 0;
    for (;; ++it) {
        const int ncur = tl.cnt[it % 3];
        if (ncur == 0) break;
        if (it == inner || (POLL && *s.stop)) {
            pending = true;
            break;
        }
        const int cb = it & 1, nb = cb ^ 1;
        int* ncnt = &tl.cnt[(it + 1) % 3];
        if (threadIdx.x == 0) {
            tl.cnt[(it + 2) % 3] = 0;
            if (POLL) {
                if (it & 1) polled = poll();
                else if (it > 0) *s.stop = polled >= stop_at ? 1 : 0;
            }
        }
        for (int i = threadIdx.x; i < ncur; i += kBlock) {
            const int q = tl.list[cb][i];
            tl.flag[cb][q] = 0u;
            int x, y, z, Lq;
            node_loc<ND, TX, TY, TZ>(q, x, y, z, Lq);
            ++my_evals;
            const T hq = s.sH[q];
            T nv[2 * ND];
            load_nb<T, ND, TX, TY, TZ>(sphi, Lq, nv);
            const T pt = eval_nb<T, ND, AN>(nv, hq, g);
            // a listed node that may not change (a fixed or barrier node
            // appended by a neighbour) is skipped here
            if (cell_free<T, AN>(hq) && pt < sphi[Lq] - eps) {
                sphi[Lq] = pt;
                tl.dirty[q] = 1;
                // the new value reaches the neighbours above it; the values
                // read for the solve are never below the current ones, so a
                // neighbour that dropped meanwhile may be listed once more
                // (an extra evaluation) but none is missed
                int up = 0;
#pragma unroll
                for (int d = 0; d < 2 * ND; ++d) up |= pt < nv[d] ? 1 << d : 0;
                const int edge = edge_bits<ND, TX, TY, TZ>(x, y, z);
                if constexpr (ND == 2) {
                    const int face = up & edge & open;
                    if (face) {
                        fm |= face;
                        kmin = tmin(kmin, pt);
                    }
                    // 2D: claim the in-tile neighbours' flags together (an OR
                    // of 0 on the node's own flag for the other directions
                    // changes nothing), then reserve a slot per claim won.
                    // In 3D this was slower (six LDS atomics per changed node
                    // where about three are needed).
                    const int in = up & ~edge;
                    uint32_t prev[2 * ND];
#pragma unroll
                    for (int d = 0; d < 2 * ND; ++d) {
                        const bool c = in & (1 << d);
                        prev[d] = atomicOr(&tl.flag[nb][c ? q + node_step<TX, TY>(d) : q], c ? 1u : 0u);
                    }
#pragma unroll
                    for (int d = 0; d < 2 * ND; ++d)
                        if ((in & (1 << d)) && prev[d] == 0u)
                            tl.list[nb][atomicAdd(ncnt, 1)] = static_cast<uint16_t>(q + node_step<TX, TY>(d));
                } else {
#pragma unroll
                    for (int d = 0; d < 2 * ND; ++d) {
                        if (!(up & (1 << d))) continue;
                        if (edge & (1 << d)) {
                            if (open & (1 << d)) {
                                fm |= 1 << d;
                                kmin = tmin(kmin, pt);
                            }
                        } else {
                            list_add(tl, nb, ncnt, q + node_step<TX, TY>(d));
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (fm) atomicOr(s.face, fm);
    if (my_evals) atomicAdd(s.evals, my_evals);
    if (ordered && kmin < inf) atomicMin(s.kmin, order_key(kmin));
    __syncthreads();
    return it;
}

// Write back the values a remedy visit changed (and count them).
template <typename T, int ND, int TX, int TY, int TZ>
__device__ __forceinline__ void remedy_write_back(T* phi, const Inst<T>& g, int x0, int y0, int z0,
                                                  const RemedyLds<T, Shape<ND, TX, TY, TZ>::NT>& s) {
    using S = Shape<ND, TX, TY, TZ>;
    int my_written = 0;
#pragma unroll
    for (int r = 0; r < S::NPT; ++r) {
        const int nn = threadIdx.x + r * kBlock;
        if (nn >= S::NT || !s.tl->dirty[nn]) continue;
        int x, y, z, L;
        node_loc<ND, TX, TY, TZ>(nn, x, y, z, L);
        phi[g.node_base + ((z0 + z) * g.ny + (y0 + y)) * g.nx + (x0 + x)] = s.sphi[L];
        ++my_written;
    }
    if (s.written && my_written) atomicAdd(s.written, my_written);
}

// ---------------------------------------------------------------------------
// STEP 2 on tiles
// ---------------------------------------------------------------------------
// Resident workgroups per CU for the update step: six for 8^3 float tiles
// (two nodes per lane), so that all 1536 default workgroups of a launch are
// resident at once (eighty registers, one value spilled); with early remedy visits a
// workgroup that waited for a slot would start its visit late and hold the
// launch.  Others unconstrained.
template <int ND, int NPT, typename T>
constexpr int update_blocks_per_cu() {
    return ND == 3 && NPT == 2 && sizeof(T) == 4 ? 6 : 1;
}

template <typename T, int ND, int TX, int TY, int TZ, bool AN>
__global__ __launch_bounds__(kBlock, (update_blocks_per_cu<ND, Shape<ND, TX, TY, TZ>::NPT, T>())) void k_tile_update(
    TileIter<T> a, BatchGeom<T> bg, T eps, int inner, TileIter<T> e, int early_inner) {
    using S = Shape<ND, TX, TY, TZ>;
    __shared__ T sphi[S::NL];
    __shared__ uint8_t sl[S::NL];
    __shared__ T sH[S::NT];
    __shared__ TileLists<S::NT> tl;
    __shared__ uint8_t schg[2][ND == 2 ? S::NT : 1];  // 2D: inputs changed in phase 1 (by iteration parity)
    __shared__ int s_len[kSub];
    __shared__ int s_slot;
    __shared__ int s_face;
    __shared__ int s_evals;
    __shared__ int s_written;
    __shared__ int s_elen[kSub];
    __shared__ uint32_t s_emask;
    __shared__ int s_stop;
    const T inf = pos_inf<T>();
    const uint32_t ntag = launch_tag(a);
    // early remedy visits exist in 3D float only (compiled out elsewhere)
    const bool early = ND == 3 && sizeof(T) == 4 && e.done != nullptr;
    if (early) {
        if (blockIdx.x == 0 && threadIdx.x < kSub) {
            e.zero_count[threadIdx.x * kPad] = 0;
            e.zero_fetch[threadIdx.x * kPad] = 0;
            if (threadIdx.x == 0) *e.fin_clear = 0;
        }
        if (threadIdx.x < kSub) s_elen[threadIdx.x] = e.cur.count[threadIdx.x * kPad];
    }
    const int n = list_open(a, s_len);
    launch_stats(a, n);
    // workgroups of group k take entries of sub-list k one at a time
    const int k = blockIdx.x & (kSub - 1);
    const int len = s_len[k];
    unsigned long long evals = 0, inner_sum = 0, written = 0, visits = 0;
    for (bool first = true;; first = false) {
        const int t = list_fetch(a.cur, k, len, &s_slot, first);
        if (t < 0) break;
        ++visits;
        const Inst<T> g = inst_of(bg, t);
        const int lt = t - g.tile_base;
        const int tx = lt % g.ntx, ty = (lt / g.ntx) % g.nty, tz = lt / (g.ntx * g.nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * (ND == 3 ? TZ : 1);
        const int open = open_bits<ND, TX, TY, TZ>(g, x0, y0, z0);
        T fv[S::NPT];
        load_owned_F<T, ND, TX, TY, TZ>(g, x0, y0, z0, a.F, fv);
        stage<T, ND, TX, TY, TZ>(g, x0, y0, z0, a.phi, a.lab, sphi, sl);
        bool ok[S::NPT];
        int G[S::NPT], L[S::NPT];
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) {
            const int nn = threadIdx.x + r * kBlock;
            int x, y, z;
            node_loc<ND, TX, TY, TZ>(nn, x, y, z, L[r]);
            G[r] = owned_index<T, ND, TX, TY, TZ>(g, x0, y0, z0, nn, ok[r]);
            if (nn < S::NT) {
                sH[nn] = ok[r] ? cell_value<T, AN>(g, fv[r]) : dead_value<T, AN>();
                tl.flag[0][nn] = 0u;
                tl.flag[1][nn] = 0u;
                if (ND == 2) {
                    schg[0][nn] = 0;
                    schg[1][nn] = 0;
                }
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
        // Inner iterations on the LDS active list, values updated in place.
        // Reads racing with updates see either value, both upper bounds of the
        // solution.  Each iteration has two phases:
        //   1. every listed node is evaluated; a value that does not move
        //      (phi - phi~ <= eps) converges the node, a value that drops is
        //      taken and marks the node's in-tile neighbours "inputs changed";
        //   2. a node whose value dropped in phase 1 while none of its inputs
        //      changed converges at once: its re-evaluation would give the
        //      same value (the convergence test of the next iteration, known
        //      in advance); the others are listed again.
        // A front thus crosses one node per iteration instead of two.  In 3D
        // phase 2 is left out (a dropped value is listed again and confirmed
        // by its next evaluation): the extra phase and its registers cost
        // more there than the shorter crossings save.
        constexpr bool TWO_PHASE = ND == 2;
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
            // the marks of the previous iteration are no longer read
            if (TWO_PHASE) {
#pragma unroll
                for (int r = 0; r < S::NPT; ++r)
                    if (threadIdx.x + r * kBlock < S::NT) schg[nb][threadIdx.x + r * kBlock] = 0;
            }
            // converged node q (LDS index Lq, tile position x, y, z): CONV,
            // its FAR neighbours become active
            auto converge = [&](int q, int Lq, int x, int y, int z) {
                sl[Lq] = (sl[Lq] & ~3u) | L_CONV;
                const int edge = edge_bits<ND, TX, TY, TZ>(x, y, z);
                // the neighbours' labels, read in one round
                uint8_t lbs[2 * ND];
#pragma unroll
                for (int d = 0; d < 2 * ND; ++d) lbs[d] = sl[Lq + lds_offset<ND, TX, TY, TZ>(d)];
#pragma unroll
                for (int d = 0; d < 2 * ND; ++d) {
                    const int Ln = Lq + lds_offset<ND, TX, TY, TZ>(d);
                    const uint8_t lb = lbs[d];
                    if (edge & (1 << d)) {
                        if ((open & (1 << d)) && (lb & 3u) == L_FAR) fm |= 1 << d;
                    } else if (!(lb & kOut) && (lb & 3u) == L_FAR && (lb & kPass)) {
                        if (list_add(tl, nb, ncnt, q + node_step<TX, TY>(d))) sl[Ln] = (lb & ~3u) | L_ACTIVE;
                    }
                }
            };
            constexpr int MAXC = (S::NT + kBlock - 1) / kBlock;
            int cq[MAXC];
            int nc = 0;
            for (int i = threadIdx.x; i < ncur; i += kBlock) {
                const int q = tl.list[cb][i];
                tl.flag[cb][q] = 0u;
                int x, y, z, Lq;
                node_loc<ND, TX, TY, TZ>(q, x, y, z, Lq);
                ++my_evals;
                const T pt = eval_lds<T, ND, TX, TY, TZ, AN>(sphi, Lq, sH[q], g);
                const T cur = sphi[Lq];
                if (pt < inf && cur - pt <= eps) {
                    converge(q, Lq, x, y, z);
                } else if (!(pt < inf)) {
                    sl[Lq] = (sl[Lq] & ~3u) | L_FAR;
                } else {
                    sphi[Lq] = pt;  // pt < cur - eps
                    if (TWO_PHASE) {
                        const int edge = edge_bits<ND, TX, TY, TZ>(x, y, z);
#pragma unroll
                        for (int d = 0; d < 2 * ND; ++d)
                            if (!(edge & (1 << d))) schg[cb][q + node_step<TX, TY>(d)] = 1;
                        cq[nc++] = q;
                    } else {
                        list_add(tl, nb, ncnt, q);
                    }
                }
            }
            if (TWO_PHASE) {
                __syncthreads();
                for (int j = 0; j < nc; ++j) {
                    const int q = cq[j];
                    int x, y, z, Lq;
                    node_loc<ND, TX, TY, TZ>(q, x, y, z, Lq);
                    if (!schg[cb][q]) converge(q, Lq, x, y, z);
                    else list_add(tl, nb, ncnt, q);
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
                if (any_active) {
                    push_tile(a.next, a.tstamp, t, ntag);
                } else if (early) {
                    // the tile's update work is done for now: queue its first
                    // remedy visit (every node) for the idle workgroups
                    e.done[t] = 1;
                    atomicOr(e.mask_next + t, kAllFaces);
                    push_tile(e.next, e.tstamp, t, ntag);
                }
            } else if (d < 2 * ND && (fmask & (1 << d))) {
                push_tile(a.next, a.tstamp, neighbour_tile(g, t, d), ntag);
            }
        }
        if (threadIdx.x == 0) {
            evals += static_cast<unsigned long long>(s_evals);
            inner_sum += static_cast<unsigned long long>(it);
            written += static_cast<unsigned long long>(s_written);
            if (early) atomicAdd(e.fin, 1);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && visits) {
        stat_add(a.blkstat, SF_EVALS2, evals);
        stat_add(a.blkstat, SF_VISITS2, visits);
        stat_add(a.blkstat, SF_INNER2, inner_sum);
        stat_add(a.blkstat, SF_WRITTEN2, written);
    }
    // Early remedy: workgroups that had no update visit in this launch run
    // remedy visits (first-in first-out, at most early_inner inner
    // iterations) on tiles whose update work is done, behind the front; the
    // remedy after the update step (detection over every node, then the
    // ordered loop) still decides the fixed point.
    if (!early || visits) return;
    const int elen = s_elen[k];
    unsigned long long eevals = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            // no new early visit once the launch's update visits are all done
            const bool over = __hip_atomic_load(e.fin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n;
            const int ei = over ? elen : atomicAdd(e.cur.fetch + k * kPad, 1);  // workgroups arrive at any time
            const int tt = ei < elen ? e.cur.data[static_cast<size_t>(k) * e.cur.cap + ei] : -1;
            if (tt >= 0) {
                s_emask = e.mask_cur[tt];  // set by an earlier launch; no writer during this one
                e.mask_cur[tt] = 0u;
            }
            s_slot = tt;
        }
        __syncthreads();
        const int t = s_slot;
        __syncthreads();
        if (t < 0) break;
        const Inst<T> g = inst_of(bg, t);
        const int lt = t - g.tile_base;
        const int tx = lt % g.ntx, ty = (lt / g.ntx) % g.nty, tz = lt / (g.ntx * g.nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * (ND == 3 ? TZ : 1);
        const int open = open_bits<ND, TX, TY, TZ>(g, x0, y0, z0);
        const RemedyLds<T, S::NT> rl{sphi, sH, &tl, &s_emask, &s_face, &s_evals, nullptr, &s_stop, nullptr};
        bool pending;
        // stop once the launch's update visits are all done
        remedy_visit<T, ND, TX, TY, TZ, AN, true>(
            e.cells, a.phi, g, t, x0, y0, z0, open, eps, early_inner, false, 0u, false, rl, pending,
            [&] { return __hip_atomic_load(e.fin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }, n);
        // a face whose neighbour tile is done with its update work marks that
        // tile; the others get their first visit when they are done
        if (threadIdx.x < 7) {
            const int d = threadIdx.x;
            if (d == 6) {
                if (pending) {
                    atomicOr(e.mask_next + t, kAllFaces);
                    push_tile(e.next, e.tstamp, t, ntag);
                }
            } else if (d < 2 * ND && (s_face & (1 << d))) {
                const int tn = neighbour_tile(g, t, d);
                if (e.done[tn]) {
                    atomicOr(e.mask_next + tn, 1u << (d ^ 1));
                    push_tile(e.next, e.tstamp, tn, ntag);
                }
            }
        }
        remedy_write_back<T, ND, TX, TY, TZ>(a.phi, g, x0, y0, z0, rl);
        if (threadIdx.x == 0) eevals += static_cast<unsigned long long>(s_evals);
        __syncthreads();
        break;  // one early visit per workgroup and launch: the launch ends with its update visits
    }
    if (threadIdx.x == 0) stat_add(a.blkstat, SF_CHECK, eevals);
}

// ---------------------------------------------------------------------------
// STEP 3: whole-grid detection, one workgroup per tile
// ---------------------------------------------------------------------------
template <typename T, int ND, int TX, int TY, int TZ, bool AN>
__global__ __launch_bounds__(kBlock) void k_tile_detect(TileIter<T> a, BatchGeom<T> bg, T eps) {
    using S = Shape<ND, TX, TY, TZ>;
    __shared__ T sphi[S::NL];
    __shared__ uint32_t s_key;
    const uint32_t ntag = launch_tag(a);
    for (int t = blockIdx.x; t < bg.ntiles; t += gridDim.x) {
        const Inst<T> g = inst_of(bg, t);
        const int lt = t - g.tile_base;
        const int tx = lt % g.ntx, ty = (lt / g.ntx) % g.nty, tz = lt / (g.ntx * g.nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * (ND == 3 ? TZ : 1);
        if (threadIdx.x == 0) s_key = kNoKey;  // ordered below the staging barrier
        T hv[S::NPT];
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) {
            const int nn = min(static_cast<int>(threadIdx.x) + r * kBlock, S::NT - 1);
            hv[r] = a.cells[static_cast<size_t>(t) * S::NT + nn];
        }
        stage<T, ND, TX, TY, TZ, false, false>(g, x0, y0, z0, a.phi, nullptr, sphi, nullptr);
        __syncthreads();
        bool flag = false;
        T low = pos_inf<T>();
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) {
            const int nn = threadIdx.x + r * kBlock;
            if (nn >= S::NT || !cell_free<T, AN>(hv[r])) continue;  // outside, barrier or fixed
            int x, y, z, L;
            node_loc<ND, TX, TY, TZ>(nn, x, y, z, L);
            const T pt = eval_lds<T, ND, TX, TY, TZ, AN>(sphi, L, hv[r], g);
            if (pt < sphi[L] - eps) {
                flag = true;
                low = tmin(low, pt);
            }
        }
        if (a.ordered && flag) atomicMin(&s_key, order_key(low));
        if (__syncthreads_or(flag) && threadIdx.x == 0) {
            a.mask_next[t] = kAllFaces;  // one writer: the workgroup of tile t
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
// Resident workgroups per CU for float tiles (the inner iterations are
// latency-bound; occupancy against spilled registers, measured): eight for
// tiles of one node per lane, six for two (the 8^3 tile: eight spill at
// 64 registers, five or fewer were slower).
template <int NPT, typename T>
constexpr int remedy_blocks_per_cu() {
    return sizeof(T) != 4 ? 1 : NPT == 1 ? 8 : NPT == 2 ? 6 : 1;
}

template <typename T, int ND, int TX, int TY, int TZ, bool AN>
__global__ __launch_bounds__(kBlock, (remedy_blocks_per_cu<Shape<ND, TX, TY, TZ>::NPT, T>())) void k_tile_remedy(
    TileIter<T> a, BatchGeom<T> bg, T eps, int inner) {
    using S = Shape<ND, TX, TY, TZ>;
    __shared__ T sphi[S::NL];
    __shared__ T sH[S::NT];
    __shared__ TileLists<S::NT> tl;
    __shared__ int s_len[kSub];
    __shared__ int s_slot;
    __shared__ int s_face;
    __shared__ int s_evals;
    __shared__ int s_written;
    __shared__ uint32_t s_mask;
    __shared__ uint32_t s_key, s_kmin;
    const uint32_t ntag = launch_tag(a);
    // ordered mode: k_tile_split has moved this launch's tiles into the work
    // list (the rest went on to the next list)
    __shared__ int s_wlen[kSub];
    const int n = list_open(a, s_len, s_wlen);
    launch_stats(a, n);
    const bool direct = list_direct(a, n);  // a short list is drained where it is
    const bool from_work = a.ordered && !direct;
    const TList src = from_work ? a.work : a.cur;
    const int k = blockIdx.x & (kSub - 1);
    const int len = from_work ? s_wlen[k] : s_len[k];
    unsigned long long evals = 0, inner_sum = 0, written = 0, visits = 0;
    for (bool first = true;; first = false) {
        if (threadIdx.x == 0) {
            const int e = fetch_index(src, k, len, first);
            const size_t idx = static_cast<size_t>(k) * src.cap + e;
            const int tt = e < len ? src.data[idx] : -1;
            if (e < len && from_work) {
                // the split moved the key and dirty faces into the work entry
                s_key = src.key[idx];
                s_mask = src.mask[idx];
            } else if (tt >= 0 && direct) {
                // the tile leaves the current list: its key goes with it
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
            if (!from_work) {
                // written by the previous launch; no writer during this one
                mask_in = a.mask_cur[t];
                a.mask_cur[t] = 0u;
            }
            s_kmin = kNoKey;
        }
        const RemedyLds<T, S::NT> rl{sphi, sH, &tl, &s_mask, &s_face, &s_evals, &s_kmin, nullptr, &s_written};
        bool pending;
        const int it = remedy_visit<T, ND, TX, TY, TZ, AN, false>(a.cells, a.phi, g, t, x0, y0, z0, open, eps, inner,
                                                                  a.ordered, mask_in, !from_work, rl, pending,
                                                                  [] { return 0; }, 0);
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
        remedy_write_back<T, ND, TX, TY, TZ>(a.phi, g, x0, y0, z0, rl);
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


// ---------------------------------------------------------------------------
// Tile-major cell values
// ---------------------------------------------------------------------------
// Entry t * NT + n holds the cell value of node n of tile t (H = h / F, or F
// itself with per-axis spacing; +inf / 0 on a barrier), -1 for a fixed node,
// the dead value outside the grid.  Built once per solve after the update
// step: a tile's detection and remedy visits then read one contiguous block
// instead of a row of F per cache line and a label byte per node, and do not
// divide.  (NT is a multiple of 64, so a wave's entries share one tile.)
template <typename T, int ND, int TX, int TY, int TZ, bool AN>
__global__ __launch_bounds__(kBlock) void k_build_cells(BatchGeom<T> bg, const T* __restrict__ F,
                                                        const uint8_t* __restrict__ lab, T* __restrict__ cells) {
    using S = Shape<ND, TX, TY, TZ>;
    static_assert(S::NT % 64 == 0, "a wave's entries must lie in one tile");
    const int64_t total = static_cast<int64_t>(bg.ntiles) * S::NT;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        const int t = static_cast<int>(i / S::NT);
        const int n = static_cast<int>(i - static_cast<int64_t>(t) * S::NT);
        const Inst<T> g = inst_of(bg, t);
        const int lt = t - g.tile_base;
        const int tx = lt % g.ntx, ty = (lt / g.ntx) % g.nty, tz = lt / (g.ntx * g.nty);
        bool ok;
        const int G = owned_index<T, ND, TX, TY, TZ>(g, tx * TX, ty * TY, tz * (ND == 3 ? TZ : 1), n, ok);
        T v = dead_value<T, AN>();
        if (ok) v = (lab[G] & 3u) == L_FIXED ? fixed_cell<T>() : cell_value<T, AN>(g, F[G]);
        cells[i] = v;
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
    void* cells;        // tile-major cell values (ntiles x tile nodes)
    SchedWs q;          // lists, stamps, masks, keys, histograms, work lists
    SchedWs eq;         // 3D: the early remedy's lists, stamps and dirty-face masks
    uint8_t* done;      // 3D: per tile, update work done
    void* table;        // instance table (batches of more than one instance)
    int* tile_inst;     // instance of every tile (idem)
    void* table_u;      // the same for the update step's tiling (2D, see solve_tile)
    int* tile_inst_u;
    size_t bytes;
};

TileWs tile_layout(char* base, int64_t n, int64_t ntiles, size_t ninst, size_t inst_bytes, bool two_tilings,
                   size_t cell_bytes) {
    TileWs w{};
    size_t off = 0;
    auto take = [&](size_t b) {
        char* p = base ? base + off : nullptr;
        off = align_up(off + b, 256);
        return p;
    };
    w.ctl = reinterpret_cast<Ctl*>(take(sizeof(Ctl)));
    w.blkstat = reinterpret_cast<unsigned long long*>(take(8 * static_cast<size_t>(kStatFields) * kMaxStatBlocks));
    w.lab = reinterpret_cast<uint8_t*>(take(static_cast<size_t>(n)));
    w.cells = take(cell_bytes);
    w.q = sched_layout(take, ntiles);
    if (!two_tilings) {  // 3D (one tiling for both steps): early remedy
        w.eq = early_layout(take, ntiles);
        w.done = reinterpret_cast<uint8_t*>(take(static_cast<size_t>(ntiles)));
    }
    if (ninst > 1) {
        w.table = take(inst_bytes * ninst);
        w.tile_inst = reinterpret_cast<int*>(take(4 * static_cast<size_t>(ntiles)));
        if (two_tilings) {  // the update step's tiling has no more tiles than this one
            w.table_u = take(inst_bytes * ninst);
            w.tile_inst_u = reinterpret_cast<int*>(take(4 * static_cast<size_t>(ntiles)));
        }
    }
    w.bytes = off;
    return w;
}

// 2D solves with the default 16 x 16 tiles run the update step on 32 x 32
// tiles: the update step's launches are bound by the front crossing a tile,
// so bigger tiles need fewer of them (2D lognormal 4096^2: update 18.6 ->
// 17.0 ms), while the remedy is faster on the smaller tiles.
bool update_tiling(const Batch& b, const eik_options& o, TileCfg& cu) {
    const bool def = o.tile[0] == 0 && o.tile[1] == 0 && o.tile[2] == 0;
    if (b.nd != 2 || !def || b.inst[0].aniso || b.cfg.tx != 16 || b.cfg.ty != 16) return false;
    cu = TileCfg{32, 32, 1};
    return true;
}

// Launches of `gt` persistent workgroups (a multiple of kSub, at most GT).
template <typename T, int ND, int TX, int TY, int TZ, bool AN>
struct TileKernels {
    static hipError_t update(const TileIter<T>& a, const BatchGeom<T>& g, T eps, int inner, int gt,
                             const TileIter<T>& e, int early_inner, hipStream_t s) {
        hipLaunchKernelGGL((k_tile_update<T, ND, TX, TY, TZ, AN>), dim3(gt), dim3(kBlock), 0, s, a, g, eps, inner, e,
                           early_inner);
        return hipGetLastError();
    }
    static hipError_t detect(const TileIter<T>& a, const BatchGeom<T>& g, T eps, int gt, hipStream_t s) {
        hipLaunchKernelGGL((k_tile_detect<T, ND, TX, TY, TZ, AN>), dim3(gt), dim3(kBlock), 0, s, a, g, eps);
        return hipGetLastError();
    }
    static hipError_t remedy(const TileIter<T>& a, const BatchGeom<T>& g, T eps, int inner, int gt, hipStream_t s) {
        hipLaunchKernelGGL((k_tile_remedy<T, ND, TX, TY, TZ, AN>), dim3(gt), dim3(kBlock), 0, s, a, g, eps, inner);
        return hipGetLastError();
    }
    static hipError_t cells(const BatchGeom<T>& g, const T* F, const uint8_t* lab, T* out, hipStream_t s) {
        using S = Shape<ND, TX, TY, TZ>;
        const int64_t total = static_cast<int64_t>(g.ntiles) * S::NT;
        const int blocks = static_cast<int>(std::min<int64_t>((total + kBlock - 1) / kBlock, 8192));
        hipLaunchKernelGGL((k_build_cells<T, ND, TX, TY, TZ, AN>), dim3(blocks), dim3(kBlock), 0, s, g, F, lab, out);
        return hipGetLastError();
    }
};

template <typename T>
struct TileOps {
    hipError_t (*update)(const TileIter<T>&, const BatchGeom<T>&, T, int, int, const TileIter<T>&, int,
                         hipStream_t) = nullptr;
    hipError_t (*detect)(const TileIter<T>&, const BatchGeom<T>&, T, int, hipStream_t) = nullptr;
    hipError_t (*remedy)(const TileIter<T>&, const BatchGeom<T>&, T, int, int, hipStream_t) = nullptr;
    hipError_t (*cells)(const BatchGeom<T>&, const T*, const uint8_t*, T*, hipStream_t) = nullptr;
};

template <typename T, int ND, int TX, int TY, int TZ, bool AN = false>
TileOps<T> ops_of() {
    TileOps<T> k;
    k.update = &TileKernels<T, ND, TX, TY, TZ, AN>::update;
    k.detect = &TileKernels<T, ND, TX, TY, TZ, AN>::detect;
    k.remedy = &TileKernels<T, ND, TX, TY, TZ, AN>::remedy;
    k.cells = &TileKernels<T, ND, TX, TY, TZ, AN>::cells;
    return k;
}

// Supported tile shapes (z, y, x); per-axis spacing only with the default
// shapes (16 x 16 in 2D, 8^3 in 3D).
template <typename T>
bool select_ops(int nd, const TileCfg& c, bool aniso, TileOps<T>& k) {
    if (aniso) {
        if (nd == 2 && c.ty == 16 && c.tx == 16) return k = ops_of<T, 2, 16, 16, 1, true>(), true;
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
        if (c.tx == 0 || c.ty == 0) c = TileCfg{16, 16, 1};
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

// Bytes of the tile-major cell array of a batch's tiling.
static size_t cell_array_bytes(const Batch& b, size_t esz) {
    return static_cast<size_t>(b.ntiles) * static_cast<size_t>(b.cfg.tx) * b.cfg.ty * b.cfg.tz * esz;
}

size_t tile_workspace_bytes(const Batch& b, size_t esz) {
    const size_t ib = esz == 8 ? sizeof(Inst<double>) : sizeof(Inst<float>);
    return tile_layout(nullptr, b.n, b.ntiles, b.inst.size(), ib, b.nd == 2, cell_array_bytes(b, esz)).bytes;
}

template <typename T>
eik_status solve_tile(const Batch& b, const T* F, double eps, T* phi, const eik_options& o, char* ws,
                      hipStream_t s, eik_stats* st) {
    const bool async = (o.flags & EIK_FLAG_ASYNC) != 0;
    const bool pageable = (o.flags & kFlagPageable) != 0;
    const TileCfg c = b.cfg;
    TileOps<T> k;
    if (!select_ops<T>(b.nd, c, b.inst[0].aniso != 0, k))
        return fail(EIK_ERR_INVALID_ARGUMENT, b.inst[0].aniso ? "per-axis spacing needs the default tile shape"
                                                              : "unsupported tile shape");
    TileWs w = tile_layout(ws, b.n, b.ntiles, b.inst.size(), sizeof(Inst<T>), b.nd == 2, cell_array_bytes(b, sizeof(T)));
    // the update step's tiling (the same unless update_tiling says otherwise)
    TileCfg cu = c;
    const bool two = update_tiling(b, o, cu);
    const Batch bu = two ? with_tiles(b, cu) : Batch{};
    const Batch& B2 = two ? bu : b;
    TileOps<T> ku = k;
    if (two && !select_ops<T>(b.nd, cu, false, ku)) return fail(EIK_ERR_INVALID_ARGUMENT, "unsupported tile shape");
    const int64_t cap = o.max_iters > 0 ? o.max_iters : 4 * b.n + 64;
    // Inner iterations per tile visit.  In 2D an update visit stops after the
    // iterations a front needs to cross the tile along an axis (one per node
    // with the 2D two-phase iteration): the front still advances a tile per
    // launch, and no visit holds its launch for a diagonal crossing (2D
    // lognormal 4096^2, 16 x 16 tiles: update 34 -> 19 ms).  In 3D the cut
    // visits leave more to the remedy than they save (256^3 maze), so update
    // and remedy visits run until their lists empty (4 x the sum of the sides
    // is a safety cap).
    const int inner = o.inner_iters > 0 ? o.inner_iters : 4 * (c.tx + c.ty + c.tz);
    const int side_u = std::max(cu.tx, std::max(cu.ty, cu.tz));
    const int inner_upd = o.inner_iters > 0 ? o.inner_iters : (b.nd == 2 ? side_u : inner);
    const int ntiles_u = static_cast<int>(B2.ntiles);
    const int gt = workgroups_of(b.nd, o.workgroups);
    const int omin = order_min_of(b.nd, o.order_min);
    int64_t launched = 0;

    Profiler prof;
    prof.start((o.flags & EIK_FLAG_PROFILE) != 0, s);
    const size_t blk_bytes = 8 * static_cast<size_t>(kStatFields) * kMaxStatBlocks;
    BatchGeom<T> geom, geom_u;
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return upload_batch_geom<T>(b, w.table, w.tile_inst, s, geom, launched); }));
    if (two)
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
            return upload_batch_geom<T>(bu, w.table_u, w.tile_inst_u, s, geom_u, launched);
        }));
    else
        geom_u = geom;
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_ctl_init(w.ctl, s); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_zero_words(w.blkstat, blk_bytes, s); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_init<T>(F, phi, w.lab, nullptr, static_cast<int>(b.n), w.ctl, s); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return sched_clear(w.q, s); }));
    launched += 7;
    const bool ordered = (o.flags & EIK_FLAG_FIFO_REMEDY) == 0;
    const bool early = b.nd == 3 && sizeof(T) == 4 && !two &&
                       !(o.flags & (EIK_FLAG_NO_EARLY_REMEDY | EIK_FLAG_SKIP_REMEDY));
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
    auto list_of = [&](int64_t t) { return w.q.list_of(t); };
    if (batches.size() <= 8) {
        // tiles next to the sources
        for (auto& sb : batches)
            HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
                hipLaunchKernelGGL(k_seed_tiles<T>, dim3(1), dim3(kMaxSrcBatch), 0, s, geom_u, b.nd, cu.tx, cu.ty, cu.tz,
                                   sb, w.q.tstamp, list_of(0));
                return hipGetLastError();
            }));
        launched += static_cast<int64_t>(batches.size());
    } else {
        // many sources: start from every tile; tiles with nothing to do drop out
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
            hipLaunchKernelGGL(k_seed_all_tiles, dim3(std::min((ntiles_u + kBlock - 1) / kBlock, 1024)), dim3(kBlock),
                               0, s, ntiles_u, w.q.tstamp, list_of(0));
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
        sched_fill(a, w.q, t, ordered && phase == 1, omin, static_cast<int>((gl + t) & 1), phase, w.ctl,
                   w.blkstat);
        a.F = F;
        a.phi = phi;
        a.lab = w.lab;
        a.cells = static_cast<const T*>(w.cells);
        return a;
    };
    auto counts = [&](int64_t t) { return w.q.count_of(static_cast<int>(t % 3)); };
    if (early) {
        // cell values (sources are fixed by now) and the early remedy's lists
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return k.cells(geom, F, w.lab, static_cast<T*>(w.cells), s); }));
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return early_clear(w.eq, s); }));
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER,
                      [&] { return launch_zero_words(w.done, align_up(static_cast<size_t>(b.ntiles), 4), s); }));
        launched += 3;
    }
    auto early_args = [&](int64_t t) {
        TileIter<T> e{};
        if (!early) return e;
        sched_fill(e, w.eq, t, false, omin, static_cast<int>((gl + t) & 1), 1, w.ctl, w.blkstat);
        e.phi = phi;
        e.cells = static_cast<const T*>(w.cells);
        e.done = w.done;
        e.fin = &w.ctl->cnt[t % 3];
        e.fin_clear = &w.ctl->cnt[(t + 1) % 3];
        return e;
    };
    // inner iterations of an early remedy visit (maze 256^3 / layered 192^3:
    // 16 gave 14.1 / 5.9 ms, 32 and 64 14.7 / 6.3 ms: deeper visits hold the
    // update launch longer than they shorten the remedy loop)
    const int early_inner = 16;

    int64_t n2 = 0;
    eik_status rc = run_loop(
        [&](int64_t t) {
            return timed(prof, EIK_KERNEL_UPDATE, [&] {
                return ku.update(iter_args(t, 0), geom_u, eT, inner_upd, gt, early_args(t), early_inner, s);
            });
        },
        counts, kSub * kPad, cap, async, s, &n2, w.ctl, pageable);
    gl += n2;
    launched += n2;
    if (rc == EIK_OK && !(o.flags & EIK_FLAG_SKIP_REMEDY)) {
        // tile-major cell values for detection and the remedy; detection
        // fills list 0 of the remedy loop
        if (!early) {
            HIP_TRY(timed(prof, EIK_KERNEL_OTHER,
                          [&] { return k.cells(geom, F, w.lab, static_cast<T*>(w.cells), s); }));
            launched += 1;
        }
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_zero_words(w.q.counters, kCounterBytes, s); }));
        TileIter<T> d = iter_args(0, 1);  // only `next` (list 0), its masks and the tag are used
        d.next = list_of(0);
        d.mask_next = w.q.tmask;  // read by remedy launch 0
        d.key_next = w.q.keys;
        d.hist_next = w.q.hist_of(0);
        d.first = 0;
        d.tag_slot = static_cast<int>(gl & 1);
        HIP_TRY(timed(prof, EIK_KERNEL_DETECT, [&] { return k.detect(d, geom, eT, gt, s); }));
        gl += 1;
        launched += 2;
        int64_t n3 = 0;
        const int split_blocks = split_blocks_of(b.ntiles);
        rc = run_loop(
            [&](int64_t t) {
                const TileIter<T> a = iter_args(t, 1);
                if (ordered) {
                    const hipError_t e = timed(prof, EIK_KERNEL_OTHER, [&] {
                        hipLaunchKernelGGL(k_tile_split, dim3(split_blocks), dim3(kBlock), 0, s, static_cast<const Sched&>(a));
                        return hipGetLastError();
                    });
                    if (e != hipSuccess) return e;
                }
                return timed(prof, EIK_KERNEL_REMEDY, [&] { return k.remedy(a, geom, eT, inner, gt, s); });
            },
            counts, kSub * kPad, cap, async, s, &n3, w.ctl, pageable);
        launched += (ordered ? 2 : 1) * n3;
    }
    if (async) return rc;
    Results res;
    const eik_status rr = read_results(w.ctl, w.blkstat, kMaxStatBlocks, pageable, s, res);
    if (rr != EIK_OK) return rr;
    if (res.ctl.err & 1) return fail(EIK_ERR_INVALID_ARGUMENT, "F has negative or non-finite values");
    if (st) {
        *st = eik_stats{};
        st->step2_iters = static_cast<int64_t>(res.ctl.iters2);
        st->step3_iters = static_cast<int64_t>(res.ctl.iters3);
        st->evals_step2 = static_cast<int64_t>(res.sum[SF_EVALS2]);
        st->evals_detect = (o.flags & EIK_FLAG_SKIP_REMEDY) ? 0 : b.n - static_cast<int64_t>(b.src.size());
        st->evals_remedy = static_cast<int64_t>(res.sum[SF_EVALS3]);
        st->remedy_initial = static_cast<int64_t>(res.ctl.remedy_init);
        st->max_active = static_cast<int64_t>(res.ctl.max_active);
        st->launches = launched;
        st->tile_visits_step2 = static_cast<int64_t>(res.sum[SF_VISITS2]);
        st->tile_visits_step3 = static_cast<int64_t>(res.sum[SF_VISITS3]);
        st->inner_step2 = static_cast<int64_t>(res.sum[SF_INNER2]);
        st->inner_step3 = static_cast<int64_t>(res.sum[SF_INNER3]);
        st->written_step2 = static_cast<int64_t>(res.sum[SF_WRITTEN2]);
        st->written_step3 = static_cast<int64_t>(res.sum[SF_WRITTEN3]);
        st->evals_early = static_cast<int64_t>(res.sum[SF_CHECK]);
        HIP_TRY(prof.collect(st));
    }
    return rc;
}

template eik_status solve_tile<float>(const Batch&, const float*, double, float*, const eik_options&, char*,
                                      hipStream_t, eik_stats*);
template eik_status solve_tile<double>(const Batch&, const double*, double, double*, const eik_options&, char*,
                                       hipStream_t, eik_stats*);

}  // namespace eik
