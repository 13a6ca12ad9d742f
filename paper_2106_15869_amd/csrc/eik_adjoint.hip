// Adjoint of the converged eikonal solve on gfx950: dL/dF for a loss L(phi).
//
// At the solution every reached non-source node i with F_i > 0 satisfies
// sum_{k in U_i} w_ik^2 = H_i^2 over its upwind axes U_i (a_k < phi_i), with
// w_ik = phi_i - a_k and H_i = h / F_i (Eq 4 / Eq 6 at the fixed point).
// Differentiating gives dphi = M dphi + D dF with M_{i,j_k} = w_ik / W_i,
// W_i = sum_k w_ik, D_i = -H_i^2 / (F_i W_i).  Hence dL/dF = D lambda with
//     lambda = dL/dphi + M^T lambda,
// a triangular system in causal order.
//
//   k_adj_prep   per node, tile by tile: the upwind neighbour on each axis
//                (lower index on a tie), the weights c_ik = w_ik / W_i, D_i.
//   Grids of a batch are tiled back to back (see eik_tile.hpp); every kernel
//   looks up the instance of the tile it works on.
//   k_adj_tile   tile work queues (eik_sched.hpp): a persistent workgroup
//                stages lambda and the stencil data of a tile plus halo in
//                LDS and recomputes
//                lambda_j = g_j + sum_{i : j upwind of i} c_{i,axis} lambda_i
//                over an LDS list: a node whose lambda changes lists the
//                nodes upwind of it (they pull from it); across a tile face it
//                marks that face dirty in the neighbour tile and queues it.
//                lambda starts at 0 and the tiles holding a nonzero dL/dphi
//                start queued, so every node with g_j != 0 changes on its
//                first evaluation and passes its value on, also across a face.
//                Tiles are taken in decreasing arrival time (order keys of
//                -phi), the direction in which lambda flows.  The system is
//                triangular, so the iteration ends at its unique solution
//                whatever the order.
//   k_adj_final  dense: dL/dF = D lambda (0 at sources and unreached nodes).
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

constexpr uint8_t kSrc = 0x80u;   // stencil byte: node is a source
// stencil byte bits: axis k present -> bit 2k; upwind on the + side -> bit 2k+1
// (axis 0 = x, 1 = y, 2 = z)

template <typename T>
struct AdjIter : Sched {
    const T* phi;
    const T* g;      // dL/dphi
    T* lam;
    const uint8_t* up;  // stencil bytes
    const T* coef;      // 3 per node (x, y, z)
};

// ---------------------------------------------------------------------------
template <typename T, int ND, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_adj_prep(BatchGeom<T> bg, const T* __restrict__ F,
                                                     const T* __restrict__ phi, uint8_t* up, T* coef, T* D,
                                                     T* lam, const T* __restrict__ g) {
    constexpr int NT = TX * TY * (ND == 3 ? TZ : 1);
    const T inf = pos_inf<T>();
    for (int t = blockIdx.x; t < bg.ntiles; t += gridDim.x) {
        const Inst<T> I = inst_of(bg, t);
        const int lt = t - I.tile_base;
        const int x0 = (lt % I.ntx) * TX, y0 = ((lt / I.ntx) % I.nty) * TY;
        const int z0 = ND == 3 ? (lt / (I.ntx * I.nty)) * TZ : 0;
        for (int q = threadIdx.x; q < NT; q += kBlock) {
            const int x = x0 + q % TX, y = y0 + (q / TX) % TY, z = ND == 3 ? z0 + q / (TX * TY) : 0;
            if (x >= I.nx || y >= I.ny || z >= I.nz) continue;
            const int sy = I.nx, sz = I.nx * I.ny;
            const int i = I.node_base + (z * I.ny + y) * I.nx + x;
            const T p = phi[i];
            const T f = F[i];
            uint8_t u = 0;
            T w[3] = {T(0), T(0), T(0)};
            T W = T(0);
            if (p < inf && f > T(0)) {
                const int st[3] = {1, sy, sz};
                const int cc[3] = {x, y, z};
                const int dd[3] = {I.nx, I.ny, I.nz};
#pragma unroll
                for (int k = 0; k < ND; ++k) {
                    T v = inf;
                    int side = -1;
                    if (cc[k] > 0 && phi[i - st[k]] < v) {
                        v = phi[i - st[k]];
                        side = 0;
                    }
                    if (cc[k] + 1 < dd[k] && phi[i + st[k]] < v) {
                        v = phi[i + st[k]];
                        side = 1;
                    }
                    if (side >= 0 && v < p) {
                        u |= static_cast<uint8_t>((1u << (2 * k)) | (static_cast<uint32_t>(side) << (2 * k + 1)));
                        // per-axis spacing weighs axis k by 1 / spacing^2 (axis k = x, y, z
                        // is dims entry ND - 1 - k)
                        const T dk = I.d[ND - 1 - k];
                        w[k] = I.aniso ? (p - v) / (dk * dk) : p - v;
                        W = W + w[k];
                    }
                }
            }
            T d = T(0);
            if (u && W > T(0)) {
                if (I.aniso) {
                    d = -T(1) / (f * f * f * W);
                } else {
                    const T Hh = I.h / f;
                    d = -(Hh * Hh) / (f * W);
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) w[k] = w[k] / W;
            } else {
                u = 0;
                w[0] = w[1] = w[2] = T(0);
            }
            up[i] = u;
            coef[3 * static_cast<size_t>(i) + 0] = w[0];
            coef[3 * static_cast<size_t>(i) + 1] = w[1];
            coef[3 * static_cast<size_t>(i) + 2] = w[2];
            D[i] = d;
            lam[i] = T(0);
        }
    }
}

template <typename T>
__global__ void k_adj_mark_sources(SrcBatch<T> b, uint8_t* up, T* coef, T* D) {
    const int k = threadIdx.x;
    if (k >= b.count) return;
    const int i = b.idx[k];
    up[i] = kSrc;
    coef[3 * static_cast<size_t>(i) + 0] = T(0);
    coef[3 * static_cast<size_t>(i) + 1] = T(0);
    coef[3 * static_cast<size_t>(i) + 2] = T(0);
    D[i] = T(0);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_final(int n, const T* __restrict__ D,
                                                      const T* __restrict__ lam, T* __restrict__ out) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) out[i] = D[i] * lam[i];
}

// ---------------------------------------------------------------------------
// Initial list: tiles holding a nonzero dL/dphi (all nodes to recompute),
// keyed by the largest arrival time among those nodes.
template <typename T, int ND, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_adj_seed(AdjIter<T> a, BatchGeom<T> bg) {
    using S = Shape<ND, TX, TY, TZ>;
    __shared__ uint32_t s_key;
    for (int t = blockIdx.x; t < bg.ntiles; t += gridDim.x) {
        const Inst<T> g = inst_of(bg, t);
        const int lt = t - g.tile_base;
        const int tx = lt % g.ntx, ty = (lt / g.ntx) % g.nty, tz = lt / (g.ntx * g.nty);
        if (threadIdx.x == 0) s_key = kNoKey;
        __syncthreads();
        bool nz = false;
        for (int q = threadIdx.x; q < S::NT; q += kBlock) {
            const int x = tx * TX + q % TX, y = ty * TY + (q / TX) % TY;
            const int z = ND == 3 ? tz * TZ + q / (TX * TY) : 0;
            if (x < g.nx && y < g.ny && z < g.nz) {
                const int i = g.node_base + (z * g.ny + y) * g.nx + x;
                if (a.g[i] != T(0)) {
                    nz = true;
                    atomicMin(&s_key, order_key(-a.phi[i]));
                }
            }
        }
        if (__syncthreads_or(nz) && threadIdx.x == 0) {
            a.mask_next[t] = kAllFaces;
            push_keyed(a, t, 1u, s_key);
        }
        __syncthreads();
    }
}

// Resident workgroups per CU: six for 8^3 float tiles, so that all 1536
// default workgroups of a launch are resident at once.  Others unconstrained.
template <int ND, int NPT, typename T>
constexpr int adj_blocks_per_cu() {
    return ND == 3 && NPT == 2 && sizeof(T) == 4 ? 6 : 1;
}

template <typename T, int ND, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock, (adj_blocks_per_cu<ND, Shape<ND, TX, TY, TZ>::NPT, T>())) void k_adj_tile(
    AdjIter<T> a, BatchGeom<T> bg, int inner) {
    using S = Shape<ND, TX, TY, TZ>;
    __shared__ T slam[S::NL];
    __shared__ T scoef[3 * S::NL];
    __shared__ uint8_t sup[S::NL];
    __shared__ T sg[S::NT];
    __shared__ TileLists<S::NT> tl;
    __shared__ int s_len[kSub];
    __shared__ int s_slot;
    __shared__ int s_face;
    __shared__ uint32_t s_mask, s_key, s_kmin;
    const uint32_t ntag = launch_tag(a);
    __shared__ int s_wlen[kSub];
    const FirstEntry pre = first_entry(a, true);
    const int n = list_open(a, s_len, s_wlen);
    if (blockIdx.x == 0 && threadIdx.x == 0 && n > 0) a.ctl->iters3 += 1;
    const bool direct = list_direct(a, n);  // a short list is drained where it is
    const bool from_work = a.ordered && !direct;
    const TList src = from_work ? a.work : a.cur;
    const int k = blockIdx.x & (kSub - 1);
    const int len = from_work ? s_wlen[k] : s_len[k];
    constexpr int SY = S::LX, SZ = S::LX * S::LY;
    unsigned long long visits = 0;
    for (bool first = true;; first = false) {
        if (threadIdx.x == 0) {
            const int e = fetch_index(src, k, len, first);
            const size_t idx = static_cast<size_t>(k) * src.cap + e;
            const int tt = e < len ? (first ? (from_work ? pre.work : pre.cur) : src.data[idx]) : -1;
            if (tt >= 0) {
                if (from_work) {
                    // the split moved the key and dirty faces into the work entry
                    s_key = first ? pre.key : src.key[idx];
                    s_mask = first ? pre.mask : src.mask[idx];
                } else {
                    if (direct) {
                        s_key = a.key_cur[tt];
                        a.key_cur[tt] = kNoKey;
                    }
                    s_mask = a.mask_cur[tt];
                    a.mask_cur[tt] = 0u;
                }
            }
            s_kmin = kNoKey;
            s_face = 0;
            tl.cnt[0] = tl.cnt[1] = tl.cnt[2] = 0;
            s_slot = tt;
        }
        __syncthreads();
        const int t = s_slot;
        if (t < 0) break;
        ++visits;
        const Inst<T> g = inst_of(bg, t);
        const int lt = t - g.tile_base;
        const int tx = lt % g.ntx, ty = (lt / g.ntx) % g.nty, tz = lt / (g.ntx * g.nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * (ND == 3 ? TZ : 1);
        const int open = open_bits<ND, TX, TY, TZ>(g, x0, y0, z0);
        // stage lambda, stencil bytes and coefficients with the halo (0 outside)
        // and dL/dphi of the tile's nodes: addresses are clamped into the grid
        // so every global load of a lane is issued before its first LDS store
        {
            constexpr int NIT = (S::NL + kBlock - 1) / kBlock;
            constexpr int NPT = (S::NT + kBlock - 1) / kBlock;
            T vl[NIT], c0[NIT], c1[NIT], c2[NIT], vg[NPT];
            uint8_t vu[NIT];
            bool in[NIT], okn[NPT];
#pragma unroll
            for (int j = 0; j < NIT; ++j) {
                const int q = min(static_cast<int>(threadIdx.x) + j * kBlock, S::NL - 1);
                const int lx = q % S::LX, ly = (q / S::LX) % S::LY, lz = q / (S::LX * S::LY);
                const int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = ND == 3 ? z0 + lz - 1 : 0;
                in[j] = gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz;
                const int cx = min(max(gx, 0), g.nx - 1), cy = min(max(gy, 0), g.ny - 1);
                const int cz = min(max(gz, 0), g.nz - 1);
                const size_t G = static_cast<size_t>(g.node_base) + (cz * g.ny + cy) * g.nx + cx;
                vl[j] = a.lam[G];
                vu[j] = a.up[G];
                c0[j] = a.coef[3 * G + 0];
                c1[j] = a.coef[3 * G + 1];
                c2[j] = a.coef[3 * G + 2];
            }
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                const int nn = min(static_cast<int>(threadIdx.x) + r * kBlock, S::NT - 1);
                int x, y, z, L;
                node_loc<ND, TX, TY, TZ>(nn, x, y, z, L);
                okn[r] = x0 + x < g.nx && y0 + y < g.ny && z0 + z < g.nz;
                const int cx = min(x0 + x, g.nx - 1), cy = min(y0 + y, g.ny - 1), cz = min(z0 + z, g.nz - 1);
                vg[r] = a.g[g.node_base + (cz * g.ny + cy) * g.nx + cx];
            }
#pragma unroll
            for (int j = 0; j < NIT; ++j) {
                const int q = threadIdx.x + j * kBlock;
                if (q >= S::NL) continue;
                slam[q] = in[j] ? vl[j] : T(0);
                sup[q] = in[j] ? vu[j] : static_cast<uint8_t>(0);
                scoef[3 * q + 0] = in[j] ? c0[j] : T(0);
                scoef[3 * q + 1] = in[j] ? c1[j] : T(0);
                scoef[3 * q + 2] = in[j] ? c2[j] : T(0);
            }
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                const int nn = threadIdx.x + r * kBlock;
                if (nn >= S::NT) continue;
                sg[nn] = okn[r] ? vg[r] : T(0);
                tl.flag[0][nn] = 0u;
                tl.flag[1][nn] = 0u;
                tl.dirty[nn] = 0;
            }
        }
        __syncthreads();
        // initial list: every node on a first visit, else the nodes on the faces
        // whose neighbour tile changed
        const uint32_t m = s_mask;
        for (int nn = threadIdx.x; nn < S::NT; nn += kBlock) {
            int x, y, z, L;
            node_loc<ND, TX, TY, TZ>(nn, x, y, z, L);
            const bool ok = x0 + x < g.nx && y0 + y < g.ny && z0 + z < g.nz;
            const int E = edge_bits<ND, TX, TY, TZ>(x, y, z) & open;
            if (ok && ((m & kAllFaces) || (E & static_cast<int>(m))))
                tl.list[0][atomicAdd(&tl.cnt[0], 1)] = static_cast<uint16_t>(nn);
        }
        __syncthreads();
        bool pending = false;
        int fm = 0;
        uint32_t kmin = kNoKey;
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
                // neighbour on the - side of axis k pulls into q if its upwind on
                // axis k is its + side; on the + side, if its upwind is its - side.
                // Every neighbour's stencil byte, coefficient and value is read
                // in one round (all inside the halo block), then summed in
                // direction order.
                const int offs[6] = {-1, 1, -SY, SY, -SZ, SZ};
                uint32_t un[2 * ND];
                T cn[2 * ND], ln[2 * ND];
#pragma unroll
                for (int d = 0; d < 2 * ND; ++d) {
                    const int p = Lq + offs[d];
                    un[d] = sup[p];
                    cn[d] = scoef[3 * p + (d >> 1)];
                    ln[d] = slam[p];
                }
                const T cur = slam[Lq];  // only this lane writes it in this iteration
                T v = sg[q];
#pragma unroll
                for (int d = 0; d < 2 * ND; ++d) {
                    const int kx = d >> 1;
                    const uint32_t u = un[d];
                    const bool present = (u & (1u << (2 * kx))) && !(u & kSrc);
                    const bool plus = (u >> (2 * kx + 1)) & 1u;
                    if (present && plus == ((d & 1) == 0)) v = v + cn[d] * ln[d];
                }
                if (v != cur) {
                    slam[Lq] = v;
                    tl.dirty[q] = 1;
                    // the nodes upwind of q pull from it: list them
                    const uint32_t u = sup[Lq];
                    const int edge = edge_bits<ND, TX, TY, TZ>(x, y, z);
#pragma unroll
                    for (int kx = 0; kx < ND; ++kx) {
                        if (!(u & (1u << (2 * kx))) || (u & kSrc)) continue;
                        const int d = 2 * kx + static_cast<int>((u >> (2 * kx + 1)) & 1u);  // face toward it
                        if (edge & (1 << d)) {
                            if (open & (1 << d)) {
                                fm |= 1 << d;
                                const int G = g.node_base + ((z0 + z) * g.ny + (y0 + y)) * g.nx + (x0 + x);
                                kmin = min(kmin, order_key(-a.phi[G]));
                            }
                        } else {
                            list_add(tl, nb, ncnt, q + node_step<TX, TY>(d));
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (fm) atomicOr(&s_face, fm);
        if (a.ordered && kmin != kNoKey) atomicMin(&s_kmin, kmin);
        __syncthreads();
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
                atomicOr(a.mask_next + tn, 1u << (d ^ 1));
                push_keyed(a, tn, ntag, key);
            }
        }
        for (int nn = threadIdx.x; nn < S::NT; nn += kBlock) {
            if (!tl.dirty[nn]) continue;
            int x, y, z, L;
            node_loc<ND, TX, TY, TZ>(nn, x, y, z, L);
            a.lam[g.node_base + ((z0 + z) * g.ny + (y0 + y)) * g.nx + (x0 + x)] = slam[L];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && visits) stat_add(a.blkstat, SF_VISITS3, visits);
}

struct AdjWs {
    Ctl* ctl;
    unsigned long long* blkstat;
    uint8_t* up;
    void* coef;
    void* D;
    void* lam;
    SchedWs q;
    void* table;
    int* tile_inst;
    size_t bytes;
};

TileCfg adj_tile(int nd) { return nd == 2 ? TileCfg{16, 16, 1} : TileCfg{8, 8, 8}; }

AdjWs adj_layout(char* base, const Batch& b, size_t esz) {
    AdjWs w{};
    size_t off = 0;
    auto take = [&](size_t n) {
        char* p = base ? base + off : nullptr;
        off = align_up(off + n, 256);
        return p;
    };
    const size_t n = static_cast<size_t>(b.n);
    w.ctl = reinterpret_cast<Ctl*>(take(sizeof(Ctl)));
    w.blkstat = reinterpret_cast<unsigned long long*>(take(8 * static_cast<size_t>(kStatFields) * kMaxStatBlocks));
    w.up = reinterpret_cast<uint8_t*>(take(n));
    w.coef = take(3 * esz * n);
    w.D = take(esz * n);
    w.lam = take(esz * n);
    w.q = sched_layout(take, b.ntiles);
    if (b.inst.size() > 1) {
        w.table = take((esz == 8 ? sizeof(Inst<double>) : sizeof(Inst<float>)) * b.inst.size());
        w.tile_inst = reinterpret_cast<int*>(take(4 * static_cast<size_t>(b.ntiles)));
    }
    w.bytes = off;
    return w;
}

template <typename T, int ND, int TX, int TY, int TZ>
eik_status adj_run(const Batch& b, const T* F, const T* phi, const T* g, T* out, const eik_options& o, char* ws,
                   hipStream_t s, eik_stats* st) {
    const bool async = (o.flags & EIK_FLAG_ASYNC) != 0;
    const bool ordered = (o.flags & EIK_FLAG_FIFO_REMEDY) == 0;
    AdjWs w = adj_layout(ws, b, sizeof(T));
    const int64_t cap = o.max_iters > 0 ? o.max_iters : 4 * b.n + 64;
    const int inner = o.inner_iters > 0 ? o.inner_iters : 4 * (TX + TY + TZ);
    const int dense = static_cast<int>(std::min<int64_t>((b.n + kBlock - 1) / kBlock, 1 << 20));
    const int tiles = static_cast<int>(std::min<int64_t>(b.ntiles, 1 << 16));
    const int split_blocks = split_blocks_of(b.ntiles);
    const size_t blk_bytes = 8 * static_cast<size_t>(kStatFields) * kMaxStatBlocks;
    int64_t launched = 0;
    Profiler prof;
    prof.start((o.flags & EIK_FLAG_PROFILE) != 0, s);

    BatchGeom<T> G;
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return upload_batch_geom<T>(b, w.table, w.tile_inst, s, G, launched); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_ctl_init(w.ctl, s); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_zero_words(w.blkstat, blk_bytes, s); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return sched_clear(w.q, s); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
        hipLaunchKernelGGL((k_adj_prep<T, ND, TX, TY, TZ>), dim3(tiles), dim3(kBlock), 0, s, G, F, phi, w.up,
                           static_cast<T*>(w.coef), static_cast<T*>(w.D), static_cast<T*>(w.lam), g);
        return hipGetLastError();
    }));
    launched += 7;
    for (size_t q = 0; q < b.src.size(); q += kMaxSrcBatch) {
        SrcBatch<T> sb{};
        sb.count = static_cast<int>(std::min<size_t>(kMaxSrcBatch, b.src.size() - q));
        for (int j = 0; j < sb.count; ++j) sb.idx[j] = b.src[q + j].first;
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
            hipLaunchKernelGGL(k_adj_mark_sources<T>, dim3(1), dim3(kMaxSrcBatch), 0, s, sb, w.up,
                               static_cast<T*>(w.coef), static_cast<T*>(w.D));
            return hipGetLastError();
        }));
        ++launched;
    }
    // launch t drains list t and fills list t + 1; the seeding fills list 0
    // with tag 1 and the tag chain starts at tag[0] = 1 (claims 2, 3, ...)
    auto iter_args = [&](int64_t t) {
        AdjIter<T> a{};
        sched_fill(a, w.q, t, ordered, order_min_of(ND, o.order_min), static_cast<int>(t & 1), 1, w.ctl, w.blkstat);
        a.phi = phi;
        a.g = g;
        a.lam = static_cast<T*>(w.lam);
        a.up = w.up;
        a.coef = static_cast<const T*>(w.coef);
        return a;
    };
    {
        AdjIter<T> a0 = iter_args(0);
        a0.next = w.q.list_of(0);
        a0.mask_next = w.q.tmask;  // read by launch 0
        a0.key_next = w.q.keys;
        a0.hist_next = w.q.hist_of(0);
        HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
            hipLaunchKernelGGL((k_adj_seed<T, ND, TX, TY, TZ>), dim3(std::min<int64_t>(b.ntiles, 4096)), dim3(kBlock), 0,
                               s, a0, G);
            return hipGetLastError();
        }));
        ++launched;
    }
    auto step = [&](int64_t t) {
        const AdjIter<T> a = iter_args(t);
        if (ordered) {
            const hipError_t e = timed(prof, EIK_KERNEL_OTHER, [&] {
                hipLaunchKernelGGL(k_tile_split, dim3(split_blocks), dim3(kBlock), 0, s, static_cast<const Sched&>(a));
                return hipGetLastError();
            });
            if (e != hipSuccess) return e;
        }
        return timed(prof, EIK_KERNEL_ADJOINT, [&] {
            hipLaunchKernelGGL((k_adj_tile<T, ND, TX, TY, TZ>), dim3(workgroups_of(ND, o.workgroups)), dim3(kBlock), 0,
                               s, a, G, inner);
            return hipGetLastError();
        });
    };
    int64_t nl = 0;
    eik_status rc = run_loop(step, [&](int64_t t) { return w.q.count_of(static_cast<int>(t % 3)); }, kSub * kPad, cap,
                             async, s, &nl, w.ctl);
    launched += (ordered ? 2 : 1) * nl;
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
        hipLaunchKernelGGL(k_adj_final<T>, dim3(dense), dim3(kBlock), 0, s, static_cast<int>(b.n),
                           static_cast<const T*>(w.D), static_cast<const T*>(w.lam), out);
        return hipGetLastError();
    }));
    ++launched;
    if (async) return rc;
    HostSlots& hs = host_slots();
    HIP_TRY(hipMemcpyAsync(hs.ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hs.blk, w.blkstat, blk_bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (st) {
        *st = eik_stats{};
        st->step3_iters = static_cast<int64_t>(hs.ctl->iters3);
        st->tile_visits_step3 = static_cast<int64_t>(blk_sum(hs.blk, SF_VISITS3, kMaxStatBlocks));
        st->launches = launched;
        HIP_TRY(prof.collect(st));
    }
    return rc;
}

}  // namespace

size_t adjoint_workspace_bytes(const Batch& b, size_t esz) {
    return adj_layout(nullptr, with_tiles(b, adj_tile(b.nd)), esz).bytes;
}

template <typename T>
eik_status adjoint_solve(const Batch& b0, const T* F, const T* phi, const T* g, T* out, const eik_options& o,
                         char* ws, hipStream_t s, eik_stats* st) {
    const Batch b = with_tiles(b0, adj_tile(b0.nd));
    if (b.nd == 2) return adj_run<T, 2, 16, 16, 1>(b, F, phi, g, out, o, ws, s, st);
    return adj_run<T, 3, 8, 8, 8>(b, F, phi, g, out, o, ws, s, st);
}

template eik_status adjoint_solve<float>(const Batch&, const float*, const float*, const float*, float*,
                                         const eik_options&, char*, hipStream_t, eik_stats*);
template eik_status adjoint_solve<double>(const Batch&, const double*, const double*, const double*, double*,
                                          const eik_options&, char*, hipStream_t, eik_stats*);

}  // namespace eik
