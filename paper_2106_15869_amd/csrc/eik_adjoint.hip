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
//   k_adj_tile   tile worklist: each workgroup stages lambda and the stencil
//                data of a tile plus halo in LDS and iterates
//                lambda_j = g_j + sum_{i : j upwind of i} c_{i,axis} lambda_i
//                until nothing in the tile changes; a change on a face
//                schedules the tile across it.  The system is triangular, so
//                the iteration ends at its unique solution whatever the order.
//   k_adj_final  dense: dL/dF = D lambda (0 at sources and unreached nodes).
#include <utility>
#include <vector>

#include "eik_device.hpp"
#include "eik_host.hpp"
#include "eik_seglist.hpp"
#include "eik_batch.hpp"
#include "eik_tile.hpp"

namespace eik {

namespace {

constexpr int GA = 1024;          // workgroups (list segments) per tile launch
constexpr uint8_t kSrc = 0x80u;   // stencil byte: node is a source
// stencil byte bits: axis k present -> bit 2k; upwind on the + side -> bit 2k+1
// (axis 0 = x, 1 = y, 2 = z)

template <typename T>
struct AdjArgs {
    const T* F;
    const T* phi;
    const T* g;      // dL/dphi
    T* lam;
    uint8_t* up;     // stencil bytes
    T* coef;         // 3 per node (x, y, z)
    T* D;
    uint32_t* tstamp;
    SegList cur, next;
    Ctl* ctl;
    int tag_slot;
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
            lam[i] = g[i];
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
template <int ND, int TX, int TY, int TZ>
struct AShape {
    static constexpr int LX = TX + 2, LY = TY + 2, LZ = ND == 3 ? TZ + 2 : 1;
    static constexpr int NT = TX * TY * (ND == 3 ? TZ : 1);
    static constexpr int NL = LX * LY * LZ;
    static constexpr int NPT = (NT + kBlock - 1) / kBlock;
};

__device__ __forceinline__ bool claim_t(uint32_t* ts, int t, uint32_t tag) {
    if (__hip_atomic_load(ts + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= tag) return false;
    return atomicMax(ts + t, tag) < tag;
}

// Initial list: tiles holding a nonzero dL/dphi.
template <typename T, int ND, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_adj_seed(AdjArgs<T> a, BatchGeom<T> bg) {
    using S = AShape<ND, TX, TY, TZ>;
    __shared__ int s_cnt;
    SegAppender app{&s_cnt};
    app.init();
    __syncthreads();
    int lo, hi;
    seg_slice(bg.ntiles, GA, lo, hi);
    for (int t = lo; t < hi; ++t) {
        const Inst<T> g = inst_of(bg, t);
        const int lt = t - g.tile_base;
        const int tx = lt % g.ntx, ty = (lt / g.ntx) % g.nty, tz = lt / (g.ntx * g.nty);
        bool nz = false;
        for (int q = threadIdx.x; q < S::NT; q += kBlock) {
            const int x = tx * TX + q % TX, y = ty * TY + (q / TX) % TY;
            const int z = ND == 3 ? tz * TZ + q / (TX * TY) : 0;
            if (x < g.nx && y < g.ny && z < g.nz) nz |= a.g[g.node_base + (z * g.ny + y) * g.nx + x] != T(0);
        }
        if (__syncthreads_or(nz) && threadIdx.x == 0 && claim_t(a.tstamp, t, 1u)) app.push_one(a.next, t);
    }
    __syncthreads();
    app.publish(a.next);
}

template <typename T, int ND, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_adj_tile(AdjArgs<T> a, BatchGeom<T> bg, int inner) {
    using S = AShape<ND, TX, TY, TZ>;
    __shared__ T slam[S::NL];
    __shared__ T scoef[3 * S::NL];
    __shared__ uint8_t sup[S::NL];
    __shared__ int s_pref[GA + 1];
    __shared__ int s_cnt;
    __shared__ int s_face;
    SegAppender app{&s_cnt};
    app.init();
    const uint32_t tag = static_cast<uint32_t>(a.ctl->tag[a.tag_slot]);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->tag[a.tag_slot ^ 1] = static_cast<int>(tag + 1);
    const uint32_t ntag = tag + 1;
    const int n = seg_prefix<GA>(a.cur.count, s_pref);
    if (blockIdx.x == 0 && threadIdx.x == 0 && n > 0) {
        a.ctl->iters3 += 1;
        a.ctl->visits3 += static_cast<unsigned long long>(n);
    }
    int lo, hi;
    seg_slice(n, GA, lo, hi);
    const int sty = S::LX, stz = S::LX * S::LY;
    for (int e = lo; e < hi; ++e) {
        const int t = seg_entry<GA>(a.cur, s_pref, e);
        const Inst<T> g = inst_of(bg, t);
        const int lt = t - g.tile_base;
        const int tx = lt % g.ntx, ty = (lt / g.ntx) % g.nty, tz = lt / (g.ntx * g.nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * (ND == 3 ? TZ : 1);
        for (int q = threadIdx.x; q < S::NL; q += kBlock) {
            const int lx = q % S::LX, ly = (q / S::LX) % S::LY, lz = q / (S::LX * S::LY);
            const int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = ND == 3 ? z0 + lz - 1 : 0;
            const bool in = gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz;
            if (in) {
                const int G = g.node_base + (gz * g.ny + gy) * g.nx + gx;
                slam[q] = a.lam[G];
                sup[q] = a.up[G];
                scoef[3 * q + 0] = a.coef[3 * static_cast<size_t>(G) + 0];
                scoef[3 * q + 1] = a.coef[3 * static_cast<size_t>(G) + 1];
                scoef[3 * q + 2] = a.coef[3 * static_cast<size_t>(G) + 2];
            } else {
                slam[q] = T(0);
                sup[q] = 0;
                scoef[3 * q + 0] = scoef[3 * q + 1] = scoef[3 * q + 2] = T(0);
            }
        }
        if (threadIdx.x == 0) s_face = 0;
        int Lr[S::NPT], Gr[S::NPT], facer[S::NPT];
        bool ok[S::NPT];
        T gr[S::NPT], lam0[S::NPT];
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) {
            const int nn = threadIdx.x + r * kBlock;
            const int x = nn % TX, y = (nn / TX) % TY, z = ND == 3 ? nn / (TX * TY) : 0;
            const int gx = x0 + x, gy = y0 + y, gz = z0 + z;
            ok[r] = nn < S::NT && gx < g.nx && gy < g.ny && gz < g.nz;
            Gr[r] = g.node_base + (gz * g.ny + gy) * g.nx + gx;
            Lr[r] = ((ND == 3 ? z + 1 : 0) * S::LY + (y + 1)) * S::LX + (x + 1);
            int f = 0;
            if (x == 0 && gx > 0) f |= 1;
            if (x == TX - 1 && gx + 1 < g.nx) f |= 2;
            if (y == 0 && gy > 0) f |= 4;
            if (y == TY - 1 && gy + 1 < g.ny) f |= 8;
            if (ND == 3) {
                if (z == 0 && gz > 0) f |= 16;
                if (z == TZ - 1 && gz + 1 < g.nz) f |= 32;
            }
            facer[r] = f;
            gr[r] = ok[r] ? a.g[Gr[r]] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < S::NPT; ++r) lam0[r] = ok[r] ? slam[Lr[r]] : T(0);
        bool pending = false;
        for (int it = 0;; ++it) {
            T nv[S::NPT];
            bool ch[S::NPT];
            bool has = false;
#pragma unroll
            for (int r = 0; r < S::NPT; ++r) {
                ch[r] = false;
                nv[r] = T(0);
                if (!ok[r]) continue;
                const int L = Lr[r];
                T v = gr[r];
                // neighbour i on the - side of axis k pulls into j if its upwind on
                // axis k is its + side; on the + side, if its upwind is its - side
                const int offs[6] = {-1, 1, -sty, sty, -stz, stz};
#pragma unroll
                for (int d = 0; d < 2 * ND; ++d) {
                    const int k = d >> 1;
                    const int q = L + offs[d];
                    const uint32_t u = sup[q];
                    const bool present = (u & (1u << (2 * k))) && !(u & kSrc);
                    const bool plus = (u >> (2 * k + 1)) & 1u;
                    if (present && plus == ((d & 1) == 0)) v = v + scoef[3 * q + k] * slam[q];
                }
                nv[r] = v;
                ch[r] = v != slam[L];
                has |= ch[r];
            }
            pending = __syncthreads_or(has);
            if (!pending || it == inner) break;
            int fm = 0;
#pragma unroll
            for (int r = 0; r < S::NPT; ++r) {
                if (!ch[r]) continue;
                slam[Lr[r]] = nv[r];
                // j's own upwind neighbours pull from j: schedule tiles across faces it
                // has an upwind neighbour on
                const uint32_t u = sup[Lr[r]];
#pragma unroll
                for (int d = 0; d < 2 * ND; ++d) {
                    const int k = d >> 1;
                    const bool present = u & (1u << (2 * k));
                    const bool plus = (u >> (2 * k + 1)) & 1u;
                    if ((facer[r] & (1 << d)) && present && plus == ((d & 1) == 1)) fm |= 1 << d;
                }
            }
            if (fm) atomicOr(&s_face, fm);
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < S::NPT; ++r)
            if (ok[r] && slam[Lr[r]] != lam0[r]) a.lam[Gr[r]] = slam[Lr[r]];
        __syncthreads();
        if (threadIdx.x == 0) {
            if (pending && claim_t(a.tstamp, t, ntag)) app.push_one(a.next, t);
            const int fm = s_face;
            for (int d = 0; d < 2 * ND; ++d) {
                if (!(fm & (1 << d))) continue;
                int tn = t;
                switch (d) {
                    case 0: tn = t - 1; break;
                    case 1: tn = t + 1; break;
                    case 2: tn = t - g.ntx; break;
                    case 3: tn = t + g.ntx; break;
                    case 4: tn = t - g.ntx * g.nty; break;
                    default: tn = t + g.ntx * g.nty; break;
                }
                if (claim_t(a.tstamp, tn, ntag)) app.push_one(a.next, tn);
            }
        }
        __syncthreads();
    }
    app.publish(a.next);
}


struct AdjWs {
    Ctl* ctl;
    uint8_t* up;
    void* coef;
    void* D;
    void* lam;
    uint32_t* tstamp;
    SegList seg[2];
    void* table;
    int* tile_inst;
    size_t bytes;
};

TileCfg adj_tile(int nd) { return nd == 2 ? TileCfg{32, 32, 1} : TileCfg{8, 8, 8}; }

AdjWs adj_layout(char* base, const Batch& b, size_t esz) {
    AdjWs w{};
    size_t off = 0;
    auto take = [&](size_t n) {
        char* p = base ? base + off : nullptr;
        off = align_up(off + n, 256);
        return p;
    };
    const size_t n = static_cast<size_t>(b.n);
    const int cap = static_cast<int>(7 * ((b.ntiles + GA - 1) / GA) + 512);
    w.ctl = reinterpret_cast<Ctl*>(take(sizeof(Ctl)));
    w.up = reinterpret_cast<uint8_t*>(take(n));
    w.coef = take(3 * esz * n);
    w.D = take(esz * n);
    w.lam = take(esz * n);
    w.tstamp = reinterpret_cast<uint32_t*>(take(4 * static_cast<size_t>(b.ntiles)));
    for (int k = 0; k < 2; ++k) {
        w.seg[k].cap = cap;
        w.seg[k].count = reinterpret_cast<int*>(take(4 * static_cast<size_t>(GA)));
        w.seg[k].data = reinterpret_cast<int*>(take(4 * static_cast<size_t>(cap) * GA));
    }
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
    AdjWs w = adj_layout(ws, b, sizeof(T));
    const int64_t cap = o.max_iters > 0 ? o.max_iters : 4 * b.n + 64;
    const int inner = o.inner_iters > 0 ? o.inner_iters : 4 * (TX + TY + TZ);
    const int dense = static_cast<int>(std::min<int64_t>((b.n + kBlock - 1) / kBlock, 1 << 20));
    const int tiles = static_cast<int>(std::min<int64_t>(b.ntiles, 1 << 16));
    int64_t launched = 0;
    Profiler prof;
    prof.start((o.flags & EIK_FLAG_PROFILE) != 0, s);

    BatchGeom<T> G;
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return upload_batch_geom<T>(b, w.table, w.tile_inst, s, G, launched); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] { return launch_ctl_init(w.ctl, s); }));
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
        hipLaunchKernelGGL((k_adj_prep<T, ND, TX, TY, TZ>), dim3(tiles), dim3(kBlock), 0, s, G, F, phi, w.up,
                           static_cast<T*>(w.coef), static_cast<T*>(w.D), static_cast<T*>(w.lam), g);
        return hipGetLastError();
    }));
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
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER,
                  [&] { return launch_zero_words(w.tstamp, 4 * static_cast<size_t>(b.ntiles), s); }));
    AdjArgs<T> a{};
    a.F = F;
    a.phi = phi;
    a.g = g;
    a.lam = static_cast<T*>(w.lam);
    a.up = w.up;
    a.coef = static_cast<T*>(w.coef);
    a.D = static_cast<T*>(w.D);
    a.tstamp = w.tstamp;
    a.ctl = w.ctl;
    a.next = w.seg[0];
    // seeding claims with tag 1; the tag chain starts at tag[0] = 1 -> claims 2, ...
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
        hipLaunchKernelGGL((k_adj_seed<T, ND, TX, TY, TZ>), dim3(GA), dim3(kBlock), 0, s, a, G);
        return hipGetLastError();
    }));
    launched += 4;
    auto step = [&](int64_t t) {
        AdjArgs<T> c = a;
        c.cur = w.seg[t & 1];
        c.next = w.seg[(t + 1) & 1];
        c.tag_slot = static_cast<int>(t & 1);
        return timed(prof, EIK_KERNEL_ADJOINT, [&] {
            hipLaunchKernelGGL((k_adj_tile<T, ND, TX, TY, TZ>), dim3(GA), dim3(kBlock), 0, s, c, G, inner);
            return hipGetLastError();
        });
    };
    int64_t nl = 0;
    eik_status rc = run_loop(step, [&](int64_t t) { return w.seg[t & 1].count; }, GA, cap, async, s, &nl);
    launched += nl;
    HIP_TRY(timed(prof, EIK_KERNEL_OTHER, [&] {
        hipLaunchKernelGGL(k_adj_final<T>, dim3(dense), dim3(kBlock), 0, s, static_cast<int>(b.n),
                           static_cast<const T*>(w.D), static_cast<const T*>(w.lam), out);
        return hipGetLastError();
    }));
    ++launched;
    if (async) return rc;
    HostSlots& hs = host_slots();
    HIP_TRY(hipMemcpyAsync(hs.ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (st) {
        *st = eik_stats{};
        st->step3_iters = static_cast<int64_t>(hs.ctl->iters3);
        st->tile_visits_step3 = static_cast<int64_t>(hs.ctl->visits3);
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
    if (b.nd == 2) return adj_run<T, 2, 32, 32, 1>(b, F, phi, g, out, o, ws, s, st);
    return adj_run<T, 3, 8, 8, 8>(b, F, phi, g, out, o, ws, s, st);
}

template eik_status adjoint_solve<float>(const Batch&, const float*, const float*, const float*, float*,
                                         const eik_options&, char*, hipStream_t, eik_stats*);
template eik_status adjoint_solve<double>(const Batch&, const double*, const double*, const double*, double*,
                                          const eik_options&, char*, hipStream_t, eik_stats*);

}  // namespace eik
