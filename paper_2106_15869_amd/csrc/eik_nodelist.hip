// Node-list IFIM kernels for gfx950: one lane per list entry (Section 3.2).
//
// Algorithm 2 in device form:
//   STEP 1  k_init / k_seed / k_seed_active   phi = +inf, sources fixed,
//           Active = FAR neighbours of the sources (F > 0).
//   STEP 2  k_step2 (in place) or k_step2_eval + k_step2_apply (synchronous
//           reads): G_i for every active node; converged nodes (phi - phi~ <=
//           eps) join the Source set and activate their FAR neighbours without
//           any convergence check of those neighbours; the rest keep the new
//           value and stay active.
//   STEP 3  k_detect: G_i for every non-source node, nodes whose value would
//           drop form the Remedy list; k_remedy (or eval + apply): changed
//           nodes take the new value and, with their neighbours, form the
//           next Remedy list.
// Lists are int32 node indices in per-workgroup segments (eik_seglist.hpp):
// each wave compacts its items with a lane prefix sum and reserves room with
// one LDS atomic.  Labels are bytes changed with word atomics.
#include <algorithm>

#include "eik_device.hpp"
#include "eik_internal.hpp"
#include "eik_seglist.hpp"

namespace eik {

static __host__ __device__ inline Grid make_grid(const GridDims& d) {
    Grid g;
    g.nx = d.nx;
    g.ny = d.ny;
    g.nz = d.nz;
    g.n = d.n;
    g.sxy = d.nx * d.ny;
    return g;
}

// Neighbour slots in a fixed order: -x, +x, -y, +y, -z, +z.
template <int ND>
__device__ __forceinline__ void neighbour_slots(const Grid& g, int i, int x, int y, int z,
                                                int (&nb)[6], uint32_t& valid) {
    valid = 0;
    nb[0] = i - 1;
    nb[1] = i + 1;
    nb[2] = i - g.nx;
    nb[3] = i + g.nx;
    nb[4] = i - g.sxy;
    nb[5] = i + g.sxy;
    if (x > 0) valid |= 1u;
    if (x + 1 < g.nx) valid |= 2u;
    if (y > 0) valid |= 4u;
    if (y + 1 < g.ny) valid |= 8u;
    if (ND == 3) {
        if (z > 0) valid |= 16u;
        if (z + 1 < g.nz) valid |= 32u;
    }
}

// ---------------------------------------------------------------------------
// STEP 1
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(const T* __restrict__ F, T* __restrict__ phi,
                                                 uint8_t* __restrict__ lab,
                                                 uint32_t* __restrict__ stamp, int n, Ctl* ctl) {
    const T inf = pos_inf<T>();
    bool bad = false;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        T f = F[i];
        bad |= !(f >= T(0)) || !(f < inf);
        phi[i] = inf;
        lab[i] = static_cast<uint8_t>(L_FAR);
        if (stamp) stamp[i] = 0u;
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(&ctl->err, 1);
}

template <typename T>
__global__ void k_seed(T* __restrict__ phi, uint8_t* __restrict__ lab, SrcBatch<T> b) {
    int k = threadIdx.x;
    if (k < b.count) {
        phi[b.idx[k]] = b.val[k];
        lab[b.idx[k]] = static_cast<uint8_t>(L_FIXED);
    }
}

// One wave: FAR neighbours (F > 0) of a batch of sources become active and are
// appended to segment `seg` of `out`.
template <typename T, int ND>
__global__ void k_seed_active(GridDims gd, const T* __restrict__ F, uint8_t* lab, SrcBatch<T> b,
                              SegList out, int seg) {
    const Grid g = make_grid(gd);
    int k = threadIdx.x;
    int items[6];
    uint32_t mask = 0;
    if (k < b.count) {
        int i = b.idx[k], x, y, z;
        decode<ND>(g, i, x, y, z);
        uint32_t valid;
        neighbour_slots<ND>(g, i, x, y, z, items, valid);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            if ((valid >> j) & 1u) {
                int q = items[j];
                if (label_get(lab, q) == L_FAR && F[q] > T(0) && label_cas(lab, q, L_FAR, L_ACTIVE))
                    mask |= 1u << j;
            }
        }
    }
    const int c = __popc(mask);
    const int incl = wave_incl_scan(c);
    const int total = __shfl(incl, 63, 64);
    if (total == 0) return;
    int base = 0;
    if (lane_id() == 63) base = atomicAdd(out.count + seg, total);
    base = __shfl(base, 63, 64);
    int* dst = out.data + static_cast<size_t>(seg) * out.cap + base + incl - c;
#pragma unroll
    for (int j = 0; j < 6; ++j)
        if (mask & (1u << j)) dst[__popc(mask & ((1u << j) - 1u))] = items[j];
}

__global__ void k_seg_clear(int* count, int nseg) {
    for (int i = threadIdx.x; i < nseg; i += blockDim.x) count[i] = 0;
}

__global__ void k_zero_words(uint32_t* p, int n) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = 0u;
}

__global__ void k_fill_words(uint32_t* p, int n, uint32_t v) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) p[i] = v;
}

// ---------------------------------------------------------------------------
// STEP 2
// ---------------------------------------------------------------------------
constexpr int G = kNodeSegs;

// Shared by the in-place and the synchronous-read apply kernels.
template <typename T, int ND>
__device__ __forceinline__ uint32_t step2_apply_node(const NodeIter<T>& a, const Grid& g, int i,
                                                     T pi, T pt, T eps, int (&items)[7], int& written) {
    const T inf = pos_inf<T>();
    uint32_t mask = 0;
    if (pt < inf && pi - pt <= eps) {
        // converged: joins the Source set; FAR neighbours become active
        label_add(a.lab, i, int(L_CONV) - int(L_ACTIVE));
        int x, y, z;
        decode<ND>(g, i, x, y, z);
        int nb[6];
        uint32_t valid;
        neighbour_slots<ND>(g, i, x, y, z, nb, valid);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            items[j] = nb[j];
            if ((valid >> j) & 1u) {
                int q = nb[j];
                if (label_get(a.lab, q) == L_FAR && a.F[q] > T(0) &&
                    label_cas(a.lab, q, L_FAR, L_ACTIVE))
                    mask |= 1u << j;
            }
        }
    } else if (!(pt < inf)) {
        // nothing finite upwind: not converged, back to FAR
        label_add(a.lab, i, int(L_FAR) - int(L_ACTIVE));
    } else {
        if (pt < pi) {
            a.phi[i] = pt;
            ++written;
        }
        items[6] = i;
        mask = 1u << 6;
    }
    return mask;
}

// Block-wide: add the lanes' counts to this workgroup's statistics column.
__device__ __forceinline__ void flush_written(unsigned long long* blkstat, int field, int* s_w, int mine) {
    if (mine) atomicAdd(s_w, mine);
    __syncthreads();
    if (threadIdx.x == 0) blk_add(blkstat, field, G, static_cast<unsigned long long>(*s_w));
}

// Loads the list lengths, updates the per-iteration counters (block 0) and
// returns this workgroup's slice.
template <typename T>
__device__ __forceinline__ int list_prologue(const NodeIter<T>& a, int* s_pref, bool step2, int& lo,
                                             int& hi) {
    const int n = seg_prefix<G>(a.cur.count, s_pref);
    if (blockIdx.x == 0 && threadIdx.x == 0 && n > 0) {
        const unsigned long long un = static_cast<unsigned long long>(n);
        if (step2) {
            a.ctl->iters2 += 1;
            a.ctl->evals2 += un;
            if (un > a.ctl->max_active) a.ctl->max_active = un;
        } else {
            a.ctl->iters3 += 1;
            a.ctl->evals_rem += un;
        }
    }
    if (!step2 && blockIdx.x == 0 && threadIdx.x == 0 && a.first)
        a.ctl->remedy_init = static_cast<unsigned long long>(n);
    seg_slice(n, G, lo, hi);
    return n;
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_step2(NodeIter<T> a, GridDims gd, Spacing<T> sp, T eps) {
    __shared__ int s_pref[G + 1];
    __shared__ int s_cnt;
    __shared__ int s_w;
    const Grid g = make_grid(gd);
    SegAppender app{&s_cnt};
    app.init();
    if (threadIdx.x == 0) s_w = 0;
    int written = 0;
    int lo, hi;
    list_prologue(a, s_pref, true, lo, hi);
    for (int base = lo; base < hi; base += kBlock) {
        const int k = base + threadIdx.x;
        int items[7];
        uint32_t mask = 0;
        if (k < hi) {
            const int i = seg_entry<G>(a.cur, s_pref, k);
            int x, y, z;
            decode<ND>(g, i, x, y, z);
            const T pi = a.phi[i];
            const T pt = eval_node<T, ND>(a.phi, a.F, g, i, x, y, z, sp);
            mask = step2_apply_node<T, ND>(a, g, i, pi, pt, eps, items, written);
        }
        app.push_mask<7>(a.next, items, mask);
    }
    flush_written(a.blkstat, SF_WRITTEN2, &s_w, written);
    app.publish(a.next);
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_step2_eval(NodeIter<T> a, GridDims gd, Spacing<T> sp) {
    __shared__ int s_pref[G + 1];
    const Grid g = make_grid(gd);
    int lo, hi;
    list_prologue(a, s_pref, true, lo, hi);
    for (int k = lo + static_cast<int>(threadIdx.x); k < hi; k += kBlock) {
        const int i = seg_entry<G>(a.cur, s_pref, k);
        int x, y, z;
        decode<ND>(g, i, x, y, z);
        a.vals[k] = eval_node<T, ND>(a.phi, a.F, g, i, x, y, z, sp);
    }
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_step2_apply(NodeIter<T> a, GridDims gd, T eps) {
    __shared__ int s_pref[G + 1];
    __shared__ int s_cnt;
    __shared__ int s_w;
    const Grid g = make_grid(gd);
    SegAppender app{&s_cnt};
    app.init();
    if (threadIdx.x == 0) s_w = 0;
    int written = 0;
    const int n = seg_prefix<G>(a.cur.count, s_pref);
    int lo, hi;
    seg_slice(n, G, lo, hi);
    for (int base = lo; base < hi; base += kBlock) {
        const int k = base + threadIdx.x;
        int items[7];
        uint32_t mask = 0;
        if (k < hi) {
            const int i = seg_entry<G>(a.cur, s_pref, k);
            mask = step2_apply_node<T, ND>(a, g, i, a.phi[i], a.vals[k], eps, items, written);
        }
        app.push_mask<7>(a.next, items, mask);
    }
    flush_written(a.blkstat, SF_WRITTEN2, &s_w, written);
    app.publish(a.next);
}

// ---------------------------------------------------------------------------
// STEP 3
// ---------------------------------------------------------------------------
template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_detect(GridDims gd, const T* __restrict__ F,
                                                   const T* __restrict__ phi,
                                                   const uint8_t* __restrict__ lab, Spacing<T> sp,
                                                   T eps, SegList out) {
    __shared__ int s_cnt;
    const Grid g = make_grid(gd);
    SegAppender app{&s_cnt};
    app.init();
    __syncthreads();
    int lo, hi;
    seg_slice(g.n, G, lo, hi);
    for (int base = lo; base < hi; base += kBlock) {
        const int i = base + threadIdx.x;
        int items[1] = {i};
        uint32_t mask = 0;
        if (i < hi && lab[i] != L_FIXED) {
            int x, y, z;
            decode<ND>(g, i, x, y, z);
            const T pt = eval_node<T, ND>(phi, F, g, i, x, y, z, sp);
            mask = pt < phi[i] - eps ? 1u : 0u;
        }
        app.push_mask<1>(out, items, mask);
    }
    __syncthreads();
    app.publish(out);
}

// claim node q for the next remedy list (first claimer this iteration wins)
__device__ __forceinline__ bool claim(uint32_t* stamp, int q, uint32_t tag) {
    if (__hip_atomic_load(stamp + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= tag) return false;
    return atomicMax(stamp + q, tag) < tag;
}

template <typename T, int ND>
__device__ __forceinline__ uint32_t remedy_apply_node(const NodeIter<T>& a, const Grid& g, int i,
                                                      T pi, T pt, T eps, uint32_t tag,
                                                      int (&items)[7], int& written) {
    uint32_t mask = 0;
    if (pt < pi - eps) {
        a.phi[i] = pt;
        ++written;
        int x, y, z;
        decode<ND>(g, i, x, y, z);
        int nb[6];
        uint32_t valid;
        neighbour_slots<ND>(g, i, x, y, z, nb, valid);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            items[j] = nb[j];
            if ((valid >> j) & 1u) {
                int q = nb[j];
                if (label_get(a.lab, q) != L_FIXED && claim(a.stamp, q, tag)) mask |= 1u << j;
            }
        }
        items[6] = i;
        if (claim(a.stamp, i, tag)) mask |= 1u << 6;
    }
    return mask;
}

// Remedy iterations advance the stamp tag: the iteration with slot p reads
// tag[p] and block 0 stores tag[p] + 1 into tag[p ^ 1] for the next one.
template <typename T>
__device__ __forceinline__ uint32_t remedy_tag(const NodeIter<T>& a, bool advance) {
    const uint32_t tag = static_cast<uint32_t>(a.ctl->tag[a.tag_slot]);
    if (advance && blockIdx.x == 0 && threadIdx.x == 0) a.ctl->tag[a.tag_slot ^ 1] = static_cast<int>(tag + 1);
    return tag;
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_remedy(NodeIter<T> a, GridDims gd, Spacing<T> sp, T eps) {
    __shared__ int s_pref[G + 1];
    __shared__ int s_cnt;
    __shared__ int s_w;
    const Grid g = make_grid(gd);
    const uint32_t tag = remedy_tag(a, true);
    SegAppender app{&s_cnt};
    app.init();
    if (threadIdx.x == 0) s_w = 0;
    int written = 0;
    int lo, hi;
    list_prologue(a, s_pref, false, lo, hi);
    for (int base = lo; base < hi; base += kBlock) {
        const int k = base + threadIdx.x;
        int items[7];
        uint32_t mask = 0;
        if (k < hi) {
            const int i = seg_entry<G>(a.cur, s_pref, k);
            int x, y, z;
            decode<ND>(g, i, x, y, z);
            const T pt = eval_node<T, ND>(a.phi, a.F, g, i, x, y, z, sp);
            mask = remedy_apply_node<T, ND>(a, g, i, a.phi[i], pt, eps, tag, items, written);
        }
        app.push_mask<7>(a.next, items, mask);
    }
    flush_written(a.blkstat, SF_WRITTEN3, &s_w, written);
    app.publish(a.next);
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_remedy_eval(NodeIter<T> a, GridDims gd, Spacing<T> sp) {
    __shared__ int s_pref[G + 1];
    const Grid g = make_grid(gd);
    remedy_tag(a, true);
    int lo, hi;
    list_prologue(a, s_pref, false, lo, hi);
    for (int k = lo + static_cast<int>(threadIdx.x); k < hi; k += kBlock) {
        const int i = seg_entry<G>(a.cur, s_pref, k);
        int x, y, z;
        decode<ND>(g, i, x, y, z);
        a.vals[k] = eval_node<T, ND>(a.phi, a.F, g, i, x, y, z, sp);
    }
}

// The apply kernel of the synchronous mode uses the tag its eval kernel read.
template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_remedy_apply(NodeIter<T> a, GridDims gd, T eps) {
    __shared__ int s_pref[G + 1];
    __shared__ int s_cnt;
    __shared__ int s_w;
    const Grid g = make_grid(gd);
    const uint32_t tag = remedy_tag(a, false);
    SegAppender app{&s_cnt};
    app.init();
    if (threadIdx.x == 0) s_w = 0;
    int written = 0;
    const int n = seg_prefix<G>(a.cur.count, s_pref);
    int lo, hi;
    seg_slice(n, G, lo, hi);
    for (int base = lo; base < hi; base += kBlock) {
        const int k = base + threadIdx.x;
        int items[7];
        uint32_t mask = 0;
        if (k < hi) {
            const int i = seg_entry<G>(a.cur, s_pref, k);
            mask = remedy_apply_node<T, ND>(a, g, i, a.phi[i], a.vals[k], eps, tag, items, written);
        }
        app.push_mask<7>(a.next, items, mask);
    }
    flush_written(a.blkstat, SF_WRITTEN3, &s_w, written);
    app.publish(a.next);
}

// ---------------------------------------------------------------------------
// FIM (Section 2.3), the method the improved variant is compared against.
// One iteration is two launches:
//   k_fim_update  every active node is updated; a node whose value no longer
//                 changes (phi - phi~ <= eps) leaves the list and goes to the
//                 converged list, the others keep the new value and stay;
//   k_fim_check   every neighbour of a converged node that is not active is
//                 evaluated; if its value drops it takes the new value and
//                 (re)joins the active list.
// Converged nodes can therefore be reactivated, and the loop ends with the
// active list empty.  The check evaluations are the work the improved method
// removes from the update step.
// ---------------------------------------------------------------------------

// phi[i] = min(phi[i], v) for any sign of the values.
__device__ __forceinline__ void atomic_min_value(float* p, float v) {
    unsigned int* w = reinterpret_cast<unsigned int*>(p);
    unsigned int old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (v < __uint_as_float(old)) {
        const unsigned int prev = atomicCAS(w, old, __float_as_uint(v));
        if (prev == old) return;
        old = prev;
    }
}
__device__ __forceinline__ void atomic_min_value(double* p, double v) {
    unsigned long long* w = reinterpret_cast<unsigned long long*>(p);
    unsigned long long old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (v < __longlong_as_double(static_cast<long long>(old))) {
        const unsigned long long prev =
            atomicCAS(w, old, static_cast<unsigned long long>(__double_as_longlong(v)));
        if (prev == old) return;
        old = prev;
    }
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_fim_update(NodeIter<T> a, GridDims gd, Spacing<T> sp, T eps) {
    __shared__ int s_pref[G + 1];
    __shared__ int s_cnt, s_cnt_conv;
    __shared__ int s_w;
    const Grid g = make_grid(gd);
    SegAppender keep{&s_cnt}, conv{&s_cnt_conv};
    keep.init();
    conv.init();
    if (threadIdx.x == 0) s_w = 0;
    int written = 0;
    int lo, hi;
    list_prologue(a, s_pref, true, lo, hi);
    const T inf = pos_inf<T>();
    for (int base = lo; base < hi; base += kBlock) {
        const int k = base + threadIdx.x;
        int item[1] = {0};
        uint32_t mkeep = 0, mconv = 0;
        if (k < hi) {
            const int i = seg_entry<G>(a.cur, s_pref, k);
            item[0] = i;
            int x, y, z;
            decode<ND>(g, i, x, y, z);
            const T pi = a.phi[i];
            const T pt = eval_node<T, ND>(a.phi, a.F, g, i, x, y, z, sp);
            if (pt < inf && pi - pt <= eps) {
                label_add(a.lab, i, int(L_CONV) - int(L_ACTIVE));
                mconv = 1u;
            } else if (!(pt < inf)) {
                label_add(a.lab, i, int(L_FAR) - int(L_ACTIVE));
            } else {
                if (pt < pi) {
                    a.phi[i] = pt;
                    ++written;
                }
                mkeep = 1u;
            }
        }
        keep.push_mask<1>(a.next, item, mkeep);
        conv.push_mask<1>(a.conv, item, mconv);
    }
    flush_written(a.blkstat, SF_WRITTEN2, &s_w, written);
    keep.publish(a.next);
    conv.publish(a.conv);
}

// Reads the converged list of this iteration and appends to the active list
// after the entries k_fim_update published there.
template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_fim_check(NodeIter<T> a, GridDims gd, Spacing<T> sp, T eps) {
    __shared__ int s_pref[G + 1];
    __shared__ int s_cnt;
    __shared__ int s_w, s_e;
    const Grid g = make_grid(gd);
    SegAppender app{&s_cnt};
    app.resume(a.next);
    if (threadIdx.x == 0) s_w = s_e = 0;
    int written = 0, evals = 0;
    const int n = seg_prefix<G>(a.conv.count, s_pref);
    int lo, hi;
    seg_slice(n, G, lo, hi);
    for (int base = lo; base < hi; base += kBlock) {
        const int k = base + threadIdx.x;
        int items[6];
        uint32_t mask = 0;
        if (k < hi) {
            const int i = seg_entry<G>(a.conv, s_pref, k);
            int x, y, z;
            decode<ND>(g, i, x, y, z);
            uint32_t valid;
            neighbour_slots<ND>(g, i, x, y, z, items, valid);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                if (!((valid >> j) & 1u)) continue;
                const int q = items[j];
                const uint32_t lb = label_get(a.lab, q);
                if (lb == L_ACTIVE || lb == L_FIXED || !(a.F[q] > T(0))) continue;
                int qx, qy, qz;
                decode<ND>(g, q, qx, qy, qz);
                ++evals;
                const T pt = eval_node<T, ND>(a.phi, a.F, g, q, qx, qy, qz, sp);
                if (pt < a.phi[q] - eps) {
                    atomic_min_value(a.phi + q, pt);
                    ++written;
                    if (label_cas(a.lab, q, lb, L_ACTIVE)) mask |= 1u << j;
                }
            }
        }
        app.push_mask<6>(a.next, items, mask);
    }
    if (evals) atomicAdd(&s_e, evals);
    flush_written(a.blkstat, SF_WRITTEN2, &s_w, written);
    if (threadIdx.x == 0) blk_add(a.blkstat, SF_CHECK, G, static_cast<unsigned long long>(s_e));
    app.publish(a.next);
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_apply_local(GridDims gd, const T* __restrict__ F,
                                                        const T* __restrict__ phi, Spacing<T> sp,
                                                        T* __restrict__ out) {
    const Grid g = make_grid(gd);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < g.n; i += gridDim.x * kBlock) {
        int x, y, z;
        decode<ND>(g, i, x, y, z);
        out[i] = eval_node<T, ND>(phi, F, g, i, x, y, z, sp);
    }
}

__global__ void k_reset_counters(Ctl* ctl) {
    if (threadIdx.x < 4) ctl->cnt[threadIdx.x] = 0;
}

// Zero the whole control block (runs before any kernel of a solve).
__global__ void k_ctl_init(Ctl* ctl) {
    if (threadIdx.x == 0) {
        for (int k = 0; k < 4; ++k) ctl->cnt[k] = 0;
        ctl->err = 0;
        ctl->open_lists = 0;
        ctl->tag[0] = 1;
        ctl->tag[1] = 1;
        ctl->iters2 = ctl->iters3 = ctl->evals2 = ctl->evals_det = ctl->evals_rem = 0;
        ctl->remedy_init = ctl->max_active = 0;
        ctl->visits2 = ctl->visits3 = ctl->inner2 = ctl->inner3 = 0;
    }
}

// Whether the list a loop would drain next still holds work (one block; the
// length words of unused slots are zero).
__global__ __launch_bounds__(kBlock) void k_loop_status(Ctl* ctl, const int* counts, int nseg) {
    int any = 0;
    for (int k = threadIdx.x; k < nseg; k += kBlock) any |= counts[k] != 0;
    if (__syncthreads_or(any) && threadIdx.x == 0) ctl->open_lists = 1;
}

// Totals of the per-workgroup statistics: field f summed over its nblocks
// columns lands in word f of the array (one block; every column is read
// before any total is written), so a read-back moves kStatFields words.
__global__ __launch_bounds__(kBlock) void k_sum_stats(unsigned long long* blk, int nblocks) {
    __shared__ unsigned long long part[kBlock];
    __shared__ unsigned long long tot[kStatFields];
    for (int f = 0; f < kStatFields; ++f) {
        unsigned long long v = 0;
        for (int b = threadIdx.x; b < nblocks; b += kBlock) v += blk[f * nblocks + b];
        part[threadIdx.x] = v;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) tot[f] = part[0];
        __syncthreads();
    }
    if (threadIdx.x < kStatFields) blk[threadIdx.x] = tot[threadIdx.x];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int dense_blocks(int n) {
    long long b = (static_cast<long long>(n) + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > (1 << 20)) b = 1 << 20;
    return static_cast<int>(b);
}

template <typename T>
hipError_t launch_init(const T* F, T* phi, uint8_t* lab, uint32_t* stamp, int n, Ctl* ctl,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_init<T>, dim3(dense_blocks(n)), dim3(kBlock), 0, s, F, phi, lab, stamp, n,
                       ctl);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_seed(T* phi, uint8_t* lab, const SrcBatch<T>& b, hipStream_t s) {
    hipLaunchKernelGGL(k_seed<T>, dim3(1), dim3(kMaxSrcBatch), 0, s, phi, lab, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_seed_active(const GridDims& g, const T* F, uint8_t* lab, const SrcBatch<T>& b,
                              const SegList& out, int seg, hipStream_t s) {
    if (g.nd == 2)
        hipLaunchKernelGGL((k_seed_active<T, 2>), dim3(1), dim3(kMaxSrcBatch), 0, s, g, F, lab, b,
                           out, seg);
    else
        hipLaunchKernelGGL((k_seed_active<T, 3>), dim3(1), dim3(kMaxSrcBatch), 0, s, g, F, lab, b,
                           out, seg);
    return hipGetLastError();
}

hipError_t launch_zero_words(void* p, size_t bytes, hipStream_t s) {
    const int n = static_cast<int>(bytes / 4);
    hipLaunchKernelGGL(k_zero_words, dim3(std::min((n + kBlock - 1) / kBlock, 1024)), dim3(kBlock), 0, s,
                       static_cast<uint32_t*>(p), n);
    return hipGetLastError();
}

hipError_t launch_fill_words(void* p, size_t n, uint32_t v, hipStream_t s) {
    const int m = static_cast<int>(n);
    hipLaunchKernelGGL(k_fill_words, dim3(std::min((m + kBlock - 1) / kBlock, 1024)), dim3(kBlock), 0, s,
                       static_cast<uint32_t*>(p), m, v);
    return hipGetLastError();
}

hipError_t launch_seg_clear(int* count, int nseg, hipStream_t s) {
    hipLaunchKernelGGL(k_seg_clear, dim3(1), dim3(kBlock), 0, s, count, nseg);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step2(const GridDims& g, const NodeIter<T>& it, const Spacing<T>& h, T eps, bool det, hipStream_t s) {
    if (det) {
        if (g.nd == 2) {
            hipLaunchKernelGGL((k_step2_eval<T, 2>), dim3(G), dim3(kBlock), 0, s, it, g, h);
            hipLaunchKernelGGL((k_step2_apply<T, 2>), dim3(G), dim3(kBlock), 0, s, it, g, eps);
        } else {
            hipLaunchKernelGGL((k_step2_eval<T, 3>), dim3(G), dim3(kBlock), 0, s, it, g, h);
            hipLaunchKernelGGL((k_step2_apply<T, 3>), dim3(G), dim3(kBlock), 0, s, it, g, eps);
        }
    } else {
        if (g.nd == 2)
            hipLaunchKernelGGL((k_step2<T, 2>), dim3(G), dim3(kBlock), 0, s, it, g, h, eps);
        else
            hipLaunchKernelGGL((k_step2<T, 3>), dim3(G), dim3(kBlock), 0, s, it, g, h, eps);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_detect(const GridDims& g, const T* F, const T* phi, const uint8_t* lab, const Spacing<T>& h, T eps,
                         const SegList& out, hipStream_t s) {
    if (g.nd == 2)
        hipLaunchKernelGGL((k_detect<T, 2>), dim3(G), dim3(kBlock), 0, s, g, F, phi, lab, h, eps, out);
    else
        hipLaunchKernelGGL((k_detect<T, 3>), dim3(G), dim3(kBlock), 0, s, g, F, phi, lab, h, eps, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_remedy(const GridDims& g, const NodeIter<T>& it, const Spacing<T>& h, T eps, bool det, hipStream_t s) {
    if (det) {
        if (g.nd == 2) {
            hipLaunchKernelGGL((k_remedy_eval<T, 2>), dim3(G), dim3(kBlock), 0, s, it, g, h);
            hipLaunchKernelGGL((k_remedy_apply<T, 2>), dim3(G), dim3(kBlock), 0, s, it, g, eps);
        } else {
            hipLaunchKernelGGL((k_remedy_eval<T, 3>), dim3(G), dim3(kBlock), 0, s, it, g, h);
            hipLaunchKernelGGL((k_remedy_apply<T, 3>), dim3(G), dim3(kBlock), 0, s, it, g, eps);
        }
    } else {
        if (g.nd == 2)
            hipLaunchKernelGGL((k_remedy<T, 2>), dim3(G), dim3(kBlock), 0, s, it, g, h, eps);
        else
            hipLaunchKernelGGL((k_remedy<T, 3>), dim3(G), dim3(kBlock), 0, s, it, g, h, eps);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_local(const GridDims& g, const T* F, const T* phi, const Spacing<T>& h, T* out,
                              hipStream_t s) {
    if (g.nd == 2)
        hipLaunchKernelGGL((k_apply_local<T, 2>), dim3(dense_blocks(g.n)), dim3(kBlock), 0, s, g, F,
                           phi, h, out);
    else
        hipLaunchKernelGGL((k_apply_local<T, 3>), dim3(dense_blocks(g.n)), dim3(kBlock), 0, s, g, F,
                           phi, h, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fim(const GridDims& g, const NodeIter<T>& it, const Spacing<T>& h, T eps, hipStream_t s) {
    if (g.nd == 2) {
        hipLaunchKernelGGL((k_fim_update<T, 2>), dim3(G), dim3(kBlock), 0, s, it, g, h, eps);
        hipLaunchKernelGGL((k_fim_check<T, 2>), dim3(G), dim3(kBlock), 0, s, it, g, h, eps);
    } else {
        hipLaunchKernelGGL((k_fim_update<T, 3>), dim3(G), dim3(kBlock), 0, s, it, g, h, eps);
        hipLaunchKernelGGL((k_fim_check<T, 3>), dim3(G), dim3(kBlock), 0, s, it, g, h, eps);
    }
    return hipGetLastError();
}

hipError_t launch_reset_counters(Ctl* ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, ctl);
    return hipGetLastError();
}

hipError_t launch_ctl_init(Ctl* ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctl);
    return hipGetLastError();
}

hipError_t launch_sum_stats(unsigned long long* blkstat, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_stats, dim3(1), dim3(kBlock), 0, s, blkstat, nblocks);
    return hipGetLastError();
}

hipError_t launch_loop_status(Ctl* ctl, const int* counts, int nseg, hipStream_t s) {
    hipLaunchKernelGGL(k_loop_status, dim3(1), dim3(kBlock), 0, s, ctl, counts, nseg);
    return hipGetLastError();
}

#define EIK_INST(T)                                                                                \
    template hipError_t launch_init<T>(const T*, T*, uint8_t*, uint32_t*, int, Ctl*, hipStream_t); \
    template hipError_t launch_seed<T>(T*, uint8_t*, const SrcBatch<T>&, hipStream_t);             \
    template hipError_t launch_seed_active<T>(const GridDims&, const T*, uint8_t*,                 \
                                              const SrcBatch<T>&, const SegList&, int, hipStream_t); \
    template hipError_t launch_step2<T>(const GridDims&, const NodeIter<T>&, const Spacing<T>&, T,  \
                                        bool, hipStream_t);                                        \
    template hipError_t launch_detect<T>(const GridDims&, const T*, const T*, const uint8_t*,       \
                                         const Spacing<T>&, T, const SegList&, hipStream_t);       \
    template hipError_t launch_remedy<T>(const GridDims&, const NodeIter<T>&, const Spacing<T>&, T, \
                                         bool, hipStream_t);                                       \
    template hipError_t launch_apply_local<T>(const GridDims&, const T*, const T*, const Spacing<T>&, \
                                              T*, hipStream_t);                                    \
    template hipError_t launch_fim<T>(const GridDims&, const NodeIter<T>&, const Spacing<T>&, T, hipStream_t);

EIK_INST(float)
EIK_INST(double)

}  // namespace eik
