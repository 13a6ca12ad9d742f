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
// Lists are int32 node indices compacted per wave (prefix sum over lanes, one
// atomic per wave).  Labels are bytes changed with word atomics.
#include "eik_device.hpp"
#include "eik_internal.hpp"

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

// Append the set bits of `mask` (slots into items[]) to list, one atomic per wave.
template <int MAXC>
__device__ __forceinline__ void wave_append_mask(int* list, int* cnt, const int (&items)[MAXC],
                                                 uint32_t mask) {
    const int c = __popc(mask);
    int incl = wave_incl_scan(c);
    int total = __shfl(incl, 63, 64);
    if (total == 0) return;
    int base = 0;
    if (lane_id() == 63) base = atomicAdd(cnt, total);
    base = __shfl(base, 63, 64);
    int pos = base + incl - c;
#pragma unroll
    for (int j = 0; j < MAXC; ++j) {
        if (mask & (1u << j)) list[pos + __popc(mask & ((1u << j) - 1u))] = items[j];
    }
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

template <typename T, int ND>
__global__ void k_seed_active(GridDims gd, const T* __restrict__ F, uint8_t* lab, SrcBatch<T> b,
                              int* list, int* cnt) {
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
    wave_append_mask<6>(list, cnt, items, mask);
}

// ---------------------------------------------------------------------------
// STEP 2
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int iter_prologue(const NodeIter<T>& a, unsigned long long* iters,
                                             unsigned long long* evals, bool track_max) {
    const int n = *a.cnt_cur;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.cnt_zero = 0;
        if (n > 0) {
            *iters += 1;
            *evals += static_cast<unsigned long long>(n);
            if (track_max && static_cast<unsigned long long>(n) > a.ctl->max_active)
                a.ctl->max_active = static_cast<unsigned long long>(n);
        }
    }
    return n;
}

// Shared by the in-place and the synchronous-read apply kernels.
template <typename T, int ND>
__device__ __forceinline__ uint32_t step2_apply_node(const NodeIter<T>& a, const Grid& g, int i,
                                                     T pi, T pt, T eps, int (&items)[7]) {
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
        if (pt < pi) a.phi[i] = pt;
        items[6] = i;
        mask = 1u << 6;
    }
    return mask;
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_step2(NodeIter<T> a, GridDims gd, T h, T eps) {
    const Grid g = make_grid(gd);
    const int n = iter_prologue(a, &a.ctl->iters2, &a.ctl->evals2, true);
    for (int base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        const int k = base + threadIdx.x;
        int items[7];
        uint32_t mask = 0;
        if (k < n) {
            const int i = a.list_cur[k];
            int x, y, z;
            decode<ND>(g, i, x, y, z);
            const T pi = a.phi[i];
            const T pt = eval_node<T, ND>(a.phi, a.F, g, i, x, y, z, h);
            mask = step2_apply_node<T, ND>(a, g, i, pi, pt, eps, items);
        }
        wave_append_mask<7>(a.list_next, a.cnt_next, items, mask);
    }
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_step2_eval(NodeIter<T> a, GridDims gd, T h) {
    const Grid g = make_grid(gd);
    const int n = iter_prologue(a, &a.ctl->iters2, &a.ctl->evals2, true);
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < n; k += gridDim.x * kBlock) {
        const int i = a.list_cur[k];
        int x, y, z;
        decode<ND>(g, i, x, y, z);
        a.vals[k] = eval_node<T, ND>(a.phi, a.F, g, i, x, y, z, h);
    }
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_step2_apply(NodeIter<T> a, GridDims gd, T eps) {
    const Grid g = make_grid(gd);
    const int n = *a.cnt_cur;
    for (int base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        const int k = base + threadIdx.x;
        int items[7];
        uint32_t mask = 0;
        if (k < n) {
            const int i = a.list_cur[k];
            mask = step2_apply_node<T, ND>(a, g, i, a.phi[i], a.vals[k], eps, items);
        }
        wave_append_mask<7>(a.list_next, a.cnt_next, items, mask);
    }
}

// ---------------------------------------------------------------------------
// STEP 3
// ---------------------------------------------------------------------------
template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_detect(GridDims gd, const T* __restrict__ F,
                                                   const T* __restrict__ phi,
                                                   const uint8_t* __restrict__ lab, T h, T eps,
                                                   int* list, int* cnt) {
    const Grid g = make_grid(gd);
    for (int base = blockIdx.x * kBlock; base < g.n; base += gridDim.x * kBlock) {
        const int i = base + threadIdx.x;
        bool flag = false;
        if (i < g.n && lab[i] != L_FIXED) {
            int x, y, z;
            decode<ND>(g, i, x, y, z);
            const T pt = eval_node<T, ND>(phi, F, g, i, x, y, z, h);
            flag = pt < phi[i] - eps;
        }
        wave_append1(list, cnt, i, flag);
    }
}

// claim node q for the next remedy list (first claimer this iteration wins)
__device__ __forceinline__ bool claim(uint32_t* stamp, int q, uint32_t tag) {
    if (__hip_atomic_load(stamp + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= tag) return false;
    return atomicMax(stamp + q, tag) < tag;
}

template <typename T, int ND>
__device__ __forceinline__ uint32_t remedy_apply_node(const NodeIter<T>& a, const Grid& g, int i,
                                                      T pi, T pt, T eps, uint32_t tag,
                                                      int (&items)[7]) {
    uint32_t mask = 0;
    if (pt < pi - eps) {
        a.phi[i] = pt;
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

template <typename T>
__device__ __forceinline__ int remedy_prologue(const NodeIter<T>& a, uint32_t& tag) {
    const int n = *a.cnt_cur;
    tag = static_cast<uint32_t>(a.ctl->tag[a.tag_slot]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.cnt_zero = 0;
        a.ctl->tag[a.tag_slot ^ 1] = static_cast<int>(tag + 1);
        if (a.first) a.ctl->remedy_init = static_cast<unsigned long long>(n);
        if (n > 0) {
            a.ctl->iters3 += 1;
            a.ctl->evals_rem += static_cast<unsigned long long>(n);
        }
    }
    return n;
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_remedy(NodeIter<T> a, GridDims gd, T h, T eps) {
    const Grid g = make_grid(gd);
    uint32_t tag;
    const int n = remedy_prologue(a, tag);
    for (int base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        const int k = base + threadIdx.x;
        int items[7];
        uint32_t mask = 0;
        if (k < n) {
            const int i = a.list_cur[k];
            int x, y, z;
            decode<ND>(g, i, x, y, z);
            const T pt = eval_node<T, ND>(a.phi, a.F, g, i, x, y, z, h);
            mask = remedy_apply_node<T, ND>(a, g, i, a.phi[i], pt, eps, tag, items);
        }
        wave_append_mask<7>(a.list_next, a.cnt_next, items, mask);
    }
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_remedy_eval(NodeIter<T> a, GridDims gd, T h) {
    const Grid g = make_grid(gd);
    uint32_t tag;
    const int n = remedy_prologue(a, tag);
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < n; k += gridDim.x * kBlock) {
        const int i = a.list_cur[k];
        int x, y, z;
        decode<ND>(g, i, x, y, z);
        a.vals[k] = eval_node<T, ND>(a.phi, a.F, g, i, x, y, z, h);
    }
}

// The apply kernel of the synchronous mode reads the tag its eval kernel used
// (the eval kernel already advanced the other slot).
template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_remedy_apply(NodeIter<T> a, GridDims gd, T eps) {
    const Grid g = make_grid(gd);
    const int n = *a.cnt_cur;
    const uint32_t tag = static_cast<uint32_t>(a.ctl->tag[a.tag_slot]);
    for (int base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        const int k = base + threadIdx.x;
        int items[7];
        uint32_t mask = 0;
        if (k < n) {
            const int i = a.list_cur[k];
            mask = remedy_apply_node<T, ND>(a, g, i, a.phi[i], a.vals[k], eps, tag, items);
        }
        wave_append_mask<7>(a.list_next, a.cnt_next, items, mask);
    }
}

template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_apply_local(GridDims gd, const T* __restrict__ F,
                                                        const T* __restrict__ phi, T h,
                                                        T* __restrict__ out) {
    const Grid g = make_grid(gd);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < g.n; i += gridDim.x * kBlock) {
        int x, y, z;
        decode<ND>(g, i, x, y, z);
        out[i] = eval_node<T, ND>(phi, F, g, i, x, y, z, h);
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
        ctl->tag[0] = 1;
        ctl->tag[1] = 1;
        ctl->iters2 = ctl->iters3 = ctl->evals2 = ctl->evals_det = ctl->evals_rem = 0;
        ctl->remedy_init = ctl->max_active = 0;
    }
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
                              int* list, int* cnt, hipStream_t s) {
    if (g.nd == 2)
        hipLaunchKernelGGL((k_seed_active<T, 2>), dim3(1), dim3(kMaxSrcBatch), 0, s, g, F, lab, b,
                           list, cnt);
    else
        hipLaunchKernelGGL((k_seed_active<T, 3>), dim3(1), dim3(kMaxSrcBatch), 0, s, g, F, lab, b,
                           list, cnt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step2(const GridDims& g, const NodeIter<T>& it, T h, T eps, bool det,
                        int blocks, hipStream_t s) {
    if (det) {
        if (g.nd == 2) {
            hipLaunchKernelGGL((k_step2_eval<T, 2>), dim3(blocks), dim3(kBlock), 0, s, it, g, h);
            hipLaunchKernelGGL((k_step2_apply<T, 2>), dim3(blocks), dim3(kBlock), 0, s, it, g, eps);
        } else {
            hipLaunchKernelGGL((k_step2_eval<T, 3>), dim3(blocks), dim3(kBlock), 0, s, it, g, h);
            hipLaunchKernelGGL((k_step2_apply<T, 3>), dim3(blocks), dim3(kBlock), 0, s, it, g, eps);
        }
    } else {
        if (g.nd == 2)
            hipLaunchKernelGGL((k_step2<T, 2>), dim3(blocks), dim3(kBlock), 0, s, it, g, h, eps);
        else
            hipLaunchKernelGGL((k_step2<T, 3>), dim3(blocks), dim3(kBlock), 0, s, it, g, h, eps);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_detect(const GridDims& g, const T* F, const T* phi, const uint8_t* lab, T h, T eps,
                         int* list, int* cnt, hipStream_t s) {
    if (g.nd == 2)
        hipLaunchKernelGGL((k_detect<T, 2>), dim3(dense_blocks(g.n)), dim3(kBlock), 0, s, g, F, phi,
                           lab, h, eps, list, cnt);
    else
        hipLaunchKernelGGL((k_detect<T, 3>), dim3(dense_blocks(g.n)), dim3(kBlock), 0, s, g, F, phi,
                           lab, h, eps, list, cnt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_remedy(const GridDims& g, const NodeIter<T>& it, T h, T eps, bool det,
                         int blocks, hipStream_t s) {
    if (det) {
        if (g.nd == 2) {
            hipLaunchKernelGGL((k_remedy_eval<T, 2>), dim3(blocks), dim3(kBlock), 0, s, it, g, h);
            hipLaunchKernelGGL((k_remedy_apply<T, 2>), dim3(blocks), dim3(kBlock), 0, s, it, g, eps);
        } else {
            hipLaunchKernelGGL((k_remedy_eval<T, 3>), dim3(blocks), dim3(kBlock), 0, s, it, g, h);
            hipLaunchKernelGGL((k_remedy_apply<T, 3>), dim3(blocks), dim3(kBlock), 0, s, it, g, eps);
        }
    } else {
        if (g.nd == 2)
            hipLaunchKernelGGL((k_remedy<T, 2>), dim3(blocks), dim3(kBlock), 0, s, it, g, h, eps);
        else
            hipLaunchKernelGGL((k_remedy<T, 3>), dim3(blocks), dim3(kBlock), 0, s, it, g, h, eps);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_local(const GridDims& g, const T* F, const T* phi, T h, T* out,
                              hipStream_t s) {
    if (g.nd == 2)
        hipLaunchKernelGGL((k_apply_local<T, 2>), dim3(dense_blocks(g.n)), dim3(kBlock), 0, s, g, F,
                           phi, h, out);
    else
        hipLaunchKernelGGL((k_apply_local<T, 3>), dim3(dense_blocks(g.n)), dim3(kBlock), 0, s, g, F,
                           phi, h, out);
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

#define EIK_INST(T)                                                                                \
    template hipError_t launch_init<T>(const T*, T*, uint8_t*, uint32_t*, int, Ctl*, hipStream_t); \
    template hipError_t launch_seed<T>(T*, uint8_t*, const SrcBatch<T>&, hipStream_t);             \
    template hipError_t launch_seed_active<T>(const GridDims&, const T*, uint8_t*,                 \
                                              const SrcBatch<T>&, int*, int*, hipStream_t);        \
    template hipError_t launch_step2<T>(const GridDims&, const NodeIter<T>&, T, T, bool, int,      \
                                        hipStream_t);                                              \
    template hipError_t launch_detect<T>(const GridDims&, const T*, const T*, const uint8_t*, T, T, \
                                         int*, int*, hipStream_t);                                 \
    template hipError_t launch_remedy<T>(const GridDims&, const NodeIter<T>&, T, T, bool, int,     \
                                         hipStream_t);                                             \
    template hipError_t launch_apply_local<T>(const GridDims&, const T*, const T*, T, T*,          \
                                              hipStream_t);

EIK_INST(float)
EIK_INST(double)

}  // namespace eik
