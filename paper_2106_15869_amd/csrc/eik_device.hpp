// Device-side building blocks of the gfx950 eikonal kernels: grid geometry,
// the exact Godunov local solve, node labels and wave64 list compaction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eik_internal.hpp"

namespace eik {

// Node labels (one byte per node).  FAR: never reached; ACTIVE: in the update
// list; CONV: converged in the update step (joins the Source set); FIXED: a
// given boundary value (Algorithm 2, STEP 1).
enum : uint32_t { L_FAR = 0u, L_ACTIVE = 1u, L_CONV = 2u, L_FIXED = 3u };

constexpr int kBlock = 256;  // threads per workgroup (4 wave64)

template <typename T> __device__ __forceinline__ T pos_inf();
template <> __device__ __forceinline__ float pos_inf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double pos_inf<double>() { return __builtin_huge_val(); }

__device__ __forceinline__ float dev_sqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double dev_sqrt(double x) { return __builtin_sqrt(x); }

template <typename T> __device__ __forceinline__ T tmin(T a, T b) { return b < a ? b : a; }

// Grid extents; 2D grids use nz = 1.  Node count < 2^31.
struct Grid {
    int nx, ny, nz;
    int n;
    int sxy;  // nx * ny
};

template <int ND>
__device__ __forceinline__ void decode(const Grid& g, int i, int& x, int& y, int& z) {
    x = i % g.nx;
    if (ND == 2) {
        y = i / g.nx;
        z = 0;
    } else {
        int t = i / g.nx;
        y = t % g.ny;
        z = t / g.ny;
    }
}

// Exact solution of sum_k ((phi - a_k)^+)^2 = H^2 over the ND per-axis minima
// (Eq 4 in 2D, Eq 6 in 3D; the quantity Algorithms 1.1 and 1.3 compute).
// Written relative to the smallest minimum (b_k = a_k - a_1) so that large
// arrival times do not cancel; an axis joins while the running root still
// exceeds its minimum.  Returns +inf when nothing upwind is finite or H = +inf.
// Branch-free: the minima are sorted with a min/max network, the one-, two-
// and three-sided roots are all formed and the progressive rule selects one
// (the same value, bit for bit, as evaluating them in turn; a root formed
// from an infinite minimum is never selected).
template <typename T, int ND>
__device__ __forceinline__ T godunov(T a0, T a1, T a2, T H) {
    const T inf = pos_inf<T>();
    const T lo = fmin(a0, a1), hi = fmax(a0, a1);
    if (ND == 3) {
        const T m = fmin(hi, a2);
        a2 = fmax(hi, a2);
        a0 = fmin(lo, m);
        a1 = fmax(lo, m);
    } else {
        a0 = lo;
        a1 = hi;
    }
    const T phi1 = a0 + H;
    T b = a1 - a0;
    T S = b;
    T Q = b * b;
    const T HH = H * H;
    T disc = S * S - T(2) * (Q - HH);
    disc = disc < T(0) ? T(0) : disc;
    const T phi2 = a0 + (S + dev_sqrt(disc)) / T(2);
    T phi = phi1 > a1 ? phi2 : phi1;
    if (ND == 3) {
        b = a2 - a0;
        S = S + b;
        Q = Q + b * b;
        disc = S * S - T(3) * (Q - HH);
        disc = disc < T(0) ? T(0) : disc;
        const T phi3 = a0 + (S + dev_sqrt(disc)) / T(3);
        phi = phi1 > a1 && phi2 > a2 ? phi3 : phi;
    }
    return H < inf && a0 < inf ? phi : inf;
}

// H_i = h / F_i, +inf for a barrier cell.
template <typename T> __device__ __forceinline__ T cell_H(T h, T f) {
    return f > T(0) ? h / f : pos_inf<T>();
}

// Per-axis spacing (Eq 5 with dx != dy, the case of Algorithm 1.2, and its 3D
// analogue): the root of sum_k ((phi - a_k)^+ / H_k)^2 = 1 with
// H_k = spacing_k / F.  Same progressive rule on the minima sorted ascending
// (a stable sort; each H_k travels with its a_k), in shifted form: with
// t = phi - a_1, b_k = a_k - a_1 and w_k = 1 / H_k^2 the active axes give
// A t^2 - 2 B t + C = 0, A = sum w_k, B = sum w_k b_k, C = sum w_k b_k^2 - 1.
template <typename T, int ND>
__device__ __forceinline__ T godunov_aniso(T a0, T a1, T a2, T H0, T H1, T H2) {
    const T inf = pos_inf<T>();
    if (a1 < a0) {
        T t = a0; a0 = a1; a1 = t;
        t = H0; H0 = H1; H1 = t;
    }
    if (ND == 3 && a2 < a1) {
        T t = a1; a1 = a2; a2 = t;
        t = H1; H1 = H2; H2 = t;
        if (a1 < a0) {
            t = a0; a0 = a1; a1 = t;
            t = H0; H0 = H1; H1 = t;
        }
    }
    if (!(a0 < inf) || !(H0 < inf)) return inf;
    T phi = a0 + H0;
    if (!(phi > a1)) return phi;
    T A = T(1) / (H0 * H0);
    T b = a1 - a0;
    T w = T(1) / (H1 * H1);
    A = A + w;
    T B = w * b;
    T C = T(-1) + w * b * b;
    T disc = B * B - A * C;
    disc = disc < T(0) ? T(0) : disc;
    phi = a0 + (B + dev_sqrt(disc)) / A;
    if (ND == 3) {
        if (!(phi > a2)) return phi;
        b = a2 - a0;
        w = T(1) / (H2 * H2);
        A = A + w;
        B = B + w * b;
        C = C + w * b * b;
        disc = B * B - A * C;
        disc = disc < T(0) ? T(0) : disc;
        phi = a0 + (B + dev_sqrt(disc)) / A;
    }
    return phi;
}

// G_i from the per-axis minima (dims order) and the node's speed.
template <typename T, int ND>
__device__ __forceinline__ T local_solve(T a0, T a1, T a2, T f, const Spacing<T>& sp) {
    if (!sp.aniso) return godunov<T, ND>(a0, a1, a2, cell_H(sp.h, f));
    if (!(f > T(0))) return pos_inf<T>();
    return godunov_aniso<T, ND>(a0, a1, a2, sp.d[0] / f, sp.d[1] / f, ND == 3 ? sp.d[2] / f : pos_inf<T>());
}

// G_i(phi) from global memory.
template <typename T, int ND>
__device__ __forceinline__ T eval_node(const T* phi, const T* F, const Grid& g, int i, int x, int y,
                                       int z, const Spacing<T>& sp) {
    const T inf = pos_inf<T>();
    T ax = inf, ay = inf, az = inf;
    if (x > 0) ax = phi[i - 1];
    if (x + 1 < g.nx) ax = tmin(ax, phi[i + 1]);
    if (y > 0) ay = phi[i - g.nx];
    if (y + 1 < g.ny) ay = tmin(ay, phi[i + g.nx]);
    if (ND == 3) {
        if (z > 0) az = phi[i - g.sxy];
        if (z + 1 < g.nz) az = tmin(az, phi[i + g.sxy]);
    }
    if (ND == 2) return local_solve<T, 2>(ay, ax, inf, F[i], sp);
    return local_solve<T, 3>(az, ay, ax, F[i], sp);
}

// ---------------------------------------------------------------------------
// Byte labels packed four to a 32-bit word; transitions use word atomics so
// that concurrent updates of neighbouring bytes never overwrite each other.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t label_get(const uint8_t* lab, int i) { return lab[i]; }

__device__ __forceinline__ bool label_cas(uint8_t* lab, int i, uint32_t expect, uint32_t desired) {
    uint32_t* w = reinterpret_cast<uint32_t*>(lab + (i & ~3));
    const int sh = (i & 3) * 8;
    uint32_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (((old >> sh) & 0xffu) != expect) return false;
        uint32_t nw = (old & ~(0xffu << sh)) | (desired << sh);
        uint32_t prev = atomicCAS(w, old, nw);
        if (prev == old) return true;
        old = prev;
    }
}

// Add a signed delta to one byte label (caller guarantees no carry/borrow).
__device__ __forceinline__ void label_add(uint8_t* lab, int i, int delta) {
    uint32_t* w = reinterpret_cast<uint32_t*>(lab + (i & ~3));
    const int sh = (i & 3) * 8;
    atomicAdd(w, static_cast<uint32_t>(delta) << sh);
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Add v to this workgroup's column of a per-workgroup statistics array
// (call from one lane only).
__device__ __forceinline__ void blk_add(unsigned long long* blkstat, int field, int nblocks,
                                        unsigned long long v) {
    if (v) blkstat[field * nblocks + blockIdx.x] += v;
}

}  // namespace eik
