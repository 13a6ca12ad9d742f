// Segmented work lists.
//
// A list is G segments, one per workgroup of the launch that produced it.
// Workgroup b appends into segment b only, reserving room with an LDS counter
// (one LDS atomic per wave after a wave prefix sum), and publishes the segment
// length at the end with a plain store.  No global atomic touches a shared
// counter, so appends never serialise across the chip.  A consumer launch of
// the same G workgroups prefix-sums the G lengths in LDS and hands workgroup b
// the contiguous slice [b*chunk, (b+1)*chunk) of the virtual concatenation.
#pragma once

#include "eik_device.hpp"
#include "eik_internal.hpp"

namespace eik {

// Block-wide: load G segment lengths, write the exclusive prefix to s_pref[0..G]
// and return the total.  s_pref must hold G + 1 ints.  All lanes must call.
template <int G>
__device__ __forceinline__ int seg_prefix(const int* __restrict__ count, int* s_pref) {
    static_assert(G % kBlock == 0, "G must be a multiple of the block size");
    constexpr int PER = G / kBlock;
    __shared__ int s_wave[kBlock / 64];
    int v[PER];
    int sum = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        v[j] = count[threadIdx.x * PER + j];
        sum += v[j];
    }
    int incl = wave_incl_scan(sum);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) s_wave[w] = incl;
    __syncthreads();
    int off = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) off += k < w ? s_wave[k] : 0;
    int run = off + incl - sum;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        s_pref[threadIdx.x * PER + j] = run;
        run += v[j];
    }
    if (threadIdx.x == kBlock - 1) s_pref[G] = run;
    __syncthreads();
    return s_pref[G];
}

// Entry k (0 <= k < total) of the virtual concatenation.
template <int G>
__device__ __forceinline__ int seg_entry(const SegList& L, const int* s_pref, int k) {
    int lo = 0, hi = G;  // find the last segment s with s_pref[s] <= k
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_pref[mid] <= k) lo = mid; else hi = mid;
    }
    return L.data[static_cast<size_t>(lo) * L.cap + (k - s_pref[lo])];
}

// Contiguous slice of the virtual list handled by this workgroup.
__device__ __forceinline__ void seg_slice(int total, int G, int& lo, int& hi) {
    const int chunk = (total + G - 1) / G;
    lo = min(total, static_cast<int>(blockIdx.x) * chunk);
    hi = min(total, lo + chunk);
}

// Per-workgroup appender into segment blockIdx.x of `out`.
struct SegAppender {
    int* s_cnt;  // LDS counter
    __device__ __forceinline__ void init() {
        if (threadIdx.x == 0) *s_cnt = 0;
    }
    // continue after what an earlier launch published into segment blockIdx.x
    __device__ __forceinline__ void resume(const SegList& out) {
        if (threadIdx.x == 0) *s_cnt = out.count[blockIdx.x];
    }
    // every lane of the wave must call; `mask` selects items[j]
    template <int MAXC>
    __device__ __forceinline__ void push_mask(const SegList& out, const int (&items)[MAXC], uint32_t mask) {
        const int c = __popc(mask);
        const int incl = wave_incl_scan(c);
        const int total = __shfl(incl, 63, 64);
        if (total == 0) return;
        int base = 0;
        if (lane_id() == 63) base = atomicAdd(s_cnt, total);
        base = __shfl(base, 63, 64);
        int* dst = out.data + static_cast<size_t>(blockIdx.x) * out.cap + base + incl - c;
#pragma unroll
        for (int j = 0; j < MAXC; ++j)
            if (mask & (1u << j)) dst[__popc(mask & ((1u << j) - 1u))] = items[j];
    }
    // single lane push (no wave-uniformity needed)
    __device__ __forceinline__ void push_one(const SegList& out, int item) {
        const int pos = atomicAdd(s_cnt, 1);
        out.data[static_cast<size_t>(blockIdx.x) * out.cap + pos] = item;
    }
    // after a __syncthreads that orders every push: publish the length
    __device__ __forceinline__ void publish(const SegList& out) {
        if (threadIdx.x == 0) out.count[blockIdx.x] = *s_cnt;
    }
};

}  // namespace eik
