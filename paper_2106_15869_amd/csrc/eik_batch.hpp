// Device-side tables of a batch (eik_tile.hpp): written by small kernels
// from kernel arguments, with no host-to-device copy, so that a solve stays
// capturable in a graph.
#pragma once

#include <algorithm>

#include "eik_device.hpp"
#include "eik_host.hpp"
#include "eik_tile.hpp"

namespace eik {

constexpr int kInstChunk = 32;
template <typename T>
struct InstChunk {
    int first, count;
    Inst<T> e[kInstChunk];
};

template <typename T>
__global__ void k_put_insts(InstChunk<T> c, Inst<T>* table) {
    if (static_cast<int>(threadIdx.x) < c.count) table[c.first + threadIdx.x] = c.e[threadIdx.x];
}

// tile_inst[t] = the instance whose tile range holds t (binary search on the
// tile bases, which increase with the instance index).
template <typename T>
__global__ void k_tile_owner(const Inst<T>* table, int ninst, int ntiles, int* tile_inst) {
    for (int t = blockIdx.x * kBlock + threadIdx.x; t < ntiles; t += gridDim.x * kBlock) {
        int lo = 0, hi = ninst;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (table[mid].tile_base <= t) lo = mid; else hi = mid;
        }
        tile_inst[t] = lo;
    }
}

template <typename T>
Inst<T> device_inst(const HostInst& h) {
    Inst<T> d;
    d.nx = h.nx;
    d.ny = h.ny;
    d.nz = h.nz;
    d.ntx = h.ntx;
    d.nty = h.nty;
    d.ntz = h.ntz;
    d.node_base = h.node_base;
    d.tile_base = h.tile_base;
    d.h = static_cast<T>(h.h);
    for (int k = 0; k < 3; ++k) d.d[k] = static_cast<T>(h.d[k]);
    d.aniso = h.aniso;
    return d;
}

// Batch geometry for the kernels; for several instances the table and the
// tile owners are written into the workspace by kernels enqueued on s.
template <typename T>
hipError_t upload_batch_geom(const Batch& b, void* table, int* tile_inst, hipStream_t s, BatchGeom<T>& g,
                             int64_t& launched) {
    g = BatchGeom<T>{};
    g.one = device_inst<T>(b.inst[0]);
    g.ninst = static_cast<int>(b.inst.size());
    g.ntiles = static_cast<int>(b.ntiles);
    if (g.ninst == 1) return hipSuccess;
    Inst<T>* tab = static_cast<Inst<T>*>(table);
    for (int f = 0; f < g.ninst; f += kInstChunk) {
        InstChunk<T> c{};
        c.first = f;
        c.count = std::min(kInstChunk, g.ninst - f);
        for (int j = 0; j < c.count; ++j) c.e[j] = device_inst<T>(b.inst[f + j]);
        hipLaunchKernelGGL(k_put_insts<T>, dim3(1), dim3(kInstChunk), 0, s, c, tab);
        ++launched;
    }
    hipLaunchKernelGGL(k_tile_owner<T>, dim3(std::min<int64_t>((b.ntiles + kBlock - 1) / kBlock, 4096)),
                       dim3(kBlock), 0, s, tab, g.ninst, g.ntiles, tile_inst);
    ++launched;
    g.table = tab;
    g.tile_inst = tile_inst;
    return hipGetLastError();
}

}  // namespace eik
