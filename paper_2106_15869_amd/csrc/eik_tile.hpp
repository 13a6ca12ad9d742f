// Tile-activated variant and adjoint: host entry points and the batch
// description they share.  A single grid is a batch of one instance.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>
#include <vector>

#include "../../include/eik.h"
#include "eik_internal.hpp"

namespace eik {

struct TileCfg {
    int tx, ty, tz;
};

// Host copy of one instance (see Inst<T>).
struct HostInst {
    int nx, ny, nz;
    int ntx, nty, ntz;
    int node_base, tile_base;
    double h;
    double d[3];  // per-axis spacing in dims order when aniso
    int aniso;
};

// Instances laid out back to back in F / phi: instance k's nodes start where
// instance k - 1's end, and likewise its tiles.
struct Batch {
    int nd = 0;
    TileCfg cfg{};
    std::vector<HostInst> inst;
    int64_t n = 0;        // nodes over all instances
    int64_t ntiles = 0;
    std::vector<std::pair<int, double>> src;  // batch-wide flat index, value (deduplicated)
    std::vector<int> src_inst;                // instance of each source
};

TileCfg pick_tile(int nd, const eik_options& o);

// Append an instance of extents (nz, ny, nx) (nz = 1 in 2D) and spacing h
// (or per-axis spacing `d` in dims order when not NULL), tiled with b.cfg.
void batch_add(Batch& b, int nx, int ny, int nz, double h, const double* d);

// The same instances and sources tiled with c.
Batch with_tiles(const Batch& b, const TileCfg& c);

size_t tile_workspace_bytes(const Batch& b, size_t esz);

template <typename T>
eik_status solve_tile(const Batch& b, const T* F, double eps, T* phi, const eik_options& o, char* ws,
                      hipStream_t s, eik_stats* st);

size_t adjoint_workspace_bytes(const Batch& b, size_t esz);

template <typename T>
eik_status adjoint_solve(const Batch& b, const T* F, const T* phi, const T* dL_dphi, T* out,
                         const eik_options& o, char* ws, hipStream_t s, eik_stats* st);

}  // namespace eik
