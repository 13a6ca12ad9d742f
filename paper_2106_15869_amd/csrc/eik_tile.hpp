// Tile-activated variant: host entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>
#include <vector>

#include "../../include/eik.h"
#include "eik_internal.hpp"

namespace eik {

size_t tile_workspace_bytes(const GridDims& g, const eik_options& o);

template <typename T>
eik_status solve_tile(const GridDims& g, const T* F, double h, double eps,
                      const std::vector<std::pair<int, double>>& src, T* phi,
                      const eik_options& o, char* ws, hipStream_t s, eik_stats* st);

size_t adjoint_workspace_bytes(const GridDims& g, const eik_options& o);

template <typename T>
eik_status adjoint_solve(const GridDims& g, const T* F, const T* phi, double h,
                         const std::vector<std::pair<int, double>>& src, const T* dL_dphi, T* out,
                         const eik_options& o, char* ws, hipStream_t s, eik_stats* st);

}  // namespace eik
