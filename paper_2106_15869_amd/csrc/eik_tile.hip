#include "eik_host.hpp"
#include "eik_tile.hpp"

namespace eik {

size_t tile_workspace_bytes(const GridDims& g, const eik_options& o) { return 256; }

template <typename T>
eik_status solve_tile(const GridDims& g, const T* F, double h, double eps,
                      const std::vector<std::pair<int, double>>& src, T* phi,
                      const eik_options& o, char* ws, hipStream_t s, eik_stats* st) {
    return fail(EIK_ERR_UNSUPPORTED, "tile variant not built yet");
}

template eik_status solve_tile<float>(const GridDims&, const float*, double, double,
                                      const std::vector<std::pair<int, double>>&, float*,
                                      const eik_options&, char*, hipStream_t, eik_stats*);
template eik_status solve_tile<double>(const GridDims&, const double*, double, double,
                                       const std::vector<std::pair<int, double>>&, double*,
                                       const eik_options&, char*, hipStream_t, eik_stats*);
}  // namespace eik
