// Local-moving decision and commit kernels (Alg. 2) for every degree bin,
// weight type and mode.
#include "scan_kernels.hpp"

namespace gvl {

void launch_decide_move(hipStream_t st, const GraphDesc& g, const ScanArgs& a, const int32_t* list,
                        const int32_t* count, const int32_t* start, bool det, int grid_cap, int hub_grid,
                        int64_t* launches) {
  if (g.w_double) {
    if (det) decide_bins<double, kMove, true>(st, g, a, list, count, start, grid_cap, hub_grid, launches);
    else decide_bins<double, kMove, false>(st, g, a, list, count, start, grid_cap, hub_grid, launches);
  } else {
    if (det) decide_bins<float, kMove, true>(st, g, a, list, count, start, grid_cap, hub_grid, launches);
    else decide_bins<float, kMove, false>(st, g, a, list, count, start, grid_cap, hub_grid, launches);
  }
}

void launch_commit_move(hipStream_t st, const GraphDesc& g, const ScanArgs& a, const int32_t* list,
                        int32_t count, int kind) {
  if (g.w_double) commit_list<double, kMove>(st, g, a, list, count, kind);
  else commit_list<float, kMove>(st, g, a, list, count, kind);
}

}  // namespace gvl
