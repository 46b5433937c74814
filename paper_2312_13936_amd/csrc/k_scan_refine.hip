// Refinement decision and commit kernels (Alg. 3) for every degree bin,
// weight type and mode.
#include "scan_kernels.hpp"

namespace gvl {

void launch_decide_refine(hipStream_t st, const GraphDesc& g, const ScanArgs& a, const int32_t* list,
                          const int32_t* count, const int32_t* start, bool det, int grid_cap, const HubArgs& h,
                          int32_t h0, int32_t h1, int64_t* launches) {
  if (g.w_double) {
    if (det) decide_bins<double, kRefine, true>(st, g, a, list, count, start, grid_cap, h, h0, h1, launches);
    else decide_bins<double, kRefine, false>(st, g, a, list, count, start, grid_cap, h, h0, h1, launches);
  } else {
    if (det) decide_bins<float, kRefine, true>(st, g, a, list, count, start, grid_cap, h, h0, h1, launches);
    else decide_bins<float, kRefine, false>(st, g, a, list, count, start, grid_cap, h, h0, h1, launches);
  }
}

}  // namespace gvl
