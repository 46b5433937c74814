// Local-moving decision and commit kernels (Alg. 2) for every degree bin,
// weight type and mode.
#include "scan_kernels.hpp"

namespace gvl {

void launch_decide_move(hipStream_t st, const GraphDesc& g, const ScanArgs& a, const int32_t* list,
                        const int32_t* count, const int32_t* start, bool det, int grid_cap, const HubArgs& h,
                        int32_t h0, int32_t h1, int64_t* launches) {
  if (g.w_double) {
    if (det) decide_bins<double, kMove, true>(st, g, a, list, count, start, grid_cap, h, h0, h1, launches);
    else decide_bins<double, kMove, false>(st, g, a, list, count, start, grid_cap, h, h0, h1, launches);
  } else {
    if (det) decide_bins<float, kMove, true>(st, g, a, list, count, start, grid_cap, h, h0, h1, launches);
    else decide_bins<float, kMove, false>(st, g, a, list, count, start, grid_cap, h, h0, h1, launches);
  }
}

void launch_commit(hipStream_t st, const GraphDesc& g, const ScanArgs& a, const HubArgs& h, const CommitLaunch& cl,
                   int phase) {
  if (phase == kMove) {
    if (g.w_double) commit_group_launch<double, kMove>(st, g, a, h, cl);
    else commit_group_launch<float, kMove>(st, g, a, h, cl);
  } else {
    if (g.w_double) commit_group_launch<double, kRefine>(st, g, a, h, cl);
    else commit_group_launch<float, kRefine>(st, g, a, h, cl);
  }
}

}  // namespace gvl
