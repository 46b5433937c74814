// Measurement aid: the random-gather rate of this device over a given index
// array (the neighbour-community scan reads one label per arc, C'[j], at
// the arc's neighbour id j).  Not part of Leiden; bench.py uses it to put
// the scan kernels' label-gather rate beside what the memory system
// delivers for the same address stream.
#include "device.hpp"
#include "host.hpp"

namespace gvl {

constexpr int kProbeUnroll = 4;

__global__ __launch_bounds__(kBlock) void k_gather_probe(const int32_t* __restrict__ idx, int64_t n_idx,
                                                         const int32_t* __restrict__ table, int64_t n_table,
                                                         unsigned long long* __restrict__ sink) {
  unsigned long long s = 0;
  const int64_t T = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_idx; b += T * kProbeUnroll) {
    int32_t j[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
      const int64_t e = b + u * T;
      if (e >= n_idx) {  // past the array: adds nothing
        j[u] = -1;
        continue;
      }
      const int32_t x = idx[e];
      j[u] = ((uint64_t)(uint32_t)x < (uint64_t)n_table) ? x : 0;  // an index outside the table reads entry 0
    }
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) s += (j[u] >= 0) ? (uint32_t)table[j[u]] : 0u;
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane_id() == 0 && s) atomicAdd(sink, s);
}

}  // namespace gvl

using namespace gvl;

gvl_status gvl_gather_probe(gvl_ctx_t ctx, const int32_t* d_idx, int64_t n_idx, const int32_t* d_table,
                            int64_t n_table, unsigned long long* d_sink) {
  if (!ctx || n_idx < 0 || n_table < 1 || !d_table || !d_sink || (n_idx > 0 && !d_idx)) return GVL_E_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return GVL_E_HIP;
  if (n_idx == 0) return GVL_OK;
  const int64_t blocks = std::min<int64_t>(4096, (n_idx + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_gather_probe, dim3((unsigned)blocks), dim3(kBlock), 0, ctx->stream, d_idx, n_idx, d_table,
                     n_table, d_sink);
  return hipGetLastError() == hipSuccess ? GVL_OK : GVL_E_HIP;
}
