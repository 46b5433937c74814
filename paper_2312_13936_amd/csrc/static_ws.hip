// gvl_leiden_static: gvl_leiden with its workspace in a device array that
// the library holds, for callers that cannot allocate device memory.
//
// The array `scratch` below is a file-scope __device__ variable: every GPU
// the library runs on holds its own copy (GVL_STATIC_WORKSPACE_BYTES) until
// the process ends.  In host code its name is only a host-side stand-in, so
// the device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress (from gvl_create, with that device current) and kept
// in g_scratch[device]; only that address is ever handed to kernels.  Every
// call on one GPU shares the array and finds the previous call's contents
// there; gvl_leiden clears everything it reads before reading it.  Calls
// that overlap on one GPU (two streams, two host threads) race on it.
#include <mutex>

#include "host.hpp"

namespace {

constexpr int kMaxDevices = 64;
static_assert(GVL_STATIC_WORKSPACE_BYTES % 256 == 0, "whole 256-byte units");

static __device__ __align__(256) unsigned char scratch[GVL_STATIC_WORKSPACE_BYTES];

std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

// Looks up the device address of `scratch` on `device` (which must be the
// current device) the first time the device is seen.
gvl_status gvl_static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return GVL_E_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return GVL_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    fprintf(stderr, "gvl: hipGetSymbolAddress(scratch) failed on device %d: %s\n", device, hipGetErrorString(e));
    return GVL_E_HIP;
  }
  g_scratch[device] = p;
  return GVL_OK;
}

extern "C" gvl_status gvl_leiden_static(gvl_ctx_t ctx, int64_t n, int64_t m, const int32_t* d_off,
                                        const int32_t* d_idx, const float* d_w, double resolution,
                                        const gvl_options* opt, int32_t* d_membership, double* modularity,
                                        gvl_stats* stats) {
  if (!ctx || !opt || n < 0 || m < 0) return GVL_E_INVALID_ARG;
  // per-kernel timing would create HIP events: not available here
  if (opt->profile) return GVL_E_INVALID_ARG;
  size_t need = 0;
  gvl_status s = gvl_workspace_bytes(n, m, opt, &need);
  if (s != GVL_OK) return s;
  if (need > (size_t)GVL_STATIC_WORKSPACE_BYTES) return GVL_E_WORKSPACE;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) ws = g_scratch[ctx->device];
  }
  if (!ws) return GVL_E_HIP;  // gvl_create did not resolve the array on this device
  return gvl_leiden(ctx, n, m, d_off, d_idx, d_w, resolution, opt, ws, (size_t)GVL_STATIC_WORKSPACE_BYTES,
                    d_membership, modularity, stats);
}
