// pifu_occupancy_grid_async_noalloc: the device-driven occupancy grid for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops, harnesses
// that forbid hipMalloc).  Its workspace is one fixed array in the library's own device
// memory instead of a caller buffer.
//
// The array is a file-scope __device__ object.  In host code its name is a host-side
// stand-in, not a device address, so host code never passes it anywhere: at set-up
// (pifu_create, once per device, with that device current) hipGetSymbolAddress gives the
// device address of this device's copy, which is kept per device and is the only handle
// host code uses.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pifu_internal.h"

static constexpr size_t kScratchBytes = (size_t)PIFU_NOALLOC_SCRATCH_MIB << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of each device's copy (null: not set up)

}  // namespace

namespace pifu {

int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return PIFU_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return PIFU_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PIFU_ERR_HIP;
  g_scratch[device] = p;
  return PIFU_OK;
}

}  // namespace pifu

extern "C" {

size_t pifu_noalloc_scratch_bytes(void) { return kScratchBytes; }

int32_t pifu_occupancy_grid_async_noalloc(pifu_ctx* ctx, const pifu_field* field,
                                          const pifu_grid_opts* opts, uint32_t max_points,
                                          float* occ, uint8_t* labels, uint8_t* eval_level,
                                          uint32_t* cells, uint32_t cells_cap,
                                          uint32_t* n_cells_dev, pifu_level_stats* stats_dev,
                                          uint32_t* status_dev, pifu_stream stream) {
  if (!ctx) return PIFU_ERR_INVALID_ARGUMENT;
  const int dev = pifu::ctx_device(ctx);
  if (dev < 0 || dev >= kMaxDevices) return PIFU_ERR_UNSUPPORTED;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    ws = g_scratch[dev];
  }
  if (!ws) return PIFU_ERR_HIP;   // set-up in pifu_create did not find the array
  size_t need = 0;
  int r = pifu_occupancy_grid_async_workspace_size(field, opts, max_points, &need);
  if (r) return r;
  if (need > kScratchBytes) return PIFU_ERR_SCRATCH_TOO_SMALL;
  // the async call clears every counter it reads with kernels and overwrites every
  // buffer before reading it, so the previous call's contents do not matter
  return pifu_occupancy_grid_async(ctx, field, opts, max_points, occ, labels, eval_level, cells,
                                   cells_cap, n_cells_dev, stats_dev, status_dev, ws,
                                   kScratchBytes, stream);
}

}  // extern "C"
