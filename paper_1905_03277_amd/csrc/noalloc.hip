// hmfsr_merge_noalloc: the merge with its per-frame maps in a static device
// array instead of the library's allocated workspace, for callers that cannot
// allocate device memory.
#include <stdint.h>

#include "host.h"

namespace hmfsr {
namespace {

constexpr size_t kScratchBytes = HMFSR_NOALLOC_SCRATCH_BYTES;

// One copy per device, held by the code object until the process ends. In
// host code this name is only a handle for hipGetSymbolAddress: the kernels
// get the device address resolved below, never the name.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* g_scratch[kMaxDevices];  // the array's address on each device (null until resolved)

// Device address of this device's scratch, resolved once per device with that
// device current (the caller holds g_mutex and made `dev` current).
hmfsr_status scratch_of(int dev, void** out) {
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return HMFSR_E_HIP;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return HMFSR_OK;
}

}  // namespace
}  // namespace hmfsr

using namespace hmfsr;

extern "C" hmfsr_status hmfsr_merge_noalloc(const hmfsr_desc* desc, const hmfsr_tuning* tuning,
                                            const uint16_t* frames, const float* motion, float* out,
                                            float* saved, void* stream) {
  hmfsr_status st = validate(desc, tuning);
  if (st != HMFSR_OK) return st;
  if (!frames || !motion || !out) return HMFSR_E_INVALID;
  if (((uintptr_t)frames & 3) || ((uintptr_t)motion & 3) || ((uintptr_t)out & 3) || ((uintptr_t)saved & 7))
    return HMFSR_E_INVALID;
  const Geometry g = make_geometry(desc);
  if (work_bytes(g) > kScratchBytes) return HMFSR_E_TOO_LARGE;
  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  if ((st = current_device(&dev)) != HMFSR_OK) return st;
  void* ws = nullptr;
  if ((st = scratch_of(dev, &ws)) != HMFSR_OK) return st;
  // every map the kernels read is written first in the same call: no clearing
  return run_merge(desc, tuning, g, frames, motion, out, saved, work_carve(ws, g), merge_variant(g),
                   (hipStream_t)stream, /*profiled=*/false);
}
