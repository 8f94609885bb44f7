// Device-data checks of HMFSR_DEBUG=1: the library normally takes frames and
// motion as they are (non-finite or huge displacements are clamped to just
// past the frame, where no sample lies in it); in debug mode every call that
// reads motion first scans it and refuses non-finite vectors.
#include <stdio.h>
#include <stdlib.h>

#include "host.h"

namespace hmfsr {
namespace {

// Smallest flat index (frame, tile, component) of a non-finite motion value
// of a frame other than the base frame, into *first (initialised to INT_MAX).
__global__ void k_check_motion(const float* __restrict__ motion, int n, int ref, int per_frame, int* first) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * per_frame || i / per_frame == ref) return;
  if (!isfinite(motion[i])) atomicMin(first, i);
}

__global__ void k_set_i32(int* p, int v) { *p = v; }

}  // namespace

bool debug_enabled() {
  const char* e = getenv("HMFSR_DEBUG");
  return e && e[0] && !(e[0] == '0' && e[1] == 0);
}

hmfsr_status debug_check_motion(int dev, const float* motion, int n, int ref, int TY, int TX, hipStream_t s) {
  DeviceState& ds = g_dev[dev];
  void* ws = nullptr;
  hmfsr_status st = grow_buffer(ds.debug_ws, ds.debug_ws_bytes, 256, s, &ws);
  if (st != HMFSR_OK) return st;
  int* first = (int*)ws;
  const int per = TY * TX * 2;
  int host = 0x7fffffff;
  hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, first, 0x7fffffff);
  hipLaunchKernelGGL(k_check_motion, dim3((n * per + 255) / 256), dim3(256), 0, s, motion, n, ref, per, first);
  if (hipGetLastError() != hipSuccess || hipMemcpyAsync(&host, first, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return HMFSR_E_HIP;
  if (host == 0x7fffffff) return HMFSR_OK;
  const int f = host / per, t = (host % per) / 2;
  fprintf(stderr, "hmfsr (HMFSR_DEBUG): non-finite motion vector: frame %d, tile row %d, column %d (%s)\n", f,
          t / TX, t % TX, (host & 1) ? "vy" : "vx");
  return HMFSR_E_DATA;
}

}  // namespace hmfsr
