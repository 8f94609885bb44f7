// Persistent batched merge: workgroups of one launch per tile shape and raw
// load batch size pull (burst, tile) items of many bursts from an XCD-chunked
// queue; the tile body is merge_tile.h.
#include "merge_tile.h"

namespace hmfsr {
namespace {

// Persistent form: workgroups pull (burst, tile) items from the XCD-chunked
// queue (for_each_item) until it is exhausted. One launch per tile shape and
// raw-load batch size (RB), so that every burst runs the code its own launch
// would.
template <int MH, int THREADS, int RB>
__global__ __launch_bounds__(THREADS, (waves_per_simd<MH, THREADS>())) void k_merge_batch(
    const BurstArgs* __restrict__ bursts, const WorkItem* __restrict__ items, ItemQueue q) {
  __shared__ MergeSmem<MH> sm;
  for_each_item(q, &sm.sItem, [&](int it) {
    const WorkItem w = items[it];
    const BurstArgs* b = bursts + w.burst;
    const Geometry g = b->g;
    const MergeConsts mc = b->mc;
    const int tx = w.tile % b->merge_tiles_x, ty = w.tile / b->merge_tiles_x;
    merge_tile<MH, THREADS, TILE_PLAIN, RB>(b->frames, b->motion, b->rmin, g, mc, b->out, nullptr,
                                         StreamState{nullptr, nullptr, 0}, tx, ty, sm);
  });
}

template <int MH, int THREADS>
hipError_t launch_batch_variant(bool wide, const BurstArgs* bursts, const WorkItem* items, const ItemQueue& q,
                                int n_groups, hipStream_t stream) {
  if (wide)
    hipLaunchKernelGGL((k_merge_batch<MH, THREADS, 8>), dim3(n_groups), dim3(THREADS), 0, stream, bursts,
                       items, q);
  else
    hipLaunchKernelGGL((k_merge_batch<MH, THREADS, 4>), dim3(n_groups), dim3(THREADS), 0, stream, bursts,
                       items, q);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_merge_batch(int cls, const BurstArgs* bursts, const WorkItem* items, const int* bounds,
                              int* counters, int n_groups, hipStream_t stream) {
  const bool wide = cls & 1;
  const ItemQueue q{bounds, counters};
  switch (cls >> 1) {
    case 1: return launch_batch_variant<32, 512>(wide, bursts, items, q, n_groups, stream);
    case 2: return launch_batch_variant<16, 256>(wide, bursts, items, q, n_groups, stream);
    case 3: return launch_batch_variant<16, 128>(wide, bursts, items, q, n_groups, stream);
    default: return launch_batch_variant<32, 256>(wide, bursts, items, q, n_groups, stream);
  }
}

namespace {
template <int MH, int THREADS>
int blocks_per_cu(bool wide) {
  int b = 0;
  const hipError_t e = wide ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_merge_batch<MH, THREADS, 8>, THREADS, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_merge_batch<MH, THREADS, 4>, THREADS, 0);
  if (e != hipSuccess) return 1;
  return b > 0 ? b : 1;
}
}  // namespace

int merge_batch_blocks_per_cu(int cls) {
  const bool wide = cls & 1;
  switch (cls >> 1) {
    case 1: return blocks_per_cu<32, 512>(wide);
    case 2: return blocks_per_cu<16, 256>(wide);
    case 3: return blocks_per_cu<16, 128>(wide);
    default: return blocks_per_cu<32, 256>(wide);
  }
}

}  // namespace hmfsr
