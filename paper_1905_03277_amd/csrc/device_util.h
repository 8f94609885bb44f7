// Small device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace hmfsr {

__host__ __device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// a * b for |a|, |b| < 2^23 (window offsets and widths, LDS indices): the
// full-rate 24-bit multiply instead of the quarter-rate 32-bit one.
__device__ __forceinline__ int mul24(int a, int b) { return __mul24(a, b); }

// Minimum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

// Row of flat index k in a row-major window of width w, given inv = 1/w
// rounded to float. (k + 1/2) / w lies at least 1/(2w) from an integer while
// the float product errs by under (k / w) * 2^-22, so the floor is exact for
// every k < 2^16.
__device__ __forceinline__ int split_row(int k, float inv) { return (int)(((float)k + 0.5f) * inv); }

// Workgroups of a launch are dispatched round-robin over the XCDs, each with
// its own L2. Tile of linear workgroup id b among n: XCD x = b % XCDS takes a
// contiguous run of tiles (row-major), so neighbouring tiles, which share
// footprint halos, meet in the same L2. A bijection on [0, n).
constexpr int XCDS = 8;
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int q = n / XCDS, r = n - q * XCDS;
  const int x = b % XCDS, l = b / XCDS;
  return x * q + min(x, r) + l;
}

// Persistent work distribution over the XCDs. A launch's items [0, n) are
// split into XCDS contiguous chunks of about equal cost (chunk x = [bounds[x],
// bounds[x + 1])), each with its own counter (zero at launch). A workgroup on
// XCD x (dispatch is round-robin) takes the items of chunk x in turn, then
// what is left of the other chunks, x + 1 first, so that neighbouring items
// (tiles of one burst) meet in one L2 and no XCD idles while another has work.
// `slot` is a workgroup-shared int; `body(item)` runs on the whole workgroup.
struct ItemQueue {
  const int* bounds;  // [XCDS + 1]
  int* counters;      // [XCDS]
};

template <typename F>
__device__ __forceinline__ void for_each_item(const ItemQueue& q, int* slot, F&& body) {
  const int home = blockIdx.x % XCDS;
  for (int k = 0; k < XCDS; ++k) {
    const int c = (home + k) % XCDS;
    const int lo = q.bounds[c], hi = q.bounds[c + 1];
    if (lo >= hi) continue;  // uniform
    while (true) {
      __syncthreads();
      if (threadIdx.x == 0) *slot = lo + atomicAdd(&q.counters[c], 1);
      __syncthreads();
      const int it = __builtin_amdgcn_readfirstlane(*slot);  // uniform: scalar loads follow
      if (it >= hi) break;
      body(it);
    }
  }
}

}  // namespace hmfsr
