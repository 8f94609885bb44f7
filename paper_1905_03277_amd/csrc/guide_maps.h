// Guide maps of the robustness (Sec. 5.2.2, eq. 6): per half-res pixel of
// every frame, the sums over its 3x3 neighbourhood (edge-replicated) of the
// guide's red value, of its two greens and of its blue value, as exact
// integers packed into 8 bytes:
//   x: R sum (below 2^20: nine 16-bit values) in bits 0-19, the low 12 bits
//      of the B sum in bits 20-31;
//   y: green sum (below 2^21: eighteen 16-bit values) in bits 0-20, the high
//      8 bits of the B sum in bits 21-28.
// The 3x3 box mean of a channel is its sum times 1/9 (the green guide is the
// mean of two greens, so its sum is halved first), rounded as a product of
// its own (never fused into a following operation), so that every reader
// sees the same float. Every partial sum is an exact float below 2^24, so
// this is the float that summing the guide's float values over the window
// and scaling by 1/9 gives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hmfsr {

__device__ __forceinline__ uint2 pack_guide_sums(uint32_t r, uint32_t g2, uint32_t b) {
  return make_uint2(r | (b << 20), g2 | ((b >> 12) << 21));
}

// The three 3x3 box means (raw units) of one packed entry.
__device__ __forceinline__ void guide_means(uint2 p, float (&m)[3]) {
  const uint32_t r = p.x & 0xfffffu;
  const uint32_t g2 = p.y & 0x1fffffu;
  const uint32_t b = (p.x >> 20) | ((p.y >> 21) << 12);
  m[0] = __fmul_rn((float)r, 1.f / 9.f);
  m[1] = __fmul_rn((float)g2 * 0.5f, 1.f / 9.f);
  m[2] = __fmul_rn((float)b, 1.f / 9.f);
}

}  // namespace hmfsr
