// Modelled noise of a guide pixel (Sec. 5.2.2): the spatial variance
// sigma_md^2 that clamps sigma_ms from below and the squared difference of two
// 3x3 means d_md^2 that drives the Wiener shrinkage of eq. (6).
#pragma once

#include "hmfsr_internal.h"

namespace hmfsr {

// At base brightness mu (raw units), channel c (1 = the two-green mean), in
// raw units squared: the Monte-Carlo table interpolated linearly at the
// normalised brightness clamped to [0, 1] when the burst has one, else the
// closed forms var = a max(mu - black, 0) + b (halved for green), 2 var / 9.
__device__ __forceinline__ void noise_md(const RobustConsts& rc, float mu, int c, float& sig2, float& dmd2) {
  if (rc.ntab) {
    const float x = fminf(fmaxf((mu - rc.black) * rc.inv_range, 0.f), 1.f) * (float)(rc.nbins - 1);
    const int i = min((int)x, rc.nbins - 2);
    const float f = x - (float)i;
    const float* t = rc.ntab + 4 * i + (c == 1 ? 2 : 0);
    sig2 = fmaf(f, t[4] - t[0], t[0]) * rc.range2;
    dmd2 = fmaf(f, t[5] - t[1], t[1]) * rc.range2;
  } else {
    float var = fmaf(rc.a_r, fmaxf(mu - rc.black, 0.f), rc.b_r);
    if (c == 1) var *= 0.5f;
    sig2 = var;
    dmd2 = var * (2.f / 9.f);
  }
}

}  // namespace hmfsr
