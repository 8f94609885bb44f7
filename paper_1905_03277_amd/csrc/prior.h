// Motion prior of eq. (7)-(8): does tile (ty, tx) of frame n use the strong
// rejection s1 (local motion) rather than s2?
#pragma once

#include <math.h>

#include "hmfsr_internal.h"

namespace hmfsr {

// M_x (M_y) is the spread of the horizontal (vertical) displacements over the
// 3x3 tile neighbourhood, tiles outside the grid skipped; M > M_th is
// evaluated as M_x^2 + M_y^2 > M_th^2, rounded operation by operation.
// A non-finite component counts as the bound the merge and robustness kernels
// clamp it to (+-(max(W, H) + 16), NaN as the negative one); finite values are
// used as they are.
__device__ __forceinline__ bool prior_moving(const float* __restrict__ motion, const Geometry& g,
                                             double m_th, int n, int ty, int tx) {
  double xmax = -INFINITY, xmin = INFINITY, ymax = -INFINITY, ymin = INFINITY;
  for (int a = -1; a <= 1; ++a) {
    for (int b = -1; b <= 1; ++b) {
      const int y = ty + a, x = tx + b;
      if (y < 0 || y >= g.TY || x < 0 || x >= g.TX) continue;
      const float* v = motion + (((size_t)n * g.TY + y) * g.TX + x) * 2;
      const float vlim = (float)(max(g.W, g.H) + 16);
      const float fx = v[0], fy = v[1];
      const double vx = isfinite(fx) ? fx : fminf(fmaxf(fx, -vlim), vlim);
      const double vy = isfinite(fy) ? fy : fminf(fmaxf(fy, -vlim), vlim);
      xmax = fmax(xmax, vx);
      xmin = fmin(xmin, vx);
      ymax = fmax(ymax, vy);
      ymin = fmin(ymin, vy);
    }
  }
  const double mx = xmax - xmin, my = ymax - ymin;
  const double m2 = __dadd_rn(__dmul_rn(mx, mx), __dmul_rn(my, my));
  return m2 > __dmul_rn(m_th, m_th);
}

}  // namespace hmfsr
