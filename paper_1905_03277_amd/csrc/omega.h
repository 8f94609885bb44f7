// Kernel covariance Omega of one half-resolution pixel (Sec. 5.1.2, eq. 3-4,
// supplement S.1), evaluated from raw 2x2-quad sums so that the structure
// tensor is exact.
//
// With L the sum of the four raw values of a quad, the luma of the quad is
// (L - 4 black) / (4 range). The cell gradient of eq. (3) (horizontal and
// vertical differences averaged over the 2x2 luma cell) is then
// g = gi / (8 range) with gi an integer built from L differences (black
// cancels), and the tensor (mean of the four cell outer products) is
// T = Ti / (256 range^2) with Ti a sum of integer products, exact in float64.
// The eigen-analysis is scale-invariant except for sqrt(lambda1), which enters
// D; that factor is folded into `inv_16_range_dtr`.
#pragma once

#include <hip/hip_runtime.h>

namespace hmfsr {

struct OmegaConsts {
  double kd_st;             // k_detail * k_stretch
  double kd_sh;             // k_detail / k_shrink
  double kd_dn;             // k_detail * k_denoise
  double d_th;
  double inv_16_range_dtr;  // 1 / (16 * range * d_tr)
};

// The hardware reciprocal and reciprocal square root are good to ~5e-8
// relative; one Newton step takes them to ~4e-15, two to the last bit or two.

// 1 / d to ~2e-15 relative (one Newton step), for values that feed only
// continuous arithmetic.
__device__ __forceinline__ double recip64_1(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return fma(r, fma(-d, r, 1.0), r);
}

// 1 / sqrt(x) for x > 0 to ~4e-15 relative (one Newton step).
__device__ __forceinline__ double rsqrt64_1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * fma(-0.5 * x, y * y, 1.5);
}

// 1 / sqrt(x) for x > 0 to ~2 ulp: the hardware reciprocal square root
// refined by two Newton steps.
__device__ __forceinline__ double rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x, y * y, 1.5);
  return y * fma(-0.5 * x, y * y, 1.5);
}

// sqrt(x) for x >= 0 to ~1e-15 relative (the correctly rounded library
// square root costs twice as many instructions, and nothing here needs the
// last bit).
__device__ __forceinline__ double sqrt64(double x) { return x > 0.0 ? x * rsqrt64(x) : 0.0; }

// sqrt(x) for x >= 0 to ~4e-15 relative (one Newton step).
__device__ __forceinline__ double sqrt64_1(double x) { return x > 0.0 ? x * rsqrt64_1(x) : 0.0; }

// What the adjoint needs of one pixel's kernel covariance besides Omega.
struct OmegaParts {
  double c2, s2;         // cos 2phi, sin 2phi of the gradient direction phi
  double A, invA, D;     // anisotropy, its inverse, denoising weight (S.1), D clamped
  double k1s, k2s;       // square roots of the edge / gradient variances
  double sqrt_l1;        // sqrt(lambda1) of the integer tensor
  bool d_free;           // D strictly inside (0, 1), i.e. not clamped
};

// l[a][b]: quad sums of the 3x3 half-res window around the pixel (edge-clamped),
// as int or as float holding integers (differences stay exact below 2^24).
template <bool PARTS, typename Q>
__device__ __forceinline__ void omega_core(const Q (&l)[3][3], const OmegaConsts& c, double& oxx,
                                           double& oxy, double& oyy, OmegaParts* parts) {
  double txx = 0.0, txy = 0.0, tyy = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const Q gxi = (l[a][b + 1] - l[a][b]) + (l[a + 1][b + 1] - l[a + 1][b]);
      const Q gyi = (l[a + 1][b] - l[a][b]) + (l[a + 1][b + 1] - l[a][b + 1]);
      const double gx = (double)gxi, gy = (double)gyi;
      txx += gx * gx;
      txy += gx * gy;
      tyy += gy * gy;
    }
  }
  // Closed-form eigen-analysis: lambda1,2 = tr/2 +- rad; lambda1 - lambda2 =
  // 2 rad. With phi the angle of the dominant eigenvector (the gradient
  // direction), cos 2phi = half / rad and sin 2phi = txy / rad, so its
  // products are (1 +- cos 2phi) / 2 and sin 2phi / 2. An isotropic tensor
  // (rad = 0, a tie of integers) takes the x axis.
  const double half = 0.5 * (txx - tyy);
  const double r2 = half * half + txy * txy;
  const double tr = txx + tyy;
  double rad = 0.0, c2 = 1.0, s2 = 0.0, A = 1.0;
  if (r2 > 0.0) {
    const double y = rsqrt64_1(r2);  // 1 / rad
    rad = r2 * y;
    c2 = half * y;
    s2 = txy * y;
    // A = 1 + sqrt((lambda1 - lambda2) / (lambda1 + lambda2)) = 1 + 1 / sqrt(tr / (2 rad)),
    // with tr >= 2 rad > 0
    A = 1.0 + rsqrt64_1(0.5 * tr * y);
  }
  const double invA = recip64_1(A);
  const double sqrt_l1 = sqrt64_1(0.5 * tr + rad);
  const double D_raw = 1.0 - sqrt_l1 * c.inv_16_range_dtr + c.d_th;
  const double D = D_raw < 0.0 ? 0.0 : (D_raw > 1.0 ? 1.0 : D_raw);
  const double k1s = (1.0 - D) * (c.kd_st * A) + D * c.kd_dn;
  const double k2s = (1.0 - D) * (c.kd_sh * invA) + D * c.kd_dn;
  const double k1 = k1s * k1s, k2 = k2s * k2s;
  // eq. (4): variance k1 along the edge (perpendicular to the gradient), k2
  // across it. With the gradient products (1 + c2) / 2, (1 - c2) / 2 and
  // s2 / 2: Omega = (k1 + k2) / 2 I + (k1 - k2) / 2 [[-c2, -s2], [-s2, c2]].
  const double hs = 0.5 * (k1 + k2), hd = 0.5 * (k1 - k2);
  oxx = fma(-c2, hd, hs);
  oxy = -(s2 * hd);
  oyy = fma(c2, hd, hs);
  if (PARTS) {
    parts->c2 = c2;
    parts->s2 = s2;
    parts->A = A;
    parts->invA = invA;
    parts->D = D;
    parts->k1s = k1s;
    parts->k2s = k2s;
    parts->sqrt_l1 = sqrt_l1;
    parts->d_free = D_raw > 0.0 && D_raw < 1.0;
  }
}

template <typename Q>
__device__ __forceinline__ void omega_from_quads(const Q (&l)[3][3], const OmegaConsts& c,
                                                 double& oxx, double& oxy, double& oyy) {
  omega_core<false>(l, c, oxx, oxy, oyy, nullptr);
}

template <typename Q>
__device__ __forceinline__ void omega_parts_from_quads(const Q (&l)[3][3], const OmegaConsts& c,
                                                       double& oxx, double& oxy, double& oyy,
                                                       OmegaParts& parts) {
  omega_core<true>(l, c, oxx, oxy, oyy, &parts);
}

}  // namespace hmfsr
