// Materialised merge pipeline: per-frame half-resolution maps written to a
// workspace, then one accumulation pass per output pixel.
//
// Stages (paper sections in brackets):
//   k_halfres     luma + guide of 2x2 quads, structure tensor (eq. 3), kernel
//                 covariance Omega (eq. 4, S.1), guide 3x3 mean / sigma  [5.1.2, 5.2.2]
//   k_prior       motion spread M per tile -> rejection strength s  [eq. 7-8]
//   k_robust      noise-corrected colour distance -> R  [eq. 5-6]
//   k_minpool     5x5 minimum of R  [eq. 9]
//   k_accumulate  nine nearest samples per frame, anisotropic Gaussian
//                 weights, per-channel normalisation  [eq. 1-2]
#include <math.h>

#include "hmfsr_internal.h"

namespace hmfsr {
namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ double raw_norm(const uint16_t* f, const Geometry& g, int r, int c) {
  return ((double)f[(size_t)r * g.W + c] - g.black) / g.range;
}

// Bilinear sample of an [h][w] map at continuous index (hx, hy), indices clamped.
template <typename T>
__device__ __forceinline__ double bilinear(const T* m, int h, int w, double hx, double hy) {
  double x0 = floor(hx), y0 = floor(hy);
  double fx = hx - x0, fy = hy - y0;
  int xi = (int)x0, yi = (int)y0;
  int xa = clampi(xi, 0, w - 1), xb = clampi(xi + 1, 0, w - 1);
  int ya = clampi(yi, 0, h - 1), yb = clampi(yi + 1, 0, h - 1);
  double top = (1.0 - fx) * (double)m[(size_t)ya * w + xa] + fx * (double)m[(size_t)ya * w + xb];
  double bot = (1.0 - fx) * (double)m[(size_t)yb * w + xa] + fx * (double)m[(size_t)yb * w + xb];
  return (1.0 - fy) * top + fy * bot;
}

// ---------------------------------------------------------------------------
// Half-resolution maps of one frame: Omega, guide mean and sigma.
__global__ void k_halfres(const uint16_t* __restrict__ frames, Geometry g, TuningD t,
                          double* __restrict__ omega, double* __restrict__ mu,
                          double* __restrict__ sd) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  const int I = blockIdx.y * blockDim.y + threadIdx.y;
  const int n = blockIdx.z;
  if (I >= g.h || J >= g.w) return;
  const uint16_t* f = frames + (size_t)n * g.H * g.W;

  double lum[3][3];
  double gd[3][3][3];  // [channel][a][b]
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) {
      const int qi = clampi(I + a - 1, 0, g.h - 1), qj = clampi(J + b - 1, 0, g.w - 1);
      double q[4];
      for (int k = 0; k < 4; ++k) q[k] = raw_norm(f, g, 2 * qi + (k >> 1), 2 * qj + (k & 1));
      lum[a][b] = (q[0] + q[1] + q[2] + q[3]) / 4.0;
      gd[0][a][b] = q[g.red_pos];
      gd[1][a][b] = (q[g.green_pos[0]] + q[g.green_pos[1]]) / 2.0;
      gd[2][a][b] = q[g.blue_pos];
    }
  }

  // eq. (3): mean of the outer products of the four cell gradients.
  double cxx[2][2], cxy[2][2], cyy[2][2];
  for (int a = 0; a < 2; ++a) {
    for (int b = 0; b < 2; ++b) {
      const double l00 = lum[a][b], l01 = lum[a][b + 1], l10 = lum[a + 1][b], l11 = lum[a + 1][b + 1];
      const double gx = ((l01 - l00) + (l11 - l10)) / 2.0;
      const double gy = ((l10 - l00) + (l11 - l01)) / 2.0;
      cxx[a][b] = gx * gx;
      cxy[a][b] = gx * gy;
      cyy[a][b] = gy * gy;
    }
  }
  const double txx = (cxx[0][0] + cxx[0][1] + cxx[1][0] + cxx[1][1]) / 4.0;
  const double txy = (cxy[0][0] + cxy[0][1] + cxy[1][0] + cxy[1][1]) / 4.0;
  const double tyy = (cyy[0][0] + cyy[0][1] + cyy[1][0] + cyy[1][1]) / 4.0;

  // Closed-form eigen-analysis; lambda1 - lambda2 = 2 rad without cancellation.
  const double half = (txx - tyy) * 0.5;
  const double rad = sqrt(half * half + txy * txy);
  const double tr = txx + tyy;
  const double lam1 = 0.5 * tr + rad;
  double ex, ey;  // unnormalised dominant eigenvector = gradient direction
  if (txy == 0.0 && txx == tyy) {
    ex = 1.0; ey = 0.0;
  } else if (half >= 0.0) {
    ex = half + rad; ey = txy;
  } else {
    ex = txy; ey = rad - half;
  }
  const double nrm2 = ex * ex + ey * ey;
  const double gx2 = ex * ex / nrm2, gy2 = ey * ey / nrm2, gxy = ex * ey / nrm2;

  // Supplement S.1 heuristics.
  const double A = tr > 0.0 ? 1.0 + sqrt(2.0 * rad / tr) : 1.0;
  double D = 1.0 - sqrt(lam1) / t.d_tr + t.d_th;
  D = D < 0.0 ? 0.0 : (D > 1.0 ? 1.0 : D);
  const double k1h = t.k_detail * (t.k_stretch * A);
  const double k2h = t.k_detail / (t.k_shrink * A);
  const double kdn = t.k_detail * t.k_denoise;
  const double k1s = (1.0 - D) * k1h + D * kdn;
  const double k2s = (1.0 - D) * k2h + D * kdn;
  const double k1 = k1s * k1s, k2 = k2s * k2s;
  // eq. (4): k1 along the edge (perpendicular to the gradient), k2 along it.
  const size_t plane = (size_t)g.h * g.w;
  const size_t o = (size_t)n * 3 * plane + (size_t)I * g.w + J;
  omega[o] = k1 * gy2 + k2 * gx2;
  omega[o + plane] = (k2 - k1) * gxy;
  omega[o + 2 * plane] = k1 * gx2 + k2 * gy2;

  // Guide 3x3 mean and population sigma (Sec. 5.2.2).
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) s += gd[c][a][b];
    const double m = s / 9.0;
    double v = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const double d = gd[c][a][b] - m;
        v += d * d;
      }
    mu[o + c * plane] = m;
    sd[o + c * plane] = sqrt(v / 9.0);
  }
}

// ---------------------------------------------------------------------------
// eq. (7)-(8): motion spread over the 3x3 tile neighbourhood -> s.
__global__ void k_prior(const float* __restrict__ motion, Geometry g, TuningD t,
                        float* __restrict__ s_tile) {
  const int tx = blockIdx.x * blockDim.x + threadIdx.x;
  const int ty = blockIdx.y * blockDim.y + threadIdx.y;
  const int n = blockIdx.z;
  if (ty >= g.TY || tx >= g.TX) return;
  const size_t idx = ((size_t)n * g.TY + ty) * g.TX + tx;
  if (n == g.ref) { s_tile[idx] = 0.0f; return; }
  double xmax = -INFINITY, xmin = INFINITY, ymax = -INFINITY, ymin = INFINITY;
  for (int a = -1; a <= 1; ++a) {
    for (int b = -1; b <= 1; ++b) {
      const int y = ty + a, x = tx + b;
      if (y < 0 || y >= g.TY || x < 0 || x >= g.TX) continue;
      const float* v = motion + (((size_t)n * g.TY + y) * g.TX + x) * 2;
      const double vx = v[0], vy = v[1];
      xmax = fmax(xmax, vx); xmin = fmin(xmin, vx);
      ymax = fmax(ymax, vy); ymin = fmin(ymin, vy);
    }
  }
  const double mx = xmax - xmin, my = ymax - ymin;
  // M > M_th as M^2 > M_th^2, rounded operation by operation (no contraction).
  const double m2 = __dadd_rn(__dmul_rn(mx, mx), __dmul_rn(my, my));
  s_tile[idx] = (float)(m2 > __dmul_rn(t.m_th, t.m_th) ? t.s1 : t.s2);
}

// ---------------------------------------------------------------------------
// eq. (5)-(6): robustness of frame n on the base frame's half-res grid.
__global__ void k_robust(const float* __restrict__ motion, Geometry g, TuningD t,
                         const double* __restrict__ mu, const double* __restrict__ sd,
                         const float* __restrict__ s_tile, float* __restrict__ robust) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  const int I = blockIdx.y * blockDim.y + threadIdx.y;
  const int n = blockIdx.z;
  if (I >= g.h || J >= g.w) return;
  const size_t plane = (size_t)g.h * g.w;
  float* out = robust + (size_t)n * plane + (size_t)I * g.w + J;
  if (n == g.ref) { *out = 1.0f; return; }
  const int ty = min((2 * I) / g.T, g.TY - 1), tx = min((2 * J) / g.T, g.TX - 1);
  const float* v = motion + (((size_t)n * g.TY + ty) * g.TX + tx) * 2;
  const double hx = (double)J + (double)v[0] / 2.0, hy = (double)I + (double)v[1] / 2.0;
  const size_t ro = (size_t)g.ref * 3 * plane + (size_t)I * g.w + J;
  double num = 0.0, den = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double m_ref = mu[ro + c * plane], s_ref = sd[ro + c * plane];
    const double m_al = bilinear(mu + ((size_t)n * 3 + c) * plane, g.h, g.w, hx, hy);
    double var = g.noise_a * fmax(m_ref, 0.0) + g.noise_b;
    if (c == 1) var = var / 2.0;
    const double sig = fmax(s_ref, sqrt(var));
    const double dms = m_ref - m_al;
    const double d = dms * (dms * dms) / (dms * dms + 2.0 * var / 9.0);
    num += d * d;
    den += sig * sig;
  }
  const double s = (double)s_tile[((size_t)n * g.TY + ty) * g.TX + tx];
  double R = s * exp(-(num / den)) - t.t;
  R = R < 0.0 ? 0.0 : (R > 1.0 ? 1.0 : R);
  *out = (float)R;
}

// eq. (9): 5x5 minimum over existing pixels.
__global__ void k_minpool(Geometry g, const float* __restrict__ robust, float* __restrict__ rmin) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  const int I = blockIdx.y * blockDim.y + threadIdx.y;
  const int n = blockIdx.z;
  if (I >= g.h || J >= g.w) return;
  const float* r = robust + (size_t)n * g.h * g.w;
  float m = 1.0f;
  for (int a = -2; a <= 2; ++a)
    for (int b = -2; b <= 2; ++b)
      m = fminf(m, r[(size_t)clampi(I + a, 0, g.h - 1) * g.w + clampi(J + b, 0, g.w - 1)]);
  rmin[(size_t)n * g.h * g.w + (size_t)I * g.w + J] = m;
}

// ---------------------------------------------------------------------------
// eq. (1)-(2): accumulate every frame's nine nearest samples per channel.
__global__ void k_accumulate(const uint16_t* __restrict__ frames, const float* __restrict__ motion,
                             Geometry g, const double* __restrict__ omega,
                             const float* __restrict__ rmin, float* __restrict__ out) {
  const int C = blockIdx.x * blockDim.x + threadIdx.x;
  const int Rr = blockIdx.y * blockDim.y + threadIdx.y;
  if (Rr >= g.OH || C >= g.OW) return;
  const double X = ((double)C + 0.5) / g.scale;
  const double Y = ((double)Rr + 0.5) / g.scale;
  const int ty = min((int)floor(Y) / g.T, g.TY - 1), tx = min((int)floor(X) / g.T, g.TX - 1);
  const size_t plane = (size_t)g.h * g.w;

  double M[3] = {-INFINITY, -INFINITY, -INFINITY};
  float num[3] = {0.f, 0.f, 0.f}, den[3] = {0.f, 0.f, 0.f};
  for (int n = 0; n < g.n; ++n) {
    double vx = 0.0, vy = 0.0;
    double rho = 1.0;
    if (n != g.ref) {
      const float* v = motion + (((size_t)n * g.TY + ty) * g.TX + tx) * 2;
      vx = v[0]; vy = v[1];
      rho = bilinear(rmin + (size_t)n * plane, g.h, g.w, X / 2.0 - 0.5, Y / 2.0 - 0.5);
      if (!(rho > 0.0)) continue;
    }
    const double px = X + vx, py = Y + vy;
    const int jc = (int)floor(px), ic = (int)floor(py);
    const double hx = px / 2.0 - 0.5, hy = py / 2.0 - 0.5;
    const double* om = omega + (size_t)n * 3 * plane;
    const double oxx = bilinear(om, g.h, g.w, hx, hy);
    const double oxy = bilinear(om + plane, g.h, g.w, hx, hy);
    const double oyy = bilinear(om + 2 * plane, g.h, g.w, hx, hy);
    const double det = oxx * oyy - oxy * oxy;
    const double ia = oyy / det, ib = -oxy / det, ic2 = oxx / det;

    double e[9];
    float val[9];
    int ch[9];
    double Mf[3] = {-INFINITY, -INFINITY, -INFINITY};
    const uint16_t* f = frames + (size_t)n * g.H * g.W;
    for (int k = 0; k < 9; ++k) {
      const int qi = ic + k / 3 - 1, qj = jc + k % 3 - 1;
      if (qi < 0 || qi >= g.H || qj < 0 || qj >= g.W) { ch[k] = -1; continue; }
      const double dx = ((double)qj + 0.5) - px, dy = ((double)qi + 0.5) - py;
      e[k] = -0.5 * (ia * dx * dx + 2.0 * ib * dx * dy + ic2 * dy * dy);
      ch[k] = g.colour[(qi & 1) * 2 + (qj & 1)];
      val[k] = (float)(((double)f[(size_t)qi * g.W + qj] - g.black) / g.range);
      Mf[ch[k]] = fmax(Mf[ch[k]], e[k]);
    }
    for (int c = 0; c < 3; ++c) {
      if (Mf[c] > M[c]) {
        if (M[c] > -INFINITY) {
          const float sc = expf((float)(M[c] - Mf[c]));
          num[c] *= sc;
          den[c] *= sc;
        }
        M[c] = Mf[c];
      }
    }
    for (int k = 0; k < 9; ++k) {
      if (ch[k] < 0) continue;
      const float wgt = (float)rho * expf((float)(e[k] - M[ch[k]]));
      num[ch[k]] += wgt * val[k];
      den[ch[k]] += wgt;
    }
  }
  const size_t oplane = (size_t)g.OH * g.OW;
  const size_t o = (size_t)Rr * g.OW + C;
  for (int c = 0; c < 3; ++c) out[o + c * oplane] = num[c] / den[c];
}

}  // namespace

size_t maps_bytes(const Geometry& g) {
  const size_t plane = (size_t)g.h * g.w;
  const size_t tiles = (size_t)g.TY * g.TX;
  return 9 * plane * g.n * sizeof(double) + 2 * plane * g.n * sizeof(float) +
         tiles * g.n * sizeof(float) + 6 * 256;
}

Maps maps_carve(void* base, const Geometry& g) {
  const size_t plane = (size_t)g.h * g.w;
  const size_t tiles = (size_t)g.TY * g.TX;
  char* p = (char*)base;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) & ~(size_t)255;
    return r;
  };
  Maps m;
  m.omega = (double*)take(3 * plane * g.n * sizeof(double));
  m.mu = (double*)take(3 * plane * g.n * sizeof(double));
  m.sd = (double*)take(3 * plane * g.n * sizeof(double));
  m.s_tile = (float*)take(tiles * g.n * sizeof(float));
  m.robust = (float*)take(plane * g.n * sizeof(float));
  m.rmin = (float*)take(plane * g.n * sizeof(float));
  return m;
}

hipError_t launch_maps(const Geometry& g, const TuningD& t, const uint16_t* frames,
                       const float* motion, const Maps& m, hipStream_t stream) {
  const dim3 blk(16, 16);
  const dim3 grid_h((g.w + 15) / 16, (g.h + 15) / 16, g.n);
  const dim3 grid_t((g.TX + 15) / 16, (g.TY + 15) / 16, g.n);
  hipLaunchKernelGGL(k_halfres, grid_h, blk, 0, stream, frames, g, t, m.omega, m.mu, m.sd);
  hipLaunchKernelGGL(k_prior, grid_t, blk, 0, stream, motion, g, t, m.s_tile);
  hipLaunchKernelGGL(k_robust, grid_h, blk, 0, stream, motion, g, t, m.mu, m.sd, m.s_tile, m.robust);
  hipLaunchKernelGGL(k_minpool, grid_h, blk, 0, stream, g, m.robust, m.rmin);
  return hipGetLastError();
}

hipError_t launch_accumulate(const Geometry& g, const uint16_t* frames, const float* motion,
                             const Maps& m, float* out, hipStream_t stream) {
  const dim3 blk(16, 16);
  const dim3 grid((g.OW + 15) / 16, (g.OH + 15) / 16);
  hipLaunchKernelGGL(k_accumulate, grid, blk, 0, stream, frames, motion, g, m.omega, m.rmin, out);
  return hipGetLastError();
}

}  // namespace hmfsr
