// Robustness of every aligned frame on the base frame's half-resolution grid
// (Sec. 5.2): noise-corrected colour distance (eq. 5-6), motion-prior strength
// (eq. 7-8, precomputed per tile) and the 5x5 minimum (eq. 9).
//
// One workgroup owns a 32x16 tile of the base half-res grid and loops over the
// frames. The base frame's 3x3 guide mean and the noise-corrected sigma are
// computed once into LDS; for each aligned frame the guide around the warped
// footprint is staged into LDS, box-filtered, sampled bilinearly at u + v/2
// for every robustness pixel of the tile plus a 2-pixel border, and the 5x5
// minimum of the result is written to global memory.
//
// All colour statistics are kept in raw units (black level subtracted only
// where the noise model needs brightness): the ratio d^2 / sigma^2 of eq. (5)
// is scale-free.
#include "hmfsr_internal.h"

namespace hmfsr {
namespace {

constexpr int RB_W = 32, RB_H = 16;              // output tile of R_hat (half-res px)
constexpr int RR_W = RB_W + 4, RR_H = RB_H + 4;  // robustness region incl. the min-pool border
constexpr int RR_N = RR_W * RR_H;
constexpr int MU_CAP = 1000;                     // frame-n box-mean region
constexpr int GU_CAP = 1150;                     // frame-n guide region
constexpr int THREADS = 256;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

// Guide pixel (I, J) of a frame in raw units: R, mean of the greens, B.
__device__ __forceinline__ void load_guide(const uint16_t* f, const Geometry& g, int I, int J,
                                           float& r, float& gr, float& b) {
  const uint32_t top = *(const uint32_t*)(f + (size_t)(2 * I) * g.W + 2 * J);
  const uint32_t bot = *(const uint32_t*)(f + (size_t)(2 * I + 1) * g.W + 2 * J);
  const int q[4] = {(int)(top & 0xffff), (int)(top >> 16), (int)(bot & 0xffff), (int)(bot >> 16)};
  r = (float)q[g.red_pos];
  gr = (float)(q[g.green_pos[0]] + q[g.green_pos[1]]) * 0.5f;
  b = (float)q[g.blue_pos];
}

// Continuous half-res index u + v/2 of base pixel (I, J) in the aligned frame.
// Clamping to [-1, w] x [-1, h] leaves the edge-clamped bilinear sample
// unchanged and keeps non-finite vectors inside the staged buffers.
__device__ __forceinline__ void warped_pos(const float* mv, const Geometry& g, int I, int J, int ty,
                                           int tx, double& hx, double& hy) {
  const float* v = mv + ((size_t)ty * g.TX + tx) * 2;
  hx = fmin(fmax((double)J + (double)v[0] * 0.5, -1.0), (double)g.w);
  hy = fmin(fmax((double)I + (double)v[1] * 0.5, -1.0), (double)g.h);
}

__global__ __launch_bounds__(THREADS) void k_robust(const uint16_t* __restrict__ frames,
                                                    const float* __restrict__ motion,
                                                    const float* __restrict__ s_tile, Geometry g,
                                                    RobustConsts rc, float* __restrict__ rmin,
                                                    float* __restrict__ robust) {
  __shared__ float sMuRef[3][RR_N];
  __shared__ float sInvDen[RR_N];
  __shared__ float sGuide[3][GU_CAP];
  __shared__ float sMu[3][MU_CAP];
  __shared__ float sR[RR_N];
  __shared__ float sTmp[RR_H * RB_W];
  __shared__ int sRed[4];

  const int tid = threadIdx.x;
  const int I0 = blockIdx.y * RB_H, J0 = blockIdx.x * RB_W;
  // robustness region (clamped to the grid): rows [ra0, ra1), cols [ca0, ca1)
  const int ra0 = max(I0 - 2, 0), ra1 = min(I0 + RB_H + 2, g.h);
  const int ca0 = max(J0 - 2, 0), ca1 = min(J0 + RB_W + 2, g.w);
  const int rw = ca1 - ca0, rh = ra1 - ra0, rn = rw * rh;
  const size_t plane = (size_t)g.h * g.w;

  // ---- base frame statistics, once ------------------------------------
  {
    const uint16_t* f = frames + (size_t)g.ref * g.H * g.W;
    const int gr0 = max(ra0 - 1, 0), gr1 = min(ra1, g.h - 1);
    const int gc0 = max(ca0 - 1, 0), gc1 = min(ca1, g.w - 1);
    const int gw = gc1 - gc0 + 1, gn = gw * (gr1 - gr0 + 1);
    for (int k = tid; k < gn; k += THREADS) {
      float r, gg, b;
      load_guide(f, g, gr0 + k / gw, gc0 + k % gw, r, gg, b);
      sGuide[0][k] = r;
      sGuide[1][k] = gg;
      sGuide[2][k] = b;
    }
    __syncthreads();
    for (int k = tid; k < rn; k += THREADS) {
      const int I = ra0 + k / rw, J = ca0 + k % rw;
      float den = 0.f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float v[9];
        float s = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            const int ii = clampi(I + a - 1, 0, g.h - 1) - gr0, jj = clampi(J + b - 1, 0, g.w - 1) - gc0;
            v[a * 3 + b] = sGuide[c][ii * gw + jj];
            s += v[a * 3 + b];
          }
        const float mu = s / 9.f;
        float var_ms = 0.f;
#pragma unroll
        for (int q = 0; q < 9; ++q) var_ms += (v[q] - mu) * (v[q] - mu);
        var_ms /= 9.f;
        // noise model in raw units at the base brightness; the guide green is
        // the mean of two greens, so its variance is halved.
        float var_md = rc.a_r * fmaxf(mu - rc.black, 0.f) + rc.b_r;
        if (c == 1) var_md *= 0.5f;
        sMuRef[c][k] = mu;
        den += fmaxf(var_ms, var_md);  // sigma = max(sigma_ms, sigma_md), eq. (6)
      }
      sInvDen[k] = 1.f / den;
    }
  }

  // ---- aligned frames -------------------------------------------------
  const int tyA = min(2 * ra0 / g.T, g.TY - 1), tyB = min(2 * (ra1 - 1) / g.T, g.TY - 1);
  const int txA = min(2 * ca0 / g.T, g.TX - 1), txB = min(2 * (ca1 - 1) / g.T, g.TX - 1);
  for (int n = 0; n < g.n; ++n) {
    if (n == g.ref) continue;
    const uint16_t* f = frames + (size_t)n * g.H * g.W;
    const float* mv = motion + (size_t)n * g.TY * g.TX * 2;
    const float* st = s_tile + (size_t)n * g.TY * g.TX;
    // Segments: the whole region when its warped footprint fits the LDS
    // buffers, otherwise one alignment tile at a time.
    int seg = -1;
    const int nseg_tiles = (tyB - tyA + 1) * (txB - txA + 1);
    bool whole = true;
    while (true) {
      const int sty = whole ? -1 : tyA + seg / (txB - txA + 1);
      const int stx = whole ? -1 : txA + seg % (txB - txA + 1);
      // bounds of the bilinear corners over the segment's pixels
      __syncthreads();
      if (tid < 4) sRed[tid] = 0x7fffffff;
      __syncthreads();
      int b0 = 0x7fffffff, b1 = 0x7fffffff, b2 = 0x7fffffff, b3 = 0x7fffffff;
      for (int k = tid; k < rn; k += THREADS) {
        const int I = ra0 + k / rw, J = ca0 + k % rw;
        const int ty = min(2 * I / g.T, g.TY - 1), tx = min(2 * J / g.T, g.TX - 1);
        if (!whole && (ty != sty || tx != stx)) continue;
        double hx, hy;
        warped_pos(mv, g, I, J, ty, tx, hx, hy);
        const int x0 = (int)floor(hx), y0 = (int)floor(hy);
        b0 = min(b0, x0); b1 = min(b1, -x0); b2 = min(b2, y0); b3 = min(b3, -y0);
      }
      b0 = wave_min(b0); b1 = wave_min(b1); b2 = wave_min(b2); b3 = wave_min(b3);
      if ((tid & 63) == 0) {
        atomicMin(&sRed[0], b0); atomicMin(&sRed[1], b1);
        atomicMin(&sRed[2], b2); atomicMin(&sRed[3], b3);
      }
      __syncthreads();
      const int xmin = sRed[0], xmax = -sRed[1], ymin = sRed[2], ymax = -sRed[3];
      bool empty = xmin > xmax;
      // box-mean region (bilinear corners) and guide region (box border), clamped
      const int mc0 = clampi(xmin, 0, g.w - 1), mc1 = clampi(xmax + 1, 0, g.w - 1);
      const int mr0 = clampi(ymin, 0, g.h - 1), mr1 = clampi(ymax + 1, 0, g.h - 1);
      const int gc0 = max(mc0 - 1, 0), gc1 = min(mc1 + 1, g.w - 1);
      const int gr0 = max(mr0 - 1, 0), gr1 = min(mr1 + 1, g.h - 1);
      const int mw = mc1 - mc0 + 1, mn = mw * (mr1 - mr0 + 1);
      const int gw = gc1 - gc0 + 1, gn = gw * (gr1 - gr0 + 1);
      if (!empty && whole && (mn > MU_CAP || gn > GU_CAP)) {
        whole = false;  // fall back to one alignment tile per pass
        seg = 0;
        continue;
      }
      if (!empty) {
        for (int k = tid; k < gn; k += THREADS) {
          float r, gg, b;
          load_guide(f, g, gr0 + k / gw, gc0 + k % gw, r, gg, b);
          sGuide[0][k] = r;
          sGuide[1][k] = gg;
          sGuide[2][k] = b;
        }
        __syncthreads();
        for (int k = tid; k < mn; k += THREADS) {
          const int I = mr0 + k / mw, J = mc0 + k % mw;
          float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const int q = (clampi(I + a - 1, 0, g.h - 1) - gr0) * gw + clampi(J + b - 1, 0, g.w - 1) - gc0;
              s0 += sGuide[0][q];
              s1 += sGuide[1][q];
              s2 += sGuide[2][q];
            }
          sMu[0][k] = s0 / 9.f;
          sMu[1][k] = s1 / 9.f;
          sMu[2][k] = s2 / 9.f;
        }
        __syncthreads();
        for (int k = tid; k < rn; k += THREADS) {
          const int I = ra0 + k / rw, J = ca0 + k % rw;
          const int ty = min(2 * I / g.T, g.TY - 1), tx = min(2 * J / g.T, g.TX - 1);
          if (!whole && (ty != sty || tx != stx)) continue;
          double hx, hy;
          warped_pos(mv, g, I, J, ty, tx, hx, hy);
          const double fhx = floor(hx), fhy = floor(hy);
          const float fx = (float)(hx - fhx), fy = (float)(hy - fhy);
          const int x0 = (int)fhx, y0 = (int)fhy;
          const int xa = clampi(x0, 0, g.w - 1) - mc0, xb = clampi(x0 + 1, 0, g.w - 1) - mc0;
          const int ya = (clampi(y0, 0, g.h - 1) - mr0) * mw, yb = (clampi(y0 + 1, 0, g.h - 1) - mr0) * mw;
          float num = 0.f;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float top = (1.f - fx) * sMu[c][ya + xa] + fx * sMu[c][ya + xb];
            const float bot = (1.f - fx) * sMu[c][yb + xa] + fx * sMu[c][yb + xb];
            const float mu_al = (1.f - fy) * top + fy * bot;
            const float mu_ref = sMuRef[c][k];
            float var = rc.a_r * fmaxf(mu_ref - rc.black, 0.f) + rc.b_r;
            if (c == 1) var *= 0.5f;
            const float dms = mu_ref - mu_al;
            const float dms2 = dms * dms;
            const float d = dms * dms2 / (dms2 + var * (2.f / 9.f));  // Wiener shrinkage, eq. (6)
            num += d * d;
          }
          const float s = st[(size_t)ty * g.TX + tx];
          float R = s * __expf(-num * sInvDen[k]) - rc.t;  // eq. (5)
          sR[k] = fminf(fmaxf(R, 0.f), 1.f);
        }
      }
      if (whole) break;
      if (++seg >= nseg_tiles) break;
    }
    __syncthreads();
    // eq. (9): 5x5 minimum, separable, over existing pixels
    const int ow = min(RB_W, g.w - J0), oh = min(RB_H, g.h - I0);
    for (int k = tid; k < rh * ow; k += THREADS) {
      const int r = k / ow, J = J0 + k % ow;
      float m = 1.f;
#pragma unroll
      for (int b = -2; b <= 2; ++b) m = fminf(m, sR[r * rw + clampi(J + b, 0, g.w - 1) - ca0]);
      sTmp[r * RB_W + (J - J0)] = m;
    }
    __syncthreads();
    for (int k = tid; k < oh * ow; k += THREADS) {
      const int I = I0 + k / ow, j = k % ow;
      float m = 1.f;
#pragma unroll
      for (int a = -2; a <= 2; ++a) m = fminf(m, sTmp[(clampi(I + a, 0, g.h - 1) - ra0) * RB_W + j]);
      const size_t o = (size_t)n * plane + (size_t)I * g.w + J0 + j;
      rmin[o] = m;
      if (robust) robust[o] = sR[(I - ra0) * rw + (J0 + j - ca0)];
    }
  }
}

}  // namespace

hipError_t launch_robust(const Geometry& g, const RobustConsts& rc, const uint16_t* frames,
                         const float* motion, const float* s_tile, float* rmin, float* robust,
                         hipStream_t stream) {
  if (g.n < 2) return hipSuccess;
  const dim3 grid((g.w + RB_W - 1) / RB_W, (g.h + RB_H - 1) / RB_H);
  hipLaunchKernelGGL(k_robust, grid, dim3(THREADS), 0, stream, frames, motion, s_tile, g, rc, rmin,
                     robust);
  return hipGetLastError();
}

}  // namespace hmfsr
