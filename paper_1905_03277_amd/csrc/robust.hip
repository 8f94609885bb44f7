// Robustness of every aligned frame on the base frame's half-resolution grid
// (Sec. 5.2): noise-corrected colour distance (eq. 5-6), motion-prior strength
// (eq. 7-8, precomputed per tile) and the 5x5 minimum (eq. 9).
//
// One workgroup owns a 32x16 tile of the base half-res grid and loops over the
// frames. The robustness is evaluated on the tile plus a 2-pixel border (the
// min-pool footprint); border pixels outside the grid repeat the edge pixel,
// which is what the edge-clamped 5x5 minimum reads. The base frame's 3x3 guide
// mean and noise-corrected sigma are computed once into LDS; for each aligned
// frame the guide around the warped footprint is staged (edge-replicated),
// box-filtered, and sampled bilinearly at u + v/2 for every robustness pixel.
//
// Colour statistics are kept in raw units (the black level enters only the
// noise model's brightness): the ratio d^2 / sigma^2 of eq. (5) is scale-free.
//
// High-frequency rejection (supplement S.3, when rc.hf > 0): with x the base
// guide doubled to integers and S its 3x3 box sums, per region pixel
// B = sum_c 9 sum x^2 - (sum x)^2 over the 3x3 window and A = the same over the
// 3x3 window of S (all integers below 2^53, so float64 holds them exactly);
// where A < hf * 81 B (variance lost to the low-pass) and the tile's motion
// prior chose s1 (eq. 8), R of the aligned frame is 0.
#include "device_util.h"
#include "hmfsr_internal.h"
#include "noise.h"

namespace hmfsr {
namespace {

constexpr int RB_W = 32, RB_H = 16;              // output tile of R_hat (half-res px)
constexpr int RR_W = RB_W + 4, RR_H = RB_H + 4;  // robustness region incl. the min-pool border
constexpr int RR_N = RR_W * RR_H;
constexpr int MU_CAP = 1000;                     // frame-n box-mean window
constexpr int GU_CAP = 1150;                     // frame-n guide window and row sums
constexpr int TT_X = RR_W / 4 + 2, TT_Y = RR_H / 4 + 2;  // alignment tiles spanned (T >= 8)
constexpr int THREADS = 256;

// Raw value at parity position pos (row-major in the 2x2 quad) from the quad's
// two 32-bit rows; pos is uniform, so this is a select and a shift.
__device__ __forceinline__ uint32_t quad_at(uint32_t top, uint32_t bot, int pos) {
  return ((pos & 2) ? bot : top) >> ((pos & 1) * 16) & 0xffffu;
}

// Guide pixel (I, J) of a frame in raw units: R, mean of the two greens, B.
__device__ __forceinline__ void load_guide(const uint16_t* f, const Geometry& g, int I, int J,
                                           float& r, float& gr, float& b) {
  const uint32_t top = *(const uint32_t*)(f + (size_t)(2 * I) * g.W + 2 * J);
  const uint32_t bot = *(const uint32_t*)(f + (size_t)(2 * I + 1) * g.W + 2 * J);
  r = (float)quad_at(top, bot, g.red_pos);
  gr = (float)(quad_at(top, bot, g.green_pos[0]) + quad_at(top, bot, g.green_pos[1])) * 0.5f;
  b = (float)quad_at(top, bot, g.blue_pos);
}

__host__ __device__ __forceinline__ int robust_tiles_x_(const Geometry& g) { return (g.w + RB_W - 1) / RB_W; }
__host__ __device__ __forceinline__ int robust_tiles_y_(const Geometry& g) { return (g.h + RB_H - 1) / RB_H; }

struct Bounds4 {
  int x0, x1, y0, y1;  // range of the bilinear base corner floor(u + v/2)
};

struct RobustSmem {
  float sMuRef[3][RR_N];
  float sInvDen[RR_N];
  float sGuide[3][GU_CAP];  // guide, then the box means
  float sHs[3][GU_CAP];     // horizontal 3-sums
  float sR[RR_N];
  float sTmp[RR_H * RB_W];
  int sTyR[RR_H], sTxR[RR_W];  // alignment tile of each region row / column
  int sRlo[TT_Y], sRhi[TT_Y], sClo[TT_X], sChi[TT_X];
  int2 sO[TT_X * TT_Y];     // floor(v / 2): integer part of the half-res displacement
  float2 sF[TT_X * TT_Y];   // v / 2 - floor(v / 2): the bilinear fractions, exact
  float sS[TT_X * TT_Y];
  Bounds4 sTB[TT_X * TT_Y];
  int sRed[5];
  int sItem;
  int sLoss[RR_N];           // S.3 variance loss of the base guide per region pixel
  int sMov[TT_X * TT_Y];     // motion prior's choice (s1) per alignment tile
  float2 sMv[(TT_X + 2) * (TT_Y + 2)];  // the frame's vectors of those tiles and a ring
};

// R_hat of one 32x16 half-res tile (tile_x, tile_y) of one burst, every aligned frame.
__device__ __forceinline__ void robust_tile(const uint16_t* __restrict__ frames,
                                            const float* __restrict__ motion,
                                            const float* __restrict__ s_tile, const Geometry& g,
                                            const RobustConsts& rc, float* __restrict__ rmin,
                                            float* __restrict__ robust, int tile_x, int tile_y,
                                            RobustSmem& sm) {
  float(*sMuRef)[RR_N] = sm.sMuRef;
  float* sInvDen = sm.sInvDen;
  float(*sGuide)[GU_CAP] = sm.sGuide;
  float(*sHs)[GU_CAP] = sm.sHs;
  float* sR = sm.sR;
  float* sTmp = sm.sTmp;
  int* sTyR = sm.sTyR;
  int* sTxR = sm.sTxR;
  int* sRlo = sm.sRlo;
  int* sRhi = sm.sRhi;
  int* sClo = sm.sClo;
  int* sChi = sm.sChi;
  int2* sO = sm.sO;
  float2* sF = sm.sF;
  float* sS = sm.sS;
  Bounds4* sTB = sm.sTB;
  int* sRed = sm.sRed;
  int* sLoss = sm.sLoss;
  int* sMov = sm.sMov;
  float2* sMv = sm.sMv;

  const int tid = threadIdx.x;
  const int I0 = tile_y * RB_H, J0 = tile_x * RB_W;
  const int ra0 = I0 - 2, ca0 = J0 - 2;  // region origin (may be outside the grid)
  const size_t plane = (size_t)g.h * g.w;

  if (tid < RR_W) sTxR[tid] = min(2 * clampi(ca0 + tid, 0, g.w - 1) / g.T, g.TX - 1);
  if (tid >= 64 && tid < 64 + RR_H) {
    const int r = tid - 64;
    sTyR[r] = min(2 * clampi(ra0 + r, 0, g.h - 1) / g.T, g.TY - 1);
  }
  __syncthreads();
  const int txA = sTxR[0], tyA = sTyR[0];
  const int ntx = sTxR[RR_W - 1] - txA + 1, nty = sTyR[RR_H - 1] - tyA + 1, ntiles = ntx * nty;
  if (tid < RR_W) {
    const int t = sTxR[tid] - txA;
    if (tid == 0 || sTxR[tid - 1] != sTxR[tid]) sClo[t] = tid;
    if (tid == RR_W - 1 || sTxR[tid + 1] != sTxR[tid]) sChi[t] = tid;
  }
  if (tid >= 64 && tid < 64 + RR_H) {
    const int r = tid - 64, t = sTyR[r] - tyA;
    if (r == 0 || sTyR[r - 1] != sTyR[r]) sRlo[t] = r;
    if (r == RR_H - 1 || sTyR[r + 1] != sTyR[r]) sRhi[t] = r;
  }

  // ---- base frame statistics, once ------------------------------------
  {
    const uint16_t* f = frames + (size_t)g.ref * g.H * g.W;
    // guide rows/cols around the clamped region, edge-replicated one step
    // further (two with the S.3 test, whose box sums need a ring more)
    const int ring = rc.hf > 0.0 ? 2 : 1;
    const int gr0 = clampi(ra0, 0, g.h - 1) - ring, gr1 = clampi(ra0 + RR_H - 1, 0, g.h - 1) + ring;
    const int gc0 = clampi(ca0, 0, g.w - 1) - ring, gc1 = clampi(ca0 + RR_W - 1, 0, g.w - 1) + ring;
    const int gw = gc1 - gc0 + 1, gn = gw * (gr1 - gr0 + 1);
    const float ginv = 1.f / (float)gw;
    for (int k = tid; k < gn; k += THREADS) {
      const int rr = split_row(k, ginv);
      float r, gg, b;
      load_guide(f, g, clampi(gr0 + rr, 0, g.h - 1), clampi(gc0 + k - rr * gw, 0, g.w - 1), r, gg, b);
      sGuide[0][k] = r;
      sGuide[1][k] = gg;
      sGuide[2][k] = b;
    }
    __syncthreads();
    const float rinv = 1.f / (float)RR_W;
    for (int k = tid; k < RR_N; k += THREADS) {
      const int rr = split_row(k, rinv), cc = k - rr * RR_W;
      const int I = clampi(ra0 + rr, 0, g.h - 1), J = clampi(ca0 + cc, 0, g.w - 1);
      const int o = (I - 1 - gr0) * gw + (J - 1 - gc0);
      float den = 0.f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float v[9];
        float s = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            v[a * 3 + b] = sGuide[c][o + a * gw + b];
            s += v[a * 3 + b];
          }
        const float mu = s * (1.f / 9.f);
        float var_ms = 0.f;
#pragma unroll
        for (int q = 0; q < 9; ++q) var_ms = fmaf(v[q] - mu, v[q] - mu, var_ms);
        var_ms *= (1.f / 9.f);
        // noise model in raw units at the base brightness (the guide green is
        // the mean of two greens)
        float var_md, dmd2_unused;
        noise_md(rc, mu, c, var_md, dmd2_unused);
        sMuRef[c][k] = mu;
        den += fmaxf(var_ms, var_md);  // sigma = max(sigma_ms, sigma_md), eq. (6)
      }
      sInvDen[k] = 1.f / den;
    }
    if (rc.hf > 0.0) {
      // box sums of the doubled guide at the image positions rows
      // [clamp(ra0) - 1, clamp(ra0 + RR_H - 1) + 1], columns alike (integers
      // below 2^24: exact in float whatever the order)
      const int sr0 = clampi(ra0, 0, g.h - 1) - 1, sc0 = clampi(ca0, 0, g.w - 1) - 1;
      const int sh = clampi(ra0 + RR_H - 1, 0, g.h - 1) + 1 - sr0 + 1;
      const int swd = clampi(ca0 + RR_W - 1, 0, g.w - 1) + 1 - sc0 + 1;
      const float sinv = 1.f / (float)swd;
      for (int k = tid; k < sh * swd; k += THREADS) {
        const int q = split_row(k, sinv);
        const int P = sr0 + q, Q = sc0 + k - q * swd;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          float sum = 0.f;
#pragma unroll
          for (int a = -1; a <= 1; ++a)
#pragma unroll
            for (int b = -1; b <= 1; ++b)
              sum += 2.f * sGuide[c][(clampi(P + a, 0, g.h - 1) - gr0) * gw + clampi(Q + b, 0, g.w - 1) - gc0];
          sHs[c][k] = sum;
        }
      }
      __syncthreads();
      const float rinv2 = 1.f / (float)RR_W;
      for (int k = tid; k < RR_N; k += THREADS) {
        const int rr = split_row(k, rinv2), cc = k - rr * RR_W;
        const int I = clampi(ra0 + rr, 0, g.h - 1), J = clampi(ca0 + cc, 0, g.w - 1);
        double A = 0.0, B = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double sx = 0.0, sxx = 0.0, ss = 0.0, sss = 0.0;
#pragma unroll
          for (int a = -1; a <= 1; ++a)
#pragma unroll
            for (int b = -1; b <= 1; ++b) {
              const int y = clampi(I + a, 0, g.h - 1), x = clampi(J + b, 0, g.w - 1);
              const double xv = 2.0 * (double)sGuide[c][(y - gr0) * gw + x - gc0];
              const double sv = (double)sHs[c][(y - sr0) * swd + x - sc0];
              sx += xv;
              sxx += xv * xv;
              ss += sv;
              sss += sv * sv;
            }
          B += 9.0 * sxx - sx * sx;
          A += 9.0 * sss - ss * ss;
        }
        sLoss[k] = A < rc.hf * (81.0 * B);
      }
    }
  }

  // ---- aligned frames -------------------------------------------------
  const float vlim = (float)(max(g.W, g.H) + 16);
  const int mvw = ntx + 2, mvn = (nty + 2) * (ntx + 2);
  for (int n = 0; n < g.n; ++n) {
    if (n == g.ref) continue;
    const uint16_t* f = frames + (size_t)n * g.H * g.W;
    __syncthreads();
    if (rc.hf > 0.0) {
      // the S.3 test takes the motion prior's decision (eq. 8) per tile: stage
      // the tiles' vectors and their ring once, in one round of loads
      for (int k = tid; k < mvn; k += THREADS) {
        const int y = tyA - 1 + k / mvw, x = txA - 1 + k % mvw;
        float2 v = make_float2(0.f, 0.f);
        if (y >= 0 && y < g.TY && x >= 0 && x < g.TX) {
          const float* p = motion + (((size_t)n * g.TY + y) * g.TX + x) * 2;  // 4-byte aligned
          v = make_float2(p[0], p[1]);
        }
        sMv[k] = v;
      }
      __syncthreads();
    }
    // per alignment tile: the bilinear base corner of u + v/2 is u + floor(v/2)
    // (u integer) with the same fractions for every pixel of the tile; and the
    // tile's footprint (monotonic in the pixel position). Wave 0 reduces the
    // footprints without atomics.
    if (tid < 64) {
      Bounds4 acc = {0x7fffffff, -0x7fffffff, 0x7fffffff, -0x7fffffff};
      int need = 0;  // largest guide window of one tile, (mw + 2) (mh + 2)
      for (int k = tid; k < ntiles; k += 64) {
        const int ky = k / ntx, kx = k - ky * ntx;
        const size_t t = ((size_t)n * g.TY + tyA + ky) * g.TX + txA + kx;
        const float* p = motion + 2 * t;
        // clamping keeps non-finite or huge vectors finite and changes no result
        const float hx = fminf(fmaxf(p[0], -vlim), vlim) * 0.5f, hy = fminf(fmaxf(p[1], -vlim), vlim) * 0.5f;
        const float fx = floorf(hx), fy = floorf(hy);
        const int2 o = make_int2((int)fx, (int)fy);
        sO[k] = o;
        sF[k] = make_float2(hx - fx, hy - fy);  // exact: v/2 has at most 24 significant bits
        sS[k] = s_tile[t];
        if (rc.hf > 0.0) {
          // eq. (7)-(8) as the motion prior takes them: spread over the existing
          // 3x3 tiles in float64, M^2 > M_th^2 rounded operation by operation
          double xmax = -INFINITY, xmin = INFINITY, ymax = -INFINITY, ymin = INFINITY;
          for (int a = -1; a <= 1; ++a)
            for (int b = -1; b <= 1; ++b) {
              const int y = tyA + ky + a, x = txA + kx + b;
              if (y < 0 || y >= g.TY || x < 0 || x >= g.TX) continue;
              const float2 v = sMv[(ky + 1 + a) * mvw + kx + 1 + b];
              xmax = fmax(xmax, (double)v.x);
              xmin = fmin(xmin, (double)v.x);
              ymax = fmax(ymax, (double)v.y);
              ymin = fmin(ymin, (double)v.y);
            }
          const double mx = xmax - xmin, my = ymax - ymin;
          sMov[k] = __dadd_rn(__dmul_rn(mx, mx), __dmul_rn(my, my)) > __dmul_rn(rc.m_th, rc.m_th);
        }
        Bounds4 b;
        b.x0 = clampi(ca0 + sClo[kx], 0, g.w - 1) + o.x;
        b.x1 = clampi(ca0 + sChi[kx], 0, g.w - 1) + o.x;
        b.y0 = clampi(ra0 + sRlo[ky], 0, g.h - 1) + o.y;
        b.y1 = clampi(ra0 + sRhi[ky], 0, g.h - 1) + o.y;
        sTB[k] = b;
        need = max(need, (b.x1 - b.x0 + 4) * (b.y1 - b.y0 + 4));
        acc.x0 = min(acc.x0, b.x0);
        acc.x1 = max(acc.x1, b.x1);
        acc.y0 = min(acc.y0, b.y0);
        acc.y1 = max(acc.y1, b.y1);
      }
      acc.x0 = wave_min(acc.x0);
      acc.x1 = -wave_min(-acc.x1);
      acc.y0 = wave_min(acc.y0);
      acc.y1 = -wave_min(-acc.y1);
      need = -wave_min(-need);
      if (tid == 0) {
        sRed[4] = need;
        sRed[0] = acc.x0;
        sRed[1] = -acc.x1;
        sRed[2] = acc.y0;
        sRed[3] = -acc.y1;
      }
    }
    __syncthreads();
    // Either one window covers every tile's footprint, or the tiles are
    // processed P at a time (one group of THREADS / P threads each, its own
    // 1 / P of the window buffers; P as large as the largest tile window
    // allows). The arithmetic per pixel is the same either way.
    const bool whole = [&] {
      const int mw = -sRed[1] - sRed[0] + 2, mh = -sRed[3] - sRed[2] + 2;
      return mw * mh <= MU_CAP && (mw + 2) * (mh + 2) <= GU_CAP && (mh + 2) * mw <= GU_CAP;
    }();
    const int need = sRed[4];
    const int P = whole ? 1 : need <= GU_CAP / 4 ? 4 : need <= GU_CAP / 2 ? 2 : 1;
    const int gsz = THREADS / P, gi = tid / gsz, lt = tid - gi * gsz, cap = GU_CAP / P;
    for (int s0 = 0; s0 < (whole ? 1 : ntiles); s0 += P) {
      const int seg = s0 + gi;
      const bool act = whole || seg < ntiles;
      Bounds4 bd = {0, 0, 0, 0};
      if (whole) {
        bd.x0 = sRed[0]; bd.x1 = -sRed[1]; bd.y0 = sRed[2]; bd.y1 = -sRed[3];
      } else if (act) {
        bd = sTB[seg];
      }
      float* G[3] = {sGuide[0] + gi * cap, sGuide[1] + gi * cap, sGuide[2] + gi * cap};
      float* Hs[3] = {sHs[0] + gi * cap, sHs[1] + gi * cap, sHs[2] + gi * cap};
      // box-mean window: every bilinear corner (unclamped; entries outside the
      // grid repeat the edge); guide window: their clamped 3x3 neighbourhoods.
      const int mc0 = bd.x0, mw = bd.x1 - bd.x0 + 2;
      const int mr0 = bd.y0, mh = bd.y1 - bd.y0 + 2;
      const int gc0 = clampi(mc0, 0, g.w - 1) - 1, gc1 = clampi(mc0 + mw - 1, 0, g.w - 1) + 1;
      const int gr0 = clampi(mr0, 0, g.h - 1) - 1, gr1 = clampi(mr0 + mh - 1, 0, g.h - 1) + 1;
      const int gw = gc1 - gc0 + 1, gn = gw * (gr1 - gr0 + 1);
      const int gh = gr1 - gr0 + 1;
      if (act) {
        const float ginv = 1.f / (float)gw;
        for (int k = lt; k < gn; k += gsz) {
          const int rr = split_row(k, ginv);
          float r, gg, b;
          load_guide(f, g, clampi(gr0 + rr, 0, g.h - 1), clampi(gc0 + k - rr * gw, 0, g.w - 1), r, gg, b);
          G[0][k] = r;
          G[1][k] = gg;
          G[2][k] = b;
        }
      }
      __syncthreads();
      // 3x3 box mean, separable: row sums over the guide rows, then column sums
      if (act) {
        const float minv = 1.f / (float)mw;
        for (int k = lt; k < gh * mw; k += gsz) {
          const int rr = split_row(k, minv), cc = k - rr * mw;
          const int q = rr * gw + clampi(mc0 + cc, 0, g.w - 1) - 1 - gc0;
#pragma unroll
          for (int c = 0; c < 3; ++c) Hs[c][k] = (G[c][q] + G[c][q + 1]) + G[c][q + 2];
        }
      }
      __syncthreads();
      if (act) {
        const float minv = 1.f / (float)mw;
        for (int k = lt; k < mw * mh; k += gsz) {
          const int rr = split_row(k, minv), cc = k - rr * mw;
          const int q = (clampi(mr0 + rr, 0, g.h - 1) - 1 - gr0) * mw + cc;
#pragma unroll
          for (int c = 0; c < 3; ++c) G[c][k] = ((Hs[c][q] + Hs[c][q + mw]) + Hs[c][q + 2 * mw]) * (1.f / 9.f);
        }
      }
      __syncthreads();
      if (act) {
        // region pixels: all of them, or the tile's own rectangle
        int rlo = 0, clo = 0, nr = RR_H, nc = RR_W;
        if (!whole) {
          const int ky = seg / ntx, kx = seg - (seg / ntx) * ntx;
          rlo = sRlo[ky];
          nr = sRhi[ky] - rlo + 1;
          clo = sClo[kx];
          nc = sChi[kx] - clo + 1;
        }
        const float cinv = 1.f / (float)nc;
        for (int q = lt; q < nr * nc; q += gsz) {
          const int qr = split_row(q, cinv);
          const int rr = rlo + qr, cc = clo + q - qr * nc;
          const int k = rr * RR_W + cc;
          const int kt = (sTyR[rr] - tyA) * ntx + (sTxR[cc] - txA);
          const int I = clampi(ra0 + rr, 0, g.h - 1), J = clampi(ca0 + cc, 0, g.w - 1);
          const int2 o = sO[kt];
          const float2 fr = sF[kt];
          const float fx = fr.x, fy = fr.y;
          const int ya = (I + o.y - mr0) * mw + (J + o.x - mc0);
          float num = 0.f;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float m00 = G[c][ya], m01 = G[c][ya + 1];
            const float m10 = G[c][ya + mw], m11 = G[c][ya + mw + 1];
            const float top = fmaf(fx, m01 - m00, m00), bot = fmaf(fx, m11 - m10, m10);
            const float mu_al = fmaf(fy, bot - top, top);
            const float mu_ref = sMuRef[c][k];
            float sig2, dmd2;
            noise_md(rc, mu_ref, c, sig2, dmd2);
            const float dms = mu_ref - mu_al;
            const float dms2 = dms * dms;
            // Wiener shrinkage of eq. (6): d = d_ms^3 / (d_ms^2 + d_md^2)
            const float dd = dms * dms2 * __builtin_amdgcn_rcpf(dms2 + dmd2);
            num = fmaf(dd, dd, num);
          }
          const float R = sS[kt] * __expf(-num * sInvDen[k]) - rc.t;  // eq. (5)
          sR[k] = rc.hf > 0.0 && sLoss[k] && sMov[kt] ? 0.f : fminf(fmaxf(R, 0.f), 1.f);
        }
      }
      __syncthreads();
    }
    // eq. (9): 5x5 minimum, separable (the region repeats edge pixels)
    const int ow = min(RB_W, g.w - J0), oh = min(RB_H, g.h - I0);
    for (int k = tid; k < RR_H * RB_W; k += THREADS) {
      const int r = k >> 5, j = k & 31;  // RB_W == 32
      const float* row = sR + r * RR_W + j;
      sTmp[k] = fminf(fminf(fminf(row[0], row[1]), fminf(row[2], row[3])), row[4]);
    }
    __syncthreads();
    for (int k = tid; k < RB_H * RB_W; k += THREADS) {
      const int i = k >> 5, j = k & 31;
      if (i >= oh || j >= ow) continue;
      const float* col = sTmp + i * RB_W + j;
      const float m = fminf(fminf(fminf(col[0], col[RB_W]), fminf(col[2 * RB_W], col[3 * RB_W])), col[4 * RB_W]);
      const size_t o = (size_t)n * plane + (size_t)(I0 + i) * g.w + J0 + j;
      rmin[o] = m;
      if (robust) robust[o] = sR[(i + 2) * RR_W + j + 2];
    }
  }
}

__global__ __launch_bounds__(THREADS) void k_robust(const uint16_t* __restrict__ frames,
                                                    const float* __restrict__ motion,
                                                    const float* __restrict__ s_tile, Geometry g,
                                                    RobustConsts rc, float* __restrict__ rmin,
                                                    float* __restrict__ robust) {
  __shared__ RobustSmem sm;
  const int tx_n = robust_tiles_x_(g), t = xcd_tile(blockIdx.x, tx_n * robust_tiles_y_(g));
  robust_tile(frames, motion, s_tile, g, rc, rmin, robust, t % tx_n, t / tx_n, sm);
}

// Persistent form over (burst, tile) items of a batch.
__global__ __launch_bounds__(THREADS) void k_robust_batch(const BurstArgs* __restrict__ bursts,
                                                          const WorkItem* __restrict__ items,
                                                          int n_items, int* __restrict__ counter) {
  __shared__ RobustSmem sm;
  while (true) {
    __syncthreads();
    if (threadIdx.x == 0) sm.sItem = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(sm.sItem);  // uniform: scalar loads below
    if (it >= n_items) break;
    const WorkItem w = items[it];
    const BurstArgs& b = bursts[w.burst];
    robust_tile(b.frames, b.motion, b.s_tile, b.g, b.rc, b.rmin, nullptr,
                w.tile % b.robust_tiles_x, w.tile / b.robust_tiles_x, sm);
  }
}

}  // namespace

int robust_tiles_x(const Geometry& g) { return robust_tiles_x_(g); }
int robust_tiles_y(const Geometry& g) { return robust_tiles_y_(g); }

hipError_t launch_robust(const Geometry& g, const RobustConsts& rc, const uint16_t* frames,
                         const float* motion, const float* s_tile, float* rmin, float* robust,
                         hipStream_t stream) {
  if (g.n < 2) return hipSuccess;
  const dim3 grid(robust_tiles_x(g) * robust_tiles_y(g));
  hipLaunchKernelGGL(k_robust, grid, dim3(THREADS), 0, stream, frames, motion, s_tile, g, rc, rmin,
                     robust);
  return hipGetLastError();
}

int robust_batch_blocks_per_cu() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_robust_batch, THREADS, 0) != hipSuccess) return 1;
  return b > 0 ? b : 1;
}

hipError_t launch_robust_batch(const BurstArgs* bursts, const WorkItem* items, int n_items,
                               int* counter, int n_groups, hipStream_t stream) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_robust_batch, dim3(n_groups), dim3(THREADS), 0, stream, bursts, items, n_items,
                     counter);
  return hipGetLastError();
}

}  // namespace hmfsr
