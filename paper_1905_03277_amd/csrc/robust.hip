// Robustness of every aligned frame on the base frame's half-resolution grid
// (Sec. 5.2): noise-corrected colour distance (eq. 5-6), motion-prior strength
// (eq. 7-8, precomputed per tile) and the 5x5 minimum (eq. 9).
//
// Two passes:
//  * k_guide_means: the 3x3 box means of every frame's guide (R, mean G, B;
//    edge-replicated) into a map [n][3][h][w]; for the base frame also the
//    reciprocal of the noise-corrected variance sum of eq. (5)-(6) into
//    [h][w], negated where the S.3 test below finds a variance loss.
//  * k_robust: one workgroup per (32x16 tile of the base half-res grid,
//    aligned frame). R is evaluated on the tile plus a 2-pixel border (the
//    min-pool footprint; border pixels outside the grid repeat the edge pixel,
//    which is what the edge-clamped 5x5 minimum reads) by sampling the frame's
//    mean map bilinearly at u + v/2 (corners clamped to the map), then the
//    5x5 minimum in LDS. Any displacement field costs the same.
//
// Colour statistics are kept in raw units (the black level enters only the
// noise model's brightness): the ratio d^2 / sigma^2 of eq. (5) is scale-free.
//
// High-frequency rejection (supplement S.3, when rc.hf > 0): with x the base
// guide doubled to integers and S its 3x3 box sums, per pixel
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
constexpr int TT_X = RR_W / 4 + 2, TT_Y = RR_H / 4 + 2;  // alignment tiles spanned (T >= 8)
constexpr int THREADS = 256;
constexpr int GM_W = 64, GM_H = 16;              // guide-means tile (half-res px)
constexpr int GW_W = GM_W + 4, GW_H = GM_H + 4;  // its guide window: two rings, edge-replicated
constexpr int GW_N = GW_W * GW_H;

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
__host__ __device__ __forceinline__ int means_tiles_x(const Geometry& g) { return (g.w + GM_W - 1) / GM_W; }
__host__ __device__ __forceinline__ int means_tiles_y(const Geometry& g) { return (g.h + GM_H - 1) / GM_H; }

// ---- pass 1: guide statistics ------------------------------------------------------
struct MeansSmem {
  float G[3][GW_N];  // guide at rows I0-2 .. I0+GM_H+1, columns J0-2 .., clamped to the grid
  float S[3][GW_N];  // row sums (aligned frames) or doubled 3x3 box sums (base frame, S.3)
  int sItem;
};

// One 64x16 tile (tile_x, tile_y) of frame n's mean map and, for the base
// frame, of the reciprocal variance sum with its S.3 sign.
__device__ __forceinline__ void guide_means_tile(const uint16_t* __restrict__ frames, const Geometry& g,
                                                 const RobustConsts& rc, float* __restrict__ gmu,
                                                 float* __restrict__ gref, int n, int tile_x, int tile_y,
                                                 MeansSmem& sm) {
  const int tid = threadIdx.x;
  const int I0 = tile_y * GM_H, J0 = tile_x * GM_W;
  const int gy0 = I0 - 2, gx0 = J0 - 2;
  const uint16_t* f = frames + (size_t)n * g.H * g.W;
  const size_t plane = (size_t)g.h * g.w;
  {
    const float ginv = 1.f / (float)GW_W;
    for (int k = tid; k < GW_N; k += THREADS) {
      const int r = split_row(k, ginv), c = k - r * GW_W;
      float vr, vg, vb;
      load_guide(f, g, clampi(gy0 + r, 0, g.h - 1), clampi(gx0 + c, 0, g.w - 1), vr, vg, vb);
      sm.G[0][k] = vr;
      sm.G[1][k] = vg;
      sm.G[2][k] = vb;
    }
  }
  __syncthreads();
  const int oh = min(GM_H, g.h - I0), ow = min(GM_W, g.w - J0);
  if (n != g.ref) {
    // 3x3 box mean, separable: row sums Hs = (g(Q-1) + g(Q)) + g(Q+1) at
    // rows I0-1 .., then (Hs(P-1) + Hs(P)) + Hs(P+1), times 1/9
    for (int k = tid; k < (GM_H + 2) * GM_W; k += THREADS) {
      const int r = k >> 6, j = k & (GM_W - 1);  // GM_W == 64
      const int q = (r + 1) * GW_W + j + 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) sm.S[c][k] = (sm.G[c][q] + sm.G[c][q + 1]) + sm.G[c][q + 2];
    }
    __syncthreads();
    for (int k = tid; k < GM_H * GM_W; k += THREADS) {
      const int i = k >> 6, j = k & (GM_W - 1);
      if (i >= oh || j >= ow) continue;
      const size_t o = (size_t)(I0 + i) * g.w + J0 + j;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float* col = sm.S[c] + i * GM_W + j;
        gmu[((size_t)n * 3 + c) * plane + o] = ((col[0] + col[GM_W]) + col[2 * GM_W]) * (1.f / 9.f);
      }
    }
    return;
  }
  if (rc.hf > 0.0) {
    // doubled 3x3 box sums at window rows and columns 1 .. GW - 2 (integers
    // below 2^24: exact in float whatever the order); the S.3 test reads them
    // only at window positions of grid pixels, whose neighbours the window
    // holds edge-replicated
    for (int k = tid; k < (GW_H - 2) * (GW_W - 2); k += THREADS) {
      const int r = k / (GW_W - 2), c0 = k - r * (GW_W - 2);
      const int q = r * GW_W + c0;  // window position of the sum's top-left neighbour
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float sum = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) sum += 2.f * sm.G[c][q + a * GW_W + b];
        sm.S[c][q + GW_W + 1] = sum;
      }
    }
    __syncthreads();
  }
  // base frame: 3x3 mean and population variance of the guide, noise-corrected
  // per channel (eq. 6), the reciprocal of their sum (eq. 5)
  for (int k = tid; k < GM_H * GM_W; k += THREADS) {
    const int i = k >> 6, j = k & (GM_W - 1);
    if (i >= oh || j >= ow) continue;
    const int P = I0 + i, Q = J0 + j;
    const int o = (i + 1) * GW_W + (j + 1);  // window position of (P - 1, Q - 1)
    float den = 0.f;
    float mu3[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float v[9];
      float s = 0.f;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          v[a * 3 + b] = sm.G[c][o + a * GW_W + b];
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
      mu3[c] = mu;
      den += fmaxf(var_ms, var_md);  // sigma = max(sigma_ms, sigma_md), eq. (6)
    }
    float inv = 1.f / den;
    if (rc.hf > 0.0) {
      // the 3x3 neighbourhood of grid positions clamped to the grid
      double A = 0.0, B = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double sx = 0.0, sxx = 0.0, ss = 0.0, sss = 0.0;
#pragma unroll
        for (int a = -1; a <= 1; ++a)
#pragma unroll
          for (int b = -1; b <= 1; ++b) {
            const int wq = (clampi(P + a, 0, g.h - 1) - gy0) * GW_W + clampi(Q + b, 0, g.w - 1) - gx0;
            const double xv = 2.0 * (double)sm.G[c][wq];
            const double sv = (double)sm.S[c][wq];
            sx += xv;
            sxx += xv * xv;
            ss += sv;
            sss += sv * sv;
          }
        B += 9.0 * sxx - sx * sx;
        A += 9.0 * sss - ss * ss;
      }
      if (A < rc.hf * (81.0 * B)) inv = -inv;
    }
    const size_t op = (size_t)P * g.w + Q;
#pragma unroll
    for (int c = 0; c < 3; ++c) gmu[((size_t)n * 3 + c) * plane + op] = mu3[c];
    gref[op] = inv;
  }
}

// Workgroup (tile, frame).
__global__ __launch_bounds__(THREADS) void k_guide_means(const uint16_t* __restrict__ frames, Geometry g,
                                                         RobustConsts rc, float* __restrict__ gmu,
                                                         float* __restrict__ gref) {
  __shared__ MeansSmem sm;
  const int tx_n = means_tiles_x(g), t = xcd_tile(blockIdx.x, tx_n * means_tiles_y(g));
  guide_means_tile(frames, g, rc, gmu, gref, blockIdx.y, t % tx_n, t / tx_n, sm);
}

// Every (burst, frame, tile) of a batch, one workgroup each.
__global__ __launch_bounds__(THREADS) void k_guide_means_batch(const BurstArgs* __restrict__ bursts,
                                                               const int* __restrict__ first, int n_bursts) {
  __shared__ MeansSmem sm;
  const int i = blockIdx.x;
  int lo = 0, hi = n_bursts - 1;  // last burst with first[b] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= i) lo = mid; else hi = mid - 1;
  }
  const BurstArgs& b = bursts[lo];
  const int tx_n = means_tiles_x(b.g), per = tx_n * means_tiles_y(b.g);
  const int k = i - first[lo], n = k / per, t = k - n * per;
  guide_means_tile(b.frames, b.g, b.rc, b.gmu, b.gref, n, t % tx_n, t / tx_n, sm);
}

// ---- pass 2: robustness and its 5x5 minimum ---------------------------------------
struct RobustSmem {
  float sR[RR_N];
  float sTmp[RR_H * RB_W];
  int sTyR[RR_H], sTxR[RR_W];  // alignment tile of each region row / column
  int2 sO[TT_X * TT_Y];        // floor(v / 2): integer part of the half-res displacement
  float2 sF[TT_X * TT_Y];      // v / 2 - floor(v / 2): the bilinear fractions, exact
  float sS[TT_X * TT_Y];
  int sMov[TT_X * TT_Y];       // motion prior's choice (s1) per alignment tile
  float2 sMv[(TT_X + 2) * (TT_Y + 2)];  // the frame's vectors of those tiles and a ring
  int sItem;
};

// R_hat of one 32x16 half-res tile (tile_x, tile_y) of aligned frame n.
__device__ __forceinline__ void robust_tile_frame(const float* __restrict__ motion,
                                                  const float* __restrict__ s_tile, const Geometry& g,
                                                  const RobustConsts& rc, const float* __restrict__ gmu,
                                                  const float* __restrict__ gref, float* __restrict__ rmin,
                                                  float* __restrict__ robust, int n, int tile_x, int tile_y,
                                                  RobustSmem& sm) {
  const int tid = threadIdx.x;
  const int I0 = tile_y * RB_H, J0 = tile_x * RB_W;
  const int ra0 = I0 - 2, ca0 = J0 - 2;  // region origin (may be outside the grid)
  const size_t plane = (size_t)g.h * g.w;

  if (tid < RR_W) sm.sTxR[tid] = min(2 * clampi(ca0 + tid, 0, g.w - 1) / g.T, g.TX - 1);
  if (tid >= 64 && tid < 64 + RR_H) {
    const int r = tid - 64;
    sm.sTyR[r] = min(2 * clampi(ra0 + r, 0, g.h - 1) / g.T, g.TY - 1);
  }
  __syncthreads();
  const int txA = sm.sTxR[0], tyA = sm.sTyR[0];
  const int ntx = sm.sTxR[RR_W - 1] - txA + 1, nty = sm.sTyR[RR_H - 1] - tyA + 1, ntiles = ntx * nty;
  const int mvw = ntx + 2, mvn = (nty + 2) * (ntx + 2);
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
      sm.sMv[k] = v;
    }
    __syncthreads();
  }
  // per alignment tile: the bilinear base corner of u + v/2 is u + floor(v/2)
  // (u integer) with the same fractions for every pixel of the tile
  const float vlim = (float)(max(g.W, g.H) + 16);
  for (int k = tid; k < ntiles; k += THREADS) {
    const int ky = k / ntx, kx = k - ky * ntx;
    const size_t t = ((size_t)n * g.TY + tyA + ky) * g.TX + txA + kx;
    const float* p = motion + 2 * t;
    // clamping keeps non-finite or huge vectors finite and changes no result
    const float hx = fminf(fmaxf(p[0], -vlim), vlim) * 0.5f, hy = fminf(fmaxf(p[1], -vlim), vlim) * 0.5f;
    const float fx = floorf(hx), fy = floorf(hy);
    sm.sO[k] = make_int2((int)fx, (int)fy);
    sm.sF[k] = make_float2(hx - fx, hy - fy);  // exact: v/2 has at most 24 significant bits
    sm.sS[k] = s_tile[t];
    if (rc.hf > 0.0) {
      // eq. (7)-(8) as the motion prior takes them: spread over the existing
      // 3x3 tiles in float64, M^2 > M_th^2 rounded operation by operation
      double xmax = -INFINITY, xmin = INFINITY, ymax = -INFINITY, ymin = INFINITY;
      for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b) {
          const int y = tyA + ky + a, x = txA + kx + b;
          if (y < 0 || y >= g.TY || x < 0 || x >= g.TX) continue;
          const float2 v = sm.sMv[(ky + 1 + a) * mvw + kx + 1 + b];
          xmax = fmax(xmax, (double)v.x);
          xmin = fmin(xmin, (double)v.x);
          ymax = fmax(ymax, (double)v.y);
          ymin = fmin(ymin, (double)v.y);
        }
      const double mx = xmax - xmin, my = ymax - ymin;
      sm.sMov[k] = __dadd_rn(__dmul_rn(mx, mx), __dmul_rn(my, my)) > __dmul_rn(rc.m_th, rc.m_th);
    }
  }
  __syncthreads();
  const float* mun = gmu + (size_t)n * 3 * plane;
  const float* muref = gmu + (size_t)g.ref * 3 * plane;
  {
    const float rinv = 1.f / (float)RR_W;
    for (int k = tid; k < RR_N; k += THREADS) {
      const int rr = split_row(k, rinv), cc = k - rr * RR_W;
      const int kt = (sm.sTyR[rr] - tyA) * ntx + (sm.sTxR[cc] - txA);
      const int I = clampi(ra0 + rr, 0, g.h - 1), J = clampi(ca0 + cc, 0, g.w - 1);
      const int2 o = sm.sO[kt];
      const float2 fr = sm.sF[kt];
      const float fx = fr.x, fy = fr.y;
      // the frame's mean map at u + v/2, corners clamped to the map
      const int ya = clampi(I + o.y, 0, g.h - 1), yb = clampi(I + o.y + 1, 0, g.h - 1);
      const int xa = clampi(J + o.x, 0, g.w - 1), xb = clampi(J + o.x + 1, 0, g.w - 1);
      const size_t p00 = (size_t)ya * g.w + xa, p01 = (size_t)ya * g.w + xb;
      const size_t p10 = (size_t)yb * g.w + xa, p11 = (size_t)yb * g.w + xb;
      const size_t pr = (size_t)I * g.w + J;
      const float ginv = gref[pr];
      float num = 0.f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float* m = mun + (size_t)c * plane;
        const float m00 = m[p00], m01 = m[p01], m10 = m[p10], m11 = m[p11];
        const float top = fmaf(fx, m01 - m00, m00), bot = fmaf(fx, m11 - m10, m10);
        const float mu_al = fmaf(fy, bot - top, top);
        const float mu_ref = muref[(size_t)c * plane + pr];
        float sig2, dmd2;
        noise_md(rc, mu_ref, c, sig2, dmd2);
        const float dms = mu_ref - mu_al;
        const float dms2 = dms * dms;
        // Wiener shrinkage of eq. (6): d = d_ms^3 / (d_ms^2 + d_md^2)
        const float dd = dms * dms2 * __builtin_amdgcn_rcpf(dms2 + dmd2);
        num = fmaf(dd, dd, num);
      }
      const float R = sm.sS[kt] * __expf(-num * fabsf(ginv)) - rc.t;  // eq. (5)
      sm.sR[k] = rc.hf > 0.0 && ginv < 0.f && sm.sMov[kt] ? 0.f : fminf(fmaxf(R, 0.f), 1.f);
    }
  }
  __syncthreads();
  // eq. (9): 5x5 minimum, separable (the region repeats edge pixels)
  const int ow = min(RB_W, g.w - J0), oh = min(RB_H, g.h - I0);
  for (int k = tid; k < RR_H * RB_W; k += THREADS) {
    const int r = k >> 5, j = k & 31;  // RB_W == 32
    const float* row = sm.sR + r * RR_W + j;
    sm.sTmp[k] = fminf(fminf(fminf(row[0], row[1]), fminf(row[2], row[3])), row[4]);
  }
  __syncthreads();
  for (int k = tid; k < RB_H * RB_W; k += THREADS) {
    const int i = k >> 5, j = k & 31;
    if (i >= oh || j >= ow) continue;
    const float* col = sm.sTmp + i * RB_W + j;
    const float m = fminf(fminf(fminf(col[0], col[RB_W]), fminf(col[2 * RB_W], col[3 * RB_W])), col[4 * RB_W]);
    const size_t o = (size_t)n * plane + (size_t)(I0 + i) * g.w + J0 + j;
    rmin[o] = m;
    if (robust) robust[o] = sm.sR[(i + 2) * RR_W + j + 2];
  }
}

// Workgroup (tile, aligned frame): blockIdx.y enumerates the frames other
// than the base.
__global__ __launch_bounds__(THREADS) void k_robust(const float* __restrict__ motion,
                                                    const float* __restrict__ s_tile, Geometry g,
                                                    RobustConsts rc, const float* __restrict__ gmu,
                                                    const float* __restrict__ gref, float* __restrict__ rmin,
                                                    float* __restrict__ robust) {
  __shared__ RobustSmem sm;
  const int tx_n = robust_tiles_x_(g), t = xcd_tile(blockIdx.x, tx_n * robust_tiles_y_(g));
  const int n = (int)blockIdx.y < g.ref ? (int)blockIdx.y : (int)blockIdx.y + 1;
  robust_tile_frame(motion, s_tile, g, rc, gmu, gref, rmin, robust, n, t % tx_n, t / tx_n, sm);
}

// Persistent form over (burst, tile) items of a batch, the tile's aligned
// frames in turn.
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
    for (int n = 0; n < b.g.n; ++n) {
      if (n == b.g.ref) continue;
      __syncthreads();  // the previous frame's LDS is no longer read
      robust_tile_frame(b.motion, b.s_tile, b.g, b.rc, b.gmu, b.gref, b.rmin, nullptr, n,
                        w.tile % b.robust_tiles_x, w.tile / b.robust_tiles_x, sm);
    }
  }
}

}  // namespace

int robust_tiles_x(const Geometry& g) { return robust_tiles_x_(g); }
int robust_tiles_y(const Geometry& g) { return robust_tiles_y_(g); }
int guide_means_groups(const Geometry& g) { return g.n > 1 ? g.n * means_tiles_x(g) * means_tiles_y(g) : 0; }

hipError_t launch_robust(const Geometry& g, const RobustConsts& rc, const uint16_t* frames,
                         const float* motion, const Work& w, float* rmin, float* robust,
                         hipStream_t stream) {
  if (g.n < 2) return hipSuccess;
  hipLaunchKernelGGL(k_guide_means, dim3(means_tiles_x(g) * means_tiles_y(g), g.n), dim3(THREADS), 0, stream,
                     frames, g, rc, w.gmu, w.gref);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_robust, dim3(robust_tiles_x(g) * robust_tiles_y(g), g.n - 1), dim3(THREADS), 0, stream,
                     motion, w.s_tile, g, rc, w.gmu, w.gref, rmin, robust);
  return hipGetLastError();
}

hipError_t launch_guide_means_batch(const BurstArgs* bursts, const int* first, int n_bursts, int total,
                                    hipStream_t stream) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_guide_means_batch, dim3(total), dim3(THREADS), 0, stream, bursts, first, n_bursts);
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
