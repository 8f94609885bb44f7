// Robustness of every aligned frame on the base frame's half-resolution grid
// (Sec. 5.2): noise-corrected colour distance (eq. 5-6), motion-prior strength
// (eq. 7-8, precomputed per tile) and the 5x5 minimum (eq. 9).
//
// Two passes:
//  * guide statistics: k_frame_means writes the 3x3 box sums of every
//    aligned frame's guide (R, the two greens, B; edge-replicated; exact
//    integers packed into 8 bytes, guide_maps.h) into a map [n][h][w + 2]
//    (the edge columns repeated once on either side, so that the two
//    horizontal bilinear corners are adjacent whatever the clamping), one
//    wave walking down a 64-column strip with the row sums in registers;
//    k_base_stats writes the base frame's sums and the reciprocal of its
//    noise-corrected variance sum of eq. (5)-(6) into [h][w], negated where
//    the S.3 test below finds a variance loss.
//  * k_robust: one workgroup per 32x32 tile of the base half-res grid, the
//    aligned frames in turn (the base statistics stay in registers; on small
//    grids the frames are split over several workgroups per tile). R is
//    evaluated on the tile plus a 2-pixel border (the min-pool footprint;
//    border pixels outside the grid repeat the edge pixel, which is what the
//    edge-clamped 5x5 minimum reads) by sampling the frame's mean map
//    bilinearly at u + v/2 (corners clamped to the map), then the 5x5 minimum
//    in LDS.
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
#include "guide_maps.h"
#include "hmfsr_internal.h"
#include "noise.h"

namespace hmfsr {
namespace {

constexpr int RB_W = 32, RB_H = 32;              // output tile of R_hat (half-res px)
constexpr int RR_W = RB_W + 4, RR_H = RB_H + 4;  // robustness region incl. the min-pool border
constexpr int RR_N = RR_W * RR_H;
constexpr int TT_X = RR_W / 4 + 2, TT_Y = RR_H / 4 + 2;  // alignment tiles spanned (T >= 8)
constexpr int THREADS = 256;
constexpr int GM_W = 64, GM_H = 16;              // base-statistics tile (half-res px)
constexpr int GW_W = GM_W + 4, GW_H = GM_H + 4;  // its guide window: two rings, edge-replicated
constexpr int GW_N = GW_W * GW_H;

// Raw value at parity position pos (row-major in the 2x2 quad) from the quad's
// two 32-bit rows; pos is uniform, so this is a select and a shift.
__device__ __forceinline__ uint32_t quad_at(uint32_t top, uint32_t bot, int pos) {
  return ((pos & 2) ? bot : top) >> ((pos & 1) * 16) & 0xffffu;
}

__host__ __device__ __forceinline__ int robust_tiles_x_(const Geometry& g) { return (g.w + RB_W - 1) / RB_W; }
__host__ __device__ __forceinline__ int robust_tiles_y_(const Geometry& g) { return (g.h + RB_H - 1) / RB_H; }
__host__ __device__ __forceinline__ int means_tiles_x(const Geometry& g) { return (g.w + GM_W - 1) / GM_W; }
__host__ __device__ __forceinline__ int means_tiles_y(const Geometry& g) { return (g.h + GM_H - 1) / GM_H; }

// Row stride of the guide maps: column Q of row P at P * mu_stride + Q + 1,
// columns -1 and w repeating columns 0 and w - 1.
__device__ __forceinline__ int mu_stride(const Geometry& g) { return g.w + 2; }

// Raw buffer resource over `bytes` bytes from p (word 3 as for gfx9 raw
// buffers; bytes below 2^31).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t bytes_rsrc(const void* p, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, 0, (int)bytes, 0x00020000);
}

// One packed guide-map entry at byte offset off (one dwordx2 load).
__device__ __forceinline__ uint2 ld_entry(__amdgpu_buffer_rsrc_t r, int off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  return make_uint2(v[0], v[1]);
}

// Last burst b with first[b] <= i.
__device__ __forceinline__ int burst_of(const int* __restrict__ first, int n_bursts, int i) {
  int lo = 0, hi = n_bursts - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---- pass 1a: the aligned frames' guide means --------------------------------------
// One wave per 64 x 8 block of half-res pixels: lane l holds guide column
// strip * 64 + l, its neighbours come from the adjacent lanes and, for lanes
// 0 and 63, from one extra column load each; the wave walks down the rows
// keeping the last two row sums.
constexpr int FM_COLS = 64, FM_ROWS = 8, FM_WAVES = THREADS / 64;

__host__ __device__ __forceinline__ int fm_strips(const Geometry& g) { return (g.w + FM_COLS - 1) / FM_COLS; }
__host__ __device__ __forceinline__ int fm_bands(const Geometry& g) {
  return (g.h + FM_ROWS * FM_WAVES - 1) / (FM_ROWS * FM_WAVES);
}

// Guide of one quad (its two 32-bit rows) as integers: R, the sum of the two
// greens, B.
__device__ __forceinline__ void guide_sums_of(uint32_t top, uint32_t bot, const Geometry& g, uint32_t (&v)[3]) {
  v[0] = quad_at(top, bot, g.red_pos);
  v[1] = quad_at(top, bot, g.green_pos[0]) + quad_at(top, bot, g.green_pos[1]);
  v[2] = quad_at(top, bot, g.blue_pos);
}

// Guide pixel of one quad (its two 32-bit rows) in raw units: R, mean of the
// two greens, B.
__device__ __forceinline__ void guide_of(uint32_t top, uint32_t bot, const Geometry& g, float (&v)[3]) {
  v[0] = (float)quad_at(top, bot, g.red_pos);
  v[1] = (float)(quad_at(top, bot, g.green_pos[0]) + quad_at(top, bot, g.green_pos[1])) * 0.5f;
  v[2] = (float)quad_at(top, bot, g.blue_pos);
}

__device__ __forceinline__ void frame_means_block(const uint16_t* __restrict__ frames, const Geometry& g,
                                                  uint2* __restrict__ gmu, int n, int strip, int band) {
  const int lane = threadIdx.x & 63;
  const int P0 = band * FM_ROWS;
  if (P0 >= g.h) return;  // uniform per wave; no barrier follows
  const int J = strip * FM_COLS + lane, Jc = min(J, g.w - 1);
  const bool edge = lane == 0 || lane == 63;
  const int Jh = clampi(lane == 0 ? J - 1 : J + 1, 0, g.w - 1);  // the edge lanes' outer neighbour
  const uint16_t* f = frames + (size_t)n * g.H * g.W;
  const int ws = mu_stride(g);
  uint2* mu = gmu + (size_t)n * g.h * ws;
  // every row's quads first, so that the loads are all in flight together
  uint32_t top[FM_ROWS + 2], bot[FM_ROWS + 2], htop[FM_ROWS + 2], hbot[FM_ROWS + 2];
#pragma unroll
  for (int i = 0; i < FM_ROWS + 2; ++i) {
    const int I = clampi(P0 - 1 + i, 0, g.h - 1);
    top[i] = *(const uint32_t*)(f + (size_t)(2 * I) * g.W + 2 * Jc);
    bot[i] = *(const uint32_t*)(f + (size_t)(2 * I + 1) * g.W + 2 * Jc);
  }
  if (edge) {
#pragma unroll
    for (int i = 0; i < FM_ROWS + 2; ++i) {
      const int I = clampi(P0 - 1 + i, 0, g.h - 1);
      htop[i] = *(const uint32_t*)(f + (size_t)(2 * I) * g.W + 2 * Jh);
      hbot[i] = *(const uint32_t*)(f + (size_t)(2 * I + 1) * g.W + 2 * Jh);
    }
  }
  // 3x3 box sums, separable: Hs = g(Q-1) + g(Q) + g(Q+1), then
  // Hs(P-1) + Hs(P) + Hs(P+1), in integers
  uint32_t h0[3] = {0u, 0u, 0u}, h1[3] = {0u, 0u, 0u};
#pragma unroll
  for (int i = 0; i < FM_ROWS + 2; ++i) {
    uint32_t v[3], hv[3] = {0u, 0u, 0u};
    guide_sums_of(top[i], bot[i], g, v);
    if (edge) guide_sums_of(htop[i], hbot[i], g, hv);
    uint32_t hs[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const uint32_t up = __shfl_up(v[c], 1, 64), dn = __shfl_down(v[c], 1, 64);
      const uint32_t l = lane == 0 ? hv[c] : up, r = lane == 63 ? hv[c] : dn;
      hs[c] = l + v[c] + r;
    }
    const int P = P0 + i - 2;  // the row whose sums are complete
    if (i >= 2 && J < g.w && P < g.h) {
      uint2* row = mu + (size_t)P * ws + J + 1;
      const uint2 m = pack_guide_sums(h0[0] + h1[0] + hs[0], h0[1] + h1[1] + hs[1], h0[2] + h1[2] + hs[2]);
      row[0] = m;
      if (J == 0) row[-1] = m;        // column -1
      if (J == g.w - 1) row[1] = m;  // column w
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      h0[c] = h1[c];
      h1[c] = hs[c];
    }
  }
}

// Workgroup (band of FM_WAVES blocks of one strip, aligned frame), mapped by
// XCD so that neighbouring strips and bands, which share the edge columns and
// rows, meet in one L2.
__global__ __launch_bounds__(THREADS) void k_frame_means(const uint16_t* __restrict__ frames, Geometry g,
                                                         uint2* __restrict__ gmu) {
  const int n = (int)blockIdx.y < g.ref ? (int)blockIdx.y : (int)blockIdx.y + 1;
  const int ns = fm_strips(g), t = xcd_tile(blockIdx.x, ns * fm_bands(g));
  frame_means_block(frames, g, gmu, n, t % ns, (t / ns) * FM_WAVES + (threadIdx.x >> 6));
}

// Every (burst, aligned frame, strip, band) of a batch, one workgroup each;
// each XCD takes a contiguous run of the flat list (neighbours share an L2).
__global__ __launch_bounds__(THREADS) void k_frame_means_batch(const BurstArgs* __restrict__ bursts,
                                                               const int* __restrict__ first, int n_bursts,
                                                               int total) {
  const int i = xcd_tile(blockIdx.x, total), bi = burst_of(first, n_bursts, i);
  const BurstArgs& b = bursts[bi];
  const int ns = fm_strips(b.g), per = ns * fm_bands(b.g);
  const int k = i - first[bi], m = k / per, t = k - m * per;
  const int n = m < b.g.ref ? m : m + 1;
  frame_means_block(b.frames, b.g, b.gmu, n, t % ns, (t / ns) * FM_WAVES + (threadIdx.x >> 6));
}

// ---- pass 1b: the base frame's statistics ------------------------------------------
struct BaseSmem {
  float G[3][GW_N];  // guide at rows I0-2 .. I0+GM_H+1, columns J0-2 .., clamped to the grid
  float S[3][GW_N];  // doubled 3x3 box sums (S.3)
};

// One 64x16 tile (tile_x, tile_y): the base frame's 3x3 guide means into
// gmu[ref] and the reciprocal variance sum, with its S.3 sign, into gref.
__device__ __forceinline__ void base_stats_tile(const uint16_t* __restrict__ frames, const Geometry& g,
                                                const RobustConsts& rc, uint2* __restrict__ gmu,
                                                float* __restrict__ gref, int tile_x, int tile_y, BaseSmem& sm) {
  const int tid = threadIdx.x;
  const int I0 = tile_y * GM_H, J0 = tile_x * GM_W;
  const int gy0 = I0 - 2, gx0 = J0 - 2;
  const uint16_t* f = frames + (size_t)g.ref * g.H * g.W;
  {
    // every quad of the window loaded before the first store
    constexpr int GPT = (GW_N + THREADS - 1) / THREADS;
    const float ginv = 1.f / (float)GW_W;
    uint32_t top[GPT], bot[GPT];
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int k = min(tid + i * THREADS, GW_N - 1);
      const int r = split_row(k, ginv), c = k - r * GW_W;
      const int I = clampi(gy0 + r, 0, g.h - 1), J = clampi(gx0 + c, 0, g.w - 1);
      top[i] = *(const uint32_t*)(f + (size_t)(2 * I) * g.W + 2 * J);
      bot[i] = *(const uint32_t*)(f + (size_t)(2 * I + 1) * g.W + 2 * J);
    }
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int k = tid + i * THREADS;
      if (k >= GW_N) continue;
      float v[3];
      guide_of(top[i], bot[i], g, v);
      sm.G[0][k] = v[0];
      sm.G[1][k] = v[1];
      sm.G[2][k] = v[2];
    }
  }
  __syncthreads();
  const int oh = min(GM_H, g.h - I0), ow = min(GM_W, g.w - J0);
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
  // 3x3 mean and population variance of the guide, noise-corrected per
  // channel (eq. 6), the reciprocal of their sum (eq. 5)
  for (int k = tid; k < GM_H * GM_W; k += THREADS) {
    const int i = k >> 6, j = k & (GM_W - 1);  // GM_W == 64
    if (i >= oh || j >= ow) continue;
    const int P = I0 + i, Q = J0 + j;
    const int o = (i + 1) * GW_W + (j + 1);  // window position of (P - 1, Q - 1)
    float den = 0.f;
    float sum3[3];
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
      const float mu = __fmul_rn(s, 1.f / 9.f);  // the map's mean (guide_maps.h)
      float var_ms = 0.f;
#pragma unroll
      for (int q = 0; q < 9; ++q) var_ms = fmaf(v[q] - mu, v[q] - mu, var_ms);
      var_ms *= (1.f / 9.f);
      // noise model in raw units at the base brightness (the guide green is
      // the mean of two greens)
      float var_md, dmd2_unused;
      noise_md(rc, mu, c, var_md, dmd2_unused);
      sum3[c] = s;
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
    // the sums are exact floats: the guide values are integers and halves
    gmu[((size_t)g.ref * g.h + P) * mu_stride(g) + Q + 1] =
        pack_guide_sums((uint32_t)sum3[0], (uint32_t)(2.f * sum3[1]), (uint32_t)sum3[2]);
    gref[(size_t)P * g.w + Q] = inv;
  }
}

__global__ __launch_bounds__(THREADS) void k_base_stats(const uint16_t* __restrict__ frames, Geometry g,
                                                        RobustConsts rc, uint2* __restrict__ gmu,
                                                        float* __restrict__ gref) {
  __shared__ BaseSmem sm;
  const int tx_n = means_tiles_x(g), t = xcd_tile(blockIdx.x, tx_n * means_tiles_y(g));
  base_stats_tile(frames, g, rc, gmu, gref, t % tx_n, t / tx_n, sm);
}

// Every (burst, tile) of a batch, one workgroup each, in XCD-contiguous runs.
__global__ __launch_bounds__(THREADS) void k_base_stats_batch(const BurstArgs* __restrict__ bursts,
                                                              const int* __restrict__ first, int n_bursts,
                                                              int total) {
  __shared__ BaseSmem sm;
  const int i = xcd_tile(blockIdx.x, total), bi = burst_of(first, n_bursts, i);
  const BurstArgs& b = bursts[bi];
  const int tx_n = means_tiles_x(b.g), t = i - first[bi];
  base_stats_tile(b.frames, b.g, b.rc, b.gmu, b.gref, t % tx_n, t / tx_n, sm);
}

// ---- pass 2: robustness and its 5x5 minimum ---------------------------------------
constexpr int TT = TT_X * TT_Y;
constexpr int NF = 4;                               // aligned frames whose tile data are staged at once
constexpr int RTHREADS = 512;                          // robustness workgroup
constexpr int PP = (RR_N + RTHREADS - 1) / RTHREADS;  // region pixels per thread
constexpr int WCAP = 2048;  // guide-map window of one frame (per channel): every corner of the region
constexpr int WPT = (WCAP + RTHREADS - 1) / RTHREADS;  // window entries per thread
constexpr long long kRobustGroups = 3072;  // target workgroup count of one robustness launch

struct RobustSmem {
  float sW[3][WCAP];           // the frame's mean maps over the region's corners
  float sR[RR_N];
  float sTmp[RR_H * RB_W];
  int sTyR[RR_H], sTxR[RR_W];  // alignment tile of each region row / column
  int sRlo[TT_Y], sRhi[TT_Y], sClo[TT_X], sChi[TT_X];  // region rows / columns of each tile
  int4 sOF[NF][TT];            // per alignment tile: floor(v/2) (x, y) and the fractions' bits
  float sS[NF][TT];            // rejection strength of eq. (8)
  unsigned char sMov[NF][TT];  // the motion prior chose s1
  int sBox[NF][4];             // per frame: corner window x0, -x1, y0, -y1 (padded columns)
  int sItem;
};

// R_hat of one 32x32 half-res tile (tile_x, tile_y), aligned frames
// m_first .. m_first + m_count - 1 (m indexes the frames other than the base).
//
// Per frame, the mean-map rows and columns that hold any bilinear corner of
// the region are copied to LDS (row-contiguous loads) when they fit WCAP,
// and the corners read from there; otherwise (a strongly divergent motion
// field) each pixel reads its corners from the maps directly. The values,
// and so the results, are the same either way.
__device__ __forceinline__ void robust_tile(const float* __restrict__ motion, const float* __restrict__ s_tile,
                                            const unsigned char* __restrict__ mov, const Geometry& g,
                                            const RobustConsts& rc, const uint2* __restrict__ gmu,
                                            const float* __restrict__ gref, float* __restrict__ rmin,
                                            float* __restrict__ robust, int tile_x, int tile_y, int m_first,
                                            int m_count, RobustSmem& sm) {
  const int tid = threadIdx.x;
  const int I0 = tile_y * RB_H, J0 = tile_x * RB_W;
  const int ra0 = I0 - 2, ca0 = J0 - 2;  // region origin (may be outside the grid)
  const size_t plane = (size_t)g.h * g.w;
  const int ws = mu_stride(g);
  const size_t mplane = (size_t)g.h * ws;  // entries of one frame's guide map

  if (tid < RR_W) sm.sTxR[tid] = min(2 * clampi(ca0 + tid, 0, g.w - 1) / g.T, g.TX - 1);
  if (tid >= 64 && tid < 64 + RR_H) {
    const int r = tid - 64;
    sm.sTyR[r] = min(2 * clampi(ra0 + r, 0, g.h - 1) / g.T, g.TY - 1);
  }
  __syncthreads();
  const int txA = sm.sTxR[0], tyA = sm.sTyR[0];
  const int ntx = sm.sTxR[RR_W - 1] - txA + 1, nty = sm.sTyR[RR_H - 1] - tyA + 1, ntiles = ntx * nty;
  // first / last region column and row of every alignment tile
  if (tid < RR_W) {
    const int t = sm.sTxR[tid] - txA;
    if (tid == 0 || sm.sTxR[tid - 1] != sm.sTxR[tid]) sm.sClo[t] = tid;
    if (tid == RR_W - 1 || sm.sTxR[tid + 1] != sm.sTxR[tid]) sm.sChi[t] = tid;
  }
  if (tid >= 64 && tid < 64 + RR_H) {
    const int r = tid - 64, t = sm.sTyR[r] - tyA;
    if (r == 0 || sm.sTyR[r - 1] != sm.sTyR[r]) sm.sRlo[t] = r;
    if (r == RR_H - 1 || sm.sTyR[r + 1] != sm.sTyR[r]) sm.sRhi[t] = r;
  }

  // this thread's region pixels: position, alignment tile, and the base
  // frame's statistics, kept for every aligned frame
  int kt[PP], Ic[PP], Jc[PP];
  float mr[PP][3], dm[PP][3], gi[PP];
  {
    const float rinv = 1.f / (float)RR_W;
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      const int k = tid + q * RTHREADS;
      const int kk = k < RR_N ? k : RR_N - 1;
      const int rr = split_row(kk, rinv), cc = kk - rr * RR_W;
      kt[q] = (sm.sTyR[rr] - tyA) * ntx + (sm.sTxR[cc] - txA);
      Ic[q] = clampi(ra0 + rr, 0, g.h - 1);
      Jc[q] = clampi(ca0 + cc, 0, g.w - 1);
      gi[q] = gref[(size_t)Ic[q] * g.w + Jc[q]];
      guide_means(gmu[(size_t)g.ref * mplane + (size_t)Ic[q] * ws + Jc[q] + 1], mr[q]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float sig2_unused;
        noise_md(rc, mr[q][c], c, sig2_unused, dm[q][c]);  // d_md^2 at the base brightness
      }
    }
  }
  const float vlim = (float)(max(g.W, g.H) + 16);
  const int na = m_first + m_count;
  const int ow = min(RB_W, g.w - J0), oh = min(RB_H, g.h - I0);

  for (int m0 = m_first; m0 < na; m0 += NF) {
    const int nf = min(NF, na - m0);
    // Readers of the previous chunk's data all passed a barrier since.
    if (tid < NF * 4) (&sm.sBox[0][0])[tid] = 0x7fffffff;
    __syncthreads();
    // per alignment tile and frame: half the displacement (the bilinear base
    // corner of u + v/2 is u + floor(v/2), u integer, with the same fractions
    // for every pixel of the tile), the rejection strength, the prior's
    // choice, and the tile's corner window (monotonic in the pixel position)
    for (int k = tid; k < nf * ntiles; k += RTHREADS) {
      const int fl = k / ntiles, kk = k - fl * ntiles;
      const int m = m0 + fl, n = m < g.ref ? m : m + 1;
      const int ky = kk / ntx, kx = kk - ky * ntx;
      const size_t t = ((size_t)n * g.TY + tyA + ky) * g.TX + txA + kx;
      const float* p = motion + 2 * t;
      // clamping keeps non-finite or huge vectors finite and changes no result
      const float hx = fminf(fmaxf(p[0], -vlim), vlim) * 0.5f, hy = fminf(fmaxf(p[1], -vlim), vlim) * 0.5f;
      const float fhx = floorf(hx), fhy = floorf(hy);
      const int ox = (int)fhx, oy = (int)fhy;
      // the fractions are exact: v/2 has at most 24 significant bits
      sm.sOF[fl][kk] = make_int4(ox, oy, __float_as_int(hx - fhx), __float_as_int(hy - fhy));
      sm.sS[fl][kk] = s_tile[t];
      sm.sMov[fl][kk] = mov[t];
      const int x0 = clampi(clampi(ca0 + sm.sClo[kx], 0, g.w - 1) + ox, -1, g.w - 1) + 1;
      const int x1 = clampi(clampi(ca0 + sm.sChi[kx], 0, g.w - 1) + ox, -1, g.w - 1) + 2;
      const int y0 = clampi(clampi(ra0 + sm.sRlo[ky], 0, g.h - 1) + oy, 0, g.h - 1);
      const int y1 = clampi(clampi(ra0 + sm.sRhi[ky], 0, g.h - 1) + oy + 1, 0, g.h - 1);
      atomicMin(&sm.sBox[fl][0], x0);
      atomicMin(&sm.sBox[fl][1], -x1);
      atomicMin(&sm.sBox[fl][2], y0);
      atomicMin(&sm.sBox[fl][3], -y1);
    }
    __syncthreads();
    // copy chunk frame fl's corner window to LDS if it fits, running
    // `between` while its loads are in flight
    auto stage = [&](int fl, auto&& between) -> bool {
      const int m = m0 + fl, n = m < g.ref ? m : m + 1;
      const int X0 = sm.sBox[fl][0], Y0 = sm.sBox[fl][2];
      const int wx = -sm.sBox[fl][1] - X0 + 1, wy = -sm.sBox[fl][3] - Y0 + 1;
      if (wx * wy > WCAP) {  // uniform
        between();
        return false;
      }
      // the map's rows Y0 .. Y0 + wy - 1 (fewer than WCAP rows of at most
      // 16386 entries: below 2^31 bytes)
      const __amdgpu_buffer_rsrc_t q =
          bytes_rsrc(gmu + ((size_t)n * g.h + Y0) * ws, (size_t)wy * ws * sizeof(uint2));
      const float inv = 1.f / (float)wx;
      const int nw = wx * wy;
      // every load of the copy in flight before the first store
      uint2 v[WPT];
#pragma unroll
      for (int i = 0; i < WPT; ++i) {
        const int k = tid + i * RTHREADS;
        if (k >= nw) continue;
        const int r = split_row(k, inv);
        v[i] = ld_entry(q, (mul24(r, ws) + X0 + (k - mul24(r, wx))) * (int)sizeof(uint2));
      }
      between();
#pragma unroll
      for (int i = 0; i < WPT; ++i) {
        const int k = tid + i * RTHREADS;
        if (k >= nw) continue;
        float m[3];
        guide_means(v[i], m);
        sm.sW[0][k] = m[0];
        sm.sW[1][k] = m[1];
        sm.sW[2][k] = m[2];
      }
      return true;
    };
    bool staged = stage(0, [] {});
    __syncthreads();
    for (int fl = 0; fl < nf; ++fl) {
      const int m = m0 + fl, n = m < g.ref ? m : m + 1;
      const uint2* mun = gmu + (size_t)n * mplane;
      const int X0 = sm.sBox[fl][0], Y0 = sm.sBox[fl][2], wx = -sm.sBox[fl][1] - X0 + 1;
#pragma unroll
      for (int q = 0; q < PP; ++q) {
        const int k = tid + q * RTHREADS;
        if (k >= RR_N) continue;
        const int4 of = sm.sOF[fl][kt[q]];
        const float fx = __int_as_float(of.z), fy = __int_as_float(of.w);
        // the frame's mean map at u + v/2, corners clamped to the map: rows
        // clamped, and columns x0, x0 + 1 of the padded map with x0 clamped
        // to [-1, w - 1], which hold the clamped corner columns
        const int ya = clampi(Ic[q] + of.y, 0, g.h - 1), yb = clampi(Ic[q] + of.y + 1, 0, g.h - 1);
        const int x0 = clampi(Jc[q] + of.x, -1, g.w - 1) + 1;
        float mm[3][4];
        if (staged) {
          const int ia = mul24(ya - Y0, wx) + x0 - X0, ib = mul24(yb - Y0, wx) + x0 - X0;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            mm[c][0] = sm.sW[c][ia];
            mm[c][1] = sm.sW[c][ia + 1];
            mm[c][2] = sm.sW[c][ib];
            mm[c][3] = sm.sW[c][ib + 1];
          }
        } else {
          const uint2* ra = mun + (size_t)ya * ws + x0;
          const uint2* rb = mun + (size_t)yb * ws + x0;
          float e[4][3];
          guide_means(ra[0], e[0]);
          guide_means(ra[1], e[1]);
          guide_means(rb[0], e[2]);
          guide_means(rb[1], e[3]);
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < 4; ++k) mm[c][k] = e[k][c];
        }
        float num = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float m00 = mm[c][0], m01 = mm[c][1], m10 = mm[c][2], m11 = mm[c][3];
          const float top = fmaf(fx, m01 - m00, m00), bot = fmaf(fx, m11 - m10, m10);
          const float mu_al = fmaf(fy, bot - top, top);
          const float mu_ref = mr[q][c];
          const float dmd2 = dm[q][c];
          const float dms = mu_ref - mu_al;
          const float dms2 = dms * dms;
          // Wiener shrinkage of eq. (6): d = d_ms^3 / (d_ms^2 + d_md^2)
          const float dd = dms * dms2 * __builtin_amdgcn_rcpf(dms2 + dmd2);
          num = fmaf(dd, dd, num);
        }
        const int ktq = kt[q];
        const float R = sm.sS[fl][ktq] * __expf(-num * fabsf(gi[q])) - rc.t;  // eq. (5)
        sm.sR[k] = rc.hf > 0.0 && gi[q] < 0.f && sm.sMov[fl][ktq] ? 0.f : fminf(fmaxf(R, 0.f), 1.f);
      }
      __syncthreads();
      // eq. (9): 5x5 minimum, separable (the region repeats edge pixels);
      // its first pass runs while the next frame's window loads (the window
      // is free again)
      auto rows_min = [&] {
        for (int k = tid; k < RR_H * RB_W; k += RTHREADS) {
          const int r = k >> 5, j = k & 31;  // RB_W == 32
          const float* row = sm.sR + r * RR_W + j;
          sm.sTmp[k] = fminf(fminf(fminf(row[0], row[1]), fminf(row[2], row[3])), row[4]);
        }
      };
      if (fl + 1 < nf) staged = stage(fl + 1, rows_min);
      else rows_min();
      __syncthreads();
      for (int k = tid; k < RB_H * RB_W; k += RTHREADS) {
        const int i = k >> 5, j = k & 31;
        if (i >= oh || j >= ow) continue;
        const float* col = sm.sTmp + i * RB_W + j;
        const float mn = fminf(fminf(fminf(col[0], col[RB_W]), fminf(col[2 * RB_W], col[3 * RB_W])), col[4 * RB_W]);
        const int o = (I0 + i) * g.w + J0 + j;  // below 2^28
        rmin[(size_t)n * plane + o] = mn;
        if (robust) robust[(size_t)n * plane + o] = sm.sR[(i + 2) * RR_W + j + 2];
      }
      // the next frame writes sR (read above before the last barrier) and,
      // after its first barrier, sTmp
    }
  }
}

// Workgroup (tile, group of m_per aligned frames).
__global__ __launch_bounds__(RTHREADS, 6) void k_robust(const float* __restrict__ motion,
                                                    const float* __restrict__ s_tile,
                                                    const unsigned char* __restrict__ mov, Geometry g,
                                                    RobustConsts rc, const uint2* __restrict__ gmu,
                                                    const float* __restrict__ gref, float* __restrict__ rmin,
                                                    float* __restrict__ robust, int m_per) {
  __shared__ RobustSmem sm;
  const int tx_n = robust_tiles_x_(g), t = xcd_tile(blockIdx.x, tx_n * robust_tiles_y_(g));
  const int m_first = blockIdx.y * m_per;
  robust_tile(motion, s_tile, mov, g, rc, gmu, gref, rmin, robust, t % tx_n, t / tx_n, m_first,
              min(m_per, g.n - 1 - m_first), sm);
}

// Persistent form over (burst, tile) items of a batch (XCD-chunked queue).
__global__ __launch_bounds__(RTHREADS, 6) void k_robust_batch(const BurstArgs* __restrict__ bursts,
                                                          const WorkItem* __restrict__ items, ItemQueue q) {
  __shared__ RobustSmem sm;
  for_each_item(q, &sm.sItem, [&](int it) {
    const WorkItem w = items[it];
    const BurstArgs& b = bursts[w.burst];
    robust_tile(b.motion, b.s_tile, b.mov, b.g, b.rc, b.gmu, b.gref, b.rmin, nullptr,
                w.tile % b.robust_tiles_x, w.tile / b.robust_tiles_x, 0, b.g.n - 1, sm);
  });
}

}  // namespace

int robust_tiles_x(const Geometry& g) { return robust_tiles_x_(g); }
int robust_tiles_y(const Geometry& g) { return robust_tiles_y_(g); }
int base_stats_groups(const Geometry& g) { return g.n > 1 ? means_tiles_x(g) * means_tiles_y(g) : 0; }
int frame_means_groups(const Geometry& g) { return g.n > 1 ? (g.n - 1) * fm_strips(g) * fm_bands(g) : 0; }

hipError_t launch_robust(const Geometry& g, const RobustConsts& rc, const uint16_t* frames,
                         const float* motion, const Work& w, float* rmin, float* robust,
                         hipStream_t stream) {
  if (g.n < 2) return hipSuccess;
  hipLaunchKernelGGL(k_base_stats, dim3(means_tiles_x(g) * means_tiles_y(g)), dim3(THREADS), 0, stream, frames, g,
                     rc, w.gmu, w.gref);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_frame_means, dim3(fm_strips(g) * fm_bands(g), g.n - 1), dim3(THREADS), 0, stream, frames,
                     g, w.gmu);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  // Frames per workgroup: all of them (the base statistics are loaded once
  // per tile) unless that leaves fewer than ~kRobustGroups workgroups, about
  // four rounds of the resident workgroups of a 256-CU device; then as few
  // as that target needs.
  const int tiles = robust_tiles_x(g) * robust_tiles_y(g), na = g.n - 1;
  const long long work = (long long)tiles * na;
  int m_per = (int)((work + kRobustGroups - 1) / kRobustGroups);
  m_per = m_per < 1 ? 1 : (m_per > na ? na : m_per);
  const int groups = (na + m_per - 1) / m_per;
  hipLaunchKernelGGL(k_robust, dim3(tiles, groups), dim3(RTHREADS), 0, stream, motion, w.s_tile, w.mov, g, rc, w.gmu,
                     w.gref, rmin, robust, m_per);
  return hipGetLastError();
}

hipError_t launch_guide_stats_batch(const BurstArgs* bursts, const int* base_first, int base_total,
                                    const int* frame_first, int frame_total, int n_bursts, hipStream_t stream) {
  if (base_total > 0) {
    hipLaunchKernelGGL(k_base_stats_batch, dim3(base_total), dim3(THREADS), 0, stream, bursts, base_first,
                       n_bursts, base_total);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  if (frame_total > 0)
    hipLaunchKernelGGL(k_frame_means_batch, dim3(frame_total), dim3(THREADS), 0, stream, bursts, frame_first,
                       n_bursts, frame_total);
  return hipGetLastError();
}

int robust_batch_blocks_per_cu() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_robust_batch, RTHREADS, 0) != hipSuccess) return 1;
  return b > 0 ? b : 1;
}

hipError_t launch_robust_batch(const BurstArgs* bursts, const WorkItem* items, const int* bounds,
                               int* counters, int n_groups, hipStream_t stream) {
  hipLaunchKernelGGL(k_robust_batch, dim3(n_groups), dim3(RTHREADS), 0, stream, bursts, items,
                     ItemQueue{bounds, counters});
  return hipGetLastError();
}

}  // namespace hmfsr
