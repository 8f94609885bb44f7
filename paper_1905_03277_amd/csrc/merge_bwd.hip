// Adjoint of the merge: given dL/dC for the output C, the gradient of L with
// respect to the tuning scalars of the kernel covariance (Sec. 5.1.2, eq. 4,
// supplement S.1: k_detail, k_denoise, D_th, D_tr, k_stretch, k_shrink) and of
// the robustness (eq. 5 and 8: s, t, s_motion), and to the per-tile
// displacement of every aligned frame.
//
// Kernel weights are recomputed, never stored: the forward keeps only the
// normaliser of eq. (1) per output pixel and channel (the value C in float64,
// the denominator, the reference exponent). With w_i = exp(e_i - m) and
// den = sum rho_i w_i,
//   dC/drho_i = w_i (c_i - C) / den,   dC/de_i = rho_i w_i (c_i - C) / den,
// and e = -1/2 d^T Omega^-1 d with d = q + 1/2 - p gives
//   de/dp = Omega^-1 d,   de/dOmega = 1/2 Omega^-1 d d^T Omega^-1.
//
// k_merge_bwd   one workgroup per 64 x 8 output tile, staging each frame as
//               the forward does. Per pixel and frame it forms dL/de for the
//               nine samples and dL/drho, then
//               - dL/dp (offsets and the Omega sampling position), summed per
//                 alignment tile into per-workgroup partials;
//               - dL/dOmega_bar, contracted at the four bilinear corners with
//                 dOmega/dtheta, which the Omega staging keeps per half-res
//                 pixel in LDS, into six per-thread sums;
//               - dL/drho, transposed through the fixed R_hat bilinear weights
//                 onto the tile's R_hat window (per-workgroup partials).
//               Both sums over a row's pixels are segmented scans across the
//               wave's lanes (lane = output column; the alignment tile and the
//               R_hat corner columns of a lane are fixed runs), then sums over
//               the tile's rows through LDS.
// k_robust_bwd  one workgroup per (aligned frame, alignment tile): gathers
//               dL/dR_hat, hands it to the 5x5 argmin of eq. (9), then
//               through the clamp and exponential of eq. (5) and the
//               noise-corrected distance of eq. (6) to s or s_motion, t and
//               the tile's displacement (through the sampled colour mean).
// k_grad_*      add the partials up.
// Every sum runs in a fixed order, so two runs give identical bits.
#include <math.h>

#include "device_util.h"
#include "guide_maps.h"
#include "hmfsr_internal.h"
#include "noise.h"
#include "merge_common.h"
#include "omega.h"
#include "prior.h"

namespace hmfsr {
namespace {

constexpr int BMH = kBwdRows;
constexpr int BTHREADS = 256;
constexpr int BWAVES = BTHREADS / 64;
constexpr int BPX = BMH / BWAVES;  // pixel rows per thread
using BCP = Caps<BMH>;
static_assert(BCP::VT == kBwdVT && BCP::RH == kBwdRH, "partial layouts follow the tile caps");
static_assert(BCP::VT <= BTHREADS, "one alignment tile per thread at most");

struct BwdSmem {
  double sX[MW], sY[BMH];
  int sTyRow[BMH], sTxCol[MW];
  int sRlo[BCP::TY], sRhi[BCP::TY], sClo[BCP::TX], sChi[BCP::TX];
  RowInfo sRow[BMH];
  int sRya[BMH], sRyb[BMH];           // R_hat window rows of each pixel row
  int sRxa[MW], sRxb[MW];             // R_hat window columns of each pixel column
  float sRfx[MW];
  int sIlo[BCP::RH_H], sIhi[BCP::RH_H];  // pixel rows touching each window row
  float2 sV[BCP::VT];
  Bounds sTB[BCP::VT];
  float sRaw[BCP::RAW];
  float sLum[BCP::LUMA];
  double sOm[3][BCP::OM];
  // dOmega/dtheta per half-res pixel: the gradient direction as (cos 2phi,
  // sin 2phi) in float64 (the edge projection of dL/dOmega cancels up to
  // (k1/k2)^2), and the per-scalar factors p0..p9.
  double2 sDir[BCP::OM];
  float4 sP[2][BCP::OM];
  float2 sP2[BCP::OM];
  float sRh[BCP::RH];
  // per frame slot (frame index & 1): a frame's sums are added up during the next frame
  double2 sHm[2][BMH][BCP::TX];  // per pixel row and alignment tile column: sum of dL/dp
  float sHa[2][BMH][BCP::RH_W];  // per pixel row and R_hat column: dL/drho through the left corners
  float sHb[2][BMH][BCP::RH_W];  // ... through the right corners
  int sRun[MW];  // per lane: first lane of its runs (alignment tile, left and right R_hat corner column)
  double sAcc[BWAVES][6];
  int sRed[8];
  int sRh0[4];
};

// Per-channel values a[R, G, B] routed to the four colour groups of a 3x3
// window (centre, left/right, up/down, corners): green centres put green on
// the centre and corners, otherwise green sits left/right and up/down; the
// other two groups take red and blue as `xIsR` says. Selects only, so the
// routing never branches.
__device__ __forceinline__ void route4(const float (&a)[3], bool isG, bool xIsR, float (&o)[4]) {
  const float X = xIsR ? a[0] : a[2], Y = xIsR ? a[2] : a[0], G = a[1];
  o[0] = isG ? G : X;
  o[1] = isG ? X : G;
  o[2] = isG ? Y : G;
  o[3] = isG ? G : Y;
}

// One 32-bit lane move of a DPP control (gfx9 encodings: row_shr:n = 0x110 +
// n within rows of 16 lanes; row_bcast:15 = 0x142, lane 15 of each row to the
// next; row_bcast:31 = 0x143, lane 31 to rows 2 and 3). Rows outside
// row_mask, and lanes without a source, receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, ROWS, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, ROWS, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Inclusive sum of v over lanes [start, lane] (start <= lane: the first lane
// of this lane's run of equal keys): Hillis-Steele steps of 1, 2, 4 and 8
// lanes inside each row of 16, then the last lane of row 0 (and of row 2) to
// row 1 (row 3), then the last lane of row 1 to rows 2 and 3, each added only
// where the source lies in the lane's run. The run's last lane then holds
// the run's sum, with the same bits on every call.
template <typename T>
__device__ __forceinline__ T run_sum(T v, int lane, int start) {
  const int in_row = lane & 15, row0 = lane & ~15;
  T u = dpp_f<0x111, 0xF>(v);
  if (in_row >= 1 && lane - 1 >= start) v += u;
  u = dpp_f<0x112, 0xF>(v);
  if (in_row >= 2 && lane - 2 >= start) v += u;
  u = dpp_f<0x114, 0xF>(v);
  if (in_row >= 4 && lane - 4 >= start) v += u;
  u = dpp_f<0x118, 0xF>(v);
  if (in_row >= 8 && lane - 8 >= start) v += u;
  u = dpp_f<0x142, 0xA>(v);  // lanes 15 and 47 to rows 1 and 3
  if ((lane & 16) && row0 - 1 >= start) v += u;
  u = dpp_f<0x143, 0xC>(v);  // lane 31 to rows 2 and 3
  if (lane >= 32 && 31 >= start) v += u;
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;  // lane 0 holds the sum, always added in the same order
}

__global__ __launch_bounds__(BTHREADS, 3) void k_merge_bwd(
    const uint16_t* __restrict__ frames, const float* __restrict__ motion,
    const float* __restrict__ rmin, const float* __restrict__ saved,
    const float* __restrict__ grad_out, Geometry g, MergeConsts mc, BwdConsts bc,
    double* __restrict__ part_theta, double* __restrict__ part_mo, float* __restrict__ part_rh) {
  __shared__ BwdSmem sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tile = xcd_tile(blockIdx.x, bc.n_tiles);
  const int tile_x = tile % bc.tiles_x, tile_y = tile / bc.tiles_x;
  const int C0 = tile_x * MW, R0 = tile_y * BMH;
  const int ncol = min(MW, g.OW - C0), nrow = min(BMH, g.OH - R0);

  // ---- per-tile geometry (as the forward) -------------------------------
  const int C = C0 + lane;
  const bool col_ok = lane < ncol;
  const double X = out_pos(C, g.scale);
  if (tid < MW) {
    sm.sX[tid] = X;
    sm.sTxCol[tid] = col_ok ? tile_of(X, g.T, g.TX) : 0;
  }
  for (int r = tid; r < BMH; r += BTHREADS) {
    const double Y = out_pos(R0 + r, g.scale);
    sm.sY[r] = Y;
    sm.sTyRow[r] = r < nrow ? tile_of(Y, g.T, g.TY) : 0;
  }
  __syncthreads();
  const int txA = sm.sTxCol[0], txB = sm.sTxCol[ncol - 1];
  const int tyA = sm.sTyRow[0], tyB = sm.sTyRow[nrow - 1];
  const int ntx = txB - txA + 1, nty = tyB - tyA + 1, ntiles = ntx * nty;
  if (tid < ncol) {
    const int t = sm.sTxCol[tid] - txA;
    if (tid == 0 || sm.sTxCol[tid - 1] != sm.sTxCol[tid]) sm.sClo[t] = tid;
    if (tid == ncol - 1 || sm.sTxCol[tid + 1] != sm.sTxCol[tid]) sm.sChi[t] = tid;
  }
  for (int r = tid; r < nrow; r += BTHREADS) {
    const int t = sm.sTyRow[r] - tyA;
    if (r == 0 || sm.sTyRow[r - 1] != sm.sTyRow[r]) sm.sRlo[t] = r;
    if (r == nrow - 1 || sm.sTyRow[r + 1] != sm.sTyRow[r]) sm.sRhi[t] = r;
  }
  if (tid == 0) {
    rh_range(C0, C0 + ncol - 1, g.scale, g.w, sm.sRh0[0], sm.sRh0[1]);
    rh_range(R0, R0 + nrow - 1, g.scale, g.h, sm.sRh0[2], sm.sRh0[3]);
  }
  __syncthreads();
  const int rhc0 = sm.sRh0[0], rhw = sm.sRh0[1] - sm.sRh0[0] + 1;
  const int rhr0 = sm.sRh0[2], rhh = sm.sRh0[3] - sm.sRh0[2] + 1;
  for (int r = tid; r < BMH; r += BTHREADS) {
    const double hy = sm.sY[r] * 0.5 - 0.5;
    const double fhy = floor(hy);
    const int y0 = (int)fhy;
    const int ya = clampi(y0, 0, g.h - 1) - rhr0, yb = clampi(y0 + 1, 0, g.h - 1) - rhr0;
    RowInfo ri;
    ri.ya = ya * rhw;
    ri.yb = yb * rhw;
    ri.fy = (float)(hy - fhy);
    sm.sRow[r] = ri;
    sm.sRya[r] = ya;
    sm.sRyb[r] = yb;
  }
  int rxa, rxb;
  float rfx;
  {
    const double hx = X * 0.5 - 0.5;
    const double fhx = floor(hx);
    rxa = clampi((int)fhx, 0, g.w - 1) - rhc0;
    rxb = clampi((int)fhx + 1, 0, g.w - 1) - rhc0;
    rfx = (float)(hx - fhx);
  }
  if (tid < MW) {
    sm.sRxa[tid] = rxa;
    sm.sRxb[tid] = rxb;
    sm.sRfx[tid] = rfx;
  }
  __syncthreads();
  // pixel rows whose R_hat corners include window row I: the corners are
  // monotonic in the pixel position.
  if (tid >= 64 && tid < 64 + rhh) {
    const int I = tid - 64;
    int lo = nrow, hi = -1;
    for (int r = 0; r < nrow; ++r) {
      if (sm.sRya[r] <= I && I <= sm.sRyb[r]) {
        lo = min(lo, r);
        hi = r;
      }
    }
    sm.sIlo[I] = lo;
    sm.sIhi[I] = hi;
  }
  const int txl = sm.sTxCol[lane] - txA;
  const float vlim = (float)(max(g.W, g.H) + 16);
  // runs of lanes (output columns) sharing an alignment tile column, a left
  // and a right R_hat corner column: each lane's first lane of its run (bits
  // 0-6, 8-14, 16-22) and whether it is the run's last (bits 7, 15, 23);
  // columns past the tile are runs of their own and never the last of one
  if (tid < MW) {
    int run_t = lane, run_a = lane, run_b = lane;
    bool end_t = false, end_a = false, end_b = false;
    if (col_ok) {
      run_t = sm.sClo[txl];
      end_t = lane == sm.sChi[txl];
      while (run_a > 0 && sm.sRxa[run_a - 1] == rxa) --run_a;
      while (run_b > 0 && sm.sRxb[run_b - 1] == rxb) --run_b;
      end_a = lane == ncol - 1 || sm.sRxa[lane + 1] != rxa;
      end_b = lane == ncol - 1 || sm.sRxb[lane + 1] != rxb;
    }
    sm.sRun[lane] = run_t | (end_t << 7) | (run_a << 8) | (end_a << 15) | (run_b << 16) | (end_b << 23);
  }

  // ---- the forward's normaliser and dL/dC per pixel ----------------------
  // C is kept as a float pair (hi + lo): x - C is then accurate to a float
  // rounding even where x and C nearly cancel, which the tuning gradients need
  // (the weights of one channel sum their (x - C) terms to zero).
  float gam[BPX][3], chi[BPX][3], clo[BPX][3], mref[BPX][3];
  {
    const size_t plane = (size_t)g.OH * g.OW;
    const double* Cs = (const double*)saved;
#pragma unroll
    for (int p = 0; p < BPX; ++p) {
      const int r = wave * BPX + p;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        gam[p][c] = 0.f;
        chi[p][c] = 0.f;
        clo[p][c] = 0.f;
        mref[p][c] = 0.f;
      }
      if (!col_ok || r >= nrow) continue;
      const size_t o = (size_t)(R0 + r) * g.OW + C;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double cv = Cs[o + c * plane];  // raw units
        chi[p][c] = (float)cv;
        clo[p][c] = (float)(cv - (double)chi[p][c]);
        mref[p][c] = saved[o + (9 + c) * plane];
        // dL/dC_raw = dL/dC * inv_range, over the denominator of eq. (1)
        gam[p][c] = grad_out[o + c * plane] * mc.inv_range / saved[o + (6 + c) * plane];
      }
    }
  }
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};

  // Over the tile's pixel rows, in fixed order, the per-row sums a frame left
  // in slot `slot`: dL/dp per alignment tile and dL/drho onto the tile's R_hat
  // window, into frame m's per-workgroup partials. Runs after the barrier
  // that opens the next frame (or follows the last), beside that frame's
  // first loads.
  auto add_rows = [&](int slot, int m) {
    const int nwin = rhh * rhw;
    for (int k = tid; k < ntiles + nwin; k += BTHREADS) {
      if (k < ntiles) {
        const int ky = k / ntx, kx = k - ky * ntx;
        double sx = 0.0, sy = 0.0;
        for (int r = sm.sRlo[ky]; r <= sm.sRhi[ky]; ++r) {
          sx += sm.sHm[slot][r][kx].x;
          sy += sm.sHm[slot][r][kx].y;
        }
        double* dst = part_mo + (((size_t)tile * g.n + m) * kBwdVT + k) * 2;
        dst[0] = sx;
        dst[1] = sy;
      } else {
        const int q = k - ntiles;
        const int I = q / rhw, J = q - I * rhw;
        float s = 0.f;
        for (int r = sm.sIlo[I]; r <= sm.sIhi[I]; ++r) {
          const float fyr = sm.sRow[r].fy;
          const float wgt = (sm.sRya[r] == I ? 1.f - fyr : 0.f) + (sm.sRyb[r] == I ? fyr : 0.f);
          s = fmaf(wgt, sm.sHa[slot][r][J] + sm.sHb[slot][r][J], s);
        }
        part_rh[((size_t)m * bc.n_tiles + tile) * kBwdRH + q] = s;
      }
    }
  };
  auto frame_of = [&](int fi) { return fi == 0 ? g.ref : (fi <= g.ref ? fi - 1 : fi); };

  for (int fi = 0; fi < g.n; ++fi) {
    const int n = fi == 0 ? g.ref : (fi <= g.ref ? fi - 1 : fi);
    const bool is_ref = n == g.ref;
    const uint16_t* f = frames + (size_t)n * g.H * g.W;
    __syncthreads();
    // this thread's alignment tile (at most one: ntiles <= VT <= BTHREADS):
    // its displacement loads in flight together with the R_hat window's
    float2 v = make_float2(0.f, 0.f);
    if (tid < ntiles && !is_ref) {
      const int ky = tid / ntx;
      const float* p = motion + (((size_t)n * g.TY + tyA + ky) * g.TX + txA + (tid - ky * ntx)) * 2;
      v = make_float2(p[0], p[1]);
    }
    if (tid < 8) sm.sRed[tid] = 0x7fffffff;
    // every load of the R_hat window in flight before its stores (entries
    // past the window re-read its last one and are not stored); the previous
    // frame's row sums are added up while they are
    constexpr int RHT = (BCP::RH + BTHREADS - 1) / BTHREADS;
    const int nrh = rhw * rhh;
    float rhv[RHT];
    if (!is_ref) {
      const float* rm = rmin + (size_t)n * g.h * g.w;
      const float inv = 1.f / (float)rhw;
#pragma unroll
      for (int i = 0; i < RHT; ++i) {
        const int k = min(tid + i * BTHREADS, nrh - 1);
        const int r = split_row(k, inv);
        rhv[i] = rm[(unsigned)((rhr0 + r) * g.w + rhc0 + k - r * rhw)];  // below 2^28
      }
    }
    if (fi >= 2) add_rows((fi - 1) & 1, frame_of(fi - 1));  // frame 0 is the base frame: no sums
    if (!is_ref) {
#pragma unroll
      for (int i = 0; i < RHT; ++i)
        if (tid + i * BTHREADS < nrh) sm.sRh[tid + i * BTHREADS] = rhv[i];
    }
    // clamping keeps non-finite or huge vectors finite and changes no result
    if (tid < ntiles) sm.sV[tid] = make_float2(fminf(fmaxf(v.x, -vlim), vlim), fminf(fmaxf(v.y, -vlim), vlim));
    // this frame's dL/drho and dL/dp of the thread's pixels (0 where skipped)
    float pgr[BPX], pgx[BPX], pgy[BPX];
#pragma unroll
    for (int p = 0; p < BPX; ++p) pgr[p] = pgx[p] = pgy[p] = 0.f;
    __syncthreads();
    for (int k = tid; k < ntiles; k += BTHREADS) {
      const int ky = k / ntx, kx = k - ky * ntx;
      const float2 v = sm.sV[k];
      const Bounds b = footprint(sm.sX[sm.sClo[kx]] + (double)v.x, sm.sX[sm.sChi[kx]] + (double)v.x,
                                 sm.sY[sm.sRlo[ky]] + (double)v.y, sm.sY[sm.sRhi[ky]] + (double)v.y, g);
      sm.sTB[k] = b;
      atomicMin(&sm.sRed[0], b.jc0); atomicMin(&sm.sRed[1], -b.jc1);
      atomicMin(&sm.sRed[2], b.ic0); atomicMin(&sm.sRed[3], -b.ic1);
      atomicMin(&sm.sRed[4], b.hj0); atomicMin(&sm.sRed[5], -b.hj1);
      atomicMin(&sm.sRed[6], b.hi0); atomicMin(&sm.sRed[7], -b.hi1);
    }
    __syncthreads();

    bool whole = true;
    int seg = 0;
    while (true) {
      Bounds bd;
      if (whole) {
        bd.jc0 = sm.sRed[0]; bd.jc1 = -sm.sRed[1]; bd.ic0 = sm.sRed[2]; bd.ic1 = -sm.sRed[3];
        bd.hj0 = sm.sRed[4]; bd.hj1 = -sm.sRed[5]; bd.hi0 = sm.sRed[6]; bd.hi1 = -sm.sRed[7];
      } else {
        bd = sm.sTB[seg];
      }
      const int sty = whole ? -1 : seg / ntx, stx = whole ? -1 : seg % ntx;
      // the forward's windows (one alignment tile's always fit: its footprint
      // stops at the frame's ring)
      const Win wn = make_win(bd, g);
      const int oc0 = wn.oc0, ow = wn.ow, or0 = wn.or0, oh = wn.oh;
      const int lc0 = wn.lc0, lr0 = wn.lr0, lw = wn.lw, lh = wn.lh;
      const int rc0 = wn.rc0, rr0 = wn.rr0, rw = wn.rw, rh = wn.rh;
      if (whole && (ow * oh > BCP::OM || lw * lh > BCP::LUMA || rw * rh > BCP::RAW)) {
        whole = false;
        seg = 0;
        continue;
      }
      {
        // loads in batches of four in flight before their stores: each reads
        // the clamped position and the zero outside the frame is chosen after
        constexpr int RB = 4;
        const float inv = 1.f / (float)rw;
        const int nr = rw * rh;
        for (int k0 = tid; k0 < nr; k0 += RB * BTHREADS) {
          uint32_t rv[RB];
          bool rin[RB];
#pragma unroll
          for (int i = 0; i < RB; ++i) {
            const int k = min(k0 + i * BTHREADS, nr - 1);
            const int r = split_row(k, inv), c = k - r * rw;
            const int gr = rr0 + r, gc = rc0 + c;
            rin[i] = gr >= 0 && gr < g.H && gc >= 0 && gc < g.W;
            rv[i] = f[(unsigned)(clampi(gr, 0, g.H - 1) * g.W + clampi(gc, 0, g.W - 1))];  // below 2^30
          }
#pragma unroll
          for (int i = 0; i < RB; ++i) {
            const int k = k0 + i * BTHREADS;
            if (k < nr) sm.sRaw[k] = rin[i] ? (float)rv[i] : 0.f;
          }
        }
      }
      __syncthreads();
      {
        const float inv = 1.f / (float)lw;
        for (int k = tid; k < lw * lh; k += BTHREADS) {
          const int r = split_row(k, inv), c = k - r * lw;
          const int o = (2 * clampi(lr0 + r, 0, g.h - 1) - rr0) * rw + 2 * clampi(lc0 + c, 0, g.w - 1) - rc0;
          sm.sLum[k] = (sm.sRaw[o] + sm.sRaw[o + 1]) + (sm.sRaw[o + rw] + sm.sRaw[o + rw + 1]);
        }
      }
      __syncthreads();
      {
        const float inv = 1.f / (float)ow;
        for (int k = tid; k < ow * oh; k += BTHREADS) {
          const int r = split_row(k, inv), c = k - r * ow;
          const int I = clampi(or0 + r, 0, g.h - 1), J = clampi(oc0 + c, 0, g.w - 1);
          const int base = (I - 1 - lr0) * lw + (J - 1 - lc0);  // the window's ring repeats the edges
          float l[3][3];
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) l[a][bb] = sm.sLum[base + a * lw + bb];
          double oxx, oxy, oyy;
          OmegaParts pt;
          omega_parts_from_quads(l, mc.om, oxx, oxy, oyy, pt);
          sm.sOm[0][k] = oxx;
          sm.sOm[1][k] = oxy;
          sm.sOm[2][k] = oyy;
          // sigma_1,2 = k1s, k2s (k1 = sigma_1^2): per unit dL/dk1, dL/dk2 the
          // derivatives of sigma_1,2 in every scalar, each times 2 sigma.
          const double D = pt.D, A = pt.A, invA = pt.invA;
          const double s1 = 2.0 * pt.k1s, s2 = 2.0 * pt.k2s;
          const double f1 = pt.d_free ? s1 * (bc.kn - bc.kst * A) : 0.0;
          const double f2 = pt.d_free ? s2 * (bc.kn - invA / bc.ksh) : 0.0;
          const double sl = pt.sqrt_l1 * bc.sl;
          sm.sDir[k] = make_double2(pt.c2, pt.s2);
          sm.sP[0][k] = make_float4((float)(s1 * pt.k1s), (float)(s2 * pt.k2s), (float)(s1 * D), (float)(s2 * D));
          sm.sP[1][k] = make_float4((float)(s1 * (1.0 - D) * A), (float)(s2 * (1.0 - D) * invA), (float)f1,
                                    (float)f2);
          sm.sP2[k] = make_float2((float)(f1 * sl), (float)(f2 * sl));
        }
      }
      __syncthreads();

      if (col_ok) {
#pragma unroll
        for (int p = 0; p < BPX; ++p) {
          const int r = wave * BPX + p;
          if (r >= nrow) continue;
          const int tyl = sm.sTyRow[r] - tyA;
          if (!whole && (tyl != sty || txl != stx)) continue;
          float rho = 1.f;
          if (!is_ref) {
            const RowInfo ri = sm.sRow[r];
            const float top = sm.sRh[ri.ya + rxa] + rfx * (sm.sRh[ri.ya + rxb] - sm.sRh[ri.ya + rxa]);
            const float bot = sm.sRh[ri.yb + rxa] + rfx * (sm.sRh[ri.yb + rxb] - sm.sRh[ri.yb + rxa]);
            rho = top + ri.fy * (bot - top);
            if (!(rho > 0.f)) continue;
          }
          const float2 v = sm.sV[tyl * ntx + txl];
          const double px = X + (double)v.x, py = sm.sY[r] + (double)v.y;
          const double fjc = floor(px), fic = floor(py);
          const double frx = px - fjc, fry = py - fic;
          const int jc = (int)fjc, ic = (int)fic;
          if (samples_outside(jc, ic, g)) continue;  // no in-frame sample: no term, no gradient
          const double hx = px * 0.5 - 0.5, hy = py * 0.5 - 0.5;
          const double fhj = floor(hx), fhi = floor(hy);
          const double fx = hx - fhj, fy = hy - fhi;
          const int ob = ((int)fhi - or0) * ow + ((int)fhj - oc0);
          double O[3], dOx[3], dOy[3];  // Omega_bar and its derivatives along hx, hy
#pragma unroll
          for (int e = 0; e < 3; ++e) {
            const double o00 = sm.sOm[e][ob], o01 = sm.sOm[e][ob + 1];
            const double o10 = sm.sOm[e][ob + ow], o11 = sm.sOm[e][ob + ow + 1];
            const double top = fma(fx, o01 - o00, o00);
            const double bot = fma(fx, o11 - o10, o10);
            O[e] = fma(fy, bot - top, top);
            dOx[e] = fma(fy, (o11 - o10) - (o01 - o00), o01 - o00);
            dOy[e] = bot - top;
          }
          const double idet = recip64_1(O[0] * O[2] - O[1] * O[1]);
          const double sc = NEG_HALF_LOG2E * idet;
          const double qa = O[2] * sc, qb2 = -2.0 * O[1] * sc, qc = O[0] * sc;
          double dx[3], dy[3];
          float dxf[3], dyf[3];  // offsets of in-frame samples, 0 elsewhere
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            dx[j] = ((double)j - 0.5) - frx;
            dy[j] = ((double)j - 0.5) - fry;
            const int qj = jc + j - 1, qi = ic + j - 1;
            const bool okx = qj >= 0 && qj < g.W, oky = qi >= 0 && qi < g.H;
            dxf[j] = okx ? (float)dx[j] : 0.f;
            dyf[j] = oky ? (float)dy[j] : 0.f;
            if (!okx) dx[j] = FAR_X;
            if (!oky) dy[j] = FAR_Y;
          }
          double E[3][3];
          {
            double ax[3], cy[3], by[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              ax[j] = qa * (dx[j] * dx[j]);
              cy[j] = qc * (dy[j] * dy[j]);
              by[j] = qb2 * dy[j];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int j = 0; j < 3; ++j) E[i][j] = fma(by[i], dx[j], ax[j] + cy[i]);
          }
          // channel of each colour group: centre (0), left/right (1), up/down (2), corners (3)
          const int pr = ic & 1, pc = jc & 1;
          const int c0 = colour_of(mc.col4, pr * 2 + pc);
          const int c1 = colour_of(mc.col4, pr * 2 + (pc ^ 1));
          const bool isG = c0 == 1;
          const bool xIsR = (isG ? c1 : c0) == 0;  // group "X" (centre or left/right) is red
          float Mg[4], Gg[4], Ch[4], Cl[4];
          route4(mref[p], isG, xIsR, Mg);
          route4(gam[p], isG, xIsR, Gg);
          route4(chi[p], isG, xIsR, Ch);
          route4(clo[p], isG, xIsR, Cl);
          const int vb = (ic - 1 - rr0) * rw + (jc - 1 - rc0);
          float a[3][3];
          float grho = 0.f;
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              const int q = (i == 1 && j == 1) ? 0 : (i == 1 ? 1 : (j == 1 ? 2 : 3));
              const float w = __builtin_amdgcn_exp2f((float)(E[i][j] - (double)Mg[q]));
              const float bq = Gg[q] * w * ((sm.sRaw[vb + i * rw + j] - Ch[q]) - Cl[q]);  // dL/drho part
              grho += bq;
              a[i][j] = rho * bq;  // dL/de
            }
          // S = sum a d d^T, t = sum a d (offsets separate into columns and rows)
          float Acol[3], Arow[3], Sxy = 0.f;
#pragma unroll
          for (int j = 0; j < 3; ++j) Acol[j] = a[0][j] + a[1][j] + a[2][j];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            Arow[i] = a[i][0] + a[i][1] + a[i][2];
            Sxy = fmaf(dyf[i], fmaf(a[i][0], dxf[0], fmaf(a[i][1], dxf[1], a[i][2] * dxf[2])), Sxy);
          }
          float Sxx = 0.f, Syy = 0.f, tx = 0.f, ty = 0.f;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            tx = fmaf(Acol[j], dxf[j], tx);
            Sxx = fmaf(Acol[j] * dxf[j], dxf[j], Sxx);
            ty = fmaf(Arow[j], dyf[j], ty);
            Syy = fmaf(Arow[j] * dyf[j], dyf[j], Syy);
          }
          // dL/dOmega_bar = 1/2 Omega^-1 S Omega^-1 (Oxy on both off-diagonal
          // entries), in float64: its edge component is ~(k2/k1)^2 of its size.
          const double ia = O[2] * idet, ib = -O[1] * idet, ic_ = O[0] * idet;
          const double Sxx_d = Sxx, Sxy_d = Sxy, Syy_d = Syy;
          const double K11 = fma(ia, Sxx_d, ib * Sxy_d), K12 = fma(ia, Sxy_d, ib * Syy_d);
          const double K21 = fma(ib, Sxx_d, ic_ * Sxy_d), K22 = fma(ib, Sxy_d, ic_ * Syy_d);
          const double Gxx = 0.5 * fma(K11, ia, K12 * ib);
          const double Gxy = fma(K11, ib, K12 * ic_);
          const double Gyy = 0.5 * fma(K21, ib, K22 * ic_);
          // dL/dp: the offsets, and Omega sampled at p / 2 - 1/2
          const float gpx = (float)(fma(ia, (double)tx, ib * (double)ty) +
                                    0.5 * fma(Gxx, dOx[0], fma(Gxy, dOx[1], Gyy * dOx[2])));
          const float gpy = (float)(fma(ib, (double)tx, ic_ * (double)ty) +
                                    0.5 * fma(Gxx, dOy[0], fma(Gxy, dOy[1], Gyy * dOy[2])));
          // dL/dk1, dL/dk2 at each corner: projections of dL/dOmega on its edge and
          // gradient directions, 1/2 tr +- (cos 2phi U + sin 2phi V); then times dk/dtheta
          const double T = 0.5 * (Gxx + Gyy), U = 0.5 * (Gyy - Gxx), V = -0.5 * Gxy;
          const float ffx = (float)fx, ffy = (float)fy;
          const float wq[4] = {(1.f - ffx) * (1.f - ffy), ffx * (1.f - ffy), (1.f - ffx) * ffy, ffx * ffy};
          const int cq[4] = {ob, ob + 1, ob + ow, ob + ow + 1};
          float s6[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double2 dir = sm.sDir[cq[q]];
            const float4 P0 = sm.sP[0][cq[q]], P1 = sm.sP[1][cq[q]];
            const float2 P2 = sm.sP2[cq[q]];
            const double qq = fma(dir.x, U, dir.y * V);
            const float k1 = wq[q] * (float)(T + qq), k2 = wq[q] * (float)(T - qq);
            s6[0] = fmaf(k1, P0.x, fmaf(k2, P0.y, s6[0]));
            s6[1] = fmaf(k1, P0.z, fmaf(k2, P0.w, s6[1]));
            s6[2] = fmaf(k1, P1.z, fmaf(k2, P1.w, s6[2]));
            s6[3] = fmaf(k1, P2.x, fmaf(k2, P2.y, s6[3]));
            s6[4] = fmaf(k1, P1.x, s6[4]);
            s6[5] = fmaf(k2, P1.y, s6[5]);
          }
#pragma unroll
          for (int e = 0; e < 6; ++e) acc[e] += (double)s6[e];
          pgr[p] = grho;
          pgx[p] = gpx;
          pgy[p] = gpy;
        }
      }
      if (whole || ++seg >= ntiles) break;
      __syncthreads();
    }

    if (!is_ref) {
      // over each of this wave's pixel rows, in registers: dL/dp summed per
      // alignment tile column (both rows at once when they share a tile row)
      // and dL/drho summed per R_hat corner column
      const int r0 = wave * BPX;
      const int runs = sm.sRun[lane];
      const int run_t = runs & 127, run_a = (runs >> 8) & 127, run_b = (runs >> 16) & 127;
      const bool end_t = (runs >> 7) & 1, end_a = (runs >> 15) & 1, end_b = (runs >> 23) & 1;
      bool joined = false;
      if (BPX == 2) joined = r0 + 1 >= nrow || sm.sTyRow[r0] == sm.sTyRow[r0 + 1];  // uniform
#pragma unroll
      for (int p = 0; p < BPX; ++p) {
        const int r = r0 + p;
        if (r >= nrow) continue;  // uniform
        if (!(joined && p == 1)) {
          double sx = (double)pgx[p], sy = (double)pgy[p];
          if (joined && BPX == 2) {
            sx += (double)pgx[1];
            sy += (double)pgy[1];
          }
          sx = run_sum(sx, lane, run_t);
          sy = run_sum(sy, lane, run_t);
          if (end_t) {
            sm.sHm[fi & 1][r][txl] = make_double2(sx, sy);
            if (joined && BPX == 2 && r + 1 < nrow) sm.sHm[fi & 1][r + 1][txl] = make_double2(0.0, 0.0);
          }
        }
        if (lane < rhw) {
          sm.sHa[fi & 1][r][lane] = 0.f;
          sm.sHb[fi & 1][r][lane] = 0.f;
        }
        const float ga = run_sum((1.f - rfx) * pgr[p], lane, run_a);
        const float gb = run_sum(rfx * pgr[p], lane, run_b);
        if (end_a) sm.sHa[fi & 1][r][rxa] = ga;
        if (end_b) sm.sHb[fi & 1][r][rxb] = gb;
      }
    }
  }
  // the last frame's row sums (a burst of the base frame alone has none)
  __syncthreads();
  if (g.n >= 2) add_rows((g.n - 1) & 1, frame_of(g.n - 1));

  // ---- the six covariance-scalar sums of the workgroup ------------------
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const double v = wave_sum(acc[e]);
    if (lane == 0) sm.sAcc[wave][e] = v;
  }
  __syncthreads();
  if (tid < 6) {
    double s = 0.0;
    for (int w = 0; w < BWAVES; ++w) s += sm.sAcc[w][tid];
    part_theta[(size_t)tile * 6 + tid] = s;
  }
}

// ---------------------------------------------------------------------------
// robustness adjoint
// ---------------------------------------------------------------------------
constexpr int RB = 8;  // half-res pixels per block edge

// Output tiles whose R_hat window holds base half-res row I (column J with
// the column geometry): at most three, ascending. Returns how many; lo[k] is
// the first window row (column) of tile t[k] and wd[k] its width.
__device__ int rh_tiles(int I, int n_out, int edge, int n_tiles_axis, int n_half, double scale, int (&t)[3],
                        int (&lo)[3], int (&wd)[3]) {
  int cnt = 0;
  const int t0 = (int)((2.0 * I + 1.0) * scale / edge);
  for (int ot = max(t0 - 2, 0); ot <= min(t0 + 2, n_tiles_axis - 1) && cnt < 3; ++ot) {
    const int o0 = ot * edge, no = min(edge, n_out - o0);
    int a, b;
    rh_range(o0, o0 + no - 1, scale, n_half, a, b);
    if (I < a || I > b) continue;
    t[cnt] = ot;
    lo[cnt] = a;
    wd[cnt] = b - a + 1;
    ++cnt;
  }
  return cnt;
}
// The guide statistics are read from the forward's maps: the 3x3 sums of
// every frame (rows of w + 2 with a replicated edge column each side) and the
// base frame's 1 / sum sigma^2 (its sign carries the S.3 test, which the
// clamped R here already reflects), so the adjoint differentiates exactly the
// values the forward used.
__global__ __launch_bounds__(64, 4) void k_robust_bwd(const uint2* __restrict__ gmu,
                                                   const float* __restrict__ gref,
                                                   const float* __restrict__ motion,
                                                   const float* __restrict__ rmap,
                                                   const float* __restrict__ part_rh, Geometry g,
                                                   RobustConsts rc, PriorConsts pc, BwdConsts bc,
                                                   double* __restrict__ part_rob) {
  const int tx = blockIdx.x, ty = blockIdx.y, n = blockIdx.z;
  const int tid = threadIdx.x;
  double* dst = part_rob + (((size_t)n * g.TY + ty) * g.TX + tx) * 5;
  if (n == g.ref) {
    if (tid < 5) dst[tid] = 0.0;
    return;
  }
  __shared__ float sR[RB + 8][RB + 8];
  // per R row of the block's window and cell column: the minimum over the
  // cell's five columns and the offset (-2..2) of its first occurrence
  __shared__ float sHv[RB + 8][RB + 4];
  __shared__ int sHj[RB + 8][RB + 4];
  __shared__ float sG[RB + 4][RB + 4];
  __shared__ int sA[RB + 4][RB + 4];
  // output tiles whose R_hat windows cover each cell row / column of the block
  __shared__ int sNr[RB + 4], sTr[RB + 4][3], sLr[RB + 4][3];
  __shared__ int sNc[RB + 4], sTc[RB + 4][3], sLc[RB + 4][3], sWc[RB + 4][3];
  const size_t plane = (size_t)g.h * g.w;
  const float* R = rmap + (size_t)n * plane;
  const int ws = g.w + 2;
  const size_t mplane = (size_t)g.h * ws;
  const uint2* mref = gmu + (size_t)g.ref * mplane;
  const uint2* mfr = gmu + (size_t)n * mplane;
  const bool moving = prior_moving(motion, g, pc.m_th, n, ty, tx);
  const float s_used = moving ? pc.s1 : pc.s2;
  const float vlim = (float)(max(g.W, g.H) + 16);
  const float* pv = motion + (((size_t)n * g.TY + ty) * g.TX + tx) * 2;
  const float vx = fminf(fmaxf(pv[0], -vlim), vlim), vy = fminf(fmaxf(pv[1], -vlim), vlim);
  const int half = g.T / 2;
  const int i0 = ty * half, i1 = min(i0 + half, g.h), j0 = tx * half, j1 = min(j0 + half, g.w);
  double gvx = 0.0, gvy = 0.0, gt = 0.0, gs = 0.0;
  for (int bi0 = i0; bi0 < i1; bi0 += RB) {
    for (int bj0 = j0; bj0 < j1; bj0 += RB) {
      __syncthreads();
      for (int k = tid; k < (RB + 8) * (RB + 8); k += 64) {
        const int rr = k / (RB + 8), cc = k - rr * (RB + 8);
        sR[rr][cc] = R[(size_t)clampi(bi0 - 4 + rr, 0, g.h - 1) * g.w + clampi(bj0 - 4 + cc, 0, g.w - 1)];
      }
      if (tid < RB + 4) {
        int t[3], lo[3], wd[3];
        const int I = bi0 - 2 + tid;
        const int cnt = (I >= 0 && I < g.h) ? rh_tiles(I, g.OH, BMH, bc.tiles_y, g.h, g.scale, t, lo, wd) : 0;
        sNr[tid] = cnt;
        for (int k = 0; k < cnt; ++k) {
          sTr[tid][k] = t[k];
          sLr[tid][k] = lo[k];
        }
      } else if (tid >= 32 && tid < 32 + RB + 4) {
        int t[3], lo[3], wd[3];
        const int c = tid - 32, J = bj0 - 2 + c;
        const int cnt = (J >= 0 && J < g.w) ? rh_tiles(J, g.OW, MW, bc.tiles_x, g.w, g.scale, t, lo, wd) : 0;
        sNc[c] = cnt;
        for (int k = 0; k < cnt; ++k) {
          sTc[c][k] = t[k];
          sLc[c][k] = lo[k];
          sWc[c][k] = wd[k];
        }
      }
      __syncthreads();
      // dL/dR_hat of the cells whose 5x5 window can reach the block: the
      // window partials of every output tile holding the cell, in tile order.
      // Beside it, the first minimum of each window row over the cells' five
      // columns (row k of the R window holds image row clamp(bi0 - 4 + k)).
      for (int k = tid; k < (RB + 4) * (RB + 4); k += 64) {
        const int r2 = k / (RB + 4), c2 = k - r2 * (RB + 4);
        const int I = bi0 - 2 + r2, J = bj0 - 2 + c2;
        float gr = 0.f;
        for (int a = 0; a < sNr[r2]; ++a) {
          const float* row = part_rh + ((size_t)n * bc.n_tiles + sTr[r2][a] * bc.tiles_x) * kBwdRH;
          for (int b2 = 0; b2 < sNc[c2]; ++b2)
            gr += row[(size_t)sTc[c2][b2] * kBwdRH + (I - sLr[r2][a]) * sWc[c2][b2] + (J - sLc[c2][b2])];
        }
        sG[r2][c2] = gr;
      }
      for (int k = tid; k < (RB + 8) * (RB + 4); k += 64) {
        const int rr = k / (RB + 4), c2 = k - rr * (RB + 4);
        float best = INFINITY;
        int bj = 0;
#pragma unroll
        for (int dj = -2; dj <= 2; ++dj) {
          const float v = sR[rr][c2 + 2 + dj];
          if (v < best) {
            best = v;
            bj = dj;
          }
        }
        sHv[rr][c2] = best;
        sHj[rr][c2] = bj;
      }
      __syncthreads();
      // where each cell's dL/dR_hat goes: the first minimum of its window in
      // scan order (rows, then columns), i.e. the first row holding the
      // window's minimum and that row's first minimum. Clamped positions
      // repeat a border cell, so ties between them name the same cell.
      for (int k = tid; k < (RB + 4) * (RB + 4); k += 64) {
        const int r2 = k / (RB + 4), c2 = k - r2 * (RB + 4);
        int arg = -1;
        if (sG[r2][c2] != 0.f) {
          float best = INFINITY;
          int bi = 0;
#pragma unroll
          for (int di = -2; di <= 2; ++di) {
            const float v = sHv[r2 + 2 + di][c2];
            if (v < best) {
              best = v;
              bi = di;
            }
          }
          if (best < INFINITY) {
            const int I = bi0 - 2 + r2, J = bj0 - 2 + c2;
            arg = clampi(I + bi, 0, g.h - 1) * g.w + clampi(J + sHj[r2 + 2 + bi][c2], 0, g.w - 1);
          }
        }
        sA[r2][c2] = arg;
      }
      __syncthreads();
      const int i = bi0 + tid / RB, j = bj0 + tid % RB;
      if (i < i1 && j < j1) {
        float gR = 0.f;
        const int me = i * g.w + j;
        for (int di = -2; di <= 2; ++di)
          for (int dj = -2; dj <= 2; ++dj) {
            const int r2 = i + di - (bi0 - 2), c2 = j + dj - (bj0 - 2);
            if (sA[r2][c2] == me) gR += sG[r2][c2];
          }
        const float Rv = sR[i - bi0 + 4][j - bj0 + 4];
        if (gR != 0.f && Rv > 0.f && Rv < 1.f) {  // unclamped R of eq. (5)
          const float inv = fabsf(gref[(size_t)i * g.w + j]);  // 1 / sum_c sigma_c^2, eq. (5)
          float mu_ref[3], dmd2[3];
          guide_means(mref[(size_t)i * ws + j + 1], mu_ref);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            float sig2;
            noise_md(rc, mu_ref[c], c, sig2, dmd2[c]);
          }
          // mu_w: frame n's box mean sampled bilinearly at (j, i) + v / 2
          const double hx = (double)j + (double)vx * 0.5, hy = (double)i + (double)vy * 0.5;
          const double fhx = floor(hx), fhy = floor(hy);
          const float fx = (float)(hx - fhx), fy = (float)(hy - fhy);
          const int xa = clampi((int)fhx, 0, g.w - 1), xb = clampi((int)fhx + 1, 0, g.w - 1);
          const int ya = clampi((int)fhy, 0, g.h - 1), yb = clampi((int)fhy + 1, 0, g.h - 1);
          float top[3], bot[3], dtop[3], dbot[3];
          float ea[3], eb[3], ec[3], ed[3];
          guide_means(mfr[(size_t)ya * ws + xa + 1], ea);
          guide_means(mfr[(size_t)ya * ws + xb + 1], eb);
          guide_means(mfr[(size_t)yb * ws + xa + 1], ec);
          guide_means(mfr[(size_t)yb * ws + xb + 1], ed);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float ma = ea[c], mb = eb[c], mc = ec[c], md = ed[c];
            dtop[c] = mb - ma;
            top[c] = fmaf(fx, dtop[c], ma);
            dbot[c] = md - mc;
            bot[c] = fmaf(fx, dbot[c], mc);
          }
          float num = 0.f, dd[3], ddp[3], dmx[3], dmy[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float mu_w = fmaf(fy, bot[c] - top[c], top[c]);
            dmx[c] = fmaf(fy, dbot[c] - dtop[c], dtop[c]);
            dmy[c] = bot[c] - top[c];
            const float dms = mu_ref[c] - mu_w, dms2 = dms * dms;
            const float q = 1.f / (dms2 + dmd2[c]);
            dd[c] = dms * dms2 * q;  // eq. (6) shrinkage
            ddp[c] = dms2 * (dms2 + 3.f * dmd2[c]) * q * q;
            num = fmaf(dd[c], dd[c], num);
          }
          const float ex = __expf(-num * inv);
          gt -= (double)gR;
          gs += (double)(gR * ex);
          const float g_r = -gR * s_used * ex;
          float gx = 0.f, gy = 0.f;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            // r = inv * sum d^2; d_ms = mu_ref - mu_w; mu_w sampled at u + v / 2
            const float g_mu = -g_r * (2.f * dd[c] * inv) * ddp[c];
            gx = fmaf(g_mu, dmx[c], gx);
            gy = fmaf(g_mu, dmy[c], gy);
          }
          gvx += 0.5 * (double)gx;
          gvy += 0.5 * (double)gy;
        }
      }
    }
  }
  gvx = wave_sum(gvx);
  gvy = wave_sum(gvy);
  gt = wave_sum(gt);
  gs = wave_sum(gs);
  if (tid == 0) {
    dst[0] = gvx;
    dst[1] = gvy;
    dst[2] = gt;
    dst[3] = moving ? 0.0 : gs;
    dst[4] = moving ? gs : 0.0;
  }
}

// ---------------------------------------------------------------------------
// fixed-order reductions
// ---------------------------------------------------------------------------
// First output row (column) whose alignment tile index is >= t.
__device__ int first_out_with_tile(int t, int n_out, double scale, int T, int nt) {
  int lo = 0, hi = n_out;  // answer in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (tile_of(out_pos(mid, scale), T, nt) >= t) hi = mid; else lo = mid + 1;
  }
  return lo;
}

__global__ void k_grad_motion(const double* __restrict__ part_mo, const double* __restrict__ part_rob,
                              Geometry g, BwdConsts bc, float* __restrict__ grad_motion) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = g.TY * g.TX;
  if (idx >= g.n * per) return;
  const int n = idx / per, t = idx - n * per, ty = t / g.TX, tx = t - ty * g.TX;
  float* out = grad_motion + (size_t)idx * 2;
  if (n == g.ref) {
    out[0] = 0.f;
    out[1] = 0.f;
    return;
  }
  const int rlo = first_out_with_tile(ty, g.OH, g.scale, g.T, g.TY);
  const int rhi = first_out_with_tile(ty + 1, g.OH, g.scale, g.T, g.TY) - 1;
  const int clo = first_out_with_tile(tx, g.OW, g.scale, g.T, g.TX);
  const int chi = first_out_with_tile(tx + 1, g.OW, g.scale, g.T, g.TX) - 1;
  double sx = 0.0, sy = 0.0;
  if (rlo <= rhi && clo <= chi) {
    for (int oty = rlo / BMH; oty <= rhi / BMH; ++oty) {
      const int tyA = tile_of(out_pos(oty * BMH, g.scale), g.T, g.TY);
      for (int otx = clo / MW; otx <= chi / MW; ++otx) {
        const int C0 = otx * MW;
        const int txA = tile_of(out_pos(C0, g.scale), g.T, g.TX);
        const int txB = tile_of(out_pos(min(C0 + MW - 1, g.OW - 1), g.scale), g.T, g.TX);
        const int k = (ty - tyA) * (txB - txA + 1) + (tx - txA);
        const double* p = part_mo + (((size_t)(oty * bc.tiles_x + otx) * g.n + n) * kBwdVT + k) * 2;
        sx += p[0];
        sy += p[1];
      }
    }
  }
  const double* rob = part_rob + (size_t)idx * 5;
  out[0] = (float)(sx + rob[0]);
  out[1] = (float)(sy + rob[1]);
}

// Tuning-gradient sums in two fixed-order stages: workgroup b adds the
// contiguous chunk b of the per-tile and per-(frame, tile) partials, then one
// workgroup adds the chunk sums in order and applies the factors left out of
// the per-tile sums.
constexpr int kSumGroups = 64;

__global__ __launch_bounds__(256) void k_grad_tuning_part(const double* __restrict__ part_theta, int n_tiles,
                                                          const double* __restrict__ part_rob, int n_rob,
                                                          double* __restrict__ part_sum) {
  __shared__ double sS[4][9];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, b = blockIdx.x;
  const int ct = (n_tiles + kSumGroups - 1) / kSumGroups, cr = (n_rob + kSumGroups - 1) / kSumGroups;
  const int t0 = b * ct, t1 = min(n_tiles, t0 + ct), r0 = b * cr, r1 = min(n_rob, r0 + cr);
  double a[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) a[e] = 0.0;
  for (int t = t0 + tid; t < t1; t += 256)
#pragma unroll
    for (int e = 0; e < 6; ++e) a[e] += part_theta[(size_t)t * 6 + e];
  for (int t = r0 + tid; t < r1; t += 256) {
    const double* r = part_rob + (size_t)t * 5;
    a[6] += r[3];
    a[7] += r[2];
    a[8] += r[4];
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    const double v = wave_sum(a[e]);
    if (lane == 0) sS[wave][e] = v;
  }
  __syncthreads();
  if (tid < 9) part_sum[b * 9 + tid] = ((sS[0][tid] + sS[1][tid]) + sS[2][tid]) + sS[3][tid];
}

__global__ __launch_bounds__(64) void k_grad_tuning(const double* __restrict__ part_sum, BwdConsts bc,
                                                    float* __restrict__ grad_tuning) {
  const int e = threadIdx.x;
  if (e >= 9) return;
  double s = 0.0;
  for (int b = 0; b < kSumGroups; ++b) s += part_sum[b * 9 + e];
  // sigma_1,2 are proportional to k_detail; the other factors were left out of the sums
  double g = s;
  if (e == 0) g = s / bc.kd;
  else if (e <= 4) g = s * bc.kd;
  else if (e == 5) g = -s * bc.kd / (bc.ksh * bc.ksh);
  grad_tuning[e] = (float)g;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

size_t bwd_bytes(const Geometry& g, bool need_saved) {
  const size_t tiles = (size_t)((g.OW + MW - 1) / MW) * ((g.OH + BMH - 1) / BMH);
  const size_t plane = (size_t)g.h * g.w;
  size_t b = align256(work_bytes(g));
  b += align256(plane * g.n * sizeof(float));
  if (need_saved) b += align256((size_t)12 * g.OH * g.OW * sizeof(float));
  b += align256((size_t)g.n * tiles * kBwdRH * sizeof(float));
  b += align256(tiles * g.n * kBwdVT * 2 * sizeof(double));
  b += align256(tiles * 6 * sizeof(double));
  b += align256((size_t)g.n * g.TY * g.TX * 5 * sizeof(double));
  b += align256((size_t)kSumGroups * 9 * sizeof(double));
  return b;
}

BwdWork bwd_carve(void* base, const Geometry& g, bool need_saved) {
  const size_t tiles = (size_t)((g.OW + MW - 1) / MW) * ((g.OH + BMH - 1) / BMH);
  const size_t plane = (size_t)g.h * g.w;
  char* p = (char*)base;
  BwdWork w;
  w.fwd = work_carve(p, g);
  p += align256(work_bytes(g));
  w.rmap = (float*)p;
  p += align256(plane * g.n * sizeof(float));
  w.saved = nullptr;
  if (need_saved) {
    w.saved = (float*)p;
    p += align256((size_t)12 * g.OH * g.OW * sizeof(float));
  }
  w.part_rh = (float*)p;
  p += align256((size_t)g.n * tiles * kBwdRH * sizeof(float));
  w.part_mo = (double*)p;
  p += align256(tiles * g.n * kBwdVT * 2 * sizeof(double));
  w.part_theta = (double*)p;
  p += align256(tiles * 6 * sizeof(double));
  w.part_rob = (double*)p;
  p += align256((size_t)g.n * g.TY * g.TX * 5 * sizeof(double));
  w.part_sum = (double*)p;
  return w;
}

hipError_t launch_merge_bwd(const Geometry& g, const MergeConsts& mc, const BwdConsts& bc,
                            const uint16_t* frames, const float* motion, const float* rmin,
                            const float* saved, const float* grad_out, const BwdWork& w,
                            hipStream_t stream) {
  const dim3 grid(bc.n_tiles);
  hipLaunchKernelGGL(k_merge_bwd, grid, dim3(BTHREADS), 0, stream, frames, motion, rmin, saved, grad_out,
                     g, mc, bc, w.part_theta, w.part_mo, w.part_rh);
  return hipGetLastError();
}

hipError_t launch_robust_bwd(const Geometry& g, const RobustConsts& rc, const PriorConsts& pc,
                             const BwdConsts& bc, const uint16_t* frames, const float* motion,
                             const BwdWork& w, hipStream_t stream) {
  const dim3 grid(g.TX, g.TY, g.n);
  (void)frames;
  hipLaunchKernelGGL(k_robust_bwd, grid, dim3(64), 0, stream, w.fwd.gmu, w.fwd.gref, motion, w.rmap, w.part_rh, g,
                     rc, pc, bc, w.part_rob);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const Geometry& g, const BwdConsts& bc, const BwdWork& w,
                              float* grad_tuning, float* grad_motion, hipStream_t stream) {
  const int total = g.n * g.TY * g.TX;
  hipLaunchKernelGGL(k_grad_motion, dim3((total + 255) / 256), dim3(256), 0, stream, w.part_mo, w.part_rob,
                     g, bc, grad_motion);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_tuning_part, dim3(kSumGroups), dim3(256), 0, stream, w.part_theta, bc.n_tiles,
                     w.part_rob, total, w.part_sum);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_tuning, dim3(1), dim3(64), 0, stream, w.part_sum, bc, grad_tuning);
  return hipGetLastError();
}

}  // namespace hmfsr
