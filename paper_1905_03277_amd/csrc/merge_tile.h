// The fused output-tile merge body (Sec. 5.1, eq. 1-2 with the kernel
// covariance of Sec. 5.1.2 / S.1 and the robustness of Sec. 5.2), shared by
// the per-burst kernels (merge.hip) and the persistent batched kernels
// (merge_batch.hip), which live in translation units of their own so that
// neither's code generation depends on the other's instantiations.
//
// One workgroup owns a 64 x MH output tile: lane = column, wave w = a band of
// PX rows, so every thread keeps the per-channel accumulators of PX pixels in
// registers for the whole burst (the paper's online merge: memory does not
// grow with the frame count). For each frame, base frame first:
//   1. the frame's tile displacements and the tile's R_hat window are staged,
//      and the footprint of every alignment tile inside the output tile is
//      derived from its displacement and the tile's extreme pixel positions;
//   2. the raw Bayer footprint is copied to LDS (zero outside the frame), the
//      2x2-quad sums (luma) and the kernel covariance Omega (float64, edge
//      values repeated outside the grid) are computed over it;
//   3. every pixel interpolates Omega and R_hat bilinearly, inverts Omega in
//      float64, forms the nine exponents and accumulates exp2-weighted raw values per
//      channel against a per-channel reference exponent that is raised only
//      when a frame would exceed it by more than 2^64 (online normalisation).
// If a frame's footprint does not fit the LDS buffers (a strongly divergent
// motion field), every alignment tile of the output tile gets its own
// windows, laid out side by side in as few groups as the buffers allow.
#pragma once

#include <math.h>

#include <type_traits>

#include "device_util.h"
#include "hmfsr_internal.h"
#include "merge_common.h"
#include "omega.h"

namespace hmfsr {
namespace {

constexpr float SLACK = 64.f;   // log2 headroom above the reference exponent

template <int MH>
struct MergeSmem {
  using CP = Caps<MH>;
  double sX[MW], sY[MH];
  int sTyRow[MH], sTxCol[MW];
  int sRlo[CP::TY], sRhi[CP::TY], sClo[CP::TX], sChi[CP::TX];
  RowInfo sRow[MH];
  float2 sV[2][CP::VT];  // displacement per alignment tile, per frame slot (loop index & 1)
  Bounds sTB[CP::VT];
  float sRaw[CP::RAW];
  float sLum[CP::LUMA];
  double sOm[3][CP::OM];
  float sRh[CP::RH];
  int sRed[16];  // footprint reduction, two slots used by alternate frames
  int sRh0[4];
  Win sWin[CP::VT];    // per alignment tile, when the whole tile's window does not fit
  int sGrp[CP::VT + 1];  // groups of alignment tiles whose windows fit side by side
  int sNGrp;
  int sItem;
};

// What a tile keeps besides the output:
//   TILE_PLAIN   nothing;
//   TILE_SAVE    the normaliser of eq. (1), accumulated in float64, for the adjoint;
//   TILE_STREAM  the accumulators themselves, loaded from and stored to a
//                caller's state, so that frames can be added one call at a time.
enum { TILE_PLAIN = 0, TILE_SAVE = 1, TILE_STREAM = 2 };

// Accumulator state of a streaming merge: [9][OH][OW] floats, per channel the
// numerator and denominator of eq. (1) (raw units, scaled by 2^-m) and the
// reference exponent m; `first` is the first frame (loop index) to add.
struct StreamState {
  const float* in;  // nullable: start from empty accumulators
  float* out;
  int first;
};

// One 64 x MH output tile (tile_x, tile_y) of one burst. RB: raw-footprint
// loads per thread in flight at once (one batch for most windows when the
// window holds more than 4 x THREADS samples, see wide_raw_window).
template <int MH, int THREADS, int MODE, int RB>
__device__ __forceinline__ void merge_tile(const uint16_t* __restrict__ frames,
                                           const float* __restrict__ motion,
                                           const float* __restrict__ rmin, const Geometry& g,
                                           const MergeConsts& mc, float* __restrict__ out,
                                           float* __restrict__ saved, StreamState st, int tile_x,
                                           int tile_y, MergeSmem<MH>& sm) {
  constexpr bool SAVE = MODE == TILE_SAVE;
  constexpr int WAVES = THREADS / 64;
  constexpr int PX = MH / WAVES;
  static_assert(PX * WAVES == MH, "tile rows must split evenly over the waves");
  static_assert(Caps<MH>::VT <= THREADS, "one alignment tile per thread at most");
  using CP = Caps<MH>;
  double* sX = sm.sX;
  double* sY = sm.sY;
  int* sTyRow = sm.sTyRow;
  int* sTxCol = sm.sTxCol;
  int* sRlo = sm.sRlo;
  int* sRhi = sm.sRhi;
  int* sClo = sm.sClo;
  int* sChi = sm.sChi;
  RowInfo* sRow = sm.sRow;
  Bounds* sTB = sm.sTB;
  float* sRaw = sm.sRaw;
  float* sLum = sm.sLum;
  double(*sOm)[CP::OM] = sm.sOm;
  float* sRh = sm.sRh;
  int* sRed = sm.sRed;
  int* sRh0 = sm.sRh0;
  Win* sWin = sm.sWin;
  int* sGrp = sm.sGrp;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int C0 = tile_x * MW, R0 = tile_y * MH;
  const int ncol = min(MW, g.OW - C0), nrow = min(MH, g.OH - R0);

  // ---- per-tile geometry ------------------------------------------------
  const int C = C0 + lane;
  const bool col_ok = lane < ncol;
  const double X = out_pos(C, g.scale);  // base-frame position of the column
  if (tid < MW) {
    sX[tid] = X;
    sTxCol[tid] = col_ok ? min((int)floor(X) / g.T, g.TX - 1) : 0;
  }
  for (int r = tid; r < MH; r += THREADS) {
    const double Y = out_pos(R0 + r, g.scale);
    sY[r] = Y;
    sTyRow[r] = r < nrow ? min((int)floor(Y) / g.T, g.TY - 1) : 0;
  }
  __syncthreads();
  const int txA = sTxCol[0], txB = sTxCol[ncol - 1];
  const int tyA = sTyRow[0], tyB = sTyRow[nrow - 1];
  const int ntx = txB - txA + 1, nty = tyB - tyA + 1, ntiles = ntx * nty;
  // first / last pixel row and column of every alignment tile in the output tile
  if (tid < ncol) {
    const int t = sTxCol[tid] - txA;
    if (tid == 0 || sTxCol[tid - 1] != sTxCol[tid]) sClo[t] = tid;
    if (tid == ncol - 1 || sTxCol[tid + 1] != sTxCol[tid]) sChi[t] = tid;
  }
  for (int r = tid; r < nrow; r += THREADS) {
    const int t = sTyRow[r] - tyA;
    if (r == 0 || sTyRow[r - 1] != sTyRow[r]) sRlo[t] = r;
    if (r == nrow - 1 || sTyRow[r + 1] != sTyRow[r]) sRhi[t] = r;
  }
  // R_hat window on the base half-res grid: bilinear corners of X/2 - 1/2.
  if (tid == 0) {
    rh_range(C0, C0 + ncol - 1, g.scale, g.w, sRh0[0], sRh0[1]);
    rh_range(R0, R0 + nrow - 1, g.scale, g.h, sRh0[2], sRh0[3]);
  }
  if (tid < 16) sRed[tid] = 0x7fffffff;  // both footprint slots
  __syncthreads();
  const int rhc0 = sRh0[0], rhw = sRh0[1] - sRh0[0] + 1;
  const int rhr0 = sRh0[2], rhh = sRh0[3] - sRh0[2] + 1;
  for (int r = tid; r < MH; r += THREADS) {
    const double hy = sY[r] * 0.5 - 0.5;
    const double fhy = floor(hy);
    const int y0 = (int)fhy;
    RowInfo ri;
    ri.ya = (clampi(y0, 0, g.h - 1) - rhr0) * rhw;
    ri.yb = (clampi(y0 + 1, 0, g.h - 1) - rhr0) * rhw;
    ri.fy = (float)(hy - fhy);
    sRow[r] = ri;
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
  const int txl = sTxCol[lane] - txA;
  // displacements beyond this put every sample outside the frame
  const float vlim = (float)(max(g.W, g.H) + 16);

  // ---- accumulators -----------------------------------------------------
  using Acc = typename std::conditional<SAVE, double, float>::type;
  using EF = typename std::conditional<SAVE, double, float>::type;  // exponent arithmetic
  Acc num[PX][3], den[PX][3];
  float M[PX][3];
#pragma unroll
  for (int p = 0; p < PX; ++p)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      num[p][c] = 0;
      den[p][c] = 0;
      M[p][c] = -INFINITY;
    }
  if (MODE == TILE_STREAM && st.in && col_ok) {
    const size_t plane = (size_t)g.OH * g.OW;
#pragma unroll
    for (int p = 0; p < PX; ++p) {
      const int r = wave * PX + p;
      if (r >= nrow) continue;
      const size_t o = (size_t)(R0 + r) * g.OW + C;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        num[p][c] = st.in[o + c * plane];
        den[p][c] = st.in[o + (3 + c) * plane];
        M[p][c] = st.in[o + (6 + c) * plane];
      }
    }
  }

  // The R_hat window: every load in flight before its stores (entries past
  // the window re-read its last one and are not stored).
  constexpr int RHT = (CP::RH + THREADS - 1) / THREADS;
  auto rh_load = [&](int n, float (&rhv)[RHT]) {
    const float* rm = rmin + (size_t)n * g.h * g.w;
    const float inv = 1.f / (float)rhw;
    const int nrh = rhw * rhh;
#pragma unroll
    for (int i = 0; i < RHT; ++i) {
      const int k = min(tid + i * THREADS, nrh - 1);
      const int r = split_row(k, inv);
      rhv[i] = rm[(unsigned)((rhr0 + r) * g.w + rhc0 + k - mul24(r, rhw))];  // below 2^28
    }
  };
  auto rh_store = [&](const float (&rhv)[RHT]) {
#pragma unroll
    for (int i = 0; i < RHT; ++i)
      if (tid + i * THREADS < rhw * rhh) sRh[tid + i * THREADS] = rhv[i];
  };

  // No barrier opens a frame: what the previous frame's pixels read is either
  // per frame slot (sV, sRed) or written only after the footprint barrier
  // below, so waves that finish their pixels start the next frame's loads.
  for (int fi = MODE == TILE_STREAM ? st.first : 0; fi < g.n; ++fi) {
    const int n = fi == 0 ? g.ref : (fi <= g.ref ? fi - 1 : fi);
    const bool is_ref = n == g.ref;
    const uint16_t* f = frames + (size_t)n * g.H * g.W;
    // the footprint reduction alternates between two slots: this frame's was
    // reset during the previous frame, the next frame's is reset now (its
    // last reader, the previous frame's window, passed that frame's staging
    // barrier before any thread got here)
    int* red = sRed + 8 * (fi & 1);
    float2* sV = sm.sV[fi & 1];
    if (tid < 8) sRed[8 * ((fi + 1) & 1) + tid] = 0x7fffffff;
    // this thread's alignment tile (at most one: ntiles <= VT <= THREADS)
    const int ky = tid < ntiles ? tid / ntx : 0, kx = tid - ky * ntx;
    float2 v = make_float2(0.f, 0.f);
    if (tid < ntiles && !is_ref) {
      const float* p = motion + (((size_t)n * g.TY + tyA + ky) * g.TX + txA + kx) * 2;
      v = make_float2(p[0], p[1]);
    }
    // per alignment tile: its displacement and its footprint (positions are
    // monotonic in X and Y, so the tile's extreme pixels give its extreme
    // window centres)
    if (tid < ntiles) {
      const int k = tid;
      // clamping keeps non-finite or huge vectors finite and changes no result
      v = make_float2(fminf(fmaxf(v.x, -vlim), vlim), fminf(fmaxf(v.y, -vlim), vlim));
      sV[k] = v;
      const Bounds b = footprint(sX[sClo[kx]] + (double)v.x, sX[sChi[kx]] + (double)v.x,
                                 sY[sRlo[ky]] + (double)v.y, sY[sRhi[ky]] + (double)v.y, g);
      sTB[k] = b;
      atomicMin(&red[0], b.jc0); atomicMin(&red[1], -b.jc1);
      atomicMin(&red[2], b.ic0); atomicMin(&red[3], -b.ic1);
      atomicMin(&red[4], b.hj0); atomicMin(&red[5], -b.hj1);
      atomicMin(&red[6], b.hi0); atomicMin(&red[7], -b.hi1);
    }
    __syncthreads();

    // Windows: the whole tile's footprint in one window when it fits the
    // buffers; otherwise every alignment tile's own window, laid out side by
    // side in groups that fit (one alignment tile always does: its pixels
    // share one displacement, and its footprint stops at the frame's ring,
    // so its windows span at most its own pixels plus the rings; the caps
    // check of the test suite replays this arithmetic for extreme vectors).
    Win W;
    {
      Bounds bd;
      bd.jc0 = red[0]; bd.jc1 = -red[1]; bd.ic0 = red[2]; bd.ic1 = -red[3];
      bd.hj0 = red[4]; bd.hj1 = -red[5]; bd.hi0 = red[6]; bd.hi1 = -red[7];
      W = make_win(bd, g);
    }
    // uniform: every thread read the same bounds
    const bool whole = W.ow * W.oh <= CP::OM && W.lw * W.lh <= CP::LUMA && W.rw * W.rh <= CP::RAW;
    int ngroups = 1;
    if (!whole) {
      if (!is_ref) {
        float rhv[RHT];
        rh_load(n, rhv);
        rh_store(rhv);
      }
      for (int k = tid; k < ntiles; k += THREADS) sWin[k] = make_win(sTB[k], g);
      __syncthreads();
      if (tid == 0) {
        int ng = 0, n_raw = 0, n_lum = 0, n_om = 0;
        sGrp[0] = 0;
        for (int k = 0; k < ntiles; ++k) {
          Win& w = sWin[k];
          const int a_raw = w.rw * w.rh, a_lum = w.lw * w.lh, a_om = w.ow * w.oh;
          if (k > sGrp[ng] && (n_raw + a_raw > CP::RAW || n_lum + a_lum > CP::LUMA || n_om + a_om > CP::OM)) {
            sGrp[++ng] = k;
            n_raw = n_lum = n_om = 0;
          }
          w.raw = n_raw;
          w.lum = n_lum;
          w.om = n_om;
          n_raw += a_raw;
          n_lum += a_lum;
          n_om += a_om;
        }
        sGrp[++ng] = ntiles;
        sm.sNGrp = ng;
      }
      __syncthreads();
      ngroups = sm.sNGrp;
    }
    for (int gi = 0; gi < ngroups; ++gi) {
      if (gi) __syncthreads();  // the previous group's windows are no longer read
      const int s0 = whole ? 0 : sGrp[gi], s1 = whole ? 0 : sGrp[gi + 1];
      // window of flat buffer entry e of this group (kind: 0 raw, 1 luma, 2 Omega)
      auto find = [&](int e, int kind) -> int {
        int k = s0;
        while (k + 1 < s1 && (kind == 0 ? sWin[k + 1].raw : kind == 1 ? sWin[k + 1].lum : sWin[k + 1].om) <= e) ++k;
        return k;
      };
      auto entries = [&](int kind) -> int {
        if (whole) return kind == 0 ? W.rw * W.rh : kind == 1 ? W.lw * W.lh : W.ow * W.oh;
        const Win& w = sWin[s1 - 1];
        return kind == 0 ? w.raw + w.rw * w.rh : kind == 1 ? w.lum + w.lw * w.lh : w.om + w.ow * w.oh;
      };
      // stage raw footprint, quad sums, Omega
      if (whole) {
        // loads in batches of RB in flight before their stores: each reads
        // the clamped position and the zero outside the frame is chosen after
        const int rc0 = W.rc0, rr0 = W.rr0, rw = W.rw, nr = W.rw * W.rh;
        const float inv = 1.f / (float)rw;
        float rhv[RHT];  // the R_hat window's loads join the first batch
        if (!is_ref) rh_load(n, rhv);
        for (int k0 = tid; k0 < nr; k0 += RB * THREADS) {
          uint32_t rv[RB];
          bool rin[RB];
#pragma unroll
          for (int i = 0; i < RB; ++i) {
            // entries past the window read its last one (no branch, so the
            // loads stay in flight together) and are not stored
            const int k = min(k0 + i * THREADS, nr - 1);
            const int r = split_row(k, inv), c = k - mul24(r, rw);
            const int gr = rr0 + r, gc = rc0 + c;
            rin[i] = gr >= 0 && gr < g.H && gc >= 0 && gc < g.W;
            rv[i] = f[(unsigned)(clampi(gr, 0, g.H - 1) * g.W + clampi(gc, 0, g.W - 1))];  // below 2^30
          }
#pragma unroll
          for (int i = 0; i < RB; ++i) {
            const int k = k0 + i * THREADS;
            if (k < nr) sRaw[k] = rin[i] ? (float)rv[i] : 0.f;
          }
        }
        if (!is_ref) rh_store(rhv);
      } else {
        const int n_e = entries(0);
        constexpr int MB = 4;  // batches of branch-free loads, as above
        for (int e0 = tid; e0 < n_e; e0 += MB * THREADS) {
          uint32_t rv[MB];
          bool rin[MB];
#pragma unroll
          for (int i = 0; i < MB; ++i) {
            const int e = min(e0 + i * THREADS, n_e - 1);
            const Win& w = sWin[find(e, 0)];
            const int k = e - w.raw, r = k / w.rw, c = k - mul24(r, w.rw);
            const int gr = w.rr0 + r, gc = w.rc0 + c;
            rin[i] = gr >= 0 && gr < g.H && gc >= 0 && gc < g.W;
            rv[i] = f[(unsigned)(clampi(gr, 0, g.H - 1) * g.W + clampi(gc, 0, g.W - 1))];
          }
#pragma unroll
          for (int i = 0; i < MB; ++i) {
            const int e = e0 + i * THREADS;
            if (e < n_e) sRaw[e] = rin[i] ? (float)rv[i] : 0.f;
          }
        }
      }
      __syncthreads();
      if (whole) {
        const int rc0 = W.rc0, rr0 = W.rr0, rw = W.rw, lc0 = W.lc0, lr0 = W.lr0, lw = W.lw, lh = W.lh;
        const float inv = 1.f / (float)lw;
        for (int k = tid; k < lw * lh; k += THREADS) {
          const int r = split_row(k, inv), c = k - mul24(r, lw);
          const int o = mul24(2 * clampi(lr0 + r, 0, g.h - 1) - rr0, rw) + 2 * clampi(lc0 + c, 0, g.w - 1) - rc0;
          sLum[k] = (sRaw[o] + sRaw[o + 1]) + (sRaw[o + rw] + sRaw[o + rw + 1]);  // exact
        }
      } else {
        const int n_e = entries(1);
        for (int e = tid; e < n_e; e += THREADS) {
          const Win& w = sWin[find(e, 1)];
          const int k = e - w.lum, r = k / w.lw, c = k - mul24(r, w.lw);
          const int o = w.raw + mul24(2 * clampi(w.lr0 + r, 0, g.h - 1) - w.rr0, w.rw) +
                        2 * clampi(w.lc0 + c, 0, g.w - 1) - w.rc0;
          sLum[e] = (sRaw[o] + sRaw[o + 1]) + (sRaw[o + w.rw] + sRaw[o + w.rw + 1]);  // exact
        }
      }
      __syncthreads();
      {
        // Omega at entry (r, c) of window w, stored at flat entry e
        auto omega_at = [&](int e, const Win& w, int r, int c) {
          const int I = clampi(w.or0 + r, 0, g.h - 1), J = clampi(w.oc0 + c, 0, g.w - 1);
          // the window's outer ring repeats the edge quads: no clamps here
          const int base = w.lum + mul24(I - 1 - w.lr0, w.lw) + (J - 1 - w.lc0);
          float l[3][3];
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) l[a][bb] = sLum[base + a * w.lw + bb];
          double oxx, oxy, oyy;
          omega_from_quads(l, mc.om, oxx, oxy, oyy);
          sOm[0][e] = oxx;
          sOm[1][e] = oxy;
          sOm[2][e] = oyy;
        };
        if (whole) {
          const float inv = 1.f / (float)W.ow;
          for (int k = tid; k < W.ow * W.oh; k += THREADS) {
            const int r = split_row(k, inv);
            omega_at(k, W, r, k - mul24(r, W.ow));
          }
        } else {
          const int n_e = entries(2);
          for (int e = tid; e < n_e; e += THREADS) {
            const Win& w = sWin[find(e, 2)];
            const int k = e - w.om, r = k / w.ow;
            omega_at(e, w, r, k - mul24(r, w.ow));
          }
        }
      }
      __syncthreads();

      // accumulate: one pixel with its windows (uniform for the whole tile,
      // else its alignment tile's)
      auto pixel = [&](const int p, const int r, const int tyl, const Win& wg) __attribute__((always_inline)) {
            float rho = 1.f;
            if (!is_ref) {
              const RowInfo ri = sRow[r];
              const float top = sRh[ri.ya + rxa] + rfx * (sRh[ri.ya + rxb] - sRh[ri.ya + rxa]);
              const float bot = sRh[ri.yb + rxa] + rfx * (sRh[ri.yb + rxb] - sRh[ri.yb + rxa]);
              rho = top + ri.fy * (bot - top);
              if (!(rho > 0.f)) return;
            }
            const float2 v = sV[mul24(tyl, ntx) + txl];
            const double px = X + (double)v.x, py = sY[r] + (double)v.y;
            const double fjc = floor(px), fic = floor(py);
            const double frx = px - fjc, fry = py - fic;  // exact
            const int jc = (int)fjc, ic = (int)fic;
            if (samples_outside(jc, ic, g)) return;  // no in-frame sample: no term
            // Omega at p / 2 - 1/2 (bilinear; the window repeats edge values)
            const double hx = px * 0.5 - 0.5, hy = py * 0.5 - 0.5;
            const double fhj = floor(hx), fhi = floor(hy);
            const double fx = hx - fhj, fy = hy - fhi;
            const int ow = wg.ow;
            const int ob = wg.om + mul24((int)fhi - wg.or0, ow) + ((int)fhj - wg.oc0);
            double O[3];
  #pragma unroll
            for (int e = 0; e < 3; ++e) {
              const double o00 = sOm[e][ob], o01 = sOm[e][ob + 1];
              const double o10 = sOm[e][ob + ow], o11 = sOm[e][ob + ow + 1];
              const double top = fma(fx, o01 - o00, o00);
              const double bot = fma(fx, o11 - o10, o10);
              O[e] = fma(fy, bot - top, top);
            }
            // eq. (2): log2 w = -1/2 log2(e) d^T Omega^-1 d. Omega_bar, its
            // determinant and inverse in float64 (Omega is ill-conditioned,
            // k1/k2 up to ~10^3); the inverse's entries, the offsets and the
            // nine exponents then in EF: float where the normaliser is not
            // kept (the exponents' terms are products of well-scaled values,
            // so each exponent carries a float rounding of its largest term,
            // a relative weight error of ~10^-5 where it matters), float64 in
            // the forward that keeps its normaliser, whose weights the adjoint
            // recomputes in float64 and must reproduce.
            const double sc = NEG_HALF_LOG2E * recip64_1(O[0] * O[2] - O[1] * O[1]);
            const EF qa = (EF)(O[2] * sc), qb2 = (EF)(-2.0 * O[1] * sc), qc = (EF)(O[0] * sc);
            // sample offsets d = q + 1/2 - p; far away where the sample is
            // outside the frame (far enough that its weight is 0, near enough
            // that no product overflows: the row distance dominates)
            EF dx[3], dy[3];
            {
              const EF fx0 = (EF)frx, fy0 = (EF)fry;
  #pragma unroll
              for (int j = 0; j < 3; ++j) {
                dx[j] = ((EF)j - (EF)0.5) - fx0;
                dy[j] = ((EF)j - (EF)0.5) - fy0;
              }
            }
            if (!(jc >= 1 && jc <= g.W - 2 && ic >= 1 && ic <= g.H - 2)) {
  #pragma unroll
              for (int j = 0; j < 3; ++j) {
                const int qj = jc + j - 1, qi = ic + j - 1;
                if (qj < 0 || qj >= g.W) dx[j] = SAVE ? (EF)FAR_X : (EF)FAR_X32;
                if (qi < 0 || qi >= g.H) dy[j] = SAVE ? (EF)FAR_Y : (EF)FAR_Y32;
              }
            }
            // exponent of sample (i, j): ax[j] + cy[i] + by[i] dx[j]
            EF ax[3], cy[3], by[3];
  #pragma unroll
            for (int j = 0; j < 3; ++j) {
              ax[j] = qa * (dx[j] * dx[j]);
              cy[j] = qc * (dy[j] * dy[j]);
              by[j] = qb2 * dy[j];
            }
            auto E = [&](int i, int j) { return fma(by[i], dx[j], ax[j] + cy[i]); };
            // Colour groups of the 3x3 window: centre (0), left/right (1), up/down (2), corners (3).
            const int pr = ic & 1, pc = jc & 1;
            const int c0 = colour_of(mc.col4, pr * 2 + pc);
            const int c1 = colour_of(mc.col4, pr * 2 + (pc ^ 1));
            const bool isG = c0 == 1;
            const bool xIsR = (isG ? c1 : c0) == 0;  // group "X" (centre or left/right) is red
            float d[3][3];
            auto exponents = [&]() {
              const float MX = xIsR ? M[p][0] : M[p][2], MY = xIsR ? M[p][2] : M[p][0], MG = M[p][1];
              const EF g0 = (EF)(isG ? MG : MX), g1 = (EF)(isG ? MX : MG);
              const EF g2 = (EF)(isG ? MY : MG), g3 = (EF)(isG ? MG : MY);
              // the group's reference joins the row term
              const EF r1c = cy[1] - g0, r1s = cy[1] - g1;
              const EF r0m = cy[0] - g2, r0c = cy[0] - g3, r2m = cy[2] - g2, r2c = cy[2] - g3;
              d[1][1] = (float)fma(by[1], dx[1], ax[1] + r1c);
              d[1][0] = (float)fma(by[1], dx[0], ax[0] + r1s);
              d[1][2] = (float)fma(by[1], dx[2], ax[2] + r1s);
              d[0][1] = (float)fma(by[0], dx[1], ax[1] + r0m);
              d[2][1] = (float)fma(by[2], dx[1], ax[1] + r2m);
              d[0][0] = (float)fma(by[0], dx[0], ax[0] + r0c);
              d[0][2] = (float)fma(by[0], dx[2], ax[2] + r0c);
              d[2][0] = (float)fma(by[2], dx[0], ax[0] + r2c);
              d[2][2] = (float)fma(by[2], dx[2], ax[2] + r2c);
            };
            exponents();
            const float dmax = fmaxf(fmaxf(fmaxf(d[0][0], d[0][1]), fmaxf(d[0][2], d[1][0])),
                                     fmaxf(fmaxf(d[1][1], d[1][2]), fmaxf(fmaxf(d[2][0], d[2][1]), d[2][2])));
            if (dmax > SLACK) {
              // raise the reference of every channel this frame would overflow
              const float m0 = (float)E(1, 1);
              const float m1 = (float)fmax(E(1, 0), E(1, 2));
              const float m2 = (float)fmax(E(0, 1), E(2, 1));
              const float m3 = (float)fmax(fmax(E(0, 0), E(0, 2)), fmax(E(2, 0), E(2, 2)));
              const float fG = isG ? fmaxf(m0, m3) : fmaxf(m1, m2);
              const float fX = isG ? m1 : m0, fY = isG ? m2 : m3;
              const float fm[3] = {xIsR ? fX : fY, fG, xIsR ? fY : fX};
  #pragma unroll
              for (int c = 0; c < 3; ++c) {
                if (fm[c] > M[p][c] + SLACK) {
                  const float s = __builtin_amdgcn_exp2f(M[p][c] - fm[c]);
                  num[p][c] *= s;
                  den[p][c] *= s;
                  M[p][c] = fm[c];
                }
              }
              exponents();
            }
            const int rw = wg.rw;
            const int vb = wg.raw + mul24(ic - 1 - wg.rr0, rw) + (jc - 1 - wg.rc0);
            float w[3][3], val[3][3];
  #pragma unroll
            for (int i = 0; i < 3; ++i)
  #pragma unroll
              for (int j = 0; j < 3; ++j) {
                w[i][j] = __builtin_amdgcn_exp2f(d[i][j]);
                val[i][j] = sRaw[vb + i * rw + j];
              }
            const float S0n = w[1][1] * val[1][1], S0d = w[1][1];
            const float S1n = fmaf(w[1][0], val[1][0], w[1][2] * val[1][2]), S1d = w[1][0] + w[1][2];
            const float S2n = fmaf(w[0][1], val[0][1], w[2][1] * val[2][1]), S2d = w[0][1] + w[2][1];
            const float S3n = fmaf(w[0][0], val[0][0], w[0][2] * val[0][2]) +
                              fmaf(w[2][0], val[2][0], w[2][2] * val[2][2]);
            const float S3d = (w[0][0] + w[0][2]) + (w[2][0] + w[2][2]);
            const float Gn = isG ? S0n + S3n : S1n + S2n, Gd = isG ? S0d + S3d : S1d + S2d;
            const float Xn = isG ? S1n : S0n, Xd = isG ? S1d : S0d;
            const float Yn = isG ? S2n : S3n, Yd = isG ? S2d : S3d;
            const Acc ra = rho;
            num[p][0] = fma(ra, (Acc)(xIsR ? Xn : Yn), num[p][0]);
            den[p][0] = fma(ra, (Acc)(xIsR ? Xd : Yd), den[p][0]);
            num[p][1] = fma(ra, (Acc)Gn, num[p][1]);
            den[p][1] = fma(ra, (Acc)Gd, den[p][1]);
            num[p][2] = fma(ra, (Acc)(xIsR ? Yn : Xn), num[p][2]);
            den[p][2] = fma(ra, (Acc)(xIsR ? Yd : Xd), den[p][2]);
      };
      if (col_ok && whole) {
#pragma unroll
        for (int p = 0; p < PX; ++p) {
          const int r = wave * PX + p;
          if (r < nrow) pixel(p, r, sTyRow[r] - tyA, W);
        }
      } else if (col_ok) {
#pragma unroll
        for (int p = 0; p < PX; ++p) {
          const int r = wave * PX + p;
          if (r >= nrow) continue;
          const int tyl = sTyRow[r] - tyA, k = mul24(tyl, ntx) + txl;
          if (k < s0 || k >= s1) continue;
          pixel(p, r, tyl, sWin[k]);
        }
      }
    }
  }

  // eq. (1): normalise and map raw units to [0, 1]
  if (col_ok) {
    const size_t plane = (size_t)g.OH * g.OW;
#pragma unroll
    for (int p = 0; p < PX; ++p) {
      const int r = wave * PX + p;
      if (r >= nrow) continue;
      const size_t o = (size_t)(R0 + r) * g.OW + C;
      if (out) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
          out[o + c * plane] = (float)((num[p][c] / den[p][c] - (Acc)mc.black) * (Acc)mc.inv_range);
      }
      if (SAVE) {  // the normaliser of eq. (1), for the adjoint
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          ((double*)saved)[o + c * plane] = (double)(num[p][c] / den[p][c]);
          saved[o + (6 + c) * plane] = (float)den[p][c];
          saved[o + (9 + c) * plane] = M[p][c];
        }
      }
      if (MODE == TILE_STREAM && st.out) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          st.out[o + c * plane] = (float)num[p][c];
          st.out[o + (3 + c) * plane] = (float)den[p][c];
          st.out[o + (6 + c) * plane] = M[p][c];
        }
      }
    }
  }
}

// Minimum resident waves per SIMD (the second launch bound), i.e. the VGPR
// budget: 4 (128 VGPRs) when a thread keeps at most four pixel rows of
// accumulators, 2 (256) otherwise.
template <int MH, int THREADS>
constexpr int waves_per_simd() {
  return (MH / (THREADS / 64) <= 4) ? 4 : 2;
}

// Whether a 64 x MH tile's raw footprint (64/s + 8 by MH/s + 8 samples with
// its rings) exceeds four loads per thread: then the loads go in batches of
// eight, else of four (entries past the window still issue a load).
inline bool wide_raw_window(int MH, int THREADS, double scale) {
  return (64.0 / scale + 8.0) * (MH / scale + 8.0) > 4.0 * THREADS;
}

}  // namespace
}  // namespace hmfsr
