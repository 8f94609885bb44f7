// Tile geometry shared by the forward merge kernel and its adjoint, so that
// both take exactly the same discrete decisions (window centres, alignment
// tiles, R_hat windows) for the same output pixel.
#pragma once

#include <math.h>

#include "device_util.h"
#include "hmfsr_internal.h"

namespace hmfsr {

constexpr int MW = 64;  // output columns per tile = lanes per wave
// -log2(e) / 2: exponent of eq. (2) in base 2.
constexpr double NEG_HALF_LOG2E = -0.72134752044448170368;
// Distances given to out-of-frame sample columns / rows: their quadratic
// form is then ~1e200 or more (Omega^-1 is bounded below), i.e. weight 0.
constexpr double FAR_X = 1e100, FAR_Y = 1e120;
// The same in float exponent arithmetic: the quadratic form's coefficients
// stay within [1e-5, 1e7] in magnitude for any practical tuning, so the far
// terms land in [1e11, 1e38] and the cross term stays below 1e31.
constexpr float FAR_X32 = 1e8f, FAR_Y32 = 1e16f;

template <int MH>
struct Caps {
  // sized for scale 1 with up to ~8 px of displacement spread inside the tile
  // (the forward's tiles take 6 more rows and columns than the adjoint's
  // 64 x 8 tile, whose LDS must leave room for three workgroups per CU)
  static constexpr int PAD = MH >= 16 ? 6 : 0;
  static constexpr int RAW = (MW + 16 + PAD) * (MH + 16 + PAD);
  static constexpr int LUMA = (MW / 2 + 8 + PAD / 2) * (MH / 2 + 8 + PAD / 2);
  static constexpr int OM = (MW / 2 + 6 + PAD / 2) * (MH / 2 + 6 + PAD / 2);
  static constexpr int RH_W = MW / 2 + 2, RH_H = MH / 2 + 2;
  static constexpr int RH = RH_W * RH_H;
  static constexpr int TX = MW / 8 + 2, TY = MH / 8 + 2;  // alignment tiles (T >= 8)
  static constexpr int VT = TX * TY;
};

__device__ __forceinline__ int colour_of(int col4, int parity) { return (col4 >> (2 * parity)) & 3; }

struct RowInfo {
  int ya, yb;  // R_hat window row offsets (already multiplied by the window width)
  float fy;
};

// Footprint of a set of output pixels in one frame: ranges of the
// nine-sample window centres (jc, ic) and of the Omega bilinear corners (hj, hi).
struct Bounds {
  int jc0, jc1, ic0, ic1, hj0, hj1, hi0, hi1;
};

// Whether every sample of the nine-sample window centred at Bayer column jc,
// row ic lies outside the frame. Such a pixel gets no term from the frame
// (eq. 1 sums over in-frame samples only) and is skipped.
__host__ __device__ __forceinline__ bool samples_outside(int jc, int ic, const Geometry& g) {
  return jc < -1 || jc > g.W || ic < -1 || ic > g.H;
}

// Footprint of pixels displaced to [pxa, pxb] x [pya, pyb] (edge
// coordinates), limited to what the pixels that are not skipped can read:
// window centres in [-1, W] x [-1, H], Omega corners from [-1, w - 1] x
// [-1, h - 1] (the positions of such pixels lie in [-1, W + 1) x [-1, H + 1)).
// A displacement that throws pixels far outside the frame therefore widens
// no window beyond the frame and a ring of two samples.
__host__ __device__ __forceinline__ Bounds footprint(double pxa, double pxb, double pya, double pyb,
                                                     const Geometry& g) {
  Bounds b;
  b.jc0 = clampi((int)floor(pxa), -1, g.W);
  b.jc1 = clampi((int)floor(pxb), -1, g.W);
  b.ic0 = clampi((int)floor(pya), -1, g.H);
  b.ic1 = clampi((int)floor(pyb), -1, g.H);
  b.hj0 = clampi((int)floor(pxa * 0.5 - 0.5), -1, g.w - 1);
  b.hj1 = clampi((int)floor(pxb * 0.5 - 0.5), -1, g.w - 1);
  b.hi0 = clampi((int)floor(pya * 0.5 - 0.5), -1, g.h - 1);
  b.hi1 = clampi((int)floor(pyb * 0.5 - 0.5), -1, g.h - 1);
  return b;
}

// Footprint windows of a set of output pixels in one frame. Omega window:
// every bilinear corner, unclamped (edge values repeated); luma window: the
// clamped corners' 3x3 neighbourhoods, whose outer ring may lie one quad
// outside the grid and then repeats the edge quad (so Omega reads it without
// clamping); raw window: the quads inside the grid and every nine-sample
// window, unclamped (zero outside the frame). raw, lum, om: the window's
// offsets in the LDS buffers.
struct Win {
  int rc0, rr0, rw, rh;
  int lc0, lr0, lw, lh;
  int oc0, or0, ow, oh;
  int raw, lum, om;
};

__host__ __device__ __forceinline__ Win make_win(const Bounds& bd, const Geometry& g) {
  Win w;
  w.oc0 = bd.hj0;
  w.ow = bd.hj1 - bd.hj0 + 2;
  w.or0 = bd.hi0;
  w.oh = bd.hi1 - bd.hi0 + 2;
  w.lc0 = clampi(bd.hj0, 0, g.w - 1) - 1;
  const int lc1 = clampi(bd.hj1 + 1, 0, g.w - 1) + 1;
  w.lr0 = clampi(bd.hi0, 0, g.h - 1) - 1;
  const int lr1 = clampi(bd.hi1 + 1, 0, g.h - 1) + 1;
  w.rc0 = min(2 * max(w.lc0, 0), bd.jc0 - 1);
  const int rc1 = max(2 * min(lc1, g.w - 1) + 1, bd.jc1 + 1);
  w.rr0 = min(2 * max(w.lr0, 0), bd.ic0 - 1);
  const int rr1 = max(2 * min(lr1, g.h - 1) + 1, bd.ic1 + 1);
  w.lw = lc1 - w.lc0 + 1;
  w.lh = lr1 - w.lr0 + 1;
  w.rw = rc1 - w.rc0 + 1;
  w.rh = rr1 - w.rr0 + 1;
  w.raw = w.lum = w.om = 0;
  return w;
}

// Base-frame position of output column C (row R): (C + 1/2) / s.
__host__ __device__ __forceinline__ double out_pos(int C, double scale) { return ((double)C + 0.5) / scale; }

// Alignment tile column of base position X (row: same with T and TY).
__host__ __device__ __forceinline__ int tile_of(double X, int T, int nt) { return min((int)floor(X) / T, nt - 1); }

// Range [lo, hi] of base half-res indices whose R_hat values the output
// pixels c0..c1 (one axis) interpolate: the bilinear corners of X/2 - 1/2.
__host__ __device__ __forceinline__ void rh_range(int c0, int c1, double scale, int n_half, int& lo, int& hi) {
  lo = clampi((int)floor(out_pos(c0, scale) * 0.5 - 0.5), 0, n_half - 1);
  hi = clampi((int)floor(out_pos(c1, scale) * 0.5 - 0.5) + 1, 0, n_half - 1);
}

}  // namespace hmfsr
