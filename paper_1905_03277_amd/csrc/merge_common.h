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

// Base-frame position of output column C (row R): (C + 1/2) / s.
__device__ __forceinline__ double out_pos(int C, double scale) { return ((double)C + 0.5) / scale; }

// Alignment tile column of base position X (row: same with T and TY).
__device__ __forceinline__ int tile_of(double X, int T, int nt) { return min((int)floor(X) / T, nt - 1); }

// Range [lo, hi] of base half-res indices whose R_hat values the output
// pixels c0..c1 (one axis) interpolate: the bilinear corners of X/2 - 1/2.
__device__ __forceinline__ void rh_range(int c0, int c1, double scale, int n_half, int& lo, int& hi) {
  lo = clampi((int)floor(out_pos(c0, scale) * 0.5 - 0.5), 0, n_half - 1);
  hi = clampi((int)floor(out_pos(c1, scale) * 0.5 - 0.5) + 1, 0, n_half - 1);
}

}  // namespace hmfsr
