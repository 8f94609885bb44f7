// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hmfsr.h"

namespace hmfsr {

// Everything a kernel needs about one burst, resolved on the host.
struct Geometry {
  int n, H, W;      // frames, Bayer rows, Bayer columns
  int h, w;         // half-resolution rows, columns
  int ref;          // base frame
  int T, TY, TX;    // tile edge, tile rows, tile columns
  int OH, OW;       // output rows, columns
  int colour[4];    // colour (0 R, 1 G, 2 B) of Bayer parity (r & 1) * 2 + (c & 1)
  int green_pos[2]; // the two green parity indices, ascending
  int red_pos, blue_pos;
  double black, range;  // x = (raw - black) / range
  double scale;
  double noise_a, noise_b;
};

// Tuning in the precision each stage uses.
struct TuningD {
  double k_detail, k_denoise, d_th, d_tr, k_stretch, k_shrink;
  double s2, t, s1, m_th;
};

// Device-side intermediate maps of the materialised pipeline.
struct Maps {
  double* omega;   // [n][3][h][w]
  double* mu;      // [n][3][h][w] 3x3 guide mean
  double* sd;      // [n][3][h][w] 3x3 guide population sigma
  float* s_tile;   // [n][TY][TX]
  float* robust;   // [n][h][w]
  float* rmin;     // [n][h][w]
};

size_t maps_bytes(const Geometry& g);
Maps maps_carve(void* base, const Geometry& g);

// Enqueue the whole materialised pipeline (maps + accumulation) on `stream`.
hipError_t launch_maps(const Geometry& g, const TuningD& t, const uint16_t* frames,
                       const float* motion, const Maps& m, hipStream_t stream);
hipError_t launch_accumulate(const Geometry& g, const uint16_t* frames, const float* motion,
                             const Maps& m, float* out, hipStream_t stream);

}  // namespace hmfsr
