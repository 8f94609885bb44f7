// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hmfsr.h"
#include "omega.h"

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
  double scale;
};

// Motion prior thresholds (eq. 7-8).
struct PriorConsts {
  double m_th;
  float s1, s2;
};

// Robustness constants in raw units (eq. 5-6).
struct RobustConsts {
  float black;
  float a_r;  // noise_a * range: variance slope per raw unit of brightness
  float b_r;  // noise_b * range^2
  float t;
  double hf;    // S.3 variance-loss threshold; 0 turns the rejection off
  const float* ntab;  // Monte-Carlo noise table [nbins][4] (normalised units), or null
  int nbins;
  float inv_range;    // 1 / (white - black)
  float range2;       // (white - black)^2
};

// Accumulation constants.
struct MergeConsts {
  OmegaConsts om;
  float black, inv_range;
  int col4;  // colour of parity k in bits 2k..2k+1
};

// One burst of a batch, as the persistent kernels see it.
struct BurstArgs {
  const uint16_t* frames;
  const float* motion;
  float* out;
  float* s_tile;  // workspace [n][TY][TX]
  unsigned char* mov;  // workspace [n][TY][TX]
  float* rmin;    // workspace [n][h][w]
  uint2* gmu;     // workspace [n][h][w + 2]
  float* gref;    // workspace [h][w]
  Geometry g;
  MergeConsts mc;
  RobustConsts rc;
  PriorConsts pc;
  int merge_tiles_x;   // output tiles per row for the batch's tile shape
  int robust_tiles_x;  // robustness tiles per row
};

// A (burst, tile) unit of work of a persistent launch.
struct WorkItem {
  int burst;
  int tile;  // row-major tile index within the burst
};

// Workspace of the merge: per-(frame, tile) rejection strength, R_hat, and
// the robustness's guide statistics.
struct Work {
  float* s_tile;  // [n][TY][TX]
  unsigned char* mov;  // [n][TY][TX] 1 where the motion prior chose s1 (eq. 8)
  float* rmin;    // [n][h][w]
  uint2* gmu;     // [n][h][w + 2] 3x3 box sums of every frame's guide (raw units, packed as
                  // guide_maps.h states), a replicated edge column on either side (column
                  // Q at Q + 1)
  float* gref;    // [h][w] base frame: 1 / sum_c sigma_c^2 of eq. (5)-(6), negated where S.3 finds a loss
};
size_t work_bytes(const Geometry& g);
Work work_carve(void* base, const Geometry& g);

// Rejection strength into w.s_tile and the prior's choice into w.mov.
hipError_t launch_prior(const Geometry& g, const PriorConsts& pc, const float* motion, const Work& w,
                        hipStream_t stream);
// Guide statistics into w.gmu / w.gref, then R_hat into rmin (and R into
// robust, nullable); reads w.s_tile.
hipError_t launch_robust(const Geometry& g, const RobustConsts& rc, const uint16_t* frames,
                         const float* motion, const Work& w, float* rmin, float* robust,
                         hipStream_t stream);
// Compiled tile shapes of the merge kernel (64 columns x rows, threads).
struct MergeVariant {
  const char* name;
  int rows, threads;
};
extern const MergeVariant kMergeVariants[];
extern const int kNumMergeVariants;
// out and saved are each nullable. saved receives the normaliser of eq. (1),
// accumulated in float64 (the 64 x 16 tile shape is then used): three float64
// planes C per channel (raw units), then three float32 planes of the
// denominator and three of the reference exponent (12 4-byte words per pixel).
hipError_t launch_merge(int variant, const Geometry& g, const MergeConsts& mc, const uint16_t* frames,
                        const float* motion, const float* rmin, float* out, float* saved,
                        hipStream_t stream);
// Class of a burst in the batched merge: 2 x tile shape + 1 where the
// raw-footprint loads go in batches of eight (the burst's own launch's choice).
constexpr int kNumMergeClasses = 8;
int merge_class(int variant, double scale);
// `bounds` [XCDS + 1] and `counters` [XCDS] of the launch's item queue (see
// for_each_item).
hipError_t launch_merge_batch(int cls, const BurstArgs* bursts, const WorkItem* items, const int* bounds,
                              int* counters, int n_groups, hipStream_t stream);
hipError_t launch_robust_batch(const BurstArgs* bursts, const WorkItem* items, const int* bounds,
                               int* counters, int n_groups, hipStream_t stream);
// Guide statistics of every burst of a batch, the base frames' and the aligned
// frames' in two flat launches: workgroup i belongs to the last burst b with
// first[b] <= i (first[b] = the workgroups of the bursts before b).
hipError_t launch_guide_stats_batch(const BurstArgs* bursts, const int* base_first, int base_total,
                                    const int* frame_first, int frame_total, int n_bursts, hipStream_t stream);
int base_stats_groups(const Geometry& g);
int frame_means_groups(const Geometry& g);
hipError_t launch_prior_batch(const BurstArgs* bursts, const int* first, int n_bursts, int total,
                              hipStream_t stream);
int merge_tile_rows(int variant);
// Streaming merge (64 x 16 tiles): frames from loop index `first` on are added
// to the accumulator state [9][OH][OW] (numerator, denominator, reference
// exponent per channel); state_in nullable (empty accumulators).
hipError_t launch_merge_stream(const Geometry& g, const MergeConsts& mc, const uint16_t* frames,
                               const float* motion, const float* rmin, const float* state_in, float* state_out,
                               int first, hipStream_t stream);
hipError_t launch_stream_finish(const Geometry& g, const MergeConsts& mc, const float* state, float* out,
                                hipStream_t stream);
int merge_batch_blocks_per_cu(int cls);
int robust_batch_blocks_per_cu();
int robust_tiles_x(const Geometry& g);
int robust_tiles_y(const Geometry& g);
hipError_t launch_fill_i32(int* p, int v, size_t n, hipStream_t stream);
hipError_t launch_fill(float* p, float v, size_t n, hipStream_t stream);
hipError_t launch_omega_map(const Geometry& g, const OmegaConsts& oc, const uint16_t* frames,
                            double* omega, hipStream_t stream);

// ---- adjoint ---------------------------------------------------------------

// Output tile of the adjoint kernel: 64 x kBwdRows pixels.
constexpr int kBwdRows = 8;
constexpr int kBwdVT = (64 / 8 + 2) * (kBwdRows / 8 + 2);   // alignment tiles per output tile, max
constexpr int kBwdRH = (64 / 2 + 2) * (kBwdRows / 2 + 2);   // R_hat window cells per output tile, max

struct BwdConsts {
  double kd, kn, kst, ksh;  // k_detail, k_denoise, k_stretch, k_shrink
  double sl;                // dD/dD_tr per unit of sqrt(lambda1) of the integer tensor
  int tiles_x, tiles_y, n_tiles;  // output tiles of the adjoint's tile shape
};

// Workspace of the adjoint (on top of the forward's s_tile and R_hat maps).
struct BwdWork {
  Work fwd;
  float* rmap;        // [n][h][w] R of eq. (5)
  float* saved;       // [12][OH][OW] words: normaliser of eq. (1) when the caller keeps none
  float* part_rh;     // [n][tiles][kBwdRH] dL/dR_hat over each tile's R_hat window
  double* part_mo;    // [tiles][n][kBwdVT][2] dL/dv of the alignment tiles each tile touches
  double* part_theta; // [tiles][6] dL/d(k_detail, k_denoise, d_th, d_tr, k_stretch, k_shrink), unscaled
  double* part_rob;   // [n][TY][TX][5] robustness part: dL/dvx, dL/dvy, dL/dt, dL/ds, dL/ds_motion
  double* part_sum;   // [64][9] chunk sums of the tuning gradient
};
size_t bwd_bytes(const Geometry& g, bool need_saved);
BwdWork bwd_carve(void* base, const Geometry& g, bool need_saved);

hipError_t launch_merge_bwd(const Geometry& g, const MergeConsts& mc, const BwdConsts& bc,
                            const uint16_t* frames, const float* motion, const float* rmin,
                            const float* saved, const float* grad_out, const BwdWork& w,
                            hipStream_t stream);
hipError_t launch_robust_bwd(const Geometry& g, const RobustConsts& rc, const PriorConsts& pc,
                             const BwdConsts& bc, const uint16_t* frames, const float* motion,
                             const BwdWork& w, hipStream_t stream);
hipError_t launch_grad_reduce(const Geometry& g, const BwdConsts& bc, const BwdWork& w,
                              float* grad_tuning, float* grad_motion, hipStream_t stream);

// ---- tile alignment ----------------------------------------------------------

constexpr int kAlignMaxLevels = 6;
constexpr int kAlignCoarseBlock = 8;   // block edge on the levels above the finest

// Pyramid and block grids of one burst's alignment, resolved on the host.
struct AlignGeom {
  int n, ref, L;                       // frames, base frame, pyramid levels built
  int lh[kAlignMaxLevels], lw[kAlignMaxLevels];    // level sizes (level 0: half resolution)
  int blk[kAlignMaxLevels];                        // block edge per level (level 0: T / 2)
  int gby[kAlignMaxLevels], gbx[kAlignMaxLevels];  // block grid per level
  long long loff[kAlignMaxLevels];     // int32 offset of each level in one frame's pyramid
  long long fstride;                   // int32 words per frame pyramid
  long long voff[kAlignMaxLevels];     // int2 offset of each level's vectors in one frame's set
  long long vstride;                   // int2 vectors per frame
  int radius_coarse, radius_fine, lk_iterations;
  // noise gate: (12 kappa) kappa (0: off), then the noise model's a, b,
  // black level and raw range white - black, as float64 from float32
  double gate_k12, na, nb, black, rng;
};

// Workspace: pyramids [n][fstride] int32, then vectors [n][vstride] int2.
size_t align_bytes(const AlignGeom& ag);
hipError_t launch_align(const AlignGeom& ag, const uint16_t* frames, int H, int W, void* ws,
                        float* motion, int* block_match, hipStream_t stream);

// ---- noise model ----------------------------------------------------------------

// Monte-Carlo noise table into `table` [bins][4] (float32).
hipError_t launch_noise_table(double a, double b, double lo, int bins, int patches, unsigned long long seed,
                              float* table, hipStream_t stream);
// Sum of one frame's raw values into *sum (device, one 64-bit word); `parts`
// holds one word per workgroup of the first pass (at most kFrameSumGroups).
constexpr int kFrameSumGroups = 1024;
hipError_t launch_frame_sum(const uint16_t* frame, long long n, unsigned long long* parts,
                            unsigned long long* sum, hipStream_t stream);

}  // namespace hmfsr
