/*
 * hmfsr.h -- C ABI of libhmfsr, the MI355X (gfx950) kernel-regression burst
 * merge of Wronski et al., "Handheld Multi-Frame Super-Resolution",
 * ACM TOG 38(4), 2019.
 *
 * The merge (the paper's Fig. 2 (b)-(g), Sec. 5 and supplement S.1) turns a
 * burst of raw Bayer frames plus per-tile alignment vectors into a linear RGB
 * image at any output scale: per-frame half-resolution structure tensors give
 * an anisotropic Gaussian kernel covariance per pixel (Sec. 5.1.2, eq. 3-4,
 * S.1); a noise-corrected robustness mask weights each aligned frame (Sec.
 * 5.2, eq. 5-9); every output pixel accumulates the nine nearest Bayer
 * samples of every frame per colour channel and normalises (Sec. 5.1, eq. 1-2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named as DEVICE pointers must point to memory of the current
 *    HIP device; host structs are read before the call returns.
 *  - All device work is enqueued asynchronously on `stream` (a hipStream_t,
 *    NULL = the default stream); no call synchronises the host.
 *  - The caller owns every buffer it passes. The library owns an internal
 *    workspace per device (intermediate per-frame maps) that it allocates on
 *    first use, grows when a larger burst arrives and frees in
 *    hmfsr_release(). Calls that run concurrently on one device must use
 *    the same stream (the workspace is shared); the library serialises its
 *    host-side bookkeeping with a mutex.
 *  - Graph capture: once an eager call of the same burst size has sized the
 *    workspace, hmfsr_merge and hmfsr_merge_backward enqueue kernel launches
 *    only (no allocation, copy, fill or synchronisation) and may be
 *    captured into a HIP graph. The graph then reads the workspace it was
 *    captured with: a later call that grows the workspace, or
 *    hmfsr_release(), frees it, and the graph must not be replayed after
 *    that. With HMFSR_DEBUG set these calls synchronise and cannot be
 *    captured. hmfsr_merge_noalloc uses a fixed scratch buffer instead.
 *  - Outputs are overwritten, never accumulated into.
 *  - Descriptor and tuning values are validated on the host before any
 *    device work: invalid values give HMFSR_E_INVALID and touch nothing.
 *    Device data (frames, motion) is not inspected: a non-finite
 *    displacement component is taken as +-(max(width, height) + 16) (NaN as
 *    the negative bound), just past the frame, where no sample lies in it, so
 *    the frame adds nothing there. With the environment variable
 *    HMFSR_DEBUG=1, hmfsr_merge, hmfsr_merge_backward, hmfsr_merge_maps,
 *    hmfsr_stream_add and hmfsr_merge_batch first scan the motion vectors of
 *    the frames other than the base frame on the device (synchronising
 *    `stream`) and return HMFSR_E_DATA, with a line on stderr naming the
 *    first non-finite value, before any other work.
 */
#ifndef HMFSR_H
#define HMFSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HMFSR_VERSION 140 /* 1.4.0 */

/* Colour filter array layout: colours of the 2x2 Bayer cell read row by row. */
typedef enum {
  HMFSR_CFA_RGGB = 0,
  HMFSR_CFA_GRBG = 1,
  HMFSR_CFA_GBRG = 2,
  HMFSR_CFA_BGGR = 3
} hmfsr_cfa;

typedef enum {
  HMFSR_OK = 0,
  HMFSR_E_INVALID = -1,     /* bad descriptor, tuning or NULL pointer          */
  HMFSR_E_UNSUPPORTED = -2, /* unknown CFA code, or a device that is not gfx950 */
  HMFSR_E_HIP = -3,         /* a HIP runtime call or kernel launch failed      */
  HMFSR_E_NOMEM = -4,       /* the internal workspace could not be allocated   */
  HMFSR_E_TOO_LARGE = -5,   /* hmfsr_merge_noalloc: the burst's maps exceed its
                               static scratch (HMFSR_NOALLOC_SCRATCH_BYTES)      */
  HMFSR_E_DATA = -6         /* HMFSR_DEBUG=1 only: device data failed a check  */
} hmfsr_status;

/*
 * Burst descriptor (host struct).
 *  n_frames     >= 1 frames in the burst (the paper merges 2..15, Sec. 6.4).
 *  height,width Bayer frame size in pixels; both even and >= 4, <= 32768.
 *  ref_frame    index of the base frame, 0 <= ref_frame < n_frames. Its
 *               robustness is 1 (Sec. 5.1, after eq. 1).
 *  cfa          hmfsr_cfa, the mosaic of every frame.
 *  black_level, white_level
 *               raw levels mapped to 0 and 1 (x = (raw - black)/(white - black),
 *               not clamped); black < white.
 *  noise_a, noise_b
 *               noise model of the normalised raw values: variance
 *               a * x + b (Sec. 5.2.2, heteroscedastic Gaussian); a >= 0, b > 0.
 *  tile_size    T_s, edge of the square alignment tiles in pixels (S.2 gives
 *               16, 32 or 64); even, 8..256.
 *  scale        output magnification s >= 1 (Sec. 7.1: 1x to 3x); <= 8.
 *  out_height, out_width
 *               must equal floor(height * scale + 0.5), floor(width * scale + 0.5).
 *               Output pixel (R, C) sits at base-frame position
 *               ((C + 1/2) / s, (R + 1/2) / s) in pixel-edge coordinates.
 *  noise_bins, noise_table
 *               0 and NULL: the robustness uses the closed forms of the noise
 *               model, sigma_md^2 = var and d_md^2 = 2 var / 9 with
 *               var = a x + b at the base brightness x (halved for the guide's
 *               two-green mean). Else a DEVICE float32 table [noise_bins][4],
 *               4-byte aligned, 2 <= noise_bins <= 65536, as hmfsr_noise_table
 *               writes it: per brightness x_i = i / (noise_bins - 1)
 *               (normalised units), sigma_md^2 and d_md^2 of an R or B guide
 *               pixel, then of the green mean (Sec. 5.2.2's Monte-Carlo
 *               tables); it is interpolated linearly at the base brightness
 *               clamped to [0, 1], and read by every call that takes the
 *               descriptor.
 */
typedef struct {
  int32_t n_frames, height, width;
  int32_t ref_frame;
  int32_t cfa;
  float black_level, white_level;
  float noise_a, noise_b;
  int32_t tile_size;
  float scale;
  int32_t out_height, out_width;
  int32_t noise_bins;
  const float* noise_table;
} hmfsr_desc;

/*
 * Tuning scalars (host struct), supplement S.1/S.2 notation.
 *  k_detail    base kernel standard deviation (px), > 0
 *  k_denoise   kernel standard deviation multiplier for denoising, > 0
 *  d_th, d_tr  denoising threshold / transition (gradient units), d_tr > 0
 *  k_stretch   kernel stretch along edges, > 0
 *  k_shrink    kernel shrink across edges, > 0
 *  s           robustness scale s_2 where the local motion is small (eq. 8), >= 0
 *  t           robustness threshold of eq. (5)
 *  s_motion    robustness scale s_1 where the motion spread M exceeds m_th, >= 0
 *  m_th        motion-spread threshold M_th (px), >= 0
 *  hf_ratio    high-frequency artefact rejection (supplement S.3), >= 0; 0
 *              turns it off. A pixel of an aligned frame is fully rejected
 *              (R = 0 before the 5x5 minimum of eq. 9) where its tile's motion
 *              prior chose s_motion (M > M_th, eq. 8) and the base frame's guide
 *              loses variance to the 3x3 low-pass: with x the guide doubled to
 *              integers and S its 3x3 box sums, summed over the channels,
 *              9 sum S^2 - (sum S)^2 < hf_ratio * 81 * (9 sum x^2 - (sum x)^2)
 *              over the 3x3 windows (edge-replicated), in exact arithmetic.
 *              The ratio of the two variances is 1/81 on a pixel checkerboard,
 *              1 on a ramp and has a median near 0.06 on white noise; 0.02 is
 *              a reasonable setting.
 * All finite.
 */
typedef struct {
  float k_detail, k_denoise, d_th, d_tr, k_stretch, k_shrink, s, t;
  float s_motion;
  float m_th;
  float hf_ratio;
} hmfsr_tuning;

/*
 * hmfsr_merge -- merge one burst (Sec. 5, eq. 1-9).
 *  frames  DEVICE uint16 [n_frames][height][width], row-major raw CFA values,
 *          4-byte aligned.
 *  motion  DEVICE float32 [n_frames][TY][TX][2], TY = ceil(height/T_s),
 *          TX = ceil(width/T_s): displacement (vx, vy) in pixels of base tile
 *          (ty, tx) in frame n, i.e. base position X is seen at X + v in
 *          frame n (Sec. 3.2 alignment vectors). motion[ref_frame] is ignored
 *          and taken as 0.
 *  out     DEVICE float32 [3][out_height][out_width], planes R, G, B of the
 *          normalised linear result (eq. 1).
 *  saved   NULL, or a DEVICE buffer of 12 * out_height * out_width 4-byte
 *          words, 8-byte aligned, that receives the normaliser of eq. (1) for
 *          hmfsr_merge_backward (which then needs no second forward): three
 *          float64 planes [3][out_height][out_width] with C per channel in raw
 *          units, then three float32 planes with the denominator (scaled by
 *          2^-m) and three with the reference exponent m (log2 units). With
 *          saved the normaliser is accumulated in float64 and the 64 x 16
 *          tile shape is used, so `out` can differ from a call without it in
 *          the last bits.
 * The internal workspace holds per-frame maps of the base half-resolution
 * grid (the guide's packed 3x3 sums and R_hat): about 12 bytes per
 * half-resolution pixel and frame.
 * Returns HMFSR_OK, or an error code with nothing enqueued.
 */
hmfsr_status hmfsr_merge(const hmfsr_desc* desc, const hmfsr_tuning* tuning,
                         const uint16_t* frames, const float* motion, float* out,
                         float* saved, void* stream);

/*
 * hmfsr_merge_noalloc -- hmfsr_merge for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Same arguments, kernels and results as hmfsr_merge (bit
 * for bit, for the same tile shape), but the per-frame maps live in a
 * static scratch array of HMFSR_NOALLOC_SCRATCH_BYTES per device, which the
 * library's code object holds from load until the process ends; the call
 * allocates nothing (no hipMalloc, hipFree, events or library allocations)
 * and profiling does not time it.
 *  Limit: the maps take about 12 bytes per half-resolution pixel and frame
 *  (up to 16 frames of 1024 x 768 and 6 frames of 2016 x 1512 fit; a
 *  12 MP x 8 burst does not): a burst whose maps exceed the scratch returns
 *  HMFSR_E_TOO_LARGE before any device work.
 *  Every call on one device shares that device's scratch and nothing in it
 *  has to start at zero (each call writes every entry it reads). Calls that
 *  overlap on one device -- on different streams, or from different threads
 *  without ordering -- race on the scratch: serialise them (one stream).
 *  The first call on a device resolves the scratch's device address
 *  (hipGetSymbolAddress) and keeps it.
 */
#define HMFSR_NOALLOC_SCRATCH_BYTES (64u << 20)
hmfsr_status hmfsr_merge_noalloc(const hmfsr_desc* desc, const hmfsr_tuning* tuning,
                                 const uint16_t* frames, const float* motion, float* out,
                                 float* saved, void* stream);

/*
 * hmfsr_merge_backward -- adjoint of hmfsr_merge. Given dL/dC for the output C
 * of hmfsr_merge on the same inputs, the gradient of L with respect to the
 * tuning scalars and to the displacements. The paper defines no gradient:
 * this is the derivative of the merge as defined by eq. (1)-(9) and S.1,
 * with every piecewise-constant decision (nine-sample window centres,
 * bilinear cells, the motion-prior choice of eq. 8, the clamps of D and of
 * R in eq. 5, the 5x5 argmin of eq. 9, first minimum in scan order) held fixed.
 *  frames, motion  as for hmfsr_merge.
 *  saved     NULL (the forward normaliser is recomputed internally) or the
 *            buffer a hmfsr_merge call on the same inputs filled.
 *  grad_out  DEVICE float32 [3][out_height][out_width]: dL/dC.
 *  grad_tuning  DEVICE float32 [9]: dL/d(k_detail, k_denoise, d_th, d_tr,
 *            k_stretch, k_shrink, s, t, s_motion). m_th and hf_ratio are
 *            thresholds with zero derivative almost everywhere and get none;
 *            pixels the S.3 test rejects have R = 0 and pass no gradient.
 *  grad_motion  DEVICE float32 [n_frames][TY][TX][2]: dL/d(vx, vy); the
 *            base frame's vectors are ignored by the merge and get 0.
 * Kernel weights are recomputed, not stored. Sums are taken in a fixed order:
 * repeated calls give identical bits. The internal workspace grows to about
 * 16 bytes per half-resolution pixel and frame (the forward's maps and R)
 * plus 3 bytes per output pixel and frame (per-tile partials), and 48 bytes
 * per output pixel more when saved is NULL.
 */
hmfsr_status hmfsr_merge_backward(const hmfsr_desc* desc, const hmfsr_tuning* tuning,
                                  const uint16_t* frames, const float* motion,
                                  const float* saved, const float* grad_out,
                                  float* grad_tuning, float* grad_motion, void* stream);

/*
 * Streaming merge -- frames added one call at a time into a caller-owned
 * accumulator state, so that memory does not grow with the frame count (the
 * paper's online merge, Sec. 5.1 and 6.5). The result equals hmfsr_merge's
 * with the 64 x 16 tile shape bit for bit when the frames are added in the
 * order hmfsr_merge visits them (base frame, then the others in index order).
 *  state  DEVICE float32 [9][out_height][out_width], caller-owned: per
 *         channel the numerator and denominator of eq. (1) (raw units, scaled
 *         by 2^-m) and the reference exponent m.
 * The descriptor's n_frames and ref_frame are not used; the other fields,
 * the tuning and the frame layout are as for hmfsr_merge.
 *
 * hmfsr_stream_begin -- initialise `state` with the base frame (weight 1).
 * hmfsr_stream_add   -- add one aligned frame: `frame` DEVICE uint16 [H][W],
 *                       `motion` DEVICE float32 [TY][TX][2] (its tile
 *                       displacements), `base_frame` the same base frame as
 *                       for begin (its statistics drive the robustness, eq.
 *                       5-9). The frames are copied into a library workspace
 *                       of two frames; calls on one device must share a stream.
 * hmfsr_stream_end   -- normalise `state` into `out` (eq. 1), as hmfsr_merge.
 */
hmfsr_status hmfsr_stream_begin(const hmfsr_desc* desc, const hmfsr_tuning* tuning,
                                const uint16_t* base_frame, float* state, void* stream);
hmfsr_status hmfsr_stream_add(const hmfsr_desc* desc, const hmfsr_tuning* tuning,
                              const uint16_t* base_frame, const uint16_t* frame,
                              const float* motion, float* state, void* stream);
hmfsr_status hmfsr_stream_end(const hmfsr_desc* desc, const hmfsr_tuning* tuning,
                              const float* state, float* out, void* stream);

/*
 * Tile-alignment parameters (host struct). The paper fixes only the number of
 * Lucas-Kanade iterations (three, Sec. 3.2); the other defaults are this
 * library's choice.
 *  levels         pyramid levels, 1..6 (default 4); fewer are built where a
 *                 coarser level would not hold an 8 x 8 block
 *  radius_coarse  search radius (pixels) on the coarsest level, 1..8 (default 4)
 *  radius_fine    search radius on every finer level, 1..8 (default 2)
 *  lk_iterations  Lucas-Kanade iterations, 0..16 (default 3)
 *  gate           noise gate kappa, 0..1000 (default 4; 0 turns it off): a
 *                 block keeps its guess unless its best candidate lowers the
 *                 cost by more than kappa standard deviations of the cost
 *                 differences that noise alone produces (below)
 */
typedef struct {
  int32_t levels, radius_coarse, radius_fine, lk_iterations;
  float gate;
} hmfsr_align_params;

/*
 * hmfsr_align -- per-tile alignment vectors of every frame against the base
 * frame (Sec. 3.2), in the layout hmfsr_merge reads, so that a raw burst goes
 * to RGB through hmfsr_align then hmfsr_merge.
 *  desc     as for hmfsr_merge; only n_frames, height, width, ref_frame,
 *           tile_size (<= 64, S.2's largest) and, for the noise gate,
 *           black_level, white_level, noise_a and noise_b are used.
 *  params   NULL for the defaults.
 *  frames   DEVICE uint16 [n_frames][height][width], 4-byte aligned.
 *  motion   DEVICE float32 [n_frames][TY][TX][2], 8-byte aligned (output):
 *           (vx, vy) in raw pixels such that base position X of tile (ty, tx)
 *           is seen at X + v in the frame; 0 for the base frame.
 *  block_match  NULL, or DEVICE int32 [n_frames][TY][TX][2], 8-byte aligned
 *           (output): the integer block-matching vector of each tile on the
 *           half-resolution grid, before the Lucas-Kanade refinement.
 * Method (the paper leaves the details open; these are the library's):
 * frames are reduced to integer 2x2-quad sums (half resolution, level 0);
 * level l + 1 holds the 2x2 sums of level l. Blocks are the merge's tiles
 * (tile_size / 2 on level 0) and 8 x 8 above. On each level, from the
 * coarsest, every block takes the integer offset that minimises the sum of
 * squared differences (edge-replicated frame) over guess + [-R, R]^2, ties to
 * the smallest offset from the guess and then to the first in row-major
 * order; the guess is twice the vector of the coarser block holding the
 * block's centre (0 on the coarsest level). Noise gate: with the noise model
 * of Sec. 5.2.2 a level-l pixel (a sum of m = 4^(l+1) raw values) has
 * variance v = m (a x + b) R^2 (R = white - black, x the block's mean
 * brightness in [0, 1]), and noise alone spreads the cost difference of two
 * candidates over N pixels by sqrt(12 N) v; the winner replaces the guess only
 * when N gain^2 > 12 kappa^2 (N v)^2, decided in float64 with the operations
 * rounded in a fixed order (S the block's integer sum, nm = N m,
 * e = clamp(S - nm black, 0, nm R), u = (a R) e + ((nm b) R) R, then
 * (N gain) gain > (((12 kappa) kappa) u) u). Each tile's vector is then
 * refined by translation-only Lucas-Kanade on level 0 over the tile grown by
 * half a tile on every side: central-difference gradients of the base frame,
 * bilinear error image, v -= H^-1 b; tiles whose normal matrix H has
 * det H <= 1e-9 (tr H)^2 keep their block-matching vector. The result is
 * twice the level-0 vector. Workspace: about 1.4 bytes per raw pixel and frame.
 */
hmfsr_status hmfsr_align(const hmfsr_desc* desc, const hmfsr_align_params* params, const uint16_t* frames,
                         float* motion, int32_t* block_match, void* stream);

/*
 * hmfsr_noise_table -- the Monte-Carlo noise tables of Sec. 5.2.2 for the
 * descriptor's noise model (noise_a, noise_b) and raw range (black_level,
 * white_level), written to `table` (DEVICE float32 [bins][4], 4-byte aligned)
 * in the layout hmfsr_desc.noise_table reads. The paper simulates constant
 * patches per brightness level so that clipping at the white point is
 * accounted for and gives no further detail; this library's simulation:
 * brightness x_i = i / (bins - 1); per patch two frames of nine guide pixels
 * (an R or B pixel is one raw sample, the green guide the mean of two), raw
 * samples x + sqrt(a max(x, 0) + b) z clipped to the raw range
 * [-black / (white - black), 1]; sigma_md^2 = the mean of the two frames'
 * unbiased 3x3 variances and d_md^2 = the mean squared difference of their
 * 3x3 means, over `patches` patches. Normals: Philox4x32-10 (Salmon et al.,
 * SC 2011) with counter (patch, bin, 16 class + j, 0), key (seed low 32 bits,
 * high 32 bits), four uniforms (u + 1/2) 2^-32 per call paired by Box-Muller;
 * sums in float64, in a fixed order (repeated calls give the same bits).
 *  bins 2..65536, patches 1..2^24.
 */
hmfsr_status hmfsr_noise_table(const hmfsr_desc* desc, int32_t bins, int32_t patches, uint64_t seed,
                               float* table, void* stream);

/*
 * hmfsr_auto_tuning -- SNR-dependent tuning (Sec. 7.2, supplement S.2): the
 * base frame's SNR x / sqrt(a max(x, 0) + b), x its mean normalised raw value
 * (an exact integer sum on the device), and tuning values piecewise linear in
 * the SNR over [6, 30] between S.2's printed ends (the paper prints no
 * breakpoints): with s = clamp((SNR - 6) / 24, 0, 1) and v = (1 - s) v_6 +
 * s v_30, k_detail 0.33 -> 0.25, k_denoise 5 -> 3, d_th 0.010 -> 0.001,
 * d_tr 0.020 -> 0.006; k_stretch 4, k_shrink 2, s 2, t 0.12, s_motion 12,
 * m_th 0.8 and hf_ratio 0 fixed; tile size 64 below SNR 14, 32 below 22, else
 * 16. Synchronises `stream` (the results are host values).
 *  frames   DEVICE uint16 [n_frames][height][width] (only the base frame is read).
 *  tuning   HOST, receives the tuning values.
 *  tile_size, snr  HOST, nullable: the suggested tile size and the SNR.
 */
hmfsr_status hmfsr_auto_tuning(const hmfsr_desc* desc, const uint16_t* frames, hmfsr_tuning* tuning,
                               int32_t* tile_size, double* snr, void* stream);

/*
 * hmfsr_merge_maps -- the per-frame intermediate maps of the merge, for
 * inspection (the paper visualises the accumulated robustness mask and the
 * kernel shapes). Same inputs as hmfsr_merge; h = height/2, w = width/2.
 *  omega     DEVICE float64 [n_frames][3][h][w]: kernel covariance
 *            (Oxx, Oxy, Oyy) per half-resolution pixel (eq. 4, S.1).
 *  robust    DEVICE float32 [n_frames][h][w]: R of eq. (5) on the base
 *            frame's half-resolution grid (1 for the base frame).
 *  robust_min DEVICE float32 [n_frames][h][w]: its 5x5 minimum (eq. 9).
 *  s_tile    DEVICE float32 [n_frames][TY][TX]: the rejection strength
 *            chosen by the motion prior (eq. 7-8; 0 for the base frame).
 * Any of the four may be NULL to skip it.
 */
hmfsr_status hmfsr_merge_maps(const hmfsr_desc* desc, const hmfsr_tuning* tuning,
                              const uint16_t* frames, const float* motion, double* omega,
                              float* robust, float* robust_min, float* s_tile, void* stream);

/*
 * hmfsr_merge_batch -- merge many independent bursts (any mix of frame counts,
 * sizes and scales) in one launch of a captured hipGraph.
 *  n_bursts        1..65536
 *  descs, tunings  HOST arrays [n_bursts], validated like hmfsr_merge's.
 *  frames, motion, out
 *                  HOST arrays [n_bursts] of DEVICE pointers with the
 *                  layouts of hmfsr_merge.
 * The graph holds a counter reset, the motion prior of every burst, one
 * persistent robustness kernel and one persistent merge kernel per tile
 * shape; persistent workgroups take (burst, tile) items from a global counter,
 * most expensive bursts first. The first call for a set of shapes and buffers
 * builds and instantiates the graph (synchronising `stream` once); later calls
 * with the same descriptors and pointers replay it, uploading changed tuning
 * values first (after synchronising `stream`). Results equal hmfsr_merge's
 * for the same tile shape bit for bit.
 */
hmfsr_status hmfsr_merge_batch(int32_t n_bursts, const hmfsr_desc* descs,
                               const hmfsr_tuning* tunings, const uint16_t* const* frames,
                               const float* const* motion, float* const* out, void* stream);

/*
 * hmfsr_batch_plan -- the work layout of the batch graph last captured on the
 * current device (host values, no device work): the (burst, tile) items of
 * the persistent robustness launch and of each persistent merge launch, and
 * the workgroups each launch starts. Merge launch c (0..7) takes the bursts
 * of tile shape c / 2 (indices as for hmfsr_autotune) whose raw footprint is
 * loaded in batches of four (c even) or eight (c odd) samples per thread, as
 * the burst's own hmfsr_merge launch would. A workgroup pulls items until the list is exhausted, so
 * items / workgroups is how many it takes in turn. By default a launch starts
 * min(items, compute units x resident workgroups per unit) workgroups;
 * HMFSR_BATCH_GROUPS=<k> (k >= 1) caps every launch at k when a graph is
 * captured (the cap is part of the graph's signature).
 *  out  HOST. HMFSR_E_INVALID when no graph was captured on this device.
 */
typedef struct {
  int32_t robust_items, robust_groups;
  int32_t merge_items[8], merge_groups[8];
} hmfsr_batch_info;
hmfsr_status hmfsr_batch_plan(hmfsr_batch_info* out);

/*
 * hmfsr_autotune -- time every compiled tile shape of the merge kernel on this
 * burst (synchronising `stream`), remember the fastest for the burst's class
 * (output scale <= 1, <= 1.5, <= 2, > 2 x frame count <= 4, <= 8, <= 15, > 15)
 * and use it for later merges of that class. With HMFSR_TUNE_CACHE=<file> the
 * table is read at first use and rewritten after each tuning. `out` receives
 * the merge; `chosen` (host, nullable) the index of the chosen shape.
 * HMFSR_MERGE_VARIANT=<index> overrides every choice.
 */
hmfsr_status hmfsr_autotune(const hmfsr_desc* desc, const hmfsr_tuning* tuning,
                            const uint16_t* frames, const float* motion, float* out, void* stream,
                            int32_t* chosen);

/*
 * Per-stage GPU timing (the tracing aid of the library). Between
 * hmfsr_profile_begin() and hmfsr_profile_end(), every kernel launch is
 * bracketed by a pair of HIP events recorded on the call's own stream;
 * hmfsr_profile_end() waits for the recorded events, adds up the elapsed
 * times per stage and turns the recording off. Not meant for use while other
 * threads issue merges.
 */
enum {
  HMFSR_STAGE_PRIOR = 0,  /* motion prior per tile (eq. 7-8)           */
  HMFSR_STAGE_ROBUST = 1, /* robustness and its 5x5 minimum (eq. 5-9)  */
  HMFSR_STAGE_MERGE = 2,  /* kernel-regression accumulation (eq. 1-4)  */
  HMFSR_STAGE_BATCH = 3,  /* one replay of a batched-merge graph       */
  HMFSR_STAGE_MERGE_BWD = 4,   /* adjoint of the accumulation              */
  HMFSR_STAGE_ROBUST_BWD = 5,  /* adjoint of the robustness                */
  HMFSR_STAGE_GRAD_REDUCE = 6, /* fixed-order sums of the gradient partials */
  HMFSR_STAGE_ALIGN = 7,       /* tile alignment (pyramid, matching, Lucas-Kanade) */
  HMFSR_NUM_STAGES = 8
};
typedef struct {
  double ms_total[HMFSR_NUM_STAGES];  /* summed kernel time per stage, milliseconds */
  int64_t launches[HMFSR_NUM_STAGES]; /* number of launches per stage             */
} hmfsr_stage_times;
hmfsr_status hmfsr_profile_begin(void);
hmfsr_status hmfsr_profile_end(hmfsr_stage_times* out);

/* Human-readable name of a status code (static storage). */
const char* hmfsr_strerror(hmfsr_status status);

/* HMFSR_VERSION of the built library. */
int32_t hmfsr_version(void);

/* Free the internal workspace of every device. Not safe to call while work
 * that uses it is still running: synchronise the streams first. */
void hmfsr_release(void);

#ifdef __cplusplus
}
#endif

#endif /* HMFSR_H */
