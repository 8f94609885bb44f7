// Tile alignment of a burst against its base frame (Sec. 3.2): a pyramid of
// integer 2x2 sums of the half-resolution luma, coarse-to-fine block matching
// by integer sum of squared differences, and Lucas-Kanade refinement of the
// finest level's vectors.
//
// Every integer step (pyramid, costs, the argmin and its tie rules) is exact,
// and the noise gate that keeps a block at its guess when the winner's gain
// is within the noise (the noise model of Sec. 5.2.2) compares float64 values
// rounded in a fixed order, so the block-matching vectors are fully
// determined by the frames and the descriptor. The
// Lucas-Kanade normal matrix is an exact integer sum as well; its solve and
// the error image run in float64.
#include <stdint.h>

#include <algorithm>

#include "device_util.h"
#include "hmfsr_internal.h"

namespace hmfsr {
namespace {

constexpr int kPyrEdge = 64;       // level-0 pixels per pyramid workgroup edge
constexpr int kAlignThreads = 256;   // pyramid workgroup

// ---- pyramid ------------------------------------------------------------------
// Workgroup = a 64 x 64 region of level 0 (128 x 128 raw pixels) of one frame;
// level l of the region (64 >> l pixels square) is summed in LDS from level
// l - 1. A level-l pixel inside the level's size has all four children inside
// level l - 1 and inside the same region, since regions are aligned to 64.
__global__ __launch_bounds__(kAlignThreads) void k_align_pyramid(const uint16_t* __restrict__ frames, int H,
                                                                 int W, int32_t* __restrict__ pyr,
                                                                 AlignGeom ag) {
  __shared__ int32_t sa[kPyrEdge * kPyrEdge];
  __shared__ int32_t sb[(kPyrEdge / 2) * (kPyrEdge / 2)];
  const int f = blockIdx.z;
  const uint16_t* fr = frames + (size_t)f * H * W;
  int32_t* P = pyr + f * ag.fstride;
  const int lane = threadIdx.x & 63, wrow = threadIdx.x >> 6;
  const int h0 = ag.lh[0], w0 = ag.lw[0];
  const int X0 = blockIdx.x * kPyrEdge, Y0 = blockIdx.y * kPyrEdge;
  for (int r = wrow; r < kPyrEdge; r += kAlignThreads / 64) {
    const int y = Y0 + r, x = X0 + lane;
    int v = 0;
    if (y < h0 && x < w0) {
      const uint32_t a = *(const uint32_t*)(fr + (size_t)(2 * y) * W + 2 * x);
      const uint32_t b = *(const uint32_t*)(fr + (size_t)(2 * y + 1) * W + 2 * x);
      v = (int)((a & 0xffffu) + (a >> 16) + (b & 0xffffu) + (b >> 16));
      P[ag.loff[0] + (long long)y * w0 + x] = v;
    }
    sa[r * kPyrEdge + lane] = v;
  }
  int32_t* src = sa;
  int32_t* dst = sb;
  int e = kPyrEdge;  // region edge on the source level
  for (int l = 1; l < ag.L; ++l) {
    __syncthreads();  // the source level is complete and the destination is free
    const int ne = e >> 1;
    const int sh = 31 - __clz(ne);
    const int oy = blockIdx.y * ne, ox = blockIdx.x * ne;
    for (int i = threadIdx.x; i < ne * ne; i += kAlignThreads) {
      const int r = i >> sh, c = i & (ne - 1);
      const int* s0 = src + (2 * r) * e + 2 * c;
      const int v = s0[0] + s0[1] + s0[e] + s0[e + 1];
      dst[i] = v;
      const int y = oy + r, x = ox + c;
      if (y < ag.lh[l] && x < ag.lw[l]) P[ag.loff[l] + (long long)y * ag.lw[l] + x] = v;
    }
    int32_t* t = src;
    src = dst;
    dst = t;
    e = ne;
  }
}

// ---- block matching ---------------------------------------------------------------
struct MatchLevel {
  int B, R;                 // block edge, search radius
  int h, w;                 // level size
  int gby, gbx;             // block grid
  long long loff, voff;     // level offset in a frame's pyramid; its vectors in a frame's set
  int parent;               // 1 when the coarser level supplies the guess
  int pB, pgby, pgbx;       // the coarser level's block edge and grid
  long long pvoff;
  int level;                // pyramid level (a pixel sums 4^(level+1) raw values)
  double k12, na, nb, black, rng;  // noise gate: (12 kappa) kappa (0: off) and the noise model
};

// Noise gate of block matching: does a winner that lowers the cost by `gain`
// below the guess's cost move the block? N pixels with integer sum S on a
// level whose pixels sum m raw values. The operations are rounded one by one
// in this order (no contraction), so that every caller takes the same
// decision for the same integers.
__device__ __forceinline__ bool gate_moves(const MatchLevel& ml, int npx, long long S, unsigned long long gain) {
  const double n = (double)npx;
  const double nm = __dmul_rn(n, (double)(1ll << (2 * ml.level + 2)));
  double e = __dsub_rn((double)S, __dmul_rn(nm, ml.black));
  e = fmin(fmax(e, 0.0), __dmul_rn(nm, ml.rng));
  const double u = __dadd_rn(__dmul_rn(__dmul_rn(ml.na, ml.rng), e), __dmul_rn(__dmul_rn(__dmul_rn(nm, ml.nb), ml.rng), ml.rng));
  const double g = (double)gain;
  return __dmul_rn(__dmul_rn(n, g), g) > __dmul_rn(__dmul_rn(ml.k12, u), u);
}

// Persistent launches: kWaves independent waves per workgroup. Wave w of
// workgroup b (XCD-aware order) takes the contiguous item range
// [(4b + w) * chunk, (4b + w + 1) * chunk), so neighbouring items share an L2.
// A wave synchronises only with itself: its LDS region is private.
constexpr int kWaves = 4;
constexpr int kGroupsPerCU = 8;

// Cross-lane visibility of a wave's own LDS writes: the LDS executes one
// wave's operations in order, so only compiler reordering must be fenced.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Raw buffer resource over n 32-bit words (word 3 as for gfx9 raw buffers).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t words_rsrc(const int32_t* p, long long n) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, 0, (int)(n * 4), 0x00020000);
}

__device__ __forceinline__ int32_t ld_word(__amdgpu_buffer_rsrc_t r, int idx) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4, 0, 0);
}

// Copy a block's base window (rows x cols from the base frame's buffer
// resource) and its search region (E x E from the frame, per-lane pointer)
// into LDS, by the LPG lanes of its group; all loads of a round before its
// stores.
template <int LPG, int U>
__device__ __forceinline__ void stage_block(int32_t* tpl, int ldt, int rows, int cols, __amdgpu_buffer_rsrc_t rs_base,
                                            int ty0, int tx0, int32_t* reg, int E, const int32_t* img, int ry0,
                                            int rx0, int h, int w, int l) {
  const int ta = rows * cols, tb = E * E;
  const float ia = 1.0f / (float)cols, ib = 1.0f / (float)E;
  for (int i0 = 0; i0 < ta || i0 < tb; i0 += LPG * U) {
    int va[U], vb[U], aa[U], ab[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * LPG + l;
      aa[u] = -1;
      ab[u] = -1;
      va[u] = 0;
      vb[u] = 0;
      if (i < ta) {
        const int r = split_row(i, ia), c = i - r * cols;
        aa[u] = r * ldt + c;
        va[u] = ld_word(rs_base, clampi(ty0 + r, 0, h - 1) * w + clampi(tx0 + c, 0, w - 1));
      }
      if (i < tb) {
        const int r = split_row(i, ib), c = i - r * E;
        ab[u] = i;
        vb[u] = img[clampi(ry0 + r, 0, h - 1) * w + clampi(rx0 + c, 0, w - 1)];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (aa[u] >= 0) tpl[aa[u]] = va[u];
      if (ab[u] >= 0) reg[ab[u]] = vb[u];
    }
  }
}

// Sum of squared differences of one block row of W pixels, every LDS read of
// the row issued before the arithmetic. Values are integers: with float64
// sums below 2^53 (or 64-bit integers) the order does not matter.
template <int W, bool EXACT_F64>
__device__ __forceinline__ void row_ssd(const int32_t* tr, const int32_t* rr, double& acc, unsigned long long& ssd) {
  int tv[W], rv[W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    tv[c] = tr[c];
    rv[c] = rr[c];
  }
#pragma unroll
  for (int c = 0; c < W; ++c) {
    if (EXACT_F64) {
      const double d = (double)(rv[c] - tv[c]);
      acc = fma(d, d, acc);
    } else {
      const long long d = (long long)(rv[c] - tv[c]);
      ssd += (unsigned long long)(d * d);
    }
  }
}

// Candidate key packed for lane exchanges: cost, then (squared offset from
// the guess) * 2^16 + scan index; the lexicographic minimum wins.
struct PKey {
  unsigned long long ssd;
  int tie;
};

template <int CTRL>
__device__ __forceinline__ PKey dpp_key(const PKey& a) {
  PKey o;
  o.ssd = ((unsigned long long)(unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(a.ssd >> 32), CTRL, 0xF, 0xF,
                                                                      true)
           << 32) |
          (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(a.ssd & 0xffffffffull), CTRL, 0xF, 0xF, true);
  o.tie = __builtin_amdgcn_update_dpp(0, a.tie, CTRL, 0xF, 0xF, true);
  return o;
}

__device__ __forceinline__ void key_min(PKey& a, const PKey& b) {
  if (b.ssd < a.ssd || (b.ssd == a.ssd && b.tie < a.tie)) a = b;
}

// Block matching of one level, four blocks per wave: the 16 lanes of group g
// take block q0 + g of the wave's chunk and split its candidates (lane l takes
// l, l + 16, ...); the group minimum of the keys is then exchanged over DPP
// (row mirror, half mirror, quad permutations: disjoint orbits, so four steps
// cover the 16 lanes). LDS per group: the base block (B x B) and the frame's
// search region ((B + 2R)^2, edge-replicated).
// EXACT_F64: every level value is below 2^22 (levels 0-2 of 16-bit frames), so
// squared differences and their sums stay below 2^53 and float64 adds them
// exactly; coarser levels add in 64-bit integers.
template <bool EXACT_F64>
__global__ __launch_bounds__(256) void k_align_match(const int32_t* __restrict__ pyr, int2* __restrict__ vecs,
                                                     MatchLevel ml, int ref, long long fstride, long long vstride,
                                                     int items, int chunk) {
  constexpr int LPG = 16, GPW = 4;
  extern __shared__ int32_t smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, l = lane & 15;
  const int B = ml.B, R = ml.R, E = B + 2 * R, D = 2 * R + 1, K = D * D;
  int32_t* tpl = smem + (wave * GPW + g) * (B * B + E * E);
  int32_t* reg = tpl + B * B;
  const int per = ml.gby * ml.gbx;
  const int gw = xcd_tile(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave;
  const int c0 = gw * chunk, c1 = min(items, c0 + chunk);
  const long long lvl_words = (long long)ml.h * ml.w;
  const __amdgpu_buffer_rsrc_t rs_base = words_rsrc(pyr + (long long)ref * fstride + ml.loff, lvl_words);
  for (int q0 = c0; q0 < c1; q0 += GPW) {
    const int item = q0 + g;
    const bool valid = item < c1;
    const int fi = valid ? item / per : 0;
    const int t = valid ? item - fi * per : 0;
    const int by = t / ml.gbx, bx = t - (t / ml.gbx) * ml.gbx;
    const int f = fi < ref ? fi : fi + 1;
    int gx = 0, gy = 0;
    if (valid && ml.parent) {
      const int cy = min(((2 * by + 1) * B) / (4 * ml.pB), ml.pgby - 1);
      const int cx = min(((2 * bx + 1) * B) / (4 * ml.pB), ml.pgbx - 1);
      const int2 pv = vecs[(long long)f * vstride + ml.pvoff + cy * ml.pgbx + cx];
      gx = 2 * pv.x;
      gy = 2 * pv.y;
    }
    const int nby = min(B, ml.h - by * B), nbx = min(B, ml.w - bx * B);
    if (valid)
      stage_block<LPG, 9>(tpl, B, nby, nbx, rs_base, by * B, bx * B, reg, E, pyr + (long long)f * fstride + ml.loff,
                          by * B + gy - R, bx * B + gx - R, ml.h, ml.w, l);
    wave_sync();
    PKey best{~0ull, 0x7fffffff};
    const int kc = R * D + R;  // the candidate at the guess
    unsigned long long ssd_c = 0;
    if (valid) {
      for (int k = l; k < K; k += LPG) {
        const int dyi = k / D, dxi = k - (k / D) * D;
        unsigned long long ssd = 0;
        if (nbx == 4 || nbx == 8 || nbx == 16 || nbx == 32) {  // full-width rows, unrolled
          double acc = 0.0;
          for (int r = 0; r < nby; ++r) {
            const int32_t* tr = tpl + r * B;
            const int32_t* rr = reg + (r + dyi) * E + dxi;
            if (nbx == 8) {
              row_ssd<8, EXACT_F64>(tr, rr, acc, ssd);
            } else if (nbx == 4) {
              row_ssd<4, EXACT_F64>(tr, rr, acc, ssd);
            } else {
              for (int c0 = 0; c0 < nbx; c0 += 8) row_ssd<8, EXACT_F64>(tr + c0, rr + c0, acc, ssd);
            }
          }
          if (EXACT_F64) ssd = (unsigned long long)acc;
        } else if (EXACT_F64) {
          double acc = 0.0;
          for (int r = 0; r < nby; ++r) {
            const int32_t* tr = tpl + r * B;
            const int32_t* rr = reg + (r + dyi) * E + dxi;
            for (int c = 0; c < nbx; ++c) {
              const double d = (double)(rr[c] - tr[c]);
              acc = fma(d, d, acc);
            }
          }
          ssd = (unsigned long long)acc;
        } else {
          for (int r = 0; r < nby; ++r) {
            const int32_t* tr = tpl + r * B;
            const int32_t* rr = reg + (r + dyi) * E + dxi;
            for (int c = 0; c < nbx; ++c) {
              const long long d = (long long)(rr[c] - tr[c]);
              ssd += (unsigned long long)(d * d);
            }
          }
        }
        const int dx = dxi - R, dy = dyi - R;
        if (k == kc) ssd_c = ssd;
        key_min(best, PKey{ssd, ((dx * dx + dy * dy) << 16) | k});
      }
    }
    key_min(best, dpp_key<0x140>(best));
    key_min(best, dpp_key<0x141>(best));
    key_min(best, dpp_key<0x4E>(best));
    key_min(best, dpp_key<0xB1>(best));
    bool keep = false;
    if (ml.k12 > 0.0) {
      // the guess's cost (one lane of the group holds it) and the block's sum
      long long S = 0;
      if (valid)
        for (int r = 0; r < nby; ++r)
          for (int c = l; c < nbx; c += LPG) S += tpl[r * B + c];
      for (int m = 8; m >= 1; m >>= 1) {
        S += __shfl_xor(S, m, LPG);
        ssd_c += __shfl_xor(ssd_c, m, LPG);
      }
      keep = !gate_moves(ml, nby * nbx, S, ssd_c - best.ssd);
    }
    if (valid && l == 0) {
      const int k = keep ? kc : best.tie & 0xffff;
      const int dyi = k / D, dxi = k - (k / D) * D;
      vecs[(long long)f * vstride + ml.voff + t] = make_int2(gx + dxi - R, gy + dyi - R);
    }
    wave_sync();  // the next blocks restage this wave's LDS
  }
}

// ---- Lucas-Kanade ----------------------------------------------------------------
struct LkArgs {
  int B, m;         // tile edge on level 0, window margin
  int h, w;         // level-0 size
  int TY, TX;       // tile grid
  int iters;
  int ref;
  long long fstride, vstride, voff0;
};

// Lane exchanges with the partner whose lane index differs in bit BIT (and,
// for BIT <= 3, possibly in lower bits too): bits 5 and 4 through the LDS
// crossbar, bits 3..0 through DPP (row_mirror: i <-> 15 - i, row_half_mirror:
// i <-> 7 - i, quad permutations [2,3,0,1] and [1,0,3,2]; gfx9 encodings).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const unsigned long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <int BIT>
__device__ __forceinline__ double partner(double v) {
  if constexpr (BIT == 5) return __shfl_xor(v, 32, 64);
  else if constexpr (BIT == 4) return __shfl_xor(v, 16, 64);
  else if constexpr (BIT == 3) return dpp_move<0x140>(v);
  else if constexpr (BIT == 2) return dpp_move<0x141>(v);
  else if constexpr (BIT == 1) return dpp_move<0x4E>(v);
  else return dpp_move<0xB1>(v);
}

// Halving step: of N values a lane keeps the half its bit BIT selects, added
// to the partner's copy of that half; the partner keeps the other half.
template <int BIT, int N>
__device__ __forceinline__ void halve(const double* in, double* out, int lane) {
  const bool up = (lane >> BIT) & 1;
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const double keep = up ? in[i + N / 2] : in[i], send = up ? in[i] : in[i + N / 2];
    out[i] = keep + partner<BIT>(send);
  }
}

// Sums of 24 per-lane values over each group of LPG (16 or 64) lanes, written
// to tbl[0..24) of the group by one lane per value. Each partner step pairs
// lanes of disjoint orbits, so after log2(LPG) steps every sum covers the
// whole group. Every value is an integer below 2^53: the sums are exact in any
// order.
template <int LPG>
__device__ __forceinline__ void group_sum24(const double* v, double* tbl, int lane, bool write) {
  constexpr int TOP = LPG == 16 ? 3 : 5;
  double a[12], b[6], c[3];
  halve<TOP, 24>(v, a, lane);
  halve<TOP - 1, 12>(a, b, lane);
  halve<TOP - 2, 6>(b, c, lane);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if constexpr (TOP - 3 >= 2) c[j] += partner<2>(c[j]);
    if constexpr (TOP - 3 >= 1) c[j] += partner<1>(c[j]);
    c[j] += partner<0>(c[j]);
  }
  if (write && (lane & ((1 << (TOP - 2)) - 1)) == 0) {
    const int i0 = 12 * ((lane >> TOP) & 1) + 6 * ((lane >> (TOP - 1)) & 1) + 3 * ((lane >> (TOP - 2)) & 1);
#pragma unroll
    for (int j = 0; j < 3; ++j) tbl[i0 + j] = c[j];
  }
}

// Copy the bordered base window and the frame's bordered patch of one tile
// into LDS, by the LPG lanes of its group (l = lane within the group). Base
// loads go through the base frame's buffer resource, frame loads through a
// per-lane pointer (the groups of a wave may hold different frames).
template <int LPG, int U>
__device__ __forceinline__ void stage_tile(int32_t* SB, int32_t* SM, int SWW, int rows, __amdgpu_buffer_rsrc_t rs_base,
                                           const int32_t* img, int h, int w, int by0, int bx0, int my0, int mx0,
                                           bool base_too, int l) {
  const int total = rows * SWW;
  const float inv = 1.0f / (float)SWW;
  for (int i0 = 0; i0 < total; i0 += LPG * U) {
    int vb[U], vm[U], at[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      at[u] = -1;
      vb[u] = 0;
      vm[u] = 0;
      const int i = i0 + u * LPG + l;
      if (i < total) {
        const int r = split_row(i, inv), c = i - r * SWW;
        at[u] = r * SWW + c;
        if (base_too) vb[u] = ld_word(rs_base, clampi(by0 + r, 0, h - 1) * w + clampi(bx0 + c, 0, w - 1));
        vm[u] = img[clampi(my0 + r, 0, h - 1) * w + clampi(mx0 + c, 0, w - 1)];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (at[u] >= 0) {
        if (base_too) SB[at[u]] = vb[u];
        SM[at[u]] = vm[u];
      }
  }
}

// Per-lane partial sums of one tile over the columns l, l + LPG, ... of its
// window, each walked top to bottom with the 3 x 3 frame neighbourhood and
// the base column kept in registers: [0, 9) sum D_x I(o), [9, 18) sum D_y I(o),
// o = (oy + 1) * 3 + ox + 1; with BASE also 18, 19: sum D_x T, sum D_y T and
// 20, 21, 22: sum D_x^2, D_x D_y, D_y^2. Products are below 2^37 and sums below
// 2^49, so float64 keeps them exact.
template <int LPG, bool BASE>
__device__ __forceinline__ void tile_sums(const int32_t* SB, const int32_t* SM, int SWW, int WH, int WW, int l,
                                          double* acc) {
#pragma unroll
  for (int i = 0; i < 24; ++i) acc[i] = 0.0;
  for (int c = l; c < WW; c += LPG) {
    const int32_t* b = SB + c + 1;
    const int32_t* m = SM + c;
    double m0[3], m1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      m0[k] = (double)m[k];
      m1[k] = (double)m[SWW + k];
    }
    int bu = b[0], bc = b[SWW];
    double m2[3];
    // window row r: the frame rows r .. r + 2 in ra, rb, rc (rc loaded here),
    // the base column's rows r, r + 1 in bu, bc (r + 2 loaded here)
    auto step = [&](int r, const double (&ra)[3], const double (&rb)[3], double (&rc)[3]) {
      const int32_t* mp = m + (r + 2) * SWW;
#pragma unroll
      for (int k = 0; k < 3; ++k) rc[k] = (double)mp[k];
      const int32_t* brow = b + (r + 1) * SWW;
      const int bd = b[(r + 2) * SWW];
      const double dx = (double)(brow[1] - brow[-1]), dy = (double)(bd - bu);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        acc[k] = fma(dx, ra[k], acc[k]);
        acc[3 + k] = fma(dx, rb[k], acc[3 + k]);
        acc[6 + k] = fma(dx, rc[k], acc[6 + k]);
        acc[9 + k] = fma(dy, ra[k], acc[9 + k]);
        acc[12 + k] = fma(dy, rb[k], acc[12 + k]);
        acc[15 + k] = fma(dy, rc[k], acc[15 + k]);
      }
      if (BASE) {
        const double tv = (double)bc;
        acc[18] = fma(dx, tv, acc[18]);
        acc[19] = fma(dy, tv, acc[19]);
        acc[20] = fma(dx, dx, acc[20]);
        acc[21] = fma(dx, dy, acc[21]);
        acc[22] = fma(dy, dy, acc[22]);
      }
      bu = bc;
      bc = bd;
    };
    if constexpr (LPG == 16) {
      // three rows per pass: the three row registers rotate by name, not by
      // copies (the wider groups keep the plain loop, whose registers allow a
      // fourth wave per SIMD)
      int r = 0;
      for (; r + 3 <= WH; r += 3) {
        step(r, m0, m1, m2);
        step(r + 1, m1, m2, m0);
        step(r + 2, m2, m0, m1);
      }
      if (r < WH) step(r++, m0, m1, m2);
      if (r < WH) step(r, m1, m2, m0);
    } else {
      for (int r = 0; r < WH; ++r) {
        step(r, m0, m1, m2);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          m0[k] = m1[k];
          m1[k] = m2[k];
        }
      }
    }
  }
}

// Lucas-Kanade, LPG lanes per (frame, tile): 16 (four tiles per wave) for
// tiles of up to 8 half-res pixels, else 64. The displacement is uniform over
// the tile, so with D = 2 g the integer central differences of the base
// window, the normal equations need only integer correlations:
//   sum_p D(p) e(p) = sum_corners w_c sum_p D(p) I(p + o_c) - sum_p D(p) T(p),
// o_c the four integer corners of the bilinear sample and w_c their weights.
// The correlations at the 3 x 3 integer offsets around a centre (first the
// block-matching vector) serve every iteration whose sample cell stays within
// them; a step that leaves them re-centres that tile and recomputes. LDS per
// group: the bordered base window and frame patch, and the 24 sums.
template <int LPG>
__global__ __launch_bounds__(256) void k_align_lk(const int32_t* __restrict__ pyr, const int2* __restrict__ vecs,
                                                  LkArgs a, float2* __restrict__ motion, int2* __restrict__ bm_out,
                                                  int items, int chunk, int sw) {
  constexpr int GPW = 64 / LPG;  // tiles per wave
  extern __shared__ int32_t smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / LPG, l = lane % LPG;
  const int grp_words = 2 * sw * sw + 48;  // two windows, then 24 doubles (sw even keeps them aligned)
  int32_t* SB = smem + (wave * GPW + g) * grp_words;
  int32_t* SM = SB + sw * sw;
  double* tbl = (double*)(SM + sw * sw);
  const int per = a.TY * a.TX;
  const int gw = xcd_tile(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave;
  const int c0 = gw * chunk, c1 = min(items, c0 + chunk);
  const long long lvl_words = (long long)a.h * a.w;
  const __amdgpu_buffer_rsrc_t rs_base = words_rsrc(pyr + (long long)a.ref * a.fstride, lvl_words);
  for (int q0 = c0; q0 < c1; q0 += GPW) {
    const int item = q0 + g;
    const int f = item / per;
    const bool valid = item < c1;
    const bool work = valid && f != a.ref;
    const int t = item - f * per;
    const int ty = t / a.TX, tx = t - (t / a.TX) * a.TX;
    const int wy0 = max(0, ty * a.B - a.m), wy1 = min(ty * a.B + a.B + a.m, a.h);
    const int wx0 = max(0, tx * a.B - a.m), wx1 = min(tx * a.B + a.B + a.m, a.w);
    const int WH = wy1 - wy0, WW = wx1 - wx0, SWW = WW + 2;
    const int32_t* img = pyr + (long long)(work ? f : a.ref) * a.fstride;
    int2 bm = make_int2(0, 0);
    if (work) bm = vecs[(long long)f * a.vstride + a.voff0 + t];
    int ccx = bm.x, ccy = bm.y;  // centre of the 3 x 3 correlation offsets
    if (work)
      stage_tile<LPG, LPG == 16 ? 11 : 8>(SB, SM, SWW, WH + 2, rs_base, img, a.h, a.w, wy0 - 1, wx0 - 1,
                                           wy0 - 1 + ccy, wx0 - 1 + ccx, true, l);
    wave_sync();
    double acc[24];
    if (work) tile_sums<LPG, true>(SB, SM, SWW, WH, WW, l, acc);
    else {
#pragma unroll
      for (int i = 0; i < 24; ++i) acc[i] = 0.0;
    }
    group_sum24<LPG>(acc, tbl, lane, true);
    wave_sync();
    const double Hxx = tbl[20], Hxy = tbl[21], Hyy = tbl[22], STx = tbl[18], STy = tbl[19];
    // Singular-window test on the exact sums, rounded step by step as written
    // (no fused multiply-add), so that it is decided identically everywhere.
    const double tr = __dadd_rn(Hxx, Hyy);
    const double det = __dsub_rn(__dmul_rn(Hxx, Hyy), __dmul_rn(Hxy, Hxy));
    const double thr = __dmul_rn(__dmul_rn(1e-9, tr), tr);
    const bool ok = work && tr > 0.0 && det > thr;
    const double k2 = ok ? 2.0 / det : 0.0;  // H and b here are 4x and 2x the half-gradient ones
    double vx = bm.x, vy = bm.y;
    for (int it = 0; it < a.iters; ++it) {
      const double fxf = floor(vx), fyf = floor(vy);
      const bool need = ok && (fxf < ccx - 1 || fxf > ccx || fyf < ccy - 1 || fyf > ccy);
      if (__any(need)) {
        // the sample cell left the correlated offsets: re-centre those tiles
        wave_sync();
        if (need) {
          ccx = (int)fmax(fmin(fxf, 1e9), -1e9);
          ccy = (int)fmax(fmin(fyf, 1e9), -1e9);
          stage_tile<LPG, LPG == 16 ? 11 : 8>(SB, SM, SWW, WH + 2, rs_base, img, a.h, a.w, 0, 0, wy0 - 1 + ccy,
                                               wx0 - 1 + ccx, false, l);
        }
        wave_sync();
        double acc2[24];
        if (need) tile_sums<LPG, false>(SB, SM, SWW, WH, WW, l, acc2);
        else {
#pragma unroll
          for (int i = 0; i < 24; ++i) acc2[i] = 0.0;
        }
        // every lane takes part in the exchanges; only re-centred groups
        // overwrite their table
        group_sum24<LPG>(acc2, tbl, lane, need);
        wave_sync();
      }
      if (ok) {
        const double fx = vx - fxf, fy = vy - fyf;
        const int o00 = ((int)(fyf - ccy) + 1) * 3 + (int)(fxf - ccx) + 1;
        const double w00 = (1.0 - fx) * (1.0 - fy), w01 = fx * (1.0 - fy), w10 = (1.0 - fx) * fy, w11 = fx * fy;
        const double sx = w00 * tbl[o00] + w01 * tbl[o00 + 1] + w10 * tbl[o00 + 3] + w11 * tbl[o00 + 4] - STx;
        const double sy =
            w00 * tbl[9 + o00] + w01 * tbl[9 + o00 + 1] + w10 * tbl[9 + o00 + 3] + w11 * tbl[9 + o00 + 4] - STy;
        vx -= k2 * (Hyy * sx - Hxy * sy);
        vy -= k2 * (Hxx * sy - Hxy * sx);
      }
    }
    if (valid && l == 0) {
      motion[item] = make_float2((float)(2.0 * vx), (float)(2.0 * vy));
      if (bm_out) bm_out[item] = bm;
    }
    wave_sync();  // the next tiles restage this wave's LDS
  }
}

unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

size_t align_bytes(const AlignGeom& ag) {
  return (size_t)ag.n * (size_t)ag.fstride * 4 + (size_t)ag.n * (size_t)ag.vstride * 8 + 256;
}

hipError_t launch_align(const AlignGeom& ag, const uint16_t* frames, int H, int W, void* ws, float* motion,
                        int* block_match, hipStream_t stream) {
  int32_t* pyr = (int32_t*)ws;
  size_t vbyte = ((size_t)ag.n * (size_t)ag.fstride * 4 + 255) & ~(size_t)255;
  int2* vecs = (int2*)((char*)ws + vbyte);
  const dim3 pg(cdiv(ag.lw[0], kPyrEdge), cdiv(ag.lh[0], kPyrEdge), ag.n);
  hipLaunchKernelGGL(k_align_pyramid, pg, dim3(kAlignThreads), 0, stream, frames, H, W, pyr, ag);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  int cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  if (ag.n > 1) {
    for (int l = ag.L - 1; l >= 0; --l) {
      MatchLevel ml;
      ml.B = ag.blk[l];
      ml.R = l == ag.L - 1 ? ag.radius_coarse : ag.radius_fine;
      ml.h = ag.lh[l];
      ml.w = ag.lw[l];
      ml.gby = ag.gby[l];
      ml.gbx = ag.gbx[l];
      ml.loff = ag.loff[l];
      ml.voff = ag.voff[l];
      ml.parent = l < ag.L - 1;
      ml.pB = ml.parent ? ag.blk[l + 1] : 1;
      ml.pgby = ml.parent ? ag.gby[l + 1] : 1;
      ml.pgbx = ml.parent ? ag.gbx[l + 1] : 1;
      ml.pvoff = ml.parent ? ag.voff[l + 1] : 0;
      ml.level = l;
      ml.k12 = ag.gate_k12;
      ml.na = ag.na;
      ml.nb = ag.nb;
      ml.black = ag.black;
      ml.rng = ag.rng;
      const int E = ml.B + 2 * ml.R;
      const int waves = ml.B <= 8 ? kWaves : 1;  // keeps LDS within 64 KiB per workgroup
      const size_t lds = (size_t)waves * 4 * (ml.B * ml.B + E * E) * 4;
      const long long items = (long long)(ag.n - 1) * ml.gby * ml.gbx;
      const long long total_waves = std::min<long long>((items + 3) / 4, (long long)cus * kGroupsPerCU * kWaves);
      long long chunk = (items + total_waves - 1) / total_waves;
      chunk = (chunk + 3) / 4 * 4;
      const unsigned groups = (unsigned)(((items + chunk - 1) / chunk + waves - 1) / waves);
      // levels 0-2 of 16-bit frames stay below 2^22 (sums of 4^(l+1) values)
      if (l <= 2)
        hipLaunchKernelGGL(k_align_match<true>, dim3(groups), dim3(64 * waves), lds, stream, pyr, vecs, ml, ag.ref,
                           ag.fstride, ag.vstride, (int)items, (int)chunk);
      else
        hipLaunchKernelGGL(k_align_match<false>, dim3(groups), dim3(64 * waves), lds, stream, pyr, vecs, ml, ag.ref,
                           ag.fstride, ag.vstride, (int)items, (int)chunk);
      if ((err = hipGetLastError()) != hipSuccess) return err;
    }
  }
  LkArgs a;
  a.B = ag.blk[0];
  a.m = a.B / 2;
  a.h = ag.lh[0];
  a.w = ag.lw[0];
  a.TY = ag.gby[0];
  a.TX = ag.gbx[0];
  a.iters = ag.lk_iterations;
  a.ref = ag.ref;
  a.fstride = ag.fstride;
  a.vstride = ag.vstride;
  a.voff0 = ag.voff[0];
  const int sw = ((a.B + 2 * a.m + 2) + 1) & ~1;  // window edge with its border, at most; even
  const long long items = (long long)ag.n * a.TY * a.TX;
  const int lpg = a.B <= 8 ? 16 : 64;
  const int gpw = 64 / lpg;
  const int waves = a.B <= 16 ? kWaves : 1;  // keeps LDS within 64 KiB per workgroup
  const size_t lds = (size_t)waves * gpw * (2 * sw * sw + 48) * 4;
  const long long total_waves =
      std::min<long long>((items + gpw - 1) / gpw, (long long)cus * kGroupsPerCU * kWaves);
  long long chunk = (items + total_waves - 1) / total_waves;
  chunk = (chunk + gpw - 1) / gpw * gpw;
  const unsigned groups = (unsigned)(((items + chunk - 1) / chunk + waves - 1) / waves);
  if (lpg == 16)
    hipLaunchKernelGGL(k_align_lk<16>, dim3(groups), dim3(64 * waves), lds, stream, pyr, vecs, a, (float2*)motion,
                       (int2*)block_match, (int)items, (int)chunk, sw);
  else
    hipLaunchKernelGGL(k_align_lk<64>, dim3(groups), dim3(64 * waves), lds, stream, pyr, vecs, a, (float2*)motion,
                       (int2*)block_match, (int)items, (int)chunk, sw);
  return hipGetLastError();
}

}  // namespace hmfsr
