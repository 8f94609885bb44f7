// Tile alignment of a burst against its base frame (Sec. 3.2): a pyramid of
// integer 2x2 sums of the half-resolution luma, coarse-to-fine block matching
// by integer sum of squared differences, and Lucas-Kanade refinement of the
// finest level's vectors.
//
// Every integer step (pyramid, costs, the argmin and its tie rules) is exact,
// so the block-matching vectors are fully determined by the frames. The
// Lucas-Kanade normal matrix is an exact integer sum as well; its solve and
// the error image run in float64.
#include <stdint.h>

#include "device_util.h"
#include "hmfsr_internal.h"

namespace hmfsr {
namespace {

constexpr int kPyrEdge = 64;       // level-0 pixels per pyramid workgroup edge
constexpr int kAlignThreads = 256;

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
};

// Candidate key: cost, squared offset from the guess, scan index; the
// lexicographic minimum wins.
struct Key {
  unsigned long long ssd;
  int d2, k;
};

__device__ __forceinline__ bool key_less(const Key& a, const Key& b) {
  if (a.ssd != b.ssd) return a.ssd < b.ssd;
  if (a.d2 != b.d2) return a.d2 < b.d2;
  return a.k < b.k;
}

__device__ __forceinline__ Key shfl_key(const Key& a, int off) {
  Key o;
  const unsigned lo = __shfl_xor((unsigned)(a.ssd & 0xffffffffull), off, 64);
  const unsigned hi = __shfl_xor((unsigned)(a.ssd >> 32), off, 64);
  o.ssd = ((unsigned long long)hi << 32) | lo;
  o.d2 = __shfl_xor(a.d2, off, 64);
  o.k = __shfl_xor(a.k, off, 64);
  return o;
}

// One wave per block of one non-base frame; the lanes take the candidates.
// LDS per wave: the base block (B x B) and the frame's search region
// ((B + 2R)^2, edge-replicated).
__global__ __launch_bounds__(kAlignThreads) void k_align_match(const int32_t* __restrict__ pyr,
                                                               int2* __restrict__ vecs, MatchLevel ml, int ref,
                                                               long long fstride, long long vstride,
                                                               int items) {
  extern __shared__ int32_t smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int B = ml.B, R = ml.R, E = B + 2 * R, D = 2 * R + 1;
  int32_t* tpl = smem + wave * (B * B + E * E);
  int32_t* reg = tpl + B * B;
  const int blk = xcd_tile(blockIdx.x, gridDim.x);
  const int item = blk * (blockDim.x >> 6) + wave;
  const bool valid = item < items;
  const int per = ml.gby * ml.gbx;
  const int fi = valid ? item / per : 0;
  const int t = valid ? item - fi * per : 0;
  const int by = t / ml.gbx, bx = t - (t / ml.gbx) * ml.gbx;
  const int f = fi < ref ? fi : fi + 1;
  const int32_t* base = pyr + (long long)ref * fstride + ml.loff;
  const int32_t* img = pyr + (long long)f * fstride + ml.loff;
  int gx = 0, gy = 0;
  if (valid && ml.parent) {
    const int cy = min(((2 * by + 1) * B) / (4 * ml.pB), ml.pgby - 1);
    const int cx = min(((2 * bx + 1) * B) / (4 * ml.pB), ml.pgbx - 1);
    const int2 pv = vecs[(long long)f * vstride + ml.pvoff + (long long)cy * ml.pgbx + cx];
    gx = 2 * pv.x;
    gy = 2 * pv.y;
  }
  const int y0 = by * B, x0 = bx * B;
  const int nby = min(B, ml.h - y0), nbx = min(B, ml.w - x0);
  if (valid) {
    for (int r = 0; r < nby; ++r)
      if (lane < nbx) tpl[r * B + lane] = base[(long long)(y0 + r) * ml.w + x0 + lane];
    for (int r = 0; r < E; ++r) {
      const int yy = clampi(y0 + gy - R + r, 0, ml.h - 1);
      if (lane < E) {
        const int xx = clampi(x0 + gx - R + lane, 0, ml.w - 1);
        reg[r * E + lane] = img[(long long)yy * ml.w + xx];
      }
    }
  }
  __syncthreads();
  if (!valid) return;
  Key best{~0ull, 0x7fffffff, 0x7fffffff};
  for (int k = lane; k < D * D; k += 64) {
    const int dyi = k / D, dxi = k - (k / D) * D;  // offsets + R
    unsigned long long ssd = 0;
    for (int r = 0; r < nby; ++r) {
      const int32_t* tr = tpl + r * B;
      const int32_t* rr = reg + (r + dyi) * E + dxi;
      for (int c = 0; c < nbx; ++c) {
        const long long d = (long long)(rr[c] - tr[c]);
        ssd += (unsigned long long)(d * d);
      }
    }
    const int dx = dxi - R, dy = dyi - R;
    const Key cand{ssd, dx * dx + dy * dy, k};
    if (key_less(cand, best)) best = cand;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const Key o = shfl_key(best, off);
    if (key_less(o, best)) best = o;
  }
  if (lane == 0) {
    const int dyi = best.k / D, dxi = best.k - (best.k / D) * D;
    vecs[(long long)f * vstride + ml.voff + t] = make_int2(gx + dxi - R, gy + dyi - R);
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned lo = __shfl_xor((unsigned)((unsigned long long)v & 0xffffffffull), off, 64);
    const int hi = __shfl_xor((int)(v >> 32), off, 64);
    v += (long long)(((unsigned long long)(unsigned)hi << 32) | lo);
  }
  return v;
}

// One wave per (frame, tile). LDS per wave: the base window with a one-pixel
// edge-replicated border, for the central differences. The butterfly sums
// leave the same bits in every lane (addition commutes), so the update is
// uniform across the wave.
__global__ __launch_bounds__(kAlignThreads) void k_align_lk(const int32_t* __restrict__ pyr,
                                                            const int2* __restrict__ vecs, LkArgs a,
                                                            float2* __restrict__ motion,
                                                            int2* __restrict__ bm_out, int items, int sw) {
  extern __shared__ int32_t smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int32_t* S = smem + wave * sw * sw;
  const int blk = xcd_tile(blockIdx.x, gridDim.x);
  const int item = blk * (blockDim.x >> 6) + wave;
  const bool valid = item < items;
  const int per = a.TY * a.TX;
  const int f = valid ? item / per : 0;
  const int t = valid ? item - f * per : 0;
  const int ty = t / a.TX, tx = t - (t / a.TX) * a.TX;
  const bool work = valid && f != a.ref;
  const int wy0 = max(0, ty * a.B - a.m), wy1 = min(ty * a.B + a.B + a.m, a.h);
  const int wx0 = max(0, tx * a.B - a.m), wx1 = min(tx * a.B + a.B + a.m, a.w);
  const int WH = wy1 - wy0, WW = wx1 - wx0, SWW = WW + 2;
  const int32_t* base = pyr + (long long)a.ref * a.fstride;
  if (work) {
    for (int r = 0; r < WH + 2; ++r) {
      const int yy = clampi(wy0 - 1 + r, 0, a.h - 1);
      for (int c = lane; c < SWW; c += 64) S[r * SWW + c] = base[(long long)yy * a.w + clampi(wx0 - 1 + c, 0, a.w - 1)];
    }
  }
  __syncthreads();
  if (!valid) return;
  if (!work) {
    if (lane == 0) {
      motion[item] = make_float2(0.f, 0.f);
      if (bm_out) bm_out[item] = make_int2(0, 0);
    }
    return;
  }
  const int2 bm = vecs[(long long)f * a.vstride + a.voff0 + t];
  const int n_px = WH * WW;
  long long hxx = 0, hxy = 0, hyy = 0;
  for (int i = lane; i < n_px; i += 64) {
    const int r = i / WW, c = i - (i / WW) * WW;
    const int32_t* s = S + (r + 1) * SWW + c + 1;
    const long long dx = s[1] - s[-1], dy = s[SWW] - s[-SWW];
    hxx += dx * dx;
    hxy += dx * dy;
    hyy += dy * dy;
  }
  const double Hxx = (double)wave_sum_ll(hxx), Hxy = (double)wave_sum_ll(hxy), Hyy = (double)wave_sum_ll(hyy);
  // Singular-window test on the exact sums, rounded step by step as written
  // (no fused multiply-add), so that it is decided identically everywhere.
  const double tr = __dadd_rn(Hxx, Hyy);
  const double det = __dsub_rn(__dmul_rn(Hxx, Hyy), __dmul_rn(Hxy, Hxy));
  const double thr = __dmul_rn(__dmul_rn(1e-9, tr), tr);
  double vx = bm.x, vy = bm.y;
  if (tr > 0.0 && det > thr) {
    const int32_t* img = pyr + (long long)f * a.fstride;
    for (int it = 0; it < a.iters; ++it) {
      double sx = 0.0, sy = 0.0;
      for (int i = lane; i < n_px; i += 64) {
        const int r = i / WW, c = i - (i / WW) * WW;
        const int32_t* s = S + (r + 1) * SWW + c + 1;
        const double x = (double)(wx0 + c) + vx, y = (double)(wy0 + r) + vy;
        const double xf = floor(x), yf = floor(y);
        const double fx = x - xf, fy = y - yf;
        const int xi = (int)fmax(fmin(xf, 1e9), -1e9), yi = (int)fmax(fmin(yf, 1e9), -1e9);
        const int xa = clampi(xi, 0, a.w - 1), xb = clampi(xi + 1, 0, a.w - 1);
        const long long ya = (long long)clampi(yi, 0, a.h - 1) * a.w;
        const long long yb = (long long)clampi(yi + 1, 0, a.h - 1) * a.w;
        const double top = (1.0 - fx) * (double)img[ya + xa] + fx * (double)img[ya + xb];
        const double bot = (1.0 - fx) * (double)img[yb + xa] + fx * (double)img[yb + xb];
        const double err = (1.0 - fy) * top + fy * bot - (double)s[0];
        sx += (double)(s[1] - s[-1]) * err;
        sy += (double)(s[SWW] - s[-SWW]) * err;
      }
      sx = wave_sum(sx);
      sy = wave_sum(sy);
      // H and b here are 4x and 2x those of the half-gradient form.
      vx -= 2.0 * (Hyy * sx - Hxy * sy) / det;
      vy -= 2.0 * (Hxx * sy - Hxy * sx) / det;
    }
  }
  if (lane == 0) {
    motion[item] = make_float2((float)(2.0 * vx), (float)(2.0 * vy));
    if (bm_out) bm_out[item] = bm;
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
      const int E = ml.B + 2 * ml.R;
      const size_t lds = (size_t)(kAlignThreads / 64) * (ml.B * ml.B + E * E) * 4;
      const long long items = (long long)(ag.n - 1) * ml.gby * ml.gbx;
      hipLaunchKernelGGL(k_align_match, dim3(cdiv(items, kAlignThreads / 64)), dim3(kAlignThreads), lds, stream,
                         pyr, vecs, ml, ag.ref, ag.fstride, ag.vstride, (int)items);
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
  const int sw = a.B + 2 * a.m + 2;  // window edge with its border, at most
  const int waves = sw > 34 ? 2 : 4;  // keeps LDS within 64 KiB per workgroup
  const long long items = (long long)ag.n * a.TY * a.TX;
  const size_t lds = (size_t)waves * sw * sw * 4;
  hipLaunchKernelGGL(k_align_lk, dim3(cdiv(items, waves)), dim3(64 * waves), lds, stream, pyr, vecs, a,
                     (float2*)motion, (int2*)block_match, (int)items, sw);
  return hipGetLastError();
}

}  // namespace hmfsr
