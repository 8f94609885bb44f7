// Per-tile motion prior (eq. 7-8) and the inspection map of Omega.
#include <math.h>

#include "hmfsr_internal.h"
#include "prior.h"

namespace hmfsr {
namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// eq. (7)-(8): rejection strength s1 or s2 per tile.
__device__ __forceinline__ void prior_one(const float* __restrict__ motion, const Geometry& g,
                                          const PriorConsts& pc, float* __restrict__ s_tile,
                                          unsigned char* __restrict__ mov, int n, int ty, int tx) {
  const size_t idx = ((size_t)n * g.TY + ty) * g.TX + tx;
  if (n == g.ref) {
    s_tile[idx] = 0.0f;
    mov[idx] = 0;
    return;
  }
  const bool moving = prior_moving(motion, g, pc.m_th, n, ty, tx);
  s_tile[idx] = moving ? pc.s1 : pc.s2;
  mov[idx] = moving;
}

__global__ void k_prior(const float* __restrict__ motion, Geometry g, PriorConsts pc,
                        float* __restrict__ s_tile, unsigned char* __restrict__ mov) {
  const int tx = blockIdx.x * blockDim.x + threadIdx.x;
  const int ty = blockIdx.y * blockDim.y + threadIdx.y;
  if (ty >= g.TY || tx >= g.TX) return;
  prior_one(motion, g, pc, s_tile, mov, blockIdx.z, ty, tx);
}

// Every (burst, frame, tile) of a batch; first[b] = first flat index of burst b.
__global__ void k_prior_batch(const BurstArgs* __restrict__ bursts, const int* __restrict__ first,
                              int n_bursts, int total) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int lo = 0, hi = n_bursts - 1;  // last burst with first[b] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= i) lo = mid; else hi = mid - 1;
  }
  const BurstArgs& b = bursts[lo];
  const int k = i - first[lo];
  const int per = b.g.TY * b.g.TX;
  const int n = k / per, t = k - n * per;
  prior_one(b.motion, b.g, b.pc, b.s_tile, b.mov, n, t / b.g.TX, t % b.g.TX);
}

// Omega per half-res pixel of every frame (inspection output).
__global__ void k_omega_map(const uint16_t* __restrict__ frames, Geometry g, OmegaConsts oc,
                            double* __restrict__ omega) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  const int I = blockIdx.y * blockDim.y + threadIdx.y;
  const int n = blockIdx.z;
  if (I >= g.h || J >= g.w) return;
  const uint16_t* f = frames + (size_t)n * g.H * g.W;
  int l[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const int qi = clampi(I + a - 1, 0, g.h - 1), qj = clampi(J + b - 1, 0, g.w - 1);
      const uint16_t* q = f + (size_t)(2 * qi) * g.W + 2 * qj;
      l[a][b] = (int)q[0] + (int)q[1] + (int)q[g.W] + (int)q[g.W + 1];
    }
  double oxx, oxy, oyy;
  omega_from_quads(l, oc, oxx, oxy, oyy);
  const size_t plane = (size_t)g.h * g.w;
  const size_t o = (size_t)n * 3 * plane + (size_t)I * g.w + J;
  omega[o] = oxx;
  omega[o + plane] = oxy;
  omega[o + 2 * plane] = oyy;
}

__global__ void k_fill(float* __restrict__ p, float v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_i32(int* __restrict__ p, int v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_fill_i32(int* p, int v, size_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, float v, size_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, v, n);
  return hipGetLastError();
}

namespace {
size_t a256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

size_t work_bytes(const Geometry& g) {
  const size_t plane = (size_t)g.h * g.w * sizeof(float);
  const size_t mu_plane = (size_t)g.h * (g.w + 2) * sizeof(uint2);
  return a256((size_t)g.TY * g.TX * g.n * sizeof(float)) + a256((size_t)g.TY * g.TX * g.n) +
         a256(plane * g.n) + a256(mu_plane * g.n) + a256(plane);
}

Work work_carve(void* base, const Geometry& g) {
  const size_t plane = (size_t)g.h * g.w * sizeof(float);
  char* p = (char*)base;
  Work w;
  w.s_tile = (float*)p;
  p += a256((size_t)g.TY * g.TX * g.n * sizeof(float));
  w.mov = (unsigned char*)p;
  p += a256((size_t)g.TY * g.TX * g.n);
  w.rmin = (float*)p;
  p += a256(plane * g.n);
  w.gmu = (uint2*)p;
  p += a256((size_t)g.h * (g.w + 2) * sizeof(uint2) * g.n);
  w.gref = (float*)p;
  return w;
}

hipError_t launch_prior(const Geometry& g, const PriorConsts& pc, const float* motion, const Work& w,
                        hipStream_t stream) {
  const dim3 blk(16, 16);
  const dim3 grid((g.TX + 15) / 16, (g.TY + 15) / 16, g.n);
  hipLaunchKernelGGL(k_prior, grid, blk, 0, stream, motion, g, pc, w.s_tile, w.mov);
  return hipGetLastError();
}

hipError_t launch_prior_batch(const BurstArgs* bursts, const int* first, int n_bursts, int total,
                              hipStream_t stream) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prior_batch, dim3((total + 255) / 256), dim3(256), 0, stream, bursts, first,
                     n_bursts, total);
  return hipGetLastError();
}

hipError_t launch_omega_map(const Geometry& g, const OmegaConsts& oc, const uint16_t* frames,
                            double* omega, hipStream_t stream) {
  const dim3 blk(16, 16);
  const dim3 grid((g.w + 15) / 16, (g.h + 15) / 16, g.n);
  hipLaunchKernelGGL(k_omega_map, grid, blk, 0, stream, frames, g, oc, omega);
  return hipGetLastError();
}

}  // namespace hmfsr
