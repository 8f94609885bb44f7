// Noise model (Sec. 5.2.2): Monte-Carlo tables of the modelled guide variance
// and of the squared difference of two 3x3 means, per brightness level, with
// the raw range's clipping; and the exact sum of a frame's raw values for the
// SNR-dependent tuning (Sec. 7.2).
#include <stdint.h>

#include "hmfsr_internal.h"

namespace hmfsr {
namespace {

constexpr int kThreads = 256;

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC 2011).
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
  constexpr unsigned M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += W0;
      k.y += W1;
    }
    const unsigned hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    const unsigned hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

// Four standard normals from one counter: uniforms (u + 1/2) 2^-32, paired
// by Box-Muller.
__device__ __forceinline__ void normals4(uint4 ctr, uint2 key, double z[4]) {
  const uint4 w = philox4x32_10(ctr, key);
  const double u0 = ((double)w.x + 0.5) * 0x1p-32, u1 = ((double)w.y + 0.5) * 0x1p-32;
  const double u2 = ((double)w.z + 0.5) * 0x1p-32, u3 = ((double)w.w + 0.5) * 0x1p-32;
  const double two_pi = 6.283185307179586;  // 2 pi rounded, as 2.0 * pi in float64
  const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
  const double t0 = two_pi * u1, t1 = two_pi * u3;
  z[0] = r0 * cos(t0);
  z[1] = r0 * sin(t0);
  z[2] = r1 * cos(t1);
  z[3] = r1 * sin(t1);
}

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kThreads / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Workgroup (bin, class): class 0 is an R or B guide pixel (one raw sample),
// class 1 the guide's green (the mean of two). Each thread takes patches
// tid, tid + 256, ...: two frames of nine guide pixels, normals consumed in
// the order ((frame * 9) + pixel) * k + sub from Philox calls
// (patch, bin, 16 class + j, 0).
__global__ __launch_bounds__(kThreads) void k_noise_table(double a, double b, double lo, int bins, int patches,
                                                          uint2 key, float* __restrict__ table) {
  __shared__ double red[kThreads / 64];
  const int bin = blockIdx.x, cls = blockIdx.y, k = cls + 1;
  const double mu = (double)bin / (double)(bins - 1);
  const double sd = sqrt(a * fmax(mu, 0.0) + b);
  double acc_s = 0.0, acc_d = 0.0;
  for (int p = threadIdx.x; p < patches; p += kThreads) {
    double g[2][9];
    double z[4];
    int q = 0;
    for (int f = 0; f < 2; ++f)
      for (int px = 0; px < 9; ++px) {
        double s = 0.0;
        for (int sub = 0; sub < k; ++sub, ++q) {
          if ((q & 3) == 0) normals4(make_uint4((unsigned)p, (unsigned)bin, 16u * cls + (q >> 2), 0u), key, z);
          const double x = fmin(fmax(mu + sd * z[q & 3], lo), 1.0);
          s = sub ? (s + x) / 2.0 : x;
        }
        g[f][px] = s;
      }
    double m[2], v[2];
    for (int f = 0; f < 2; ++f) {
      double t = 0.0;
      for (int px = 0; px < 9; ++px) t += g[f][px];
      m[f] = t / 9.0;
      double e = 0.0;
      for (int px = 0; px < 9; ++px) e += (g[f][px] - m[f]) * (g[f][px] - m[f]);
      v[f] = e / 8.0;
    }
    acc_s += 0.5 * (v[0] + v[1]);
    acc_d += (m[0] - m[1]) * (m[0] - m[1]);
  }
  const double ts = block_sum(acc_s, red);
  const double td = block_sum(acc_d, red);
  if (threadIdx.x == 0) {
    table[4 * bin + 2 * cls] = (float)(ts / (double)patches);
    table[4 * bin + 2 * cls + 1] = (float)(td / (double)patches);
  }
}

// Exact sum of n uint16 values (n even, 4-byte aligned): per-workgroup partial
// sums in a grid-stride loop over 32-bit pairs, then one workgroup adds them.
__global__ __launch_bounds__(kThreads) void k_frame_sum(const uint32_t* __restrict__ pairs, long long n_pairs,
                                                        unsigned long long* __restrict__ parts) {
  __shared__ unsigned long long red[kThreads / 64];
  unsigned long long acc = 0;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n_pairs; i += (long long)gridDim.x * kThreads) {
    const uint32_t w = pairs[i];
    acc += (w & 0xffffu) + (w >> 16);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned lo = __shfl_xor((unsigned)(acc & 0xffffffffull), off, 64);
    const unsigned hi = __shfl_xor((unsigned)(acc >> 32), off, 64);
    acc += ((unsigned long long)hi << 32) | lo;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kThreads / 64; ++w) t += red[w];
    parts[blockIdx.x] = t;
  }
}

// One wave adds the partial sums (integers: exact in any order).
__global__ __launch_bounds__(64) void k_sum_parts(const unsigned long long* __restrict__ parts, int n,
                                                  unsigned long long* __restrict__ sum) {
  unsigned long long t = 0;
  for (int i = threadIdx.x; i < n; i += 64) t += parts[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned lo = __shfl_xor((unsigned)(t & 0xffffffffull), off, 64);
    const unsigned hi = __shfl_xor((unsigned)(t >> 32), off, 64);
    t += ((unsigned long long)hi << 32) | lo;
  }
  if (threadIdx.x == 0) *sum = t;
}

}  // namespace

hipError_t launch_noise_table(double a, double b, double lo, int bins, int patches, unsigned long long seed,
                              float* table, hipStream_t stream) {
  const uint2 key = make_uint2((unsigned)(seed & 0xffffffffull), (unsigned)(seed >> 32));
  hipLaunchKernelGGL(k_noise_table, dim3(bins, 2), dim3(kThreads), 0, stream, a, b, lo, bins, patches, key, table);
  return hipGetLastError();
}

hipError_t launch_frame_sum(const uint16_t* frame, long long n, unsigned long long* parts, unsigned long long* sum,
                            hipStream_t stream) {
  const long long n_pairs = n / 2;
  const long long want = (n_pairs + kThreads * 8 - 1) / (kThreads * 8);
  const int groups = (int)(want < 1 ? 1 : (want > kFrameSumGroups ? kFrameSumGroups : want));
  hipLaunchKernelGGL(k_frame_sum, dim3(groups), dim3(kThreads), 0, stream, (const uint32_t*)frame, n_pairs, parts);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, stream, parts, groups, sum);
  return hipGetLastError();
}

}  // namespace hmfsr
