// Per-burst forward merge kernels (one launch over a burst's output tiles),
// the normaliser-keeping forward of the adjoint and the streaming merge; the
// tile body is merge_tile.h.
#include "merge_tile.h"

namespace hmfsr {
namespace {

template <int MH, int THREADS, int RB>
__global__ __launch_bounds__(THREADS, (waves_per_simd<MH, THREADS>())) void k_merge(
    const uint16_t* __restrict__ frames, const float* __restrict__ motion,
    const float* __restrict__ rmin, Geometry g, MergeConsts mc, float* __restrict__ out) {
  __shared__ MergeSmem<MH> sm;
  const int tiles_x = (g.OW + MW - 1) / MW, n = tiles_x * ((g.OH + MH - 1) / MH);
  const int t = xcd_tile(blockIdx.x, n);
  merge_tile<MH, THREADS, TILE_PLAIN, RB>(frames, motion, rmin, g, mc, out, nullptr, StreamState{nullptr, nullptr, 0},
                                      t % tiles_x, t / tiles_x, sm);
}

// Forward that also keeps the normaliser for the adjoint (float64 accumulation).
template <int RB>
__global__ __launch_bounds__(256, 2) void k_merge_save(
    const uint16_t* __restrict__ frames, const float* __restrict__ motion,
    const float* __restrict__ rmin, Geometry g, MergeConsts mc, float* __restrict__ out,
    float* __restrict__ saved) {
  __shared__ MergeSmem<16> sm;
  const int tiles_x = (g.OW + MW - 1) / MW, n = tiles_x * ((g.OH + 15) / 16);
  const int t = xcd_tile(blockIdx.x, n);
  merge_tile<16, 256, TILE_SAVE, RB>(frames, motion, rmin, g, mc, out, saved, StreamState{nullptr, nullptr, 0},
                                 t % tiles_x, t / tiles_x, sm);
}

// Streaming form: frames from loop index st.first on are added to the state.
template <int RB>
__global__ __launch_bounds__(256, 4) void k_merge_stream(
    const uint16_t* __restrict__ frames, const float* __restrict__ motion,
    const float* __restrict__ rmin, Geometry g, MergeConsts mc, StreamState st) {
  __shared__ MergeSmem<16> sm;
  const int tiles_x = (g.OW + MW - 1) / MW, n = tiles_x * ((g.OH + 15) / 16);
  const int t = xcd_tile(blockIdx.x, n);
  merge_tile<16, 256, TILE_STREAM, RB>(frames, motion, rmin, g, mc, nullptr, nullptr, st, t % tiles_x, t / tiles_x,
                                   sm);
}

// eq. (1) on a streaming state: C = num / den per channel, mapped to [0, 1].
__global__ void k_stream_finish(const float* __restrict__ state, size_t plane, float black, float inv_range,
                                float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= plane) return;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    out[i + c * plane] = (state[i + c * plane] / state[i + (3 + c) * plane] - black) * inv_range;
}

template <int MH, int THREADS>
hipError_t launch_variant(const Geometry& g, const MergeConsts& mc, const uint16_t* frames,
                          const float* motion, const float* rmin, float* out, hipStream_t stream) {
  const dim3 grid(((g.OW + MW - 1) / MW) * ((g.OH + MH - 1) / MH));
  if (wide_raw_window(MH, THREADS, g.scale))
    hipLaunchKernelGGL((k_merge<MH, THREADS, 8>), grid, dim3(THREADS), 0, stream, frames, motion, rmin, g,
                       mc, out);
  else
    hipLaunchKernelGGL((k_merge<MH, THREADS, 4>), grid, dim3(THREADS), 0, stream, frames, motion, rmin, g,
                       mc, out);
  return hipGetLastError();
}

}  // namespace

const MergeVariant kMergeVariants[] = {
    {"64x32/256", 32, 256}, {"64x32/512", 32, 512}, {"64x16/256", 16, 256}, {"64x16/128", 16, 128},
};
const int kNumMergeVariants = sizeof(kMergeVariants) / sizeof(kMergeVariants[0]);

hipError_t launch_merge(int variant, const Geometry& g, const MergeConsts& mc, const uint16_t* frames,
                        const float* motion, const float* rmin, float* out, float* saved,
                        hipStream_t stream) {
  if (saved) {  // one tile shape keeps the normaliser
    const dim3 grid(((g.OW + MW - 1) / MW) * ((g.OH + 15) / 16));
    if (wide_raw_window(16, 256, g.scale))
      hipLaunchKernelGGL(k_merge_save<8>, grid, dim3(256), 0, stream, frames, motion, rmin, g, mc, out, saved);
    else
      hipLaunchKernelGGL(k_merge_save<4>, grid, dim3(256), 0, stream, frames, motion, rmin, g, mc, out, saved);
    return hipGetLastError();
  }
  switch (variant) {
    case 1: return launch_variant<32, 512>(g, mc, frames, motion, rmin, out, stream);
    case 2: return launch_variant<16, 256>(g, mc, frames, motion, rmin, out, stream);
    case 3: return launch_variant<16, 128>(g, mc, frames, motion, rmin, out, stream);
    default: return launch_variant<32, 256>(g, mc, frames, motion, rmin, out, stream);
  }
}

int merge_class(int variant, double scale) {
  return 2 * variant + (wide_raw_window(kMergeVariants[variant].rows, kMergeVariants[variant].threads, scale) ? 1 : 0);
}

int merge_tile_rows(int variant) { return kMergeVariants[variant].rows; }

hipError_t launch_merge_stream(const Geometry& g, const MergeConsts& mc, const uint16_t* frames,
                               const float* motion, const float* rmin, const float* state_in, float* state_out,
                               int first, hipStream_t stream) {
  const dim3 grid(((g.OW + MW - 1) / MW) * ((g.OH + 15) / 16));
  if (wide_raw_window(16, 256, g.scale))
    hipLaunchKernelGGL(k_merge_stream<8>, grid, dim3(256), 0, stream, frames, motion, rmin, g, mc,
                       StreamState{state_in, state_out, first});
  else
    hipLaunchKernelGGL(k_merge_stream<4>, grid, dim3(256), 0, stream, frames, motion, rmin, g, mc,
                       StreamState{state_in, state_out, first});
  return hipGetLastError();
}

hipError_t launch_stream_finish(const Geometry& g, const MergeConsts& mc, const float* state, float* out,
                                hipStream_t stream) {
  const size_t plane = (size_t)g.OH * g.OW;
  hipLaunchKernelGGL(k_stream_finish, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, stream, state, plane,
                     mc.black, mc.inv_range, out);
  return hipGetLastError();
}

}  // namespace hmfsr
