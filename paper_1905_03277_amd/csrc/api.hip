// C ABI entry points: validation, per-device workspace, single-burst dispatch,
// inspection maps, profiling.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "host.h"

namespace hmfsr {

std::mutex g_mutex;
DeviceState g_dev[kMaxDevices];
Timing g_timing;

hipEvent_t Timing::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

namespace {

bool finite(float v) { return isfinite(v) != 0; }

// Colours of the 2x2 mosaic read row by row: 0 R, 1 G, 2 B.
bool cfa_colours(int cfa, int out[4]) {
  static const int table[4][4] = {{0, 1, 1, 2}, {1, 0, 2, 1}, {1, 2, 0, 1}, {2, 1, 1, 0}};
  if (cfa < 0 || cfa > 3) return false;
  for (int k = 0; k < 4; ++k) out[k] = table[cfa][k];
  return true;
}

double range_of(const hmfsr_desc* d) { return (double)d->white_level - (double)d->black_level; }

}  // namespace

hmfsr_status validate_desc(const hmfsr_desc* d) {
  if (!d) return HMFSR_E_INVALID;
  if (d->n_frames < 1 || d->n_frames > 4096) return HMFSR_E_INVALID;
  if (d->ref_frame < 0 || d->ref_frame >= d->n_frames) return HMFSR_E_INVALID;
  if (d->height < 4 || d->width < 4 || d->height > 32768 || d->width > 32768) return HMFSR_E_INVALID;
  if ((d->height & 1) || (d->width & 1)) return HMFSR_E_INVALID;
  if (!finite(d->black_level) || !finite(d->white_level) || !(d->black_level < d->white_level))
    return HMFSR_E_INVALID;
  if (!finite(d->noise_a) || !finite(d->noise_b) || d->noise_a < 0.f || !(d->noise_b > 0.f))
    return HMFSR_E_INVALID;
  if (d->tile_size < 8 || d->tile_size > 256 || (d->tile_size & 1)) return HMFSR_E_INVALID;
  if (!finite(d->scale) || !(d->scale >= 1.f) || d->scale > 8.f) return HMFSR_E_INVALID;
  const double s = (double)d->scale;
  if (d->out_height != (int32_t)floor((double)d->height * s + 0.5) ||
      d->out_width != (int32_t)floor((double)d->width * s + 0.5))
    return HMFSR_E_INVALID;
  if (d->noise_table ? (d->noise_bins < 2 || d->noise_bins > 65536 || ((uintptr_t)d->noise_table & 3))
                     : d->noise_bins != 0)
    return HMFSR_E_INVALID;
  int cols[4];
  if (!cfa_colours(d->cfa, cols)) return HMFSR_E_UNSUPPORTED;
  return HMFSR_OK;
}

hmfsr_status validate(const hmfsr_desc* d, const hmfsr_tuning* t) {
  if (!d || !t) return HMFSR_E_INVALID;
  const hmfsr_status st = validate_desc(d);
  if (st != HMFSR_OK) return st;
  const float vals[11] = {t->k_detail, t->k_denoise, t->d_th, t->d_tr, t->k_stretch,
                          t->k_shrink, t->s, t->t, t->s_motion, t->m_th, t->hf_ratio};
  for (float v : vals)
    if (!finite(v)) return HMFSR_E_INVALID;
  if (!(t->k_detail > 0.f) || !(t->k_denoise > 0.f) || !(t->d_tr > 0.f) || !(t->k_stretch > 0.f) ||
      !(t->k_shrink > 0.f) || t->s < 0.f || t->s_motion < 0.f || t->m_th < 0.f || t->hf_ratio < 0.f)
    return HMFSR_E_INVALID;
  return HMFSR_OK;
}

Geometry make_geometry(const hmfsr_desc* d) {
  Geometry g;
  g.n = d->n_frames;
  g.H = d->height;
  g.W = d->width;
  g.h = g.H / 2;
  g.w = g.W / 2;
  g.ref = d->ref_frame;
  g.T = d->tile_size;
  g.TY = (g.H + g.T - 1) / g.T;
  g.TX = (g.W + g.T - 1) / g.T;
  g.OH = d->out_height;
  g.OW = d->out_width;
  cfa_colours(d->cfa, g.colour);
  int ng = 0;
  for (int k = 0; k < 4; ++k) {
    if (g.colour[k] == 0) g.red_pos = k;
    if (g.colour[k] == 2) g.blue_pos = k;
    if (g.colour[k] == 1) g.green_pos[ng++] = k;
  }
  g.scale = (double)d->scale;
  return g;
}

OmegaConsts make_omega(const hmfsr_desc* d, const hmfsr_tuning* t) {
  OmegaConsts c;
  const double kd = t->k_detail;
  c.kd_st = kd * (double)t->k_stretch;
  c.kd_sh = kd / (double)t->k_shrink;
  c.kd_dn = kd * (double)t->k_denoise;
  c.d_th = t->d_th;
  c.inv_16_range_dtr = 1.0 / (16.0 * range_of(d) * (double)t->d_tr);
  return c;
}

PriorConsts make_prior(const hmfsr_tuning* t) {
  PriorConsts p;
  p.m_th = t->m_th;
  p.s1 = t->s_motion;
  p.s2 = t->s;
  return p;
}

RobustConsts make_robust(const hmfsr_desc* d, const hmfsr_tuning* t) {
  RobustConsts r;
  const double range = range_of(d);
  r.black = d->black_level;
  r.a_r = (float)((double)d->noise_a * range);
  r.b_r = (float)((double)d->noise_b * range * range);
  r.t = t->t;
  r.hf = t->hf_ratio;
  r.ntab = d->noise_table;
  r.nbins = d->noise_bins;
  r.inv_range = (float)(1.0 / range);
  r.range2 = (float)(range * range);
  return r;
}

MergeConsts make_merge(const hmfsr_desc* d, const hmfsr_tuning* t, const Geometry& g) {
  MergeConsts m;
  m.om = make_omega(d, t);
  m.black = d->black_level;
  m.inv_range = (float)(1.0 / range_of(d));
  m.col4 = 0;
  for (int k = 0; k < 4; ++k) m.col4 |= g.colour[k] << (2 * k);
  return m;
}

hmfsr_status current_device(int* dev_out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HMFSR_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return HMFSR_E_UNSUPPORTED;
  DeviceState& st = g_dev[dev];
  if (st.checked == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return HMFSR_E_HIP;
    st.checked = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
    st.cus = prop.multiProcessorCount;
  }
  if (st.checked < 0) return HMFSR_E_UNSUPPORTED;
  *dev_out = dev;
  return HMFSR_OK;
}

namespace {
// Growing a workspace frees the old one only after the stream that may still
// use it has drained.
hmfsr_status grow(void*& buf, size_t& have, size_t bytes, hipStream_t stream, void** out) {
  if (have < bytes) {
    if (buf) {
      if (hipStreamSynchronize(stream) != hipSuccess) return HMFSR_E_HIP;
      (void)hipFree(buf);
      buf = nullptr;
      have = 0;
    }
    if (hipMalloc(&buf, bytes) != hipSuccess) {
      (void)hipGetLastError();
      buf = nullptr;
      return HMFSR_E_NOMEM;
    }
    have = bytes;
  }
  *out = buf;
  return HMFSR_OK;
}
}  // namespace

hmfsr_status workspace(int dev, size_t bytes, hipStream_t stream, void** out) {
  return grow(g_dev[dev].workspace, g_dev[dev].workspace_bytes, bytes, stream, out);
}

hmfsr_status bwd_workspace(int dev, size_t bytes, hipStream_t stream, void** out) {
  return grow(g_dev[dev].bwd_ws, g_dev[dev].bwd_ws_bytes, bytes, stream, out);
}

hmfsr_status stream_workspace(int dev, size_t bytes, hipStream_t stream, void** out) {
  return grow(g_dev[dev].stream_ws, g_dev[dev].stream_ws_bytes, bytes, stream, out);
}

hmfsr_status align_workspace(int dev, size_t bytes, hipStream_t stream, void** out) {
  return grow(g_dev[dev].align_ws, g_dev[dev].align_ws_bytes, bytes, stream, out);
}

hmfsr_status grow_buffer(void*& buf, size_t& have, size_t bytes, hipStream_t stream, void** out) {
  return grow(buf, have, bytes, stream, out);
}

namespace {
// Pyramid sizes and block grids: level l + 1 holds the 2x2 sums of level l
// while it still holds a whole coarse block, up to params->levels levels.
hmfsr_status make_align_geom(const hmfsr_desc* d, const hmfsr_align_params* p, AlignGeom* ag) {
  if (d->tile_size > 64) return HMFSR_E_INVALID;
  if (p->levels < 1 || p->levels > kAlignMaxLevels || p->radius_coarse < 1 || p->radius_coarse > 8 ||
      p->radius_fine < 1 || p->radius_fine > 8 || p->lk_iterations < 0 || p->lk_iterations > 16 ||
      !(p->gate >= 0.0f && p->gate <= 1000.0f))
    return HMFSR_E_INVALID;
  AlignGeom a;
  memset(&a, 0, sizeof(a));
  a.n = d->n_frames;
  a.ref = d->ref_frame;
  a.lh[0] = d->height / 2;
  a.lw[0] = d->width / 2;
  a.L = 1;
  while (a.L < p->levels) {
    const int nh = a.lh[a.L - 1] / 2, nw = a.lw[a.L - 1] / 2;
    if (nh < kAlignCoarseBlock || nw < kAlignCoarseBlock) break;
    a.lh[a.L] = nh;
    a.lw[a.L] = nw;
    ++a.L;
  }
  long long off = 0, voff = 0;
  for (int l = 0; l < a.L; ++l) {
    a.blk[l] = l == 0 ? d->tile_size / 2 : kAlignCoarseBlock;
    a.gby[l] = (a.lh[l] + a.blk[l] - 1) / a.blk[l];
    a.gbx[l] = (a.lw[l] + a.blk[l] - 1) / a.blk[l];
    a.loff[l] = off;
    off += (long long)a.lh[l] * a.lw[l];
    a.voff[l] = voff;
    voff += (long long)a.gby[l] * a.gbx[l];
  }
  a.fstride = (off + 63) / 64 * 64;
  a.vstride = (voff + 31) / 32 * 32;
  if ((long long)a.n * a.gby[0] * a.gbx[0] >= (1ll << 31)) return HMFSR_E_INVALID;  // work items are int
  a.radius_coarse = p->radius_coarse;
  a.radius_fine = p->radius_fine;
  a.lk_iterations = p->lk_iterations;
  const double kappa = (double)p->gate;
  a.gate_k12 = (12.0 * kappa) * kappa;
  a.na = (double)d->noise_a;
  a.nb = (double)d->noise_b;
  a.black = (double)d->black_level;
  a.rng = (double)d->white_level - (double)d->black_level;
  *ag = a;
  return HMFSR_OK;
}
}  // namespace

hmfsr_status run_merge(const hmfsr_desc* desc, const hmfsr_tuning* tuning, const Geometry& g,
                       const uint16_t* frames, const float* motion, float* out, float* saved,
                       const Work& w, int variant, hipStream_t s, bool profiled) {
  const PriorConsts pc = make_prior(tuning);
  const RobustConsts rc = make_robust(desc, tuning);
  const MergeConsts mc = make_merge(desc, tuning, g);
  auto run = [&](int stage, auto fn) { return profiled ? timed(stage, s, fn) : fn(); };
  if (run(HMFSR_STAGE_PRIOR, [&] { return launch_prior(g, pc, motion, w, s); }) != hipSuccess)
    return HMFSR_E_HIP;
  if (run(HMFSR_STAGE_ROBUST, [&] { return launch_robust(g, rc, frames, motion, w, w.rmin, nullptr, s); }) !=
      hipSuccess)
    return HMFSR_E_HIP;
  if (run(HMFSR_STAGE_MERGE, [&] { return launch_merge(variant, g, mc, frames, motion, w.rmin, out, saved, s); }) !=
      hipSuccess)
    return HMFSR_E_HIP;
  return HMFSR_OK;
}

}  // namespace hmfsr

using namespace hmfsr;

extern "C" {

hmfsr_status hmfsr_merge(const hmfsr_desc* desc, const hmfsr_tuning* tuning, const uint16_t* frames,
                         const float* motion, float* out, float* saved, void* stream) {
  hmfsr_status st = validate(desc, tuning);
  if (st != HMFSR_OK) return st;
  if (!frames || !motion || !out) return HMFSR_E_INVALID;
  if (((uintptr_t)frames & 3) || ((uintptr_t)motion & 3) || ((uintptr_t)out & 3) || ((uintptr_t)saved & 7))
    return HMFSR_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  if ((st = current_device(&dev)) != HMFSR_OK) return st;
  const Geometry g = make_geometry(desc);
  void* ws = nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (debug_enabled() && (st = debug_check_motion(dev, motion, g.n, g.ref, g.TY, g.TX, s)) != HMFSR_OK) return st;
  if ((st = workspace(dev, work_bytes(g), s, &ws)) != HMFSR_OK) return st;
  return run_merge(desc, tuning, g, frames, motion, out, saved, work_carve(ws, g), merge_variant(g), s);
}

hmfsr_status hmfsr_stream_begin(const hmfsr_desc* desc, const hmfsr_tuning* tuning, const uint16_t* base_frame,
                                float* state, void* stream) {
  hmfsr_status st = validate(desc, tuning);
  if (st != HMFSR_OK) return st;
  if (!base_frame || !state || ((uintptr_t)base_frame & 3) || ((uintptr_t)state & 3)) return HMFSR_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  if ((st = current_device(&dev)) != HMFSR_OK) return st;
  Geometry g = make_geometry(desc);
  g.n = 1;
  g.ref = 0;
  hipStream_t s = (hipStream_t)stream;
  // the base frame alone: its weights are 1 and it reads no motion or R_hat
  return timed(HMFSR_STAGE_MERGE, s, [&] {
           return launch_merge_stream(g, make_merge(desc, tuning, g), base_frame, nullptr, nullptr, nullptr,
                                      state, 0, s);
         }) == hipSuccess
             ? HMFSR_OK
             : HMFSR_E_HIP;
}

hmfsr_status hmfsr_stream_add(const hmfsr_desc* desc, const hmfsr_tuning* tuning, const uint16_t* base_frame,
                              const uint16_t* frame, const float* motion, float* state, void* stream) {
  hmfsr_status st = validate(desc, tuning);
  if (st != HMFSR_OK) return st;
  if (!base_frame || !frame || !motion || !state) return HMFSR_E_INVALID;
  for (const void* p : {(const void*)base_frame, (const void*)frame, (const void*)motion, (const void*)state})
    if ((uintptr_t)p & 3) return HMFSR_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  if ((st = current_device(&dev)) != HMFSR_OK) return st;
  // a two-frame view [base, frame] in the library's stream workspace
  Geometry g = make_geometry(desc);
  g.n = 2;
  g.ref = 0;
  const size_t fbytes = (size_t)g.H * g.W * sizeof(uint16_t);
  const size_t mbytes = (size_t)g.TY * g.TX * 2 * sizeof(float);
  const size_t off_m = (2 * fbytes + 255) / 256 * 256, off_w = off_m + (2 * mbytes + 255) / 256 * 256;
  hipStream_t s = (hipStream_t)stream;
  if (debug_enabled() && (st = debug_check_motion(dev, motion, 1, -1, g.TY, g.TX, s)) != HMFSR_OK) return st;
  void* ws = nullptr;
  if ((st = stream_workspace(dev, off_w + work_bytes(g), s, &ws)) != HMFSR_OK) return st;
  uint16_t* frames = (uint16_t*)ws;
  float* mo = (float*)((char*)ws + off_m);
  const Work w = work_carve((char*)ws + off_w, g);
  if (hipMemcpyAsync(frames, base_frame, fbytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(frames + (size_t)g.H * g.W, frame, fbytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync((char*)mo + mbytes, motion, mbytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return HMFSR_E_HIP;
  const PriorConsts pc = make_prior(tuning);
  const RobustConsts rc = make_robust(desc, tuning);
  const MergeConsts mc = make_merge(desc, tuning, g);
  if (timed(HMFSR_STAGE_PRIOR, s, [&] { return launch_prior(g, pc, mo, w, s); }) != hipSuccess ||
      timed(HMFSR_STAGE_ROBUST, s, [&] {
        return launch_robust(g, rc, frames, mo, w, w.rmin, nullptr, s);
      }) != hipSuccess ||
      timed(HMFSR_STAGE_MERGE, s, [&] {
        return launch_merge_stream(g, mc, frames, mo, w.rmin, state, state, 1, s);
      }) != hipSuccess)
    return HMFSR_E_HIP;
  return HMFSR_OK;
}

hmfsr_status hmfsr_stream_end(const hmfsr_desc* desc, const hmfsr_tuning* tuning, const float* state, float* out,
                              void* stream) {
  hmfsr_status st = validate(desc, tuning);
  if (st != HMFSR_OK) return st;
  if (!state || !out || ((uintptr_t)state & 3) || ((uintptr_t)out & 3)) return HMFSR_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  if ((st = current_device(&dev)) != HMFSR_OK) return st;
  const Geometry g = make_geometry(desc);
  return launch_stream_finish(g, make_merge(desc, tuning, g), state, out, (hipStream_t)stream) == hipSuccess
             ? HMFSR_OK
             : HMFSR_E_HIP;
}

hmfsr_status hmfsr_merge_backward(const hmfsr_desc* desc, const hmfsr_tuning* tuning,
                                  const uint16_t* frames, const float* motion, const float* saved,
                                  const float* grad_out, float* grad_tuning, float* grad_motion,
                                  void* stream) {
  hmfsr_status st = validate(desc, tuning);
  if (st != HMFSR_OK) return st;
  if (!frames || !motion || !grad_out || !grad_tuning || !grad_motion) return HMFSR_E_INVALID;
  for (const void* p : {(const void*)frames, (const void*)motion, (const void*)grad_out,
                        (const void*)grad_tuning, (const void*)grad_motion})
    if ((uintptr_t)p & 3) return HMFSR_E_INVALID;
  if ((uintptr_t)saved & 7) return HMFSR_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  if ((st = current_device(&dev)) != HMFSR_OK) return st;
  const Geometry g = make_geometry(desc);
  hipStream_t s = (hipStream_t)stream;
  if (debug_enabled() && (st = debug_check_motion(dev, motion, g.n, g.ref, g.TY, g.TX, s)) != HMFSR_OK) return st;
  void* ws = nullptr;
  const bool need_saved = saved == nullptr;
  if ((st = bwd_workspace(dev, bwd_bytes(g, need_saved), s, &ws)) != HMFSR_OK) return st;
  const BwdWork w = bwd_carve(ws, g, need_saved);
  const PriorConsts pc = make_prior(tuning);
  const RobustConsts rc = make_robust(desc, tuning);
  const MergeConsts mc = make_merge(desc, tuning, g);
  BwdConsts bc;
  bc.kd = tuning->k_detail;
  bc.kn = tuning->k_denoise;
  bc.kst = tuning->k_stretch;
  bc.ksh = tuning->k_shrink;
  bc.sl = mc.om.inv_16_range_dtr / (double)tuning->d_tr;
  bc.tiles_x = (g.OW + 63) / 64;
  bc.tiles_y = (g.OH + kBwdRows - 1) / kBwdRows;
  bc.n_tiles = bc.tiles_x * bc.tiles_y;
  if (timed(HMFSR_STAGE_PRIOR, s, [&] { return launch_prior(g, pc, motion, w.fwd, s); }) != hipSuccess)
    return HMFSR_E_HIP;
  if (timed(HMFSR_STAGE_ROBUST, s, [&] {
        return launch_robust(g, rc, frames, motion, w.fwd, w.fwd.rmin, w.rmap, s);
      }) != hipSuccess)
    return HMFSR_E_HIP;
  if (need_saved) {
    if (timed(HMFSR_STAGE_MERGE, s, [&] {
          return launch_merge(merge_variant(g), g, mc, frames, motion, w.fwd.rmin, nullptr, w.saved, s);
        }) != hipSuccess)
      return HMFSR_E_HIP;
    saved = w.saved;
  }
  if (timed(HMFSR_STAGE_MERGE_BWD, s, [&] {
        return launch_merge_bwd(g, mc, bc, frames, motion, w.fwd.rmin, saved, grad_out, w, s);
      }) != hipSuccess)
    return HMFSR_E_HIP;
  if (timed(HMFSR_STAGE_ROBUST_BWD, s, [&] {
        return launch_robust_bwd(g, rc, pc, bc, frames, motion, w, s);
      }) != hipSuccess)
    return HMFSR_E_HIP;
  if (timed(HMFSR_STAGE_GRAD_REDUCE, s, [&] {
        return launch_grad_reduce(g, bc, w, grad_tuning, grad_motion, s);
      }) != hipSuccess)
    return HMFSR_E_HIP;
  return HMFSR_OK;
}

hmfsr_status hmfsr_merge_maps(const hmfsr_desc* desc, const hmfsr_tuning* tuning,
                              const uint16_t* frames, const float* motion, double* omega,
                              float* robust, float* robust_min, float* s_tile, void* stream) {
  hmfsr_status st = validate(desc, tuning);
  if (st != HMFSR_OK) return st;
  if (!frames || !motion) return HMFSR_E_INVALID;
  if (((uintptr_t)frames & 3) || ((uintptr_t)motion & 3)) return HMFSR_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  if ((st = current_device(&dev)) != HMFSR_OK) return st;
  const Geometry g = make_geometry(desc);
  void* ws = nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (debug_enabled() && (st = debug_check_motion(dev, motion, g.n, g.ref, g.TY, g.TX, s)) != HMFSR_OK) return st;
  if ((st = workspace(dev, work_bytes(g), s, &ws)) != HMFSR_OK) return st;
  const Work w = work_carve(ws, g);
  const size_t plane = (size_t)g.h * g.w;
  if (omega && launch_omega_map(g, make_omega(desc, tuning), frames, omega, s) != hipSuccess)
    return HMFSR_E_HIP;
  if (launch_prior(g, make_prior(tuning), motion, w, s) != hipSuccess) return HMFSR_E_HIP;
  float* rmin = robust_min ? robust_min : w.rmin;
  if (launch_robust(g, make_robust(desc, tuning), frames, motion, w, rmin, robust, s) !=
      hipSuccess)
    return HMFSR_E_HIP;
  // the base frame's robustness is 1 by definition
  for (float* m : {robust, robust_min}) {
    if (!m) continue;
    if (launch_fill(m + g.ref * plane, 1.0f, plane, s) != hipSuccess) return HMFSR_E_HIP;
  }
  if (s_tile && hipMemcpyAsync(s_tile, w.s_tile, (size_t)g.TY * g.TX * g.n * sizeof(float),
                               hipMemcpyDeviceToDevice, s) != hipSuccess)
    return HMFSR_E_HIP;
  return HMFSR_OK;
}

hmfsr_status hmfsr_align(const hmfsr_desc* desc, const hmfsr_align_params* params, const uint16_t* frames,
                         float* motion, int32_t* block_match, void* stream) {
  hmfsr_status st = validate_desc(desc);
  if (st != HMFSR_OK) return st;
  if (!frames || !motion || ((uintptr_t)frames & 3) || ((uintptr_t)motion & 7) || ((uintptr_t)block_match & 7))
    return HMFSR_E_INVALID;
  const hmfsr_align_params defaults = {4, 4, 2, 3, 4.0f};
  AlignGeom ag;
  if ((st = make_align_geom(desc, params ? params : &defaults, &ag)) != HMFSR_OK) return st;
  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  if ((st = current_device(&dev)) != HMFSR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  void* ws = nullptr;
  if ((st = align_workspace(dev, align_bytes(ag), s, &ws)) != HMFSR_OK) return st;
  return timed(HMFSR_STAGE_ALIGN, s, [&] {
           return launch_align(ag, frames, desc->height, desc->width, ws, motion, block_match, s);
         }) == hipSuccess
             ? HMFSR_OK
             : HMFSR_E_HIP;
}

hmfsr_status hmfsr_noise_table(const hmfsr_desc* desc, int32_t bins, int32_t patches, uint64_t seed, float* table,
                               void* stream) {
  hmfsr_status st = validate_desc(desc);
  if (st != HMFSR_OK) return st;
  if (bins < 2 || bins > 65536 || patches < 1 || patches > (1 << 24) || !table || ((uintptr_t)table & 3))
    return HMFSR_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  if ((st = current_device(&dev)) != HMFSR_OK) return st;
  const double lo = -(double)desc->black_level / ((double)desc->white_level - (double)desc->black_level);
  return launch_noise_table((double)desc->noise_a, (double)desc->noise_b, lo, bins, patches,
                            (unsigned long long)seed, table, (hipStream_t)stream) == hipSuccess
             ? HMFSR_OK
             : HMFSR_E_HIP;
}

hmfsr_status hmfsr_auto_tuning(const hmfsr_desc* desc, const uint16_t* frames, hmfsr_tuning* tuning,
                               int32_t* tile_size, double* snr_out, void* stream) {
  hmfsr_status st = validate_desc(desc);
  if (st != HMFSR_OK) return st;
  if (!frames || ((uintptr_t)frames & 3) || !tuning) return HMFSR_E_INVALID;
  unsigned long long total = 0;
  {
    std::lock_guard<std::mutex> lock(g_mutex);
    int dev = 0;
    if ((st = current_device(&dev)) != HMFSR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    void* ws = nullptr;
    DeviceState& ds = g_dev[dev];
    if ((st = grow_buffer(ds.sum_ws, ds.sum_ws_bytes, (kFrameSumGroups + 1) * sizeof(unsigned long long), s, &ws)) !=
        HMFSR_OK)
      return st;
    unsigned long long* parts = (unsigned long long*)ws;
    const long long n = (long long)desc->height * desc->width;
    if (launch_frame_sum(frames + (size_t)desc->ref_frame * n, n, parts, parts + kFrameSumGroups, s) != hipSuccess ||
        hipMemcpyAsync(&total, parts + kFrameSumGroups, sizeof(total), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return HMFSR_E_HIP;
  }
  // SNR at the mean brightness, rounded operation by operation (one statement
  // per operation: no contraction)
  const double n = (double)desc->height * (double)desc->width;
  const double mean_raw = (double)total / n;
  const double black = desc->black_level, white = desc->white_level;
  const double mu = (mean_raw - black) / (white - black);
  double var = (double)desc->noise_a * fmax(mu, 0.0);
  var = var + (double)desc->noise_b;
  const double snr = mu / sqrt(var);
  double f = (snr - 6.0) / (30.0 - 6.0);
  f = fmin(fmax(f, 0.0), 1.0);
  auto lerp = [f](double lo, double hi) {
    const double p = (1.0 - f) * lo;
    const double q = f * hi;
    return (float)(p + q);
  };
  hmfsr_tuning t;
  t.k_detail = lerp(0.33, 0.25);
  t.k_denoise = lerp(5.0, 3.0);
  t.d_th = lerp(0.010, 0.001);
  t.d_tr = lerp(0.020, 0.006);
  t.k_stretch = 4.f;
  t.k_shrink = 2.f;
  t.s = 2.f;
  t.t = 0.12f;
  t.s_motion = 12.f;
  t.m_th = 0.8f;
  t.hf_ratio = 0.f;
  *tuning = t;
  if (tile_size) *tile_size = snr < 14.0 ? 64 : (snr < 22.0 ? 32 : 16);
  if (snr_out) *snr_out = snr;
  return HMFSR_OK;
}

const char* hmfsr_strerror(hmfsr_status status) {
  switch (status) {
    case HMFSR_OK: return "HMFSR_OK";
    case HMFSR_E_INVALID: return "HMFSR_E_INVALID: invalid descriptor, tuning or pointer";
    case HMFSR_E_UNSUPPORTED: return "HMFSR_E_UNSUPPORTED: unknown CFA or device is not gfx950";
    case HMFSR_E_HIP: return "HMFSR_E_HIP: HIP runtime or launch error";
    case HMFSR_E_NOMEM: return "HMFSR_E_NOMEM: workspace allocation failed";
    case HMFSR_E_DATA: return "HMFSR_E_DATA: device data failed an HMFSR_DEBUG check (non-finite motion)";
    case HMFSR_E_TOO_LARGE:
      return "HMFSR_E_TOO_LARGE: the burst's maps exceed hmfsr_merge_noalloc's static scratch (64 MiB)";
  }
  return "HMFSR: unknown status";
}

int32_t hmfsr_version(void) { return HMFSR_VERSION; }

hmfsr_status hmfsr_profile_begin(void) {
  std::lock_guard<std::mutex> lock(g_mutex);
  for (auto& p : g_timing.pairs) {
    g_timing.pool.push_back(p.a);
    g_timing.pool.push_back(p.b);
  }
  g_timing.pairs.clear();
  g_timing.on = true;
  return HMFSR_OK;
}

hmfsr_status hmfsr_profile_end(hmfsr_stage_times* out) {
  std::lock_guard<std::mutex> lock(g_mutex);
  g_timing.on = false;
  if (!out) return HMFSR_E_INVALID;
  memset(out, 0, sizeof(*out));
  hmfsr_status st = HMFSR_OK;
  for (auto& p : g_timing.pairs) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) {
      st = HMFSR_E_HIP;
    } else if (p.stage >= 0 && p.stage < HMFSR_NUM_STAGES) {
      out->ms_total[p.stage] += ms;
      out->launches[p.stage] += 1;
    }
    g_timing.pool.push_back(p.a);
    g_timing.pool.push_back(p.b);
  }
  g_timing.pairs.clear();
  return st;
}

void hmfsr_release(void) {
  std::lock_guard<std::mutex> lock(g_mutex);
  int cur = 0;
  const bool have_cur = hipGetDevice(&cur) == hipSuccess;
  for (int d = 0; d < kMaxDevices; ++d) {
    DeviceState& st = g_dev[d];
    if (!st.workspace && !st.batch_ws && !st.bwd_ws && !st.stream_ws && !st.align_ws && !st.sum_ws && !st.debug_ws &&
        !st.plan.exec && !st.capture_stream)
      continue;
    if (hipSetDevice(d) != hipSuccess) continue;
    if (st.plan.exec) (void)hipGraphExecDestroy(st.plan.exec);
    if (st.plan.graph) (void)hipGraphDestroy(st.plan.graph);
    st.plan = BatchPlan();
    if (st.workspace) (void)hipFree(st.workspace);
    if (st.batch_ws) (void)hipFree(st.batch_ws);
    if (st.bwd_ws) (void)hipFree(st.bwd_ws);
    if (st.stream_ws) (void)hipFree(st.stream_ws);
    st.stream_ws = nullptr;
    st.stream_ws_bytes = 0;
    if (st.align_ws) (void)hipFree(st.align_ws);
    st.align_ws = nullptr;
    st.align_ws_bytes = 0;
    if (st.sum_ws) (void)hipFree(st.sum_ws);
    st.sum_ws = nullptr;
    st.sum_ws_bytes = 0;
    if (st.debug_ws) (void)hipFree(st.debug_ws);
    st.debug_ws = nullptr;
    st.debug_ws_bytes = 0;
    if (st.capture_stream) (void)hipStreamDestroy(st.capture_stream);
    st.workspace = st.batch_ws = st.bwd_ws = nullptr;
    st.workspace_bytes = st.batch_ws_bytes = st.bwd_ws_bytes = 0;
    st.capture_stream = nullptr;
  }
  if (have_cur) (void)hipSetDevice(cur);
}

}  // extern "C"
