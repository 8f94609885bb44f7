// Host-side state and helpers shared by the C ABI translation units.
#pragma once

#include <mutex>
#include <vector>

#include "hmfsr_internal.h"

namespace hmfsr {

constexpr int kMaxDevices = 64;

// A captured batch graph and the signature it was built for.
struct BatchPlan {
  std::vector<hmfsr_desc> descs;
  std::vector<const void*> ptrs;  // frames, motion, out of every burst
  std::vector<int> variants;
  void* ws = nullptr;             // batch workspace the graph's arguments point into
  std::vector<hmfsr_tuning> tunings;  // the tunings of the uploaded argument blocks
  int groups_cap = 0;             // HMFSR_BATCH_GROUPS when captured (0: none)
  hmfsr_batch_info info = {};     // items and workgroups of the persistent launches
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct DeviceState {
  int checked = 0;  // 0 unknown, 1 gfx950, -1 unsupported
  int cus = 0;      // compute units
  void* workspace = nullptr;  // single-burst workspace
  size_t workspace_bytes = 0;
  void* batch_ws = nullptr;   // batch workspace
  size_t batch_ws_bytes = 0;
  void* bwd_ws = nullptr;     // adjoint workspace
  size_t bwd_ws_bytes = 0;
  void* stream_ws = nullptr;  // streaming merge: two-frame view and its maps
  size_t stream_ws_bytes = 0;
  void* align_ws = nullptr;   // tile alignment: pyramids and block vectors
  size_t align_ws_bytes = 0;
  void* sum_ws = nullptr;     // frame sums for the SNR-dependent tuning
  size_t sum_ws_bytes = 0;
  void* debug_ws = nullptr;   // HMFSR_DEBUG: the device checks' result word
  size_t debug_ws_bytes = 0;
  hipStream_t capture_stream = nullptr;
  BatchPlan plan;
};

extern std::mutex g_mutex;
extern DeviceState g_dev[kMaxDevices];

// Optional per-stage timing: an event pair around every kernel launch.
struct Timing {
  bool on = false;
  struct Pair {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Pair> pairs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
};
extern Timing g_timing;

// Launch `fn` on `s`, bracketed by timing events when profiling is on.
template <typename F>
hipError_t timed(int stage, hipStream_t s, F fn) {
  if (!g_timing.on) return fn();
  hipEvent_t a = g_timing.get(), b = g_timing.get();
  if (a) (void)hipEventRecord(a, s);  // profiling only: a failed record leaves the pair out below
  const hipError_t err = fn();
  if (b) (void)hipEventRecord(b, s);
  if (a && b) g_timing.pairs.push_back({stage, a, b});
  return err;
}

hmfsr_status validate_desc(const hmfsr_desc* d);
hmfsr_status validate(const hmfsr_desc* d, const hmfsr_tuning* t);
Geometry make_geometry(const hmfsr_desc* d);
PriorConsts make_prior(const hmfsr_tuning* t);
RobustConsts make_robust(const hmfsr_desc* d, const hmfsr_tuning* t);
MergeConsts make_merge(const hmfsr_desc* d, const hmfsr_tuning* t, const Geometry& g);
OmegaConsts make_omega(const hmfsr_desc* d, const hmfsr_tuning* t);
hmfsr_status current_device(int* dev_out);  // caller holds g_mutex
hmfsr_status workspace(int dev, size_t bytes, hipStream_t stream, void** out);  // caller holds g_mutex
hmfsr_status bwd_workspace(int dev, size_t bytes, hipStream_t stream, void** out);  // caller holds g_mutex
hmfsr_status stream_workspace(int dev, size_t bytes, hipStream_t stream, void** out);  // caller holds g_mutex
hmfsr_status align_workspace(int dev, size_t bytes, hipStream_t stream, void** out);  // caller holds g_mutex
// Grow a per-device buffer (caller holds g_mutex).
hmfsr_status grow_buffer(void*& buf, size_t& have, size_t bytes, hipStream_t stream, void** out);

// HMFSR_DEBUG set (and not "0"): calls check their device data first.
bool debug_enabled();
// Scan motion [n][TY][TX][2] (frame `ref` skipped; ref < 0: none) for
// non-finite values; synchronises `s`. HMFSR_E_DATA (and a line on stderr
// naming the first one) if any (caller holds g_mutex).
hmfsr_status debug_check_motion(int dev, const float* motion, int n, int ref, int TY, int TX, hipStream_t s);

// Merge tile shape for a burst: HMFSR_MERGE_VARIANT, else the autotuned
// choice for the burst's (scale, frame count) class, else the default.
int merge_variant(const Geometry& g);
// The three kernels of one merge on `s` (workspace from `workspace`). With
// `profiled` false the launches are never bracketed by timing events (which
// the event pool may have to create).
hmfsr_status run_merge(const hmfsr_desc* desc, const hmfsr_tuning* tuning, const Geometry& g,
                       const uint16_t* frames, const float* motion, float* out, float* saved,
                       const Work& w, int variant, hipStream_t s, bool profiled = true);

}  // namespace hmfsr
