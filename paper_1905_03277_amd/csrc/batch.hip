// Batched merge of many bursts of uneven frame count, size and scale in one
// captured graph of persistent kernels, and the tile-shape autotuner.
//
// hmfsr_merge_batch lays out one workspace for every burst (rejection
// strengths, R_hat), per-burst argument blocks and cost-ordered work lists,
// then records into a hipGraph: a counter reset, the motion prior of every
// (burst, frame, tile), the guide statistics, one persistent robustness
// launch over all (burst, tile) items and one persistent merge launch per
// class (tile shape, raw-load batch size), each with an XCD-chunked queue. The graph is
// kept and replayed while the bursts' shapes and buffers stay the same;
// changed tuning values are uploaded before the replay.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <numeric>

#include "device_util.h"
#include "host.h"

namespace hmfsr {
namespace {

constexpr int kDefaultVariant = 2;  // 64x16 tile, 256 threads

// ---- autotuner --------------------------------------------------------------
// The best tile shape depends mostly on the output scale (footprint per output
// pixel) and on the frame count (how long accumulators live per workgroup).
struct TuneTable {
  int v[4][4];
  bool tuned[4][4];
  bool loaded = false;
};
TuneTable g_tune;

int scale_class(double s) { return s <= 1.0 ? 0 : (s <= 1.5 ? 1 : (s <= 2.0 ? 2 : 3)); }
int frame_bucket(int n) { return n <= 4 ? 0 : (n <= 8 ? 1 : (n <= 15 ? 2 : 3)); }

void tune_load() {
  if (g_tune.loaded) return;
  g_tune.loaded = true;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      g_tune.v[a][b] = kDefaultVariant;
      g_tune.tuned[a][b] = false;
    }
  const char* path = getenv("HMFSR_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  int a, b, v;
  while (fscanf(f, "%d %d %d", &a, &b, &v) == 3) {
    if (a >= 0 && a < 4 && b >= 0 && b < 4 && v >= 0 && v < kNumMergeVariants) {
      g_tune.v[a][b] = v;
      g_tune.tuned[a][b] = true;
    }
  }
  fclose(f);
}

void tune_save() {
  const char* path = getenv("HMFSR_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "w");
  if (!f) return;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      if (g_tune.tuned[a][b]) fprintf(f, "%d %d %d\n", a, b, g_tune.v[a][b]);
  fclose(f);
}

// ---- batch layout -------------------------------------------------------------
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t counters = 0, bounds = 0, args = 0, first = 0, bfirst = 0, ffirst = 0, ritems = 0, mitems = 0, work = 0,
         total = 0;
  std::vector<size_t> burst_work;  // offset of each burst's Work inside the workspace
};

// HMFSR_BATCH_GROUPS: a cap on the workgroups of every persistent launch
// (0 = none), so that each workgroup takes many items in turn.
int batch_groups_cap() {
  const char* env = getenv("HMFSR_BATCH_GROUPS");
  if (!env) return 0;
  const int k = atoi(env);
  return k > 0 ? k : 0;
}

// Persistent launches of a batch: the robustness launch (0), then one merge
// launch per class (1 + class). Each has an XCD-chunked item queue.
constexpr int kQueues = 1 + kNumMergeClasses;

// Bounds of XCDS contiguous chunks of items [0, n) of about equal cost
// (cost(i) per item), into out[0 .. XCDS].
template <typename C>
void xcd_chunks(int n, C cost, int* out) {
  double total = 0.0;
  for (int i = 0; i < n; ++i) total += cost(i);
  double acc = 0.0;
  int x = 1;
  out[0] = 0;
  for (int i = 0; i < n && x < XCDS; ++i) {
    acc += cost(i);
    while (x < XCDS && acc >= total * x / XCDS) out[x++] = i + 1;
  }
  while (x <= XCDS) out[x++] = n;
}

int capped(size_t items, size_t resident, int cap) {
  size_t g = std::min(items, resident);
  if (cap > 0) g = std::min(g, (size_t)cap);
  return (int)std::max<size_t>(g, 1);
}

}  // namespace

int merge_variant(const Geometry& g) {
  const char* env = getenv("HMFSR_MERGE_VARIANT");
  if (env) {
    const int v = atoi(env);
    if (v >= 0 && v < kNumMergeVariants) return v;
  }
  tune_load();
  return g_tune.v[scale_class(g.scale)][frame_bucket(g.n)];
}

}  // namespace hmfsr

using namespace hmfsr;

extern "C" {

hmfsr_status hmfsr_autotune(const hmfsr_desc* desc, const hmfsr_tuning* tuning,
                            const uint16_t* frames, const float* motion, float* out, void* stream,
                            int32_t* chosen) {
  hmfsr_status st = validate(desc, tuning);
  if (st != HMFSR_OK) return st;
  if (!frames || !motion || !out) return HMFSR_E_INVALID;
  if (((uintptr_t)frames & 3) || ((uintptr_t)motion & 3) || ((uintptr_t)out & 3)) return HMFSR_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  if ((st = current_device(&dev)) != HMFSR_OK) return st;
  const Geometry g = make_geometry(desc);
  void* ws = nullptr;
  hipStream_t s = (hipStream_t)stream;
  if ((st = workspace(dev, work_bytes(g), s, &ws)) != HMFSR_OK) return st;
  const Work w = work_carve(ws, g);
  // robustness once, then every tile shape: one warm-up and three timed launches
  if ((st = run_merge(desc, tuning, g, frames, motion, out, nullptr, w, kDefaultVariant, s)) != HMFSR_OK) return st;
  const MergeConsts mc = make_merge(desc, tuning, g);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return HMFSR_E_HIP;
  int best = kDefaultVariant;
  float best_ms = 1e30f;
  for (int v = 0; v < kNumMergeVariants && st == HMFSR_OK; ++v) {
    if (launch_merge(v, g, mc, frames, motion, w.rmin, out, nullptr, s) != hipSuccess) st = HMFSR_E_HIP;
    if (hipEventRecord(a, s) != hipSuccess) st = HMFSR_E_HIP;
    for (int r = 0; r < 3 && st == HMFSR_OK; ++r)
      if (launch_merge(v, g, mc, frames, motion, w.rmin, out, nullptr, s) != hipSuccess) st = HMFSR_E_HIP;
    float ms = 0.f;
    if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess)
      st = HMFSR_E_HIP;
    if (st == HMFSR_OK && ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != HMFSR_OK) return st;
  // leave `out` holding the merge of the chosen shape
  if (launch_merge(best, g, mc, frames, motion, w.rmin, out, nullptr, s) != hipSuccess) return HMFSR_E_HIP;
  tune_load();
  g_tune.v[scale_class(g.scale)][frame_bucket(g.n)] = best;
  g_tune.tuned[scale_class(g.scale)][frame_bucket(g.n)] = true;
  tune_save();
  if (chosen) *chosen = best;
  return HMFSR_OK;
}

hmfsr_status hmfsr_merge_batch(int32_t n_bursts, const hmfsr_desc* descs, const hmfsr_tuning* tunings,
                               const uint16_t* const* frames, const float* const* motion,
                               float* const* out, void* stream) {
  if (n_bursts < 1 || n_bursts > 65536 || !descs || !tunings || !frames || !motion || !out)
    return HMFSR_E_INVALID;
  hmfsr_status st;
  for (int i = 0; i < n_bursts; ++i) {
    if ((st = validate(&descs[i], &tunings[i])) != HMFSR_OK) return st;
    if (!frames[i] || !motion[i] || !out[i]) return HMFSR_E_INVALID;
    if (((uintptr_t)frames[i] & 3) || ((uintptr_t)motion[i] & 3) || ((uintptr_t)out[i] & 3))
      return HMFSR_E_INVALID;
  }
  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  if ((st = current_device(&dev)) != HMFSR_OK) return st;
  DeviceState& ds = g_dev[dev];
  hipStream_t s = (hipStream_t)stream;
  if (debug_enabled())
    for (int i = 0; i < n_bursts; ++i) {
      const Geometry gi = make_geometry(&descs[i]);
      if ((st = debug_check_motion(dev, motion[i], gi.n, gi.ref, gi.TY, gi.TX, s)) != HMFSR_OK) return st;
    }

  // per-burst geometry, tile shape and work sizes
  std::vector<Geometry> geo(n_bursts);
  std::vector<int> var(n_bursts), mtx(n_bursts), mtiles(n_bursts), rtiles(n_bursts);
  std::vector<double> cost(n_bursts);
  Layout L;
  size_t n_prior = 0, n_base = 0, n_fmeans = 0, n_ritems = 0, n_mitems = 0;
  for (int i = 0; i < n_bursts; ++i) {
    geo[i] = make_geometry(&descs[i]);
    var[i] = merge_variant(geo[i]);
    const int rows = merge_tile_rows(var[i]);
    mtx[i] = (geo[i].OW + 63) / 64;
    mtiles[i] = mtx[i] * ((geo[i].OH + rows - 1) / rows);
    rtiles[i] = geo[i].n > 1 ? robust_tiles_x(geo[i]) * robust_tiles_y(geo[i]) : 0;
    cost[i] = (double)geo[i].n * geo[i].OH * geo[i].OW;
    n_prior += (size_t)geo[i].n * geo[i].TY * geo[i].TX;
    n_base += (size_t)base_stats_groups(geo[i]);
    n_fmeans += (size_t)frame_means_groups(geo[i]);
    n_ritems += rtiles[i];
    n_mitems += mtiles[i];
  }
  if (n_prior > 0x7fffffff || n_base > 0x7fffffff || n_fmeans > 0x7fffffff || n_ritems > 0x7fffffff || n_mitems > 0x7fffffff)
    return HMFSR_E_INVALID;
  size_t off = 0;
  L.counters = off; off += align256(sizeof(int) * kQueues * XCDS);
  L.bounds = off; off += align256(sizeof(int) * kQueues * (XCDS + 1));
  L.args = off; off += align256(sizeof(BurstArgs) * n_bursts);
  L.first = off; off += align256(sizeof(int) * n_bursts);
  L.bfirst = off; off += align256(sizeof(int) * n_bursts);
  L.ffirst = off; off += align256(sizeof(int) * n_bursts);
  L.ritems = off; off += align256(sizeof(WorkItem) * n_ritems);
  L.mitems = off; off += align256(sizeof(WorkItem) * n_mitems);
  L.burst_work.resize(n_bursts);
  for (int i = 0; i < n_bursts; ++i) {
    L.burst_work[i] = off;
    off += align256(work_bytes(geo[i]));
  }
  L.total = off;

  // workspace (grown only; the old graph points into the old one)
  if (ds.batch_ws_bytes < L.total) {
    if (hipStreamSynchronize(s) != hipSuccess) return HMFSR_E_HIP;
    if (ds.plan.exec) (void)hipGraphExecDestroy(ds.plan.exec);
    if (ds.plan.graph) (void)hipGraphDestroy(ds.plan.graph);
    ds.plan = BatchPlan();
    if (ds.batch_ws) (void)hipFree(ds.batch_ws);
    ds.batch_ws = nullptr;
    ds.batch_ws_bytes = 0;
    if (hipMalloc(&ds.batch_ws, L.total) != hipSuccess) {
      (void)hipGetLastError();
      return HMFSR_E_NOMEM;
    }
    ds.batch_ws_bytes = L.total;
  }
  char* base = (char*)ds.batch_ws;

  // argument blocks
  std::vector<BurstArgs> args(n_bursts);
  for (int i = 0; i < n_bursts; ++i) {
    BurstArgs& a = args[i];
    const Work w = work_carve(base + L.burst_work[i], geo[i]);
    a.frames = frames[i];
    a.motion = motion[i];
    a.out = out[i];
    a.s_tile = w.s_tile;
    a.mov = w.mov;
    a.rmin = w.rmin;
    a.gmu = w.gmu;
    a.gref = w.gref;
    a.g = geo[i];
    a.mc = make_merge(&descs[i], &tunings[i], geo[i]);
    a.rc = make_robust(&descs[i], &tunings[i]);
    a.pc = make_prior(&tunings[i]);
    a.merge_tiles_x = mtx[i];
    a.robust_tiles_x = geo[i].n > 1 ? robust_tiles_x(geo[i]) : 1;
  }

  // same shapes and buffers as the captured graph: refresh arguments, replay
  // (descriptors and tunings are plain int32 / float structs: memcmp is exact)
  std::vector<const void*> ptrs;
  for (int i = 0; i < n_bursts; ++i) {
    ptrs.push_back(frames[i]);
    ptrs.push_back(motion[i]);
    ptrs.push_back(out[i]);
  }
  BatchPlan& P = ds.plan;
  const int cap = batch_groups_cap();
  const bool same = P.exec && P.ws == ds.batch_ws && P.variants == var && P.ptrs == ptrs && P.groups_cap == cap &&
                    P.descs.size() == (size_t)n_bursts &&
                    memcmp(P.descs.data(), descs, sizeof(hmfsr_desc) * n_bursts) == 0;
  if (same) {
    if (memcmp(P.tunings.data(), tunings, sizeof(hmfsr_tuning) * n_bursts) != 0) {
      // the previous replay may still read the old arguments
      if (hipStreamSynchronize(s) != hipSuccess) return HMFSR_E_HIP;
      if (hipMemcpy(base + L.args, args.data(), sizeof(BurstArgs) * n_bursts, hipMemcpyHostToDevice) !=
          hipSuccess)
        return HMFSR_E_HIP;
      P.tunings.assign(tunings, tunings + n_bursts);
    }
    return timed(HMFSR_STAGE_BATCH, s, [&] { return hipGraphLaunch(P.exec, s); }) == hipSuccess
               ? HMFSR_OK
               : HMFSR_E_HIP;
  }

  // work lists: most expensive bursts first, tiles in order within a burst
  std::vector<int> order(n_bursts);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<WorkItem> ritems;
  ritems.reserve(n_ritems);
  for (int i : order)
    for (int t = 0; t < rtiles[i]; ++t) ritems.push_back({i, t});
  // one merge list per class (tile shape, load batch), stored back to back
  std::vector<int> mcls(n_bursts);
  for (int i = 0; i < n_bursts; ++i) mcls[i] = merge_class(var[i], geo[i].scale);
  std::vector<WorkItem> mitems;
  mitems.reserve(n_mitems);
  std::vector<int> group_start(kNumMergeClasses + 1, 0);
  for (int c = 0; c < kNumMergeClasses; ++c) {
    group_start[c] = (int)mitems.size();
    for (int i : order)
      if (mcls[i] == c)
        for (int t = 0; t < mtiles[i]; ++t) mitems.push_back({i, t});
  }
  group_start[kNumMergeClasses] = (int)mitems.size();
  // XCD chunks of every persistent launch, balanced by frames per item
  std::vector<int> bounds(kQueues * (XCDS + 1), 0);
  xcd_chunks((int)n_ritems, [&](int i) { return (double)(geo[ritems[i].burst].n - 1); }, &bounds[0]);
  for (int c = 0; c < kNumMergeClasses; ++c)
    xcd_chunks(group_start[c + 1] - group_start[c],
               [&](int i) { return (double)geo[mitems[group_start[c] + i].burst].n; }, &bounds[(1 + c) * (XCDS + 1)]);
  std::vector<int> first(n_bursts), bfirst(n_bursts), ffirst(n_bursts);
  {
    size_t acc = 0, bacc = 0, facc = 0;
    for (int i = 0; i < n_bursts; ++i) {
      first[i] = (int)acc;
      acc += (size_t)geo[i].n * geo[i].TY * geo[i].TX;
      bfirst[i] = (int)bacc;
      bacc += (size_t)base_stats_groups(geo[i]);
      ffirst[i] = (int)facc;
      facc += (size_t)frame_means_groups(geo[i]);
    }
  }

  // rebuild: wait for any replay that reads the lists, upload, capture
  if (hipStreamSynchronize(s) != hipSuccess) return HMFSR_E_HIP;
  if (P.exec) (void)hipGraphExecDestroy(P.exec);
  if (P.graph) (void)hipGraphDestroy(P.graph);
  P = BatchPlan();
  if (hipMemcpy(base + L.args, args.data(), sizeof(BurstArgs) * n_bursts, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(base + L.first, first.data(), sizeof(int) * n_bursts, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(base + L.bfirst, bfirst.data(), sizeof(int) * n_bursts, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(base + L.ffirst, ffirst.data(), sizeof(int) * n_bursts, hipMemcpyHostToDevice) != hipSuccess ||
      (n_ritems && hipMemcpy(base + L.ritems, ritems.data(), sizeof(WorkItem) * n_ritems,
                             hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(base + L.mitems, mitems.data(), sizeof(WorkItem) * n_mitems, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(base + L.bounds, bounds.data(), sizeof(int) * bounds.size(), hipMemcpyHostToDevice) != hipSuccess)
    return HMFSR_E_HIP;
  if (!ds.capture_stream && hipStreamCreateWithFlags(&ds.capture_stream, hipStreamNonBlocking) != hipSuccess)
    return HMFSR_E_HIP;

  const BurstArgs* d_args = (const BurstArgs*)(base + L.args);
  const int* d_first = (const int*)(base + L.first);
  const int* d_bfirst = (const int*)(base + L.bfirst);
  const int* d_ffirst = (const int*)(base + L.ffirst);
  const WorkItem* d_ritems = (const WorkItem*)(base + L.ritems);
  const WorkItem* d_mitems = (const WorkItem*)(base + L.mitems);
  int* d_counters = (int*)(base + L.counters);  // [queue][XCDS]: robustness, then merge class c
  const int* d_bounds = (const int*)(base + L.bounds);  // [queue][XCDS + 1]
  const int cus = ds.cus > 0 ? ds.cus : 256;
  hipStream_t cs = ds.capture_stream;
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return HMFSR_E_HIP;
  hipError_t err = launch_fill_i32(d_counters, 0, kQueues * XCDS, cs);
  if (err == hipSuccess) err = launch_prior_batch(d_args, d_first, n_bursts, (int)n_prior, cs);
  if (err == hipSuccess)
    err = launch_guide_stats_batch(d_args, d_bfirst, (int)n_base, d_ffirst, (int)n_fmeans, n_bursts, cs);
  hmfsr_batch_info info = {};
  if (err == hipSuccess && n_ritems) {
    const int groups = capped(n_ritems, (size_t)cus * robust_batch_blocks_per_cu(), cap);
    err = launch_robust_batch(d_args, d_ritems, d_bounds, d_counters, groups, cs);
    info.robust_items = (int32_t)n_ritems;
    info.robust_groups = groups;
  }
  for (int c = 0; c < kNumMergeClasses && err == hipSuccess; ++c) {
    const int cnt = group_start[c + 1] - group_start[c];
    if (cnt == 0) continue;
    const int groups = capped(cnt, (size_t)cus * merge_batch_blocks_per_cu(c), cap);
    err = launch_merge_batch(c, d_args, d_mitems + group_start[c], d_bounds + (1 + c) * (XCDS + 1),
                             d_counters + (1 + c) * XCDS, groups, cs);
    info.merge_items[c] = cnt;
    info.merge_groups[c] = groups;
  }
  const hipError_t end = hipStreamEndCapture(cs, &graph);
  if (err != hipSuccess || end != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return HMFSR_E_HIP;
  }
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return HMFSR_E_HIP;
  }
  P.graph = graph;
  P.exec = exec;
  P.ws = ds.batch_ws;
  P.variants = var;
  P.ptrs = ptrs;
  P.descs.assign(descs, descs + n_bursts);
  P.tunings.assign(tunings, tunings + n_bursts);
  P.groups_cap = cap;
  P.info = info;
  return timed(HMFSR_STAGE_BATCH, s, [&] { return hipGraphLaunch(P.exec, s); }) == hipSuccess
             ? HMFSR_OK
             : HMFSR_E_HIP;
}

hmfsr_status hmfsr_batch_plan(hmfsr_batch_info* out) {
  if (!out) return HMFSR_E_INVALID;
  std::lock_guard<std::mutex> lock(g_mutex);
  int dev = 0;
  hmfsr_status st;
  if ((st = current_device(&dev)) != HMFSR_OK) return st;
  if (!g_dev[dev].plan.exec) return HMFSR_E_INVALID;
  *out = g_dev[dev].plan.info;
  return HMFSR_OK;
}

}  // extern "C"
