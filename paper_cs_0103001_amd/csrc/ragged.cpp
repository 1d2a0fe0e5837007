// ragged.cpp -- ragged batches of square images of mixed power-of-two sides:
// plan (image table and per-pass tile lists on the device), execution as one
// persistent launch per pass captured in a HIP graph, and the autotuner that
// picks the launch schedule.
//
// Schedule knobs:
//   block   threads per workgroup (256 or 512): a tile is block/TPT(s)
//           transforms of side s, so block*16 points for every side
//   wg_cap  resident workgroups per CU (0: as many as fit)
//   chunk   0: each pass covers the whole batch; otherwise images are taken
//           in runs whose complex64 intermediate is at most `chunk` bytes,
//           the three passes run per run (the run's intermediate then stays
//           in the memory-side cache between passes), and the workspace
//           region is reused by every run
//   order   0: tiles of the largest images first; 1: the images' own order
//   small   images of side <= 2^small run in one pass from LDS (one launch
//           of their own, beside the three passes of the larger images);
//           -1: every image takes the three passes
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/fftmi.h"
#include "fft_schedule.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace fftmi {

struct RaggedSchedule {
  int block = 256;
  int wg_cap = 0;
  int64_t chunk = 0;
  int order = 0;
  int small = kRaggedSmallMaxLog2;
};

struct RaggedRun {  // one run of images: the tile range of each pass
  int64_t begin[3], count[3];
};

struct RaggedState {
  std::vector<int64_t> sizes;
  std::vector<RaggedImage> imgs;
  int64_t total = 0;     // sum of s^2
  int64_t ws_total = 0;  // workspace elements (blocked layouts with padded strides)
  RaggedSchedule sched;
  std::vector<RaggedRun> runs;
  RaggedImage* d_imgs = nullptr;
  int2* d_tiles[3] = {nullptr, nullptr, nullptr};
  // images of the single-pass LDS path: their indices (largest side first)
  // and the work items {first entry, count}
  int* d_small_idx = nullptr;
  int2* d_small_items = nullptr;
  int n_small_items = 0;
  // the small images' launch runs on a second stream, forked from and
  // joined to the caller's stream (a parallel branch of the captured graph)
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  TwTable tw{};
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // what the instantiated graph was captured with
  const void* g_in = nullptr;
  void* g_out = nullptr;
  void* g_ws = nullptr;
  MaskArgs g_mask{};
  bool use_graph = true;
  // real input: the first row pass takes the rows in pairs (twice the rows
  // per tile)
  bool in_f32 = false;
};

namespace {

int rb_for(int64_t s) { return (int)std::min<int64_t>(4, threads_per_transform((int)s)); }
// block stride and workspace elements of one image of side s
int64_t bs_for(int64_t s) { return rb_for(s) * s + block_pad(rb_for(s) * s); }
int64_t ws_elems_for(int64_t s) { return (s / rb_for(s)) * bs_for(s); }

void drop_graph(RaggedState* r) {
  if (r->exec) (void)hipGraphExecDestroy(r->exec);
  if (r->graph) (void)hipGraphDestroy(r->graph);
  r->exec = nullptr;
  r->graph = nullptr;
}

void free_lists(RaggedState* r) {
  if (r->d_imgs) (void)hipFree(r->d_imgs);
  for (auto& t : r->d_tiles)
    if (t) (void)hipFree(t);
  if (r->d_small_idx) (void)hipFree(r->d_small_idx);
  if (r->d_small_items) (void)hipFree(r->d_small_items);
  r->d_imgs = nullptr;
  r->d_tiles[0] = r->d_tiles[1] = r->d_tiles[2] = nullptr;
  r->d_small_idx = nullptr;
  r->d_small_items = nullptr;
  r->n_small_items = 0;
}

bool is_small(const RaggedState* r, int64_t s) { return r->sched.small >= 0 && s <= (int64_t(1) << r->sched.small); }

// Image table, runs and tile lists for the current schedule; uploads them.
int build_lists(RaggedState* r) {
  drop_graph(r);
  free_lists(r);
  r->runs.clear();
  const int64_t n = (int64_t)r->sizes.size();
  r->imgs.assign(n, RaggedImage{});
  // runs of consecutive images
  std::vector<std::pair<int64_t, int64_t>> spans;  // [first, last)
  int64_t first = 0, bytes = 0, off = 0, ws_off = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t s = r->sizes[i], b = is_small(r, s) ? 0 : ws_elems_for(s) * 8;
    if (r->sched.chunk > 0 && i > first && b > 0 && bytes + b > r->sched.chunk) {
      spans.push_back({first, i});
      first = i;
      bytes = 0;
    }
    RaggedImage& im = r->imgs[i];
    im.off = off;
    im.ws_off = r->sched.chunk > 0 ? bytes / 8 : ws_off;
    im.lg = ilog2c((int)s);
    im.rb = rb_for(s);
    im.bs = bs_for(s);
    bytes += b;
    off += s * s;
    ws_off += ws_elems_for(s);
  }
  if (n > first) spans.push_back({first, n});
  std::vector<int2> lists[3];
  for (const auto& sp : spans) {
    std::vector<int64_t> idx(sp.second - sp.first);
    std::iota(idx.begin(), idx.end(), sp.first);
    if (r->sched.order == 0)
      std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return r->sizes[a] > r->sizes[b]; });
    RaggedRun run{};
    for (int p = 0; p < 3; ++p) {
      run.begin[p] = (int64_t)lists[p].size();
      for (int64_t i : idx) {
        const int64_t s = r->sizes[i];
        if (is_small(r, s)) continue;
        // rows or columns per tile: one per transform, two per transform
        // in the first row pass of real input
        const int per = std::max(1, r->sched.block / threads_per_transform((int)s)) * (p == 0 && r->in_f32 ? 2 : 1);
        const int64_t tiles = (s + per - 1) / per;
        for (int64_t t = 0; t < tiles; ++t) lists[p].push_back(make_int2((int)i, (int)t));
      }
      run.count[p] = (int64_t)lists[p].size() - run.begin[p];
    }
    r->runs.push_back(run);
  }
  // small images: largest side first, in items of at most ragged_small_ipw
  // images of one side
  std::vector<int> sidx;
  std::vector<int2> items;
  for (int64_t i = 0; i < n; ++i)
    if (is_small(r, r->sizes[i])) sidx.push_back((int)i);
  std::stable_sort(sidx.begin(), sidx.end(), [&](int a, int b) { return r->sizes[a] > r->sizes[b]; });
  for (size_t a = 0; a < sidx.size();) {
    const int lg = ilog2c((int)r->sizes[sidx[a]]), ipw = ragged_small_ipw(lg);
    size_t b = a;
    while (b < sidx.size() && b - a < (size_t)ipw && r->sizes[sidx[b]] == r->sizes[sidx[a]]) ++b;
    items.push_back(make_int2((int)a, (int)(b - a)));
    a = b;
  }
  if (n == 0) return FFT_OK;
  hipError_t e = hipMalloc(&r->d_imgs, n * sizeof(RaggedImage));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? FFT_ERR_NOMEM : hip_fail(e);
  e = hipMemcpy(r->d_imgs, r->imgs.data(), n * sizeof(RaggedImage), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e);
  for (int p = 0; p < 3; ++p) {
    e = hipMalloc(&r->d_tiles[p], std::max<size_t>(lists[p].size(), 1) * sizeof(int2));
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? FFT_ERR_NOMEM : hip_fail(e);
    e = hipMemcpy(r->d_tiles[p], lists[p].data(), lists[p].size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (!items.empty()) {
    e = hipMalloc(&r->d_small_idx, sidx.size() * sizeof(int));
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? FFT_ERR_NOMEM : hip_fail(e);
    e = hipMemcpy(r->d_small_idx, sidx.data(), sidx.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
    e = hipMalloc(&r->d_small_items, items.size() * sizeof(int2));
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? FFT_ERR_NOMEM : hip_fail(e);
    e = hipMemcpy(r->d_small_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
    r->n_small_items = (int)items.size();
  }
  return FFT_OK;
}

// Launch every run's three passes on `st`.  The grid sizes are worked out
// first (occupancy queries are host calls, kept out of a stream capture).
hipError_t enqueue(const fftmi_plan* p, RaggedState* r, const void* in, void* out, void* ws, const MaskArgs& mk,
                   hipStream_t st, bool capturing = false) {
  const bool in_f32 = p->flags & FFT_IN_REAL_F32, out_f32 = p->flags & FFT_OUT_REAL_F32;
  const bool numpy = p->flags & FFT_NORM_NUMPY;
  int small_grid = 0;
  hipError_t se = ragged_small_grid(in_f32, out_f32, mk.kind, r->n_small_items, &small_grid);
  if (se != hipSuccess) return se;
  std::vector<int> grids;
  for (const RaggedRun& run : r->runs)
    for (int pass = 0; pass < 3; ++pass) {
      int g = 0;
      hipError_t e = ragged_grid(pass, in_f32, out_f32, mk.kind, r->sched.block, r->sched.wg_cap,
                                 (int)run.count[pass], &g);
      if (e != hipSuccess) return e;
      grids.push_back(g);
    }
  if (capturing) {
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
  }
  size_t k = 0;
  hipError_t err = hipSuccess;
  // small images: forked onto the side stream, so that they run beside the
  // passes of the larger images (in a captured graph: a parallel branch)
  const bool fork = r->n_small_items > 0;
  if (r->n_small_items > 0) {
    hipStream_t ss = st;
    if (fork) {
      err = hipEventRecord(r->ev_fork, st);
      if (err == hipSuccess) err = hipStreamWaitEvent(r->side_stream, r->ev_fork, 0);
      ss = r->side_stream;
    }
    if (err == hipSuccess)
      err = launch_ragged_small(in, in_f32, out, out_f32, r->d_imgs, r->d_small_idx, r->d_small_items,
                                r->n_small_items, small_grid, mk, r->tw, numpy, ss);
    if (fork && err == hipSuccess) err = hipEventRecord(r->ev_join, r->side_stream);
  }
  for (const RaggedRun& run : r->runs) {
    for (int pass = 0; pass < 3 && err == hipSuccess; ++pass, ++k)
      err = launch_ragged_pass(pass, in, in_f32, static_cast<float2*>(ws), out, out_f32, r->d_imgs,
                               r->d_tiles[pass] + run.begin[pass], (int)run.count[pass], r->sched.block, grids[k],
                               mk, r->tw, numpy, st);
    if (err != hipSuccess) break;
  }
  if (fork && err == hipSuccess) err = hipStreamWaitEvent(st, r->ev_join, 0);
  return err;
}

// Capture one call's launches (on the plan's capture stream) into an
// instantiated graph.
hipError_t capture(const fftmi_plan* p, RaggedState* r, const void* in, void* out, void* ws, const MaskArgs& mk,
                   hipGraph_t* graph, hipGraphExec_t* exec) {
  *graph = nullptr;
  *exec = nullptr;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t le = enqueue(p, r, in, out, ws, mk, r->cap_stream, true);
  hipError_t e = hipSuccess;
  if (hipStreamIsCapturing(r->cap_stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive)
    e = hipStreamEndCapture(r->cap_stream, graph);
  if (le != hipSuccess || e != hipSuccess) {
    if (*graph) (void)hipGraphDestroy(*graph);
    *graph = nullptr;
    return le != hipSuccess ? le : e;
  }
  e = hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(*graph);
    *graph = nullptr;
    *exec = nullptr;
  }
  return e;
}

// ----------------------------------------------------------- tuning cache
std::mutex g_cache_mu;

std::string cache_key(const fftmi_plan* p, const RaggedState* r) {
  hipDeviceProp_t prop;
  std::string dev = "unknown";
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) dev = prop.gcnArchName;
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the side list
  for (int64_t s : r->sizes) {
    h ^= (uint64_t)s;
    h *= 1099511628211ull;
  }
  std::ostringstream k;
  k << "ragged/" << dev << "/n" << r->sizes.size() << "/h" << std::hex << h << "/f" << p->flags;
  std::string out = k.str();
  for (char& c : out)
    if (c == ' ' || c == ':') c = '_';
  return out;
}

// A schedule the launchers accept: a record from the cache file that is not
// (a hand edit, another library version) is ignored, so a plan never adopts a
// schedule that would fail at every later exec.
bool schedule_valid(const RaggedSchedule& s) {
  return (s.block == 128 || s.block == 256 || s.block == 512) && s.wg_cap >= 0 && s.wg_cap <= 64 &&
         s.chunk >= 0 && s.chunk <= (int64_t(1) << 40) && (s.order == 0 || s.order == 1) && s.small >= -1 &&
         s.small <= kRaggedSmallMaxLog2;
}

bool cache_lookup(const std::string& key, RaggedSchedule* s) {
  const char* path = std::getenv("FFTMI_TUNE_CACHE");
  if (!path || !*path) return false;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    std::string k;
    RaggedSchedule t;
    std::string rest;
    if (ls >> k >> t.block >> t.wg_cap >> t.chunk >> t.order >> t.small && k == key && !(ls >> rest) &&
        schedule_valid(t)) {
      *s = t;
      found = true;  // the last record of a key wins
    }
  }
  return found;
}

void cache_store(const std::string& key, const RaggedSchedule& s) {
  const char* path = std::getenv("FFTMI_TUNE_CACHE");
  if (!path || !*path) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  std::ofstream f(path, std::ios::app);
  f << key << ' ' << s.block << ' ' << s.wg_cap << ' ' << s.chunk << ' ' << s.order << ' ' << s.small << '\n';
}

bool valid_side(int64_t s) { return s >= 1 && s <= (int64_t(1) << kRaggedMaxLog2) && (s & (s - 1)) == 0; }

}  // namespace

void destroy_ragged_state(fftmi_plan* p) {
  RaggedState* r = p->ragged;
  if (!r) return;
  drop_graph(r);
  free_lists(r);
  if (r->cap_stream) (void)hipStreamDestroy(r->cap_stream);
  if (r->side_stream) (void)hipStreamDestroy(r->side_stream);
  if (r->ev_fork) (void)hipEventDestroy(r->ev_fork);
  if (r->ev_join) (void)hipEventDestroy(r->ev_join);
  delete r;
  p->ragged = nullptr;
}

// Candidate schedules, timed on the caller's buffers; the fastest is kept.
int tune_ragged(fftmi_plan* p, const void* in, void* out, const fft_mask* mask, void* ws, hipStream_t st,
                RaggedSchedule* chosen) {
  RaggedState* r = p->ragged;
  MaskArgs mk;
  int rc = mask_args(mask, p, &mk);
  if (rc != FFT_OK) return rc;
  std::vector<RaggedSchedule> cands;
  // launch shape (threads per workgroup, workgroups per CU, runs) and
  // transform shape: the largest side done in one pass from LDS
  for (int small : {-1, 6, kRaggedSmallMaxLog2})
    for (int block : {256, 512})
      for (int cap : {0, 2})
        for (int64_t chunk : {int64_t(0), int64_t(128) << 20}) {
          RaggedSchedule s;
          s.block = block;
          s.wg_cap = cap;
          s.chunk = chunk;
          s.order = 0;
          s.small = small;
          cands.push_back(s);
        }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return FFT_ERR_HIP;
  }
  float best = 1e30f;
  RaggedSchedule best_s = r->sched;
  int status = FFT_OK;
  for (const RaggedSchedule& s : cands) {
    r->sched = s;
    rc = build_lists(r);
    if (rc != FFT_OK) {
      status = rc;
      break;
    }
    // each candidate runs the way calls will run it: as a graph replay
    // (or eagerly when graphs are off), once to warm up, then three timed
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    hipError_t e = r->use_graph ? capture(p, r, in, out, ws, mk, &g, &x) : hipSuccess;
    auto run = [&]() { return x ? hipGraphLaunch(x, st) : enqueue(p, r, in, out, ws, mk, st); };
    if (e == hipSuccess) e = run();
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) e = run();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      status = hip_fail(e);
      break;
    }
    if (ms < best) {
      best = ms;
      best_s = s;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  r->sched = best_s;
  rc = build_lists(r);
  if (status == FFT_OK) status = rc;
  if (chosen) *chosen = best_s;
  return status;
}

}  // namespace fftmi

using namespace fftmi;

extern "C" {

int fft_plan_ragged(fft_plan_t* out, int64_t count, const int64_t* sizes, uint32_t flags) {
  if (!out) return FFT_ERR_ARG;
  *out = nullptr;
  if (count < 0 || (count > 0 && !sizes)) return FFT_ERR_ARG;
  if (flags & ~(FFT_IN_REAL_F32 | FFT_OUT_REAL_F32 | FFT_NORM_NUMPY)) return FFT_ERR_ARG;
  for (int64_t i = 0; i < count; ++i)
    if (!valid_side(sizes[i])) return FFT_ERR_SIZE;
  std::unique_ptr<fftmi_plan> p(new (std::nothrow) fftmi_plan());
  if (!p) return FFT_ERR_NOMEM;
  std::unique_ptr<RaggedState> r(new (std::nothrow) RaggedState());
  if (!r) return FFT_ERR_NOMEM;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  p->magic = kPlanMagic;
  p->kind = 3;
  p->device = dev;
  p->batch = count;
  p->flags = flags;
  p->n = p->m = 1;
  int rc = device_tables(dev, &p->tables);
  if (rc != FFT_OK) return rc;
  r->sizes.assign(sizes, sizes + count);
  r->in_f32 = (flags & FFT_IN_REAL_F32) != 0;
  for (int64_t s : r->sizes) {
    r->total += s * s;
    r->ws_total += ws_elems_for(s);
  }
  for (int lg = 0; lg <= kRaggedMaxLog2; ++lg) r->tw.p[lg] = blob_for(p->tables, lg);
  if (const char* g = std::getenv("FFTMI_RAGGED_GRAPH")) r->use_graph = std::atoi(g) != 0;
  e = hipStreamCreateWithFlags(&r->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e);
  p->ragged = r.get();
  e = hipStreamCreateWithFlags(&r->side_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ev_join, hipEventDisableTiming);
  if (e != hipSuccess) {
    destroy_ragged_state(p.get());
    r.release();
    return hip_fail(e);
  }

  RaggedSchedule cached;
  if (cache_lookup(cache_key(p.get(), r.get()), &cached)) r->sched = cached;
  // FFTMI_RAGGED_SMALL (log2 of the largest single-pass side, -1 for none)
  // overrides the single-pass limit, for tests and measurements
  if (const char* sm = std::getenv("FFTMI_RAGGED_SMALL")) {
    const int v = std::atoi(sm);
    if (v >= -1 && v <= kRaggedSmallMaxLog2) r->sched.small = v;
  }
  rc = build_lists(r.get());
  if (rc != FFT_OK) {
    destroy_ragged_state(p.get());
    r.release();
    return rc;
  }
  p->ws_bytes = (size_t)std::max<int64_t>(r->ws_total, 1) * sizeof(float2);
  r.release();
  plan_register(p.get());
  *out = p.release();
  return FFT_OK;
}

int fft2d_filter_ragged(fft_plan_t p, const void* in, void* out, const fft_mask* mask, void* workspace, void* stream) {
  TraceRange tr("fft2d_filter_ragged");
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (p->kind != 3 || !p->ragged) return FFT_ERR_STATE;
  RaggedState* r = p->ragged;
  MaskArgs mk;
  int rc = mask_args(mask, p, &mk);
  if (rc != FFT_OK) return rc;
  if (mk.kind != FFT_MASK_NONE && mk.kind != FFT_MASK_GAUSSIAN && mk.kind != FFT_MASK_BUTTERWORTH)
    return FFT_ERR_UNSUPPORTED;
  if (p->batch == 0) return FFT_OK;
  if (!in || !out) return FFT_ERR_ARG;
  if (!workspace) return FFT_ERR_WORKSPACE;
  if (ws_misaligned(workspace)) return FFT_ERR_ARG;
  rc = plan_check(p, nullptr);
  if (rc != FFT_OK) return rc;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (!r->use_graph) {
    hipError_t e = enqueue(p, r, in, out, workspace, mk, st);
    return e == hipSuccess ? FFT_OK : hip_fail(e);
  }
  const bool same = r->exec && r->g_in == in && r->g_out == out && r->g_ws == workspace &&
                    std::memcmp(&r->g_mask, &mk, sizeof(MaskArgs)) == 0;
  if (!same) {
    drop_graph(r);
    hipError_t e = capture(p, r, in, out, workspace, mk, &r->graph, &r->exec);
    if (e != hipSuccess) return hip_fail(e);
    r->g_in = in;
    r->g_out = out;
    r->g_ws = workspace;
    r->g_mask = mk;
  }
  hipError_t e = hipGraphLaunch(r->exec, st);
  return e == hipSuccess ? FFT_OK : hip_fail(e);
}

int fft_plan_tune(fft_plan_t p, const void* in, void* out, const fft_mask* mask, void* workspace, void* stream) {
  TraceRange tr("fft_plan_tune");
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (p->kind != 3 || !p->ragged) return FFT_ERR_UNSUPPORTED;
  if (p->batch == 0) return FFT_OK;
  if (!in || !out) return FFT_ERR_ARG;
  if (!workspace) return FFT_ERR_WORKSPACE;
  if (ws_misaligned(workspace)) return FFT_ERR_ARG;
  int rc = plan_check(p, nullptr);
  if (rc != FFT_OK) return rc;
  MaskArgs mk;
  rc = mask_args(mask, p, &mk);
  if (rc != FFT_OK) return rc;
  if (mk.kind != FFT_MASK_NONE && mk.kind != FFT_MASK_GAUSSIAN && mk.kind != FFT_MASK_BUTTERWORTH)
    return FFT_ERR_UNSUPPORTED;
  RaggedSchedule s;
  rc = tune_ragged(p, in, out, mask, workspace, static_cast<hipStream_t>(stream), &s);
  if (rc != FFT_OK) return rc;
  cache_store(cache_key(p, p->ragged), s);
  return FFT_OK;
}

int fft_plan_schedule(fft_plan_t p, int* block, int* wg_cap, int64_t* chunk_bytes, int* order, int* small_side) {
  if (!plan_live(p)) return FFT_ERR_ARG;
  if (p->kind != 3 || !p->ragged) return FFT_ERR_UNSUPPORTED;
  const RaggedSchedule& s = p->ragged->sched;
  if (block) *block = s.block;
  if (wg_cap) *wg_cap = s.wg_cap;
  if (chunk_bytes) *chunk_bytes = s.chunk;
  if (order) *order = s.order;
  if (small_side) *small_side = s.small >= 0 ? 1 << s.small : 0;
  return FFT_OK;
}

}  // extern "C"
