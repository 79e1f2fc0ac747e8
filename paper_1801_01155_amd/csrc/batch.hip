// Batched rendering: many views of many resident line sets in one persistent
// launch, optionally replayed from a hipGraph, with a tile-shape / grid-size
// autotuner. The per-pixel work is the plain renderer's (render.hip), so a
// view renders the same image alone and in a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "render_args.h"

struct ls_batch {
  int device = 0;
  int n_views = 0;
  int total_tiles = 0;
  int32_t flags = 0;
  bool vdi = false;          // some view uses per-fragment illumination
  BatchPlan plan{2, 2, 0};
  BatchQueues queues{};
  std::vector<ls_view> views;
  std::vector<RenderArgs> args;
  std::vector<int32_t> tile_start;
  RenderArgs* d_args = nullptr;
  int32_t* d_tile_start = nullptr;
  unsigned* d_queue = nullptr;  // 8 queue counters + RenderCounters
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  float tuned_ms = 0.f;
  int autotuned = 0;
  int candidates = 0;
};

namespace {

constexpr int kQueueWords = 8 + (int)(sizeof(RenderCounters) / sizeof(unsigned));

std::mutex g_cache_mu;
std::map<std::string, BatchPlan> g_plan_cache;

// The extended kernel instance (see view_dependent in render_args.h).
bool view_dependent_params(const ls_view& v) {
  return (v.params.shading == 2 && (v.params.ao_mode != 0 || v.params.shadow_mode != 0)) ||
         (v.set && v.set->ends != nullptr) || (!v.params.opaque && v.params.accel_depth > 0.f);
}

std::string signature(const std::vector<ls_view>& v) {
  std::string k;
  for (const auto& x : v) {
    k += std::to_string(x.cam.width) + "x" + std::to_string(x.cam.height) + "m" +
         std::to_string(x.params.mode) + "o" + std::to_string(x.params.opaque) +
         (view_dependent_params(x) ? "v;" : ";");
  }
  return k;
}

void free_batch(ls_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->d_args) (void)hipFree(b->d_args);
  if (b->d_tile_start) (void)hipFree(b->d_tile_start);
  if (b->d_queue) (void)hipFree(b->d_queue);
  b->exec = nullptr;
  b->graph = nullptr;
  b->cap_stream = nullptr;
  b->d_args = nullptr;
  b->d_tile_start = nullptr;
  b->d_queue = nullptr;
}

// Builds the descriptors for a tile shape and uploads them.
int prepare(ls_batch* b, const BatchPlan& plan, hipStream_t st) {
  b->plan = plan;
  b->args.resize(b->n_views);
  b->tile_start.resize(b->n_views + 1);
  int64_t total = 0;
  for (int v = 0; v < b->n_views; ++v) {
    const ls_view& x = b->views[v];
    make_render_args(x.set, &x.cam, &x.params, x.rgba_out, plan.wx, plan.wy, nullptr, &b->args[v]);
    b->tile_start[v] = (int32_t)total;
    total += b->args[v].n_tiles;
  }
  if (total > (1ll << 30)) {
    ls_set_error("batch has too many tiles");
    return LS_EINVAL;
  }
  b->tile_start[b->n_views] = (int32_t)total;
  b->total_tiles = (int)total;
  b->queues = make_queues(b->total_tiles);
  LS_HIP(hipMemcpyAsync(b->d_args, b->args.data(), sizeof(RenderArgs) * b->n_views,
                        hipMemcpyHostToDevice, st));
  LS_HIP(hipMemcpyAsync(b->d_tile_start, b->tile_start.data(), sizeof(int32_t) * (b->n_views + 1),
                        hipMemcpyHostToDevice, st));
  LS_HIP(hipStreamSynchronize(st));
  return LS_OK;
}

int launch(ls_batch* b, bool count, hipStream_t st) {
  int rc;
  if ((rc = fill_u32(b->d_queue, 0u, count ? kQueueWords : 8, st))) return rc;
  return launch_render_batch(b->d_args, b->d_tile_start, b->n_views, b->queues, b->d_queue,
                             b->plan, count, b->vdi, st);
}

int plan_blocks(int wx, int wy, int mult, bool vdi, int* blocks) {
  int dev = 0, per_cu = 1;
  LS_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  LS_HIP(hipGetDeviceProperties(&prop, dev));
  int rc;
  if ((rc = batch_blocks_per_cu(wx, wy, vdi, &per_cu))) return rc;
  *blocks = prop.multiProcessorCount * per_cu * mult;
  return LS_OK;
}

// Times every candidate (tile shape x persistent grid size) on this batch and
// keeps the fastest; results are cached per batch signature.
constexpr int kShapes[][2] = {{2, 2}, {4, 1}, {1, 4}, {2, 1}, {1, 2}, {1, 1}};
constexpr int kMults[] = {1, 2};

int autotune(ls_batch* b, hipStream_t st) {
  const auto& shapes = kShapes;
  const auto& mults = kMults;
  hipEvent_t e0, e1;
  LS_HIP(hipEventCreate(&e0));
  LS_HIP(hipEventCreate(&e1));
  BatchPlan best{2, 2, 0};
  float best_ms = 1e30f;
  int rc = LS_OK, n = 0;
  for (const auto& sh : shapes) {
    for (int mult : mults) {
      BatchPlan p{sh[0], sh[1], 0};
      if ((rc = plan_blocks(p.wx, p.wy, mult, b->vdi, &p.blocks))) break;
      if ((rc = prepare(b, p, st))) break;
      if ((rc = launch(b, false, st))) break;  // warm
      LS_HIP(hipEventRecord(e0, st));
      for (int r = 0; r < 2 && !rc; ++r) rc = launch(b, false, st);
      LS_HIP(hipEventRecord(e1, st));
      LS_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      LS_HIP(hipEventElapsedTime(&ms, e0, e1));
      ms *= 0.5f;
      ++n;
      if (ms < best_ms) {
        best_ms = ms;
        best = p;
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  b->tuned_ms = best_ms;
  b->autotuned = 1;
  b->candidates = n;
  return prepare(b, best, st);
}

int capture(ls_batch* b) {
  LS_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  LS_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = launch(b, false, b->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) {
    ls_set_error("hipStreamEndCapture: %s", hipGetErrorString(e));
    return LS_EDEVICE;
  }
  b->graph = g;
  LS_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return LS_OK;
}

// Allocation-free one-shot batch (lineset_render_batch_static): queue
// counters, tile starts and view descriptors live in one file-scope device
// array per GPU instead of hipMalloc'd buffers.
constexpr int kStaticViews = 256;
constexpr size_t kStaticQueueOff = 0;
constexpr size_t kStaticTileOff = 256;  // after the queue words
constexpr size_t kStaticArgsOff =
    (kStaticTileOff + sizeof(int32_t) * (kStaticViews + 1) + 255) / 256 * 256;
constexpr size_t kStaticBytes = kStaticArgsOff + sizeof(RenderArgs) * kStaticViews;
static_assert(sizeof(unsigned) * 8 <= kStaticTileOff, "queue words overlap the tile starts");

constexpr int kStaticDevices = 64;
std::mutex g_static_mu;
unsigned char* g_static_ptr[kStaticDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the array's host-side name is not an address).
int static_scratch(int dev, unsigned char** out);

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
int static_scratch(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kStaticDevices) {
    ls_set_error("lineset_render_batch_static: device %d out of range", dev);
    return LS_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      ls_set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
      return LS_EDEVICE;
    }
    g_static_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_static_ptr[dev];
  return LS_OK;
}
}  // namespace

extern "C" {

// fixed: a plan (wx, wy, grid multiplier) chosen by the caller instead of the
// cache / autotuner / default.
static int create_batch(const ls_view* views, int32_t n_views, int32_t flags, const int32_t* fixed,
                        void* hip_stream, ls_batch_t* out) {
  if (!out) {
    ls_set_error("lineset_batch_create: out is NULL");
    return LS_EINVAL;
  }
  *out = nullptr;
  if (!views || n_views < 1 || n_views > (1 << 20)) {
    ls_set_error("lineset_batch_create: need 1 .. 2^20 views");
    return LS_EINVAL;
  }
  int rc;
  for (int v = 0; v < n_views; ++v)
    if ((rc = check_render(views[v].set, &views[v].cam, &views[v].params, views[v].rgba_out))) {
      return rc;
    }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  ls_batch* b = new (std::nothrow) ls_batch();
  if (!b) {
    ls_set_error("host allocation failed");
    return LS_ENOMEM;
  }
  b->n_views = n_views;
  b->flags = flags;
  b->views.assign(views, views + n_views);
  for (const ls_view& x : b->views) b->vdi = b->vdi || view_dependent_params(x);
  (void)hipGetDevice(&b->device);
  auto fail = [&](int code) {
    (void)hipStreamSynchronize(st);
    free_batch(b);
    delete b;
    return code;
  };
  if (hipMalloc(&b->d_args, sizeof(RenderArgs) * n_views) != hipSuccess ||
      hipMalloc(&b->d_tile_start, sizeof(int32_t) * (n_views + 1)) != hipSuccess ||
      hipMalloc(&b->d_queue, sizeof(unsigned) * kQueueWords) != hipSuccess) {
    (void)hipGetLastError();
    ls_set_error("device allocation failed");
    return fail(LS_ENOMEM);
  }
  const std::string key = signature(b->views);
  BatchPlan cached{0, 0, 0};
  if (!fixed) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_plan_cache.find(key);
    if (it != g_plan_cache.end()) cached = it->second;
  }
  if (fixed) {
    BatchPlan p{fixed[0], fixed[1], 0};
    rc = plan_blocks(p.wx, p.wy, fixed[2], b->vdi, &p.blocks);
    if (!rc) rc = prepare(b, p, st);
  } else if (cached.blocks > 0) {
    rc = prepare(b, cached, st);
    b->autotuned = 2;  // from the cache
  } else if (flags & LS_BATCH_AUTOTUNE) {
    rc = autotune(b, st);
    if (!rc) {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      g_plan_cache[key] = b->plan;
    }
  } else {
    BatchPlan p{2, 2, 0};
    rc = plan_blocks(p.wx, p.wy, 1, b->vdi, &p.blocks);
    if (!rc) rc = prepare(b, p, st);
  }
  if (!rc && (flags & LS_BATCH_GRAPH)) rc = capture(b);
  if (rc) return fail(rc);
  *out = b;
  return LS_OK;
}

int lineset_batch_create(const ls_view* views, int32_t n_views, int32_t flags, void* hip_stream,
                         ls_batch_t* out) {
  return create_batch(views, n_views, flags, nullptr, hip_stream, out);
}

int lineset_batch_candidates(int32_t* waves_x, int32_t* waves_y, int32_t* grid_mult, int32_t cap,
                             int32_t* n) {
  if (!n || (cap > 0 && (!waves_x || !waves_y || !grid_mult))) {
    ls_set_error("lineset_batch_candidates: null argument");
    return LS_EINVAL;
  }
  int k = 0;
  for (const auto& sh : kShapes)
    for (int m : kMults) {
      if (k < cap) {
        waves_x[k] = sh[0];
        waves_y[k] = sh[1];
        grid_mult[k] = m;
      }
      ++k;
    }
  *n = k;
  return LS_OK;
}

int lineset_batch_create_plan(const ls_view* views, int32_t n_views, int32_t waves_x,
                              int32_t waves_y, int32_t grid_mult, int32_t flags, void* hip_stream,
                              ls_batch_t* out) {
  bool known = false;
  for (const auto& sh : kShapes) known = known || (sh[0] == waves_x && sh[1] == waves_y);
  if (!known || grid_mult < 1 || grid_mult > 8) {
    if (out) *out = nullptr;
    ls_set_error("lineset_batch_create_plan: tile shape not one of the candidates, or grid "
                 "multiplier outside [1, 8]");
    return LS_EINVAL;
  }
  if (flags & LS_BATCH_AUTOTUNE) {
    if (out) *out = nullptr;
    ls_set_error("lineset_batch_create_plan: a fixed plan is not autotuned");
    return LS_EINVAL;
  }
  const int32_t fixed[3] = {waves_x, waves_y, grid_mult};
  return create_batch(views, n_views, flags, fixed, hip_stream, out);
}

int lineset_batch_render(ls_batch_t b, void* hip_stream) {
  if (!b) {
    ls_set_error("lineset_batch_render: batch is NULL");
    return LS_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (b->exec) {
    LS_HIP(hipGraphLaunch(b->exec, st));
    return LS_OK;
  }
  return launch(b, false, st);
}

int lineset_batch_render_counted(ls_batch_t b, ls_render_counters* c, void* hip_stream) {
  if (!b || !c) {
    ls_set_error("lineset_batch_render_counted: null argument");
    return LS_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int rc;
  if ((rc = launch(b, true, st))) return rc;
  RenderCounters h{};
  LS_HIP(hipMemcpyAsync(&h, b->d_queue + 8, sizeof(h), hipMemcpyDeviceToHost, st));
  LS_HIP(hipStreamSynchronize(st));
  export_counters(h, c);
  return LS_OK;
}

int lineset_batch_config(ls_batch_t b, ls_batch_config* o) {
  if (!b || !o) {
    ls_set_error("lineset_batch_config: null argument");
    return LS_EINVAL;
  }
  o->waves_x = b->plan.wx;
  o->waves_y = b->plan.wy;
  o->blocks = b->plan.blocks;
  o->n_tiles = b->total_tiles;
  o->autotuned = b->autotuned;
  o->candidates = b->candidates;
  o->tuned_ms = b->tuned_ms;
  o->graph = b->exec != nullptr;
  return LS_OK;
}

void lineset_batch_destroy(ls_batch_t b) {
  if (!b) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != b->device) (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  free_batch(b);
  if (cur != b->device) (void)hipSetDevice(cur);
  delete b;
}

int lineset_render_batch_static(const ls_view* views, int32_t n_views, void* hip_stream) {
  if (!views || n_views < 1 || n_views > kStaticViews) {
    ls_set_error("lineset_render_batch_static: need 1 .. %d views", kStaticViews);
    return LS_EINVAL;
  }
  int rc;
  for (int v = 0; v < n_views; ++v)
    if ((rc = check_render(views[v].set, &views[v].cam, &views[v].params, views[v].rgba_out))) {
      return rc;
    }
  int dev = 0;
  LS_HIP(hipGetDevice(&dev));
  unsigned char* base = nullptr;
  if ((rc = static_scratch(dev, &base))) return rc;
  // Host staging on the stack (no heap): the copies below read it before the
  // stream synchronisation at the end returns.
  RenderArgs args[kStaticViews];
  int32_t tile_start[kStaticViews + 1];
  BatchPlan plan{2, 2, 0};
  bool vdi = false;
  for (int v = 0; v < n_views; ++v) vdi = vdi || view_dependent_params(views[v]);
  if ((rc = plan_blocks(plan.wx, plan.wy, 1, vdi, &plan.blocks))) return rc;
  int64_t total = 0;
  for (int v = 0; v < n_views; ++v) {
    const ls_view& x = views[v];
    make_render_args(x.set, &x.cam, &x.params, x.rgba_out, plan.wx, plan.wy, nullptr, &args[v]);
    tile_start[v] = (int32_t)total;
    total += args[v].n_tiles;
  }
  if (total > (1ll << 30)) {
    ls_set_error("lineset_render_batch_static: batch has too many tiles");
    return LS_EINVAL;
  }
  tile_start[n_views] = (int32_t)total;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  unsigned* d_queue = reinterpret_cast<unsigned*>(base + kStaticQueueOff);
  int32_t* d_tiles = reinterpret_cast<int32_t*>(base + kStaticTileOff);
  RenderArgs* d_args = reinterpret_cast<RenderArgs*>(base + kStaticArgsOff);
  LS_HIP(hipMemcpyAsync(d_args, args, sizeof(RenderArgs) * n_views, hipMemcpyHostToDevice, st));
  LS_HIP(hipMemcpyAsync(d_tiles, tile_start, sizeof(int32_t) * (n_views + 1),
                        hipMemcpyHostToDevice, st));
  rc = fill_u32(d_queue, 0u, 8, st);
  if (!rc) {
    rc = launch_render_batch(d_args, d_tiles, n_views, make_queues((int)total), d_queue, plan,
                             false, vdi, st);
  }
  // Synchronise on every path from here: the copies read the stack arrays.
  if (hipStreamSynchronize(st) != hipSuccess && !rc) {
    ls_set_error("lineset_render_batch_static: stream synchronisation failed");
    rc = LS_EDEVICE;
  }
  return rc;
}

int lineset_render_batch(const ls_view* views, int32_t n_views, void* hip_stream) {
  ls_batch_t b = nullptr;
  int rc = lineset_batch_create(views, n_views, 0, hip_stream, &b);
  if (rc) return rc;
  rc = lineset_batch_render(b, hip_stream);
  if (!rc && hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)) != hipSuccess) {
    ls_set_error("lineset_render_batch: stream synchronisation failed");
    rc = LS_EDEVICE;
  }
  lineset_batch_destroy(b);
  return rc;
}

}  // extern "C"
