// Render server: resident line sets, admission by an HBM budget, continuous
// batching of render requests into persistent batched launches.
//
// A scheduler thread owns `n_slots` launch slots (a stream, an event and
// pre-allocated descriptor buffers each). Whenever a slot is free and
// requests wait, it takes the queue's head requests (FIFO) whose memory
// reservation fits the budget into one batched launch on that slot's stream;
// requests that arrive while batches run are admitted into the next free
// slot, so several batches overlap on the device. Completion is observed by
// polling the slots' events.
//
// Memory: the budget holds the resident sets, the optional output arena
// (device memory the server owns, allocated at creation) and the outputs
// being written by requests in flight. A request submitted without an
// output buffer renders into a block of the arena, taken first-fit at
// admission and returned when the caller copies the image out; a request
// whose block does not fit waits at the head of the queue. Device memory is
// allocated only at creation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "render_args.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket;
  int32_t set_id;
  ls_camera cam;
  ls_render_params params;
  float* out;            // caller's buffer, or the arena block once admitted
  bool arena = false;    // output in the server's arena
  size_t bytes;          // caller's buffer: output bytes in flight; arena: block size
  size_t arena_off = 0;
  Clock::time_point t_submit, t_done;
  int state;             // 0 queued, 1 running, 2 done
  bool held = false;     // was once at the queue head without room in the budget
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
};

constexpr int kQueueWords = 8 + (int)(sizeof(RenderCounters) / sizeof(unsigned));

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  RenderArgs* d_args = nullptr;
  int32_t* d_tile_start = nullptr;
  unsigned* d_queue = nullptr;
  RenderArgs* h_args = nullptr;      // pinned
  int32_t* h_tile_start = nullptr;   // pinned
  std::vector<Request*> reqs;
  size_t bytes = 0;      // output bytes of the caller-owned requests in the batch
  bool busy = false;
};

}  // namespace

struct ls_server {
  ls_server_config cfg{};
  int device = 0;
  BatchPlan plan{2, 2, 0};
  std::vector<ls_lineset_t> sets;
  size_t resident = 0;      // bytes of the sets at the last admission pass
  std::vector<hipEvent_t> free_events;  // submission events, reused
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> by_ticket;
  std::vector<Slot> slots;
  std::thread sched;
  bool stop = false;
  size_t inflight = 0;      // output bytes of caller-owned requests in flight
  uint64_t next_ticket = 1;
  // output arena: base, size, free blocks (offset -> size, coalesced), bytes in use
  char* arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  std::map<size_t, size_t> arena_free;
  uint64_t arena_returns = 0;   // blocks given back (wakes a scheduler waiting for space)
  // statistics
  std::vector<double> lat_ms;
  uint64_t rays_done = 0, batches = 0, batched_views = 0, rejected = 0, max_depth = 0;
  uint64_t held = 0;
  bool have_first = false;
  Clock::time_point t_first, t_last;
  int launch_error = 0;
};

namespace {

constexpr size_t kArenaAlign = 256;

size_t image_bytes(const ls_camera& c) { return (size_t)c.width * (size_t)c.height * 16; }

size_t reservation(const ls_camera& c) { return image_bytes(c) + sizeof(RenderArgs); }

size_t arena_block(const ls_camera& c) {
  return (image_bytes(c) + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
}

// First-fit block of `len` bytes from the arena's free list.
bool arena_take(ls_server* S, size_t len, size_t* off) {
  for (auto it = S->arena_free.begin(); it != S->arena_free.end(); ++it) {
    if (it->second < len) continue;
    *off = it->first;
    const size_t rest = it->second - len;
    const size_t at = it->first + len;
    S->arena_free.erase(it);
    if (rest) S->arena_free[at] = rest;
    S->arena_used += len;
    return true;
  }
  return false;
}

void arena_give(ls_server* S, size_t off, size_t len) {
  S->arena_used -= len;
  auto it = S->arena_free.emplace(off, len).first;
  auto nx = std::next(it);
  if (nx != S->arena_free.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    S->arena_free.erase(nx);
  }
  if (it != S->arena_free.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      S->arena_free.erase(it);
    }
  }
}

// Device bytes of the resident sets now: a set grows when its density
// pyramid or illumination grids are built after it was added.
size_t resident_bytes(const ls_server* S) {
  size_t b = 0;
  for (const ls_lineset* s : S->sets) b += s->bytes;
  return b;
}

// Builds and launches one batch on slot `sl` (caller holds the lock).
int launch_slot(ls_server* S, Slot& sl) {
  const int n = (int)sl.reqs.size();
  int64_t total = 0;
  for (int k = 0; k < n; ++k) {
    Request* r = sl.reqs[k];
    make_render_args(S->sets[r->set_id], &r->cam, &r->params, r->out, S->plan.wx, S->plan.wy,
                     nullptr, &sl.h_args[k]);
    sl.h_tile_start[k] = (int32_t)total;
    total += sl.h_args[k].n_tiles;
  }
  sl.h_tile_start[n] = (int32_t)total;
  const BatchQueues q = make_queues((int)total);
  bool vdi = false;
  for (int k = 0; k < n; ++k) vdi = vdi || view_dependent(sl.h_args[k]);
  // each request's inputs and output were produced on its submitter's stream
  for (Request* r : sl.reqs) LS_HIP(hipStreamWaitEvent(sl.stream, r->ready, 0));
  LS_HIP(hipMemcpyAsync(sl.d_args, sl.h_args, sizeof(RenderArgs) * n, hipMemcpyHostToDevice,
                        sl.stream));
  LS_HIP(hipMemcpyAsync(sl.d_tile_start, sl.h_tile_start, sizeof(int32_t) * (n + 1),
                        hipMemcpyHostToDevice, sl.stream));
  int rc;
  if ((rc = fill_u32(sl.d_queue, 0u, 8, sl.stream))) return rc;
  if ((rc = launch_render_batch(sl.d_args, sl.d_tile_start, n, q, sl.d_queue, S->plan, false,
                                vdi, sl.stream)))
    return rc;
  LS_HIP(hipEventRecord(sl.done, sl.stream));
  return LS_OK;
}

void scheduler(ls_server* S) {
  (void)hipSetDevice(S->device);
  const size_t budget = S->cfg.hbm_budget_bytes;
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    // retire finished batches
    bool any_busy = false;
    for (Slot& sl : S->slots) {
      if (!sl.busy) continue;
      hipError_t e = hipEventQuery(sl.done);
      if (e == hipErrorNotReady) {
        any_busy = true;
        continue;
      }
      const auto now = Clock::now();
      for (Request* r : sl.reqs) {
        S->free_events.push_back(r->ready);
        r->ready = nullptr;
        r->state = 2;
        r->t_done = now;
        S->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
        S->rays_done += (uint64_t)r->cam.width * r->cam.height;
      }
      S->t_last = now;
      S->inflight -= sl.bytes;
      sl.reqs.clear();
      sl.bytes = 0;
      sl.busy = false;
      if (e != hipSuccess) S->launch_error = LS_EDEVICE;
      S->cv_done.notify_all();
    }
    // admit queued requests into free slots
    S->resident = resident_bytes(S);
    bool head_blocked = false;
    for (Slot& sl : S->slots) {
      if (sl.busy || S->queue.empty()) continue;
      while (!S->queue.empty() && (int)sl.reqs.size() < S->cfg.max_batch_views) {
        Request* r = S->queue.front();
        size_t off = 0;
        const bool fits =
            r->arena ? arena_take(S, r->bytes, &off)
                     : S->resident + S->arena_bytes + S->inflight + sl.bytes + r->bytes <= budget;
        if (!fits) {
          if (!r->held) {
            r->held = true;
            S->held++;
          }
          head_blocked = true;
          break;
        }
        S->queue.pop_front();
        r->state = 1;
        sl.reqs.push_back(r);
        if (r->arena) {
          r->arena_off = off;
          r->out = reinterpret_cast<float*>(S->arena + off);
        } else {
          sl.bytes += r->bytes;
        }
      }
      if (sl.reqs.empty()) break;  // the head does not fit until memory frees
      S->inflight += sl.bytes;
      sl.busy = true;
      any_busy = true;
      S->batches++;
      S->batched_views += sl.reqs.size();
      if (launch_slot(S, sl) != LS_OK) S->launch_error = LS_EDEVICE;
    }
    // nothing in flight and the head waits for arena blocks the caller has
    // not collected: at shutdown it can never run
    if (S->stop && !any_busy && (S->queue.empty() || head_blocked)) break;
    if (any_busy) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else if (head_blocked) {
      const uint64_t seen = S->arena_returns;
      S->cv_work.wait(lk, [&] { return S->stop || S->arena_returns != seen; });
    } else {
      S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
    }
  }
}

void free_server(ls_server* S) {
  for (Slot& sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.d_args) (void)hipFree(sl.d_args);
    if (sl.d_tile_start) (void)hipFree(sl.d_tile_start);
    if (sl.d_queue) (void)hipFree(sl.d_queue);
    if (sl.h_args) (void)hipHostFree(sl.h_args);
    if (sl.h_tile_start) (void)hipHostFree(sl.h_tile_start);
  }
  if (S->arena) (void)hipFree(S->arena);
  S->arena = nullptr;
  for (auto& kv : S->by_ticket) {
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    delete kv.second;
  }
  for (Request* r : S->queue) {
    if (S->by_ticket.count(r->ticket)) continue;
    if (r->ready) (void)hipEventDestroy(r->ready);
    delete r;
  }
  for (hipEvent_t e : S->free_events) (void)hipEventDestroy(e);
  S->free_events.clear();
}

}  // namespace

extern "C" {

int ls_server_create(const ls_server_config* cfg, ls_server_t* out) {
  if (!out || !cfg) {
    ls_set_error("ls_server_create: null argument");
    return LS_EINVAL;
  }
  *out = nullptr;
  if (cfg->n_slots < 1 || cfg->n_slots > 16 || cfg->max_batch_views < 1 ||
      cfg->max_batch_views > 4096 || cfg->max_queue < 1 || cfg->hbm_budget_bytes == 0 ||
      cfg->output_arena_bytes > cfg->hbm_budget_bytes) {
    ls_set_error("ls_server_create: need 1..16 slots, 1..4096 views per batch, max_queue >= 1, "
                 "a non-zero budget holding the output arena");
    return LS_EINVAL;
  }
  ls_server* S = new (std::nothrow) ls_server();
  if (!S) {
    ls_set_error("host allocation failed");
    return LS_ENOMEM;
  }
  S->cfg = *cfg;
  (void)hipGetDevice(&S->device);
  int per_cu = 1;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, S->device) != hipSuccess ||
      batch_blocks_per_cu(2, 2, false, &per_cu) != LS_OK) {
    delete S;
    ls_set_error("ls_server_create: device query failed");
    return LS_EDEVICE;
  }
  S->plan = BatchPlan{2, 2, prop.multiProcessorCount * per_cu};
  S->slots.resize(cfg->n_slots);
  const int nv = cfg->max_batch_views;
  for (Slot& sl : S->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&sl.d_args, sizeof(RenderArgs) * nv) != hipSuccess ||
        hipMalloc(&sl.d_tile_start, sizeof(int32_t) * (nv + 1)) != hipSuccess ||
        hipMalloc(&sl.d_queue, sizeof(unsigned) * kQueueWords) != hipSuccess ||
        hipHostMalloc(&sl.h_args, sizeof(RenderArgs) * nv, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&sl.h_tile_start, sizeof(int32_t) * (nv + 1), hipHostMallocDefault) !=
            hipSuccess) {
      (void)hipGetLastError();
      free_server(S);
      delete S;
      ls_set_error("ls_server_create: allocation failed");
      return LS_ENOMEM;
    }
  }
  if (cfg->output_arena_bytes > 0) {
    S->arena_bytes = cfg->output_arena_bytes / kArenaAlign * kArenaAlign;
    if (S->arena_bytes == 0 || hipMalloc(&S->arena, S->arena_bytes) != hipSuccess) {
      (void)hipGetLastError();
      S->arena = nullptr;
      free_server(S);
      delete S;
      ls_set_error("ls_server_create: output arena of %zu bytes not allocated",
                   (size_t)cfg->output_arena_bytes);
      return LS_ENOMEM;
    }
    S->arena_free[0] = S->arena_bytes;
  }
  S->sched = std::thread(scheduler, S);
  *out = S;
  return LS_OK;
}

int ls_server_add_lineset(ls_server_t S, ls_lineset_t set, int32_t* set_id) {
  if (!S || !set || !set_id) {
    ls_set_error("ls_server_add_lineset: null argument");
    return LS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  S->resident = resident_bytes(S);
  if (S->resident + S->arena_bytes + set->bytes > S->cfg.hbm_budget_bytes) {
    ls_set_error("ls_server_add_lineset: resident sets would exceed the HBM budget");
    return LS_ENOMEM;
  }
  S->resident += set->bytes;
  S->sets.push_back(set);
  *set_id = (int32_t)S->sets.size() - 1;
  return LS_OK;
}

int ls_server_submit(ls_server_t S, int32_t set_id, const ls_camera* cam,
                     const ls_render_params* params, float* rgba_out, void* hip_stream,
                     uint64_t* ticket) {
  if (!S || !cam || !params || !ticket) {
    ls_set_error("ls_server_submit: null argument");
    return LS_EINVAL;
  }
  int rc;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (set_id < 0 || set_id >= (int32_t)S->sets.size()) {
      ls_set_error("ls_server_submit: unknown set id %d", set_id);
      return LS_EINVAL;
    }
    const bool in_arena = rgba_out == nullptr;
    if (in_arena && !S->arena) {
      ls_set_error("ls_server_submit: rgba_out is NULL and the server has no output arena");
      return LS_EINVAL;
    }
    // an arena request is validated against the (aligned) arena base
    if ((rc = check_render(S->sets[set_id], cam, params,
                           in_arena ? reinterpret_cast<const float*>(S->arena) : rgba_out)))
      return rc;
    const size_t bytes = in_arena ? arena_block(*cam) : reservation(*cam);
    S->resident = resident_bytes(S);
    if (in_arena ? bytes > S->arena_bytes
                 : S->resident + S->arena_bytes + bytes > S->cfg.hbm_budget_bytes) {
      ls_set_error("ls_server_submit: request needs %zu bytes, more than the %s can hold", bytes,
                   in_arena ? "output arena" : "budget");
      return LS_ENOMEM;
    }
    if ((int)S->queue.size() >= S->cfg.max_queue) {
      S->rejected++;
      ls_set_error("ls_server_submit: queue full");
      return LS_EBUSY;
    }
    Request* r = new (std::nothrow) Request();
    if (!r) {
      ls_set_error("host allocation failed");
      return LS_ENOMEM;
    }
    if (!S->free_events.empty()) {
      r->ready = S->free_events.back();
      S->free_events.pop_back();
    } else if (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      delete r;
      ls_set_error("ls_server_submit: event creation failed");
      return LS_EDEVICE;
    }
    if (hipEventRecord(r->ready, static_cast<hipStream_t>(hip_stream)) != hipSuccess) {
      (void)hipGetLastError();
      S->free_events.push_back(r->ready);
      delete r;
      ls_set_error("ls_server_submit: recording on the caller's stream failed");
      return LS_EDEVICE;
    }
    r->ticket = S->next_ticket++;
    r->set_id = set_id;
    r->cam = *cam;
    r->params = *params;
    r->out = rgba_out;
    r->arena = in_arena;
    r->bytes = bytes;
    r->state = 0;
    r->t_submit = Clock::now();
    if (!S->have_first) {
      S->have_first = true;
      S->t_first = r->t_submit;
    }
    S->queue.push_back(r);
    S->by_ticket[r->ticket] = r;
    S->max_depth = std::max<uint64_t>(S->max_depth, S->queue.size());
    *ticket = r->ticket;
  }
  S->cv_work.notify_one();
  return LS_OK;
}

int ls_server_wait(ls_server_t S, uint64_t ticket, int64_t timeout_us) {
  if (!S) {
    ls_set_error("ls_server_wait: null server");
    return LS_EINVAL;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->by_ticket.find(ticket);
  if (it == S->by_ticket.end()) {
    ls_set_error("ls_server_wait: unknown or already collected ticket");
    return LS_EINVAL;
  }
  Request* r = it->second;
  auto done = [&] { return r->state == 2; };
  if (timeout_us < 0) {
    S->cv_done.wait(lk, done);
  } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
    ls_set_error("ls_server_wait: timed out");
    return LS_ETIMEOUT;
  }
  if (!r->arena) {
    // an arena request stays until ls_server_result copies its image out
    S->by_ticket.erase(it);
    delete r;
  }
  if (S->launch_error) {
    ls_set_error("ls_server_wait: a batched launch failed");
    return S->launch_error;
  }
  return LS_OK;
}

int ls_server_result(ls_server_t S, uint64_t ticket, float* dst, size_t dst_bytes,
                     int32_t dst_on_device, void* hip_stream) {
  if (!S || !dst) {
    ls_set_error("ls_server_result: null argument");
    return LS_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->by_ticket.find(ticket);
    if (it == S->by_ticket.end() || !it->second->arena) {
      ls_set_error("ls_server_result: unknown ticket, already collected, or not an arena request");
      return LS_EINVAL;
    }
    r = it->second;
    if (r->state != 2) {
      ls_set_error("ls_server_result: request not complete (ls_server_wait first)");
      return LS_EBUSY;
    }
    if (dst_bytes < image_bytes(r->cam)) {
      ls_set_error("ls_server_result: destination holds %zu bytes, %zu needed", dst_bytes,
                   image_bytes(r->cam));
      return LS_EINVAL;
    }
  }
  // the block is still held: no other request writes it until it is returned
  const hipError_t e1 = hipMemcpyAsync(dst, r->out, image_bytes(r->cam),
                                       dst_on_device ? hipMemcpyDeviceToDevice
                                                     : hipMemcpyDeviceToHost, st);
  const hipError_t e2 = e1 == hipSuccess ? hipStreamSynchronize(st) : e1;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    arena_give(S, r->arena_off, r->bytes);
    S->arena_returns++;
    S->by_ticket.erase(ticket);
    delete r;
  }
  S->cv_work.notify_one();   // a request held for arena space may fit now
  if (e2 != hipSuccess) {
    (void)hipGetLastError();
    ls_set_error("ls_server_result: copy failed: %s", hipGetErrorString(e2));
    return LS_EDEVICE;
  }
  return LS_OK;
}

int ls_server_stats(ls_server_t S, ls_server_report* o) {
  if (!S || !o) {
    ls_set_error("ls_server_stats: null argument");
    return LS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  std::vector<double> l = S->lat_ms;
  std::sort(l.begin(), l.end());
  auto pct = [&](double p) {
    if (l.empty()) return 0.0;
    size_t k = (size_t)std::min<double>((double)l.size() - 1, p * (double)(l.size() - 1) + 0.5);
    return l[k];
  };
  o->completed = (int64_t)l.size();
  o->p50_ms = pct(0.50);
  o->p99_ms = pct(0.99);
  o->max_ms = l.empty() ? 0.0 : l.back();
  double span = S->have_first && !l.empty()
                    ? std::chrono::duration<double>(S->t_last - S->t_first).count()
                    : 0.0;
  o->mrays_per_s = span > 0 ? (double)S->rays_done / span / 1e6 : 0.0;
  o->batches = (int64_t)S->batches;
  o->mean_batch = S->batches ? (double)S->batched_views / (double)S->batches : 0.0;
  o->queued = (int64_t)S->queue.size();
  o->max_queue_depth = (int64_t)S->max_depth;
  o->rejected = (int64_t)S->rejected;
  o->held_for_memory = (int64_t)S->held;
  o->resident_bytes = S->resident;
  o->inflight_bytes = S->inflight;
  o->arena_bytes = S->arena_bytes;
  o->arena_in_use = S->arena_used;
  return LS_OK;
}

void ls_server_destroy(ls_server_t S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->sched.joinable()) S->sched.join();
  free_server(S);
  delete S;
}

}  // extern "C"
