// Device memory cache for the library's own buffers.
//
// hipMalloc and hipFree of the large per-set arrays (CSR, density pyramid,
// illumination grids) and of the voxelizer's temporaries cost milliseconds
// per call, and hipFree synchronises the device. Blocks released by the
// library are therefore kept per device and handed out again to requests
// that fit; hipMalloc runs only on a miss. Sizes are rounded up (powers of
// two below 1 MiB, multiples of 2 MiB above) so repeated work of the same
// shape reuses the same blocks. Cached blocks are returned to the runtime
// when an allocation fails, or by lineset_pool_trim().
//
// Callers must make sure no queued device work still uses a block when they
// release it (the library releases set buffers after a device
// synchronisation and temporaries after synchronising their stream).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "ls_internal.h"

namespace {

constexpr size_t kSmall = 1u << 20;
constexpr size_t kGranule = 2u << 20;

struct DevicePool {
  std::multimap<size_t, void*> free_blocks;   // size -> block
  std::unordered_map<void*, size_t> live;     // block -> size
  size_t cached = 0;
  size_t held = 0;                            // live + cached
};

std::mutex g_mu;
std::vector<DevicePool> g_pools;

DevicePool& pool_for(int device) {
  if ((int)g_pools.size() <= device) g_pools.resize(device + 1);
  return g_pools[device];
}

size_t round_size(size_t bytes) {
  if (bytes == 0) bytes = 1;
  if (bytes < kSmall) {
    size_t r = 512;
    while (r < bytes) r <<= 1;
    return r;
  }
  return (bytes + kGranule - 1) / kGranule * kGranule;
}

// Frees every cached block of `P` (lock held; `device` current).
void release_cached(DevicePool& P) {
  for (auto& kv : P.free_blocks) (void)hipFree(kv.second);
  P.held -= P.cached;
  P.cached = 0;
  P.free_blocks.clear();
}

}  // namespace

int pool_alloc(size_t bytes, void** out, size_t* rounded) {
  *out = nullptr;
  int device = 0;
  LS_HIP(hipGetDevice(&device));
  const size_t need = round_size(bytes);
  std::lock_guard<std::mutex> lk(g_mu);
  DevicePool& P = pool_for(device);
  // smallest cached block that fits, if it wastes at most 1/8 of itself
  auto it = P.free_blocks.lower_bound(need);
  if (it != P.free_blocks.end() && it->first - need <= it->first / 8) {
    *out = it->second;
    if (rounded) *rounded = it->first;
    P.live[it->second] = it->first;
    P.cached -= it->first;
    P.free_blocks.erase(it);
    return LS_OK;
  }
  void* p = nullptr;
  if (hipMalloc(&p, need) != hipSuccess) {
    (void)hipGetLastError();
    release_cached(P);
    if (hipMalloc(&p, need) != hipSuccess) {
      (void)hipGetLastError();
      ls_set_error("device allocation of %zu bytes failed", bytes);
      return LS_ENOMEM;
    }
  }
  P.live[p] = need;
  P.held += need;
  *out = p;
  if (rounded) *rounded = need;
  return LS_OK;
}

void pool_free(void* p) {
  if (!p) return;
  int device = 0;
  (void)hipGetDevice(&device);
  std::lock_guard<std::mutex> lk(g_mu);
  DevicePool& P = pool_for(device);
  auto it = P.live.find(p);
  if (it == P.live.end()) {
    // not ours on this device: look on the others (set freed from another device)
    for (DevicePool& Q : g_pools) {
      auto jt = Q.live.find(p);
      if (jt != Q.live.end()) {
        Q.free_blocks.emplace(jt->second, p);
        Q.cached += jt->second;
        Q.live.erase(jt);
        return;
      }
    }
    return;
  }
  P.free_blocks.emplace(it->second, p);
  P.cached += it->second;
  P.live.erase(it);
}

extern "C" {

void lineset_pool_trim(void) {
  int cur = 0;
  (void)hipGetDevice(&cur);
  std::lock_guard<std::mutex> lk(g_mu);
  for (int d = 0; d < (int)g_pools.size(); ++d) {
    if (g_pools[d].free_blocks.empty()) continue;
    (void)hipSetDevice(d);
    (void)hipDeviceSynchronize();
    release_cached(g_pools[d]);
  }
  (void)hipSetDevice(cur);
}

int lineset_pool_stats(int32_t device, size_t* cached_bytes, size_t* held_bytes) {
  if (device < 0) {
    ls_set_error("lineset_pool_stats: negative device");
    return LS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  size_t c = 0, h = 0;
  if (device < (int)g_pools.size()) {
    c = g_pools[device].cached;
    h = g_pools[device].held;
  }
  if (cached_bytes) *cached_bytes = c;
  if (held_bytes) *held_bytes = h;
  return LS_OK;
}

}  // extern "C"
