// Incremental update of a voxelized line set: curves removed by id and new
// curves appended, without re-voxelizing the curves that stay (section
// "Voxel-based curve discretization", first paragraph: on the GPU the
// pre-process allows instant updates when curves are removed or added; the
// conclusion names local updates and time-varying line sets as the next
// step).
//
// The result equals voxelizing the edited curve list from scratch: the old
// curves keep their ids (a removed curve contributes nothing) and the added
// ones take the ids that follow. A voxel's list is ordered by (curve id,
// position along the curve), so its new list is its old records minus the
// removed curves' followed by the added curves' records:
//   1. the added curves are voxelized on their own (same kernels, curve tags
//      offset by the old curve count), mapped with the set's grid set-up;
//   2. k_merge_count: thread per voxel, kept old records + added records;
//   3. exclusive scan -> new offsets;
//   4. k_merge_scatter: thread per voxel, copies the kept records, then the
//      added ones, into the new record array;
//   5. occupancy words and list statistics of the new lists.
// Curve ids live in the records' 24-bit curve tag, so updates need at most
// 2^24 curves. The density pyramid and illumination grids describe the old
// lines: they are released, and lineset_build_lod rebuilds them.
#include <hip/hip_runtime.h>

#include <new>
#include <vector>

#include "ls_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int64_t kMaxTagged = 1ll << 24;

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__device__ inline bool removed(const uint32_t* mask, uint64_t rec) {
  if (!mask) return false;
  const uint32_t tag = (uint32_t)(rec >> 40);
  return (mask[tag >> 5] >> (tag & 31)) & 1u;
}

__global__ __launch_bounds__(kBlock) void k_mark_removed(const int64_t* ids, int64_t n,
                                                         int64_t n_curves, uint32_t* mask,
                                                         int* err) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const int64_t id = ids[k];
  if (id < 0 || id >= n_curves) {
    atomicOr(err, 1);
    return;
  }
  atomicOr(mask + (id >> 5), 1u << (id & 31));
}

// counts[v] = kept records of v + added records of v
__global__ __launch_bounds__(kBlock) void k_merge_count(const uint32_t* off, const uint64_t* rec,
                                                        const uint32_t* mask,
                                                        const uint32_t* add_off, int64_t nvox,
                                                        uint32_t* counts) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nvox) return;
  const uint32_t lo = off[v], hi = off[v + 1];
  uint32_t n = 0;
  if (mask) {
    for (uint32_t k = lo; k < hi; ++k) n += removed(mask, rec[k]) ? 0u : 1u;
  } else {
    n = hi - lo;
  }
  if (add_off) n += add_off[v + 1] - add_off[v];
  counts[v] = n;
}

__global__ __launch_bounds__(kBlock) void k_merge_scatter(const uint32_t* off, const uint64_t* rec,
                                                          const uint32_t* mask,
                                                          const uint32_t* add_off,
                                                          const uint64_t* add_rec, int64_t nvox,
                                                          const uint32_t* new_off,
                                                          uint64_t* out) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nvox) return;
  uint32_t w = new_off[v];
  for (uint32_t k = off[v]; k < off[v + 1]; ++k) {
    const uint64_t r = rec[k];
    if (!removed(mask, r)) out[w++] = r;
  }
  if (add_off)
    for (uint32_t k = add_off[v]; k < add_off[v + 1]; ++k) out[w++] = add_rec[k];
}

// Pool blocks released after the stream has drained.
struct Temps {
  hipStream_t st;
  std::vector<void*> v;
  explicit Temps(hipStream_t s) : st(s) {}
  ~Temps() {
    if (!v.empty()) (void)hipStreamSynchronize(st);
    for (void* p : v) pool_free(p);
  }
  template <typename T>
  int get(T** out, size_t n) {
    void* p = nullptr;
    const int rc = pool_alloc(sizeof(T) * (n ? n : 1), &p, nullptr);
    if (rc) return rc;
    v.push_back(p);
    *out = static_cast<T*>(p);
    return LS_OK;
  }
  // a device copy of host or device input
  template <typename T>
  int input(const T* p, int64_t n, bool on_device, const T** out) {
    *out = nullptr;
    if (!p) return LS_OK;
    if (on_device) {
      *out = p;
      return LS_OK;
    }
    T* d = nullptr;
    int rc;
    if ((rc = get(&d, (size_t)n))) return rc;
    if (n > 0) LS_HIP(hipMemcpyAsync(d, p, sizeof(T) * (size_t)n, hipMemcpyHostToDevice, st));
    *out = d;
    return LS_OK;
  }
};

}  // namespace

extern "C" int lineset_update(ls_lineset_t s, const ls_update_desc* d, void* hip_stream) {
  if (!s || !d) {
    ls_set_error("lineset_update: null set or desc");
    return LS_EINVAL;
  }
  if (d->n_curves < 0 || d->n_vertices < 0 || d->n_remove < 0 ||
      (d->n_curves > 0 && !d->curve_off) || (d->n_remove > 0 && !d->remove_ids)) {
    ls_set_error("lineset_update: negative size or missing curve_off / remove_ids");
    return LS_EINVAL;
  }
  if (d->n_vertices > 0 && (d->xyz == nullptr) == (d->lattice == nullptr)) {
    ls_set_error("lineset_update: give exactly one of xyz and lattice for the added curves");
    return LS_EINVAL;
  }
  if (d->xyz && d->n_vertices > 0 && !(s->lo_scale[3] > 0.0)) {
    ls_set_error("lineset_update: xyz needs a set voxelized from xyz (its grid set-up)");
    return LS_EINVAL;
  }
  if (s->ends) {
    ls_set_error("lineset_update: sets voxelized with per-vertex attributes are not updated "
                 "in place (voxelize the edited curve list)");
    return LS_EUNSUPPORTED;
  }
  if (s->n_curves + d->n_curves > kMaxTagged) {
    ls_set_error("lineset_update: more than 2^24 curves (curve tags would repeat)");
    return LS_EUNSUPPORTED;
  }
  if (d->n_curves == 0 && d->n_remove == 0) return LS_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int cur = 0;
  LS_HIP(hipGetDevice(&cur));
  if (cur != s->device) {
    ls_set_error("lineset_update: the set lives on device %d, device %d is current", s->device,
                 cur);
    return LS_EINVAL;
  }
  if (!d->on_device && d->n_curves > 0) {
    if (d->curve_off[0] != 0 || d->curve_off[d->n_curves] > d->n_vertices) {
      ls_set_error("lineset_update: curve_off must start at 0 and end at most at n_vertices");
      return LS_EINVAL;
    }
    for (int64_t c = 0; c < d->n_curves; ++c)
      if (d->curve_off[c + 1] < d->curve_off[c]) {
        ls_set_error("lineset_update: curve_off must be non-decreasing");
        return LS_EINVAL;
      }
  }
  Temps T(st);
  int rc;
  const int64_t nvox = s->nvox;

  // 1. the added curves alone, with the set's grid set-up and following ids
  ls_lineset* add = nullptr;
  struct AddGuard {
    ls_lineset* p = nullptr;
    ~AddGuard() {
      if (p) {
        ls_free_all(p);
        delete p;
      }
    }
  } add_guard;
  if (d->n_curves > 0) {
    const float* xyz = nullptr;
    const int32_t* lat = nullptr;
    const int64_t* off = nullptr;
    const uint8_t* attr = nullptr;
    if ((rc = T.input(d->xyz, 3 * d->n_vertices, d->on_device, &xyz)) ||
        (rc = T.input(d->lattice, 3 * d->n_vertices, d->on_device, &lat)) ||
        (rc = T.input(d->curve_off, d->n_curves + 1, d->on_device, &off)) ||
        (rc = T.input(d->curve_attr, d->n_curves, d->on_device, &attr)))
      return rc;
    if (xyz && d->n_vertices > 0) {
      int32_t* snapped = nullptr;
      if ((rc = T.get(&snapped, 3 * (size_t)d->n_vertices))) return rc;
      SnapArgs sa;
      for (int a = 0; a < 3; ++a) sa.lo[a] = s->lo_scale[a];
      sa.scale = s->lo_scale[3];
      if ((rc = vox_snap(xyz, d->n_vertices, sa, snapped, st))) return rc;
      lat = snapped;
    }
    add = new (std::nothrow) ls_lineset();
    if (!add) {
      ls_set_error("host allocation failed");
      return LS_ENOMEM;
    }
    add_guard.p = add;
    for (int a = 0; a < 3; ++a) add->grid[a] = s->grid[a];
    add->bins = s->bins;
    add->nvox = nvox;
    add->n_curves = d->n_curves;
    add->n_vertices = d->n_vertices;
    add->curve_base = s->n_curves;
    add->device = s->device;
    // lattice input: vox_build checks the range (a vertex outside the grid
    // is an error, and the set stays as it was)
    if ((rc = vox_build(add, nullptr, lat, off, attr, nullptr, st))) return rc;
  }

  // 2. removal mask over the old curve ids
  uint32_t* mask = nullptr;
  if (d->n_remove > 0) {
    const int64_t* ids = nullptr;
    if ((rc = T.input(d->remove_ids, d->n_remove, d->on_device, &ids))) return rc;
    const int64_t words = (s->n_curves + 31) / 32;
    int* err = nullptr;
    if ((rc = T.get(&mask, (size_t)words)) || (rc = T.get(&err, 1))) return rc;
    if ((rc = fill_u32(mask, 0u, words, st)) || (rc = fill_u32((uint32_t*)err, 0u, 1, st)))
      return rc;
    hipLaunchKernelGGL(k_mark_removed, dim3(blocks_for(d->n_remove)), dim3(kBlock), 0, st, ids,
                       d->n_remove, s->n_curves, mask, err);
    LS_HIP(hipGetLastError());
    int herr = 0;
    LS_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    LS_HIP(hipStreamSynchronize(st));
    if (herr) {
      ls_set_error("lineset_update: a removed curve id is outside [0, %lld)",
                   (long long)s->n_curves);
      return LS_EINVAL;
    }
  }

  // 3. new offsets: counts, then an exclusive scan in place
  if ((uint64_t)s->n_records + (add ? (uint64_t)add->n_records : 0) >= 0xFFFFFFFFull) {
    ls_set_error("lineset_update: too many per-voxel lines");
    return LS_ENOMEM;
  }
  ls_lineset fresh{};
  for (int a = 0; a < 3; ++a) fresh.grid[a] = s->grid[a];
  fresh.bins = s->bins;
  fresh.nvox = nvox;
  fresh.device = s->device;
  struct FreshGuard {
    ls_lineset* p;
    bool keep = false;
    ~FreshGuard() {
      if (!keep) ls_free_all(p);
    }
  } fresh_guard{&fresh};
  uint32_t* sums = nullptr;
  if ((rc = ls_alloc(&fresh, (void**)&fresh.offsets, sizeof(uint32_t) * (nvox + 1))) ||
      (rc = T.get(&sums, (size_t)scan_block_sums_len(nvox))))
    return rc;
  const uint32_t* add_off = add ? add->offsets : nullptr;
  hipLaunchKernelGGL(k_merge_count, dim3(blocks_for(nvox)), dim3(kBlock), 0, st, s->offsets,
                     s->records, mask, add_off, nvox, fresh.offsets);
  LS_HIP(hipGetLastError());
  if ((rc = exclusive_scan_u32(fresh.offsets, fresh.offsets, nvox, sums, st))) return rc;
  uint32_t total = 0;
  LS_HIP(hipMemcpyAsync(&total, fresh.offsets + nvox, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  LS_HIP(hipStreamSynchronize(st));

  // 4. records
  if ((rc = ls_alloc(&fresh, (void**)&fresh.records, sizeof(uint64_t) * (total ? total : 1))))
    return rc;
  hipLaunchKernelGGL(k_merge_scatter, dim3(blocks_for(nvox)), dim3(kBlock), 0, st, s->offsets,
                     s->records, mask, add_off, add ? add->records : nullptr, nvox, fresh.offsets,
                     fresh.records);
  LS_HIP(hipGetLastError());

  // 5. occupancy and statistics of the new lists
  if ((rc = vox_occupancy(&fresh, st))) return rc;
  LS_HIP(hipStreamSynchronize(st));

  // the new arrays replace the old ones; the pyramid and grids are stale
  const int64_t add_slots = add ? add->n_slots - add->n_records : 0;
  ls_free_all(s);
  s->offsets = fresh.offsets;
  s->records = fresh.records;
  s->occupancy = fresh.occupancy;
  for (int a = 0; a < 3; ++a) s->macro[a] = fresh.macro[a];
  s->stats_pending = true;
  s->bytes = fresh.bytes;
  fresh_guard.keep = true;
  s->n_records = total;
  s->n_slots = (int64_t)total + add_slots;
  s->n_curves += d->n_curves;
  s->n_vertices += d->n_vertices;
  s->n_levels = 0;
  return LS_OK;
}
