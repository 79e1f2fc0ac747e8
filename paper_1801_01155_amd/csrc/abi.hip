// C-ABI of liblineset: argument validation, object lifetime, error text.
// Every exported function returns an ls_status and leaves nothing half-built.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>
#include <mutex>
#include <vector>

#include "render_args.h"

namespace {
thread_local char g_err[512] = "no error";

struct Stream {
  hipStream_t s;
  explicit Stream(void* p) : s(static_cast<hipStream_t>(p)) {}
};

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_grid(const int32_t g[3], int lo) {
  for (int a = 0; a < 3; ++a)
    if (g[a] < lo || g[a] > 1024) {
      ls_set_error("grid sides must be in [%d, 1024]", lo);
      return LS_EINVAL;
    }
  if ((int64_t)g[0] * g[1] * g[2] > (1ll << 30)) {
    ls_set_error("grid has more than 2^30 voxels");
    return LS_EINVAL;
  }
  return LS_OK;
}

bool finite3(const float v[3]) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

// Copies `n` elements of host or device memory into a fresh device buffer
// (returns the original pointer when it already is device memory).
template <typename T>
int to_device(const T* p, int64_t n, bool on_device, T** out, std::vector<void*>& owned,
              hipStream_t st) {
  *out = nullptr;
  if (!p) return LS_OK;
  if (on_device) {
    *out = const_cast<T*>(p);
    return LS_OK;
  }
  void* d = nullptr;
  size_t bytes = sizeof(T) * (size_t)(n > 0 ? n : 1);
  int rc = pool_alloc(bytes, &d, nullptr);
  if (rc) return rc;
  owned.push_back(d);
  if (n > 0) LS_HIP(hipMemcpyAsync(d, p, sizeof(T) * (size_t)n, hipMemcpyHostToDevice, st));
  *out = static_cast<T*>(d);
  return LS_OK;
}

struct Owned {
  std::vector<void*> v;
  hipStream_t st = nullptr;
  ~Owned() {
    if (!v.empty()) (void)hipStreamSynchronize(st);
    for (void* p : v) pool_free(p);
  }
};

}  // namespace

namespace {

// One side stream (default priority, non-blocking) and a fork/join event pair
// per device, created on first use and kept for the process; the mutex keeps
// one caller's fork, side work and join together.
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::mutex mu;
};

std::mutex g_side_mu;
SideStream g_side[64];

SideStream* side_stream(int device) {
  if (device < 0 || device >= 64) {
    ls_set_error("device index %d out of range", device);
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_side_mu);
  SideStream& S = g_side[device];
  if (!S.stream) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != device) (void)hipSetDevice(device);
    const bool ok = hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking) == hipSuccess &&
                    hipEventCreateWithFlags(&S.fork, hipEventDisableTiming) == hipSuccess &&
                    hipEventCreateWithFlags(&S.join, hipEventDisableTiming) == hipSuccess;
    if (cur != device) (void)hipSetDevice(cur);
    if (!ok) {
      (void)hipGetLastError();
      ls_set_error("side stream creation failed");
      S.stream = nullptr;
      return nullptr;
    }
  }
  return &S;
}

}  // namespace

void ls_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int ls_alloc(ls_lineset* s, void** p, size_t bytes) {
  size_t got = 0;
  const int rc = pool_alloc(bytes, p, &got);
  if (rc) return rc;
  s->bytes += got;
  return LS_OK;
}

void ls_free_all(ls_lineset* s) {
  void* ptrs[] = {s->offsets, s->records, s->occupancy, s->lod_count, s->lod_len,
                  s->lod_rho, s->ao,      s->sh,        s->cone_tab, s->rep, s->ends,
                  s->lod_rgb};
  bool any = false;
  for (void* p : ptrs) any = any || p;
  // work queued on any stream may still read the set (hipFree would wait too)
  if (any) (void)hipDeviceSynchronize();
  for (void* p : ptrs) pool_free(p);
  s->offsets = nullptr;
  s->records = nullptr;
  s->occupancy = nullptr;
  s->stats_pending = false;
  s->lod_count = s->lod_len = s->lod_rho = s->ao = s->sh = s->lod_rgb = nullptr;
  s->cone_tab = nullptr;
  s->cone_tab_bytes = 0;
  s->rep = nullptr;
  s->rep_levels = 0;
  s->ends = nullptr;
  s->bytes = 0;
}

int check_render(const ls_lineset* s, const ls_camera* c, const ls_render_params* p,
                 const float* out) {
  if (!s || !c || !p || !out || !p->lut_rgba) {
    ls_set_error("lineset_render: null set, camera, params, lut or output");
    return LS_EINVAL;
  }
  if (c->width <= 0 || c->height <= 0 || (int64_t)c->width * c->height > (1ll << 31)) {
    ls_set_error("lineset_render: image size must be positive and below 2^31 pixels");
    return LS_EINVAL;
  }
  if (!finite3(c->eye) || !finite3(c->forward) || !finite3(c->right) || !finite3(c->up)) {
    ls_set_error("lineset_render: non-finite camera");
    return LS_EINVAL;
  }
  if (c->forward[0] == 0.f && c->forward[1] == 0.f && c->forward[2] == 0.f) {
    ls_set_error("lineset_render: forward is zero");
    return LS_EINVAL;
  }
  if (!(p->radius > 0.f) || !std::isfinite(p->radius) || (p->mode == 1 && !(p->radius < 1.f))) {
    ls_set_error("lineset_render: radius must be > 0 (and < 1 voxel in mode 1)");
    return LS_EINVAL;
  }
  if (p->mode != 0 && p->mode != 1) {
    ls_set_error("lineset_render: mode must be 0 or 1");
    return LS_EINVAL;
  }
  if (p->shading < 0 || p->shading > 2) {
    ls_set_error("lineset_render: shading must be 0, 1 or 2");
    return LS_EINVAL;
  }
  if (p->shading == 2) {
    if (p->ao_mode < 0 || p->ao_mode > 1 || p->shadow_mode < 0 || p->shadow_mode > 2) {
      ls_set_error("lineset_render: ao_mode must be 0 or 1, shadow_mode 0, 1 or 2");
      return LS_EINVAL;
    }
    if ((p->ao_mode == 0 && !s->ao) || (p->shadow_mode == 0 && !s->sh)) {
      ls_set_error("lineset_render: shading 2 from the per-voxel grids needs them built "
                   "(lineset_build_lod with build_ao / build_shadow)");
      return LS_EINVAL;
    }
    if ((p->ao_mode == 1 || p->shadow_mode == 1) && !s->lod_rho) {
      ls_set_error("lineset_render: per-fragment AO or shadow cones need the density pyramid");
      return LS_EINVAL;
    }
    if (p->ao_mode == 1 && (p->ao_rays < 1 || p->ao_rays > 256 || !(p->ao_radius > 0.f) ||
                            !std::isfinite(p->ao_radius))) {
      ls_set_error("lineset_render: ao_rays must be in [1, 256] and ao_radius finite and > 0");
      return LS_EINVAL;
    }
    if (p->shadow_mode == 2 && (!s->rep || p->rep_level < 0 || p->rep_level >= s->rep_levels)) {
      ls_set_error("lineset_render: shadow_mode 2 needs the representative lines "
                   "(build_rep_lines) and rep_level in [0, levels)");
      return LS_EINVAL;
    }
    if (p->shadow_mode != 0 && !finite3(p->light_dir)) {
      ls_set_error("lineset_render: non-finite light_dir");
      return LS_EINVAL;
    }
  }
  if (!(p->accel_depth >= 0.f) || !std::isfinite(p->accel_depth)) {
    ls_set_error("lineset_render: accel_depth must be finite and >= 0");
    return LS_EINVAL;
  }
  if (p->accel_depth > 0.f && !p->opaque && (!s->lod_rho || !s->lod_rgb)) {
    ls_set_error("lineset_render: opacity acceleration needs the density and colour pyramids "
                 "(lineset_build_lod with build_color)");
    return LS_EINVAL;
  }
  if (!aligned16(out) || !aligned16(p->lut_rgba)) {
    ls_set_error("lineset_render: rgba_out and lut_rgba must be 16-byte aligned");
    return LS_EINVAL;
  }
  return LS_OK;
}

extern "C" {

const char* ls_last_error(void) { return g_err; }

int ls_version(void) { return 100; }

int lineset_grid_setup(const float* xyz, int64_t n_vertices, const int32_t grid[3],
                       int32_t* lattice, double* lo_scale, void* hip_stream) {
  if (!grid || (n_vertices > 0 && (!xyz || !lattice)) || n_vertices < 0) {
    ls_set_error("lineset_grid_setup: null pointer or negative size");
    return LS_EINVAL;
  }
  int rc;
  if ((rc = check_grid(grid, 3))) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double lo[3], hi[3];
  if ((rc = vox_bbox(xyz, n_vertices, lo, hi, st))) return rc;
  SnapArgs sa;
  for (int a = 0; a < 3; ++a) sa.lo[a] = lo[a];
  sa.scale = vox_scale(lo, hi, grid);
  if ((rc = vox_snap(xyz, n_vertices, sa, lattice, st))) return rc;
  LS_HIP(hipStreamSynchronize(st));
  if (lo_scale) {
    for (int a = 0; a < 3; ++a) lo_scale[a] = lo[a];
    lo_scale[3] = sa.scale;
  }
  return LS_OK;
}

int lineset_voxelize(const ls_voxelize_desc* d, void* hip_stream, ls_lineset_t* out) {
  if (!out) {
    ls_set_error("lineset_voxelize: out is NULL");
    return LS_EINVAL;
  }
  *out = nullptr;
  if (!d) {
    ls_set_error("lineset_voxelize: desc is NULL");
    return LS_EINVAL;
  }
  if ((d->xyz == nullptr) == (d->lattice == nullptr) && d->n_vertices > 0) {
    ls_set_error("lineset_voxelize: give exactly one of xyz and lattice");
    return LS_EINVAL;
  }
  if (d->n_vertices < 0 || d->n_curves < 0 || (d->n_curves > 0 && !d->curve_off)) {
    ls_set_error("lineset_voxelize: negative size or missing curve_off");
    return LS_EINVAL;
  }
  if (d->bins < 1 || d->bins > 64 || (d->bins & (d->bins - 1))) {
    ls_set_error("lineset_voxelize: bins must be a power of two in [1, 64]");
    return LS_EINVAL;
  }
  int rc;
  if ((rc = check_grid(d->grid, d->xyz ? 3 : 1))) return rc;
  if (d->n_vertices >= (1ll << 40)) {
    ls_set_error("lineset_voxelize: too many vertices");
    return LS_ENOMEM;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  LS_HIP(hipGetDevice(&dev));

  // host inputs: validate curve_off on the host, then upload
  if (!d->on_device && d->n_curves > 0) {
    if (d->curve_off[0] != 0) {
      ls_set_error("curve_off must start at 0");
      return LS_EINVAL;
    }
    for (int64_t c = 0; c < d->n_curves; ++c)
      if (d->curve_off[c + 1] < d->curve_off[c]) {
        ls_set_error("curve_off must be non-decreasing");
        return LS_EINVAL;
      }
    if (d->curve_off[d->n_curves] > d->n_vertices) {
      ls_set_error("curve_off ends beyond n_vertices");
      return LS_EINVAL;
    }
  }
  Owned own;
  own.st = st;
  const float* xyz = nullptr;
  const int32_t* lat = nullptr;
  const int64_t* off = nullptr;
  const uint8_t* attr = nullptr;
  const uint8_t* vattr = nullptr;
  {
    float* x = nullptr;
    int32_t* l = nullptr;
    int64_t* o = nullptr;
    uint8_t* a = nullptr;
    uint8_t* va = nullptr;
    if ((rc = to_device(d->xyz, 3 * d->n_vertices, d->on_device, &x, own.v, st)) ||
        (rc = to_device(d->lattice, 3 * d->n_vertices, d->on_device, &l, own.v, st)) ||
        (rc = to_device(d->curve_off, d->n_curves + 1, d->on_device, &o, own.v, st)) ||
        (rc = to_device(d->curve_attr, d->n_curves, d->on_device, &a, own.v, st)) ||
        (rc = to_device(d->vertex_attr, d->n_vertices, d->on_device, &va, own.v, st)))
      return rc;
    xyz = x;
    lat = l;
    off = o;
    attr = a;
    vattr = va;
  }

  ls_lineset* s = new (std::nothrow) ls_lineset();
  if (!s) {
    ls_set_error("host allocation failed");
    return LS_ENOMEM;
  }
  for (int a = 0; a < 3; ++a) s->grid[a] = d->grid[a];
  s->bins = d->bins;
  s->nvox = (int64_t)d->grid[0] * d->grid[1] * d->grid[2];
  s->n_curves = d->n_curves;
  s->n_vertices = d->n_vertices;
  s->device = dev;
  if ((rc = vox_build(s, xyz, lat, off, attr, vattr, st))) {
    (void)hipStreamSynchronize(st);
    ls_free_all(s);
    delete s;
    return rc;
  }
  *out = s;
  return LS_OK;
}

void lineset_destroy(ls_lineset_t s) {
  if (!s) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != s->device) (void)hipSetDevice(s->device);
  ls_free_all(s);
  if (cur != s->device) (void)hipSetDevice(cur);
  delete s;
}

int lineset_build_lod(ls_lineset_t s, const ls_lod_desc* d, void* hip_stream) {
  if (!s || !d || !d->lut_rgba) {
    ls_set_error("lineset_build_lod: null set, desc or lut");
    return LS_EINVAL;
  }
  if (d->build_ao && (d->ao_cones < 1 || !(d->ao_radius > 0.f) || !std::isfinite(d->ao_radius))) {
    ls_set_error("lineset_build_lod: ao_cones >= 1 and a finite ao_radius > 0 required");
    return LS_EINVAL;
  }
  if ((d->build_ao || d->build_shadow) &&
      (!(d->cone_aperture >= 0.f) || !std::isfinite(d->cone_aperture))) {
    ls_set_error("lineset_build_lod: cone_aperture must be finite and >= 0");
    return LS_EINVAL;
  }
  if (d->build_shadow) {
    float n = d->light_dir[0] * d->light_dir[0] + d->light_dir[1] * d->light_dir[1] +
              d->light_dir[2] * d->light_dir[2];
    if (!finite3(d->light_dir) || !(n > 0.f)) {
      ls_set_error("lineset_build_lod: light_dir must be a finite non-zero vector");
      return LS_EINVAL;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int rc;
  if ((rc = lod_build(s, d->lut_rgba, d->opaque, st))) return rc;
  if (d->build_rep_lines && (rc = rep_build(s, st))) return rc;
  if (d->build_color && (rc = lod_color_build(s, d->lut_rgba, d->opaque, st))) return rc;
  if (d->build_ao && d->build_shadow) {
    bool applied = false;
    if ((rc = illum_ao_shadow(s, d->ao_cones, d->ao_radius, d->light_dir, d->cone_aperture, st,
                              &applied)))
      return rc;
    if (applied) return LS_OK;
    // Otherwise the shadow cone (latency-bound gathers) runs on a second
    // stream beside the AO cones, both after the pyramid, joined before return.
    SideStream* side = side_stream(s->device);
    if (!side) return LS_EDEVICE;
    std::lock_guard<std::mutex> lk(side->mu);
    LS_HIP(hipEventRecord(side->fork, st));
    LS_HIP(hipStreamWaitEvent(side->stream, side->fork, 0));
    rc = illum_shadow(s, d->light_dir, d->cone_aperture, side->stream);
    LS_HIP(hipEventRecord(side->join, side->stream));
    if (!rc) rc = illum_ao(s, d->ao_cones, d->ao_radius, d->cone_aperture, st);
    LS_HIP(hipStreamWaitEvent(st, side->join, 0));
    return rc;
  }
  if (d->build_ao && (rc = illum_ao(s, d->ao_cones, d->ao_radius, d->cone_aperture, st))) return rc;
  if (d->build_shadow && (rc = illum_shadow(s, d->light_dir, d->cone_aperture, st))) return rc;
  return LS_OK;
}


int lineset_render(ls_lineset_t s, const ls_camera* cam, const ls_render_params* p,
                   float* rgba_out, void* hip_stream) {
  int rc;
  if ((rc = check_render(s, cam, p, rgba_out))) return rc;
  return render_frame(s, cam, p, rgba_out, nullptr, static_cast<hipStream_t>(hip_stream));
}

int lineset_render_counted(ls_lineset_t s, const ls_camera* cam, const ls_render_params* p,
                           float* rgba_out, ls_render_counters* counters, void* hip_stream) {
  int rc;
  if ((rc = check_render(s, cam, p, rgba_out))) return rc;
  if (!counters) {
    ls_set_error("lineset_render_counted: counters is NULL");
    return LS_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  RenderCounters* dc = nullptr;
  if ((rc = pool_alloc(sizeof(RenderCounters), (void**)&dc, nullptr))) return rc;
  RenderCounters h{};
  rc = LS_OK;
  if (hipMemcpyAsync(dc, &h, sizeof(h), hipMemcpyHostToDevice, st) != hipSuccess) rc = LS_EDEVICE;
  if (!rc) rc = render_frame(s, cam, p, rgba_out, dc, st);
  if (!rc && (hipMemcpyAsync(&h, dc, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
              hipStreamSynchronize(st) != hipSuccess)) {
    ls_set_error("lineset_render_counted: copy of counters failed");
    rc = LS_EDEVICE;
  }
  (void)hipStreamSynchronize(st);
  pool_free(dc);
  if (rc) return rc;
  export_counters(h, counters);
  return LS_OK;
}

int lineset_render_limits(int32_t* merge_slots) {
  if (!merge_slots) {
    ls_set_error("lineset_render_limits: null argument");
    return LS_EINVAL;
  }
  *merge_slots = render_merge_slots();
  return LS_OK;
}

int lineset_info(ls_lineset_t s, ls_info* o) {
  if (!s || !o) {
    ls_set_error("lineset_info: null argument");
    return LS_EINVAL;
  }
  if (s->stats_pending) {
    // the voxelizer synchronised its stream: the statistics are final
    const int64_t nm = (int64_t)s->macro[0] * s->macro[1] * s->macro[2];
    unsigned long long h[2] = {0, 0};
    LS_HIP(hipMemcpy(h, s->occupancy + nm, sizeof(h), hipMemcpyDeviceToHost));
    s->nonempty = (int64_t)h[0];
    s->max_list = (int64_t)(uint32_t)h[1];
    s->stats_pending = false;
  }
  std::memset(o, 0, sizeof(*o));
  for (int a = 0; a < 3; ++a) o->grid[a] = s->grid[a];
  o->bins = s->bins;
  o->n_curves = s->n_curves;
  o->n_vertices = s->n_vertices;
  o->n_records = s->n_records;
  o->n_record_slots = s->n_slots;
  o->nonempty_voxels = s->nonempty;
  o->max_list = s->max_list;
  o->n_levels = s->lod_rho ? s->n_levels : 0;
  o->has_ao = s->ao != nullptr;
  o->has_shadow = s->sh != nullptr;
  o->has_rep_lines = s->rep != nullptr;
  o->has_vertex_attr = s->ends != nullptr;
  o->has_color = s->lod_rgb != nullptr;
  for (int l = 0; l < s->n_levels && l < 32; ++l)
    for (int a = 0; a < 3; ++a) o->level_dims[l][a] = s->level_dims[l][a];
  for (int l = 0; l <= s->n_levels && l < 33; ++l) o->level_off[l] = s->level_off[l];
  for (int k = 0; k < 4; ++k) o->lo_scale[k] = s->lo_scale[k];
  o->device_bytes = s->bytes;
  return LS_OK;
}

int lineset_export(ls_lineset_t s, int32_t what, void* dst, size_t dst_bytes,
                   int32_t dst_on_device, void* hip_stream) {
  if (!s || !dst) {
    ls_set_error("lineset_export: null argument");
    return LS_EINVAL;
  }
  const void* src = nullptr;
  size_t bytes = 0;
  const size_t lod_bytes = s->lod_rho ? sizeof(float) * (size_t)s->level_off[s->n_levels] : 0;
  switch (what) {
    case LS_EXPORT_OFFSETS: src = s->offsets; bytes = sizeof(uint32_t) * (size_t)(s->nvox + 1); break;
    case LS_EXPORT_RECORDS: src = s->records; bytes = sizeof(uint64_t) * (size_t)s->n_records; break;
    case LS_EXPORT_LOD_COUNT: src = s->lod_count; bytes = lod_bytes; break;
    case LS_EXPORT_LOD_LEN: src = s->lod_len; bytes = lod_bytes; break;
    case LS_EXPORT_LOD_RHO: src = s->lod_rho; bytes = lod_bytes; break;
    case LS_EXPORT_AO: src = s->ao; bytes = s->ao ? sizeof(float) * (size_t)s->nvox : 0; break;
    case LS_EXPORT_SHADOW: src = s->sh; bytes = s->sh ? sizeof(float) * (size_t)s->nvox : 0; break;
    case LS_EXPORT_LOD_COLOR: src = s->lod_rgb; bytes = s->lod_rgb ? 3 * lod_bytes : 0; break;
    case LS_EXPORT_ENDS:
      src = s->ends;
      bytes = s->ends ? sizeof(uint16_t) * (size_t)s->n_records : 0;
      break;
    case LS_EXPORT_REP_LINES:
      src = s->rep;
      bytes = s->rep ? sizeof(uint32_t) * (size_t)s->level_off[s->rep_levels] : 0;
      break;
    default:
      ls_set_error("lineset_export: unknown buffer %d", what);
      return LS_EINVAL;
  }
  if (!src) {
    ls_set_error("lineset_export: buffer %d has not been built", what);
    return LS_EINVAL;
  }
  if (dst_bytes < bytes) {
    ls_set_error("lineset_export: destination holds %zu bytes, %zu needed", dst_bytes, bytes);
    return LS_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (bytes) {
    LS_HIP(hipMemcpyAsync(dst, src, bytes, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          st));
  }
  LS_HIP(hipStreamSynchronize(st));
  return LS_OK;
}

}  // extern "C"
