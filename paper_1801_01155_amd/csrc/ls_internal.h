// Internal declarations shared by the HIP translation units of liblineset.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "lineset.h"

#define LS_MAX_LEVELS 32
#define LS_INVALID_VOXEL 0xFFFFFFFFu

// ---------------------------------------------------------------------------
// Error reporting (per-thread text behind ls_last_error).
void ls_set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

#define LS_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ls_set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                   __LINE__);                                                     \
      return LS_EDEVICE;                                                          \
    }                                                                             \
  } while (0)

// ---------------------------------------------------------------------------
// The line set object behind ls_lineset_t.
struct ls_lineset {
  int32_t grid[3];
  int32_t bins;
  int64_t nvox;
  int64_t n_curves, n_vertices;
  int64_t curve_base;  // id of the first curve voxelized by vox_build (curve tag offset)
  int64_t n_records, n_slots;
  int64_t nonempty, max_list;
  bool stats_pending;  // nonempty and max_list still on the device (after the occupancy words)
  uint32_t* offsets;   // [nvox + 1]
  uint64_t* records;   // [n_records] (at least one element allocated)
  uint16_t* ends;      // [n_records] endpoint attributes entry | exit << 8 (per-vertex input), or null
  uint64_t* occupancy; // per 4^3 macro cell: 64-bit mask of its non-empty voxels;
                       // then the non-empty voxel count (u64) and the longest list (u32)
  int32_t macro[3];    // macro-cell grid dims (ceil(grid / 4))
  // density pyramid
  int32_t n_levels;
  int32_t level_dims[LS_MAX_LEVELS][3];
  int64_t level_off[LS_MAX_LEVELS + 1];
  float* lod_count;
  float* lod_len;
  float* lod_rho;
  float* lod_rgb;         // colour pyramid [level_off][3] (opacity acceleration), or null
  float* ao;
  float* sh;
  uint32_t* rep;          // representative lines, levels flat at level_off (or null)
  int32_t rep_levels;
  void* cone_tab;         // plane and tap tables of the column cone tracer
  size_t cone_tab_bytes;
  double lo_scale[4];
  size_t bytes;
  int device;
};

// Device allocation tracked on the set (from the device memory cache).
int ls_alloc(ls_lineset* s, void** p, size_t bytes);
void ls_free_all(ls_lineset* s);

// Device memory cache (pool.hip): blocks of the current device, rounded up;
// `rounded` (optional) receives the block size. pool_free requires that no
// queued device work still uses the block.
int pool_alloc(size_t bytes, void** out, size_t* rounded);
void pool_free(void* p);

// ---------------------------------------------------------------------------
// Scans (scan.hip). out may alias in; writes n + 1 values (out[n] = total).
// `block_sums` needs scan_block_sums_len(n) elements of T.
int64_t scan_block_sums_len(int64_t n);
int exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* block_sums,
                       hipStream_t st);
int exclusive_scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* block_sums,
                       hipStream_t st);

// Fill kernels (no hipMemset, so callers may capture them in graphs).
int fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);

// ---------------------------------------------------------------------------
// Voxelization (vox.hip).
struct SnapArgs {
  double lo[3];
  double scale;
};

int vox_bbox(const float* xyz, int64_t nv, double lo[3], double hi[3], hipStream_t st);
double vox_scale(const double lo[3], const double hi[3], const int32_t grid[3]);
int vox_snap(const float* xyz, int64_t nv, SnapArgs sa, int32_t* lat, hipStream_t st);
// Builds the set's CSR. Float input (xyz): the grid set-up runs on the
// device and s->lo_scale is set; lattice input (lat): used as given.
int vox_build(ls_lineset* s, const float* xyz, const int32_t* lat, const int64_t* curve_off,
              const uint8_t* attr, const uint8_t* vattr, hipStream_t st);
// Occupancy words and list statistics of s->offsets (allocates s->occupancy).
int vox_occupancy(ls_lineset* s, hipStream_t st);

// ---------------------------------------------------------------------------
// Density pyramid and illumination (lod.hip, illum.hip).
void lod_plan(const int32_t grid[3], int32_t* n_levels, int32_t dims[][3], int64_t* level_off);
int lod_build(ls_lineset* s, const float* lut, int opaque, hipStream_t st);
// Colour pyramid beside rho (after lod_build): sum of length * sigma * rgb.
int lod_color_build(ls_lineset* s, const float* lut, int opaque, hipStream_t st);
int illum_ao(ls_lineset* s, int n_cones, float radius, float aperture, hipStream_t st);
// Both grids in one pass of the column cone tracer (the shadow cone rides
// along with the AO cones) when the schedules allow it; *applied = false
// (nothing launched) otherwise.
int illum_ao_shadow(ls_lineset* s, int n_cones, float radius, const float light[3],
                    float aperture, hipStream_t st, bool* applied);
int illum_shadow(ls_lineset* s, const float light[3], float aperture, hipStream_t st);
// Representative lines of every level (replines.hip); allocates s->rep.
int rep_build(ls_lineset* s, hipStream_t st);

// ---------------------------------------------------------------------------
// Rendering (render.hip).
struct RenderCounters {
  unsigned long long visited, nonempty, tested, hits, fragments, list_bytes, sort_passes,
      merge_evictions, macro_skips, merge_live_evictions, merge_overflow_rays;
};

inline void export_counters(const RenderCounters& h, ls_render_counters* c) {
  c->visited = (int64_t)h.visited;
  c->nonempty = (int64_t)h.nonempty;
  c->tested = (int64_t)h.tested;
  c->hits = (int64_t)h.hits;
  c->fragments = (int64_t)h.fragments;
  c->list_bytes = (int64_t)h.list_bytes;
  c->sort_passes = (int64_t)h.sort_passes;
  c->merge_evictions = (int64_t)h.merge_evictions;
  c->macro_skips = (int64_t)h.macro_skips;
  c->merge_live_evictions = (int64_t)h.merge_live_evictions;
  c->merge_overflow_rays = (int64_t)h.merge_overflow_rays;
}

// Validates one view's camera / parameters / output (sets the error text).
int check_render(const ls_lineset* s, const ls_camera* c, const ls_render_params* p,
                 const float* out);

int render_frame(const ls_lineset* s, const ls_camera* cam, const ls_render_params* p,
                 float* out, RenderCounters* dev_counters, hipStream_t st);
