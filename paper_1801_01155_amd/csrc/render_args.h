// Per-view render descriptor shared by the plain, batched and served paths.
#pragma once

#include "ls_internal.h"

// Everything one view needs, passed by value to the plain kernel and read
// from device memory (uniform, scalar loads) by the persistent kernel.
struct RenderArgs {
  const uint32_t* offsets;
  const uint64_t* records;
  const unsigned long long* occ;  // per 4^3 macro cell: mask of non-empty voxels
  int32_t g[3];
  int32_t mg[3];                  // macro grid dims
  float inv_bins;
  const float* lut;
  const float* ao;
  const float* sh;
  float eye[3], fwd[3], right[3], up[3];
  int32_t ortho, W, H;
  float radius, r2, alpha_stop;
  int32_t mode, opaque, merge, shading;
  int32_t dist_alpha;             // opacity from the chord length inside the tube
  float inv_2r;                   // 1 / (2 radius)
  float ka, kd, ks, shin;
  float light[3];
  // shading 2 sources: ao_mode 0 grid / 1 hemisphere rays per fragment;
  // shadow_mode 0 grid / 1 cone per fragment / 2 representative-line ray
  int32_t ao_mode, shadow_mode, ao_rays, rep_level, n_levels;
  float ao_radius;
  const float* rho;               // density pyramid, levels flat
  const uint32_t* rep;            // representative lines, levels flat
  const uint16_t* ends;           // per-record endpoint attributes (or null)
  // opacity acceleration: switch at A >= accel_A0 (2: off), depth scale
  float accel_A0, accel_depth;
  const float* rgb;               // colour pyramid, levels flat, 3 floats per cell
  float* out;
  RenderCounters* counters;
  int32_t wx, wy;                 // tile = wx x wy waves of 8 x 8 pixels
  int32_t tiles_x, n_tiles, tiles_per_xcd;
  // plain launch order: tiles in square rings around the tile (spiral_x,
  // spiral_y) out to ring spiral_r, or rows interleaved over the XCDs when
  // spiral_r < 0
  int32_t spiral_x, spiral_y, spiral_r;
  // the tiles of the first split_n spiral positions (the innermost rings)
  // are rendered by split_s workgroups each, on 8 / split_s pixel rows, so
  // the waves over the densest part of the image hold fewer rays
  int32_t split_n, split_s;
  // ordered frames: the first top_n launch positions (the longest measured
  // tiles) are split top_s ways (4 or 8), before the split_n ones above
  int32_t top_n, top_s;
  // plain launch order by measured cost (tile_order): workgroup position p
  // renders tile order[p]; null: the ring order above. times (or null):
  // each workgroup adds its duration (10 ns ticks) to its tile's entry
  const int32_t* order;
  uint32_t* times;
};

// Tile queues of the persistent kernel: one contiguous range per XCD.
struct BatchQueues {
  int32_t begin[8];
  int32_t len[8];
};

struct BatchPlan {
  int32_t wx, wy;     // tile shape in waves
  int32_t blocks;     // persistent workgroups
};

int make_render_args(const ls_lineset* s, const ls_camera* cam, const ls_render_params* p,
                     float* out, int wx, int wy, RenderCounters* dev_counters, RenderArgs* R);
int launch_render(const RenderArgs& R, hipStream_t st);
// True when the view needs the kernels' extended instance: it samples the
// pyramid or the representative lines per fragment (view-dependent
// illumination), or its set carries per-line endpoint attributes.
inline bool view_dependent(const RenderArgs& R) {
  return (R.shading == 2 && (R.ao_mode != 0 || R.shadow_mode != 0)) || R.ends != nullptr ||
         R.accel_A0 <= 1.f;
}
BatchQueues make_queues(int total_tiles);
// dev_queue: 8 queue counters (zeroed before the launch), followed by a
// RenderCounters block when `count` is set.
// vdi: some view uses view-dependent illumination (view_dependent).
int launch_render_batch(const RenderArgs* dev_views, const int32_t* dev_tile_start, int n_views,
                        const BatchQueues& q, unsigned* dev_queue, const BatchPlan& plan,
                        bool count, bool vdi, hipStream_t st);
int batch_blocks_per_cu(int wx, int wy, bool vdi, int* out);
int render_merge_slots();   // intervals in the per-ray curve-merge table
