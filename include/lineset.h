/*
 * lineset — voxel-based ray-casting of large 3D line sets on AMD Instinct
 * MI355X (gfx950).
 *
 * Method: Kanzler, Rautenhaus, Westermann, "A Voxel-based Rendering Pipeline
 * for Large 3D Line Sets". Curves are clipped per voxel, the per-voxel line
 * endpoints are quantized to N x N bins of the voxel faces and stored in
 * per-voxel lists; every pixel's ray walks the grid (3D-DDA), intersects the
 * tubes of the lines in the voxels it visits, sorts those hits per voxel and
 * composites them front to back with early termination. A density pyramid
 * drives cone-traced ambient occlusion and soft shadows.
 *
 * Conventions for every entry point:
 *  - Returns an ls_status; on failure nothing is allocated or left half-built
 *    and ls_last_error() (per thread) describes the cause.
 *  - `hip_stream` is a hipStream_t (NULL = the default stream). Work is
 *    enqueued on it; calls that must know device-side sizes synchronise it.
 *  - Pointers documented as "device" are HIP device (or managed) memory owned
 *    by the caller, and must stay valid until the stream has passed the call.
 *  - No exception crosses this boundary.
 */
#ifndef LINESET_H
#define LINESET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LS_OK = 0,
  LS_EINVAL = -1,        /* invalid argument or input data */
  LS_ENOMEM = -2,        /* device or host allocation failed, or a size limit */
  LS_EDEVICE = -3,       /* a HIP runtime call failed */
  LS_EUNSUPPORTED = -4,  /* valid request this library does not implement */
  LS_EBUSY = -5,         /* server cannot queue the request now */
  LS_ETIMEOUT = -6       /* wait ended before completion */
} ls_status;

/* Text of the last non-OK status returned on this thread. Never NULL. */
const char* ls_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int ls_version(void);

/* An opaque voxelized line set. Owns every device buffer it allocates
 * (CSR offsets and records, density pyramid, illumination grids) until
 * lineset_destroy. */
typedef struct ls_lineset* ls_lineset_t;

/* ------------------------------------------------------------------------ */
/* Grid set-up (section "Curve voxelization", first paragraph): cube voxels of
 * side 1; the curves' bounding box is mapped into the grid keeping its aspect
 * ratio, with one voxel of margin on each side, and every vertex is rounded to
 * a lattice of 1/256 voxel:
 *     q = floor((v - lo) * S + 0.5) + 256,
 *     S = min over axes with extent > 0 of 256 (grid_a - 2) / extent_a,
 * evaluated in fp64 (S = 0 when all extents are 0).
 *   xyz       device, float [n_vertices][3]
 *   lattice   device, int32 [n_vertices][3] (output)
 *   lo_scale  host, double [4] (output, may be NULL): lo[3], S
 * Errors: LS_EINVAL for a grid side outside [3, 1024] or a non-finite
 * coordinate. Synchronises the stream. */
int lineset_grid_setup(const float* xyz, int64_t n_vertices, const int32_t grid[3],
                       int32_t* lattice, double* lo_scale, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Voxelization (sections "Curve voxelization", "Line quantization", "GPU
 * implementation").
 *
 * Input curves are vertex sequences: curve c owns vertices
 * [curve_off[c], curve_off[c+1]). Give either world coordinates (`xyz`,
 * mapped by the grid set-up above) or lattice coordinates (`lattice`, int32
 * in 1/256 voxel, each in [0, 256 * grid_a)).
 *
 * Each curve segment is clipped against the voxel faces in order of
 * occurrence (half-open voxels; simultaneous crossings of several planes are
 * one event whose face is that of the lowest axis). Consecutive events of a
 * curve bound one per-voxel line; the pieces before the first and after the
 * last event are dropped, as are lines whose two exact event points or two
 * quantized endpoints coincide. Endpoints are quantized to the centres of
 * N x N bins per face: bin = min(floor(local * N), N - 1).
 *
 * Output layout (CSR), exported by lineset_export:
 *   offsets  uint32 [gx*gy*gz + 1], voxel id = x + gx * (y + gy * z)
 *   records  uint64 [n_records], a voxel's lines consecutive, in order of
 *            (curve id, position along the curve):
 *     bits  0..2  entry face   3..8  entry bin u   9..14 entry bin w
 *     bits 15..17 exit face   18..23 exit bin u   24..29 exit bin w
 *     bits 32..39 attribute byte   40..63 curve id mod 2^24
 *   Faces 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z; (u, w) are the face's other
 *   two axes in increasing order.
 *
 * Per-vertex attributes (section "Curve voxelization": line attributes
 * interpolated to the line-face intersection points): with vertex_attr each
 * event on segment v_i -> v_{i+1} at exact parameter t gets
 * a_i + (a_{i+1} - a_i) t rounded to the nearest integer (halves up); every
 * line keeps its entry and exit attributes (LS_EXPORT_ENDS, uint16
 * entry | exit << 8 per record, CSR order) and its record's attribute byte is
 * their mean rounded down (curve_attr is then ignored). Rendering reads the
 * transfer function linearly at the attribute interpolated along the line at
 * the segment point closest to the fragment's entry. Such sets are not
 * updated in place (lineset_update returns LS_EUNSUPPORTED).
 * Errors: LS_EINVAL for grid sides outside [1, 1024] (3 with xyz input),
 * more than 2^30 voxels, bins not a power of two in [1, 64], non-monotone
 * curve_off, a lattice coordinate out of range; LS_ENOMEM if the lines
 * exceed 2^32 - 1 records or memory runs out. `*out` is NULL on failure.
 * Synchronises the stream (it reads device-side totals to size buffers). */
typedef struct {
  const float* xyz;          /* [n_vertices][3] world coordinates, or NULL */
  const int32_t* lattice;    /* [n_vertices][3] lattice coordinates, or NULL */
  const int64_t* curve_off;  /* [n_curves + 1] */
  const uint8_t* curve_attr; /* [n_curves], or NULL for 255 */
  int64_t n_vertices;
  int64_t n_curves;
  int32_t on_device;         /* 1: the pointers are device memory; 0: host */
  int32_t grid[3];
  int32_t bins;              /* N */
  const uint8_t* vertex_attr; /* [n_vertices] per-vertex attribute, or NULL (see below) */
} ls_voxelize_desc;

int lineset_voxelize(const ls_voxelize_desc* desc, void* hip_stream, ls_lineset_t* out);

/* Incremental update (section "Voxel-based curve discretization", first
 * paragraph: on the GPU the pre-process permits instant updates when curves
 * are removed or added; section "Conclusion and future work": local updates
 * and time-varying line sets). Removes the curves listed in remove_ids (ids
 * of the set, duplicates allowed) and appends the given curves, without
 * re-voxelizing the curves that stay. The set then holds exactly what
 * lineset_voxelize returns for the edited curve list in lattice form: old
 * curves keep their ids and removed ones contribute nothing, added curves
 * take ids n_curves, n_curves + 1, ... (lineset_info's n_curves grows by
 * the added count). Added vertices are given like lineset_voxelize's: `xyz`
 * is mapped with the set's own grid set-up (the set must come from xyz
 * input), `lattice` is used as given; either must lie in [0, 256 * grid).
 * The density pyramid and illumination grids are released (they describe
 * the old lines): call lineset_build_lod again.
 * Errors: LS_EINVAL for a removed id outside [0, n_curves), a vertex outside
 * the grid, malformed curve_off; LS_EUNSUPPORTED when the set would hold more
 * than 2^24 curves (the records' curve tags would repeat); LS_ENOMEM. On an
 * error the set is unchanged. Synchronises the stream. */
typedef struct {
  const float* xyz;          /* added curves: [n_vertices][3] world coordinates, or NULL */
  const int32_t* lattice;    /* [n_vertices][3] lattice coordinates, or NULL */
  const int64_t* curve_off;  /* [n_curves + 1] */
  const uint8_t* curve_attr; /* [n_curves], or NULL for 255 */
  int64_t n_vertices;
  int64_t n_curves;
  const int64_t* remove_ids; /* [n_remove] curve ids to remove */
  int64_t n_remove;
  int32_t on_device;         /* 1: the pointers are device memory; 0: host */
} ls_update_desc;

int lineset_update(ls_lineset_t set, const ls_update_desc* desc, void* hip_stream);

void lineset_destroy(ls_lineset_t set);

/* ------------------------------------------------------------------------ */
/* Density pyramid (section "LoD construction"): per voxel
 *   count = number of lines, len = sum of line lengths (voxel units),
 *   rho = sum of length * sigma, sigma = lut[attr].a (1 when opaque);
 * level l+1 averages the 2^3 children of level l (children beyond an odd side
 * count as 0), down to 1^3. Stored as float per level.
 *
 * Optionally the per-voxel illumination grids (sections "Shadow simulation",
 * "Ambient occlusion", "Illumination effects"), computed by cone tracing on
 * rho: from the voxel centre p along direction u, samples at distance s with
 * cone diameter D = max(1, aperture * s) on level min(L, floor(log2 D))
 * (cell-centred trilinear, clamp to edge), occlusion += rho * D, s += D, while
 * s < s_max and the point is inside the grid; occlusion is capped at 1.
 *   ao[v] = 1 - mean over ao_cones spherical-Fibonacci directions
 *           (s_max = ao_radius)
 *   sh[v] = 1 - occlusion towards light_dir (s_max = infinity)
 *   lut_rgba   device, float [256][4] straight alpha
 *
 * Optionally one representative line per voxel of every level (section "LoD
 * construction"), exported as uint32 codes (LS_EXPORT_REP_LINES, levels flat
 * at level_off; the record layout's low 30 bits with start = entry, end =
 * exit; 0xFFFFFFFF where a voxel has no lines): the start and end points of
 * the voxel's lines are averaged separately, a line flipped first when its
 * direction has a negative dot product with the previous line (list order,
 * as flipped); each average goes to the closest bin centre on the boundary
 * (first face, lowest bins on ties); then two face-adjacent voxels with one
 * endpoint each on their common face move both to the bin of the points'
 * mean (a mean on a bin boundary to the upper bin). Level l + 1 averages the
 * joined lines of its children (x fastest, then y, z) in its own frame and
 * joins again. Exact integer arithmetic; bit-identical to the definition.
 *
 * Optionally a colour pyramid beside rho (LS_EXPORT_LOD_COLOR, float
 * [level_off][3]): per voxel the sum over its lines of length * sigma * lut
 * rgb, averaged up the levels like rho; rgb / rho is the density-weighted
 * mean colour that opacity acceleration composites.
 * Errors: LS_EINVAL (bad cone count, radius, aperture or light), LS_ENOMEM;
 * LS_EUNSUPPORTED when a cone needs more than 48 samples or sample distances
 * not exact in fp32 (apertures far below 1). */
typedef struct {
  const float* lut_rgba;
  int32_t opaque;
  int32_t build_ao;
  int32_t ao_cones;          /* default 16, at most 32 */
  float ao_radius;           /* default 15 voxels */
  float cone_aperture;       /* default 1: the cone subtends one voxel at s = 1 */
  int32_t build_shadow;
  float light_dir[3];        /* unit vector towards a directional light */
  int32_t build_rep_lines;   /* 1: representative lines of every level (see below) */
  int32_t build_color;       /* 1: colour pyramid for opacity acceleration (see below) */
} ls_lod_desc;

int lineset_build_lod(ls_lineset_t set, const ls_lod_desc* desc, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Rendering (sections "Line Raycasting", "Ray-tube intersections",
 * "Rendering effects", "Transparency rendering").
 *
 * Camera: pixel (i, j), row 0 at the top, sampled at its centre:
 *   u = 2(i + 0.5)/W - 1, v = 1 - 2(j + 0.5)/H;
 *   perspective: origin = eye, direction = forward + u right + v up;
 *   orthographic: origin = eye + u right + v up, direction = forward;
 * evaluated in fp64 and rounded to fp32 (right/up are half-extent vectors).
 *
 * Each ray is clipped to the grid box and walks it voxel by voxel; the next
 * crossing of axis a is (plane - o_a) * (1 / d_a) in fp64, ties to the lowest
 * axis. Lines are capsules of `radius` (tube plus joint spheres). mode 0
 * tests the lines of the visited voxel only and accepts hits with t >= 0
 * (interactive mode); mode 1 also tests the 26 neighbour voxels and accepts a
 * hit in the voxel whose [t0, t1) holds its entry t (still-camera mode).
 * Accepted hits of a voxel are composited in (entry t, record index) order:
 * with merge_curves, a hit whose entry lies inside the open interval of the
 * same curve extends it and is not blended again. Colour per fragment:
 *   shading 0: lut rgb
 *   shading 1: rgb (ka + kd |n.v|) + ks |n.v|^shininess
 *   shading 2: rgb (ka AO(x) + kd SH(x) max(0, n.L)) + ks SH(x) max(0, n.h)^shininess
 * (v towards the eye, h = normalize(L + v), AO/SH trilinear at the entry).
 * In shading 2 the AO and shadow factors come from (view-dependent
 * illumination, sections "Shadow simulation" and "Ambient occlusion"):
 *   ao_mode 0: the per-voxel AO grid, trilinear at the entry point x;
 *   ao_mode 1: per fragment, ao_rays hemisphere rays about the tube normal n
 *     (equal-area heights 1 - (i + 0.5)/ao_rays, azimuth i * pi (3 - sqrt 5),
 *     in the Duff et al. orthonormal frame of n), each sampling the finest
 *     density level at distances 1, 2, ... < ao_radius until the density sum
 *     reaches 1; AO = 1 - mean occlusion;
 *   shadow_mode 0: the per-voxel shadow grid at x;
 *   shadow_mode 1: per fragment, 1 - the cone occlusion from x towards
 *     light_dir (aperture 1, as the shadow grid's cones);
 *   shadow_mode 2: per fragment, a shadow ray from x towards light_dir walks
 *     level rep_level and is tested against the representative lines there,
 *     tubes of `radius` in that level's voxel units: 0 if it enters one at a
 *     positive distance, else 1.
 * Premultiplied front-to-back: C += (1 - A) a c, A += (1 - A) a; the ray stops
 * once A >= alpha_stop (opaque lines: a = 1). Opacity a = lut alpha, or with
 * distance_alpha (section "Transparency rendering": opacity dependent on the
 * distance the ray travels inside the tube) a = 1 - (1 - lut alpha)^(l / 2r),
 * l = |d| (t_out - t_in) the chord of the composited hit (a merged hit adds
 * nothing; a tangent hit, l = 0, is transparent).
 *   lut_rgba   device, float [256][4] straight alpha
 *   rgba_out   device, float [height][width][4], premultiplied (C, A)
 * Opacity acceleration (section "Transparency rendering", after Danskin and
 * Hanrahan), transparent lines only: once the accumulated optical depth
 * -ln(1 - A) reaches accel_depth > 0 after a fragment, the ray leaves the
 * lines at the end of that voxel and samples the density pyramid instead:
 * at optical depth d, level l = min(top, 1 + floor(log2(d / accel_depth))),
 * step 2^l voxels, one trilinear sample at each step's midpoint with opacity
 * min(1, rho 2^l) and the colour pyramid's mean colour (unlit), front to
 * back until alpha_stop or the grid's edge. The image then differs from the
 * exact one by at most exp(-accel_depth) per channel.
 * Errors: LS_EINVAL for a zero or negative size, radius <= 0 (or >= 1 in
 * mode 1), a zero forward/direction, shading 2 without the grids, pyramid or
 * representative lines its sources need, ao_rays outside [1, 256], a
 * negative or non-finite accel_depth, acceleration without the pyramids. */
typedef struct {
  float eye[3], forward[3], right[3], up[3];
  int32_t orthographic, width, height;
} ls_camera;

typedef struct {
  float radius;
  int32_t mode;
  int32_t opaque;
  float alpha_stop;          /* default 0.95 */
  int32_t merge_curves;
  const float* lut_rgba;
  int32_t shading;
  float ka, kd, ks, shininess;
  float light_dir[3];
  int32_t distance_alpha;    /* 1: opacity from the chord length (see below) */
  int32_t ao_mode;           /* shading 2: 0 per-voxel grid, 1 per-fragment hemisphere */
  int32_t shadow_mode;       /* shading 2: 0 per-voxel grid, 1 per-fragment cone,
                                2 representative-line shadow ray */
  int32_t ao_rays;           /* ao_mode 1: rays per fragment (default 16) */
  float ao_radius;           /* ao_mode 1: radius of influence in voxels (default 15) */
  int32_t rep_level;         /* shadow_mode 2: pyramid level of the representative lines */
  float accel_depth;         /* opacity acceleration from this optical depth (0: off; see above) */
} ls_render_params;

/* Launch order (no effect on the image): a frame with more screen
 * tiles than the device runs at once records each tile's duration (the
 * first frame of a transparent view starts its tiles in the order of a cost
 * estimate from the occupancy words along four rays per tile); when the
 * same stream renders the same view again (same set shape and record count,
 * camera, image size and parameters), or the view with its camera moved
 * slightly (eye within 2 % of the grid's diagonal, each camera vector within
 * 2 degrees and 1 % in length), its tiles start longest first by the times
 * of that earlier frame and the 32 longest are split four ways (eight ways
 * in frames that split no other tile). The library
 * keeps, per (device, stream), the tile times of the stream's last 64 such
 * views (4 bytes per tile each) and one ordering buffer, until the process
 * ends; enlarging them synchronises the stream once. */
int lineset_render(ls_lineset_t set, const ls_camera* cam, const ls_render_params* params,
                   float* rgba_out, void* hip_stream);

/* Same image as lineset_render, with per-frame work counters (host struct,
 * filled after the call synchronises the stream). */
typedef struct {
  int64_t visited;          /* voxels whose list header was read */
  int64_t nonempty;         /* visited voxels whose own list is not empty */
  int64_t tested;           /* ray-capsule tests */
  int64_t hits;             /* accepted hits */
  int64_t fragments;        /* composited fragments */
  int64_t list_bytes;       /* bytes of offsets and records read */
  int64_t sort_passes;      /* extra passes for voxels with more hits than the sort buffer */
  int64_t merge_evictions;  /* open intervals evicted from the bounded merge table */
  int64_t macro_skips;      /* empty 4^3 macro cells jumped over */
  int64_t merge_live_evictions; /* evictions of intervals still open at the new hit's entry
                                   (a later hit of that curve may be blended again) */
  int64_t merge_overflow_rays;  /* rays with at least one such eviction: an upper bound on
                                   the pixels that differ from an unbounded table */
} ls_render_counters;

int lineset_render_counted(ls_lineset_t set, const ls_camera* cam,
                           const ls_render_params* params, float* rgba_out,
                           ls_render_counters* counters, void* hip_stream);

/* The per-curve merge table of a ray holds `merge_slots` open intervals.
 * When it is full, the interval that closed first is evicted; the image then
 * equals that of an unbounded table unless an evicted interval is still open
 * at the new hit and its curve is hit again (merge_live_evictions and
 * merge_overflow_rays count this). A ray along which at most merge_slots
 * curves are open at once is exact. */
int lineset_render_limits(int32_t* merge_slots);

/* ------------------------------------------------------------------------ */
/* Batched rendering: many views of many resident line sets (uneven sizes,
 * mixed modes) in ONE persistent launch. The screen tiles of all views form
 * one list split into 8 queues (one per XCD); workgroups pop tiles from their
 * XCD's queue and steal from the others. Each view's pixels are computed
 * exactly as lineset_render computes them.
 *   flags LS_BATCH_AUTOTUNE: time every tile shape (1x1 .. 4x1 waves of 8x8
 *         pixels) and persistent grid size on this batch at creation and keep
 *         the fastest (cached per batch signature for the process);
 *   flags LS_BATCH_GRAPH: capture the launch in a hipGraph replayed by
 *         lineset_batch_render.
 * The batch borrows the views' sets, LUTs and outputs: they must outlive it.
 * Creation renders the batch while autotuning (outputs are overwritten).
 * Errors: LS_EINVAL for an invalid view (same rules as lineset_render) or
 * n_views outside [1, 2^20]; LS_ENOMEM. */
typedef struct {
  ls_lineset_t set;
  ls_camera cam;
  ls_render_params params;
  float* rgba_out;           /* device, float [height][width][4] */
} ls_view;

typedef struct ls_batch* ls_batch_t;

enum { LS_BATCH_AUTOTUNE = 1, LS_BATCH_GRAPH = 2 };

typedef struct {
  int32_t waves_x, waves_y;  /* tile shape: waves_x x waves_y waves of 8 x 8 pixels */
  int32_t blocks;            /* persistent workgroups */
  int32_t n_tiles;
  int32_t autotuned;         /* 0 default plan, 1 tuned now, 2 from the cache */
  int32_t candidates;        /* plans timed */
  float tuned_ms;            /* best candidate's time per launch */
  int32_t graph;             /* replayed from a hipGraph */
} ls_batch_config;

int lineset_batch_create(const ls_view* views, int32_t n_views, int32_t flags, void* hip_stream,
                         ls_batch_t* out);
/* The plans the autotuner times, in its order: tile shape (waves_x x
 * waves_y waves) and persistent grid size (grid_mult x CUs x workgroups per
 * CU). Writes min(cap, count) entries and the count to *n. */
int lineset_batch_candidates(int32_t* waves_x, int32_t* waves_y, int32_t* grid_mult, int32_t cap,
                             int32_t* n);
/* lineset_batch_create with a fixed plan (one of the candidates' tile shapes,
 * grid_mult in [1, 8]; no autotuning, no plan cache; flags may hold
 * LS_BATCH_GRAPH only), so every plan the autotuner can pick can be run and
 * checked. Errors: LS_EINVAL for an unknown shape or multiplier, or with
 * LS_BATCH_AUTOTUNE; otherwise as lineset_batch_create. */
int lineset_batch_create_plan(const ls_view* views, int32_t n_views, int32_t waves_x,
                              int32_t waves_y, int32_t grid_mult, int32_t flags, void* hip_stream,
                              ls_batch_t* out);
int lineset_batch_render(ls_batch_t batch, void* hip_stream);
int lineset_batch_render_counted(ls_batch_t batch, ls_render_counters* counters,
                                 void* hip_stream);
int lineset_batch_config(ls_batch_t batch, ls_batch_config* out);
void lineset_batch_destroy(ls_batch_t batch);   /* waits for the device */

/* One-shot: create (default plan, no graph), render, synchronise, destroy. */
int lineset_render_batch(const ls_view* views, int32_t n_views, void* hip_stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same one-shot
 * batch as lineset_render_batch (same default plan, same images), with its
 * queue counters, tile starts and view descriptors in a fixed device array of
 * the library (about 80 KB per GPU, held until the process ends) instead of
 * allocated buffers. Calls no hipMalloc / hipFree. At most 256 views per call
 * (LS_EINVAL beyond); the views' sets, LUTs and outputs are the caller's as
 * in lineset_render_batch. Synchronises hip_stream before returning. Every
 * call on one GPU uses that GPU's one array: calls that overlap on the same
 * GPU (from several host threads) race and must be serialised by the caller. */
int lineset_render_batch_static(const ls_view* views, int32_t n_views, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Render server: keeps voxelized line sets resident, admits render requests
 * by an HBM budget and batches them continuously (section "GPU
 * implementation": the voxel model stays resident and rendering runs per
 * view). A scheduler thread owns n_slots launch slots (stream + event +
 * descriptor buffers). Whenever a slot is free it takes the queue's head
 * requests, in arrival order, while their memory fits, and renders them in
 * one batched launch; requests arriving meanwhile go into the next free slot,
 * so batches overlap on the device. Each request's image equals its
 * lineset_render image.
 *
 * Memory. The budget holds the resident sets (their current device bytes,
 * re-read at every admission, so grids built after ls_server_add_lineset
 * count), the output arena and the outputs being written:
 *   - output_arena_bytes > 0: the server allocates that much device memory at
 *     creation. A request submitted with rgba_out == NULL renders into an
 *     arena block of W*H*16 bytes (rounded up to 256), taken first-fit when
 *     the request reaches the head of the queue; while no block fits, the
 *     head waits (held_for_memory). The block returns to the arena when
 *     ls_server_result copies the image out. Arena requests must be
 *     collected, or the queue behind them stalls.
 *   - rgba_out != NULL: the caller owns the output; the request reserves
 *     W*H*16 bytes plus a descriptor while in flight, within
 *     budget - resident sets - arena.
 * Device memory is allocated only by ls_server_create.
 *
 * Ordering. ls_server_submit records an event on hip_stream; the render
 * waits for it, so work queued on that stream before the call (building the
 * set's grids, filling the LUT, clearing rgba_out) is done before the render
 * reads or writes. Completion is observed on the host (ls_server_wait).
 *
 *   ls_server_add_lineset: the set's device bytes count against the budget
 *     (LS_ENOMEM if they do not fit); the server borrows the set.
 *   ls_server_submit: non-blocking; LS_EBUSY when max_queue requests wait,
 *     LS_ENOMEM when the request alone exceeds the arena (rgba_out NULL) or
 *     what the budget leaves, LS_EINVAL for invalid views (lineset_render's
 *     rules) or rgba_out NULL without an arena. rgba_out and the LUT must
 *     stay valid until the request completes.
 *   ls_server_wait: blocks up to timeout_us (negative: forever); LS_OK once
 *     the image is written, LS_ETIMEOUT else. A caller-owned request's
 *     ticket is then retired; an arena request's stays until
 *     ls_server_result.
 *   ls_server_result: for a completed arena request, copies the H*W*4 floats
 *     into dst (device or host memory, dst_bytes large enough) on hip_stream,
 *     synchronises that stream, returns the block and retires the ticket.
 *     LS_EBUSY if the request has not completed, LS_EINVAL for other tickets.
 *   ls_server_stats: latency percentiles from submission to observed
 *     completion over all completed requests; Mrays/s over the span from the
 *     first submission to the last completion.
 *   ls_server_destroy: finishes the work in flight; requests still queued
 *     behind uncollected arena blocks are dropped. */
typedef struct ls_server* ls_server_t;

typedef struct {
  size_t hbm_budget_bytes;
  int32_t n_slots;           /* concurrent batched launches, 1..16 */
  int32_t max_batch_views;   /* requests per launch, 1..4096 */
  int32_t max_queue;         /* waiting requests before LS_EBUSY */
  size_t output_arena_bytes; /* server-owned output memory (0: none), within the budget */
} ls_server_config;

typedef struct {
  int64_t completed;
  double p50_ms, p99_ms, max_ms;
  double mrays_per_s;
  int64_t batches;
  double mean_batch;
  int64_t queued, max_queue_depth, rejected;
  size_t resident_bytes, inflight_bytes;
  int64_t held_for_memory;   /* requests that waited at the queue head because
                                their memory did not fit */
  size_t arena_bytes, arena_in_use;
} ls_server_report;

int ls_server_create(const ls_server_config* cfg, ls_server_t* out);
int ls_server_add_lineset(ls_server_t server, ls_lineset_t set, int32_t* set_id);
int ls_server_submit(ls_server_t server, int32_t set_id, const ls_camera* cam,
                     const ls_render_params* params, float* rgba_out, void* hip_stream,
                     uint64_t* ticket);
int ls_server_wait(ls_server_t server, uint64_t ticket, int64_t timeout_us);
int ls_server_result(ls_server_t server, uint64_t ticket, float* dst, size_t dst_bytes,
                     int32_t dst_on_device, void* hip_stream);
int ls_server_stats(ls_server_t server, ls_server_report* out);
void ls_server_destroy(ls_server_t server);   /* finishes queued work first */

/* ------------------------------------------------------------------------ */
/* Device memory cache. The library takes every device buffer it owns (set
 * arrays, voxelizer temporaries) from a per-device cache: released blocks
 * are kept and handed out again to requests that fit (sizes rounded up to a
 * power of two below 1 MiB, to a multiple of 2 MiB above), so repeated work
 * of one shape does not call hipMalloc / hipFree. lineset_destroy waits for
 * the device before its blocks return to the cache. Cached blocks go back to
 * the runtime when an allocation fails, or here:
 *   lineset_pool_trim: frees every cached (not live) block on every device.
 *   lineset_pool_stats: bytes cached (free, kept) and held (live + cached) on
 *     `device`; LS_EINVAL for a negative device. */
void lineset_pool_trim(void);
int lineset_pool_stats(int32_t device, size_t* cached_bytes, size_t* held_bytes);

/* ------------------------------------------------------------------------ */
/* Inspection. */
typedef struct {
  int32_t grid[3];
  int32_t bins;
  int64_t n_curves, n_vertices;
  int64_t n_records;
  int64_t n_record_slots;    /* records emitted before dropping */
  int64_t nonempty_voxels;
  int64_t max_list;          /* longest per-voxel list */
  int32_t n_levels;          /* density pyramid levels (0 before build_lod) */
  int32_t has_ao, has_shadow;
  int32_t has_rep_lines;
  int32_t has_vertex_attr;   /* per-line endpoint attributes (LS_EXPORT_ENDS) */
  int32_t has_color;         /* colour pyramid (LS_EXPORT_LOD_COLOR) */
  int32_t level_dims[32][3];
  int64_t level_off[33];
  double lo_scale[4];        /* grid set-up of xyz input: lo[3], S */
  size_t device_bytes;       /* bytes held by the set */
} ls_info;

int lineset_info(ls_lineset_t set, ls_info* out);

enum {
  LS_EXPORT_OFFSETS = 0,     /* uint32 [voxels + 1] */
  LS_EXPORT_RECORDS = 1,     /* uint64 [n_records] */
  LS_EXPORT_LOD_COUNT = 2,   /* float, all levels flat (level_off) */
  LS_EXPORT_LOD_LEN = 3,
  LS_EXPORT_LOD_RHO = 4,
  LS_EXPORT_AO = 5,          /* float [voxels] */
  LS_EXPORT_SHADOW = 6,      /* float [voxels] */
  LS_EXPORT_REP_LINES = 7,   /* uint32, all levels flat (level_off) */
  LS_EXPORT_ENDS = 8,        /* uint16 [n_records]: entry | exit << 8 attributes */
  LS_EXPORT_LOD_COLOR = 9    /* float [level_off][3], all levels flat */
};

/* Copies one buffer of the set into `dst` (host or device). Errors:
 * LS_EINVAL if the buffer does not exist or dst_bytes is too small. */
int lineset_export(ls_lineset_t set, int32_t what, void* dst, size_t dst_bytes,
                   int32_t dst_on_device, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LINESET_H */
