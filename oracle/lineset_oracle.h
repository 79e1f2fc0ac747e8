/*
 * CPU oracle for voxel-based ray-casting of 3D line sets
 * (Kanzler, Rautenhaus, Westermann, "A Voxel-based Rendering Pipeline for
 * Large 3D Line Sets").
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, plain reference the
 * GPU path is checked against. Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code with the HIP library.
 *
 * Integer work (grid set-up, voxelization, CSR) is exact; floating-point
 * work is fp64 except where the method fixes a value to fp32 (the ray itself,
 * see or_ray).
 */
#ifndef LINESET_ORACLE_H
#define LINESET_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Per-voxel record (8 bytes):
 *   bits  0..2   entry face     bits  3..8  entry bin u   bits  9..14 entry bin w
 *   bits 15..17  exit face      bits 18..23 exit bin u    bits 24..29 exit bin w
 *   bits 32..39  attribute      bits 40..63 curve id mod 2^24
 * Faces: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z. In-plane axes (u, w) are the two
 * other axes in increasing order. */

/* Section "Curve voxelization": grid set-up. Maps float vertices to a
 * 1/256-voxel lattice inside grid[0..2] voxels with a one-voxel margin. */
int or_grid_setup(const float* xyz, int64_t n_vertices, const int32_t grid[3],
                  int32_t* lattice_out, double* lo_out, double* scale_out);

typedef struct {
  int64_t n_records;
  int64_t n_voxels;
  uint32_t* offsets;   /* [n_voxels + 1] */
  uint64_t* records;   /* [n_records] */
  int64_t n_events;
  int64_t n_dropped;
  uint16_t* ends;      /* [n_records] endpoint attributes entry | exit << 8, or NULL */
} or_csr;

/* Sections "Curve voxelization", "Line quantization", "GPU implementation". */
int or_voxelize(const int32_t* lattice, const int64_t* curve_off,
                const uint8_t* attr, int64_t n_curves, const int32_t grid[3],
                int32_t bins, or_csr* out);
/* The same with per-vertex attributes (section "Curve voxelization": line
 * attributes interpolated to the line-face intersection points): vattr holds
 * one byte per vertex (NULL: none); out->ends gets each line's endpoint
 * attributes and its record's attribute byte their mean (rounded down). */
int or_voxelize_attr(const int32_t* lat, const int64_t* curve_off, const uint8_t* attr,
                     const uint8_t* vattr, int64_t n_curves, const int32_t grid[3], int32_t bins,
                     or_csr* out);
void or_csr_free(or_csr* c);

/* Section "Memory statistics": bytes per quantized line in the paper's
 * packed format (two 3-bit face ids, two 2*log2(N)-bit bin indices, one
 * attribute byte, a 5-bit local line id, rounded up to whole bytes). */
int or_paper_record_bytes(int32_t bins);

/* Section "LoD construction": level dims and the count / length / density
 * pyramid. level_off[l] is the first voxel of level l in the flat arrays. */
int or_lod_levels(const int32_t grid[3], int32_t* dims_out /* [32][3] */,
                  int64_t* level_off_out /* [33] */);
int or_lod(const uint32_t* offsets, const uint64_t* records, const int32_t grid[3],
           int32_t bins, const float* lut_rgba, int32_t opaque,
           double* count, double* len, double* rho);

/* Colour pyramid for opacity acceleration: rgb[v][3] = sum of length *
 * sigma * lut colour over the voxel's lines, averaged up the levels. */
int or_lod_color(const uint32_t* offsets, const uint64_t* records, const int32_t grid[3],
                 int32_t bins, const float* lut_rgba, int32_t opaque, double* rgb);

/* Sections "Shadow simulation" and "Ambient occlusion": per-voxel cone-traced
 * occlusion grids on the density pyramid. */
double or_cone(const double* rho, const int32_t grid[3], const double p[3],
               const double dir[3], double s_max, double aperture);
void or_fibonacci_dirs(int32_t n, double* dirs /* [n][3] */);
int or_ao_grid(const double* rho, const int32_t grid[3], int32_t n_cones,
               double radius, double aperture, double* ao, int32_t n_threads);
int or_shadow_grid(const double* rho, const int32_t grid[3], const double light[3],
                   double aperture, double* sh, int32_t n_threads);
/* The same grids over voxels [v0, v1) only (out[v - v0]): bounded samples. */
int or_ao_grid_part(const double* rho, const int32_t grid[3], int32_t n_cones, double radius,
                    double aperture, int64_t v0, int64_t v1, double* ao, int32_t n_threads);
int or_shadow_grid_part(const double* rho, const int32_t grid[3], const double light[3],
                        double aperture, int64_t v0, int64_t v1, double* sh, int32_t n_threads);

/* Section "LoD construction": one representative line per voxel and level
 * (code = record bits 0..29, 0xFFFFFFFF for none), levels flat at the
 * density pyramid's level offsets. Returns the level count. */
int or_rep_lines(const uint32_t* offsets, const uint64_t* records, const int32_t grid[3],
                 int32_t bins, uint32_t* rep);
/* Section "Shadow simulation", first approach: 1 if the ray from x towards
 * `light` enters a representative line of `level` (radius in that level's
 * voxel units) at a positive distance. */
int or_rep_shadow(const uint32_t* rep, const int32_t grid[3], int32_t bins, int32_t level,
                  double radius, const double x[3], const double light[3]);
/* Section "Ambient occlusion", first approach: k hemisphere directions
 * around n, and 1 - mean occlusion of level-0 rays of the given radius. */
void or_hemi_dirs(const double n[3], int32_t k, double* dirs /* [k][3] */);
double or_ao_hemi(const double* rho, const int32_t grid[3], const double x[3],
                  const double n[3], int32_t k, double radius);

/* Section "Line Raycasting" and "Rendering effects". */
typedef struct {
  float eye[3], forward[3], right[3], up[3];
  int32_t orthographic, width, height;
} or_camera;

typedef struct {
  float radius;
  int32_t mode;          /* 0 own-voxel lists, 1 with 26 neighbour lists */
  int32_t opaque;
  float alpha_stop;
  int32_t merge_curves;
  const float* lut_rgba; /* [256][4] straight alpha */
  int32_t shading;       /* 0 flat colour, 1 head-light Phong, 2 AO + shadow */
  float ka, kd, ks, shininess;
  float light_dir[3];    /* towards the light, unit length */
  int32_t distance_alpha; /* 1: opacity from the chord length inside the tube */
  /* shading 2, view-dependent sources (sections "Shadow simulation",
   * "Ambient occlusion"): */
  int32_t ao_mode;       /* 0 per-voxel AO grid, 1 per-fragment hemisphere rays on level 0 */
  int32_t shadow_mode;   /* 0 per-voxel shadow grid, 1 per-fragment cone,
                            2 shadow ray against the representative lines */
  int32_t ao_rays;       /* hemisphere rays (ao_mode 1) */
  float ao_radius;       /* radius of influence (ao_mode 1), voxels */
  int32_t rep_level;     /* level of the representative lines (shadow_mode 2) */
  const double* rho;     /* density pyramid, levels flat (ao_mode 1, shadow_mode 1) */
  const uint32_t* rep;   /* representative lines, levels flat (shadow_mode 2) */
  const uint16_t* ends;  /* per-record endpoint attributes (or NULL): colour and
                            opacity from the attribute interpolated along the line */
  float accel_depth;     /* opacity acceleration from this optical depth (0: off) */
  const double* rgb;     /* colour pyramid [level_off][3] (or_lod_color), accel_depth > 0 */
} or_params;

typedef struct {
  int64_t visited, nonempty, tested, hits, fragments;
} or_counters;

void or_ray(const or_camera* cam, int32_t i, int32_t j, float o[3], float d[3]);

/* Voxels visited by a ray, in order, with their [t0, t1). Returns the count
 * (may exceed cap; only cap entries are written). */
int64_t or_dda(const int32_t grid[3], const float o[3], const float d[3],
               int32_t* cells, double* t0, double* t1, int64_t cap);

/* Ray vs capsule (segment a-b, radius r). Returns 1 on hit. */
int or_capsule(const double o[3], const double d[3], const double a[3],
               const double b[3], double r, double* t_in, double* t_out,
               double n_out[3]);

/* Decoded endpoints of a record in voxel-local units. */
void or_decode(uint64_t rec, int32_t bins, double entry[3], double exit_[3]);

/* Render pixels. pixels == NULL renders the full W*H image into
 * rgba[(j*W+i)*4]; otherwise renders the n_pixels listed (index j*W+i) into
 * rgba[k*4]. ao/sh may be NULL unless shading == 2. */
int or_render(const uint32_t* offsets, const uint64_t* records,
              const int32_t grid[3], int32_t bins, const or_camera* cam,
              const or_params* p, const double* ao, const double* sh,
              const int64_t* pixels, int64_t n_pixels, double* rgba,
              or_counters* counters, int32_t n_threads);

#ifdef __cplusplus
}
#endif
#endif
