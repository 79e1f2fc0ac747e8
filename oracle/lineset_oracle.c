/*
 * CPU oracle for voxel-based ray-casting of 3D line sets.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path. It shares no
 * code with the HIP library. Plain loops, no blocking or fusion: each
 * function follows the paper section it cites, in the order the paper states
 * the steps. Integer work is exact (int64); floating point is fp64 except the
 * ray, which the method fixes to fp32 values (or_ray).
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off
 */
#define _GNU_SOURCE
#include "lineset_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAX_DIM 1024

/* ------------------------------------------------------------------------ */
/* Section "Curve voxelization", first paragraph: cube voxels of side 1, the
 * curves' bounding box mapped into [0, r]^3 keeping its aspect ratio. Reading
 * used: the longest extent spans r - 2 voxels (one empty voxel of margin on
 * each side) and vertices are rounded to a lattice of 1/256 voxel so that the
 * voxelization below is exact integer arithmetic. */
int or_grid_setup(const float* xyz, int64_t nv, const int32_t grid[3],
                  int32_t* lat, double* lo_out, double* scale_out) {
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a)
    if (grid[a] < 3 || grid[a] > MAX_DIM) return -1;
  if (nv > 0) {
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int64_t v = 0; v < nv; ++v)
      for (int a = 0; a < 3; ++a) {
        double x = (double)xyz[3 * v + a];
        if (!(x == x) || isinf(x)) return -1;
        if (x < lo[a]) lo[a] = x;
        if (x > hi[a]) hi[a] = x;
      }
  }
  double s = INFINITY;
  for (int a = 0; a < 3; ++a) {
    double ext = hi[a] - lo[a];
    if (ext > 0) {
      double cand = (256.0 * (double)(grid[a] - 2)) / ext;
      if (cand < s) s = cand;
    }
  }
  if (isinf(s)) s = 0.0;
  for (int64_t v = 0; v < nv; ++v)
    for (int a = 0; a < 3; ++a) {
      double x = (double)xyz[3 * v + a];
      double y = (x - lo[a]) * s;
      y = y + 0.5;
      lat[3 * v + a] = (int32_t)floor(y) + 256;
    }
  if (lo_out) for (int a = 0; a < 3; ++a) lo_out[a] = lo[a];
  if (scale_out) *scale_out = s;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Sections "Curve voxelization" and "Line quantization".
 *
 * Each curve segment P0 -> P1 (lattice units, 256 per voxel) is clipped
 * against the voxel faces in the order the crossings occur. A crossing of the
 * plane x_a = 256 k happens going up iff P0_a < 256k <= P1_a and going down
 * iff P1_a < 256k <= P0_a (half-open voxels), at t = (256k - P0_a)/(P1_a - P0_a).
 * Crossings of several axes at equal t are one event (through an edge or a
 * corner); its face is that of the lowest axis involved. Consecutive events
 * of a curve bound one per-voxel line; the pieces before the first and after
 * the last event are dropped. Each endpoint is quantized to one of N x N
 * bins of its face: bin = min(floor(local * N / 256), N - 1), local being the
 * exact rational in-face coordinate. A line is dropped when its two exact
 * event points coincide or its two quantized endpoints coincide. */

typedef struct {
  int64_t xn[3];   /* event point * den, exact */
  int64_t den;
  uint32_t entry_code, exit_code;
  uint32_t attr;   /* vertex attribute interpolated to the event point */
} or_event;

/* Section "Curve voxelization": line attributes interpolated to the
 * line-face intersection points. The event lies at t = num / den along the
 * segment whose vertices carry a0 and a1; its attribute is a0 + (a1 - a0) t
 * rounded to the nearest integer (halves up), in exact integer arithmetic. */
static uint32_t event_attr(uint32_t a0, uint32_t a1, int64_t num, int64_t den) {
  int64_t s = 2 * ((int64_t)a0 * den + ((int64_t)a1 - (int64_t)a0) * num) + den;
  return (uint32_t)(s / (2 * den));
}

static uint32_t face_code(int axis, int side, const int64_t xn[3], int64_t den,
                          const int32_t cell[3], int32_t bins) {
  int ua = (axis == 0) ? 1 : 0;
  int wa = (axis == 2) ? 1 : 2;
  int64_t step = (int64_t)(256 / bins) * den;
  int64_t lu = xn[ua] - (int64_t)256 * cell[ua] * den;
  int64_t lw = xn[wa] - (int64_t)256 * cell[wa] * den;
  int64_t bu = lu / step, bw = lw / step;
  if (lu < 0 || lw < 0) abort(); /* an event point always lies on the voxel */
  if (bu > bins - 1) bu = bins - 1;
  if (bw > bins - 1) bw = bins - 1;
  return (uint32_t)(2 * axis + side) | (uint32_t)bu << 3 | (uint32_t)bw << 9;
}

typedef struct {
  uint32_t* vox;
  uint64_t* rec;
  uint16_t* ends;
  int64_t n, cap;
} rec_buf;

static int push_rec(rec_buf* b, uint32_t vox, uint64_t rec, uint16_t ends) {
  if (b->n == b->cap) {
    int64_t nc = b->cap ? 2 * b->cap : 1024;
    uint32_t* v2 = (uint32_t*)realloc(b->vox, (size_t)nc * sizeof(uint32_t));
    if (!v2) return -1;
    b->vox = v2;
    uint64_t* r2 = (uint64_t*)realloc(b->rec, (size_t)nc * sizeof(uint64_t));
    if (!r2) return -1;
    b->rec = r2;
    uint16_t* e2 = (uint16_t*)realloc(b->ends, (size_t)nc * sizeof(uint16_t));
    if (!e2) return -1;
    b->ends = e2;
    b->cap = nc;
  }
  b->vox[b->n] = vox;
  b->rec[b->n] = rec;
  b->ends[b->n] = ends;
  b->n++;
  return 0;
}

int or_voxelize(const int32_t* lat, const int64_t* curve_off, const uint8_t* attr,
                int64_t n_curves, const int32_t grid[3], int32_t bins, or_csr* out) {
  return or_voxelize_attr(lat, curve_off, attr, NULL, n_curves, grid, bins, out);
}

/* With per-vertex attributes (vattr, one byte per vertex), every event gets
 * the attribute interpolated to its point, each line keeps the attributes of
 * its two endpoints (out->ends: entry | exit << 8, in CSR order), and the
 * record's attribute byte is their mean rounded down, (entry + exit) / 2. */
int or_voxelize_attr(const int32_t* lat, const int64_t* curve_off, const uint8_t* attr,
                     const uint8_t* vattr, int64_t n_curves, const int32_t grid[3], int32_t bins,
                     or_csr* out) {
  memset(out, 0, sizeof(*out));
  for (int a = 0; a < 3; ++a)
    if (grid[a] < 1 || grid[a] > MAX_DIM) return -1;
  if (bins < 1 || bins > 64 || (bins & (bins - 1))) return -1;
  int64_t nvox = (int64_t)grid[0] * grid[1] * grid[2];
  int64_t nv = n_curves > 0 ? curve_off[n_curves] : 0;
  if (n_curves > 0 && curve_off[0] != 0) return -1;
  for (int64_t c = 0; c < n_curves; ++c)
    if (curve_off[c + 1] < curve_off[c]) return -1;
  for (int64_t v = 0; v < nv; ++v)
    for (int a = 0; a < 3; ++a)
      if (lat[3 * v + a] < 0 || lat[3 * v + a] >= 256 * grid[a]) return -1;

  rec_buf buf = {0};
  int64_t n_events = 0, n_dropped = 0;
  for (int64_t c = 0; c < n_curves; ++c) {
    int64_t v0 = curve_off[c], v1 = curve_off[c + 1];
    if (v1 - v0 < 2) continue;
    uint64_t hi_bits = ((uint64_t)(attr ? attr[c] : 255) << 32) |
                       ((uint64_t)(c & 0xFFFFFF) << 40);
    int32_t cell[3];
    for (int a = 0; a < 3; ++a) cell[a] = lat[3 * v0 + a] >> 8;
    int have_prev = 0;
    or_event prev;
    memset(&prev, 0, sizeof(prev));
    for (int64_t i = v0; i + 1 < v1; ++i) {
      const int32_t* P0 = lat + 3 * i;
      const int32_t* P1 = lat + 3 * (i + 1);
      int64_t d[3], k[3], remaining[3];
      int sgn[3];
      for (int a = 0; a < 3; ++a) {
        d[a] = (int64_t)P1[a] - P0[a];
        int64_t c0 = P0[a] >> 8, c1 = P1[a] >> 8;
        if (d[a] > 0) { sgn[a] = 1; k[a] = c0 + 1; remaining[a] = c1 - c0; }
        else if (d[a] < 0) { sgn[a] = -1; k[a] = c0; remaining[a] = c0 - c1; }
        else { sgn[a] = 0; k[a] = 0; remaining[a] = 0; }
      }
      for (;;) {
        /* next crossing: smallest t = num/den over the axes */
        int best = -1;
        int64_t bnum = 0, bden = 1;
        for (int a = 0; a < 3; ++a) {
          if (remaining[a] == 0) continue;
          int64_t num = sgn[a] > 0 ? 256 * k[a] - P0[a] : P0[a] - 256 * k[a];
          int64_t den = sgn[a] > 0 ? d[a] : -d[a];
          if (best < 0 || num * bden < bnum * den) { best = a; bnum = num; bden = den; }
        }
        if (best < 0) break;
        int in_group[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {
          if (remaining[a] == 0) continue;
          int64_t num = sgn[a] > 0 ? 256 * k[a] - P0[a] : P0[a] - 256 * k[a];
          int64_t den = sgn[a] > 0 ? d[a] : -d[a];
          if (num * bden == bnum * den) in_group[a] = 1;
        }
        int fa = in_group[0] ? 0 : (in_group[1] ? 1 : 2);
        int32_t ncell[3] = {cell[0], cell[1], cell[2]};
        for (int a = 0; a < 3; ++a) if (in_group[a]) ncell[a] += sgn[a];
        or_event ev;
        ev.den = sgn[fa] > 0 ? d[fa] : -d[fa];
        int64_t num = sgn[fa] > 0 ? 256 * k[fa] - P0[fa] : P0[fa] - 256 * k[fa];
        for (int b = 0; b < 3; ++b) ev.xn[b] = (int64_t)P0[b] * ev.den + num * d[b];
        int exit_side = sgn[fa] > 0 ? 1 : 0;
        ev.exit_code = face_code(fa, exit_side, ev.xn, ev.den, cell, bins);
        ev.entry_code = face_code(fa, 1 - exit_side, ev.xn, ev.den, ncell, bins);
        ev.attr = vattr ? event_attr(vattr[i], vattr[i + 1], num, ev.den) : 0;
        n_events++;
        if (have_prev) {
          /* the line inside `cell` runs from prev's entry to this exit */
          int same_point = 1;
          for (int b = 0; b < 3; ++b)
            if (prev.xn[b] * ev.den != ev.xn[b] * prev.den) same_point = 0;
          if (same_point || prev.entry_code == ev.exit_code) {
            n_dropped++;
          } else {
            uint32_t vox = (uint32_t)(cell[0] + (int64_t)grid[0] * (cell[1] + (int64_t)grid[1] * cell[2]));
            uint64_t rec = (uint64_t)prev.entry_code | ((uint64_t)ev.exit_code << 15) | hi_bits;
            uint16_t ends = 0;
            if (vattr) {
              rec = (rec & ~((uint64_t)0xFF << 32)) | ((uint64_t)((prev.attr + ev.attr) / 2) << 32);
              ends = (uint16_t)(prev.attr | (ev.attr << 8));
            }
            if (push_rec(&buf, vox, rec, ends)) goto oom;
          }
        }
        prev = ev;
        have_prev = 1;
        for (int a = 0; a < 3; ++a) cell[a] = ncell[a];
        for (int a = 0; a < 3; ++a)
          if (in_group[a]) { remaining[a]--; k[a] += sgn[a]; }
      }
    }
  }

  /* Section "GPU implementation": lines of a voxel stored consecutively, with
   * a per-voxel start index. A stable counting sort by voxel id keeps each
   * voxel's lines in (curve, order along the curve) order. */
  out->n_voxels = nvox;
  out->n_records = buf.n;
  out->n_events = n_events;
  out->n_dropped = n_dropped;
  out->offsets = (uint32_t*)calloc((size_t)nvox + 1, sizeof(uint32_t));
  out->records = (uint64_t*)malloc((size_t)(buf.n > 0 ? buf.n : 1) * sizeof(uint64_t));
  if (!out->offsets || !out->records) goto oom;
  if (vattr) {
    out->ends = (uint16_t*)malloc((size_t)(buf.n > 0 ? buf.n : 1) * sizeof(uint16_t));
    if (!out->ends) goto oom;
  }
  if (buf.n > 0xFFFFFFFFll) goto oom;
  for (int64_t r = 0; r < buf.n; ++r) out->offsets[buf.vox[r] + 1]++;
  for (int64_t v = 0; v < nvox; ++v) out->offsets[v + 1] += out->offsets[v];
  {
    uint32_t* cursor = (uint32_t*)malloc((size_t)(nvox > 0 ? nvox : 1) * sizeof(uint32_t));
    if (!cursor) goto oom;
    memcpy(cursor, out->offsets, (size_t)nvox * sizeof(uint32_t));
    for (int64_t r = 0; r < buf.n; ++r) {
      uint32_t at = cursor[buf.vox[r]]++;
      out->records[at] = buf.rec[r];
      if (vattr) out->ends[at] = buf.ends[r];
    }
    free(cursor);
  }
  free(buf.vox);
  free(buf.rec);
  free(buf.ends);
  return 0;
oom:
  free(buf.vox);
  free(buf.rec);
  free(buf.ends);
  or_csr_free(out);
  return -2;
}

void or_csr_free(or_csr* c) {
  free(c->offsets);
  free(c->records);
  free(c->ends);
  c->offsets = NULL;
  c->records = NULL;
  c->ends = NULL;
}

int or_paper_record_bytes(int32_t bins) {
  int lg = 0;
  while ((1 << lg) < bins) ++lg;
  int bits = 2 * 3 + 2 * (2 * lg) + 8 + 5;
  return (bits + 7) / 8;
}

/* ------------------------------------------------------------------------ */
/* Decoding (section "Line quantization"): an endpoint is the centre of its
 * bin on its face; the face coordinate is 0 or 1 in voxel units. */
static void decode_code(uint32_t code, int32_t bins, double p[3]) {
  int face = (int)(code & 7u);
  int axis = face >> 1, side = face & 1;
  int ua = (axis == 0) ? 1 : 0;
  int wa = (axis == 2) ? 1 : 2;
  double bu = (double)((code >> 3) & 63u), bw = (double)((code >> 9) & 63u);
  p[axis] = (double)side;
  p[ua] = (bu + 0.5) / (double)bins;
  p[wa] = (bw + 0.5) / (double)bins;
}

void or_decode(uint64_t rec, int32_t bins, double entry[3], double exit_[3]) {
  decode_code((uint32_t)(rec & 0x7FFFu), bins, entry);
  decode_code((uint32_t)((rec >> 15) & 0x7FFFu), bins, exit_);
}

/* ------------------------------------------------------------------------ */
/* Section "LoD construction": rho = sum over the voxel's lines of
 * length * opacity; coarser levels average 2^3 children (children outside an
 * odd-sized level count as 0). */
int or_lod_levels(const int32_t grid[3], int32_t* dims, int64_t* level_off) {
  int n = 0;
  int32_t cur[3] = {grid[0], grid[1], grid[2]};
  level_off[0] = 0;
  for (;;) {
    dims[3 * n + 0] = cur[0];
    dims[3 * n + 1] = cur[1];
    dims[3 * n + 2] = cur[2];
    level_off[n + 1] = level_off[n] + (int64_t)cur[0] * cur[1] * cur[2];
    ++n;
    if (cur[0] == 1 && cur[1] == 1 && cur[2] == 1) break;
    for (int a = 0; a < 3; ++a) cur[a] = (cur[a] + 1) / 2;
  }
  return n;
}

int or_lod(const uint32_t* offsets, const uint64_t* records, const int32_t grid[3],
           int32_t bins, const float* lut, int32_t opaque,
           double* count, double* len, double* rho) {
  int32_t dims[96];
  int64_t loff[33];
  int nl = or_lod_levels(grid, dims, loff);
  int64_t nvox = (int64_t)grid[0] * grid[1] * grid[2];
  for (int64_t v = 0; v < nvox; ++v) {
    double c = 0, l = 0, r = 0;
    for (uint32_t k = offsets[v]; k < offsets[v + 1]; ++k) {
      double a[3], b[3];
      or_decode(records[k], bins, a, b);
      double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
      double L = sqrt(dx * dx + dy * dy + dz * dz);
      int attr = (int)((records[k] >> 32) & 0xFF);
      double sigma = opaque ? 1.0 : (double)lut[4 * attr + 3];
      c += 1.0;
      l += L;
      r += L * sigma;
    }
    count[v] = c;
    len[v] = l;
    rho[v] = r;
  }
  for (int lv = 1; lv < nl; ++lv) {
    const int32_t* dc = dims + 3 * (lv - 1);
    const int32_t* dp = dims + 3 * lv;
    for (int32_t z = 0; z < dp[2]; ++z)
      for (int32_t y = 0; y < dp[1]; ++y)
        for (int32_t x = 0; x < dp[0]; ++x) {
          double sc = 0, sl = 0, sr = 0;
          for (int k = 0; k < 8; ++k) {
            int32_t cx = 2 * x + (k & 1), cy = 2 * y + ((k >> 1) & 1), cz = 2 * z + (k >> 2);
            if (cx >= dc[0] || cy >= dc[1] || cz >= dc[2]) continue;
            int64_t ci = loff[lv - 1] + cx + (int64_t)dc[0] * (cy + (int64_t)dc[1] * cz);
            sc += count[ci];
            sl += len[ci];
            sr += rho[ci];
          }
          int64_t pi = loff[lv] + x + (int64_t)dp[0] * (y + (int64_t)dp[1] * z);
          count[pi] = sc / 8.0;
          len[pi] = sl / 8.0;
          rho[pi] = sr / 8.0;
        }
  }
  return nl;
}

/* Colour beside the density (the opacity-acceleration reading of section
 * "Transparency rendering"): per voxel rgb[v] = sum over its lines of
 * length * sigma * (transfer-function colour), averaged up the levels like
 * rho, so rgb / rho is the density-weighted mean colour of a cell. */
int or_lod_color(const uint32_t* offsets, const uint64_t* records, const int32_t grid[3],
                 int32_t bins, const float* lut, int32_t opaque, double* rgb) {
  int32_t dims[96];
  int64_t loff[33];
  int nl = or_lod_levels(grid, dims, loff);
  int64_t nvox = (int64_t)grid[0] * grid[1] * grid[2];
  for (int64_t v = 0; v < nvox; ++v) {
    double c[3] = {0, 0, 0};
    for (uint32_t k = offsets[v]; k < offsets[v + 1]; ++k) {
      double a[3], b[3];
      or_decode(records[k], bins, a, b);
      double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
      double L = sqrt(dx * dx + dy * dy + dz * dz);
      int attr = (int)((records[k] >> 32) & 0xFF);
      double sigma = opaque ? 1.0 : (double)lut[4 * attr + 3];
      for (int q = 0; q < 3; ++q) c[q] += L * sigma * (double)lut[4 * attr + q];
    }
    for (int q = 0; q < 3; ++q) rgb[3 * v + q] = c[q];
  }
  for (int lv = 1; lv < nl; ++lv) {
    const int32_t* dc = dims + 3 * (lv - 1);
    const int32_t* dp = dims + 3 * lv;
    for (int32_t z = 0; z < dp[2]; ++z)
      for (int32_t y = 0; y < dp[1]; ++y)
        for (int32_t x = 0; x < dp[0]; ++x) {
          double s[3] = {0, 0, 0};
          for (int k = 0; k < 8; ++k) {
            int32_t cx = 2 * x + (k & 1), cy = 2 * y + ((k >> 1) & 1), cz = 2 * z + (k >> 2);
            if (cx >= dc[0] || cy >= dc[1] || cz >= dc[2]) continue;
            int64_t ci = loff[lv - 1] + cx + (int64_t)dc[0] * (cy + (int64_t)dc[1] * cz);
            for (int q = 0; q < 3; ++q) s[q] += rgb[3 * ci + q];
          }
          int64_t pi = loff[lv] + x + (int64_t)dp[0] * (y + (int64_t)dp[1] * z);
          for (int q = 0; q < 3; ++q) rgb[3 * pi + q] = s[q] / 8.0;
        }
  }
  return nl;
}

/* ------------------------------------------------------------------------ */
/* Sections "Shadow simulation" (cone tracing on the density levels, cone
 * subtending one voxel at the finest level) and "Ambient occlusion" (density
 * accumulated until it reaches 1 or the ray leaves the radius of influence or
 * the domain; averaged over the rays; per-voxel spherical occlusion).
 * Reading used: the cone diameter at distance s is D = max(1, aperture * s),
 * the sample is taken on level floor(log2 D) (cell-centred trilinear,
 * clamp-to-edge), weighted by D, and the next sample is D further along. */
static double sample_level(const double* rho_level, const int32_t* dim, int lv,
                           const double x[3]) {
  double scale = ldexp(1.0, -lv);
  int64_t i0[3], i1[3];
  double f[3];
  for (int a = 0; a < 3; ++a) {
    double g = x[a] * scale - 0.5;
    double fl = floor(g);
    f[a] = g - fl;
    int64_t lo = (int64_t)fl, hi = lo + 1;
    if (lo < 0) lo = 0;
    if (lo > dim[a] - 1) lo = dim[a] - 1;
    if (hi < 0) hi = 0;
    if (hi > dim[a] - 1) hi = dim[a] - 1;
    i0[a] = lo;
    i1[a] = hi;
  }
  double acc = 0;
  for (int k = 0; k < 8; ++k) {
    int bx = k & 1, by = (k >> 1) & 1, bz = k >> 2;
    int64_t ix = bx ? i1[0] : i0[0], iy = by ? i1[1] : i0[1], iz = bz ? i1[2] : i0[2];
    double w = (bx ? f[0] : 1 - f[0]) * (by ? f[1] : 1 - f[1]) * (bz ? f[2] : 1 - f[2]);
    acc += w * rho_level[ix + (int64_t)dim[0] * (iy + (int64_t)dim[1] * iz)];
  }
  return acc;
}

/* sample_level over an interleaved array (element k at lev[k * stride]) */
static double sample_level_stride(const double* lev, const int32_t* dim, int lv, const double x[3],
                                  int stride) {
  double scale = ldexp(1.0, -lv);
  int64_t i0[3], i1[3];
  double f[3];
  for (int a = 0; a < 3; ++a) {
    double g = x[a] * scale - 0.5;
    double fl = floor(g);
    f[a] = g - fl;
    int64_t lo = (int64_t)fl, hi = lo + 1;
    if (lo < 0) lo = 0;
    if (lo > dim[a] - 1) lo = dim[a] - 1;
    if (hi < 0) hi = 0;
    if (hi > dim[a] - 1) hi = dim[a] - 1;
    i0[a] = lo;
    i1[a] = hi;
  }
  double acc = 0;
  for (int k = 0; k < 8; ++k) {
    int bx = k & 1, by = (k >> 1) & 1, bz = k >> 2;
    int64_t ix = bx ? i1[0] : i0[0], iy = by ? i1[1] : i0[1], iz = bz ? i1[2] : i0[2];
    double w = (bx ? f[0] : 1 - f[0]) * (by ? f[1] : 1 - f[1]) * (bz ? f[2] : 1 - f[2]);
    acc += w * lev[stride * (ix + (int64_t)dim[0] * (iy + (int64_t)dim[1] * iz))];
  }
  return acc;
}

double or_cone(const double* rho, const int32_t grid[3], const double p[3],
               const double dir[3], double s_max, double aperture) {
  int32_t dims[96];
  int64_t loff[33];
  int nl = or_lod_levels(grid, dims, loff);
  int top = nl - 1;
  double occ = 0.0;
  double s = 1.0;
  while (s < s_max) {
    double x[3];
    int inside = 1;
    for (int a = 0; a < 3; ++a) {
      x[a] = p[a] + s * dir[a];
      if (!(x[a] >= 0.0 && x[a] < (double)grid[a])) inside = 0;
    }
    if (!inside) break;
    double D = aperture * s;
    if (D < 1.0) D = 1.0;
    int e;
    frexp(D, &e);           /* D = m * 2^e, m in [0.5, 1): floor(log2 D) = e - 1 */
    int lv = e - 1;
    if (lv > top) lv = top;
    occ += sample_level(rho + loff[lv], dims + 3 * lv, lv, x) * D;
    if (occ >= 1.0) break;
    s += D;
  }
  return occ < 1.0 ? occ : 1.0;
}

/* Spherical Fibonacci point set: z_i = 1 - (2i+1)/n, azimuth i * pi(3 - sqrt 5). */
void or_fibonacci_dirs(int32_t n, double* dirs) {
  double ga = 3.14159265358979323846 * (3.0 - sqrt(5.0));
  for (int32_t i = 0; i < n; ++i) {
    double z = 1.0 - (2.0 * i + 1.0) / (double)n;
    double r = sqrt(1.0 - z * z);
    double ph = ga * (double)i;
    dirs[3 * i + 0] = r * cos(ph);
    dirs[3 * i + 1] = r * sin(ph);
    dirs[3 * i + 2] = z;
  }
}

int or_ao_grid(const double* rho, const int32_t grid[3], int32_t n_cones,
               double radius, double aperture, double* ao, int32_t n_threads) {
  return or_ao_grid_part(rho, grid, n_cones, radius, aperture, 0,
                         (int64_t)grid[0] * grid[1] * grid[2], ao, n_threads);
}

/* Voxels [v0, v1) of the AO grid into ao[v - v0]. */
int or_ao_grid_part(const double* rho, const int32_t grid[3], int32_t n_cones, double radius,
                    double aperture, int64_t v0, int64_t v1, double* ao, int32_t n_threads) {
  double* dirs = (double*)malloc((size_t)n_cones * 3 * sizeof(double));
  if (!dirs) return -2;
  or_fibonacci_dirs(n_cones, dirs);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
  for (int64_t v = v0; v < v1; ++v) {
    int64_t x = v % grid[0], y = (v / grid[0]) % grid[1], z = v / ((int64_t)grid[0] * grid[1]);
    double p[3] = {x + 0.5, y + 0.5, z + 0.5};
    double sum = 0;
    for (int32_t c = 0; c < n_cones; ++c) sum += or_cone(rho, grid, p, dirs + 3 * c, radius, aperture);
    ao[v - v0] = 1.0 - sum / (double)n_cones;
  }
  free(dirs);
  return 0;
}

int or_shadow_grid(const double* rho, const int32_t grid[3], const double light[3],
                   double aperture, double* sh, int32_t n_threads) {
  return or_shadow_grid_part(rho, grid, light, aperture, 0,
                             (int64_t)grid[0] * grid[1] * grid[2], sh, n_threads);
}

/* Voxels [v0, v1) of the shadow grid into sh[v - v0]. */
int or_shadow_grid_part(const double* rho, const int32_t grid[3], const double light[3],
                        double aperture, int64_t v0, int64_t v1, double* sh, int32_t n_threads) {
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
  for (int64_t v = v0; v < v1; ++v) {
    int64_t x = v % grid[0], y = (v / grid[0]) % grid[1], z = v / ((int64_t)grid[0] * grid[1]);
    double p[3] = {x + 0.5, y + 0.5, z + 0.5};
    sh[v - v0] = 1.0 - or_cone(rho, grid, p, light, INFINITY, aperture);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Ray per pixel. Pixel (i, j), row 0 at the top, through the pixel centre:
 * u = 2(i + 0.5)/W - 1, v = 1 - 2(j + 0.5)/H. Perspective: o = eye,
 * d = F + u R + v U. Orthographic: o = eye + u R + v U, d = F. Evaluated in
 * fp64 from the fp32 camera, then rounded to fp32: those fp32 values are the
 * ray. */
void or_ray(const or_camera* cam, int32_t i, int32_t j, float o[3], float d[3]) {
  double u = (2.0 * ((double)i + 0.5)) / (double)cam->width - 1.0;
  double v = 1.0 - (2.0 * ((double)j + 0.5)) / (double)cam->height;
  for (int a = 0; a < 3; ++a) {
    double su = u * (double)cam->right[a];
    double sv = v * (double)cam->up[a];
    if (cam->orthographic) {
      double oo = (double)cam->eye[a] + su;
      oo = oo + sv;
      o[a] = (float)oo;
      d[a] = cam->forward[a];
    } else {
      double dd = (double)cam->forward[a] + su;
      dd = dd + sv;
      o[a] = cam->eye[a];
      d[a] = (float)dd;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Section "Line Raycasting": the ray walks the grid from voxel face to voxel
 * face (3D-DDA). After clipping the ray to the grid box, the next crossing of
 * each axis is t_a = (plane_a - o_a) * (1 / d_a) in fp64, recomputed from the
 * plane at every step; the smallest wins, ties go to the lowest axis. */
typedef struct {
  int ok;
  int32_t cell[3];
  int step[3];
  double inv[3], tnext[3], t0, o[3];
  int32_t R[3];
} dda_state;

static void dda_init(dda_state* s, const int32_t grid[3], const double of[3], const double df[3]) {
  double tn = 0.0, tf = INFINITY;
  s->ok = 0;
  if (df[0] == 0.0 && df[1] == 0.0 && df[2] == 0.0) return;
  for (int a = 0; a < 3; ++a) {
    s->R[a] = grid[a];
    s->o[a] = of[a];
    double d = df[a];
    /* an axis whose 1/d overflows is treated as parallel to the ray */
    if (d != 0.0 && !isinf(1.0 / d)) {
      s->inv[a] = 1.0 / d;
      double ta = (0.0 - s->o[a]) * s->inv[a];
      double tb = ((double)grid[a] - s->o[a]) * s->inv[a];
      double lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
      if (lo > tn) tn = lo;
      if (hi < tf) tf = hi;
      s->step[a] = d > 0 ? 1 : -1;
    } else {
      s->inv[a] = 0.0;
      s->step[a] = 0;
      if (!(s->o[a] >= 0.0 && s->o[a] < (double)grid[a])) return;
    }
  }
  if (!(tn < tf)) return;
  for (int a = 0; a < 3; ++a) {
    double p = df[a] * tn;
    p = s->o[a] + p;
    double fl = floor(p);
    int64_t c = (int64_t)fl;
    if (c < 0) c = 0;
    if (c > grid[a] - 1) c = grid[a] - 1;
    s->cell[a] = (int32_t)c;
    if (s->step[a] > 0) s->tnext[a] = ((double)(c + 1) - s->o[a]) * s->inv[a];
    else if (s->step[a] < 0) s->tnext[a] = ((double)c - s->o[a]) * s->inv[a];
    else s->tnext[a] = INFINITY;
  }
  s->t0 = tn;
  s->ok = 1;
}

/* Returns the current voxel and its [t0, t1); advances. 0 when done. */
static int dda_next(dda_state* s, int32_t cell[3], double* t0, double* t1) {
  if (!s->ok) return 0;
  int a = 0;
  if (s->tnext[1] < s->tnext[a]) a = 1;
  if (s->tnext[2] < s->tnext[a]) a = 2;
  cell[0] = s->cell[0];
  cell[1] = s->cell[1];
  cell[2] = s->cell[2];
  *t0 = s->t0;
  *t1 = s->tnext[a];
  s->t0 = s->tnext[a];
  s->cell[a] += s->step[a];
  if (s->cell[a] < 0 || s->cell[a] >= s->R[a]) {
    s->ok = 0;
  } else {
    double plane = (double)(s->step[a] > 0 ? s->cell[a] + 1 : s->cell[a]);
    s->tnext[a] = (plane - s->o[a]) * s->inv[a];
  }
  return 1;
}

int64_t or_dda(const int32_t grid[3], const float o[3], const float d[3],
               int32_t* cells, double* t0, double* t1, int64_t cap) {
  dda_state s;
  double od[3] = {o[0], o[1], o[2]}, dd[3] = {d[0], d[1], d[2]};
  dda_init(&s, grid, od, dd);
  int64_t n = 0;
  int32_t c[3];
  double a, b;
  while (dda_next(&s, c, &a, &b)) {
    if (n < cap) {
      cells[3 * n + 0] = c[0];
      cells[3 * n + 1] = c[1];
      cells[3 * n + 2] = c[2];
      t0[n] = a;
      t1[n] = b;
    }
    ++n;
  }
  return n;
}

/* ------------------------------------------------------------------------ */
/* Sections "Line Raycasting" and "Ray-tube intersections": each line is a
 * tube of the user radius with spheres of the same radius at both endpoints
 * (joint spheres), i.e. the capsule {x : dist(x, segment ab) <= r}. Being
 * convex, its ray interval is [min entry, max exit] over the finite cylinder
 * and the two spheres. The normal at the entry point is the direction from
 * the closest point of the segment. */
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static int sphere_interval(const double o[3], const double d[3], const double c[3],
                           double r, double* t0, double* t1) {
  double oc[3] = {o[0] - c[0], o[1] - c[1], o[2] - c[2]};
  double A = dot3(d, d), B = dot3(oc, d), C = dot3(oc, oc) - r * r;
  double disc = B * B - A * C;
  if (disc < 0) return 0;
  double sq = sqrt(disc);
  *t0 = (-B - sq) / A;
  *t1 = (-B + sq) / A;
  return 1;
}

int or_capsule(const double o[3], const double d[3], const double a[3],
               const double b[3], double r, double* t_in, double* t_out, double n_out[3]) {
  double lo = INFINITY, hi = -INFINITY, t0, t1;
  if (sphere_interval(o, d, a, r, &t0, &t1)) { if (t0 < lo) lo = t0; if (t1 > hi) hi = t1; }
  if (sphere_interval(o, d, b, r, &t0, &t1)) { if (t0 < lo) lo = t0; if (t1 > hi) hi = t1; }
  double ba[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  double oa[3] = {o[0] - a[0], o[1] - a[1], o[2] - a[2]};
  double L2 = dot3(ba, ba);
  double dba = dot3(d, ba), oba = dot3(oa, ba);
  double dp[3], op[3];
  for (int k = 0; k < 3; ++k) {
    dp[k] = d[k] - (dba / L2) * ba[k];
    op[k] = oa[k] - (oba / L2) * ba[k];
  }
  double A = dot3(dp, dp);
  if (A > 0) {
    double B = dot3(op, dp), C = dot3(op, op) - r * r;
    double disc = B * B - A * C;
    if (disc >= 0) {
      double sq = sqrt(disc);
      double c0 = (-B - sq) / A, c1 = (-B + sq) / A;
      double s0, s1;
      if (dba != 0) {
        s0 = (0.0 - oba) / dba;
        s1 = (L2 - oba) / dba;
        if (s0 > s1) { double tt = s0; s0 = s1; s1 = tt; }
      } else if (oba >= 0 && oba <= L2) {
        s0 = -INFINITY;
        s1 = INFINITY;
      } else {
        s0 = INFINITY;
        s1 = -INFINITY;
      }
      double e0 = c0 > s0 ? c0 : s0, e1 = c1 < s1 ? c1 : s1;
      if (e0 <= e1) { if (e0 < lo) lo = e0; if (e1 > hi) hi = e1; }
    }
  }
  if (!(lo <= hi)) return 0;
  *t_in = lo;
  *t_out = hi;
  if (n_out) {
    double P[3] = {o[0] + lo * d[0], o[1] + lo * d[1], o[2] + lo * d[2]};
    double pa[3] = {P[0] - a[0], P[1] - a[1], P[2] - a[2]};
    double u = dot3(pa, ba) / L2;
    if (u < 0) u = 0;
    if (u > 1) u = 1;
    double nn[3] = {P[0] - (a[0] + u * ba[0]), P[1] - (a[1] + u * ba[1]), P[2] - (a[2] + u * ba[2])};
    double l = sqrt(dot3(nn, nn));
    for (int k = 0; k < 3; ++k) n_out[k] = l > 0 ? nn[k] / l : 0.0;
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Section "LoD construction", representative lines. Every voxel gets one
 * average line: the start points and the end points of its lines are
 * averaged separately, a line being flipped first when it makes an angle of
 * more than 90 degrees with the line taken before it (list order, that line
 * as possibly flipped); each of the two averages is snapped to the closest
 * bin centre on the voxel's boundary. Then representative lines of two
 * face-adjacent voxels that both end on their common face are joined: both
 * endpoints move to the bin holding the mean of the two points. Coarser
 * levels average the joined lines of the (up to 8) children the same way, in
 * the parent's frame, and join again.
 *
 * Readings: the angle test is a negative dot product of the two direction
 * vectors; a voxel whose two endpoints lie on one face is not joined, nor is
 * a neighbour whose two endpoints lie on the common face; children are taken
 * in order x fastest, then y, then z; a bin boundary belongs to the upper
 * bin (as in the voxelizer). The representative line of level l has radius
 * (tube radius) * 2^l in finest-voxel units: the same radius in its own
 * level's voxel units.
 *
 * Exact integer arithmetic: a point of a voxel is held in units of 1/(4N) of
 * its side (a bin centre is 4k + 2, a face plane 0 or 4N; a child's bin
 * centre is an integer of the parent), sums of points in int64, squared
 * distances scaled by n^2 in 128-bit integers. A line's code is the record
 * layout's low 30 bits (start = entry, end = exit); voxels without lines hold
 * 0xFFFFFFFF. */
#define OR_REP_NONE 0xFFFFFFFFu

static void face_axes(int face, int* axis, int* ua, int* wa) {
  *axis = face >> 1;
  *ua = (*axis == 0) ? 1 : 0;
  *wa = (*axis == 2) ? 1 : 2;
}

/* bin centre of a 15-bit endpoint code, in units of 1/(4N) of its voxel */
static void end_units(uint32_t code, int32_t bins, int64_t p[3]) {
  int axis, ua, wa;
  int face = (int)(code & 7u);
  face_axes(face, &axis, &ua, &wa);
  p[axis] = (face & 1) ? 4 * (int64_t)bins : 0;
  p[ua] = 4 * (int64_t)((code >> 3) & 63u) + 2;
  p[wa] = 4 * (int64_t)((code >> 9) & 63u) + 2;
}

/* bin index k in [0, N) minimising |S - n (4k + 2)|, the lowest on ties */
static int nearest_bin(int64_t S, int64_t n, int32_t bins, __int128* d2) {
  int best = 0;
  __int128 bd = -1;
  for (int k = 0; k < bins; ++k) {
    __int128 d = (__int128)S - (__int128)n * (4 * (int64_t)k + 2);
    __int128 q = d * d;
    if (bd < 0 || q < bd) {
      bd = q;
      best = k;
    }
  }
  *d2 = bd;
  return best;
}

/* Closest bin centre on the voxel boundary to the point S / n (units of
 * 1/(4N)); 15-bit endpoint code. On one face the squared distance is the
 * plane term plus one term per in-plane axis, so the face's closest centre
 * takes the closest bin on each axis; faces are compared in order, the first
 * one kept on ties. */
static uint32_t snap_point(const int64_t S[3], int64_t n, int32_t bins) {
  __int128 best = -1;
  uint32_t code = 0;
  for (int f = 0; f < 6; ++f) {
    int axis, ua, wa;
    face_axes(f, &axis, &ua, &wa);
    __int128 da = (__int128)S[axis] - (__int128)n * ((f & 1) ? 4 * (int64_t)bins : 0);
    __int128 du2, dw2;
    int bu = nearest_bin(S[ua], n, bins, &du2);
    int bw = nearest_bin(S[wa], n, bins, &dw2);
    __int128 d2 = da * da + du2 + dw2;
    if (best < 0 || d2 < best) {
      best = d2;
      code = (uint32_t)f | ((uint32_t)bu << 3) | ((uint32_t)bw << 9);
    }
  }
  return code;
}

typedef struct {
  int64_t S[3], E[3], prev[3];
  int64_t n;
} rep_acc;

static void rep_add(rep_acc* r, const int64_t a_in[3], const int64_t b_in[3]) {
  int64_t a[3], b[3], dir[3];
  for (int q = 0; q < 3; ++q) { a[q] = a_in[q]; b[q] = b_in[q]; }
  if (r->n > 0) {
    int64_t dot = 0;
    for (int q = 0; q < 3; ++q) dot += (b[q] - a[q]) * r->prev[q];
    if (dot < 0) {
      for (int q = 0; q < 3; ++q) { int64_t t = a[q]; a[q] = b[q]; b[q] = t; }
    }
  }
  for (int q = 0; q < 3; ++q) {
    dir[q] = b[q] - a[q];
    r->S[q] += a[q];
    r->E[q] += b[q];
    r->prev[q] = dir[q];
  }
  r->n++;
}

static uint32_t rep_code(const rep_acc* r, int32_t bins) {
  if (r->n == 0) return OR_REP_NONE;
  uint32_t s = snap_point(r->S, r->n, bins);
  uint32_t e = snap_point(r->E, r->n, bins);
  return s | (e << 15);
}

/* Joins representative lines across shared faces (pre -> out, one level). */
static void rep_connect(const uint32_t* pre, uint32_t* out, const int32_t dim[3]) {
  for (int32_t z = 0; z < dim[2]; ++z)
    for (int32_t y = 0; y < dim[1]; ++y)
      for (int32_t x = 0; x < dim[0]; ++x) {
        int64_t v = x + (int64_t)dim[0] * (y + (int64_t)dim[1] * z);
        uint32_t code = pre[v];
        if (code == OR_REP_NONE) {
          out[v] = code;
          continue;
        }
        uint32_t ends[2] = {code & 0x7FFFu, (code >> 15) & 0x7FFFu};
        int f0 = (int)(ends[0] & 7u), f1 = (int)(ends[1] & 7u);
        if (f0 != f1) {
          for (int e = 0; e < 2; ++e) {
            int f = (int)(ends[e] & 7u), axis = f >> 1;
            int32_t c[3] = {x, y, z};
            c[axis] += (f & 1) ? 1 : -1;
            if (c[axis] < 0 || c[axis] >= dim[axis]) continue;
            uint32_t nb = pre[c[0] + (int64_t)dim[0] * (c[1] + (int64_t)dim[1] * c[2])];
            if (nb == OR_REP_NONE) continue;
            uint32_t n0 = nb & 0x7FFFu, n1 = (nb >> 15) & 0x7FFFu;
            int g = f ^ 1;
            uint32_t other;
            if ((int)(n0 & 7u) == g && (int)(n1 & 7u) != g) other = n0;
            else if ((int)(n1 & 7u) == g && (int)(n0 & 7u) != g) other = n1;
            else continue;
            uint32_t bu = (((ends[e] >> 3) & 63u) + ((other >> 3) & 63u) + 1u) >> 1;
            uint32_t bw = (((ends[e] >> 9) & 63u) + ((other >> 9) & 63u) + 1u) >> 1;
            ends[e] = (uint32_t)f | (bu << 3) | (bw << 9);
          }
        }
        out[v] = ends[0] | (ends[1] << 15);
      }
}

int or_rep_lines(const uint32_t* offsets, const uint64_t* records, const int32_t grid[3],
                 int32_t bins, uint32_t* rep) {
  int32_t dims[96];
  int64_t loff[33];
  int nl = or_lod_levels(grid, dims, loff);
  uint32_t* pre = (uint32_t*)malloc((size_t)loff[1] * sizeof(uint32_t));
  if (!pre) return -2;
  /* level 0 from the voxels' line lists */
  int64_t nvox = loff[1];
  for (int64_t v = 0; v < nvox; ++v) {
    rep_acc r;
    memset(&r, 0, sizeof(r));
    for (uint32_t k = offsets[v]; k < offsets[v + 1]; ++k) {
      int64_t a[3], b[3];
      end_units((uint32_t)(records[k] & 0x7FFFu), bins, a);
      end_units((uint32_t)((records[k] >> 15) & 0x7FFFu), bins, b);
      rep_add(&r, a, b);
    }
    pre[v] = rep_code(&r, bins);
  }
  rep_connect(pre, rep, dims);
  /* coarser levels from the joined lines of the children */
  for (int lv = 1; lv < nl; ++lv) {
    const int32_t* dc = dims + 3 * (lv - 1);
    const int32_t* dp = dims + 3 * lv;
    for (int32_t z = 0; z < dp[2]; ++z)
      for (int32_t y = 0; y < dp[1]; ++y)
        for (int32_t x = 0; x < dp[0]; ++x) {
          rep_acc r;
          memset(&r, 0, sizeof(r));
          for (int k = 0; k < 8; ++k) {
            int32_t off[3] = {k & 1, (k >> 1) & 1, k >> 2};
            int32_t cx = 2 * x + off[0], cy = 2 * y + off[1], cz = 2 * z + off[2];
            if (cx >= dc[0] || cy >= dc[1] || cz >= dc[2]) continue;
            uint32_t cc = rep[loff[lv - 1] + cx + (int64_t)dc[0] * (cy + (int64_t)dc[1] * cz)];
            if (cc == OR_REP_NONE) continue;
            int64_t a[3], b[3];
            end_units(cc & 0x7FFFu, bins, a);
            end_units((cc >> 15) & 0x7FFFu, bins, b);
            /* child units 1/(4N) of the child = 1/(8N) of the parent: halve
             * (bin centres and planes are even) and add the child's offset */
            for (int q = 0; q < 3; ++q) {
              a[q] = a[q] / 2 + (int64_t)off[q] * 2 * bins;
              b[q] = b[q] / 2 + (int64_t)off[q] * 2 * bins;
            }
            rep_add(&r, a, b);
          }
          pre[x + (int64_t)dp[0] * (y + (int64_t)dp[1] * z)] = rep_code(&r, bins);
        }
    rep_connect(pre, rep + loff[lv], dp);
  }
  free(pre);
  return nl;
}

/* Section "Shadow simulation", first approach: a shadow ray from the point x
 * (finest-voxel units) towards the light walks the voxels of level `level`
 * and is tested against each voxel's representative line, a tube of radius
 * `radius` in that level's voxel units (so thicker than the lines it stands
 * for). Returns 1 when the ray enters one of them at a positive distance (a
 * line the point already lies inside does not shadow it), else 0. */
int or_rep_shadow(const uint32_t* rep, const int32_t grid[3], int32_t bins, int32_t level,
                  double radius, const double x[3], const double light[3]) {
  int32_t dims[96];
  int64_t loff[33];
  int nl = or_lod_levels(grid, dims, loff);
  if (level < 0 || level >= nl) return 0;
  const int32_t* dm = dims + 3 * level;
  double scale = ldexp(1.0, -level);
  double o[3] = {x[0] * scale, x[1] * scale, x[2] * scale};
  double d[3] = {light[0], light[1], light[2]};
  dda_state s;
  dda_init(&s, dm, o, d);
  int32_t cell[3];
  double t0, t1;
  while (dda_next(&s, cell, &t0, &t1)) {
    uint32_t code = rep[loff[level] + cell[0] + (int64_t)dm[0] * (cell[1] + (int64_t)dm[1] * cell[2])];
    if (code == OR_REP_NONE) continue;
    double A[3], B[3];
    decode_code(code & 0x7FFFu, bins, A);
    decode_code((code >> 15) & 0x7FFFu, bins, B);
    for (int q = 0; q < 3; ++q) { A[q] += cell[q]; B[q] += cell[q]; }
    double ti, to;
    if (or_capsule(o, d, A, B, radius, &ti, &to, NULL) && ti > 0.0) return 1;
  }
  return 0;
}

/* Section "Ambient occlusion", first approach: from a visible point, rays
 * into the hemisphere around the surface normal sample the finest density
 * level (trilinear), one sample per voxel of distance, accumulating until the
 * density reaches 1 or the ray passes the radius of influence or leaves the
 * grid; the occlusion is averaged over the rays. Directions (reading): k
 * points of equal area, heights z_i = 1 - (i + 0.5)/k over the hemisphere,
 * azimuths i times the golden angle pi (3 - sqrt 5), in the orthonormal frame
 * (t1, t2, n) of Duff et al., "Building an Orthonormal Basis, Revisited"
 * (JCGT 2017), with the sign taken as +1 for n_z >= 0. */
void or_hemi_dirs(const double n[3], int32_t k, double* dirs) {
  double sgn = n[2] >= 0.0 ? 1.0 : -1.0;
  double a = -1.0 / (sgn + n[2]);
  double b = n[0] * n[1] * a;
  double t1[3] = {1.0 + sgn * n[0] * n[0] * a, sgn * b, -sgn * n[0]};
  double t2[3] = {b, sgn + n[1] * n[1] * a, -n[1]};
  double ga = 3.14159265358979323846 * (3.0 - sqrt(5.0));
  for (int32_t i = 0; i < k; ++i) {
    double z = 1.0 - ((double)i + 0.5) / (double)k;
    double r = sqrt(1.0 - z * z);
    double ph = ga * (double)i;
    double cx = r * cos(ph), cy = r * sin(ph);
    for (int q = 0; q < 3; ++q) dirs[3 * i + q] = cx * t1[q] + cy * t2[q] + z * n[q];
  }
}

double or_ao_hemi(const double* rho, const int32_t grid[3], const double x[3],
                  const double n[3], int32_t k, double radius) {
  double dirs[3 * 256];
  if (k < 1 || k > 256) return 1.0;
  or_hemi_dirs(n, k, dirs);
  double sum = 0.0;
  for (int32_t i = 0; i < k; ++i) sum += or_cone(rho, grid, x, dirs + 3 * i, radius, 0.0);
  return 1.0 - sum / (double)k;
}

/* ------------------------------------------------------------------------ */
/* Rendering (sections "Line Raycasting", "Rendering effects", "Transparency
 * rendering"). Per visited voxel: test the candidate lines, sort the accepted
 * hits by (entry t, record index), then per hit in that order: per-curve
 * interval merge (a hit whose entry lies inside the still-open interval of
 * the same curve extends it and is not blended again, the reading used for
 * the joint-sphere de-duplication), shading at the entry point, front-to-back
 * premultiplied compositing, and termination once the accumulated opacity
 * reaches the threshold (opaque lines: the first hit). */

typedef struct {
  double t_in, t_out;
  uint32_t idx;
  double n[3];
  double x[3];
  int32_t cell[3];   /* the voxel owning the line */
} or_hit;

static int cmp_hit(const void* pa, const void* pb) {
  const or_hit* a = (const or_hit*)pa;
  const or_hit* b = (const or_hit*)pb;
  if (a->t_in < b->t_in) return -1;
  if (a->t_in > b->t_in) return 1;
  return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

static double trilinear_grid(const double* g, const int32_t grid[3], const double x[3]) {
  return sample_level(g, grid, 0, x);
}

/* Section "Transparency rendering", opacity acceleration (after Danskin and
 * Hanrahan): once the accumulated optical depth -ln(1 - A) has reached
 * accel_depth, the ray leaves the lines at the end of the voxel holding that
 * fragment and continues on the density pyramid: with the optical depth
 * delta, the level is l = min(top, 1 + floor(log2(delta / accel_depth))) and
 * the step D = 2^l voxels (both grow with the depth); each step samples
 * level l at its midpoint (trilinear), takes the opacity min(1, rho D) (the
 * density as blocking per unit length, as in the cone tracer) and the
 * density-weighted mean colour rgb / rho, unlit, and composites them front to
 * back, until A reaches alpha_stop or the midpoint leaves the grid. The
 * image then differs from the exact one by at most 1 - (1 - e^-accel_depth)
 * per channel (what remains after the switch). */
static void accel_phase(const double* rho, const double* rgb, const int32_t grid[3],
                        const double o[3], const double d[3], double t_start, double depth0,
                        double alpha_stop, double C[3], double* Acc) {
  int32_t dims[96];
  int64_t loff[33];
  int nl = or_lod_levels(grid, dims, loff);
  int top = nl - 1;
  double dl = sqrt(dot3(d, d));
  double u[3] = {d[0] / dl, d[1] / dl, d[2] / dl};
  double s = t_start * dl;
  while (*Acc < alpha_stop) {
    double delta = -log(1.0 - *Acc);
    int lv = 1 + (int)floor(log2(delta / depth0));
    if (lv < 1) lv = 1;
    if (lv > top) lv = top;
    double D = ldexp(1.0, lv);
    double x[3];
    int inside = 1;
    for (int a = 0; a < 3; ++a) {
      x[a] = o[a] + (s + 0.5 * D) * u[a];
      if (!(x[a] >= 0.0 && x[a] < (double)grid[a])) inside = 0;
    }
    if (!inside) break;
    double r = sample_level(rho + loff[lv], dims + 3 * lv, lv, x);
    double alpha = r * D;
    if (alpha > 1.0) alpha = 1.0;
    if (r > 0.0 && alpha > 0.0) {
      double w = (1.0 - *Acc) * alpha;
      for (int q = 0; q < 3; ++q) {
        /* the colour pyramid's channel q, sampled like rho */
        double cq = sample_level_stride(rgb + 3 * loff[lv] + q, dims + 3 * lv, lv, x, 3) / r;
        C[q] += w * cq;
      }
      *Acc += w;
    }
    s += D;
  }
}

typedef struct {
  const uint32_t* offsets;
  const uint64_t* records;
  const int32_t* grid;
  int32_t bins;
  const or_camera* cam;
  const or_params* p;
  const double* ao;
  const double* sh;
} rctx;

typedef struct {
  uint32_t tag;
  double t_out;
} open_iv;

static void test_list(const rctx* c, int64_t vox, const int32_t cell[3], const double o[3],
                      const double d[3], int exact, double t0, double t1,
                      or_hit** hits, int64_t* nh, int64_t* cap, or_counters* k) {
  for (uint32_t r = c->offsets[vox]; r < c->offsets[vox + 1]; ++r) {
    double ea[3], eb[3], A[3], B[3];
    or_decode(c->records[r], c->bins, ea, eb);
    for (int q = 0; q < 3; ++q) { A[q] = cell[q] + ea[q]; B[q] = cell[q] + eb[q]; }
    k->tested++;
    double ti, to, n[3];
    if (!or_capsule(o, d, A, B, (double)c->p->radius, &ti, &to, n)) continue;
    if (exact) { if (!(ti >= t0 && ti < t1)) continue; }
    else if (!(ti >= 0.0)) continue;
    if (*nh == *cap) {
      *cap = *cap ? 2 * *cap : 16;
      *hits = (or_hit*)realloc(*hits, (size_t)*cap * sizeof(or_hit));
    }
    or_hit* h = *hits + (*nh)++;
    h->t_in = ti;
    h->t_out = to;
    h->idx = r;
    for (int q = 0; q < 3; ++q) { h->n[q] = n[q]; h->x[q] = o[q] + ti * d[q]; h->cell[q] = cell[q]; }
  }
}

static void render_pixel(const rctx* c, int32_t i, int32_t j, double out[4], or_counters* k) {
  const or_params* p = c->p;
  float of[3], df[3];
  or_ray(c->cam, i, j, of, df);
  double o[3] = {of[0], of[1], of[2]}, d[3] = {df[0], df[1], df[2]};
  double dl = sqrt(dot3(d, d));
  double v[3] = {-d[0] / dl, -d[1] / dl, -d[2] / dl};
  double L[3] = {p->light_dir[0], p->light_dir[1], p->light_dir[2]};
  double h[3] = {L[0] + v[0], L[1] + v[1], L[2] + v[2]};
  double hl = sqrt(dot3(h, h));
  for (int q = 0; q < 3; ++q) h[q] = hl > 0 ? h[q] / hl : 0.0;
  double C[3] = {0, 0, 0}, Acc = 0;
  or_hit* hits = NULL;
  int64_t cap = 0;
  open_iv* open = NULL;
  int64_t n_open = 0, cap_open = 0;
  dda_state s;
  dda_init(&s, c->grid, o, d);
  int32_t cell[3];
  double t0, t1;
  int done = 0, switched = 0;
  double t_switch = 0.0;
  const double accel_A0 = p->accel_depth > 0.0f ? 1.0 - exp(-(double)p->accel_depth) : 2.0;
  const int32_t* G = c->grid;
  while (!done && dda_next(&s, cell, &t0, &t1)) {
    k->visited++;
    int64_t vox = cell[0] + (int64_t)G[0] * (cell[1] + (int64_t)G[1] * cell[2]);
    if (c->offsets[vox + 1] > c->offsets[vox]) k->nonempty++;
    int64_t nh = 0;
    if (p->mode == 0) {
      test_list(c, vox, cell, o, d, 0, t0, t1, &hits, &nh, &cap, k);
    } else {
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            int32_t nc[3] = {cell[0] + dx, cell[1] + dy, cell[2] + dz};
            if (nc[0] < 0 || nc[1] < 0 || nc[2] < 0 || nc[0] >= G[0] || nc[1] >= G[1] || nc[2] >= G[2])
              continue;
            int64_t nv = nc[0] + (int64_t)G[0] * (nc[1] + (int64_t)G[1] * nc[2]);
            test_list(c, nv, nc, o, d, 1, t0, t1, &hits, &nh, &cap, k);
          }
    }
    if (nh == 0) continue;
    k->hits += nh;
    qsort(hits, (size_t)nh, sizeof(or_hit), cmp_hit);
    for (int64_t m = 0; m < nh && !done; ++m) {
      const or_hit* H = hits + m;
      uint64_t rec = c->records[H->idx];
      uint32_t tag = (uint32_t)(rec >> 40);
      int attr = (int)((rec >> 32) & 0xFF);
      if (!p->opaque && p->merge_curves) {
        int64_t f = -1;
        for (int64_t q = 0; q < n_open; ++q) if (open[q].tag == tag) { f = q; break; }
        if (f >= 0 && H->t_in <= open[f].t_out) {
          if (H->t_out > open[f].t_out) open[f].t_out = H->t_out;
          continue;
        }
        if (f >= 0) {
          open[f].t_out = H->t_out;
        } else {
          if (n_open == cap_open) {
            cap_open = cap_open ? 2 * cap_open : 16;
            open = (open_iv*)realloc(open, (size_t)cap_open * sizeof(open_iv));
          }
          open[n_open].tag = tag;
          open[n_open].t_out = H->t_out;
          n_open++;
        }
      }
      const float* lut = p->lut_rgba + 4 * attr;
      double base[3] = {lut[0], lut[1], lut[2]};
      double alpha = p->opaque ? 1.0 : (double)lut[3];
      if (p->ends) {
        /* Attributes interpolated along the line: the endpoint attributes
         * taken linearly at the segment point closest to the entry point
         * (clamped to the segment), and the transfer function read linearly
         * between its two neighbouring entries. */
        double ea[3], eb[3], A[3], B[3];
        or_decode(rec, c->bins, ea, eb);
        for (int q = 0; q < 3; ++q) { A[q] = H->cell[q] + ea[q]; B[q] = H->cell[q] + eb[q]; }
        double ba[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        double pa[3] = {H->x[0] - A[0], H->x[1] - A[1], H->x[2] - A[2]};
        double u = dot3(pa, ba) / dot3(ba, ba);
        if (u < 0) u = 0;
        if (u > 1) u = 1;
        uint16_t en = p->ends[H->idx];
        double a0 = (double)(en & 0xFF), a1 = (double)(en >> 8);
        double af = a0 + u * (a1 - a0);
        int i0 = (int)floor(af);
        if (i0 > 255) i0 = 255;
        int i1 = i0 < 255 ? i0 + 1 : 255;
        double f = af - (double)i0;
        const float* l0 = p->lut_rgba + 4 * i0;
        const float* l1 = p->lut_rgba + 4 * i1;
        for (int q = 0; q < 3; ++q) base[q] = (1.0 - f) * (double)l0[q] + f * (double)l1[q];
        if (!p->opaque) alpha = (1.0 - f) * (double)l0[3] + f * (double)l1[3];
      }
      if (!p->opaque && p->distance_alpha) {
        /* Section "Transparency rendering": opacity dependent on the distance
         * travelled inside the tube. Reading: the transfer function's alpha
         * is that of a chord of one diameter (2r); a chord of length l has
         * 1 - (1 - alpha)^(l / 2r), the Beer-Lambert law for a uniform
         * medium. l is the chord of this (composited) hit. */
        double chord = (H->t_out - H->t_in) * dl;
        alpha = 1.0 - pow(1.0 - alpha, chord / (2.0 * (double)p->radius));
      }
      double col[3];
      if (p->shading == 0) {
        for (int q = 0; q < 3; ++q) col[q] = base[q];
      } else if (p->shading == 1) {
        double ndv = fabs(dot3(H->n, v));
        double spec = (double)p->ks * pow(ndv, (double)p->shininess);
        for (int q = 0; q < 3; ++q) col[q] = base[q] * ((double)p->ka + (double)p->kd * ndv) + spec;
      } else {
        double aov, shv;
        if (p->ao_mode == 1)
          aov = or_ao_hemi(p->rho, G, H->x, H->n, p->ao_rays, (double)p->ao_radius);
        else
          aov = trilinear_grid(c->ao, G, H->x);
        if (p->shadow_mode == 1)
          shv = 1.0 - or_cone(p->rho, G, H->x, L, INFINITY, 1.0);
        else if (p->shadow_mode == 2)
          shv = or_rep_shadow(p->rep, G, c->bins, p->rep_level, (double)p->radius, H->x, L) ? 0.0 : 1.0;
        else
          shv = trilinear_grid(c->sh, G, H->x);
        double ndl = dot3(H->n, L);
        if (ndl < 0) ndl = 0;
        double ndh = dot3(H->n, h);
        if (ndh < 0) ndh = 0;
        double spec = (double)p->ks * shv * pow(ndh, (double)p->shininess);
        for (int q = 0; q < 3; ++q)
          col[q] = base[q] * ((double)p->ka * aov + (double)p->kd * shv * ndl) + spec;
      }
      double w = (1.0 - Acc) * alpha;
      for (int q = 0; q < 3; ++q) C[q] += w * col[q];
      Acc += w;
      k->fragments++;
      if (Acc >= (double)p->alpha_stop) {
        done = 1;
      } else if (Acc >= accel_A0) {
        done = 1;
        switched = 1;
        t_switch = t1;
      }
    }
  }
  if (switched)
    accel_phase(p->rho, p->rgb, G, o, d, t_switch, (double)p->accel_depth,
                (double)p->alpha_stop, C, &Acc);
  free(hits);
  free(open);
  out[0] = C[0];
  out[1] = C[1];
  out[2] = C[2];
  out[3] = Acc;
}

int or_render(const uint32_t* offsets, const uint64_t* records, const int32_t grid[3],
              int32_t bins, const or_camera* cam, const or_params* p, const double* ao,
              const double* sh, const int64_t* pixels, int64_t n_pixels, double* rgba,
              or_counters* counters, int32_t n_threads) {
  rctx c = {offsets, records, grid, bins, cam, p, ao, sh};
  if (p->shading == 2) {
    if (p->ao_mode == 0 && !ao) return -1;
    if (p->shadow_mode == 0 && !sh) return -1;
    if ((p->ao_mode == 1 || p->shadow_mode == 1) && !p->rho) return -1;
    if (p->shadow_mode == 2 && !p->rep) return -1;
    if (p->ao_mode == 1 && p->ao_rays < 1) return -1;
  }
  if (p->accel_depth > 0.0f && (!p->rho || !p->rgb)) return -1;
  int64_t W = cam->width, H = cam->height;
  int64_t n = pixels ? n_pixels : W * H;
  int64_t kv = 0, kn = 0, kt = 0, kh = 0, kf = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : kv, kn, kt, kh, kf)
#endif
  for (int64_t m = 0; m < n; ++m) {
    int64_t pix = pixels ? pixels[m] : m;
    or_counters k = {0, 0, 0, 0, 0};
    render_pixel(&c, (int32_t)(pix % W), (int32_t)(pix / W), rgba + 4 * m, &k);
    kv += k.visited;
    kn += k.nonempty;
    kt += k.tested;
    kh += k.hits;
    kf += k.fragments;
  }
  if (counters) {
    counters->visited = kv;
    counters->nonempty = kn;
    counters->tested = kt;
    counters->hits = kh;
    counters->fragments = kf;
  }
  return 0;
}
