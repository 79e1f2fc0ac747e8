// Ray-casting of the voxelized line set on gfx950 (sections "Line
// Raycasting", "Ray-tube intersections", "Rendering effects", "Transparency
// rendering").
//
// One ray per lane; a wave renders an 8 x 8 screen tile, so its 64 rays walk
// nearly the same voxels and their list loads coalesce in the L1/L2. The
// plain launch uses one wave per workgroup (a finished wave frees its slot
// at once; measured faster than 2 x 2-wave workgroups on dense frames).
// Workgroup b runs on XCD b mod 8, and XCD x renders tile rows x, x + 8, ...
// so neighbouring tiles share one L2 and every XCD gets part of the busy
// screen region.
//
// Per ray:
//  1. ray from the camera in fp64, rounded to fp32 (these fp32 values are the
//     ray);
//  2. clip to the grid box and walk it voxel by voxel (3D-DDA) with the
//     next crossing of each axis t = (plane - o) * (1/d) in fp64, ties to the
//     lowest axis: voxel order and [t0, t1) match the CPU oracle bit for bit;
//     an empty 4^3 macro cell (one 64-bit occupancy word) is crossed in one
//     step;
//  3. per non-empty voxel, capsule tests in fp32 in a voxel-local frame
//     (origin = ray point at t0 minus the voxel corner, formed in fp64); in
//     own-list mode the lists of all lanes that entered a non-empty voxel in
//     the same step are tested by the whole wave together (voxels_coop);
//  4. accepted hits go into a 4-slot register-resident sorted buffer keyed
//     by (entry t, record index); a voxel with more hits is swept again for
//     the next 4;
//  5. per hit in order: per-curve interval merge in an 8-entry LDS table
//     (the interval that closed first is evicted when full), shading,
//     premultiplied front-to-back compositing, termination at alpha_stop.
#include "render_args.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace {

constexpr int kBlock = 256;
constexpr int kSortSlots = 4;   // sorted hit buffer of the neighbour mode
// Split tiles of the innermost launch rings: workgroups per tile, the radius
// of the split rings as a fraction of the grid's projected radius, and the
// largest frame split, in estimated ray-records (pixels the grid covers times
// the mean records per grid column). A transparent frame below that size is
// set by the waves over the dense core (a wave's time is that of its slowest
// ray), and half as many rays per wave there shortens them; bigger or opaque
// frames are bound by total work, which splitting raises. Measured (ms,
// unsplit -> split, identical images):
//   100k x 200 lines, 256^3 (144 records per column), perspective:
//     1920x1080 1.12 -> 1.04 (AO/shadow shading 1.25 -> 1.14),
//     960x540 1.02 -> 0.79, distant view 1.04 -> 0.78,
//     but 3840x2160 1.83 -> 2.17 and opaque 1920x1080 0.36 -> 0.44;
//   1M x 100 lines, 512^3 (536 records per column):
//     960x540 1.63 -> 1.36, but 1920x1080 2.10 -> 2.18.
// The limit lies between the largest split case (1.1e8 ray-records) and the
// smallest unsplit one (4.1e8). On the first set any radius of 0.5 to 1.25
// measured the same, 0.35 and 0.25 worse than no split; on the second,
// 960x540 took 1.56 ms at 0.5 and 1.36 at 0.75-1.25.
// Frames of at most kSplit4MaxWork split four ways (two rows per
// workgroup): first set 960x540 0.78 -> 0.66 ms, distant view 0.79 -> 0.61
// (2.1e7 to 2.8e7 ray-records), while at 1.0e8 and above (first set
// 1920x1080 1.02 -> 1.21, second set 960x540 1.36 -> 1.48) two ways are
// better.
constexpr double kSplitFrac = 1.0;
constexpr double kSplitMaxWork = 2.0e8;
constexpr double kSplit4MaxWork = 5.0e7;
constexpr int kCoopSlots = 4;   // sorted hit buffer of the wave-cooperative own-list mode (8 measured slower)
// Intervals of the per-curve merge table (LDS, 12 bytes each per lane).
#ifndef LS_MERGE_SLOTS
#define LS_MERGE_SLOTS 8
#endif
constexpr int kMergeSlots = LS_MERGE_SLOTS;
constexpr int kXcds = 8;



struct Counts {
  uint32_t visited = 0, nonempty = 0, tested = 0, hits = 0, fragments = 0, passes = 0,
           evictions = 0, skips = 0, live_evictions = 0, overflow_rays = 0;
  uint32_t list_bytes = 0;
};

__device__ inline void decode_point(uint32_t code, float inv_bins, float p[3]) {
  const int face = (int)(code & 7u);
  const int axis = face >> 1;
  const float side = (float)(face & 1);
  const float u = ((float)((code >> 3) & 63u) + 0.5f) * inv_bins;
  const float w = ((float)((code >> 9) & 63u) + 0.5f) * inv_bins;
  p[0] = axis == 0 ? side : u;
  p[1] = axis == 1 ? side : (axis == 0 ? u : w);
  p[2] = axis == 2 ? side : w;
}

__device__ inline float dot3(const float a[3], const float b[3]) {
  #pragma clang fp contract(fast)
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Ray vs capsule {x : dist(x, ab) <= r}: [min entry, max exit] over the two
// spheres and the finite cylinder. q, d in the voxel-local frame.
__device__ inline bool capsule(const float q[3], const float d[3], float dd, float inv_dd,
                               const float a[3], const float b[3], float r2, float& t_in,
                               float& t_out) {
  // fp32 shading and intersection arithmetic may fuse multiply-adds (the
  // grid walk and ray set-up use explicitly rounded fp64 operations)
  #pragma clang fp contract(fast)
  float lo = INFINITY, hi = -INFINITY;
  float oa[3] = {q[0] - a[0], q[1] - a[1], q[2] - a[2]};
  float ob[3] = {q[0] - b[0], q[1] - b[1], q[2] - b[2]};
  {
    float B = dot3(oa, d), C = dot3(oa, oa) - r2;
    float disc = B * B - dd * C;
    if (disc >= 0.f) {
      float s = __builtin_sqrtf(disc);
      lo = fminf(lo, (-B - s) * inv_dd);
      hi = fmaxf(hi, (-B + s) * inv_dd);
    }
  }
  {
    float B = dot3(ob, d), C = dot3(ob, ob) - r2;
    float disc = B * B - dd * C;
    if (disc >= 0.f) {
      float s = __builtin_sqrtf(disc);
      lo = fminf(lo, (-B - s) * inv_dd);
      hi = fmaxf(hi, (-B + s) * inv_dd);
    }
  }
  float ba[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  float L2 = dot3(ba, ba);
  float iL2 = rcp(L2);
  float dba = dot3(d, ba), oba = dot3(oa, ba);
  float kd = dba * iL2, ko = oba * iL2;
  float dp[3] = {d[0] - kd * ba[0], d[1] - kd * ba[1], d[2] - kd * ba[2]};
  float op[3] = {oa[0] - ko * ba[0], oa[1] - ko * ba[1], oa[2] - ko * ba[2]};
  float A = dot3(dp, dp);
  if (A > 0.f) {
    float B = dot3(op, dp), C = dot3(op, op) - r2;
    float disc = B * B - A * C;
    if (disc >= 0.f) {
      float s = __builtin_sqrtf(disc);
      float iA = rcp(A);
      float c0 = (-B - s) * iA, c1 = (-B + s) * iA;
      float s0, s1;
      if (dba != 0.f) {
        float idba = rcp(dba);
        float u0 = -oba * idba, u1 = (L2 - oba) * idba;
        s0 = fminf(u0, u1);
        s1 = fmaxf(u0, u1);
      } else if (oba >= 0.f && oba <= L2) {
        s0 = -INFINITY;
        s1 = INFINITY;
      } else {
        s0 = INFINITY;
        s1 = -INFINITY;
      }
      float e0 = fmaxf(c0, s0), e1 = fminf(c1, s1);
      if (e0 <= e1) {
        lo = fminf(lo, e0);
        hi = fmaxf(hi, e1);
      }
    }
  }
  t_in = lo;
  t_out = hi;
  return lo <= hi;
}

// Trilinear, cell-centred, clamp-to-edge lookup of a per-voxel grid at the
// point cell + p (p local).
__device__ inline float grid_lookup(const float* grid, const int32_t g[3], const int32_t cell[3],
                                    const float p[3]) {
  #pragma clang fp contract(fast)
  int32_t i0[3], i1[3];
  float f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float x = p[a] - 0.5f;
    float fl = floorf(x);
    f[a] = x - fl;
    int32_t lo = cell[a] + (int32_t)fl;
    int32_t hi = lo + 1;
    lo = lo < 0 ? 0 : (lo > g[a] - 1 ? g[a] - 1 : lo);
    hi = hi < 0 ? 0 : (hi > g[a] - 1 ? g[a] - 1 : hi);
    i0[a] = lo;
    i1[a] = hi;
  }
  const int64_t sy = g[0], sz = (int64_t)g[0] * g[1];
  const int64_t z0 = i0[2] * sz, z1 = i1[2] * sz, y0 = i0[1] * sy, y1 = i1[1] * sy;
  float c00 = grid[i0[0] + y0 + z0] * (1.f - f[0]) + grid[i1[0] + y0 + z0] * f[0];
  float c10 = grid[i0[0] + y1 + z0] * (1.f - f[0]) + grid[i1[0] + y1 + z0] * f[0];
  float c01 = grid[i0[0] + y0 + z1] * (1.f - f[0]) + grid[i1[0] + y0 + z1] * f[0];
  float c11 = grid[i0[0] + y1 + z1] * (1.f - f[0]) + grid[i1[0] + y1 + z1] * f[0];
  float c0 = c00 * (1.f - f[1]) + c10 * f[1];
  float c1 = c01 * (1.f - f[1]) + c11 * f[1];
  return c0 * (1.f - f[2]) + c1 * f[2];
}

// Per-ray compositing state. The merge table (curve tag, end of the open
// interval) lives in dynamically sized LDS, one block per wave, slot-major
// with a stride of 64 lanes so each lane's accesses are conflict-free and
// every slot is a constant offset from one base: per thread kMergeSlots
// doubles and kMergeSlots tags (12 * kMergeSlots bytes).
constexpr int kWave = 64;

struct MergeLds {
  double* out;     // this lane's slot 0; slot k at out[k * 64]
  uint32_t* tag;   // this lane's slot 0; slot k at tag[k * 64]
};

// Per wave: [kMergeSlots][64] doubles, then [kMergeSlots][64] tags.
__device__ inline MergeLds merge_lds_view(double* base) {
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = (int)(threadIdx.x & (kWave - 1));
  double* w = base + wave * (kMergeSlots * kWave * 3 / 2);
  MergeLds m;
  m.out = w + lane;
  m.tag = reinterpret_cast<uint32_t*>(w + kMergeSlots * kWave) + lane;
  return m;
}

inline size_t merge_lds_bytes(unsigned threads) {
  return (size_t)threads * kMergeSlots * (sizeof(double) + sizeof(uint32_t));
}

struct Accum {
  float C[3] = {0.f, 0.f, 0.f};
  float A = 0.f;
  bool done = false;
  bool switched = false;   // opacity acceleration: leave the lines for the pyramid
  MergeLds mt;
  __device__ Accum(const MergeLds& m) : mt(m) {
#pragma unroll
    for (int k = 0; k < kMergeSlots; ++k) {
      mt.tag[k * kWave] = 0xFFFFFFFFu;
      mt.out[k * kWave] = -INFINITY;
    }
  }
};

// Returns true if the hit merges into an open interval of its curve.
__device__ inline bool merge_hit(Accum& acc, uint32_t tag, double t_in, double t_out,
                                 Counts& cnt) {
  const MergeLds& M = acc.mt;
  const int l = 0, st = kWave;
  int f = -1;
#pragma unroll
  for (int m = 0; m < kMergeSlots; ++m)
    if (M.tag[m * st + l] == tag) f = m;
  if (f >= 0) {
    const bool inside = t_in <= M.out[f * st + l];
    M.out[f * st + l] = inside ? fmax(M.out[f * st + l], t_out) : t_out;
    return inside;
  }
  // new curve: take an empty slot, else evict the interval that closed first
  int slot = 0;
  double best = M.out[0 * st + l];
#pragma unroll
  for (int m = 1; m < kMergeSlots; ++m) {
    const double o = M.out[m * st + l];
    if (o < best) {
      best = o;
      slot = m;
    }
  }
  if (M.tag[slot * st + l] != 0xFFFFFFFFu) {
    // an evicted interval still open at this hit's entry could have merged
    // a later hit of its curve (with hits in global t order, as in the
    // neighbour mode, one that closed before t_in never can)
    cnt.evictions++;
    if (best >= t_in) cnt.live_evictions++;
  }
  M.tag[slot * st + l] = tag;
  M.out[slot * st + l] = t_out;
  return false;
}

struct Shade {
  float v[3];   // towards the eye, unit
  float h[3];   // half vector for the directional light
  float dlen;   // |d|: ray parameter -> distance
};

// Opacity of a fragment. Constant per line, or (distance_alpha) dependent on
// the distance the ray travels inside the tube (section "Transparency
// rendering"): the LUT opacity a holds for a chord of one tube diameter, so a
// chord of length l has opacity 1 - (1 - a)^(l / 2r) (a tangent hit, l = 0,
// has none).
__device__ inline float fragment_alpha(const RenderArgs& R, float a, float chord) {
  if (R.opaque) return 1.f;
  if (!R.dist_alpha) return a;
  if (!(chord > 0.f)) return 0.f;
  if (a >= 1.f) return 1.f;
  return 1.f - __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(1.f - a) * (chord * R.inv_2r));
}

// ---------------------------------------------------------------------------
// View-dependent illumination per fragment (sections "Shadow simulation" and
// "Ambient occlusion"), used by shading 2 when ao_mode / shadow_mode select
// it. The fragment is the entry point p in the frame of voxel `cell`.

// Dimensions and flat offset of pyramid level lv (each level halves the
// sides, rounding up, down to 1^3).
__device__ inline void level_geom(const int32_t g[3], int lv, int32_t dim[3], int64_t& off) {
  dim[0] = g[0];
  dim[1] = g[1];
  dim[2] = g[2];
  off = 0;
  for (int l = 0; l < lv; ++l) {
    off += (int64_t)dim[0] * dim[1] * dim[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) dim[a] = (dim[a] + 1) >> 1;
  }
}

// Cell-centred trilinear sample, clamped to the edge, of a pyramid level at
// the point cell + q (finest-voxel units; q may reach far outside the cell).
__device__ inline float sample_level(const float* lev, const int32_t dim[3], int lv,
                                     const int32_t cell[3], const float q[3]) {
  #pragma clang fp contract(fast)
  const float scale = __builtin_ldexpf(1.0f, -lv);
  const int32_t mask = (1 << lv) - 1;
  int32_t i0[3], i1[3];
  float f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float x = ((float)(cell[a] & mask) + q[a]) * scale - 0.5f;
    const float fl = floorf(x);
    f[a] = x - fl;
    const int32_t lo = (cell[a] >> lv) + (int32_t)fl;
    i0[a] = min(max(lo, 0), dim[a] - 1);
    i1[a] = min(max(lo + 1, 0), dim[a] - 1);
  }
  const int64_t sy = dim[0], sz = (int64_t)dim[0] * dim[1];
  const int64_t z0 = i0[2] * sz, z1 = i1[2] * sz, y0 = i0[1] * sy, y1 = i1[1] * sy;
  const float c00 = lev[i0[0] + y0 + z0] * (1.f - f[0]) + lev[i1[0] + y0 + z0] * f[0];
  const float c10 = lev[i0[0] + y1 + z0] * (1.f - f[0]) + lev[i1[0] + y1 + z0] * f[0];
  const float c01 = lev[i0[0] + y0 + z1] * (1.f - f[0]) + lev[i1[0] + y0 + z1] * f[0];
  const float c11 = lev[i0[0] + y1 + z1] * (1.f - f[0]) + lev[i1[0] + y1 + z1] * f[0];
  const float c0 = c00 * (1.f - f[1]) + c10 * f[1];
  const float c1 = c01 * (1.f - f[1]) + c11 * f[1];
  return c0 * (1.f - f[2]) + c1 * f[2];
}

__device__ inline bool inside_grid(const RenderArgs& R, const int32_t cell[3], const float q[3]) {
  bool in = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) in &= q[a] >= -(float)cell[a] && q[a] < (float)(R.g[a] - cell[a]);
  return in;
}

// First AO approach: ao_rays rays about the unit normal n, directions of
// equal area (heights 1 - (i + 0.5)/k) at azimuths i * pi (3 - sqrt 5) in
// the orthonormal frame of Duff et al. ("Building an Orthonormal Basis,
// Revisited", JCGT 2017; sign +1 for n_z >= 0). Each ray samples the finest
// density level at distances s = 1, 2, ... < ao_radius, adding the sample,
// until the sum reaches 1 or the ray leaves the grid. Returns 1 - mean.
__device__ inline float hemi_ao(const RenderArgs& R, const int32_t cell[3], const float p[3],
                                const float n[3]) {
  #pragma clang fp contract(fast)
  const float sgn = n[2] >= 0.f ? 1.f : -1.f;
  const float a = -1.f / (sgn + n[2]);
  const float b = n[0] * n[1] * a;
  const float t1[3] = {1.f + sgn * n[0] * n[0] * a, sgn * b, -sgn * n[0]};
  const float t2[3] = {b, sgn + n[1] * n[1] * a, -n[1]};
  const int k = R.ao_rays;
  const float ik = 1.f / (float)k;
  float sum = 0.f;
  for (int i = 0; i < k; ++i) {
    const float z = 1.f - ((float)i + 0.5f) * ik;
    const float r = sqrtf(fmaxf(1.f - z * z, 0.f));
    // azimuth i * golden angle, reduced in fp64 so large i keeps its accuracy
    const double ph = (double)i * 2.3999632297286531;
    const float phr = (float)(ph - 6.283185307179586 * floor(ph * 0.15915494309189535));
    float sn, cs;
    sincosf(phr, &sn, &cs);
    float d[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c] = r * cs * t1[c] + r * sn * t2[c] + z * n[c];
    float occ = 0.f;
    for (float s = 1.f; s < R.ao_radius; s += 1.f) {
      float q[3] = {p[0] + s * d[0], p[1] + s * d[1], p[2] + s * d[2]};
      if (!inside_grid(R, cell, q)) break;
      occ += sample_level(R.rho, R.g, 0, cell, q);
      if (occ >= 1.f) break;
    }
    sum += fminf(occ, 1.f);
  }
  return 1.f - sum * ik;
}

// Second shadow approach at the fragment: a cone of aperture 1 towards the
// light, samples at s = 1, 2, 4, ... (diameter D = s) on level
// min(top, log2 s) weighted by D, until the sum reaches 1 or the point leaves
// the grid. Returns the occlusion (capped at 1).
__device__ inline float point_cone(const RenderArgs& R, const int32_t cell[3], const float p[3]) {
  #pragma clang fp contract(fast)
  int32_t dim[3] = {R.g[0], R.g[1], R.g[2]};
  int64_t off = 0;
  int lv = 0;
  const int top = R.n_levels - 1;
  float occ = 0.f, s = 1.f;
  for (int k = 0; k < 64; ++k) {
    const float q[3] = {p[0] + s * R.light[0], p[1] + s * R.light[1], p[2] + s * R.light[2]};
    if (!inside_grid(R, cell, q)) break;
    const int want = min(top, k);
    while (lv < want) {
      off += (int64_t)dim[0] * dim[1] * dim[2];
#pragma unroll
      for (int a = 0; a < 3; ++a) dim[a] = (dim[a] + 1) >> 1;
      ++lv;
    }
    occ += sample_level(R.rho + off, dim, lv, cell, q) * s;
    if (occ >= 1.f) break;
    s += s;
  }
  return fminf(occ, 1.f);
}

// First shadow approach: a ray from the fragment towards the light walks the
// voxels of level rep_level (the grid walk's fp64 formula, ties to the lowest
// axis) and tests each voxel's representative line, a capsule of `radius` in
// that level's voxel units. True when it enters one at a positive distance.
__device__ inline bool rep_shadow(const RenderArgs& R, const int32_t cell[3], const float p[3]) {
  const int lv = R.rep_level;
  int32_t dim[3];
  int64_t off;
  level_geom(R.g, lv, dim, off);
  const uint32_t* rep = R.rep + off;
  const double scale = ldexp(1.0, -lv);
  double o[3], d[3], inv[3], tn[3];
  int32_t c[3], st[3];
  double tnear = 0.0, tfar = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    o[a] = __dmul_rn(__dadd_rn((double)cell[a], (double)p[a]), scale);
    d[a] = (double)R.light[a];
    const double iv = __ddiv_rn(1.0, d[a]);
    if (d[a] != 0.0 && !isinf(iv)) {
      inv[a] = iv;
      const double ta = __dmul_rn(__dadd_rn(0.0, -o[a]), iv);
      const double tb = __dmul_rn(__dadd_rn((double)dim[a], -o[a]), iv);
      tnear = fmax(tnear, fmin(ta, tb));
      tfar = fmin(tfar, fmax(ta, tb));
      st[a] = d[a] > 0.0 ? 1 : -1;
    } else {
      inv[a] = 0.0;
      st[a] = 0;
      if (!(o[a] >= 0.0 && o[a] < (double)dim[a])) tfar = -INFINITY;
    }
  }
  if (!(tnear < tfar)) return false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double x = __dadd_rn(o[a], __dmul_rn(d[a], tnear));
    const double fl = floor(x);
    c[a] = fl < 0.0 ? 0 : (fl > (double)(dim[a] - 1) ? dim[a] - 1 : (int32_t)fl);
    if (st[a] > 0) tn[a] = __dmul_rn(__dadd_rn((double)(c[a] + 1), -o[a]), inv[a]);
    else if (st[a] < 0) tn[a] = __dmul_rn(__dadd_rn((double)c[a], -o[a]), inv[a]);
    else tn[a] = INFINITY;
  }
  const float Lf[3] = {R.light[0], R.light[1], R.light[2]};
  const float dd = dot3(Lf, Lf), inv_dd = 1.f / dd;
  double t0 = tnear;
  const int max_steps = dim[0] + dim[1] + dim[2] + 3;
  for (int it = 0; it < max_steps; ++it) {
    const uint32_t code = rep[c[0] + (int64_t)dim[0] * (c[1] + (int64_t)dim[1] * c[2])];
    if (code != 0xFFFFFFFFu) {
      float a[3], b[3], q[3];
      decode_point(code & 0x7FFFu, R.inv_bins, a);
      decode_point((code >> 15) & 0x7FFFu, R.inv_bins, b);
#pragma unroll
      for (int k = 0; k < 3; ++k) q[k] = (float)__dadd_rn(__dadd_rn(o[k], __dmul_rn(d[k], t0)), -(double)c[k]);
      float si, so;
      if (capsule(q, Lf, dd, inv_dd, a, b, R.r2, si, so) && t0 + (double)si > 0.0) return true;
    }
    int ax = 0;
    if (tn[1] < tn[ax]) ax = 1;
    if (tn[2] < tn[ax]) ax = 2;
    t0 = tn[ax];
    c[ax] += st[ax];
    if (c[ax] < 0 || c[ax] >= dim[ax]) break;
    const double plane = (double)(st[ax] > 0 ? c[ax] + 1 : c[ax]);
    tn[ax] = __dmul_rn(__dadd_rn(plane, -o[ax]), inv[ax]);
  }
  return false;
}

// Colour pyramid sample (three interleaved floats per cell), as sample_level.
__device__ inline void sample_level3(const float* lev, const int32_t dim[3], int lv,
                                     const int32_t cell[3], const float q[3], float out[3]) {
  #pragma clang fp contract(fast)
  const float scale = __builtin_ldexpf(1.0f, -lv);
  const int32_t mask = (1 << lv) - 1;
  int32_t i0[3], i1[3];
  float f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float x = ((float)(cell[a] & mask) + q[a]) * scale - 0.5f;
    const float fl = floorf(x);
    f[a] = x - fl;
    const int32_t lo = (cell[a] >> lv) + (int32_t)fl;
    i0[a] = min(max(lo, 0), dim[a] - 1);
    i1[a] = min(max(lo + 1, 0), dim[a] - 1);
  }
  const int64_t sy = dim[0], sz = (int64_t)dim[0] * dim[1];
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c] = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int bx = k & 1, by = (k >> 1) & 1, bz = k >> 2;
    const float w = (bx ? f[0] : 1.f - f[0]) * (by ? f[1] : 1.f - f[1]) * (bz ? f[2] : 1.f - f[2]);
    const int64_t i = (bx ? i1[0] : i0[0]) + (by ? i1[1] : i0[1]) * sy + (bz ? i1[2] : i0[2]) * sz;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] += w * lev[3 * i + c];
  }
}

// Shade and composite one fragment. p is the entry point in the frame of
// `cell`, a/b the record's endpoints in the same frame, dt the ray-parameter
// length of the hit (exit - entry).
// Transfer function at the line attribute interpolated along the line (the
// record's endpoint attributes taken linearly at the segment point closest
// to p), read linearly between its two neighbouring entries.
__device__ inline float4 lut_along(const float4* lut_lds, uint32_t en, const float p[3],
                                   const float a[3], const float b[3]) {
  #pragma clang fp contract(fast)
  const float ba[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  const float pa[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
  const float u = fminf(fmaxf(dot3(pa, ba) / dot3(ba, ba), 0.f), 1.f);
  const float e = (float)(en & 0xFFu), x = (float)(en >> 8);
  const float af = e + u * (x - e);
  const int i0 = min((int)floorf(af), 255), i1 = min(i0 + 1, 255);
  const float f = af - (float)i0;
  const float4 l0 = lut_lds[i0], l1 = lut_lds[i1];
  return make_float4(l0.x + f * (l1.x - l0.x), l0.y + f * (l1.y - l0.y), l0.z + f * (l1.z - l0.z),
                     l0.w + f * (l1.w - l0.w));
}

template <bool kVdi>
__device__ __attribute__((always_inline)) inline void composite(const RenderArgs& R, const float4* lut_lds, const Shade& S, Accum& acc, uint64_t rec,
                                 uint32_t k, const int32_t cell[3], const float p[3],
                                 const float a[3], const float b[3], float dt, Counts& cnt) {
  #pragma clang fp contract(fast)
  const int attr = (int)((rec >> 32) & 0xFF);
  const float4 lut = (kVdi && R.ends) ? lut_along(lut_lds, R.ends[k], p, a, b) : lut_lds[attr];
  const float alpha = fragment_alpha(R, lut.w, dt * S.dlen);
  float col[3] = {lut.x, lut.y, lut.z};
  if (R.shading != 0) {
    float ba[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    float pa[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    float u = dot3(pa, ba) * rcp(dot3(ba, ba));
    u = fminf(fmaxf(u, 0.f), 1.f);
    float n[3] = {pa[0] - u * ba[0], pa[1] - u * ba[1], pa[2] - u * ba[2]};
    float nl = dot3(n, n);
    float inl = nl > 0.f ? __builtin_amdgcn_rsqf(nl) : 0.f;
    n[0] *= inl;
    n[1] *= inl;
    n[2] *= inl;
    if (R.shading == 1) {
      float ndv = fabsf(dot3(n, S.v));
      float spec = R.ks * __builtin_amdgcn_exp2f(R.shin * __builtin_amdgcn_logf(ndv));
      spec = ndv > 0.f ? spec : 0.f;
      float diff = R.ka + R.kd * ndv;
#pragma unroll
      for (int c = 0; c < 3; ++c) col[c] = col[c] * diff + spec;
    } else {
      float aov, shv;
      if (kVdi && R.ao_mode == 1) aov = hemi_ao(R, cell, p, n);
      else aov = grid_lookup(R.ao, R.g, cell, p);
      if (kVdi && R.shadow_mode == 1) shv = 1.f - point_cone(R, cell, p);
      else if (kVdi && R.shadow_mode == 2) shv = rep_shadow(R, cell, p) ? 0.f : 1.f;
      else shv = grid_lookup(R.sh, R.g, cell, p);
      float ndl = fmaxf(dot3(n, R.light), 0.f);
      float ndh = fmaxf(dot3(n, S.h), 0.f);
      float spec = R.ks * shv * __builtin_amdgcn_exp2f(R.shin * __builtin_amdgcn_logf(ndh));
      spec = ndh > 0.f ? spec : 0.f;
      float diff = R.ka * aov + R.kd * shv * ndl;
#pragma unroll
      for (int c = 0; c < 3; ++c) col[c] = col[c] * diff + spec;
    }
  }
  const float w = (1.f - acc.A) * alpha;
  acc.C[0] += w * col[0];
  acc.C[1] += w * col[1];
  acc.C[2] += w * col[2];
  acc.A += w;
  cnt.fragments++;
  if (acc.A >= R.alpha_stop) {
    acc.done = true;
  } else if (kVdi && acc.A >= R.accel_A0) {
    acc.done = true;
    acc.switched = true;
  }
}

// Sorted register buffer of hits. Key (t, idx) lexicographic.
template <typename TKey, int K = kSortSlots>
struct HitBuf {
  TKey t[K];
  float so[K];
  uint32_t idx[K];
  uint32_t aux[K];
  uint64_t rec[K];
  int n = 0;
  int dropped = 0;

  __device__ inline static bool less(TKey ta, uint32_t ia, TKey tb, uint32_t ib) {
    return ta < tb || (ta == tb && ia < ib);
  }

  __device__ inline void insert(TKey tk, float sout, uint32_t id, uint32_t ax, uint64_t rc) {
    if (n == K && !less(tk, id, t[K - 1], idx[K - 1])) {
      ++dropped;
      return;
    }
    if (n == K) ++dropped;
    // carry the new entry down the sorted array, swapping with larger keys
#pragma unroll
    for (int i = 0; i < K; ++i) {
      bool occupied = i < n;
      bool sw = !occupied || less(tk, id, t[i], idx[i]);
      if (sw) {
        TKey t2 = t[i];
        float s2 = so[i];
        uint32_t i2 = idx[i], a2 = aux[i];
        uint64_t r2 = rec[i];
        t[i] = tk;
        so[i] = sout;
        idx[i] = id;
        aux[i] = ax;
        rec[i] = rc;
        tk = t2;
        sout = s2;
        id = i2;
        ax = a2;
        rc = r2;
        if (!occupied) break;
      }
    }
    if (n < K) ++n;
  }

  // Removes the smallest entry (slot 0), shifting the others down.
  __device__ inline void pop_front() {
#pragma unroll
    for (int i = 0; i + 1 < K; ++i) {
      t[i] = t[i + 1];
      so[i] = so[i + 1];
      idx[i] = idx[i + 1];
      aux[i] = aux[i + 1];
      rec[i] = rec[i + 1];
    }
    --n;
  }
};

struct Ray {
  float o[3], d[3];
  double od[3], inv[3];
  double tnext[3];
  int32_t cell[3];
  int32_t step[3];
  double t0;
  bool alive;
};

// Opacity acceleration (section "Transparency rendering", after Danskin and
// Hanrahan): from the ray parameter t0 (the end of the voxel where the
// optical depth passed accel_depth) the ray samples the density pyramid, at
// depth d on level min(top, 1 + floor(log2(d / accel_depth))) with step
// D = 2^level voxels, one trilinear sample per step at its midpoint: opacity
// min(1, rho D), colour the colour pyramid's mean (unlit); front to back until
// alpha_stop or the grid's edge.
__device__ inline void accel_phase(const RenderArgs& R, const Ray& ray, double t0, Accum& acc) {
  const double dx = ray.d[0], dy = ray.d[1], dz = ray.d[2];
  const double dl = sqrt(dx * dx + dy * dy + dz * dz);
  const double u[3] = {dx / dl, dy / dl, dz / dl};
  double s = t0 * dl;
  const int top = R.n_levels - 1;
  for (int it = 0; it < 4096 && acc.A < R.alpha_stop; ++it) {
    const double delta = -log(1.0 - (double)acc.A);
    int lv = 1 + (int)floor(log2(delta / (double)R.accel_depth));
    lv = lv < 1 ? 1 : lv;
    lv = lv > top ? top : lv;
    const double D = ldexp(1.0, lv);
    double x[3];
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      x[a] = ray.od[a] + (s + 0.5 * D) * u[a];
      inside &= x[a] >= 0.0 && x[a] < (double)R.g[a];
    }
    if (!inside) break;
    int32_t dim[3], cell[3];
    int64_t off;
    level_geom(R.g, lv, dim, off);
    float q[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double fl = floor(x[a]);
      cell[a] = (int32_t)fl;
      q[a] = (float)(x[a] - fl);
    }
    const float r = sample_level(R.rho + off, dim, lv, cell, q);
    const float alpha = fminf(r * (float)D, 1.f);
    if (r > 0.f && alpha > 0.f) {
      float c[3];
      sample_level3(R.rgb + 3 * off, dim, lv, cell, q, c);
      const float w = (1.f - acc.A) * alpha, ir = 1.f / r;
      acc.C[0] += w * (c[0] * ir);
      acc.C[1] += w * (c[1] * ir);
      acc.C[2] += w * (c[2] * ir);
      acc.A += w;
    }
    s += D;
  }
}

__device__ inline void make_ray(const RenderArgs& R, int i, int j, float o[3], float d[3]) {
  double u = __dadd_rn(__ddiv_rn(__dmul_rn(2.0, __dadd_rn((double)i, 0.5)), (double)R.W), -1.0);
  double v = __dadd_rn(1.0, -__ddiv_rn(__dmul_rn(2.0, __dadd_rn((double)j, 0.5)), (double)R.H));
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double su = __dmul_rn(u, (double)R.right[a]);
    double sv = __dmul_rn(v, (double)R.up[a]);
    if (R.ortho) {
      o[a] = (float)__dadd_rn(__dadd_rn((double)R.eye[a], su), sv);
      d[a] = R.fwd[a];
    } else {
      o[a] = R.eye[a];
      d[a] = (float)__dadd_rn(__dadd_rn((double)R.fwd[a], su), sv);
    }
  }
}

__device__ inline void dda_init(const RenderArgs& R, Ray& ray) {
  double tn = 0.0, tf = INFINITY;
  ray.alive = false;
  if (ray.d[0] == 0.f && ray.d[1] == 0.f && ray.d[2] == 0.f) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ray.od[a] = (double)ray.o[a];
    double d = (double)ray.d[a];
    const double inv = __ddiv_rn(1.0, d);
    // an axis whose 1/d overflows (d == 0 or denormal) is parallel to the ray
    if (d != 0.0 && !isinf(inv)) {
      ray.inv[a] = inv;
      double ta = __dmul_rn(__dadd_rn(0.0, -ray.od[a]), ray.inv[a]);
      double tb = __dmul_rn(__dadd_rn((double)R.g[a], -ray.od[a]), ray.inv[a]);
      double lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
      tn = lo > tn ? lo : tn;
      tf = hi < tf ? hi : tf;
      ray.step[a] = d > 0.0 ? 1 : -1;
    } else {
      ray.inv[a] = 0.0;
      ray.step[a] = 0;
      if (!(ray.od[a] >= 0.0 && ray.od[a] < (double)R.g[a])) tf = -INFINITY;
    }
  }
  if (!(tn < tf)) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double p = __dadd_rn(ray.od[a], __dmul_rn((double)ray.d[a], tn));
    double fl = floor(p);
    int32_t c = fl < 0.0 ? 0 : (fl > (double)(R.g[a] - 1) ? R.g[a] - 1 : (int32_t)fl);
    ray.cell[a] = c;
    if (ray.step[a] > 0)
      ray.tnext[a] = __dmul_rn(__dadd_rn((double)(c + 1), -ray.od[a]), ray.inv[a]);
    else if (ray.step[a] < 0)
      ray.tnext[a] = __dmul_rn(__dadd_rn((double)c, -ray.od[a]), ray.inv[a]);
    else
      ray.tnext[a] = INFINITY;
  }
  ray.t0 = tn;
  ray.alive = true;
}

// Advance to the next voxel; returns the t1 of the voxel just left.
__device__ inline double dda_step(const RenderArgs& R, Ray& ray) {
  int a = 0;
  if (ray.tnext[1] < ray.tnext[0]) a = 1;
  if (ray.tnext[2] < (a == 0 ? ray.tnext[0] : ray.tnext[1])) a = 2;
  double t1;
  if (a == 0) {
    t1 = ray.tnext[0];
    ray.cell[0] += ray.step[0];
    if (ray.cell[0] < 0 || ray.cell[0] >= R.g[0]) ray.alive = false;
    double plane = (double)(ray.step[0] > 0 ? ray.cell[0] + 1 : ray.cell[0]);
    ray.tnext[0] = __dmul_rn(__dadd_rn(plane, -ray.od[0]), ray.inv[0]);
  } else if (a == 1) {
    t1 = ray.tnext[1];
    ray.cell[1] += ray.step[1];
    if (ray.cell[1] < 0 || ray.cell[1] >= R.g[1]) ray.alive = false;
    double plane = (double)(ray.step[1] > 0 ? ray.cell[1] + 1 : ray.cell[1]);
    ray.tnext[1] = __dmul_rn(__dadd_rn(plane, -ray.od[1]), ray.inv[1]);
  } else {
    t1 = ray.tnext[2];
    ray.cell[2] += ray.step[2];
    if (ray.cell[2] < 0 || ray.cell[2] >= R.g[2]) ray.alive = false;
    double plane = (double)(ray.step[2] > 0 ? ray.cell[2] + 1 : ray.cell[2]);
    ray.tnext[2] = __dmul_rn(__dadd_rn(plane, -ray.od[2]), ray.inv[2]);
  }
  return t1;
}

__device__ inline double peek_t1(const Ray& ray) {
  double m = ray.tnext[0];
  m = ray.tnext[1] < m ? ray.tnext[1] : m;
  m = ray.tnext[2] < m ? ray.tnext[2] : m;
  return m;
}

// Empty-space skipping. The fine walk handles plane crossings in
// lexicographic (t, axis) order. Leaving an empty 4^3 macro cell M, it stops
// at the first crossing of M's boundary, (T*, a*) = lexicographic minimum over
// the axes of (t of the boundary plane, axis). Jumping there directly gives the
// same state: on the exit axis the cell moves to the first cell past the
// boundary; on every other axis the cell advances by the number of its planes
// inside M with (t, axis) < (T*, a*) (at most 3, tested with the same fp64
// formula); the next crossings are recomputed from the new cells. Voxel order
// and t values of every non-empty voxel are therefore unchanged.
__device__ inline void macro_jump(const RenderArgs& R, Ray& ray, const int32_t m[3]) {
  double T[3];
  int32_t B[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (ray.step[a] > 0) {
      B[a] = min(4 * (m[a] + 1), R.g[a]);
      T[a] = __dmul_rn(__dadd_rn((double)B[a], -ray.od[a]), ray.inv[a]);
    } else if (ray.step[a] < 0) {
      B[a] = 4 * m[a];
      T[a] = __dmul_rn(__dadd_rn((double)B[a], -ray.od[a]), ray.inv[a]);
    } else {
      B[a] = 0;
      T[a] = INFINITY;
    }
  }
  int ax = 0;
  if (T[1] < T[0]) ax = 1;
  if (T[2] < (ax == 0 ? T[0] : T[1])) ax = 2;
  const double Ts = ax == 0 ? T[0] : (ax == 1 ? T[1] : T[2]);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    if (ray.step[b] == 0) continue;
    int32_t c = ray.cell[b];
    if (b == ax) {
      c = ray.step[b] > 0 ? B[b] : B[b] - 1;
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int32_t plane = ray.step[b] > 0 ? c + 1 : c;
        if (plane == B[b]) break;
        const double t = __dmul_rn(__dadd_rn((double)plane, -ray.od[b]), ray.inv[b]);
        if (t < Ts || (t == Ts && b < ax)) c += ray.step[b];
        else break;
      }
    }
    ray.cell[b] = c;
    const double plane = (double)(ray.step[b] > 0 ? c + 1 : c);
    ray.tnext[b] = __dmul_rn(__dadd_rn(plane, -ray.od[b]), ray.inv[b]);
  }
  ray.t0 = Ts;
  // (selects rather than an indexed access keep the arrays in registers)
  const int32_t ce = ax == 0 ? ray.cell[0] : (ax == 1 ? ray.cell[1] : ray.cell[2]);
  const int32_t ge = ax == 0 ? R.g[0] : (ax == 1 ? R.g[1] : R.g[2]);
  if (ce < 0 || ce >= ge) ray.alive = false;
}

__device__ inline void local_origin(const Ray& ray, double t, const int32_t cell[3], float q[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) q[a] = (float)(fma(t, (double)ray.d[a], ray.od[a]) - (double)cell[a]);
}

// ---------------------------------------------------------------------------
// Wave-cooperative list tests (own-list mode). In one step of the grid walk
// only some lanes stand in a non-empty voxel, and their lists differ in
// length; testing each lane's own list leaves most lanes idle while the
// longest list is tested. Instead the (ray, line) pairs of the whole wave are
// numbered by a prefix sum over the list lengths and dealt out 64 at a time:
// pair w belongs to the last lane r with P_r <= w (a binary search over the
// lanes' prefixes), and the tester reads r's ray frame by cross-lane reads.
// Hits go back to their owners through a ballot: owner r pulls the hits of
// the testers in its pair range one by one, so every owner sees the same set
// of hits (and the same sorted buffer) as if it had tested its list itself.
__device__ inline int wave_lane() { return (int)(threadIdx.x & 63); }

__device__ inline uint32_t wave_excl_scan(uint32_t v, uint32_t& total) {
  const int lane = wave_lane();
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d, 64);
    if (lane >= d) inc += y;
  }
  total = __shfl(inc, 63, 64);
  return inc - v;
}

// Last lane r with P_r <= w (P non-decreasing over the lanes).
__device__ inline int pair_owner(uint32_t P, uint32_t w) {
  int r = 0;
#pragma unroll
  for (int step = 32; step >= 1; step >>= 1) {
    const uint32_t pc = __shfl(P, r + step, 64);
    if (pc <= w) r += step;
  }
  return r;
}

// Bits [a, b) of a 64-bit mask (0 <= a <= b <= 64).
__device__ inline unsigned long long bit_range(int a, int b) {
  if (a >= b) return 0ull;
  const unsigned long long hi = b >= 64 ? ~0ull : ((1ull << b) - 1ull);
  return hi & ~((1ull << a) - 1ull);
}

__device__ inline double shfl_f64(double v, int src) {
  return __hiloint2double(__shfl(__double2hiint(v), src, 64), __shfl(__double2loint(v), src, 64));
}

// Called by all 64 lanes together. Lane `mine` owns the voxel vcell entered
// at vt0 with lines [lo, hi).
template <bool kVdi>
__device__ __attribute__((always_inline)) inline void voxels_coop(
    const RenderArgs& R, const float4* lut_lds, const Ray& ray, const int32_t vcell[3],
    double vt0, const Shade& S, float dd, float inv_dd, bool mine, uint32_t lo, uint32_t hi,
    Accum& acc, Counts& cnt) {
  const int lane = wave_lane();
  const uint32_t n = mine ? hi - lo : 0u;
  if (__ballot(n != 0u) == 0ull) return;
  float q[3] = {0.f, 0.f, 0.f};
  if (mine) local_origin(ray, vt0, vcell, q);
  if (R.opaque) {
    uint32_t N;
    const uint32_t P = wave_excl_scan(n, N);
    float best = INFINITY;
    uint32_t bi = 0xFFFFFFFFu;
    for (uint32_t base = 0; base < N; base += 64) {
      const uint32_t w = base + (uint32_t)lane;
      const int r = pair_owner(P, w);
      const float qr[3] = {__shfl(q[0], r, 64), __shfl(q[1], r, 64), __shfl(q[2], r, 64)};
      const float dr[3] = {__shfl(ray.d[0], r, 64), __shfl(ray.d[1], r, 64),
                           __shfl(ray.d[2], r, 64)};
      const float ddr = __shfl(dd, r, 64), iddr = __shfl(inv_dd, r, 64);
      const uint32_t lor = __shfl(lo, r, 64), Pr = __shfl(P, r, 64);
      const double vt0r = shfl_f64(vt0, r);
      bool hit = false;
      float si = 0.f, so = 0.f;
      uint32_t k = 0;
      if (w < N) {
        k = lor + (w - Pr);
        const uint64_t rec = R.records[k];
        float a[3], b[3];
        decode_point((uint32_t)(rec & 0x7FFFu), R.inv_bins, a);
        decode_point((uint32_t)((rec >> 15) & 0x7FFFu), R.inv_bins, b);
        cnt.tested++;
        hit = capsule(qr, dr, ddr, iddr, a, b, R.r2, si, so) && vt0r + (double)si >= 0.0;
      }
      unsigned long long m =
          __ballot(hit) & bit_range(max((int)P - (int)base, 0), min((int)(P + n) - (int)base, 64));
      while (__ballot(m != 0ull) != 0ull) {
        const int src = m ? __builtin_ctzll(m) : 0;
        const float ts = __shfl(si, src, 64);
        const uint32_t ks = __shfl(k, src, 64);
        if (m) {
          cnt.hits++;
          if (ts < best || (ts == best && ks < bi)) {
            best = ts;
            bi = ks;
          }
          m &= m - 1ull;
        }
      }
    }
    if (mine) {
      cnt.list_bytes += 8u * n;
      if (bi != 0xFFFFFFFFu) {
        const uint64_t rec = R.records[bi];
        float a[3], b[3], p[3];
        decode_point((uint32_t)(rec & 0x7FFFu), R.inv_bins, a);
        decode_point((uint32_t)((rec >> 15) & 0x7FFFu), R.inv_bins, b);
#pragma unroll
        for (int c = 0; c < 3; ++c) p[c] = q[c] + best * ray.d[c];
        composite<kVdi>(R, lut_lds, S, acc, rec, bi, vcell, p, a, b, 0.f, cnt);
        acc.done = true;
      }
    }
    return;
  }
  // transparent: passes of up to kCoopSlots hits per owner, in (t, index) order
  bool need = n != 0u;
  bool first = true;
  float last_t = -INFINITY;
  uint32_t last_i = 0;
  while (__ballot(need) != 0ull) {
    const uint32_t np = need ? n : 0u;
    uint32_t N;
    const uint32_t P = wave_excl_scan(np, N);
    HitBuf<float, kCoopSlots> buf;
    for (uint32_t base = 0; base < N; base += 64) {
      const uint32_t w = base + (uint32_t)lane;
      const int r = pair_owner(P, w);
      const float qr[3] = {__shfl(q[0], r, 64), __shfl(q[1], r, 64), __shfl(q[2], r, 64)};
      const float dr[3] = {__shfl(ray.d[0], r, 64), __shfl(ray.d[1], r, 64),
                           __shfl(ray.d[2], r, 64)};
      const float ddr = __shfl(dd, r, 64), iddr = __shfl(inv_dd, r, 64);
      const uint32_t lor = __shfl(lo, r, 64), Pr = __shfl(P, r, 64);
      const double vt0r = shfl_f64(vt0, r);
      const bool firstr = __shfl((int)first, r, 64) != 0;
      const float ltr = __shfl(last_t, r, 64);
      const uint32_t lir = __shfl(last_i, r, 64);
      bool hit = false;
      float si = 0.f, so = 0.f;
      uint32_t k = 0;
      if (w < N) {
        k = lor + (w - Pr);
        const uint64_t rec = R.records[k];
        float a[3], b[3];
        decode_point((uint32_t)(rec & 0x7FFFu), R.inv_bins, a);
        decode_point((uint32_t)((rec >> 15) & 0x7FFFu), R.inv_bins, b);
        cnt.tested++;
        // t >= 0 and the pass filter are applied here, so only kept hits are pulled
        hit = capsule(qr, dr, ddr, iddr, a, b, R.r2, si, so) && vt0r + (double)si >= 0.0 &&
              (firstr || HitBuf<float, kCoopSlots>::less(ltr, lir, si, k));
      }
      unsigned long long m =
          __ballot(hit) & bit_range(max((int)P - (int)base, 0), min((int)(P + np) - (int)base, 64));
      while (__ballot(m != 0ull) != 0ull) {
        const int src = m ? __builtin_ctzll(m) : 0;
        const float ts = __shfl(si, src, 64), os = __shfl(so, src, 64);
        const uint32_t ks = __shfl(k, src, 64);
        if (m) {
          if (first) cnt.hits++;
          buf.insert(ts, os, ks, 0u, 0ull);   // the record is reloaded when composited
          m &= m - 1ull;
        }
      }
    }
    if (need) {
      cnt.list_bytes += 8u * n;
      // the pass's last key bounds the next pass (read before consuming)
      last_t = buf.t[kCoopSlots - 1];
      last_i = buf.idx[kCoopSlots - 1];
      const bool more = buf.dropped != 0;
      while (buf.n > 0 && !acc.done) {
        const float t_in = buf.t[0], t_out = buf.so[0];
        const uint32_t ki = buf.idx[0];
        const uint64_t rc = R.records[ki];
        buf.pop_front();
        if (R.merge) {
          const uint32_t tag = (uint32_t)(rc >> 40);
          if (merge_hit(acc, tag, vt0 + (double)t_in, vt0 + (double)t_out, cnt)) continue;
        }
        float a[3], b[3], p[3];
        decode_point((uint32_t)(rc & 0x7FFFu), R.inv_bins, a);
        decode_point((uint32_t)((rc >> 15) & 0x7FFFu), R.inv_bins, b);
#pragma unroll
        for (int c = 0; c < 3; ++c) p[c] = q[c] + t_in * ray.d[c];
        composite<kVdi>(R, lut_lds, S, acc, rc, ki, vcell, p, a, b, t_out - t_in, cnt);
      }
      need = more && !acc.done;
      if (need) cnt.passes++;
      first = false;
    }
  }
}

// Neighbour mode: lines of the 27 voxels around the visited one; a hit is
// accepted by the visited voxel whose [t0, t1) holds its entry t. Each
// line's t is computed in the frame of its own voxel, with the origin at the
// ray point nearest the voxel centre, so every visited voxel sees the same t
// for a line and the hits are partitioned exactly.
__device__ inline double owner_ref(const Ray& ray, const int32_t w[3], double idd) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) s += ((double)w[a] + 0.5 - ray.od[a]) * (double)ray.d[a];
  return s * idd;
}

// Ray vs capsule for the neighbour mode, as absolute ray parameters. The
// cylinder is intersected in the owner voxel's frame (origin at the ray point
// tr); each joint sphere in a frame of its own, with the origin at the ray
// point nearest its centre c = owner corner + endpoint (exact in fp32). Two
// consecutive lines of a curve share that sphere: a ray entering through it
// then gets bit-identical entry parameters from both lines, and their order
// falls to the record index, as with exact arithmetic.
__device__ inline bool capsule_abs(const Ray& ray, double tr, const float q[3], const int32_t w[3],
                                   float dd, float inv_dd, double idd, const float a[3],
                                   const float b[3], float r2, double& t_in, double& t_out) {
  #pragma clang fp contract(fast)
  double lo = INFINITY, hi = -INFINITY;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const float* p = e ? b : a;
    double c[3], tc = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      c[k] = (double)w[k] + (double)p[k];
      tc += (c[k] - ray.od[k]) * (double)ray.d[k];
    }
    tc *= idd;
    float qs[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) qs[k] = (float)(fma(tc, (double)ray.d[k], ray.od[k]) - c[k]);
    const float B = dot3(qs, ray.d), C = dot3(qs, qs) - r2;
    const float disc = B * B - dd * C;
    if (disc >= 0.f) {
      const float s = __builtin_sqrtf(disc);
      lo = fmin(lo, tc + (double)((-B - s) * inv_dd));
      hi = fmax(hi, tc + (double)((-B + s) * inv_dd));
    }
  }
  float ba[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  float oa[3] = {q[0] - a[0], q[1] - a[1], q[2] - a[2]};
  float L2 = dot3(ba, ba);
  float iL2 = rcp(L2);
  float dba = dot3(ray.d, ba), oba = dot3(oa, ba);
  float kd = dba * iL2, ko = oba * iL2;
  float dp[3] = {ray.d[0] - kd * ba[0], ray.d[1] - kd * ba[1], ray.d[2] - kd * ba[2]};
  float op[3] = {oa[0] - ko * ba[0], oa[1] - ko * ba[1], oa[2] - ko * ba[2]};
  float A = dot3(dp, dp);
  if (A > 0.f) {
    float B = dot3(op, dp), C = dot3(op, op) - r2;
    float disc = B * B - A * C;
    if (disc >= 0.f) {
      float s = __builtin_sqrtf(disc);
      float iA = rcp(A);
      float c0 = (-B - s) * iA, c1 = (-B + s) * iA;
      float s0, s1;
      if (dba != 0.f) {
        float idba = rcp(dba);
        float u0 = -oba * idba, u1 = (L2 - oba) * idba;
        s0 = fminf(u0, u1);
        s1 = fmaxf(u0, u1);
      } else if (oba >= 0.f && oba <= L2) {
        s0 = -INFINITY;
        s1 = INFINITY;
      } else {
        s0 = INFINITY;
        s1 = -INFINITY;
      }
      float e0 = fmaxf(c0, s0), e1 = fminf(c1, s1);
      if (e0 <= e1) {
        lo = fmin(lo, tr + (double)e0);
        hi = fmax(hi, tr + (double)e1);
      }
    }
  }
  t_in = lo;
  t_out = hi;
  return lo <= hi;
}

template <bool kVdi>
__device__ __attribute__((always_inline)) inline void voxel_exact(const RenderArgs& R, const float4* lut_lds, const Ray& ray, const Shade& S, float dd,
                                   float inv_dd, double idd, double t1, Accum& acc, Counts& cnt) {
  double last_t = -INFINITY;
  uint32_t last_i = 0;
  bool first = true;
  for (;;) {
    HitBuf<double> buf;
    for (int nb = 0; nb < 27; ++nb) {
      int32_t w[3] = {ray.cell[0] + nb % 3 - 1, ray.cell[1] + (nb / 3) % 3 - 1,
                      ray.cell[2] + nb / 9 - 1};
      if (w[0] < 0 || w[1] < 0 || w[2] < 0 || w[0] >= R.g[0] || w[1] >= R.g[1] || w[2] >= R.g[2])
        continue;
      const int64_t vid = w[0] + (int64_t)R.g[0] * (w[1] + (int64_t)R.g[1] * w[2]);
      const uint32_t lo = R.offsets[vid], hi = R.offsets[vid + 1];
      cnt.list_bytes += 8u + 8u * (hi - lo);
      if (lo == hi) continue;
      const double tr = owner_ref(ray, w, idd);
      float q[3];
      local_origin(ray, tr, w, q);
      for (uint32_t k = lo; k < hi; ++k) {
        const uint64_t rec = R.records[k];
        float a[3], b[3];
        decode_point((uint32_t)(rec & 0x7FFFu), R.inv_bins, a);
        decode_point((uint32_t)((rec >> 15) & 0x7FFFu), R.inv_bins, b);
        cnt.tested++;
        double ti, to;
        if (!capsule_abs(ray, tr, q, w, dd, inv_dd, idd, a, b, R.r2, ti, to)) continue;
        if (!(ti >= ray.t0 && ti < t1)) continue;
        if (!first && !HitBuf<double>::less(last_t, last_i, ti, k)) continue;
        if (first) cnt.hits++;
        buf.insert(ti, (float)(to - ti), k, (uint32_t)nb, rec);
      }
    }
    last_t = buf.t[kSortSlots - 1];
    last_i = buf.idx[kSortSlots - 1];
    const bool more = buf.dropped != 0;
    while (buf.n > 0 && !acc.done) {
      const double t_in = buf.t[0];
      const float len = buf.so[0];
      const int nb = (int)buf.aux[0];
      const uint64_t rec = buf.rec[0];
      const uint32_t ki = buf.idx[0];
      buf.pop_front();
      if (!R.opaque && R.merge) {
        const uint32_t tag = (uint32_t)(rec >> 40);
        if (merge_hit(acc, tag, t_in, t_in + (double)len, cnt)) continue;
      }
      int32_t w[3] = {ray.cell[0] + nb % 3 - 1, ray.cell[1] + (nb / 3) % 3 - 1,
                      ray.cell[2] + nb / 9 - 1};
      const double tr = owner_ref(ray, w, idd);
      float q[3], a[3], b[3], p[3];
      local_origin(ray, tr, w, q);
      const float s_in = (float)(t_in - tr);
      decode_point((uint32_t)(rec & 0x7FFFu), R.inv_bins, a);
      decode_point((uint32_t)((rec >> 15) & 0x7FFFu), R.inv_bins, b);
#pragma unroll
      for (int c = 0; c < 3; ++c) p[c] = q[c] + s_in * ray.d[c];
      composite<kVdi>(R, lut_lds, S, acc, rec, ki, w, p, a, b, len, cnt);
      if (R.opaque) acc.done = true;
    }
    if (acc.done || !more) break;
    first = false;
    cnt.passes++;
  }
}

__device__ inline void flush_counts(RenderCounters* out, const Counts& c) {
  unsigned long long v[11] = {c.visited, c.nonempty, c.tested, c.hits, c.fragments, c.list_bytes,
                              c.passes, c.evictions, c.skips, c.live_evictions, c.overflow_rays};
#pragma unroll
  for (int k = 0; k < 11; ++k) {
    unsigned long long x = v[k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    v[k] = x;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&out->visited, v[0]);
    atomicAdd(&out->nonempty, v[1]);
    atomicAdd(&out->tested, v[2]);
    atomicAdd(&out->hits, v[3]);
    atomicAdd(&out->fragments, v[4]);
    atomicAdd(&out->list_bytes, v[5]);
    atomicAdd(&out->sort_passes, v[6]);
    atomicAdd(&out->merge_evictions, v[7]);
    atomicAdd(&out->macro_skips, v[8]);
    atomicAdd(&out->merge_live_evictions, v[9]);
    atomicAdd(&out->merge_overflow_rays, v[10]);
  }
}

template <int kMode, bool kVdi>
// All 64 lanes of the wave call this together (mode 0 tests lists
// cooperatively); a lane whose pixel lies outside the image takes part
// with a dead ray and writes nothing.
__device__ __attribute__((always_inline)) inline void render_pixel(const RenderArgs& R, const float4* lut_lds, const MergeLds& mt, int i,
                                                             int j, bool valid, Counts& cnt) {
  Ray ray;
  make_ray(R, valid ? i : 0, valid ? j : 0, ray.o, ray.d);
  dda_init(R, ray);
  if (!valid) ray.alive = false;
  Accum acc(mt);
  const uint32_t live_ev0 = cnt.live_evictions;
  {
    const float dd = dot3(ray.d, ray.d);
    const float inv_dd = 1.f / dd;
    const double idd = 1.0 / ((double)ray.d[0] * ray.d[0] + (double)ray.d[1] * ray.d[1] +
                              (double)ray.d[2] * ray.d[2]);
    Shade S;
    const float il = __builtin_amdgcn_rsqf(dd);
    S.v[0] = -ray.d[0] * il;
    S.v[1] = -ray.d[1] * il;
    S.v[2] = -ray.d[2] * il;
    float h[3] = {R.light[0] + S.v[0], R.light[1] + S.v[1], R.light[2] + S.v[2]};
    float hl = dot3(h, h);
    float ih = hl > 0.f ? __builtin_amdgcn_rsqf(hl) : 0.f;
    S.h[0] = h[0] * ih;
    S.h[1] = h[1] * ih;
    S.h[2] = h[2] * ih;
    S.dlen = __builtin_sqrtf(dd);
    // every step moves one cell monotonically along one axis: at most
    // gx + gy + gz steps (the cap only guards against malformed input)
    const int max_steps = R.g[0] + R.g[1] + R.g[2] + 3;
    if (kMode == 0) {
      // One 64-bit occupancy word per 4^3 macro cell: an empty macro cell is
      // jumped in one step, and an empty voxel inside an occupied one is
      // stepped over without touching the lists. Each step, the lanes that
      // entered a non-empty voxel test their lists together (voxels_coop).
      int64_t last_mid = -1;
      unsigned long long occ = 0;
      for (int it = 0;; ++it) {
        const bool live = it < max_steps && ray.alive && !acc.done;
        if (__ballot(live) == 0ull) break;
        bool mine = false;
        uint32_t lo = 0, hi = 0;
        int32_t vc[3] = {0, 0, 0};
        double vt0 = 0.0;
        if (live) {
          const int32_t m[3] = {ray.cell[0] >> 2, ray.cell[1] >> 2, ray.cell[2] >> 2};
          const int64_t mid = m[0] + (int64_t)R.mg[0] * (m[1] + (int64_t)R.mg[1] * m[2]);
          if (mid != last_mid) {
            last_mid = mid;
            occ = R.occ[mid];
            cnt.list_bytes += 8u;
          }
          if (occ == 0ull) {
            cnt.skips++;
            macro_jump(R, ray, m);
          } else {
            cnt.visited++;
            const int bit = (ray.cell[0] & 3) + 4 * (ray.cell[1] & 3) + 16 * (ray.cell[2] & 3);
            if ((occ >> bit) & 1ull) {
              const int64_t vid =
                  ray.cell[0] + (int64_t)R.g[0] * (ray.cell[1] + (int64_t)R.g[1] * ray.cell[2]);
              lo = R.offsets[vid];
              hi = R.offsets[vid + 1];
              cnt.list_bytes += 8u;
              cnt.nonempty++;
              mine = true;
              vc[0] = ray.cell[0];
              vc[1] = ray.cell[1];
              vc[2] = ray.cell[2];
              vt0 = ray.t0;
            }
            ray.t0 = dda_step(R, ray);
          }
        }
        voxels_coop<kVdi>(R, lut_lds, ray, vc, vt0, S, dd, inv_dd, mine, lo, hi, acc, cnt);
      }
    } else {
      for (int it = 0; it < max_steps && ray.alive && !acc.done; ++it) {
        cnt.visited++;
        const int64_t vid =
            ray.cell[0] + (int64_t)R.g[0] * (ray.cell[1] + (int64_t)R.g[1] * ray.cell[2]);
        if (R.offsets[vid + 1] > R.offsets[vid]) cnt.nonempty++;
        voxel_exact<kVdi>(R, lut_lds, ray, S, dd, inv_dd, idd, peek_t1(ray), acc, cnt);
        ray.t0 = dda_step(R, ray);
      }
    }
  }
  if (kVdi && acc.switched && valid) accel_phase(R, ray, ray.t0, acc);
  if (cnt.live_evictions != live_ev0) cnt.overflow_rays++;
  if (valid) {
    float4 px = make_float4(acc.C[0], acc.C[1], acc.C[2], acc.A);
    reinterpret_cast<float4*>(R.out)[(int64_t)j * R.W + i] = px;
  }
}

// Pixel of lane `lane` in wave `wave` of tile `tile` (tile = wx x wy waves of 8 x 8).
__device__ inline void tile_pixel(const RenderArgs& R, int tile, int wave, int lane, int& i, int& j) {
  const int tx = tile % R.tiles_x, ty = tile / R.tiles_x;
  i = tx * 8 * R.wx + (wave % R.wx) * 8 + (lane & 7);
  j = ty * 8 * R.wy + (wave / R.wx) * 8 + (lane >> 3);
}

template <bool kVdi>
__device__ __attribute__((always_inline)) inline void render_any(const RenderArgs& R, const float4* lut_lds, const MergeLds& mt, int i, int j,
                       bool valid, Counts& cnt) {
  if (R.mode == 0) render_pixel<0, kVdi>(R, lut_lds, mt, i, j, valid, cnt);
  else render_pixel<1, kVdi>(R, lut_lds, mt, i, j, valid, cnt);
}

// Stages a view's transfer function (256 RGBA) in LDS.
__device__ inline void load_lut(const RenderArgs& R, float4* lut_lds) {
  for (int k = threadIdx.x; k < 256; k += blockDim.x)
    lut_lds[k] = reinterpret_cast<const float4*>(R.lut)[k];
}

template <int kMode, bool kCount, bool kVdi>
__global__ __launch_bounds__(kBlock) void k_render(RenderArgs R) {
  const unsigned long long t_start = R.times ? wall_clock64() : 0ull;
  int b = blockIdx.x;
  int tile;
  bool live;
  int sub = 0, nsub = 1;   // sub-tile (rows sub * 8 / nsub ...) of a split tile
  if (R.spiral_r >= 0) {
    // launch positions: the first top_n tiles (the longest measured ones of
    // an ordered frame) split four ways, the next split_n split_s ways, the
    // rest whole; in groups of kXcds tiles x nsub parts, as workgroups are
    // dealt to the XCDs round-robin, so in a full group the parts of a tile
    // share an XCD (and its L2) as its lists are read again
    int first = 0;   // launch positions before this region
    if (b < R.top_s * R.top_n) {
      nsub = R.top_s;
      const int grp = b / (kXcds * nsub), r = b - grp * kXcds * nsub;
      const int w = min(kXcds, R.top_n - grp * kXcds);   // tiles in the group
      sub = r / w;
      b = grp * kXcds + r % w;
    } else {
      b -= R.top_s * R.top_n;
      first = R.top_n;
      if (R.split_s > 1) {
        const int ns = R.split_n * R.split_s;
        if (b < ns) {
          nsub = R.split_s;
          const int grp = b / (kXcds * nsub), r = b - grp * kXcds * nsub;
          const int w = min(kXcds, R.split_n - grp * kXcds);
          sub = r / w;
          b = grp * kXcds + r % w;
        } else {
          b -= ns - R.split_n;
        }
      }
      b += first;
    }
    if (R.order) {
      // tiles by decreasing measured time
      tile = R.order[b];
      live = tile >= 0 && tile < R.n_tiles;
    } else {
    // Tiles in square rings around the projection of the grid centre, where
    // rays cross the most voxels: the costliest tiles start first instead of
    // setting the frame's tail. Ring r holds workgroups [(2r-1)^2, (2r+1)^2).
    int s = (int)sqrtf((float)b);
    while (s * s > b) --s;
    while ((s + 1) * (s + 1) <= b) ++s;
    const int r = (s + 1) / 2;
    int dx = 0, dy = 0;
    if (r > 0) {
      const int k = b - (2 * r - 1) * (2 * r - 1), side = 2 * r;
      if (k < side) {
        dx = r;
        dy = -r + 1 + k;
      } else if (k < 2 * side) {
        dx = r - 1 - (k - side);
        dy = r;
      } else if (k < 3 * side) {
        dx = -r;
        dy = r - 1 - (k - 2 * side);
      } else {
        dx = -r + 1 + (k - 3 * side);
        dy = -r;
      }
    }
    const int tx = R.spiral_x + dx, ty = R.spiral_y + dy;
    const int tiles_y = R.n_tiles / R.tiles_x;
    live = tx >= 0 && ty >= 0 && tx < R.tiles_x && ty < tiles_y;
    tile = ty * R.tiles_x + tx;
    }
  } else {
    // Workgroup b runs on XCD b % 8. XCD x renders the tile rows x, x + 8,
    // x + 16, ...: whole rows keep neighbouring tiles in one L2, and every
    // XCD gets a share of the part of the screen the grid covers.
    const int x = b % kXcds, l = b / kXcds;
    const int row = x + kXcds * (l / R.tiles_x);
    tile = row * R.tiles_x + l % R.tiles_x;
    live = row * R.tiles_x < R.n_tiles;
  }
  __shared__ float4 lut_lds[256];
  extern __shared__ double dyn_lds[];
  const MergeLds merge_lds = merge_lds_view(dyn_lds);
  Counts cnt;
  if (!live) {
    if (kCount) flush_counts(R.counters, cnt);
    return;
  }
  load_lut(R, lut_lds);
  __syncthreads();
  {
    int i, j;
    const int lane = threadIdx.x & 63;
    bool valid = true;
    if (nsub > 1) {
      // a split tile (1 x 1 waves): this workgroup's 8 / nsub rows, on the
      // first 64 / nsub lanes
      const int rows = 8 / nsub;
      i = (tile % R.tiles_x) * 8 + (lane & 7);
      j = (tile / R.tiles_x) * 8 + sub * rows + (lane >> 3);
      valid = lane < 8 * rows;
    } else {
      tile_pixel(R, tile, threadIdx.x >> 6, lane, i, j);
    }
    render_pixel<kMode, kVdi>(R, lut_lds, merge_lds, i, j, valid && i < R.W && j < R.H, cnt);
  }
  if (kCount) flush_counts(R.counters, cnt);
  if (R.times && threadIdx.x == 0) {
    const unsigned long long dt = wall_clock64() - t_start;
    atomicAdd(R.times + tile, dt < 0xFFFFFFFFull ? (uint32_t)dt : 0xFFFFFFFFu);
  }
}

// Persistent batched renderer: one launch renders the tiles of many views.
// The global tile list (views concatenated, tile_start = prefix of the
// views' tile counts) is cut into 8 contiguous queues, one per XCD; a
// workgroup pops tiles from its own XCD's queue and then steals from the
// others. Every workgroup reaches the exit once all queues are drained.
template <bool kCount, bool kVdi>
__global__ __launch_bounds__(kBlock) void k_render_batch(const RenderArgs* __restrict__ views,
                                                         const int32_t* __restrict__ tile_start,
                                                         int32_t n_views, BatchQueues q,
                                                         unsigned* __restrict__ counters) {
  __shared__ int s_tile;
  __shared__ float4 lut_lds[256];
  extern __shared__ double dyn_lds[];
  const MergeLds merge_lds = merge_lds_view(dyn_lds);
  int lut_view = -1;
  const int home = blockIdx.x % kXcds;
  int qi = 0;
  Counts cnt;
  for (;;) {
    if (threadIdx.x == 0) {
      int t = -1;
      while (qi < kXcds) {
        const int qq = (home + qi) % kXcds;
        int qb = 0, ql = 0;
#pragma unroll
        for (int x = 0; x < kXcds; ++x)
          if (x == qq) {
            qb = q.begin[x];
            ql = q.len[x];
          }
        const unsigned k = atomicAdd(counters + qq, 1u);
        if (k < (unsigned)ql) {
          t = qb + (int)k;
          break;
        }
        ++qi;
      }
      s_tile = t;
    }
    __syncthreads();
    const int t = s_tile;
    __syncthreads();
    if (t < 0) break;
    // view owning tile t: last v with tile_start[v] <= t
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tile_start[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const int v = __builtin_amdgcn_readfirstlane(lo);
    const RenderArgs R = views[v];
    if (v != lut_view) {
      load_lut(R, lut_lds);
      lut_view = v;
    }
    __syncthreads();
    int i, j;
    tile_pixel(R, t - tile_start[v], threadIdx.x >> 6, threadIdx.x & 63, i, j);
    render_any<kVdi>(R, lut_lds, merge_lds, i, j, i < R.W && j < R.H, cnt);
    __syncthreads();
  }
  if (kCount && counters) flush_counts(reinterpret_cast<RenderCounters*>(counters + kXcds), cnt);
}

// ---------------------------------------------------------------------------
// Launch order by measured cost. A frame lasts as long as its slowest
// workgroups, and the costly tiles are wherever the line set is dense along
// the view (not necessarily the middle of the image, where the ring order
// starts). Every workgroup adds its duration to its tile's time; when the
// same view is rendered again on the same stream, the tiles are bucketed by
// that time, eight buckets per octave (k_tile_hist), and launched by
// decreasing bucket (k_tile_order), so the longest start first and are the
// ones split.
constexpr int kCostBuckets = 256;
// Ordered frames split their kTopTiles longest tiles four ways (frames split
// two ways) or eight ways (frames not split; frames split four ways
// throughout keep that). Measured on the scale workload's 1080p frame (split
// two ways; render 0.89 ms): 32 -> 0.815, 64 -> 0.819, 256 -> 0.845, 1024 ->
// 0.953 ms, every split tile four ways -> 1.37 ms; eight ways: 0.81 (16, 32
// tiles), 0.85 ms for the moving camera; batch-workload views rendered one at
// a time moved by +1 % at 32. On the unsplit 512^3 global-illumination 1080p
// frame: 2.0 -> 1.46 ms (four ways), 1.22 ms (eight ways; 64 tiles the same);
// opaque frames (unsplit), batch-workload sets 12-18 % faster (four ways).
constexpr int kTopTiles = 32;

__device__ inline int cost_bucket(uint32_t c) {
  if (c == 0u) return 0;
  const int lz = 31 - __builtin_clz(c);
  const int frac = lz >= 3 ? (int)((c >> (lz - 3)) & 7u) : (int)((c << (3 - lz)) & 7u);
  return min(kCostBuckets - 1, 1 + 8 * lz + frac);
}

// Buckets of the tiles' times (kept, so the order pass sees the same ones)
// and their histogram.
// Buckets of the tiles' times (kept, so the order pass sees the same ones)
// and their histogram.
__global__ __launch_bounds__(kBlock) void k_tile_hist(const uint32_t* __restrict__ cost,
                                                      int32_t n_tiles,
                                                      uint8_t* __restrict__ bucket,
                                                      uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kCostBuckets];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t < n_tiles) {
    const int q = cost_bucket(cost[t]);
    bucket[t] = (uint8_t)q;
    atomicAdd(h + q, 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(hist + threadIdx.x, h[threadIdx.x]);
}

// The first frame of a transparent view has no measured times: each tile's
// cost is estimated instead from the occupancy words its rays cross, four
// rays per tile (at the centres of its quadrants), one sample per macro-cell
// length between grid entry and exit, adding the non-empty voxels of the
// sampled macro cell. Only the launch order depends on it. Each ray's
// samples are shared by kProbeSegs lanes (every kProbeSegs-th sample).
constexpr int kProbeRays = 4, kProbeSegs = 4, kProbeLanes = kProbeRays * kProbeSegs;

__global__ __launch_bounds__(kBlock) void k_tile_probe(RenderArgs R, uint32_t* __restrict__ cost) {
  const int t = blockIdx.x * (kBlock / kProbeLanes) + (int)threadIdx.x / kProbeLanes;
  const int l = threadIdx.x % kProbeLanes, r = l % kProbeRays, seg = l / kProbeRays;
  uint32_t c = 0;
  if (t < R.n_tiles) {
    const int tw = 8 * R.wx, th = 8 * R.wy;
    const int i = min((t % R.tiles_x) * tw + ((r & 1) ? 3 * tw / 4 : tw / 4), R.W - 1);
    const int j = min((t / R.tiles_x) * th + ((r & 2) ? 3 * th / 4 : th / 4), R.H - 1);
    float o[3], d[3];
    make_ray(R, i, j, o, d);
    float tn = 0.f, tf = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (d[a] != 0.f) {
        const float inv = 1.f / d[a];
        const float ta = -o[a] * inv, tb = ((float)R.g[a] - o[a]) * inv;
        tn = fmaxf(tn, fminf(ta, tb));
        tf = fminf(tf, fmaxf(ta, tb));
      } else if (!(o[a] >= 0.f && o[a] < (float)R.g[a])) {
        tf = -1.f;
      }
    }
    const float len = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (tn < tf && len > 0.f) {
      const float dt = 4.f / len;
      const int steps = (int)fminf((tf - tn) / dt + 1.f, 4096.f);
#pragma unroll 2
      for (int k = seg; k < steps; k += kProbeSegs) {
        const float tt = tn + ((float)k + 0.5f) * dt;
        int m[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
          m[a] = min(max((int)floorf(o[a] + tt * d[a]) >> 2, 0), R.mg[a] - 1);
        c += (uint32_t)__popcll(R.occ[m[0] + (int64_t)R.mg[0] * (m[1] + (int64_t)R.mg[1] * m[2])]);
      }
    }
  }
#pragma unroll
  for (int m = 1; m < kProbeLanes; m <<= 1) c += __shfl_xor(c, m);
  if (l == 0 && t < R.n_tiles) cost[t] = c;
}

// order[p]: the tile at position p, by decreasing bucket (the order inside a
// bucket depends on atomic order; every tile appears once). Clears the
// times for the frame about to be measured.
__global__ __launch_bounds__(kBlock) void k_tile_order(uint32_t* __restrict__ cost,
                                                       const uint8_t* __restrict__ bucket,
                                                       int32_t n_tiles,
                                                       const uint32_t* __restrict__ hist,
                                                       uint32_t* __restrict__ cursor,
                                                       int32_t* __restrict__ order) {
  static_assert(kBlock == kCostBuckets, "one thread per bucket");
  __shared__ uint32_t pre[kCostBuckets];   // tiles in higher buckets
  __shared__ uint32_t cnt[kCostBuckets];
  __shared__ uint32_t base[kCostBuckets];
  const int b = threadIdx.x;
  // suffix sum of the histogram (exclusive), by a block scan
  uint32_t x = hist[kCostBuckets - 1 - b];
  pre[b] = x;
  cnt[b] = 0u;
  __syncthreads();
  for (int d = 1; d < kCostBuckets; d <<= 1) {
    const uint32_t y = b >= d ? pre[b - d] : 0u;
    __syncthreads();
    pre[b] += y;
    __syncthreads();
  }
  // pre[k] = sum of hist[255 - k .. 255] (inclusive); bucket q's start is
  // the sum over buckets above it = pre[254 - q] for q < 255, 0 for q = 255
  const uint32_t start = b == kCostBuckets - 1 ? 0u : pre[kCostBuckets - 2 - b];
  __syncthreads();
  base[b] = start;
  __syncthreads();
  const int t = blockIdx.x * kBlock + threadIdx.x;
  int q = 0;
  uint32_t r = 0;
  if (t < n_tiles) {
    q = bucket[t];
    cost[t] = 0u;
    r = atomicAdd(cnt + q, 1u);
  }
  __syncthreads();
  if (cnt[b]) base[b] += atomicAdd(cursor + b, cnt[b]);
  __syncthreads();
  if (t < n_tiles) order[base[q] + r] = t;
}

}  // namespace

int make_render_args(const ls_lineset* s, const ls_camera* cam, const ls_render_params* p,
                     float* out, int wx, int wy, RenderCounters* dev_counters, RenderArgs* Rp) {
  RenderArgs R{};
  R.offsets = s->offsets;
  R.records = s->records;
  R.occ = reinterpret_cast<const unsigned long long*>(s->occupancy);
  for (int a = 0; a < 3; ++a) {
    R.mg[a] = s->macro[a];
    R.g[a] = s->grid[a];
    R.eye[a] = cam->eye[a];
    R.fwd[a] = cam->forward[a];
    R.right[a] = cam->right[a];
    R.up[a] = cam->up[a];
    R.light[a] = p->light_dir[a];
  }
  R.inv_bins = 1.0f / (float)s->bins;
  R.lut = p->lut_rgba;
  R.ao = s->ao;
  R.sh = s->sh;
  R.ortho = cam->orthographic;
  R.W = cam->width;
  R.H = cam->height;
  R.radius = p->radius;
  R.r2 = p->radius * p->radius;
  R.alpha_stop = p->alpha_stop;
  R.mode = p->mode;
  R.opaque = p->opaque;
  R.merge = p->merge_curves;
  R.dist_alpha = p->distance_alpha;
  R.inv_2r = 0.5f / p->radius;
  R.shading = p->shading;
  R.ka = p->ka;
  R.kd = p->kd;
  R.ks = p->ks;
  R.shin = p->shininess;
  R.ao_mode = p->shading == 2 ? p->ao_mode : 0;
  R.shadow_mode = p->shading == 2 ? p->shadow_mode : 0;
  R.ao_rays = p->ao_rays;
  R.ao_radius = p->ao_radius;
  R.rep_level = p->rep_level;
  R.n_levels = s->lod_rho ? s->n_levels : 0;
  R.rho = s->lod_rho;
  R.rep = s->rep;
  R.ends = s->ends;
  R.accel_depth = p->accel_depth;
  R.accel_A0 = (!p->opaque && p->accel_depth > 0.f) ? (float)(1.0 - std::exp(-(double)p->accel_depth))
                                                    : 2.f;
  R.rgb = s->lod_rgb;
  R.out = out;
  R.counters = dev_counters;
  R.wx = wx;
  R.wy = wy;
  R.tiles_x = (R.W + 8 * wx - 1) / (8 * wx);
  const int tiles_y = (R.H + 8 * wy - 1) / (8 * wy);
  R.n_tiles = R.tiles_x * tiles_y;
  R.tiles_per_xcd = (R.n_tiles + kXcds - 1) / kXcds;
  R.spiral_r = -1;
  R.order = nullptr;
  R.top_n = 0;
  R.top_s = 4;
  R.split_n = 0;
  R.split_s = 1;
  {
    // screen position of the grid centre (camera vectors taken as orthogonal;
    // this only orders the launch)
    double p[3], F2 = 0, R2 = 0, U2 = 0, pF = 0, pR = 0, pU = 0;
    for (int a = 0; a < 3; ++a) {
      p[a] = 0.5 * s->grid[a] - cam->eye[a];
      F2 += (double)cam->forward[a] * cam->forward[a];
      R2 += (double)cam->right[a] * cam->right[a];
      U2 += (double)cam->up[a] * cam->up[a];
      pF += p[a] * cam->forward[a];
      pR += p[a] * cam->right[a];
      pU += p[a] * cam->up[a];
    }
    double u = 0, v = 0;
    bool ok = R2 > 0 && U2 > 0;
    if (ok && !cam->orthographic) {
      ok = F2 > 0 && pF > 0;
      const double sc = ok ? pF / F2 : 1.0;
      u = pR / (sc * R2);
      v = pU / (sc * U2);
    } else if (ok) {
      u = pR / R2;
      v = pU / U2;
    }
    if (ok && std::isfinite(u) && std::isfinite(v)) {
      const double fi = (u + 1.0) * 0.5 * R.W, fj = (1.0 - v) * 0.5 * R.H;
      const int ty_n = R.n_tiles / R.tiles_x;
      int cx = (int)std::floor(fi / (8.0 * wx)), cy = (int)std::floor(fj / (8.0 * wy));
      cx = std::min(std::max(cx, 0), R.tiles_x - 1);
      cy = std::min(std::max(cy, 0), ty_n - 1);
      R.spiral_x = cx;
      R.spiral_y = cy;
      R.spiral_r = std::max(std::max(cx, R.tiles_x - 1 - cx), std::max(cy, ty_n - 1 - cy));
      // projected radius of the grid's bounding sphere, in tiles; the rings
      // within kSplitFrac of it are split when the frame's estimated work
      // (rays over the grid times records per grid column) is small
      double rad = 0;
      for (int a = 0; a < 3; ++a) rad += 0.25 * (double)s->grid[a] * s->grid[a];
      rad = std::sqrt(rad);
      const double scale = cam->orthographic ? 1.0 : pF / F2;
      const double r_tiles = rad * R.W / (16.0 * wx * scale * std::sqrt(R2));
      const double cols = std::cbrt((double)s->grid[0] * s->grid[1] * s->grid[2]);
      const double covered = std::min((double)R.n_tiles, M_PI * r_tiles * r_tiles);
      const double work = 64.0 * covered * (double)s->n_records / (cols * cols);
      if (wx == 1 && wy == 1 && !R.opaque && std::isfinite(r_tiles) &&
          work <= kSplitMaxWork) {
        const int rs = (int)std::min(kSplitFrac * r_tiles, (double)R.spiral_r);
        R.split_n = (2 * rs + 1) * (2 * rs + 1);
        R.split_s = work <= kSplit4MaxWork ? 4 : 2;
      }
    }
  }
  *Rp = R;
  return LS_OK;
}

int launch_render(const RenderArgs& R, hipStream_t st) {
  const int tiles_y = R.n_tiles / R.tiles_x;
  const unsigned blocks =
      R.order ? (unsigned)(R.n_tiles + (R.top_s - 1) * R.top_n + R.split_n * (R.split_s - 1))
      : R.spiral_r >= 0 ? (unsigned)((2 * R.spiral_r + 1) * (2 * R.spiral_r + 1) +
                                     R.split_n * (R.split_s - 1))
                        : (unsigned)(kXcds * ((tiles_y + kXcds - 1) / kXcds) * R.tiles_x);
  const unsigned threads = (unsigned)(64 * R.wx * R.wy);
  const size_t lds = merge_lds_bytes(threads);
  const dim3 grid(blocks), block(threads);
  const bool vdi = view_dependent(R), cnt = R.counters != nullptr;
  // one instance per (mode, counters, view-dependent illumination): the
  // per-fragment illumination code stays out of the other instances
  if (R.mode == 0) {
    if (vdi) {
      if (cnt) hipLaunchKernelGGL((k_render<0, true, true>), grid, block, lds, st, R);
      else hipLaunchKernelGGL((k_render<0, false, true>), grid, block, lds, st, R);
    } else {
      if (cnt) hipLaunchKernelGGL((k_render<0, true, false>), grid, block, lds, st, R);
      else hipLaunchKernelGGL((k_render<0, false, false>), grid, block, lds, st, R);
    }
  } else {
    if (vdi) {
      if (cnt) hipLaunchKernelGGL((k_render<1, true, true>), grid, block, lds, st, R);
      else hipLaunchKernelGGL((k_render<1, false, true>), grid, block, lds, st, R);
    } else {
      if (cnt) hipLaunchKernelGGL((k_render<1, true, false>), grid, block, lds, st, R);
      else hipLaunchKernelGGL((k_render<1, false, false>), grid, block, lds, st, R);
    }
  }
  LS_HIP(hipGetLastError());
  return LS_OK;
}

namespace {

// Launch-order state per (device, stream): the tile times of the stream's
// last kOrderViews distinct views (least recently used replaced), and one
// work buffer (bucket counters, per-tile buckets, the order). Work queued on
// one stream runs in order, so its frames share these buffers. A buffer that
// must grow is replaced after synchronising the stream; all are kept until
// the process ends.
constexpr int kOrderViews = 64;

struct OrderKey {
  int32_t grid[3];
  int64_t n_records;
  ls_camera cam;
  ls_render_params params;
  int32_t split;
};

// Same view but for a slightly moved camera: everything else equal, the eye
// within 2 % of the grid's diagonal and each camera vector within 2 degrees
// and 1 % in length of the other's.
bool near_view(const OrderKey& a, const OrderKey& b) {
  OrderKey x = a, y = b;
  std::memset(&x.cam, 0, sizeof(x.cam));
  std::memset(&y.cam, 0, sizeof(y.cam));
  if (std::memcmp(&x, &y, sizeof(x)) != 0) return false;
  const ls_camera &p = a.cam, &q = b.cam;
  if (p.width != q.width || p.height != q.height || p.orthographic != q.orthographic)
    return false;
  double diag2 = 0, de2 = 0;
  for (int k = 0; k < 3; ++k) {
    diag2 += (double)a.grid[k] * a.grid[k];
    de2 += ((double)p.eye[k] - q.eye[k]) * ((double)p.eye[k] - q.eye[k]);
  }
  if (!(de2 <= 4e-4 * diag2)) return false;
  const float* const u[3] = {p.forward, p.right, p.up};
  const float* const w[3] = {q.forward, q.right, q.up};
  for (int k = 0; k < 3; ++k) {
    double uu = 0, ww = 0, uw = 0;
    for (int c = 0; c < 3; ++c) {
      uu += (double)u[k][c] * u[k][c];
      ww += (double)w[k][c] * w[k][c];
      uw += (double)u[k][c] * w[k][c];
    }
    if (!(uu > 0 && ww > 0)) return false;
    const double r = std::sqrt(ww / uu);
    if (!(r > 0.99 && r < 1.01)) return false;
    if (!(uw / std::sqrt(uu * ww) >= 0.99939)) return false;   // cos 2 degrees
  }
  return true;
}

struct ViewTimes {
  OrderKey key;
  void* times = nullptr;
  size_t bytes = 0;
  uint64_t used = 0;
};

struct StreamOrder {
  void* work = nullptr;
  size_t work_bytes = 0;
  std::vector<ViewTimes> views;
  uint64_t clock = 0;
};

std::mutex g_order_mu;
std::map<std::pair<int, hipStream_t>, StreamOrder> g_order;

// Replaces *p (after synchronising st) by a block of at least `bytes`.
int grow(void** p, size_t* have, size_t bytes, hipStream_t st) {
  if (*have >= bytes) return LS_OK;
  if (*p) {
    LS_HIP(hipStreamSynchronize(st));
    pool_free(*p);
    *p = nullptr;
    *have = 0;
  }
  return pool_alloc(bytes, p, have);
}

// Workgroups the plain launch keeps resident on the device at once.
int resident_blocks(int* out) {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  LS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it == cache.end()) {
    hipDeviceProp_t prop;
    LS_HIP(hipGetDeviceProperties(&prop, dev));
    int per_cu = 0;
    LS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(k_render<0, false, false>), kWave,
        merge_lds_bytes(kWave)));
    it = cache.emplace(dev, prop.multiProcessorCount * (per_cu > 0 ? per_cu : 1)).first;
  }
  *out = it->second;
  return LS_OK;
}

// Plain frames with more workgroups than the device holds at once: tile
// times are measured, and a frame of a view the stream rendered before (same
// set shape, image, camera and parameters), or of one with the camera moved
// slightly, is launched in the order of those times.
int tile_order(const ls_lineset* s, const ls_camera* cam, const ls_render_params* p,
               RenderArgs& R, hipStream_t st) {
  int resident = 0, rc;
  if ((rc = resident_blocks(&resident))) return rc;
  if ((int64_t)R.n_tiles + (int64_t)R.split_n * (R.split_s - 1) <= resident) return LS_OK;
  OrderKey key;
  std::memset(&key, 0, sizeof(key));
  for (int a = 0; a < 3; ++a) key.grid[a] = s->grid[a];
  key.n_records = s->n_records;
  key.cam = *cam;
  key.params = *p;
  key.split = R.split_n * 8 + R.split_s;
  int dev = 0;
  LS_HIP(hipGetDevice(&dev));
  const int64_t n = R.n_tiles;
  std::lock_guard<std::mutex> lk(g_order_mu);
  StreamOrder& so = g_order[{dev, st}];
  ++so.clock;
  int v = -1;
  for (int k = 0; k < (int)so.views.size(); ++k)
    if (std::memcmp(&so.views[k].key, &key, sizeof(key)) == 0) v = k;
  // else a view with the camera only slightly moved (a camera in motion):
  // its times order this frame, and the entry follows the camera
  for (int k = 0; v < 0 && k < (int)so.views.size(); ++k)
    if (near_view(so.views[k].key, key)) {
      v = k;
      so.views[v].key = key;
    }
  bool repeat = v >= 0;
  if (!repeat) {
    if ((int)so.views.size() < kOrderViews) {
      so.views.emplace_back();
      v = (int)so.views.size() - 1;
    } else {
      v = 0;
      for (int k = 1; k < kOrderViews; ++k)
        if (so.views[k].used < so.views[v].used) v = k;
    }
    so.views[v].key = key;
  }
  ViewTimes& vt = so.views[v];
  vt.used = so.clock;
  if (vt.bytes < sizeof(uint32_t) * n) repeat = false;
  if ((rc = grow(&vt.times, &vt.bytes, sizeof(uint32_t) * n, st))) return rc;
  // work: hist, cursor (256 words each), order (int32 per tile), bucket
  // (uint8 per tile)
  if ((rc = grow(&so.work, &so.work_bytes,
                 sizeof(uint32_t) * (2 * kCostBuckets + n) + (size_t)n, st)))
    return rc;
  uint32_t* times = static_cast<uint32_t*>(vt.times);
  uint32_t* hist = static_cast<uint32_t*>(so.work);
  uint32_t* cursor = hist + kCostBuckets;
  int32_t* order = reinterpret_cast<int32_t*>(cursor + kCostBuckets);
  uint8_t* bucket = reinterpret_cast<uint8_t*>(order + n);
  // first frame of a transparent view: estimated costs order it
  const bool probe = !repeat && !R.opaque;
  if (probe) {
    const unsigned pb = (unsigned)((n + kBlock / kProbeLanes - 1) / (kBlock / kProbeLanes));
    hipLaunchKernelGGL(k_tile_probe, dim3(pb), dim3(kBlock), 0, st, R, times);
    LS_HIP(hipGetLastError());
  }
  if (repeat || probe) {
    if ((rc = fill_u32(hist, 0u, 2 * kCostBuckets, st))) return rc;
    const unsigned tb = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_tile_hist, dim3(tb), dim3(kBlock), 0, st, times, (int32_t)n, bucket,
                       hist);
    hipLaunchKernelGGL(k_tile_order, dim3(tb), dim3(kBlock), 0, st, times, bucket, (int32_t)n,
                       hist, cursor, order);
    LS_HIP(hipGetLastError());
    R.order = order;
    // the longest measured tiles split four ways in frames split two ways,
    // eight ways in frames not split at all (the light frames split four
    // ways throughout already). Not in an estimated frame: a split tile's
    // parts add their durations, up to nsub times the tile's unsplit
    // duration (each part takes about as long as its slowest ray), which
    // keeps the longest tiles on top once measured but would keep tiles the
    // estimate wrongly put on top there too.
    if (probe) {
    } else if (R.split_s == 2) {
      R.top_n = std::min(kTopTiles, R.split_n);
      R.top_s = 4;
      R.split_n -= R.top_n;
    } else if (R.split_s == 1) {
      R.top_n = (int)std::min<int64_t>(kTopTiles, n);
      R.top_s = 8;
    }
  } else {
    if ((rc = fill_u32(times, 0u, n, st))) return rc;
  }
  R.times = times;
  return LS_OK;
}

}  // namespace

int render_frame(const ls_lineset* s, const ls_camera* cam, const ls_render_params* p, float* out,
                 RenderCounters* dev_counters, hipStream_t st) {
  RenderArgs R;
  make_render_args(s, cam, p, out, 1, 1, dev_counters, &R);
  int rc;
  if (R.spiral_r >= 0 && (rc = tile_order(s, cam, p, R, st))) return rc;
  return launch_render(R, st);
}

BatchQueues make_queues(int total_tiles) {
  BatchQueues q{};
  for (int k = 0; k < kXcds; ++k) {
    const int b = (int)((int64_t)total_tiles * k / kXcds);
    const int e = (int)((int64_t)total_tiles * (k + 1) / kXcds);
    q.begin[k] = b;
    q.len[k] = e - b;
  }
  return q;
}

int launch_render_batch(const RenderArgs* dev_views, const int32_t* dev_tile_start, int n_views,
                        const BatchQueues& q, unsigned* dev_queue, const BatchPlan& plan,
                        bool count, bool vdi, hipStream_t st) {
  const unsigned threads = (unsigned)(64 * plan.wx * plan.wy);
  const size_t lds = merge_lds_bytes(threads);
  const dim3 grid(plan.blocks), block(threads);
  if (vdi) {
    if (count)
      hipLaunchKernelGGL((k_render_batch<true, true>), grid, block, lds, st, dev_views,
                         dev_tile_start, n_views, q, dev_queue);
    else
      hipLaunchKernelGGL((k_render_batch<false, true>), grid, block, lds, st, dev_views,
                         dev_tile_start, n_views, q, dev_queue);
  } else {
    if (count)
      hipLaunchKernelGGL((k_render_batch<true, false>), grid, block, lds, st, dev_views,
                         dev_tile_start, n_views, q, dev_queue);
    else
      hipLaunchKernelGGL((k_render_batch<false, false>), grid, block, lds, st, dev_views,
                         dev_tile_start, n_views, q, dev_queue);
  }
  LS_HIP(hipGetLastError());
  return LS_OK;
}

int render_merge_slots() { return kMergeSlots; }

int batch_blocks_per_cu(int wx, int wy, bool vdi, int* out) {
  int n = 0;
  const void* k = vdi ? (const void*)k_render_batch<false, true> : (const void*)k_render_batch<false, false>;
  LS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64 * wx * wy,
                                                      merge_lds_bytes(64u * wx * wy)));
  *out = n > 0 ? n : 1;
  return LS_OK;
}
