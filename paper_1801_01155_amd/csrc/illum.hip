// Per-voxel ambient occlusion and soft-shadow grids by cone tracing the
// density pyramid (sections "Shadow simulation", "Ambient occlusion",
// "Illumination effects") on gfx950.
//
// From the voxel centre p along a unit direction u, samples are taken at
// distance s with cone diameter D = max(1, aperture * s) on level
// min(L, floor(log2 D)) (cell-centred trilinear, clamp to edge); each adds
// rho * D to the occlusion, then s += D, while s < s_max and the point is
// inside the grid; occlusion saturates at 1. Sample positions and lattice
// inside-the-grid tests are made in fp64; lattice coordinates and weights in
// fp32 relative to the voxel, accumulation in fp32. One thread per voxel; the
// pyramid levels are small enough past level 2 to stay in L2.
#include "ls_internal.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int kBlock = 256;
constexpr int kMaxCones = 32;

struct Pyramid {
  const float* rho;
  int32_t n_levels;
  int32_t dims[LS_MAX_LEVELS][3];
  int64_t off[LS_MAX_LEVELS];
  int32_t g[3];
};

struct Cones {
  int32_t n;
  double s_max;
  double aperture;
  double dir[kMaxCones][3];
};

// Sample schedule along a cone: distances s_k < s_max, diameters D_k and
// levels l_k. With D = max(1, aperture s) and s_{k+1} = s_k + D_k it depends
// only on the aperture and s_max, so all cones and voxels share it.
constexpr int kMaxSamples = 48;
struct Sched {
  int32_t n;
  float reach;             // s_max of the schedule + 1 (voxels farther from every face skip inside tests)
  float s[kMaxSamples];
  float D[kMaxSamples];
  int32_t lv[kMaxSamples];
};

// Trilinear sample of level `lv` at the point v + f (v the voxel corner,
// integer; f a local offset in voxel units). The level coordinate is formed
// from v's low bits and f in fp32, so it keeps ~1e-7 cell precision at every
// level. The two x-neighbour taps are one 8-byte load: the pair starts at
// j = clamp(i0, 0, D - 2) and the x weight is clamp(x - j, 0, 1), which is
// clamp-to-edge interpolation. Level sizes are below 2^31: int32 indices.
__device__ inline float sample(const Pyramid& P, int lv, const int32_t v[3], const float f[3]) {
  const float scale = __builtin_ldexpf(1.0f, -lv);
  const int32_t mask = (1 << lv) - 1;
  const int32_t dx = P.dims[lv][0], dy = P.dims[lv][1], dz = P.dims[lv][2];
  int32_t i0[3];
  float fr[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float x = ((float)(v[a] & mask) + f[a]) * scale - 0.5f;
    const float fl = floorf(x);
    fr[a] = x - fl;
    i0[a] = (v[a] >> lv) + (int32_t)fl;
  }
  const float* r = P.rho + P.off[lv];
  const int32_t y0 = min(max(i0[1], 0), dy - 1), y1 = min(max(i0[1] + 1, 0), dy - 1);
  const int32_t z0 = min(max(i0[2], 0), dz - 1), z1 = min(max(i0[2] + 1, 0), dz - 1);
  const int32_t rows[4] = {(y0 + dy * z0) * dx, (y1 + dy * z0) * dx, (y0 + dy * z1) * dx,
                           (y1 + dy * z1) * dx};
  float c[4];
  if (dx >= 2) {
    const int32_t j = min(max(i0[0], 0), dx - 2);
    const float wx = fminf(fmaxf((float)(i0[0] - j) + fr[0], 0.f), 1.f);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float2 pr;
      __builtin_memcpy(&pr, r + rows[k] + j, sizeof(pr));
      c[k] = __builtin_fmaf(wx, pr.y - pr.x, pr.x);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = r[rows[k]];
  }
  const float c0 = __builtin_fmaf(fr[1], c[1] - c[0], c[0]);
  const float c1 = __builtin_fmaf(fr[1], c[3] - c[2], c[2]);
  return __builtin_fmaf(fr[2], c1 - c0, c0);
}

// Occlusion along one cone from the centre of voxel v. A sample point
// p + s u (p the voxel centre) is tested against the grid in fp64, the same
// expression as the definition; voxels farther than the schedule's reach
// from every face have all samples inside and skip the test. The sample
// itself uses the local offset f = 0.5 + s u in fp32.
__device__ inline float cone(const Pyramid& P, const Sched& S, const int32_t v[3], const double u[3],
                             bool near_face) {
  const float u32[3] = {(float)u[0], (float)u[1], (float)u[2]};
  float occ = 0.f;
  for (int k = 0; k < S.n; ++k) {
    const float s = S.s[k];
    if (near_face) {
      bool inside = true;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double x = ((double)v[a] + 0.5) + (double)s * u[a];
        inside &= x >= 0.0 && x < (double)P.g[a];
      }
      if (!inside) break;
    }
    const float f[3] = {0.5f + s * u32[0], 0.5f + s * u32[1], 0.5f + s * u32[2]};
    occ = __builtin_fmaf(sample(P, S.lv[k], v, f), S.D[k], occ);
    if (occ >= 1.f) break;
  }
  return occ < 1.f ? occ : 1.f;
}

__device__ inline bool near_any_face(const Pyramid& P, const int32_t v[3], float reach) {
  bool n = false;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    n |= (float)v[a] < reach || (float)(P.g[a] - 1 - v[a]) < reach;
  return n;
}

__global__ __launch_bounds__(kBlock) void k_ao(Pyramid P, Cones C, Sched S, int64_t nvox,
                                               float* ao) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nvox) return;
  const int32_t p[3] = {(int32_t)(v % P.g[0]), (int32_t)((v / P.g[0]) % P.g[1]),
                        (int32_t)(v / ((int64_t)P.g[0] * P.g[1]))};
  const bool near_face = near_any_face(P, p, S.reach);
  float sum = 0.f;
  for (int c = 0; c < C.n; ++c) sum += cone(P, S, p, C.dir[c], near_face);
  ao[v] = 1.f - sum / (float)C.n;
}

__global__ __launch_bounds__(kBlock) void k_shadow(Pyramid P, Cones C, Sched S, int64_t nvox,
                                                   float* sh) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nvox) return;
  const int32_t p[3] = {(int32_t)(v % P.g[0]), (int32_t)((v / P.g[0]) % P.g[1]),
                        (int32_t)(v / ((int64_t)P.g[0] * P.g[1]))};
  sh[v] = 1.f - cone(P, S, p, C.dir[0], near_any_face(P, p, S.reach));
}

// LDS-tiled cone tracing by voxel columns. A block handles a tile of
// 16 x 16 x 8 voxels; each of its 256 threads owns one (x, y) column of the
// tile and walks its 8 voxels along z. Every sample k of every cone lies
// within s_k (voxel units) of its voxel, so on level l the taps of the whole
// tile fall inside a box of (tile extent on l) + 2 m_l cells per axis,
// m_l = ceil(max s_k / 2^l) + 2 over the samples on l. The block first
// copies each level's box into LDS (coordinates clamped to the level, which
// makes plain trilinear interpolation of the copy the clamp-to-edge
// interpolation of the level).
//
// With the tile origin a multiple of 8 and every level at most 3, a sample's
// lattice coordinate on axis a depends only on the cone, the sample and the
// voxel's position p_a = v_a - t0_a in the tile: x = ((p_a mod 2^l) + 0.5 +
// s u_a) 2^-l - 0.5 (the arithmetic of sample()), cell floor(x) + (p_a >> l)
// and weight frac(x). Along z, the voxels of one phase ph = p_z mod 2^l take
// consecutive cells c_ph + (p_z >> l), and c_ph is c_0 or c_0 + 1. So for
// one cone and sample a thread interpolates the (x, y) bilinear value of the
// few z-planes c_0 .. c_0 + (8 >> l) + 1 once, and each voxel of the column
// takes its z interpolation from two of them: the 8 voxels of a column share
// 9 planes on level 0 and 3 on level 3, where per-voxel trilinear samples
// would read 8 taps each. The x and y taps (per thread) come from a small
// table in global memory, the z taps, plane choices and inside-the-grid
// ranges of each (cone, sample) are wave-uniform (scalar loads). The order of
// the interpolations (x, then y, then z) is that of sample().
//
// The inside-the-grid test of sample k (the fp64 expression of the
// definition) holds on an interval of each voxel coordinate; the table
// kernel finds the intervals by bisection, so the kernel compares integers.
// A sample outside the grid adds nothing, and since the test is monotone
// along the cone every later sample is outside too, which is where the
// definition stops. Occlusion terms are non-negative, so accumulating past
// saturation and clamping at the end gives the definition's value.
constexpr int kColX = 16, kColY = 16, kColZ = 8;
constexpr int kColThreads = kColX * kColY;
constexpr int kColTab = kColX > kColY ? kColX : kColY;   // x / y tap entries per axis
constexpr int kColSlots = 4;             // levels 0..3
constexpr int kColLdsBytes = 65536;
constexpr int kColMaxSamples = 8;        // instantiated schedule lengths

struct ColLevels {
  int32_t n;                        // distinct levels of the schedule
  int32_t lv[kColSlots];
  int32_t m[kColSlots];             // margin per side, cells
  int32_t sz[kColSlots][3];         // box extent per axis, cells
  int32_t base[kColSlots + 1];      // LDS offset (floats) of each box; base[n] = total
  int32_t slot[kMaxSamples];        // box of each sample
  int32_t tiles[3];
  int32_t tiles_per_xcd;
};

// Tap offset (bytes, within the sample's box) and weight of one axis.
struct Tap {
  int32_t off;
  float w;
};

// Per (cone, sample): the z planes and the inside-the-grid ranges.
struct alignas(64) ZRec {
  int32_t c0;          // byte offset in LDS of plane c_0 (box base included)
  int32_t delta;       // bit ph: c_ph - c_0 (0 or 1)
  int32_t lo[3], hi[3];  // inside-the-grid voxel ranges (lo > hi: none)
  float w[8];          // z weight of phase ph
};
static_assert(sizeof(ZRec) == 64, "ZRec is one 64-byte scalar load");

// Planes a column interpolates on level L for 8 voxels: (8 >> L) + 1 on
// level 0 (one phase), one more on coarser levels (the phases' c_ph may
// exceed c_0 by one).
template <int L>
constexpr int col_planes() {
  return L == 0 ? 9 : (kColZ >> L) + 2;
}

__host__ __device__ inline int col_planes_rt(int L) { return L == 0 ? 9 : (kColZ >> L) + 2; }

// Table layout (global memory): ZRec[n_cones * kN], then
// Tap[n_cones * kN][2][kColTab] (x taps by p_x, y taps by p_y).
inline size_t col_table_bytes(int n_cones, int n_samples) {
  return (size_t)n_cones * n_samples * (sizeof(ZRec) + 2 * kColTab * sizeof(Tap));
}
constexpr size_t kMaxTabBytes = (size_t)kMaxCones * kColMaxSamples * (sizeof(ZRec) + 2 * kColTab * sizeof(Tap));

// Smallest v in [0, g) whose sample coordinate (v + 0.5) + s u is >= 0, and
// the largest whose coordinate is < g (the coordinate grows with v).
__device__ inline void inside_range(double s, double u, int32_t g, int32_t* lo, int32_t* hi) {
  int32_t a = 0, b = g;                  // first v with x >= 0 lies in [a, b]
  while (a < b) {
    const int32_t mid = (a + b) >> 1;
    if (((double)mid + 0.5) + s * u >= 0.0) b = mid; else a = mid + 1;
  }
  *lo = a;
  a = -1;
  b = g - 1;                             // last v with x < g lies in [a, b]
  while (a < b) {
    const int32_t mid = (a + b + 1) >> 1;
    if (((double)mid + 0.5) + s * u < (double)g) a = mid; else b = mid - 1;
  }
  *hi = a;
}

// Lattice cell (before the tile offset) and weight of axis coordinate p on
// level lv for local offset f; the arithmetic of sample().
__device__ inline void col_coord(int32_t p, int lv, float f, float* fl, float* w) {
  const float x = ((float)(p & ((1 << lv) - 1)) + f) * __builtin_ldexpf(1.0f, -lv) - 0.5f;
  *fl = floorf(x);
  *w = x - *fl;
}

template <int kN>
__global__ __launch_bounds__(kColThreads) void k_col_table(Pyramid P, Cones C, Sched S,
                                                           ColLevels CL, ZRec* zt, Tap* xyt) {
  const int n_ck = C.n * kN;
  for (int e = threadIdx.x; e < n_ck * 2 * kColTab; e += kColThreads) {
    const int p = e % kColTab, a = (e / kColTab) & 1, ck = e / (2 * kColTab);
    const int c = ck / kN, k = ck % kN;
    const int q = CL.slot[k], lv = S.lv[k];
    const float f = 0.5f + S.s[k] * (float)C.dir[c][a];
    float fl, w;
    col_coord(p, lv, f, &fl, &w);
    const int32_t li = min(max((p >> lv) + (int32_t)fl + CL.m[q], 0), CL.sz[q][a] - 2);
    const int32_t stride = a == 0 ? 1 : CL.sz[q][0];
    xyt[e] = Tap{li * stride * (int32_t)sizeof(float), w};
  }
  for (int ck = threadIdx.x; ck < n_ck; ck += kColThreads) {
    const int c = ck / kN, k = ck % kN;
    const int q = CL.slot[k], lv = S.lv[k];
    const float f = 0.5f + S.s[k] * (float)C.dir[c][2];
    ZRec r{};
    float fl0, w;
    col_coord(0, lv, f, &fl0, &w);
    const int nph = 1 << lv;
    for (int ph = 0; ph < 8; ++ph) {
      float fl;
      col_coord(ph, lv, f, &fl, &w);
      r.w[ph] = ph < nph ? w : 0.f;
      if (ph < nph && fl > fl0) r.delta |= 1 << ph;
    }
    const int32_t c0 = min(max((int32_t)fl0 + CL.m[q], 0), CL.sz[q][2] - col_planes_rt(lv));
    r.c0 = (CL.base[q] + c0 * CL.sz[q][0] * CL.sz[q][1]) * (int32_t)sizeof(float);
    for (int ax = 0; ax < 3; ++ax)
      inside_range((double)S.s[k], C.dir[c][ax], P.g[ax], &r.lo[ax], &r.hi[ax]);
    zt[ck] = r;
  }
}

// One (cone, sample) on level L for a thread's column: the planes' bilinear
// values, then each voxel's z interpolation. Dm is the sample's weight D, or
// 0 when the column is outside the grid in x or y.
// kRowB, kPlaneB > 0: the box strides (bytes) are compile-time constants, so
// every read of the sample is an immediate offset from one address.
template <int L, int kRowB = 0, int kPlaneB = 0>
__device__ inline void col_sample(const char* box, const ZRec& z, int32_t plane_bytes,
                                  int32_t row_bytes, float wx, float wy, float Dm, int32_t vz0,
                                  float occ[kColZ]) {
  constexpr int R = col_planes<L>();
  if (kRowB > 0) {
    plane_bytes = kPlaneB;
    row_bytes = kRowB;
  }
  float pl[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const float* r0 = reinterpret_cast<const float*>(box + j * plane_bytes);
    const float* r1 = reinterpret_cast<const float*>(box + j * plane_bytes + row_bytes);
    const float a = __builtin_fmaf(wx, r0[1] - r0[0], r0[0]);
    const float b = __builtin_fmaf(wx, r1[1] - r1[0], r1[0]);
    pl[j] = __builtin_fmaf(wy, b - a, a);
  }
  float val[kColZ];
#pragma unroll
  for (int pz = 0; pz < kColZ; ++pz) {
    constexpr int kMask = (1 << L) - 1;
    const int ph = pz & kMask, i = pz >> L;
    float p0 = pl[i], p1 = pl[i + 1];
    if (L > 0 && ((z.delta >> ph) & 1)) {
      p0 = pl[i + 1];
      p1 = pl[(L > 0 ? i + 2 : i + 1)];
    }
    val[pz] = __builtin_fmaf(z.w[ph], p1 - p0, p0);
  }
  if (vz0 >= z.lo[2] && vz0 + kColZ - 1 <= z.hi[2]) {
    // the common case: every voxel of the column segment is inside along z
#pragma unroll
    for (int pz = 0; pz < kColZ; ++pz) occ[pz] = __builtin_fmaf(val[pz], Dm, occ[pz]);
  } else {
#pragma unroll
    for (int pz = 0; pz < kColZ; ++pz) {
      const int32_t vz = vz0 + pz;
      const float d = vz >= z.lo[2] && vz <= z.hi[2] ? Dm : 0.f;
      occ[pz] = __builtin_fmaf(val[pz], d, occ[pz]);
    }
  }
}

// kN = S.n: the sample loop is unrolled, so the schedule's per-sample
// constants stay in scalar registers for the whole block. With kShadow the
// last cone of C is the shadow cone: its first kN samples are the AO
// schedule's (same distances, diameters and levels, so the same boxes) and
// are traced like the AO cones; its remaining samples SH[kN..) lie on
// levels >= 3 and are interpolated per column (see below). AO averages the
// other C.n - 1 cones.
// kStd: the schedule samples levels 0, 1, 2, 3 (one sample each) with box
// margin 3 on every level (the 16-cone radius-15 AO of aperture 1), so box
// k has the compile-time extent kStdBox[k] and sample k the level k.
constexpr int kStdBox[4][3] = {{22, 22, 14}, {14, 14, 10}, {10, 10, 8}, {8, 8, 7}};
constexpr int std_row(int q) { return kStdBox[q][0] * 4; }
constexpr int std_plane(int q) { return kStdBox[q][0] * kStdBox[q][1] * 4; }

template <int kN, bool kShadow, bool kStd>
__global__ __launch_bounds__(kColThreads) void k_cones_col(Pyramid P, Cones C, Sched S,
                                                           ColLevels CL,
                                                           const ZRec* __restrict__ zt,
                                                           const Tap* __restrict__ xyt,
                                                           float* out, Sched SH, float* sh_out) {
  extern __shared__ float lds[];
  // XCD x (= block mod 8) works through a contiguous run of tiles, so the
  // boxes neighbouring tiles share are fetched into one L2.
  const int b = blockIdx.x;
  const int tile = (b % 8) * CL.tiles_per_xcd + b / 8;
  const int nt = CL.tiles[0] * CL.tiles[1] * CL.tiles[2];
  if (tile >= nt) return;
  const int32_t t0[3] = {kColX * (tile % CL.tiles[0]),
                         kColY * ((tile / CL.tiles[0]) % CL.tiles[1]),
                         kColZ * (tile / (CL.tiles[0] * CL.tiles[1]))};
  // box copy: one flat loop over each box's cells (compile-time boxes divide
  // by constants)
  if (kStd) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int sx = kStdBox[q][0], sy = kStdBox[q][1], n = sx * sy * kStdBox[q][2];
      const int32_t dx = P.dims[q][0], dy = P.dims[q][1], dz = P.dims[q][2];
      const int32_t o0 = (t0[0] >> q) - 3, o1 = (t0[1] >> q) - 3, o2 = (t0[2] >> q) - 3;
      const float* __restrict__ rho = P.rho + P.off[q];
      float* box = lds + CL.base[q];
      // unrolled: eight independent loads in flight per thread (LoD + AO +
      // shadow 0.69 -> 0.63 ms at 256^3, 6.2 -> 5.4 ms at 512^3)
#pragma unroll 8
      for (int i = threadIdx.x; i < n; i += kColThreads) {
        const int x = i % sx, y = (i / sx) % sy, z = i / (sx * sy);
        const int32_t gx = min(max(o0 + x, 0), dx - 1), gy = min(max(o1 + y, 0), dy - 1),
                      gz = min(max(o2 + z, 0), dz - 1);
        box[i] = rho[((int64_t)gz * dy + gy) * dx + gx];
      }
    }
  } else {
    for (int q = 0; q < CL.n; ++q) {
      const int lv = CL.lv[q], sx = CL.sz[q][0], sxy = sx * CL.sz[q][1];
      const int n = sxy * CL.sz[q][2];
      const int32_t dx = P.dims[lv][0], dy = P.dims[lv][1], dz = P.dims[lv][2];
      const int32_t o0 = (t0[0] >> lv) - CL.m[q], o1 = (t0[1] >> lv) - CL.m[q],
                    o2 = (t0[2] >> lv) - CL.m[q];
      const float* __restrict__ rho = P.rho + P.off[lv];
      float* box = lds + CL.base[q];
      // cell i = x + sx (y + sy z) of a box below 2^14 cells: (i + 0.5) / s
      // lies at least 0.5 / s from an integer, far beyond the fp32 error of
      // (i + 0.5) * (1 / s), so the truncation is the exact quotient
      const float isx = 1.f / (float)sx, isxy = 1.f / (float)sxy;
#pragma unroll 8
      for (int i = threadIdx.x; i < n; i += kColThreads) {
        const int z = (int)(((float)i + 0.5f) * isxy), rem = i - z * sxy;
        const int y = (int)(((float)rem + 0.5f) * isx), x = rem - y * sx;
        const int32_t gx = min(max(o0 + x, 0), dx - 1), gy = min(max(o1 + y, 0), dy - 1),
                      gz = min(max(o2 + z, 0), dz - 1);
        box[i] = rho[((int64_t)gz * dy + gy) * dx + gx];
      }
    }
  }
  __syncthreads();
  const int px = threadIdx.x & (kColX - 1), py = threadIdx.x / kColX;
  const int32_t vx = t0[0] + px, vy = t0[1] + py;
  const int n_ao = kShadow ? C.n - 1 : C.n;
  const float inv_n = 1.f / (float)n_ao;
  float sum[kColZ];
#pragma unroll
  for (int i = 0; i < kColZ; ++i) sum[i] = 0.f;
  float occ[kColZ];
  // the next cone's x/y taps are loaded while the current one is sampled
  Tap ntx[kN], nty[kN];
#pragma unroll
  for (int k = 0; k < kN; ++k) {
    ntx[k] = C.n > 0 ? xyt[2 * kColTab * k + px] : Tap{0, 0.f};
    nty[k] = C.n > 0 ? xyt[2 * kColTab * k + kColTab + py] : Tap{0, 0.f};
  }
  for (int c = 0; c < C.n; ++c) {
    const ZRec* zc = zt + kN * c;
    Tap ctx[kN], cty[kN];
#pragma unroll
    for (int k = 0; k < kN; ++k) {
      ctx[k] = ntx[k];
      cty[k] = nty[k];
    }
    if (c + 1 < C.n) {
      const Tap* tn = xyt + 2 * kColTab * kN * (c + 1);
#pragma unroll
      for (int k = 0; k < kN; ++k) {
        ntx[k] = tn[2 * kColTab * k + px];
        nty[k] = tn[2 * kColTab * k + kColTab + py];
      }
    }
#pragma unroll
    for (int i = 0; i < kColZ; ++i) occ[i] = 0.f;
#pragma unroll
    for (int k = 0; k < kN; ++k) {
      const ZRec z = zc[k];
      const Tap tx = ctx[k], ty = cty[k];
      const bool in_xy = vx >= z.lo[0] && vx <= z.hi[0] && vy >= z.lo[1] && vy <= z.hi[1];
      const float Dm = in_xy ? S.D[k] : 0.f;
      const int q = CL.slot[k];
      const int32_t row_bytes = CL.sz[q][0] * (int32_t)sizeof(float);
      const int32_t plane_bytes = row_bytes * CL.sz[q][1];
      const char* box = reinterpret_cast<const char*>(lds) + z.c0 + tx.off + ty.off;
      if (kStd) {
        switch (k) {   // k is a constant of the unrolled loop
          case 0: col_sample<0, std_row(0), std_plane(0)>(box, z, 0, 0, tx.w, ty.w, Dm, t0[2], occ); break;
          case 1: col_sample<1, std_row(1), std_plane(1)>(box, z, 0, 0, tx.w, ty.w, Dm, t0[2], occ); break;
          case 2: col_sample<2, std_row(2), std_plane(2)>(box, z, 0, 0, tx.w, ty.w, Dm, t0[2], occ); break;
          default: col_sample<3, std_row(3), std_plane(3)>(box, z, 0, 0, tx.w, ty.w, Dm, t0[2], occ); break;
        }
      } else {
        switch (S.lv[k]) {
          case 0: col_sample<0>(box, z, plane_bytes, row_bytes, tx.w, ty.w, Dm, t0[2], occ); break;
          case 1: col_sample<1>(box, z, plane_bytes, row_bytes, tx.w, ty.w, Dm, t0[2], occ); break;
          case 2: col_sample<2>(box, z, plane_bytes, row_bytes, tx.w, ty.w, Dm, t0[2], occ); break;
          default: col_sample<3>(box, z, plane_bytes, row_bytes, tx.w, ty.w, Dm, t0[2], occ); break;
        }
      }
    }
    if (kShadow && c == n_ao) break;   // the shadow cone's occ stays in occ[]
#pragma unroll
    for (int i = 0; i < kColZ; ++i) sum[i] += occ[i] < 1.f ? occ[i] : 1.f;
  }
  if (vx >= P.g[0] || vy >= P.g[1]) return;
  const int64_t col = vx + (int64_t)P.g[0] * vy, plane = (int64_t)P.g[0] * P.g[1];
#pragma unroll
  for (int i = 0; i < kColZ; ++i)
    if (t0[2] + i < P.g[2]) out[col + plane * (t0[2] + i)] = 1.f - sum[i] * inv_n;
  if (kShadow) {
    // The shadow cone's coarse samples (levels >= 3, the schedule's tail):
    // the column's 8 voxels share their x and y taps, and their level-z
    // cells c(pz) = (vz >> l) + floor(z) span at most two neighbours, so a
    // sample costs the (x, y) bilinear values of three planes (paired x
    // loads, clamp to edge as in sample()) and one z interpolation per
    // voxel, in sample()'s order. Outside samples add nothing (every later
    // one is outside too); saturation is applied at the end.
    const double* u = C.dir[n_ao];
    const float u32[3] = {(float)u[0], (float)u[1], (float)u[2]};
    for (int k = kN; k < SH.n; ++k) {
      const int lv = SH.lv[k];
      const float sk = SH.s[k], Dk = SH.D[k];
      const float scale = __builtin_ldexpf(1.0f, -lv);
      const int32_t mask = (1 << lv) - 1;
      const int32_t dx = P.dims[lv][0], dy = P.dims[lv][1], dz = P.dims[lv][2];
      // x and y taps of the column
      const float fx = 0.5f + sk * u32[0], fy = 0.5f + sk * u32[1], fz = 0.5f + sk * u32[2];
      const float xx = ((float)(vx & mask) + fx) * scale - 0.5f;
      const float xy = ((float)(vy & mask) + fy) * scale - 0.5f;
      const float flx = floorf(xx), fly = floorf(xy);
      const float frx = xx - flx, fry = xy - fly;
      const int32_t i0x = (vx >> lv) + (int32_t)flx, i0y = (vy >> lv) + (int32_t)fly;
      const int32_t y0 = min(max(i0y, 0), dy - 1), y1 = min(max(i0y + 1, 0), dy - 1);
      int32_t jx = 0;
      float wx = 0.f;
      if (dx >= 2) {
        jx = min(max(i0x, 0), dx - 2);
        wx = fminf(fmaxf((float)(i0x - jx) + frx, 0.f), 1.f);
      }
      // inside the grid in x and y (fp64, the definition's expression)
      const double ax = ((double)vx + 0.5) + (double)sk * u[0];
      const double ay = ((double)vy + 0.5) + (double)sk * u[1];
      const bool in_xy = ax >= 0.0 && ax < (double)P.g[0] && ay >= 0.0 && ay < (double)P.g[1];
      // z cells of the column's voxels: c(0) <= c(pz) <= c(0) + 1
      float frz[kColZ];
      int32_t iz0[kColZ];
#pragma unroll
      for (int i = 0; i < kColZ; ++i) {
        const int32_t vz = t0[2] + i;
        const float zz = ((float)(vz & mask) + fz) * scale - 0.5f;
        const float flz = floorf(zz);
        frz[i] = zz - flz;
        iz0[i] = (vz >> lv) + (int32_t)flz;
      }
      const float* __restrict__ r = P.rho + P.off[lv];
      float pl[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int32_t zj = min(max(iz0[0] + j, 0), dz - 1);
        const int32_t r0 = (y0 + dy * zj) * dx, r1 = (y1 + dy * zj) * dx;
        float c0, c1;
        if (dx >= 2) {
          float2 a, b;
          __builtin_memcpy(&a, r + r0 + jx, sizeof(a));
          __builtin_memcpy(&b, r + r1 + jx, sizeof(b));
          c0 = __builtin_fmaf(wx, a.y - a.x, a.x);
          c1 = __builtin_fmaf(wx, b.y - b.x, b.x);
        } else {
          c0 = r[r0];
          c1 = r[r1];
        }
        pl[j] = __builtin_fmaf(fry, c1 - c0, c0);
      }
      const double bz = (double)sk * u[2];
#pragma unroll
      for (int i = 0; i < kColZ; ++i) {
        const bool up = iz0[i] != iz0[0];
        const float p0 = up ? pl[1] : pl[0], p1 = up ? pl[2] : pl[1];
        const float val = __builtin_fmaf(frz[i], p1 - p0, p0);
        const double az = ((double)(t0[2] + i) + 0.5) + bz;
        const bool in = in_xy && az >= 0.0 && az < (double)P.g[2];
        occ[i] = in ? __builtin_fmaf(val, Dk, occ[i]) : occ[i];
      }
    }
#pragma unroll
    for (int i = 0; i < kColZ; ++i)
      if (t0[2] + i < P.g[2]) sh_out[col + plane * (t0[2] + i)] = 1.f - (occ[i] < 1.f ? occ[i] : 1.f);
  }
}

// Builds the schedule; fails (returns false) if it needs more than
// kMaxSamples entries. Every sample of a cone starting inside the grid lies
// within distance gmax * sqrt(3) of its voxel, so longer schedules stop there.
bool make_sched(const ls_lineset* s, double s_max, double aperture, Sched* S) {
  const int top = s->n_levels - 1;
  const double limit = 1.7320508075688772 * (double)std::max(s->grid[0], std::max(s->grid[1], s->grid[2])) + 2.0;
  S->n = 0;
  double t = 1.0;
  while (t < s_max && t <= limit) {
    if (S->n == kMaxSamples) return false;
    double D = aperture * t;
    D = D < 1.0 ? 1.0 : D;
    int lv = std::ilogb(D);
    lv = lv > top ? top : lv;
    S->s[S->n] = (float)t;
    S->D[S->n] = (float)D;
    S->lv[S->n] = lv;
    // distances and diameters must be exact in fp32 for the sample offsets
    // to match the definition
    if ((double)S->s[S->n] != t || (double)S->D[S->n] != D) return false;
    S->n++;
    t += D;
  }
  const double last = S->n ? (double)S->s[S->n - 1] : 0.0;
  S->reach = (float)(last + 2.0);
  return true;
}

Pyramid make_pyramid(const ls_lineset* s) {
  Pyramid P{};
  P.rho = s->lod_rho;
  P.n_levels = s->n_levels;
  for (int l = 0; l < s->n_levels; ++l) {
    for (int a = 0; a < 3; ++a) P.dims[l][a] = s->level_dims[l][a];
    P.off[l] = s->level_off[l];
  }
  for (int a = 0; a < 3; ++a) P.g[a] = s->grid[a];
  return P;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Boxes of the column kernel for schedule S; false if a level above 3 is
// sampled or the boxes exceed the LDS budget (then the untiled kernels run).
bool make_col_levels(const ls_lineset* s, const Sched& S, ColLevels* T) {
  *T = ColLevels{};
  for (int k = 0; k < S.n; ++k) {
    const int lv = S.lv[k];
    if (lv > 3) return false;
    int q = 0;
    while (q < T->n && T->lv[q] != lv) ++q;
    if (q == T->n) {
      T->lv[q] = lv;
      T->m[q] = 0;
      T->n++;
    }
    const int m = (int)std::ceil((double)S.s[k] / (double)(1 << lv)) + 2;
    T->m[q] = std::max(T->m[q], m);
    T->slot[k] = q;
  }
  const int ext[3] = {kColX, kColY, kColZ};
  int64_t total = 0;
  for (int q = 0; q < T->n; ++q) {
    for (int a = 0; a < 3; ++a) T->sz[q][a] = std::max(ext[a] >> T->lv[q], 1) + 2 * T->m[q];
    if (T->sz[q][2] < col_planes_rt(T->lv[q])) return false;
    T->base[q] = (int32_t)total;
    total += (int64_t)T->sz[q][0] * T->sz[q][1] * T->sz[q][2];
  }
  T->base[T->n] = (int32_t)total;
  if (total * 4 > kColLdsBytes) return false;
  for (int a = 0; a < 3; ++a) T->tiles[a] = (s->grid[a] + ext[a] - 1) / ext[a];
  const int64_t nt = (int64_t)T->tiles[0] * T->tiles[1] * T->tiles[2];
  T->tiles_per_xcd = (int32_t)((nt + 7) / 8);
  return true;
}

// Column kernel when it applies, else the per-voxel kernels (ao: k_ao, else
// k_shadow). With sh_out, C's last cone is the shadow cone with schedule SH
// (see k_cones_col); the call then fails with LS_EUNSUPPORTED instead of
// falling back when the column kernel does not apply.
int launch_cones(ls_lineset* s, const Cones& C, const Sched& S, float* out, hipStream_t st,
                 bool ao, const Sched* SH = nullptr, float* sh_out = nullptr) {
  // the column kernel pays one LDS fill per tile; with few samples per voxel
  // (the single shadow cone) direct gathers are cheaper
  ColLevels T;
  if (C.n >= 4 && S.n >= 1 && S.n <= kColMaxSamples && make_col_levels(s, S, &T)) {
    const size_t lds = sizeof(float) * (size_t)T.base[T.n];
    const dim3 grid((unsigned)(8 * T.tiles_per_xcd)), block(kColThreads);
    const Pyramid P = make_pyramid(s);
    // the plane and tap tables: one small launch, read by every block
    int rc;
    if (!s->cone_tab) {
      if ((rc = ls_alloc(s, &s->cone_tab, kMaxTabBytes))) return rc;
      s->cone_tab_bytes = kMaxTabBytes;
    }
    ZRec* zt = static_cast<ZRec*>(s->cone_tab);
    Tap* xyt = reinterpret_cast<Tap*>(zt + (size_t)C.n * S.n);
    bool std4 = S.n == 4 && T.n == 4;
    for (int q = 0; std4 && q < 4; ++q)
      std4 = S.lv[q] == q && T.lv[q] == q && T.slot[q] == q && T.m[q] == 3 &&
             T.sz[q][0] == kStdBox[q][0] && T.sz[q][1] == kStdBox[q][1] &&
             T.sz[q][2] == kStdBox[q][2];
    if (std4) {
      hipLaunchKernelGGL(k_col_table<4>, dim3(1), block, 0, st, P, C, S, T, zt, xyt);
      if (sh_out)
        hipLaunchKernelGGL((k_cones_col<4, true, true>), grid, block, lds, st, P, C, S, T, zt,
                           xyt, out, *SH, sh_out);
      else
        hipLaunchKernelGGL((k_cones_col<4, false, true>), grid, block, lds, st, P, C, S, T, zt,
                           xyt, out, S, nullptr);
      LS_HIP(hipGetLastError());
      return LS_OK;
    }
    switch (S.n) {
#define LS_CONES_CASE(N)                                                                        \
  case N:                                                                                       \
    hipLaunchKernelGGL(k_col_table<N>, dim3(1), block, 0, st, P, C, S, T, zt, xyt);            \
    if (sh_out)                                                                                 \
      hipLaunchKernelGGL((k_cones_col<N, true, false>), grid, block, lds, st, P, C, S, T, zt,  \
                         xyt, out, *SH, sh_out);                                                \
    else                                                                                        \
      hipLaunchKernelGGL((k_cones_col<N, false, false>), grid, block, lds, st, P, C, S, T, zt, \
                         xyt, out, S, nullptr);                                                 \
    break;
      LS_CONES_CASE(1) LS_CONES_CASE(2) LS_CONES_CASE(3) LS_CONES_CASE(4)
      LS_CONES_CASE(5) LS_CONES_CASE(6) LS_CONES_CASE(7) LS_CONES_CASE(8)
#undef LS_CONES_CASE
    }
  } else if (sh_out) {
    return LS_EUNSUPPORTED;
  } else if (ao) {
    hipLaunchKernelGGL(k_ao, dim3(blocks_for(s->nvox)), dim3(kBlock), 0, st, make_pyramid(s), C,
                       S, s->nvox, out);
  } else {
    hipLaunchKernelGGL(k_shadow, dim3(blocks_for(s->nvox)), dim3(kBlock), 0, st, make_pyramid(s),
                       C, S, s->nvox, out);
  }
  LS_HIP(hipGetLastError());
  return LS_OK;
}

}  // namespace

namespace {

// AO cone set: spherical Fibonacci directions z_i = 1 - (2i + 1)/n, azimuth
// i * pi (3 - sqrt 5).
Cones ao_cones(int n_cones, float radius, float aperture) {
  Cones C{};
  C.n = n_cones;
  C.s_max = (double)radius;
  C.aperture = (double)aperture;
  const double ga = 3.14159265358979323846 * (3.0 - std::sqrt(5.0));
  for (int i = 0; i < n_cones; ++i) {
    double z = 1.0 - (2.0 * i + 1.0) / (double)n_cones;
    double r = std::sqrt(1.0 - z * z);
    double ph = ga * (double)i;
    C.dir[i][0] = r * std::cos(ph);
    C.dir[i][1] = r * std::sin(ph);
    C.dir[i][2] = z;
  }
  return C;
}

}  // namespace

int illum_ao_shadow(ls_lineset* s, int n_cones, float radius, const float light[3],
                    float aperture, hipStream_t st, bool* applied) {
  *applied = false;
  if (n_cones < 1 || n_cones + 1 > kMaxCones) return LS_OK;
  Sched S, SH;
  if (!make_sched(s, (double)radius, (double)aperture, &S) ||
      !make_sched(s, INFINITY, (double)aperture, &SH) || SH.n < S.n)
    return LS_OK;
  for (int k = 0; k < S.n; ++k)
    if (SH.s[k] != S.s[k] || SH.D[k] != S.D[k] || SH.lv[k] != S.lv[k]) return LS_OK;
  // the column kernel's shadow tail takes samples on levels >= 3 (a column's
  // 8 voxels then span at most two level cells along z)
  for (int k = S.n; k < SH.n; ++k)
    if (SH.lv[k] < 3) return LS_OK;
  ColLevels T;
  if (S.n < 1 || S.n > kColMaxSamples || !make_col_levels(s, S, &T)) return LS_OK;
  int rc;
  if (!s->ao && (rc = ls_alloc(s, (void**)&s->ao, sizeof(float) * (size_t)s->nvox))) return rc;
  if (!s->sh && (rc = ls_alloc(s, (void**)&s->sh, sizeof(float) * (size_t)s->nvox))) return rc;
  Cones C = ao_cones(n_cones, radius, aperture);
  for (int a = 0; a < 3; ++a) C.dir[n_cones][a] = (double)light[a];
  C.n = n_cones + 1;
  if ((rc = launch_cones(s, C, S, s->ao, st, true, &SH, s->sh))) return rc;
  *applied = true;
  return LS_OK;
}

int illum_ao(ls_lineset* s, int n_cones, float radius, float aperture, hipStream_t st) {
  if (n_cones < 1 || n_cones > kMaxCones) {
    ls_set_error("ao_cones must be in [1, %d]", kMaxCones);
    return LS_EINVAL;
  }
  int rc;
  if (!s->ao && (rc = ls_alloc(s, (void**)&s->ao, sizeof(float) * (size_t)s->nvox))) return rc;
  const Cones C = ao_cones(n_cones, radius, aperture);
  Sched S;
  if (!make_sched(s, (double)radius, (double)aperture, &S)) {
    ls_set_error("cone schedule longer than %d samples or not exact in fp32 (aperture too small?)",
                 kMaxSamples);
    return LS_EUNSUPPORTED;
  }
  return launch_cones(s, C, S, s->ao, st, true);
}

int illum_shadow(ls_lineset* s, const float light[3], float aperture, hipStream_t st) {
  int rc;
  if (!s->sh && (rc = ls_alloc(s, (void**)&s->sh, sizeof(float) * (size_t)s->nvox))) return rc;
  Cones C{};
  C.n = 1;
  C.aperture = (double)aperture;
  for (int a = 0; a < 3; ++a) C.dir[0][a] = (double)light[a];
  Sched S;
  if (!make_sched(s, INFINITY, (double)aperture, &S)) {
    ls_set_error("cone schedule longer than %d samples or not exact in fp32 (aperture too small?)",
                 kMaxSamples);
    return LS_EUNSUPPORTED;
  }
  return launch_cones(s, C, S, s->sh, st, false);
}
