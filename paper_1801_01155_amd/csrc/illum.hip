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

// LDS-tiled cone tracing. A block handles an 8^3 tile of voxels. Every
// sample k of every cone lies within s_k (voxel units) of its voxel, so on
// level l the taps of the whole tile fall inside a box of
// (tile extent on l) + 2 m_l cells per axis, m_l = ceil(max s_k / 2^l) + 2
// over the samples on l. The block first copies each level's box into LDS
// (coordinates clamped to the level, which makes plain trilinear
// interpolation of the copy the clamp-to-edge interpolation of the level).
//
// With the tile origin a multiple of 8 and every level at most 3, a sample's
// lattice coordinate on axis a depends only on the cone, the sample and the
// voxel's position p_a = v_a - t0_a in the tile: x = ((p_a mod 2^l) + 0.5 +
// s u_a) 2^-l - 0.5 (the arithmetic of sample()). The block tabulates, per
// (cone, sample, axis, p_a), the tap's offset in the box and the weight
// frac(x); a sample then costs three table reads, eight tap reads and the
// seven interpolations.
constexpr int kTile = 8;
constexpr int kTileThreads = 256;
constexpr int kTileSlots = 4;            // levels 0..3
constexpr int kTileLdsBytes = 49152;
constexpr int kTileMaxSamples = 8;       // instantiated schedule lengths
constexpr size_t kMaxTabBytes = 8u * kMaxCones * kTileMaxSamples * 24;   // Tap tables

struct TileLevels {
  int32_t n;                        // distinct levels of the schedule
  int32_t lv[kTileSlots];
  int32_t m[kTileSlots];            // margin per side, cells
  int32_t sz[kTileSlots];           // box edge, cells
  int32_t base[kTileSlots + 1];     // LDS offset (floats) of each box; base[n] = total
  int32_t slot[kMaxSamples];        // box of each sample
  int32_t table;                    // LDS offset (floats, even) of the tap tables
  int32_t tiles[3];
  int32_t tiles_per_xcd;
};

// Tap offset (in bytes, within the sample's box) and weight of one axis.
struct Tap {
  int32_t off;
  float w;
};

// kN = S.n: the sample loop is unrolled, so the schedule's per-sample
// constants (box, edge, weight) stay in scalar registers for the whole block.
// Tap table entry ((c * S.n + k) * 3 + a) * 8 + p: the box offset and
// weight of cone c, sample k, axis a for a voxel at position p of the tile.
template <int kN>
__global__ __launch_bounds__(kTileThreads) void k_cone_table(Cones C, Sched S, TileLevels TL,
                                                             Tap* tab) {
  const int n_tab = C.n * kN * 24;
  for (int e = threadIdx.x; e < n_tab; e += kTileThreads) {
    const int p = e & 7, a = (e >> 3) % 3, ck = e / 24;
    const int c = ck / kN, k = ck % kN;
    const int q = TL.slot[k], lv = S.lv[k], sz = TL.sz[q];
    const float u = (float)C.dir[c][a];
    const float f = 0.5f + S.s[k] * u;
    const float x = ((float)(p & ((1 << lv) - 1)) + f) * __builtin_ldexpf(1.0f, -lv) - 0.5f;
    const float fl = floorf(x);
    const int32_t li = min(max((p >> lv) + (int32_t)fl + TL.m[q], 0), sz - 2);
    const int32_t stride = a == 0 ? 1 : (a == 1 ? sz : sz * sz);
    tab[e] = Tap{li * stride * (int32_t)sizeof(float), x - fl};
  }
}

template <int kN>
__global__ __launch_bounds__(kTileThreads) void k_cones_tiled(Pyramid P, Cones C, Sched S,
                                                              TileLevels TL,
                                                              const Tap* __restrict__ tab_g,
                                                              float* out) {
  extern __shared__ float lds[];
  // XCD x (= block mod 8) works through a contiguous run of tiles, so the
  // boxes neighbouring tiles share are fetched into one L2.
  const int b = blockIdx.x;
  const int tile = (b % 8) * TL.tiles_per_xcd + b / 8;
  const int nt = TL.tiles[0] * TL.tiles[1] * TL.tiles[2];
  if (tile >= nt) return;
  const int32_t t0[3] = {kTile * (tile % TL.tiles[0]),
                         kTile * ((tile / TL.tiles[0]) % TL.tiles[1]),
                         kTile * (tile / (TL.tiles[0] * TL.tiles[1]))};
  for (int q = 0; q < TL.n; ++q) {
    const int lv = TL.lv[q], sz = TL.sz[q], n = sz * sz * sz;
    const int32_t dx = P.dims[lv][0], dy = P.dims[lv][1], dz = P.dims[lv][2];
    const int32_t o0 = (t0[0] >> lv) - TL.m[q], o1 = (t0[1] >> lv) - TL.m[q],
                  o2 = (t0[2] >> lv) - TL.m[q];
    const float* __restrict__ r = P.rho + P.off[lv];
    float* box = lds + TL.base[q];
    for (int i = threadIdx.x; i < n; i += kTileThreads) {
      const int lx = i % sz, ly = (i / sz) % sz, lz = i / (sz * sz);
      const int32_t x = min(max(o0 + lx, 0), dx - 1), y = min(max(o1 + ly, 0), dy - 1),
                    z = min(max(o2 + lz, 0), dz - 1);
      box[i] = r[(z * dy + y) * dx + x];
    }
  }
  // tap tables (built once per launch by k_cone_table) into LDS
  Tap* tab = reinterpret_cast<Tap*>(lds + TL.table);
  {
    const int n4 = C.n * kN * 24 / 2;   // two Taps per 16-byte word
    const int4* src = reinterpret_cast<const int4*>(tab_g);
    int4* dst = reinterpret_cast<int4*>(tab);
    for (int e = threadIdx.x; e < n4; e += kTileThreads) dst[e] = src[e];
  }
  __syncthreads();
  const float inv_n = 1.f / (float)C.n;
  // per-sample constants, read once (wave-uniform, scalar registers)
  int32_t kbase[kN], ksz[kN];
  float kD[kN], ks[kN];
#pragma unroll
  for (int k = 0; k < kN; ++k) {
    const int q = TL.slot[k];
    kbase[k] = TL.base[q];
    ksz[k] = TL.sz[q];
    kD[k] = S.D[k];
    ks[k] = S.s[k];
  }
#pragma unroll 1
  for (int half = 0; half < kTile * kTile * kTile / kTileThreads; ++half) {
    const int loc = threadIdx.x + half * kTileThreads;
    const int32_t pl[3] = {loc & 7, (loc >> 3) & 7, loc >> 6};
    const int32_t v[3] = {t0[0] + pl[0], t0[1] + pl[1], t0[2] + pl[2]};
    if (v[0] >= P.g[0] || v[1] >= P.g[1] || v[2] >= P.g[2]) continue;
    const bool near_face = near_any_face(P, v, S.reach);
    float sum = 0.f;
    const Tap* tc = tab;
    for (int c = 0; c < C.n; ++c, tc += 24 * kN) {
      float occ = 0.f;
      bool go = true;
#pragma unroll
      for (int k = 0; k < kN; ++k) {
        if (go && near_face) {
          const double s = (double)ks[k];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const double x = ((double)v[a] + 0.5) + s * C.dir[c][a];
            go &= x >= 0.0 && x < (double)P.g[a];
          }
        }
        if (go) {
          const Tap* tk = tc + 24 * k;
          const Tap ex = tk[pl[0]], ey = tk[8 + pl[1]], ez = tk[16 + pl[2]];
          const int sz = ksz[k], sz2 = sz * sz;
          const float* bp = reinterpret_cast<const float*>(
              reinterpret_cast<const char*>(lds + kbase[k]) + (ex.off + ey.off + ez.off));
          // lerp(a, b, w) = a + w (b - a), fused
          const float c00 = __builtin_fmaf(ex.w, bp[1] - bp[0], bp[0]);
          const float c10 = __builtin_fmaf(ex.w, bp[sz + 1] - bp[sz], bp[sz]);
          const float c01 = __builtin_fmaf(ex.w, bp[sz2 + 1] - bp[sz2], bp[sz2]);
          const float c11 = __builtin_fmaf(ex.w, bp[sz2 + sz + 1] - bp[sz2 + sz], bp[sz2 + sz]);
          const float c0 = __builtin_fmaf(ey.w, c10 - c00, c00);
          const float c1 = __builtin_fmaf(ey.w, c11 - c01, c01);
          occ = __builtin_fmaf(__builtin_fmaf(ez.w, c1 - c0, c0), kD[k], occ);
          go = occ < 1.f;
        }
      }
      sum += occ < 1.f ? occ : 1.f;
    }
    out[v[0] + (int64_t)P.g[0] * (v[1] + (int64_t)P.g[1] * v[2])] = 1.f - sum * inv_n;
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

// Boxes and tap tables of the tiled kernel for schedule S and n_cones cones;
// false if a level above 3 is sampled or LDS would exceed the budget (then
// the untiled kernels run).
bool make_tile_levels(const ls_lineset* s, const Sched& S, int n_cones, TileLevels* T) {
  *T = TileLevels{};
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
  int64_t total = 0;
  for (int q = 0; q < T->n; ++q) {
    const int ext = std::max(kTile >> T->lv[q], 1);
    T->sz[q] = ext + 2 * T->m[q];
    T->base[q] = (int32_t)total;
    total += (int64_t)T->sz[q] * T->sz[q] * T->sz[q];
  }
  T->base[T->n] = (int32_t)total;
  total = (total + 3) & ~(int64_t)3;           // 16-byte alignment of the tables
  T->table = (int32_t)total;
  total += (int64_t)n_cones * S.n * 24 * 2;    // Tap = 2 floats
  if (total * 4 > kTileLdsBytes) return false;
  for (int a = 0; a < 3; ++a) T->tiles[a] = (s->grid[a] + kTile - 1) / kTile;
  const int64_t nt = (int64_t)T->tiles[0] * T->tiles[1] * T->tiles[2];
  T->tiles_per_xcd = (int32_t)((nt + 7) / 8);
  return true;
}

// LDS bytes of the tiled kernel's plan T.
size_t tile_lds_bytes(const TileLevels& T, int n_cones, int n_samples) {
  return sizeof(float) * ((size_t)T.table + (size_t)n_cones * n_samples * 24 * 2);
}

int launch_cones(ls_lineset* s, const Cones& C, const Sched& S, float* out, hipStream_t st,
                 bool ao) {
  // the tiled kernel pays one LDS fill per tile; with few samples per voxel
  // (the single shadow cone) direct gathers are cheaper
  TileLevels T;
  if (C.n >= 4 && S.n >= 1 && S.n <= kTileMaxSamples && make_tile_levels(s, S, C.n, &T)) {
    const size_t lds = tile_lds_bytes(T, C.n, S.n);
    const dim3 grid((unsigned)(8 * T.tiles_per_xcd)), block(kTileThreads);
    const Pyramid P = make_pyramid(s);
    // the tap tables: one small launch, then copied by every block
    const size_t tab_bytes = sizeof(Tap) * (size_t)C.n * S.n * 24;
    int rc;
    if (!s->cone_tab || s->cone_tab_bytes < tab_bytes) {
      if ((rc = ls_alloc(s, &s->cone_tab, kMaxTabBytes))) return rc;
      s->cone_tab_bytes = kMaxTabBytes;
    }
    Tap* tab = static_cast<Tap*>(s->cone_tab);
    switch (S.n) {
#define LS_CONES_CASE(N)                                                                        \
  case N:                                                                                       \
    hipLaunchKernelGGL(k_cone_table<N>, dim3(1), block, 0, st, C, S, T, tab);                   \
    hipLaunchKernelGGL(k_cones_tiled<N>, grid, block, lds, st, P, C, S, T, tab, out);          \
    break;
      LS_CONES_CASE(1) LS_CONES_CASE(2) LS_CONES_CASE(3) LS_CONES_CASE(4)
      LS_CONES_CASE(5) LS_CONES_CASE(6) LS_CONES_CASE(7) LS_CONES_CASE(8)
#undef LS_CONES_CASE
    }
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

int illum_ao(ls_lineset* s, int n_cones, float radius, float aperture, hipStream_t st) {
  if (n_cones < 1 || n_cones > kMaxCones) {
    ls_set_error("ao_cones must be in [1, %d]", kMaxCones);
    return LS_EINVAL;
  }
  int rc;
  if (!s->ao && (rc = ls_alloc(s, (void**)&s->ao, sizeof(float) * (size_t)s->nvox))) return rc;
  Cones C{};
  C.n = n_cones;
  C.s_max = (double)radius;
  C.aperture = (double)aperture;
  // spherical Fibonacci directions: z_i = 1 - (2i + 1)/n, azimuth i * pi (3 - sqrt 5)
  const double ga = 3.14159265358979323846 * (3.0 - std::sqrt(5.0));
  for (int i = 0; i < n_cones; ++i) {
    double z = 1.0 - (2.0 * i + 1.0) / (double)n_cones;
    double r = std::sqrt(1.0 - z * z);
    double ph = ga * (double)i;
    C.dir[i][0] = r * std::cos(ph);
    C.dir[i][1] = r * std::sin(ph);
    C.dir[i][2] = z;
  }
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
