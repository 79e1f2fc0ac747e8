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
      c[k] = pr.x + wx * (pr.y - pr.x);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = r[rows[k]];
  }
  const float c0 = c[0] * (1.f - fr[1]) + c[1] * fr[1];
  const float c1 = c[2] * (1.f - fr[1]) + c[3] * fr[1];
  return c0 * (1.f - fr[2]) + c1 * fr[2];
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
    occ += sample(P, S.lv[k], v, f) * S.D[k];
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
  hipLaunchKernelGGL(k_ao, dim3(blocks_for(s->nvox)), dim3(kBlock), 0, st, make_pyramid(s), C, S,
                     s->nvox, s->ao);
  LS_HIP(hipGetLastError());
  return LS_OK;
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
  hipLaunchKernelGGL(k_shadow, dim3(blocks_for(s->nvox)), dim3(kBlock), 0, st, make_pyramid(s), C,
                     S, s->nvox, s->sh);
  LS_HIP(hipGetLastError());
  return LS_OK;
}
