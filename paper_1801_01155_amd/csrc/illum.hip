// Per-voxel ambient occlusion and soft-shadow grids by cone tracing the
// density pyramid (sections "Shadow simulation", "Ambient occlusion",
// "Illumination effects") on gfx950.
//
// From the voxel centre p along a unit direction u, samples are taken at
// distance s with cone diameter D = max(1, aperture * s) on level
// min(L, floor(log2 D)) (cell-centred trilinear, clamp to edge); each adds
// rho * D to the occlusion, then s += D, while s < s_max and the point is
// inside the grid; occlusion saturates at 1. Sample positions and lattice
// coordinates are formed in fp64 (they reach hundreds of voxels along the
// shadow cone), weights and accumulation in fp32. One thread per voxel; the
// pyramid levels are small enough past level 2 to stay in L2.
#include "ls_internal.h"

#include <cmath>

namespace {

constexpr int kBlock = 256;
constexpr int kMaxCones = 64;

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

__device__ inline float sample(const Pyramid& P, int lv, const double x[3]) {
  const double scale = ldexp(1.0, -lv);
  const int32_t* dm = P.dims[lv];
  int32_t i0[3], i1[3];
  float f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double g = x[a] * scale - 0.5;
    double fl = floor(g);
    f[a] = (float)(g - fl);
    int32_t lo = (int32_t)fl;
    int32_t hi = lo + 1;
    lo = lo < 0 ? 0 : (lo > dm[a] - 1 ? dm[a] - 1 : lo);
    hi = hi < 0 ? 0 : (hi > dm[a] - 1 ? dm[a] - 1 : hi);
    i0[a] = lo;
    i1[a] = hi;
  }
  const float* r = P.rho + P.off[lv];
  const int64_t sy = dm[0], sz = (int64_t)dm[0] * dm[1];
  const int64_t z0 = i0[2] * sz, z1 = i1[2] * sz, y0 = i0[1] * sy, y1 = i1[1] * sy;
  float c00 = r[i0[0] + y0 + z0] * (1.f - f[0]) + r[i1[0] + y0 + z0] * f[0];
  float c10 = r[i0[0] + y1 + z0] * (1.f - f[0]) + r[i1[0] + y1 + z0] * f[0];
  float c01 = r[i0[0] + y0 + z1] * (1.f - f[0]) + r[i1[0] + y0 + z1] * f[0];
  float c11 = r[i0[0] + y1 + z1] * (1.f - f[0]) + r[i1[0] + y1 + z1] * f[0];
  float c0 = c00 * (1.f - f[1]) + c10 * f[1];
  float c1 = c01 * (1.f - f[1]) + c11 * f[1];
  return c0 * (1.f - f[2]) + c1 * f[2];
}

__device__ inline float cone(const Pyramid& P, const double p[3], const double u[3], double s_max,
                             double aperture) {
  const int top = P.n_levels - 1;
  float occ = 0.f;
  double s = 1.0;
  while (s < s_max) {
    double x[3];
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      x[a] = p[a] + s * u[a];
      inside &= x[a] >= 0.0 && x[a] < (double)P.g[a];
    }
    if (!inside) break;
    double D = aperture * s;
    D = D < 1.0 ? 1.0 : D;
    int lv = ilogb(D);
    lv = lv > top ? top : lv;
    occ += sample(P, lv, x) * (float)D;
    if (occ >= 1.f) break;
    s += D;
  }
  return occ < 1.f ? occ : 1.f;
}

__global__ __launch_bounds__(kBlock) void k_ao(Pyramid P, Cones C, int64_t nvox, float* ao) {
  int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nvox) return;
  const double p[3] = {(double)(v % P.g[0]) + 0.5, (double)((v / P.g[0]) % P.g[1]) + 0.5,
                       (double)(v / ((int64_t)P.g[0] * P.g[1])) + 0.5};
  float sum = 0.f;
  for (int c = 0; c < C.n; ++c) sum += cone(P, p, C.dir[c], C.s_max, C.aperture);
  ao[v] = 1.f - sum / (float)C.n;
}

__global__ __launch_bounds__(kBlock) void k_shadow(Pyramid P, Cones C, int64_t nvox, float* sh) {
  int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nvox) return;
  const double p[3] = {(double)(v % P.g[0]) + 0.5, (double)((v / P.g[0]) % P.g[1]) + 0.5,
                       (double)(v / ((int64_t)P.g[0] * P.g[1])) + 0.5};
  sh[v] = 1.f - cone(P, p, C.dir[0], INFINITY, C.aperture);
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
  hipLaunchKernelGGL(k_ao, dim3(blocks_for(s->nvox)), dim3(kBlock), 0, st, make_pyramid(s), C,
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
  hipLaunchKernelGGL(k_shadow, dim3(blocks_for(s->nvox)), dim3(kBlock), 0, st, make_pyramid(s), C,
                     s->nvox, s->sh);
  LS_HIP(hipGetLastError());
  return LS_OK;
}
