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

// Trilinear sample of level `lv` at the point v + f (v the voxel corner,
// integer; f a local offset in voxel units). The level coordinate is formed
// from v's low bits and f in fp32, so it keeps ~1e-7 cell precision at every
// level. The two x-neighbour taps are one 8-byte load: the pair starts at
// j = clamp(i0, 0, D - 2) and the x weight is clamp(x - j, 0, 1), which is
// clamp-to-edge interpolation.
__device__ inline float sample(const Pyramid& P, int lv, const int32_t v[3], const float f[3]) {
  const float scale = __builtin_ldexpf(1.0f, -lv);
  const int32_t mask = (1 << lv) - 1;
  const int32_t* dm = P.dims[lv];
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
  const int64_t sy = dm[0], sz = (int64_t)dm[0] * dm[1];
  const int32_t y0 = min(max(i0[1], 0), dm[1] - 1), y1 = min(max(i0[1] + 1, 0), dm[1] - 1);
  const int32_t z0 = min(max(i0[2], 0), dm[2] - 1), z1 = min(max(i0[2] + 1, 0), dm[2] - 1);
  float c[4];
  const int64_t rows[4] = {y0 * sy + z0 * sz, y1 * sy + z0 * sz, y0 * sy + z1 * sz, y1 * sy + z1 * sz};
  if (dm[0] >= 2) {
    const int32_t j = min(max(i0[0], 0), dm[0] - 2);
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

// Occlusion along one cone from the centre of voxel v. The inside-the-grid
// test is made in fp64 on p + s u (the same expression as the definition);
// the sample itself uses the local offset f = 0.5 + s u in fp32.
__device__ inline float cone(const Pyramid& P, const int32_t v[3], const double u[3],
                             double s_max, double aperture) {
  const int top = P.n_levels - 1;
  const float u32[3] = {(float)u[0], (float)u[1], (float)u[2]};
  float occ = 0.f;
  double s = 1.0;
  while (s < s_max) {
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double x = ((double)v[a] + 0.5) + s * u[a];
      inside &= x >= 0.0 && x < (double)P.g[a];
    }
    if (!inside) break;
    double D = aperture * s;
    D = D < 1.0 ? 1.0 : D;
    int lv = ilogb(D);
    lv = lv > top ? top : lv;
    const float sf = (float)s;
    const float f[3] = {0.5f + sf * u32[0], 0.5f + sf * u32[1], 0.5f + sf * u32[2]};
    occ += sample(P, lv, v, f) * (float)D;
    if (occ >= 1.f) break;
    s += D;
  }
  return occ < 1.f ? occ : 1.f;
}

__global__ __launch_bounds__(kBlock) void k_ao(Pyramid P, Cones C, int64_t nvox, float* ao) {
  int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nvox) return;
  const int32_t p[3] = {(int32_t)(v % P.g[0]), (int32_t)((v / P.g[0]) % P.g[1]),
                        (int32_t)(v / ((int64_t)P.g[0] * P.g[1]))};
  float sum = 0.f;
  for (int c = 0; c < C.n; ++c) sum += cone(P, p, C.dir[c], C.s_max, C.aperture);
  ao[v] = 1.f - sum / (float)C.n;
}

__global__ __launch_bounds__(kBlock) void k_shadow(Pyramid P, Cones C, int64_t nvox, float* sh) {
  int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nvox) return;
  const int32_t p[3] = {(int32_t)(v % P.g[0]), (int32_t)((v / P.g[0]) % P.g[1]),
                        (int32_t)(v / ((int64_t)P.g[0] * P.g[1]))};
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
