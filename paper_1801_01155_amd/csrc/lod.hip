// Density pyramid (section "LoD construction") on gfx950.
//
// Level 0 over each voxel's contiguous line list:
//   count = #lines, len = sum |exit - entry|, rho = sum |exit - entry| * sigma
// (sigma = lut[attr].a, or 1 for opaque lines). Each coarser level averages
// the 2^3 children of the finer one (children beyond an odd side count as 0).
// The three fields are written as separate float arrays (structure of arrays)
// so the renderer and the cone tracer read only rho.
#include "ls_internal.h"

namespace {

constexpr int kBlock = 256;

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

// Level 0, a wave per 64 consecutive voxels. Their lists are one contiguous
// run of records, read 64 at a time by the whole wave (coalesced); each
// line's length goes through a segmented scan over the lanes holding its
// voxel's lines, and the voxel's lane collects its segment's total. A wave
// costs (lines of its voxels) / 64 steps instead of its longest list.
__device__ inline int wave_lane() { return (int)(threadIdx.x & 63); }

__global__ __launch_bounds__(kBlock) void k_lod0(const uint32_t* offsets, const uint64_t* records,
                                                 int64_t nvox, float inv_bins, const float* lut,
                                                 int opaque, float* count, float* len, float* rho) {
  const int lane = wave_lane();
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool in = v < nvox;
  uint32_t lo = 0, hi = 0;
  if (in) {
    lo = offsets[v];
    hi = offsets[v + 1];
  }
  const uint32_t n = hi - lo;
  // exclusive scan of the list lengths: this voxel's lines are the wave's
  // lines [P, P + n), i.e. records lo0 + [P, P + n)
  uint32_t inc = n;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d, 64);
    if (lane >= d) inc += y;
  }
  const uint32_t P = inc - n;
  const uint32_t N = __shfl(inc, 63, 64);
  const uint32_t lo0 = __shfl(lo, 0, 64);
  float l = 0.f, r = 0.f;
  for (uint32_t base = 0; base < N; base += 64) {
    const uint32_t w = base + (uint32_t)lane;
    // owner: the last lane whose P <= w (lists are in lane order)
    int o = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
      const uint32_t pq = __shfl(P, o + step, 64);
      if (pq <= w) o += step;
    }
    float L = 0.f, Ls = 0.f;
    if (w < N) {
      const uint64_t rec = records[lo0 + w];
      float a[3], b[3];
      decode_point((uint32_t)(rec & 0x7FFFu), inv_bins, a);
      decode_point((uint32_t)((rec >> 15) & 0x7FFFu), inv_bins, b);
      const float dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
      L = sqrtf(dx * dx + dy * dy + dz * dz);
      const float sigma = opaque ? 1.f : lut[4 * ((rec >> 32) & 0xFF) + 3];
      Ls = L * sigma;
    }
    // segmented inclusive scan: lanes of one owner form a contiguous run
    const uint32_t po = __shfl(P, o, 64);
    const int seg0 = po > base ? (int)(po - base) : 0;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const float yl = __shfl_up(L, d, 64), yr = __shfl_up(Ls, d, 64);
      if (lane - d >= seg0) {
        L += yl;
        Ls += yr;
      }
    }
    // this voxel's run in the chunk ends at lane min(P + n, base + 64) - 1
    // (all lanes shuffle; lanes without a run here discard the value)
    const bool here = n != 0 && P < base + 64u && P + n > base;
    const int end = here ? (int)((P + n < base + 64u ? P + n : base + 64u) - 1u - base) : 0;
    const float tl = __shfl(L, end, 64), tr = __shfl(Ls, end, 64);
    if (here) {
      l += tl;
      r += tr;
    }
  }
  if (!in) return;
  count[v] = (float)n;
  len[v] = l;
  rho[v] = r;
}

struct MipArgs {
  int32_t cx, cy, cz;  // child dims
  int32_t px, py, pz;  // parent dims
};

__global__ __launch_bounds__(kBlock) void k_mip(const float* __restrict__ c_count,
                                                const float* __restrict__ c_len,
                                                const float* __restrict__ c_rho, float* p_count,
                                                float* p_len, float* p_rho, MipArgs m) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int64_t n = (int64_t)m.px * m.py * m.pz;
  if (i >= n) return;
  int32_t x = (int32_t)(i % m.px), y = (int32_t)((i / m.px) % m.py),
          z = (int32_t)(i / ((int64_t)m.px * m.py));
  float sc = 0.f, sl = 0.f, sr = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int32_t ax = 2 * x + (k & 1), ay = 2 * y + ((k >> 1) & 1), az = 2 * z + (k >> 2);
    if (ax < m.cx && ay < m.cy && az < m.cz) {
      int64_t ci = ax + (int64_t)m.cx * (ay + (int64_t)m.cy * az);
      sc += c_count[ci];
      sl += c_len[ci];
      sr += c_rho[ci];
    }
  }
  p_count[i] = sc * 0.125f;
  p_len[i] = sl * 0.125f;
  p_rho[i] = sr * 0.125f;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

void lod_plan(const int32_t grid[3], int32_t* n_levels, int32_t dims[][3], int64_t* level_off) {
  int n = 0;
  int32_t cur[3] = {grid[0], grid[1], grid[2]};
  level_off[0] = 0;
  for (;;) {
    for (int a = 0; a < 3; ++a) dims[n][a] = cur[a];
    level_off[n + 1] = level_off[n] + (int64_t)cur[0] * cur[1] * cur[2];
    ++n;
    if ((cur[0] == 1 && cur[1] == 1 && cur[2] == 1) || n == LS_MAX_LEVELS) break;
    for (int a = 0; a < 3; ++a) cur[a] = (cur[a] + 1) / 2;
  }
  *n_levels = n;
}

int lod_build(ls_lineset* s, const float* lut, int opaque, hipStream_t st) {
  int rc;
  if (!s->lod_rho) {
    lod_plan(s->grid, &s->n_levels, s->level_dims, s->level_off);
    size_t bytes = sizeof(float) * (size_t)s->level_off[s->n_levels];
    if ((rc = ls_alloc(s, (void**)&s->lod_count, bytes)) ||
        (rc = ls_alloc(s, (void**)&s->lod_len, bytes)) || (rc = ls_alloc(s, (void**)&s->lod_rho, bytes)))
      return rc;
  }
  if (s->nvox > 0) {
    hipLaunchKernelGGL(k_lod0, dim3(blocks_for(s->nvox)), dim3(kBlock), 0, st, s->offsets,
                       s->records, s->nvox, 1.0f / (float)s->bins, lut, opaque, s->lod_count,
                       s->lod_len, s->lod_rho);
    LS_HIP(hipGetLastError());
  }
  for (int l = 1; l < s->n_levels; ++l) {
    MipArgs m{s->level_dims[l - 1][0], s->level_dims[l - 1][1], s->level_dims[l - 1][2],
              s->level_dims[l][0],     s->level_dims[l][1],     s->level_dims[l][2]};
    int64_t c0 = s->level_off[l - 1], p0 = s->level_off[l];
    int64_t n = s->level_off[l + 1] - p0;
    hipLaunchKernelGGL(k_mip, dim3(blocks_for(n)), dim3(kBlock), 0, st, s->lod_count + c0,
                       s->lod_len + c0, s->lod_rho + c0, s->lod_count + p0, s->lod_len + p0,
                       s->lod_rho + p0, m);
    LS_HIP(hipGetLastError());
  }
  return LS_OK;
}
