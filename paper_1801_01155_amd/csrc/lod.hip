// Density pyramid (section "LoD construction") on gfx950.
//
// Level 0 over each voxel's contiguous line list:
//   count = #lines, len = sum |exit - entry|, rho = sum |exit - entry| * sigma
// (sigma = lut[attr].a, or 1 for opaque lines). Each coarser level averages
// the 2^3 children of the finer one (children beyond an odd side count as 0).
// The three fields are written as separate float arrays (structure of arrays)
// so the renderer and the cone tracer read only rho.
#include <algorithm>

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
  // the transfer function's opacities, staged once per block (a record's
  // opacity is then not a global load that waits for the record)
  static_assert(kBlock == 256, "one thread per transfer-function entry");
  __shared__ float s_alpha[256];
  s_alpha[threadIdx.x] = opaque ? 1.f : lut[4 * threadIdx.x + 3];
  __syncthreads();
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
      const float sigma = s_alpha[(rec >> 32) & 0xFF];
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

// Small levels, up to kBrickLevels per launch: each
// workgroup takes an 8^3 brick of the first level it writes and reduces it
// to one voxel through LDS (8^3 -> 4^3 -> 2^3 -> 1), so a small level costs
// a few LDS passes instead of a launch. Sums run over the children in the
// same order as k_mip, so every level is bit-identical to one k_mip per level.
// Levels larger than kBrickMaxVoxels keep one k_mip launch each: a brick's
// few loads in flight per thread read a big level slower than a thread per
// voxel does (measured at 512^3: 128^3 bricked 1.31 ms for the pyramid,
// 1.27 ms with k_mip).
constexpr int kBrick = 8;
constexpr int kBrickLevels = 4;
constexpr int64_t kBrickMaxVoxels = 1 << 18;

struct BrickArgs {
  int32_t dims[kBrickLevels + 1][3];   // level L (children) .. L + nl
  int64_t off[kBrickLevels + 1];       // their element offsets in the pyramid
  int32_t nl;                          // levels written, 1..kBrickLevels
  int32_t bx, by;                      // bricks along x and y of level L + 1
};

__global__ __launch_bounds__(kBlock) void k_mip_brick(float* count, float* len, float* rho,
                                                      BrickArgs a) {
  // level L + j of the brick (side kBrick >> (j - 1)) at lds[c][base[j] + v]
  __shared__ float lds[3][512 + 64 + 8];
  const int base[4] = {0, 0, 512, 576};
  const int b = blockIdx.x;
  const int ox = b % a.bx, oy = (b / a.bx) % a.by, oz = b / (a.bx * a.by);
  float* const ch[3] = {count, len, rho};
  for (int j = 1; j <= a.nl; ++j) {
    const int side = kBrick >> (j - 1);
    const int32_t* cd = a.dims[j - 1];
    const int32_t* pd = a.dims[j];
    const int32_t gx0 = ox * side, gy0 = oy * side, gz0 = oz * side;
    for (int v = threadIdx.x; v < side * side * side; v += kBlock) {
      const int x = v % side, y = (v / side) % side, z = v / (side * side);
      const int32_t gx = gx0 + x, gy = gy0 + y, gz = gz0 + z;
      if (gx >= pd[0] || gy >= pd[1] || gz >= pd[2]) continue;
      float sum[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
        const int32_t ax = 2 * gx + kx, ay = 2 * gy + ky, az = 2 * gz + kz;
        if (ax < cd[0] && ay < cd[1] && az < cd[2]) {
          if (j == 1) {
            const int64_t ci = a.off[0] + ax + (int64_t)cd[0] * (ay + (int64_t)cd[1] * az);
#pragma unroll
            for (int c = 0; c < 3; ++c) sum[c] += ch[c][ci];
          } else {
            const int s2 = 2 * side;
            const int li = base[j - 1] + (2 * x + kx) + s2 * ((2 * y + ky) + s2 * (2 * z + kz));
#pragma unroll
            for (int c = 0; c < 3; ++c) sum[c] += lds[c][li];
          }
        }
      }
      const int64_t pi = a.off[j] + gx + (int64_t)pd[0] * (gy + (int64_t)pd[1] * gz);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float m = sum[c] * 0.125f;
        ch[c][pi] = m;
        if (j < a.nl) lds[c][base[j] + v] = m;
      }
    }
    __syncthreads();
  }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Colour beside the density for opacity acceleration: per voxel the sum over
// its lines of length * sigma * (transfer-function colour), three floats
// interleaved; a thread per voxel walks its list.
__global__ __launch_bounds__(kBlock) void k_lodc0(const uint32_t* offsets, const uint64_t* records,
                                                  int64_t nvox, float inv_bins, const float* lut,
                                                  int opaque, float* rgb) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nvox) return;
  float c[3] = {0.f, 0.f, 0.f};
  for (uint32_t k = offsets[v]; k < offsets[v + 1]; ++k) {
    const uint64_t rec = records[k];
    float a[3], b[3];
    decode_point((uint32_t)(rec & 0x7FFFu), inv_bins, a);
    decode_point((uint32_t)((rec >> 15) & 0x7FFFu), inv_bins, b);
    const float dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
    const float L = sqrtf(dx * dx + dy * dy + dz * dz);
    const float* l = lut + 4 * ((rec >> 32) & 0xFF);
    const float w = L * (opaque ? 1.f : l[3]);
    c[0] += w * l[0];
    c[1] += w * l[1];
    c[2] += w * l[2];
  }
  rgb[3 * v + 0] = c[0];
  rgb[3 * v + 1] = c[1];
  rgb[3 * v + 2] = c[2];
}

// One coarser colour level: a thread per parent averages its 8 children
// (x fastest, missing children beyond an odd side count as 0).
__global__ __launch_bounds__(kBlock) void k_mipc(const float* child, float* parent, MipArgs m) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t np = (int64_t)m.px * m.py * m.pz;
  if (v >= np) return;
  const int32_t x = (int32_t)(v % m.px), y = (int32_t)((v / m.px) % m.py),
                z = (int32_t)(v / ((int64_t)m.px * m.py));
  float s[3] = {0.f, 0.f, 0.f};
  for (int k = 0; k < 8; ++k) {
    const int32_t cx = 2 * x + (k & 1), cy = 2 * y + ((k >> 1) & 1), cz = 2 * z + (k >> 2);
    if (cx >= m.cx || cy >= m.cy || cz >= m.cz) continue;
    const int64_t ci = cx + (int64_t)m.cx * (cy + (int64_t)m.cy * cz);
    s[0] += child[3 * ci + 0];
    s[1] += child[3 * ci + 1];
    s[2] += child[3 * ci + 2];
  }
  parent[3 * v + 0] = s[0] * 0.125f;
  parent[3 * v + 1] = s[1] * 0.125f;
  parent[3 * v + 2] = s[2] * 0.125f;
}

}  // namespace

int lod_color_build(ls_lineset* s, const float* lut, int opaque, hipStream_t st) {
  int rc;
  if (!s->lod_rgb) {
    if ((rc = ls_alloc(s, (void**)&s->lod_rgb,
                       3 * sizeof(float) * (size_t)s->level_off[s->n_levels])))
      return rc;
  }
  if (s->nvox > 0) {
    hipLaunchKernelGGL(k_lodc0, dim3(blocks_for(s->nvox)), dim3(kBlock), 0, st, s->offsets,
                       s->records, s->nvox, 1.0f / (float)s->bins, lut, opaque, s->lod_rgb);
    LS_HIP(hipGetLastError());
  }
  for (int L = 0; L + 1 < s->n_levels; ++L) {
    const int64_t n = s->level_off[L + 2] - s->level_off[L + 1];
    MipArgs m{s->level_dims[L][0],     s->level_dims[L][1],     s->level_dims[L][2],
              s->level_dims[L + 1][0], s->level_dims[L + 1][1], s->level_dims[L + 1][2]};
    hipLaunchKernelGGL(k_mipc, dim3(blocks_for(n)), dim3(kBlock), 0, st,
                       s->lod_rgb + 3 * s->level_off[L], s->lod_rgb + 3 * s->level_off[L + 1], m);
    LS_HIP(hipGetLastError());
  }
  return LS_OK;
}

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
  // large levels stream their children at full occupancy (a thread per
  // voxel); the small rest goes kBrickLevels levels per launch through LDS
  int L = 0;
  for (; L + 1 < s->n_levels; ++L) {
    const int64_t p0 = s->level_off[L + 1];
    const int64_t n = s->level_off[L + 2] - p0;
    if (n <= kBrickMaxVoxels) break;
    const int64_t c0 = s->level_off[L];
    MipArgs m{s->level_dims[L][0],     s->level_dims[L][1],     s->level_dims[L][2],
              s->level_dims[L + 1][0], s->level_dims[L + 1][1], s->level_dims[L + 1][2]};
    hipLaunchKernelGGL(k_mip, dim3(blocks_for(n)), dim3(kBlock), 0, st, s->lod_count + c0,
                       s->lod_len + c0, s->lod_rho + c0, s->lod_count + p0, s->lod_len + p0,
                       s->lod_rho + p0, m);
    LS_HIP(hipGetLastError());
  }
  for (; L + 1 < s->n_levels; L += kBrickLevels) {
    BrickArgs a{};
    a.nl = std::min(kBrickLevels, s->n_levels - 1 - L);
    for (int j = 0; j <= a.nl; ++j) {
      for (int c = 0; c < 3; ++c) a.dims[j][c] = s->level_dims[L + j][c];
      a.off[j] = s->level_off[L + j];
    }
    a.bx = (a.dims[1][0] + kBrick - 1) / kBrick;
    a.by = (a.dims[1][1] + kBrick - 1) / kBrick;
    const int64_t bz = (a.dims[1][2] + kBrick - 1) / kBrick;
    const int64_t blocks = (int64_t)a.bx * a.by * bz;
    hipLaunchKernelGGL(k_mip_brick, dim3((unsigned)blocks), dim3(kBlock), 0, st, s->lod_count,
                       s->lod_len, s->lod_rho, a);
    LS_HIP(hipGetLastError());
  }
  return LS_OK;
}
