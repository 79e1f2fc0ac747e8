// Representative lines (section "LoD construction") on gfx950: one average
// line per voxel of every level of the pyramid, used by the shadow rays of
// the first shadow approach (section "Shadow simulation").
//
// Per voxel, the lines' start and end points are summed separately, a line
// being flipped first when its direction has a negative dot product with the
// line before it (list order, as flipped), and each of the two averages goes
// to the closest bin centre on the voxel boundary. Then the lines of two
// face-adjacent voxels that have one endpoint each on their common face are
// joined: both endpoints move to the bin holding the mean of the two points
// (a mean on a bin boundary goes to the upper bin). Level l + 1 averages the
// joined lines of its (up to 8) children, x fastest, in its own frame, and
// joins again.
//
// All arithmetic is exact in int64. A point of a voxel is held in units of
// 1/(4N) of its side: a bin centre is 4k + 2, a face plane 0 or 4N, and a
// child's point p becomes p / 2 + 2N * (child offset) in its parent. For the
// average S / n the closest centre is found without squares: on one face the
// squared distance to its closest centre is the plane term plus the in-plane
// terms, and between two faces the difference reduces to comparing
// t^2 - r(t)^2 (t a plane distance, r(t) the distance of the same coordinate
// to its nearest bin centre), which increases with t; so the closest centre
// lies on the face whose plane is nearest (the first such face on ties), at
// the nearest bin of each in-plane axis (the lowest on ties).
//
// Code of a line: the record layout's low 30 bits (start = entry face and
// bins, end = exit face and bins); 0xFFFFFFFF for a voxel without lines.
#include "ls_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kNone = 0xFFFFFFFFu;

// Bin centre of a 15-bit endpoint code, units of 1/(4N).
__device__ inline void end_units(uint32_t code, int32_t bins, int32_t p[3]) {
  const int face = (int)(code & 7u);
  const int axis = face >> 1;
  const int32_t plane = (face & 1) ? 4 * bins : 0;
  const int32_t u = 4 * (int32_t)((code >> 3) & 63u) + 2;
  const int32_t w = 4 * (int32_t)((code >> 9) & 63u) + 2;
  p[0] = axis == 0 ? plane : u;
  p[1] = axis == 1 ? plane : (axis == 0 ? u : w);
  p[2] = axis == 2 ? plane : w;
}

// Bin k in [0, N) minimising |S - n (4k + 2)|, the lower one on ties.
__device__ inline uint32_t nearest_bin(int64_t S, int64_t n, int32_t bins) {
  const int64_t num = S - 2 * n, den = 4 * n;
  int64_t q = num >= 0 ? num / den : -((-num + den - 1) / den);   // floor(num / den)
  const int64_t e0 = S - n * (4 * q + 2), e1 = S - n * (4 * q + 6);
  if ((e1 < 0 ? -e1 : e1) < (e0 < 0 ? -e0 : e0)) ++q;
  q = q < 0 ? 0 : (q > bins - 1 ? bins - 1 : q);
  return (uint32_t)q;
}

// Closest bin centre on the boundary to the point S / n (see above).
__device__ inline uint32_t snap_point(const int64_t S[3], int64_t n, int32_t bins) {
  const int64_t far = n * 4 * (int64_t)bins;
  int face = 0;
  int64_t best = S[0];
#pragma unroll
  for (int f = 1; f < 6; ++f) {
    const int64_t d = (f & 1) ? far - S[f >> 1] : S[f >> 1];
    if (d < best) {
      best = d;
      face = f;
    }
  }
  const int axis = face >> 1;
  const int ua = axis == 0 ? 1 : 0, wa = axis == 2 ? 1 : 2;
  return (uint32_t)face | (nearest_bin(S[ua], n, bins) << 3) | (nearest_bin(S[wa], n, bins) << 9);
}

struct RepAcc {
  int64_t S[3] = {0, 0, 0}, E[3] = {0, 0, 0};
  int32_t prev[3] = {0, 0, 0};
  int64_t n = 0;

  __device__ void add(const int32_t a_in[3], const int32_t b_in[3]) {
    int32_t a[3] = {a_in[0], a_in[1], a_in[2]}, b[3] = {b_in[0], b_in[1], b_in[2]};
    if (n > 0) {
      const int32_t dot = (b[0] - a[0]) * prev[0] + (b[1] - a[1]) * prev[1] + (b[2] - a[2]) * prev[2];
      if (dot < 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const int32_t t = a[q];
          a[q] = b[q];
          b[q] = t;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      S[q] += a[q];
      E[q] += b[q];
      prev[q] = b[q] - a[q];
    }
    ++n;
  }

  __device__ uint32_t code(int32_t bins) const {
    if (n == 0) return kNone;
    return snap_point(S, n, bins) | (snap_point(E, n, bins) << 15);
  }
};

// Level 0 from the voxels' line lists (thread per voxel).
__global__ __launch_bounds__(kBlock) void k_rep0(const uint32_t* __restrict__ offsets,
                                                 const uint64_t* __restrict__ records, int64_t nvox,
                                                 int32_t bins, uint32_t* __restrict__ pre) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nvox) return;
  const uint32_t lo = offsets[v], hi = offsets[v + 1];
  RepAcc acc;
  for (uint32_t k = lo; k < hi; ++k) {
    const uint64_t rec = records[k];
    int32_t a[3], b[3];
    end_units((uint32_t)(rec & 0x7FFFu), bins, a);
    end_units((uint32_t)((rec >> 15) & 0x7FFFu), bins, b);
    acc.add(a, b);
  }
  pre[v] = acc.code(bins);
}

// Level l + 1 from the joined lines of level l (thread per parent).
__global__ __launch_bounds__(kBlock) void k_rep_up(const uint32_t* __restrict__ child, int32_t cx,
                                                   int32_t cy, int32_t cz, int32_t px, int32_t py,
                                                   int32_t pz, int32_t bins,
                                                   uint32_t* __restrict__ pre) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t np = (int64_t)px * py * pz;
  if (v >= np) return;
  const int32_t x = (int32_t)(v % px), y = (int32_t)((v / px) % py), z = (int32_t)(v / ((int64_t)px * py));
  RepAcc acc;
  for (int k = 0; k < 8; ++k) {
    const int32_t off[3] = {k & 1, (k >> 1) & 1, k >> 2};
    const int32_t c[3] = {2 * x + off[0], 2 * y + off[1], 2 * z + off[2]};
    if (c[0] >= cx || c[1] >= cy || c[2] >= cz) continue;
    const uint32_t code = child[c[0] + (int64_t)cx * (c[1] + (int64_t)cy * c[2])];
    if (code == kNone) continue;
    int32_t a[3], b[3];
    end_units(code & 0x7FFFu, bins, a);
    end_units((code >> 15) & 0x7FFFu, bins, b);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      a[q] = a[q] / 2 + off[q] * 2 * bins;
      b[q] = b[q] / 2 + off[q] * 2 * bins;
    }
    acc.add(a, b);
  }
  pre[v] = acc.code(bins);
}

// Joins the lines of one level across shared faces (thread per voxel).
__global__ __launch_bounds__(kBlock) void k_rep_join(const uint32_t* __restrict__ pre, int32_t dx,
                                                     int32_t dy, int32_t dz,
                                                     uint32_t* __restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t nv = (int64_t)dx * dy * dz;
  if (v >= nv) return;
  const uint32_t code = pre[v];
  if (code == kNone) {
    out[v] = kNone;
    return;
  }
  const int32_t dim[3] = {dx, dy, dz};
  const int32_t cell[3] = {(int32_t)(v % dx), (int32_t)((v / dx) % dy), (int32_t)(v / ((int64_t)dx * dy))};
  uint32_t ends[2] = {code & 0x7FFFu, (code >> 15) & 0x7FFFu};
  if ((ends[0] & 7u) != (ends[1] & 7u)) {
    for (int e = 0; e < 2; ++e) {
      const uint32_t f = ends[e] & 7u;
      const int axis = (int)(f >> 1);
      int32_t c[3] = {cell[0], cell[1], cell[2]};
      c[axis] += (f & 1u) ? 1 : -1;
      if (c[axis] < 0 || c[axis] >= dim[axis]) continue;
      const uint32_t nb = pre[c[0] + (int64_t)dx * (c[1] + (int64_t)dy * c[2])];
      if (nb == kNone) continue;
      const uint32_t n0 = nb & 0x7FFFu, n1 = (nb >> 15) & 0x7FFFu, g = f ^ 1u;
      uint32_t other;
      if ((n0 & 7u) == g && (n1 & 7u) != g) other = n0;
      else if ((n1 & 7u) == g && (n0 & 7u) != g) other = n1;
      else continue;
      const uint32_t bu = (((ends[e] >> 3) & 63u) + ((other >> 3) & 63u) + 1u) >> 1;
      const uint32_t bw = (((ends[e] >> 9) & 63u) + ((other >> 9) & 63u) + 1u) >> 1;
      ends[e] = f | (bu << 3) | (bw << 9);
    }
  }
  out[v] = ends[0] | (ends[1] << 15);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int rep_build(ls_lineset* s, hipStream_t st) {
  int32_t n_levels = 0;
  int32_t dims[LS_MAX_LEVELS][3];
  int64_t loff[LS_MAX_LEVELS + 1];
  lod_plan(s->grid, &n_levels, dims, loff);
  int rc;
  if (!s->rep) {
    if ((rc = ls_alloc(s, (void**)&s->rep, sizeof(uint32_t) * (size_t)loff[n_levels]))) return rc;
  }
  uint32_t* pre = nullptr;
  if ((rc = pool_alloc(sizeof(uint32_t) * (size_t)(s->nvox > 0 ? s->nvox : 1), (void**)&pre,
                       nullptr)))
    return rc;
  hipLaunchKernelGGL(k_rep0, dim3(blocks_for(s->nvox)), dim3(kBlock), 0, st, s->offsets,
                     s->records, s->nvox, s->bins, pre);
  hipLaunchKernelGGL(k_rep_join, dim3(blocks_for(s->nvox)), dim3(kBlock), 0, st, pre,
                     dims[0][0], dims[0][1], dims[0][2], s->rep);
  for (int l = 1; l < n_levels; ++l) {
    const int64_t np = (int64_t)dims[l][0] * dims[l][1] * dims[l][2];
    hipLaunchKernelGGL(k_rep_up, dim3(blocks_for(np)), dim3(kBlock), 0, st,
                       s->rep + loff[l - 1], dims[l - 1][0], dims[l - 1][1], dims[l - 1][2],
                       dims[l][0], dims[l][1], dims[l][2], s->bins, pre);
    hipLaunchKernelGGL(k_rep_join, dim3(blocks_for(np)), dim3(kBlock), 0, st, pre, dims[l][0],
                       dims[l][1], dims[l][2], s->rep + loff[l]);
  }
  const hipError_t e = hipGetLastError();
  // the temporary returns to the cache once the stream has passed its readers
  const hipError_t e2 = hipStreamSynchronize(st);
  pool_free(pre);
  if (e != hipSuccess || e2 != hipSuccess) {
    ls_set_error("representative lines: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    return LS_EDEVICE;
  }
  s->rep_levels = n_levels;
  return LS_OK;
}
