// Voxelization of curves into per-voxel quantized line lists (CSR) on gfx950.
//
// Sections "Curve voxelization", "Line quantization" and "GPU
// implementation". The paper's GPU construction appends per-curve lines
// tagged with voxel ids, sorts by voxel and prefix-sums the counts. Here the
// append is replaced by a count pass that sizes every curve's output range
// exactly (so the emit pass writes without global atomics on a cursor), the
// sort by a histogram + scan + scatter, and determinism inside a voxel by a
// rank pass:
//   k_count   wave per curve: upper bound of the curve's lines (plane
//             crossings - 1); validates the input
//   scan      curve ranges
//   k_emit    wave per curve, lane per segment: exact integer clipping,
//             quantization and packing; a wave prefix sum numbers the events
//             along the curve, so lanes write their lines to consecutive slots
//             (coalesced) in curve order, each taking its rank in its voxel
//             with one atomic on the histogram
//   scan      voxel offsets (CSR)
//   k_scatter thread per emitted line: index into its voxel's range
//   k_rank    thread per CSR slot: ranks the voxel's lines by emission order
//             and gathers the record, so each list is in (curve, position
//             along curve) order regardless of atomic order
// All arithmetic deciding a line's voxel, faces and bins is exact integer
// arithmetic on the 1/256-voxel lattice.
#include "ls_internal.h"

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

namespace {

constexpr int kBlock = 256;

struct GridArgs {
  int32_t g[3];
  int32_t bins;
  int32_t bin_shift;  // log2(256 / bins)
};

// Grid set-up (section "Curve voxelization"): fp64 without contraction, the
// same expression as documented in lineset.h.
__device__ inline int32_t snap_coord(float x, double lo, double scale) {
  double y = __dmul_rn(__dadd_rn((double)x, -lo), scale);
  y = __dadd_rn(y, 0.5);
  return (int32_t)floor(y) + 256;
}

template <bool kFloatIn>
__device__ inline void load_vertex(const float* xyz, const int32_t* lat, int64_t v,
                                   const SnapArgs& sa, int32_t q[3]) {
  if (kFloatIn) {
    const float* p = xyz + 3 * v;
    q[0] = snap_coord(p[0], sa.lo[0], sa.scale);
    q[1] = snap_coord(p[1], sa.lo[1], sa.scale);
    q[2] = snap_coord(p[2], sa.lo[2], sa.scale);
  } else {
    const int32_t* p = lat + 3 * v;
    q[0] = p[0];
    q[1] = p[1];
    q[2] = p[2];
  }
}

__device__ inline bool in_range(const int32_t q[3], const GridArgs& ga) {
  return q[0] >= 0 && q[1] >= 0 && q[2] >= 0 && q[0] < 256 * ga.g[0] && q[1] < 256 * ga.g[1] &&
         q[2] < 256 * ga.g[2];
}

// error codes written to err[0]
constexpr int kErrOffsets = 1;
constexpr int kErrRange = 2;
constexpr int kErrNonFinite = 4;

// Lattice scale 256 (G_a - 2) / extent_a, minimised over the axes with a
// positive extent (0 if none): the grid set-up of section "Curve
// voxelization", the same expression on the host and the device.
__host__ __device__ inline double lattice_scale(const double lo[3], const double hi[3],
                                                const int32_t grid[3]) {
  double s = INFINITY;
  for (int a = 0; a < 3; ++a) {
    const double ext = hi[a] - lo[a];
    if (ext > 0) {
      const double cand = (256.0 * (double)(grid[a] - 2)) / ext;
      if (cand < s) s = cand;
    }
  }
  return s == INFINITY ? 0.0 : s;
}

// Low 32 bits of a * b for a, b below 2^24: one full-rate 24-bit multiply
// (written out because the operands' range is not visible to instruction
// selection across basic blocks, which then picks the quarter-rate 32-bit one).
__device__ inline uint32_t mul_lo24(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// floor(num / den) for 0 <= num <= 256 den, 0 < den < 2^18 (quotient at
// most 256): an fp32 estimate (relative error below 1e-6, so off by at most
// one) corrected by one exact step either way; 24-bit products.
__device__ inline int32_t floor_div_small(int32_t num, int32_t den) {
  __builtin_assume(den > 0 && den < (1 << 18));
  int32_t q = (int32_t)((float)num * __builtin_amdgcn_rcpf((float)den));
  __builtin_assume(q >= 0 && q <= 512);
  if ((int32_t)mul_lo24((uint32_t)q, (uint32_t)den) > num) --q;
  else if ((int32_t)mul_lo24((uint32_t)(q + 1), (uint32_t)den) <= num) ++q;
  return q;
}

// Low 32 bits of the exact event point times den: P0 den + nf d, with
// lattice coordinates and den below 2^18 (24-bit products, wrapping sum).
__device__ inline void event_low(const int32_t P0[3], const int32_t d[3], int32_t den, int32_t nf,
                                 uint32_t xl[3]) {
#pragma unroll
  for (int b = 0; b < 3; ++b)
    xl[b] = mul_lo24((uint32_t)P0[b], (uint32_t)den) + (uint32_t)__mul24(nf, d[b]);
}

// In-face bins of an event point on voxel `cell`, face normal `axis`.
// xl = low 32 bits of (event point * den); the local coordinate
// xn - 256 cell den lies in [0, 256 den] (below 2^26), so it is exact in
// wrapping 32-bit arithmetic.
__device__ inline uint32_t face_code(int axis, int side, const uint32_t xl[3], int32_t den,
                                     const int32_t cell[3], const GridArgs& ga) {
  const uint32_t x_u = axis == 0 ? xl[1] : xl[0];
  const uint32_t x_w = axis == 2 ? xl[1] : xl[2];
  const int32_t c_u = axis == 0 ? cell[1] : cell[0];
  const int32_t c_w = axis == 2 ? cell[1] : cell[2];
  const int32_t lu = (int32_t)(x_u - mul_lo24((uint32_t)(c_u << 8), (uint32_t)den));
  const int32_t lw = (int32_t)(x_w - mul_lo24((uint32_t)(c_w << 8), (uint32_t)den));
  // bin = floor(l / (den 256 / N)) = floor(floor(l / 2^sh) / den), 256 / N = 2^sh
  int32_t bu = floor_div_small(lu >> ga.bin_shift, den);
  int32_t bw = floor_div_small(lw >> ga.bin_shift, den);
  bu = bu < ga.bins - 1 ? bu : ga.bins - 1;
  bw = bw < ga.bins - 1 ? bw : ga.bins - 1;
  return (uint32_t)(2 * axis + side) | ((uint32_t)bu << 3) | ((uint32_t)bw << 9);
}

// One wave per curve; lane l of the wave handles segment s0 + l, 64 segments
// at a time, so vertex loads and record writes are contiguous across lanes.
constexpr int kWavesPerBlock = kBlock / 64;

// Per-curve count of line slots: plane crossings - 1 (an upper bound of the
// lines; simultaneous crossings merge into one event). Validates the input.
template <bool kFloatIn>
__global__ __launch_bounds__(kBlock) void k_count(const float* xyz, const int32_t* lat,
                                                  const int64_t* curve_off, int64_t n_curves,
                                                  int64_t n_vertices, const SnapArgs* sap,
                                                  GridArgs ga, uint64_t* slots, int* err) {
  const int lane = threadIdx.x & 63;
  const SnapArgs sa = kFloatIn ? *sap : SnapArgs{};
  const int64_t c = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (c >= n_curves) return;  // wave-uniform
  const int64_t v0 = curve_off[c], v1 = curve_off[c + 1];
  if (v0 < 0 || v1 < v0 || v1 > n_vertices || (c == 0 && v0 != 0)) {
    if (lane == 0) {
      atomicOr(err, kErrOffsets);
      slots[c] = 0;
    }
    return;
  }
  unsigned long long crossings = 0;
  bool bad = false;
  // two 64-vertex chunks per pass, every load issued before any is used;
  // indices are clamped to the curve's last vertex (v1 > v0 inside the loop)
  // so the loads need no branch, and clamped lanes add nothing
  for (int64_t s0 = v0; s0 < v1; s0 += 128) {
    int32_t q[2][3], r[2][3];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t v = s0 + 64 * h + lane;
      load_vertex<kFloatIn>(xyz, lat, v < v1 ? v : v1 - 1, sa, q[h]);
      load_vertex<kFloatIn>(xyz, lat, v + 1 < v1 ? v + 1 : v1 - 1, sa, r[h]);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t v = s0 + 64 * h + lane;
      if (v < v1) bad |= !in_range(q[h], ga);
      if (v + 1 < v1) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
          crossings += (unsigned long long)abs((r[h][a] >> 8) - (q[h][a] >> 8));
      }
    }
  }
  if (bad) atomicOr(err, kErrRange);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) crossings += __shfl_xor(crossings, d, 64);
  if (lane == 0) slots[c] = crossings > 0 ? crossings - 1 : 0;
}

// An event: the curve crosses from `cell` into the next voxel at the exact
// segment parameter nf / den (den = |d| of the face axis, nf the numerator on
// that axis), i.e. at the point xn / den with xn = P0 den + nf d.
struct Ev {
  int32_t den, nf;
  uint32_t exit_code, entry_code;   // set when face codes are requested
  int fa, exit_side;                // face axis, side of the exited voxel's face
  int planes;                       // planes crossed at this event (1 to 3)
  int32_t ncell[3];                 // the entered voxel
};

// a * b for a, b below 2^24: two full-rate 24-bit multiplies.
__device__ inline uint64_t mul_wide24(uint32_t a, uint32_t b) {
  return (uint64_t)(a & 0xFFFFFFu) * (b & 0xFFFFFFu);
}

// Enumerates the events of segment P0 -> P1 in order: crossings of the
// planes x_a = 256 k (up iff P0_a < 256k <= P1_a, down iff P1_a < 256k <=
// P0_a), ordered by their exact parameter; equal parameters are one event
// whose face is the lowest axis's. f(ev, cell_before) per event.
template <bool kCodes, typename F>
__device__ inline void for_each_event(const int32_t P0[3], const int32_t P1[3], const GridArgs& ga,
                                      F&& f) {
  // lattice coordinates are below 2^18 (grid sides <= 1024): differences,
  // plane offsets and the numerators num_a = distance from P0 to the next
  // plane along a (below 2^19) fit 24 bits, their cross products 48
  int32_t d[3], dn[3], num[3], left[3], cell[3], sg[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    d[a] = P1[a] - P0[a];
    const int32_t c0 = P0[a] >> 8, c1 = P1[a] >> 8;
    cell[a] = c0;
    sg[a] = d[a] > 0 ? 1 : (d[a] < 0 ? -1 : 0);
    dn[a] = d[a] > 0 ? d[a] : -d[a];
    num[a] = d[a] > 0 ? 256 * (c0 + 1) - P0[a] : P0[a] - 256 * c0;
    left[a] = abs(c1 - c0);
  }
  while (left[0] + left[1] + left[2] > 0) {
    // next crossing parameter of axis a: num_a / dn_a; compared exactly by
    // cross products. grp: the axes whose next crossing is the earliest
    // (several at once make one event; its face is the lowest axis's).
    const uint64_t a01 = mul_wide24(num[0], dn[1]), a10 = mul_wide24(num[1], dn[0]);
    const uint64_t a02 = mul_wide24(num[0], dn[2]), a20 = mul_wide24(num[2], dn[0]);
    const uint64_t a12 = mul_wide24(num[1], dn[2]), a21 = mul_wide24(num[2], dn[1]);
    const bool n0 = left[0] == 0, n1 = left[1] == 0, n2 = left[2] == 0;
    bool grp[3];
    grp[0] = !n0 && (n1 || a01 <= a10) && (n2 || a02 <= a20);
    grp[1] = !n1 && (n0 || a10 <= a01) && (n2 || a12 <= a21);
    grp[2] = !n2 && (n0 || a20 <= a02) && (n1 || a21 <= a12);
    const int fa = grp[0] ? 0 : (grp[1] ? 1 : 2);
    int32_t ncell[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) ncell[a] = cell[a] + (grp[a] ? sg[a] : 0);
    Ev ev;
    ev.den = fa == 0 ? dn[0] : (fa == 1 ? dn[1] : dn[2]);
    ev.nf = fa == 0 ? num[0] : (fa == 1 ? num[1] : num[2]);
    const int exit_side = (fa == 0 ? sg[0] : (fa == 1 ? sg[1] : sg[2])) > 0 ? 1 : 0;
    ev.fa = fa;
    ev.exit_side = exit_side;
    ev.planes = (int)grp[0] + (int)grp[1] + (int)grp[2];
#pragma unroll
    for (int b = 0; b < 3; ++b) ev.ncell[b] = ncell[b];
    if (kCodes) {
      uint32_t xl[3];
      event_low(P0, d, ev.den, ev.nf, xl);
      ev.exit_code = face_code(fa, exit_side, xl, ev.den, cell, ga);
      // one plane crossed: the entered voxel has the same in-face cells, so
      // the entry face has the exit face's bins and the other side
      ev.entry_code = ev.planes == 1 ? ev.exit_code ^ 1u
                                     : face_code(fa, 1 - exit_side, xl, ev.den, ncell, ga);
    }
    f(ev, cell);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cell[a] = ncell[a];
      if (grp[a]) {
        --left[a];
        num[a] += 256;
      }
    }
  }
}

// The last event of the lanes before this one (or of earlier chunks).
struct Last {
  int has;
  long long xn0, xn1, xn2, den;
  unsigned entry;
  unsigned attr;   // vertex attribute interpolated to the event (attribute input)
};

template <bool kAttr>
__device__ inline Last shfl_last(const Last& v, int src) {
  Last o;
  o.has = __shfl(v.has, src, 64);
  o.xn0 = __shfl(v.xn0, src, 64);
  o.xn1 = __shfl(v.xn1, src, 64);
  o.xn2 = __shfl(v.xn2, src, 64);
  o.den = __shfl(v.den, src, 64);
  o.entry = __shfl(v.entry, src, 64);
  o.attr = kAttr ? __shfl(v.attr, src, 64) : 0u;
  return o;
}

// Section "Curve voxelization": a line attribute interpolated to the face
// crossing at parameter num / den of the segment whose vertices carry a0 and
// a1, rounded to the nearest integer (halves up), exactly.
__device__ inline unsigned event_attr(unsigned a0, unsigned a1, long long num, long long den) {
  const long long s = 2 * ((long long)a0 * den + ((long long)a1 - (long long)a0) * num) + den;
  return (unsigned)(s / (2 * den));
}

// Plane crossings of segment P0 -> P1 and its last event, without walking
// the events: the last event is the crossing of the largest parameter
// (exact cross-multiplied comparison; on a tie the lowest axis, the face the
// walk in for_each_event gives a simultaneous event), and it enters the
// segment's final voxel.
// (kAttr: also the vertex attribute a0 -> a1 interpolated to that event.)
template <bool kAttr>
__device__ inline uint32_t last_event(const int32_t P0[3], const int32_t P1[3],
                                      const GridArgs& ga, Last& out, unsigned a0 = 0,
                                      unsigned a1 = 0) {
  int64_t d[3], num[3], dn[3];
  int32_t c1[3];
  uint32_t cross = 0;
  bool has[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    d[a] = (int64_t)P1[a] - P0[a];
    const int32_t c0 = P0[a] >> 8;
    c1[a] = P1[a] >> 8;
    const uint32_t n = (uint32_t)abs(c1[a] - c0);
    cross += n;
    has[a] = n != 0;
    num[a] = d[a] > 0 ? 256 * (int64_t)c1[a] - P0[a] : P0[a] - 256 * ((int64_t)c1[a] + 1);
    dn[a] = d[a] > 0 ? d[a] : -d[a];
  }
  if (cross == 0) return 0;
  int fa = -1;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!has[a]) continue;
    if (fa < 0) {
      fa = a;
    } else {
      const int64_t nf = fa == 0 ? num[0] : (fa == 1 ? num[1] : num[2]);
      const int64_t df = fa == 0 ? dn[0] : (fa == 1 ? dn[1] : dn[2]);
      if (num[a] * df > nf * dn[a]) fa = a;
    }
  }
  const int64_t den = fa == 0 ? dn[0] : (fa == 1 ? dn[1] : dn[2]);
  const int64_t nf = fa == 0 ? num[0] : (fa == 1 ? num[1] : num[2]);
  const int64_t df = fa == 0 ? d[0] : (fa == 1 ? d[1] : d[2]);
  int64_t xn[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) xn[b] = (int64_t)P0[b] * den + nf * d[b];
  out.has = 1;
  out.xn0 = xn[0];
  out.xn1 = xn[1];
  out.xn2 = xn[2];
  out.den = den;
  uint32_t xl[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) xl[b] = (uint32_t)xn[b];
  out.entry = face_code(fa, df > 0 ? 0 : 1, xl, (int32_t)den, c1, ga);
  out.attr = kAttr ? event_attr(a0, a1, nf, den) : 0u;
  return cross;
}

// Brick-major index of voxel (x, y, z): bricks of 8^3 voxels, nbx bricks
// along x and nbxy in a z layer of bricks; inside a brick x fastest. A curve's
// consecutive voxels then share cache lines of a per-voxel array far more
// often than in row-major order, where a step in z jumps a whole layer.
__device__ inline uint32_t brick_index(uint32_t x, uint32_t y, uint32_t z, uint32_t nbx,
                                       uint32_t nbxy) {
  return (((x >> 3) + nbx * (y >> 3) + nbxy * (z >> 3)) << 9) |
         ((x & 7u) | (y & 7u) << 3 | (z & 7u) << 6);
}

// Segments with events wait in a per-wave ring in LDS until 64 of them
// (or the curve's last ones) can be walked together, so the event walk runs
// on full waves instead of on the lanes of each 64-segment chunk that happen
// to cross a plane. An entry holds what the walk needs: the segment's
// lattice end points, the curve's crossings before it and the event before
// it (entry code and exact point; den = 0: none).
constexpr int kEmitRing = 128;   // >= 2 * 64 - 1 pending entries
struct EmitRing {
  int32_t p[6][kEmitRing];
  uint32_t g[kEmitRing];
  uint32_t entry[kEmitRing];
  int32_t den[kEmitRing];
  long long x[3][kEmitRing];
};

struct EmitRingAttr : EmitRing {
  uint32_t va[kEmitRing];   // a0 | a1 << 8 | (attribute at the event before) << 16
};

// Lines of every curve in curve order: the line inside a voxel runs from
// one event's entry point to the next event's exit point; it is dropped if
// the two exact points or the two quantized endpoints coincide. The line
// ending at an event goes to slot slot_off[c] + (plane crossings of the curve
// before that event) - 1; slots no line takes keep the invalid mark written
// before the launch. Each line takes its rank in its voxel with one atomic on
// the histogram. With per-vertex attributes (kAttr) every event carries the
// attribute interpolated to it; a line writes its two endpoint attributes to
// ends_out and their mean (rounded down) as its record's attribute byte.
template <bool kFloatIn, bool kAttr>
__global__ __launch_bounds__(kBlock, 4) void k_emit(const float* xyz, const int32_t* lat,
                                                 const int64_t* curve_off, const uint8_t* attr,
                                                 const uint8_t* vattr,
                                                 int64_t n_curves, int64_t curve_base,
                                                 const SnapArgs* sap,
                                                 GridArgs ga, const uint64_t* slot_off,
                                                 uint64_t* rec_out, uint16_t* ends_out,
                                                 uint32_t* vox_out, uint32_t* rank_out,
                                                 uint32_t* hist, uint32_t hist_nbx,
                                                 uint32_t hist_nbxy) {
  using Ring = std::conditional_t<kAttr, EmitRingAttr, EmitRing>;
  __shared__ Ring rings[kWavesPerBlock];
  const int lane = threadIdx.x & 63;
  const SnapArgs sa = kFloatIn ? *sap : SnapArgs{};
  const int64_t c = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (c >= n_curves) return;  // wave-uniform
  Ring& Q = rings[threadIdx.x >> 6];
  const int64_t v0 = curve_off[c], v1 = curve_off[c + 1];
  const uint64_t w0 = slot_off[c], w_end = slot_off[c + 1];
  const uint64_t hi_bits =
      ((uint64_t)(attr ? attr[c] : 255) << 32) | ((uint64_t)((curve_base + c) & 0xFFFFFF) << 40);
  const int64_t gx = ga.g[0], gxy = (int64_t)ga.g[0] * ga.g[1];
  const unsigned long long below = (1ull << lane) - 1ull;

  // walks the first `count` ring entries from `head`, one per lane
  auto walk = [&](uint32_t head, uint32_t count) {
    // ring writes by other lanes of this wave precede these reads (LDS
    // operations of a wave complete in order; the fence keeps the compiler
    // from moving them)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if ((uint32_t)lane >= count) return;
    const uint32_t k = (head + (uint32_t)lane) & (kEmitRing - 1);
    const int32_t P0[3] = {Q.p[0][k], Q.p[1][k], Q.p[2][k]};
    const int32_t P1[3] = {Q.p[3][k], Q.p[4][k], Q.p[5][k]};
    const int32_t bden = Q.den[k];
    const long long bx0 = Q.x[0][k], bx1 = Q.x[1][k], bx2 = Q.x[2][k];
    uint64_t g = Q.g[k];
    bool has_prev = bden != 0, first = true;
    uint32_t prev_entry = Q.entry[k];
    uint32_t va = 0u;
    if constexpr (kAttr) va = Q.va[k];
    uint32_t prev_attr = va >> 16;
    for_each_event<true>(P0, P1, ga, [&](const Ev& ev, const int32_t* cell) {
      const uint32_t ea = kAttr ? event_attr(va & 0xFFu, (va >> 8) & 0xFFu, ev.nf, ev.den) : 0u;
      if (has_prev) {
        const uint64_t w = w0 + (g - 1);
        if (w < w_end) {
          // events of one segment have distinct parameters, so only its
          // first event can coincide with the event before it
          bool same = false;
          if (first) {
            int64_t xn[3];
#pragma unroll
            for (int b = 0; b < 3; ++b)
              xn[b] = (int64_t)P0[b] * ev.den + (int64_t)ev.nf * (P1[b] - P0[b]);
            same = bx0 * ev.den == xn[0] * bden && bx1 * ev.den == xn[1] * bden &&
                   bx2 * ev.den == xn[2] * bden;
          }
          if (!same && prev_entry != ev.exit_code) {
            const uint32_t vid = (uint32_t)(cell[0] + gx * cell[1] + gxy * cell[2]);
            uint64_t hb = hi_bits;
            if (kAttr) {
              hb = (hb & ~(0xFFull << 32)) | ((uint64_t)((prev_attr + ea) >> 1) << 32);
              ends_out[w] = (uint16_t)(prev_attr | (ea << 8));
            }
            rec_out[w] = (uint64_t)prev_entry | ((uint64_t)ev.exit_code << 15) | hb;
            vox_out[w] = vid;
            const uint32_t hv =
                hist_nbx ? brick_index(cell[0], cell[1], cell[2], hist_nbx, hist_nbxy) : vid;
            rank_out[w] = atomicAdd(hist + hv, 1u);
          }
        }
      }
      has_prev = true;
      first = false;
      prev_entry = ev.entry_code;
      prev_attr = ea;
      g += (uint64_t)ev.planes;
    });
  };

  Last carry{0, 0, 0, 0, 1, 0u, 0u};
  uint64_t g0 = 0;       // crossings of the curve before this chunk
  uint32_t q_head = 0, q_n = 0;   // ring state (wave-uniform)
  for (int64_t s0 = v0; s0 + 1 < v1; s0 += 64) {
    const int64_t i = s0 + lane;
    const bool valid = i + 1 < v1;
    int32_t P0[3] = {0, 0, 0}, P1[3] = {0, 0, 0};
    if (valid) {
      load_vertex<kFloatIn>(xyz, lat, i, sa, P0);
      load_vertex<kFloatIn>(xyz, lat, i + 1, sa, P1);
    }
    // plane crossings and the last event. Lines are numbered by crossings
    // (an event of k simultaneous planes uses k numbers), so the numbering
    // needs no walk; the unused numbers stay invalid slots.
    uint32_t e = 0;
    Last mine{0, 0, 0, 0, 1, 0u, 0u};
    uint32_t a01 = 0;
    if (kAttr && valid) a01 = (uint32_t)vattr[i] | ((uint32_t)vattr[i + 1] << 8);
    if (valid) e = last_event<kAttr>(P0, P1, ga, mine, a01 & 0xFFu, a01 >> 8);
    // exclusive prefix sum of the crossing counts
    uint32_t inc = e;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(inc, d, 64);
      if (lane >= d) inc += y;
    }
    const uint32_t base = inc - e;
    const uint32_t total = __shfl(inc, 63, 64);
    // latest lane at or before this one with an event (max scan), then the
    // last event strictly before this lane is that lane's of lane - 1
    int src = mine.has ? lane : -1;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int o = __shfl_up(src, d, 64);
      if (lane >= d) src = o > src ? o : src;
    }
    int prev_src = __shfl_up(src, 1, 64);
    if (lane == 0) prev_src = -1;
    Last before = shfl_last<kAttr>(mine, prev_src >= 0 ? prev_src : 0);
    if (prev_src < 0) before = carry;
    // queue the segments with events
    const bool act = valid && e > 0;
    const unsigned long long am = __ballot(act);
    if (act) {
      const uint32_t k = (q_head + q_n + (uint32_t)__popcll(am & below)) & (kEmitRing - 1);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        Q.p[a][k] = P0[a];
        Q.p[3 + a][k] = P1[a];
      }
      Q.g[k] = (uint32_t)(g0 + base);
      Q.entry[k] = before.entry;
      Q.den[k] = before.has ? (int32_t)before.den : 0;
      Q.x[0][k] = before.xn0;
      Q.x[1][k] = before.xn1;
      Q.x[2][k] = before.xn2;
      if constexpr (kAttr) Q.va[k] = a01 | (before.attr << 16);
    }
    q_n += (uint32_t)__popcll(am);
    // carry the chunk's last event
    const int last_src = __shfl(src, 63, 64);
    if (last_src >= 0) carry = shfl_last<kAttr>(mine, last_src);
    g0 += total;
    if (q_n >= 64) {
      walk(q_head, 64);
      q_head = (q_head + 64) & (kEmitRing - 1);
      q_n -= 64;
    }
  }
  if (q_n > 0) walk(q_head, q_n);
}

// Each emitted line e of voxel v goes to slot offsets[v] + rank[e] of its
// voxel's range, as the pair (v, e): one 8-byte write, so the rank pass reads
// the voxel with the index instead of gathering it.
__global__ __launch_bounds__(kBlock) void k_scatter(const uint32_t* vox, const uint32_t* rank,
                                                    int64_t n_slots, const uint32_t* offsets,
                                                    uint64_t* idx) {
  int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n_slots) return;
  uint32_t v = vox[e];
  if (v == LS_INVALID_VOXEL) return;
  idx[offsets[v] + rank[e]] = ((uint64_t)v << 32) | (uint32_t)e;
}

struct BrickGrid {
  int32_t g[3];          // voxel grid (row-major ids)
  uint32_t nbx, nbxy;    // brick grid (brick_index)
};

// Brick-major -> row-major copy of a per-voxel array. A workgroup moves 8
// bricks consecutive along x (4096 words, one contiguous read) through LDS
// and writes their 64 rows of up to 64 voxels (contiguous writes); grid
// (ceil(nbx / 8), bricks along y, bricks along z).
constexpr int kRunBricks = 8;

__global__ __launch_bounds__(kBlock) void k_from_bricks(const uint32_t* brick, BrickGrid bg,
                                                        uint32_t* rows) {
  __shared__ uint32_t s_b[kRunBricks * 513];   // one padding word per brick: no bank conflicts
  const uint32_t bx0 = blockIdx.x * kRunBricks, by = blockIdx.y, bz = blockIdx.z;
  const uint32_t nb = bg.nbx - bx0 < (uint32_t)kRunBricks ? bg.nbx - bx0 : kRunBricks;
  const uint32_t* src = brick + ((size_t)(bx0 + bg.nbx * by + bg.nbxy * bz) << 9);
  for (uint32_t i = threadIdx.x; i < nb * 512; i += kBlock) s_b[(i >> 9) * 513 + (i & 511)] = src[i];
  __syncthreads();
  const int32_t x0 = 8 * (int32_t)bx0;
#pragma unroll 4
  for (int i = threadIdx.x; i < 64 * 64; i += kBlock) {
    const int xx = i & 63, row = i >> 6;
    const int32_t x = x0 + xx, y = 8 * (int32_t)by + (row & 7), z = 8 * (int32_t)bz + (row >> 3);
    if (x < bg.g[0] && y < bg.g[1] && z < bg.g[2])
      rows[x + (int64_t)bg.g[0] * (y + (int64_t)bg.g[1] * z)] =
          s_b[(xx >> 3) * 513 + ((xx & 7) | (row & 7) << 3 | (row >> 3) << 6)];
  }
}

// Each CSR slot p holds some emitted line e of voxel v; its final position is
// offsets[v] + (number of lines of v emitted before e). A block handles 256
// consecutive slots; the lists overlapping them (slots are grouped by voxel,
// so they span [lo of the first slot's voxel, hi of the last's)) are staged
// in LDS when they fit, else counted from memory.
constexpr int kRankLds = 4096;

__global__ __launch_bounds__(kBlock) void k_rank(const uint64_t* idx, const uint64_t* rec,
                                                 const uint16_t* ends_in, int64_t n_records,
                                                 const uint32_t* offsets, uint64_t* records,
                                                 uint16_t* ends) {
  __shared__ uint32_t s_idx[kRankLds];
  __shared__ uint32_t s_range[2];
  const int64_t p0 = (int64_t)blockIdx.x * kBlock;
  const int64_t p = p0 + threadIdx.x;
  const int64_t n_here = n_records - p0 < kBlock ? n_records - p0 : kBlock;
  uint32_t e = 0, lo = 0, hi = 0;
  if (p < n_records) {
    const uint64_t ve = idx[p];
    e = (uint32_t)ve;
    const uint32_t v = (uint32_t)(ve >> 32);
    lo = offsets[v];
    hi = offsets[v + 1];
  }
  if (threadIdx.x == 0) s_range[0] = lo;
  if ((int64_t)threadIdx.x == n_here - 1) s_range[1] = hi;
  __syncthreads();
  const uint32_t blo = s_range[0], bhi = s_range[1];
  const bool staged = bhi - blo <= (uint32_t)kRankLds;   // block-uniform
  if (staged)
    for (uint32_t q = blo + threadIdx.x; q < bhi; q += kBlock) s_idx[q - blo] = (uint32_t)idx[q];
  __syncthreads();
  if (p >= n_records) return;
  uint32_t r = 0;
  if (staged) {
    for (uint32_t q = lo; q < hi; ++q) r += s_idx[q - blo] < e;
  } else {
    for (uint32_t q = lo; q < hi; ++q) r += (uint32_t)idx[q] < e;
  }
  records[lo + r] = rec[e];
  if (ends) ends[lo + r] = ends_in[e];
}

// Occupancy mask per 4^3 macro cell: bit (x & 3) + 4 (y & 3) + 16 (z & 3) of
// the cell's 64-bit word is set when that voxel's list is not empty. One
// load tells the ray caster which voxels of the macro cell it can skip
// (a zero word: the whole macro cell). The same pass counts the non-empty
// voxels and the longest list (wave and block reduction, one atomic each per
// workgroup).
__global__ __launch_bounds__(kBlock) void k_occupancy(const uint32_t* offsets, GridArgs ga,
                                                      int32_t mx, int32_t my, int32_t mz,
                                                      unsigned long long* occ,
                                                      unsigned long long* nonempty,
                                                      unsigned int* max_list) {
  __shared__ unsigned long long s_ne[kBlock / 64];
  __shared__ unsigned s_mx[kBlock / 64];
  int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int64_t nm = (int64_t)mx * my * mz;
  unsigned long long ne = 0;
  unsigned mxl = 0;
  if (m < nm) {
    int32_t bx = (int32_t)(m % mx), by = (int32_t)((m / mx) % my),
            bz = (int32_t)(m / ((int64_t)mx * my));
    unsigned long long bits = 0;
    if ((ga.g[0] & 3) == 0) {
      // whole macro cells along x: a row of 4 voxels is one aligned 16-byte
      // load of their offsets plus the next row start
#pragma unroll 4
      for (int r = 0; r < 16; ++r) {
        const int32_t y = 4 * by + (r & 3), z = 4 * bz + (r >> 2);
        if (y >= ga.g[1] || z >= ga.g[2]) continue;
        const int64_t v = 4 * (int64_t)bx + (int64_t)ga.g[0] * (y + (int64_t)ga.g[1] * z);
        const uint4 a = *reinterpret_cast<const uint4*>(offsets + v);
        const uint32_t e = offsets[v + 4];
        const unsigned n[4] = {a.y - a.x, a.z - a.y, a.w - a.z, e - a.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (n[c] > 0) bits |= 1ull << (4 * r + c);
          mxl = n[c] > mxl ? n[c] : mxl;
        }
      }
    } else {
      for (int k = 0; k < 64; ++k) {
        const int32_t x = 4 * bx + (k & 3), y = 4 * by + ((k >> 2) & 3), z = 4 * bz + (k >> 4);
        if (x >= ga.g[0] || y >= ga.g[1] || z >= ga.g[2]) continue;
        const int64_t v = x + (int64_t)ga.g[0] * (y + (int64_t)ga.g[1] * z);
        const unsigned n = offsets[v + 1] - offsets[v];
        if (n > 0) bits |= 1ull << k;
        mxl = n > mxl ? n : mxl;
      }
    }
    occ[m] = bits;
    ne = (unsigned long long)__popcll(bits);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    ne += __shfl_xor(ne, d, 64);
    const unsigned o = __shfl_xor(mxl, d, 64);
    mxl = o > mxl ? o : mxl;
  }
  if ((threadIdx.x & 63) == 0) {
    s_ne[threadIdx.x >> 6] = ne;
    s_mx[threadIdx.x >> 6] = mxl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
      ne += s_ne[w];
      mxl = s_mx[w] > mxl ? s_mx[w] : mxl;
    }
    if (ne) atomicAdd(nonempty, ne);
    if (mxl) atomicMax(max_list, mxl);
  }
}


// Per-block bounds of the vertices (min and max are exact in fp32; widened
// to fp64 for the set-up). kVec: xyz 16-byte aligned, read as three float4
// per 4 vertices.
template <bool kVec>
__global__ __launch_bounds__(kBlock) void k_bbox(const float* xyz, int64_t nv, double* part,
                                                 int* bad) {
  __shared__ double s[6][kBlock];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool fin = true;
  auto take = [&](int a, float x) {
    fin &= isfinite(x);
    lo[a] = fminf(lo[a], x);
    hi[a] = fmaxf(hi[a], x);
  };
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t v_tail = 0;
  if (kVec) {
    const float4* g4 = reinterpret_cast<const float4*>(xyz);
    const int64_t ng = nv / 4;
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < ng; g += stride) {
      const float4 a = g4[3 * g], b = g4[3 * g + 1], c = g4[3 * g + 2];
      take(0, a.x); take(1, a.y); take(2, a.z);
      take(0, a.w); take(1, b.x); take(2, b.y);
      take(0, b.z); take(1, b.w); take(2, c.x);
      take(0, c.y); take(1, c.z); take(2, c.w);
    }
    v_tail = 4 * ng;
  }
  for (int64_t v = v_tail + (int64_t)blockIdx.x * kBlock + threadIdx.x; v < nv; v += stride) {
#pragma unroll
    for (int a = 0; a < 3; ++a) take(a, xyz[3 * v + a]);
  }
  if (!fin) *bad = 1;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    s[a][threadIdx.x] = (double)lo[a];
    s[3 + a][threadIdx.x] = (double)hi[a];
  }
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = fmin(s[a][threadIdx.x], s[a][threadIdx.x + st]);
        s[3 + a][threadIdx.x] = fmax(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + st]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int a = 0; a < 6; ++a) part[6 * blockIdx.x + a] = s[a][0];
}

// Reduces k_bbox's per-block bounds and writes the lattice set-up; flags
// non-finite input (bad, from k_bbox) in err.
__global__ __launch_bounds__(kBlock) void k_lattice(const double* part, int blocks, int64_t nv,
                                                    GridArgs ga, const int* bad, SnapArgs* out,
                                                    int* err) {
  __shared__ double s[6][kBlock];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < blocks; b += kBlock) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fmin(lo[a], part[6 * b + a]);
      hi[a] = fmax(hi[a], part[6 * b + 3 + a]);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    s[a][threadIdx.x] = lo[a];
    s[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = fmin(s[a][threadIdx.x], s[a][threadIdx.x + st]);
        s[3 + a][threadIdx.x] = fmax(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + st]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double l[3], h[3];
    for (int a = 0; a < 3; ++a) {
      l[a] = nv > 0 ? s[a][0] : 0.0;
      h[a] = nv > 0 ? s[3 + a][0] : 0.0;
    }
    SnapArgs r;
    for (int a = 0; a < 3; ++a) r.lo[a] = l[a];
    r.scale = lattice_scale(l, h, ga.g);
    *out = r;
    if (*bad) atomicOr(err, kErrNonFinite);
  }
}

__global__ __launch_bounds__(kBlock) void k_snap(const float* xyz, int64_t nv, SnapArgs sa,
                                                 int32_t* lat) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= 3 * nv) return;
  int a = (int)(i % 3);
  lat[i] = snap_coord(xyz[i], sa.lo[a], sa.scale);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Grids from this many voxels count lines in brick-major order: their 4-byte
// per-voxel array (128 MiB and up) no longer sits comfortably in the 256 MB
// last-level cache, so the emit's row-major atomics would go to HBM at random.
constexpr int64_t kBrickMinVoxels = int64_t(1) << 25;
inline unsigned curve_blocks(int64_t n) {
  return (unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock);
}

// Temporary device buffer from the memory cache; released after the stream
// it was used on has drained.
struct DeviceBuf {
  void* p = nullptr;
  hipStream_t st = nullptr;
  explicit DeviceBuf(hipStream_t s) : st(s) {}
  DeviceBuf(const DeviceBuf&) = delete;
  DeviceBuf& operator=(const DeviceBuf&) = delete;
  ~DeviceBuf() {
    if (p) {
      (void)hipStreamSynchronize(st);
      pool_free(p);
    }
  }
  int alloc(size_t bytes) { return pool_alloc(bytes, &p, nullptr); }
  template <typename T>
  T* as() { return static_cast<T*>(p); }
};

}  // namespace

int vox_bbox(const float* xyz, int64_t nv, double lo[3], double hi[3], hipStream_t st) {
  for (int a = 0; a < 3; ++a) {
    lo[a] = 0.0;
    hi[a] = 0.0;
  }
  if (nv <= 0) return LS_OK;
  int64_t blocks = (nv + kBlock - 1) / kBlock;
  if (blocks > 1024) blocks = 1024;
  DeviceBuf part(st), bad(st);
  int rc;
  if ((rc = part.alloc(sizeof(double) * 6 * blocks)) || (rc = bad.alloc(sizeof(int)))) return rc;
  LS_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), st));
  if ((reinterpret_cast<uintptr_t>(xyz) & 15) == 0)
    hipLaunchKernelGGL(k_bbox<true>, dim3((unsigned)blocks), dim3(kBlock), 0, st, xyz, nv,
                       part.as<double>(), bad.as<int>());
  else
    hipLaunchKernelGGL(k_bbox<false>, dim3((unsigned)blocks), dim3(kBlock), 0, st, xyz, nv,
                       part.as<double>(), bad.as<int>());
  LS_HIP(hipGetLastError());
  std::vector<double> h(6 * blocks);
  int hbad = 0;
  LS_HIP(hipMemcpyAsync(h.data(), part.p, sizeof(double) * 6 * blocks, hipMemcpyDeviceToHost, st));
  LS_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  LS_HIP(hipStreamSynchronize(st));
  if (hbad) {
    ls_set_error("non-finite vertex coordinate");
    return LS_EINVAL;
  }
  for (int a = 0; a < 3; ++a) {
    lo[a] = INFINITY;
    hi[a] = -INFINITY;
  }
  for (int64_t b = 0; b < blocks; ++b)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::fmin(lo[a], h[6 * b + a]);
      hi[a] = std::fmax(hi[a], h[6 * b + 3 + a]);
    }
  return LS_OK;
}

double vox_scale(const double lo[3], const double hi[3], const int32_t grid[3]) {
  return lattice_scale(lo, hi, grid);
}

int vox_snap(const float* xyz, int64_t nv, SnapArgs sa, int32_t* lat, hipStream_t st) {
  if (nv <= 0) return LS_OK;
  hipLaunchKernelGGL(k_snap, dim3(blocks_for(3 * nv)), dim3(kBlock), 0, st, xyz, nv, sa, lat);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

int vox_build(ls_lineset* s, const float* xyz, const int32_t* lat, const int64_t* curve_off,
              const uint8_t* attr, const uint8_t* vattr, hipStream_t st) {
  GridArgs ga;
  for (int a = 0; a < 3; ++a) ga.g[a] = s->grid[a];
  ga.bins = s->bins;
  int sh = 0;
  while ((256 >> sh) > s->bins) ++sh;
  ga.bin_shift = sh;  // 256 / bins = 2^sh
  const int64_t C = s->n_curves;
  const bool float_in = xyz != nullptr;
  int rc;

  // 0. float input: grid set-up on the device (bounds, then the lattice
  //    scale), read back with the slot count below
  const int64_t nv = s->n_vertices;
  const int bb_blocks = (int)std::min<int64_t>(std::max<int64_t>((nv + kBlock - 1) / kBlock, 1), 1024);
  // The slot counts [C + 1] (the scan leaves their total at [C]) are
  // followed in the same buffer by the grid set-up and the error flags, so
  // one copy reads all three back.
  struct Header {
    uint64_t n_slots;
    SnapArgs sa;
    int err[2];
  };
  static_assert(sizeof(Header) == sizeof(uint64_t) + sizeof(SnapArgs) + 2 * sizeof(int),
                "header layout");
  const size_t slot_bytes = sizeof(uint64_t) * (C + 1);
  DeviceBuf slots(st), sums64(st), lattice(st);
  if ((rc = slots.alloc(slot_bytes + sizeof(SnapArgs) + 2 * sizeof(int))) ||
      (rc = sums64.alloc(sizeof(uint64_t) * scan_block_sums_len(C))) ||
      (rc = lattice.alloc(sizeof(double) * 6 * bb_blocks)))
    return rc;
  SnapArgs* sad = reinterpret_cast<SnapArgs*>(slots.as<char>() + slot_bytes);
  int* errp = reinterpret_cast<int*>(sad + 1);
  LS_HIP(hipMemsetAsync(errp, 0, 2 * sizeof(int), st));
  if (float_in) {
    double* part = lattice.as<double>();
    if ((reinterpret_cast<uintptr_t>(xyz) & 15) == 0)
      hipLaunchKernelGGL(k_bbox<true>, dim3((unsigned)bb_blocks), dim3(kBlock), 0, st, xyz, nv,
                         part, errp + 1);
    else
      hipLaunchKernelGGL(k_bbox<false>, dim3((unsigned)bb_blocks), dim3(kBlock), 0, st, xyz, nv,
                         part, errp + 1);
    hipLaunchKernelGGL(k_lattice, dim3(1), dim3(kBlock), 0, st, part, bb_blocks, nv, ga,
                       errp + 1, sad, errp);
    LS_HIP(hipGetLastError());
  }
  // 1. per-curve slot counts + validation
  if (C > 0) {
    if (float_in)
      hipLaunchKernelGGL((k_count<true>), dim3(curve_blocks(C)), dim3(kBlock), 0, st, xyz, lat,
                         curve_off, C, s->n_vertices, sad, ga, slots.as<uint64_t>(), errp);
    else
      hipLaunchKernelGGL((k_count<false>), dim3(curve_blocks(C)), dim3(kBlock), 0, st, xyz, lat,
                         curve_off, C, s->n_vertices, sad, ga, slots.as<uint64_t>(), errp);
    LS_HIP(hipGetLastError());
  }
  if ((rc = exclusive_scan_u64(slots.as<uint64_t>(), slots.as<uint64_t>(), C, sums64.as<uint64_t>(),
                               st)))
    return rc;
  Header hh{};
  LS_HIP(hipMemcpyAsync(&hh, slots.as<uint64_t>() + C, sizeof(Header), hipMemcpyDeviceToHost, st));
  LS_HIP(hipStreamSynchronize(st));
  const uint64_t n_slots = hh.n_slots;
  const int herr = hh.err[0];
  const SnapArgs hsa = hh.sa;
  if (herr & kErrNonFinite) {
    ls_set_error("non-finite vertex coordinate");
    return LS_EINVAL;
  }
  if (float_in) {
    for (int a = 0; a < 3; ++a) s->lo_scale[a] = hsa.lo[a];
    s->lo_scale[3] = hsa.scale;
  }
  if (herr & kErrOffsets) {
    ls_set_error("curve_off must start at 0, be non-decreasing and end at most at n_vertices");
    return LS_EINVAL;
  }
  if (herr & kErrRange) {
    ls_set_error("a vertex lies outside [0, 256 * grid) in lattice units");
    return LS_EINVAL;
  }
  if (n_slots >= 0xFFFFFFFFull) {
    ls_set_error("too many per-voxel lines (%llu slots >= 2^32 - 1)", (unsigned long long)n_slots);
    return LS_ENOMEM;
  }
  s->n_slots = (int64_t)n_slots;

  // 2. offsets array (owned by the set) doubles as the histogram; on grids
  // whose per-voxel array outgrows the last-level cache the lines are counted
  // in a brick-major array instead (the emit's atomics then follow a curve
  // through nearby cache lines), copied to row-major order before the scan
  if ((rc = ls_alloc(s, (void**)&s->offsets, sizeof(uint32_t) * (s->nvox + 1)))) return rc;
  const bool bricks = s->nvox >= kBrickMinVoxels;
  BrickGrid bg{};
  for (int a = 0; a < 3; ++a) bg.g[a] = s->grid[a];
  DeviceBuf hist_b(st);
  if (bricks) {
    bg.nbx = (uint32_t)(s->grid[0] + 7) / 8;
    bg.nbxy = bg.nbx * (uint32_t)((s->grid[1] + 7) / 8);
    const int64_t nb = (int64_t)bg.nbxy * ((s->grid[2] + 7) / 8) * 512;
    if ((rc = hist_b.alloc(sizeof(uint32_t) * nb))) return rc;
    if ((rc = fill_u32(hist_b.as<uint32_t>(), 0u, nb, st))) return rc;
  } else if ((rc = fill_u32(s->offsets, 0u, s->nvox + 1, st))) {
    return rc;
  }
  uint32_t* hist = bricks ? hist_b.as<uint32_t>() : s->offsets;

  // 3. emit
  DeviceBuf rec(st), vox(st), rank(st), sums32(st), ends_slots(st);
  if ((rc = rec.alloc(sizeof(uint64_t) * n_slots)) || (rc = vox.alloc(sizeof(uint32_t) * n_slots)) ||
      (rc = rank.alloc(sizeof(uint32_t) * n_slots)) ||
      (rc = sums32.alloc(sizeof(uint32_t) * scan_block_sums_len(s->nvox))))
    return rc;
  if (vattr && (rc = ends_slots.alloc(sizeof(uint16_t) * (n_slots ? n_slots : 1)))) return rc;
  if ((rc = fill_u32(vox.as<uint32_t>(), LS_INVALID_VOXEL, (int64_t)n_slots, st))) return rc;
  if (C > 0) {
    const dim3 grid(curve_blocks(C)), block(kBlock);
    uint16_t* eo = vattr ? ends_slots.as<uint16_t>() : nullptr;
    if (float_in && vattr)
      hipLaunchKernelGGL((k_emit<true, true>), grid, block, 0, st, xyz, lat, curve_off, attr,
                         vattr, C, s->curve_base, sad, ga, slots.as<uint64_t>(),
                         rec.as<uint64_t>(), eo, vox.as<uint32_t>(), rank.as<uint32_t>(),
                         hist, bg.nbx, bg.nbxy);
    else if (float_in)
      hipLaunchKernelGGL((k_emit<true, false>), grid, block, 0, st, xyz, lat, curve_off, attr,
                         vattr, C, s->curve_base, sad, ga, slots.as<uint64_t>(),
                         rec.as<uint64_t>(), eo, vox.as<uint32_t>(), rank.as<uint32_t>(),
                         hist, bg.nbx, bg.nbxy);
    else if (vattr)
      hipLaunchKernelGGL((k_emit<false, true>), grid, block, 0, st, xyz, lat, curve_off, attr,
                         vattr, C, s->curve_base, sad, ga, slots.as<uint64_t>(),
                         rec.as<uint64_t>(), eo, vox.as<uint32_t>(), rank.as<uint32_t>(),
                         hist, bg.nbx, bg.nbxy);
    else
      hipLaunchKernelGGL((k_emit<false, false>), grid, block, 0, st, xyz, lat, curve_off, attr,
                         vattr, C, s->curve_base, sad, ga, slots.as<uint64_t>(),
                         rec.as<uint64_t>(), eo, vox.as<uint32_t>(), rank.as<uint32_t>(),
                         hist, bg.nbx, bg.nbxy);
    LS_HIP(hipGetLastError());
  }

  // 4. counts -> offsets (in place)
  if (bricks) {
    const dim3 grid((bg.nbx + kRunBricks - 1) / kRunBricks, (s->grid[1] + 7) / 8,
                    (s->grid[2] + 7) / 8);
    hipLaunchKernelGGL(k_from_bricks, grid, dim3(kBlock), 0, st, hist_b.as<uint32_t>(), bg,
                       s->offsets);
    LS_HIP(hipGetLastError());
  }
  if ((rc = exclusive_scan_u32(s->offsets, s->offsets, s->nvox, sums32.as<uint32_t>(), st)))
    return rc;
  uint32_t n_rec = 0;
  LS_HIP(hipMemcpyAsync(&n_rec, s->offsets + s->nvox, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  LS_HIP(hipStreamSynchronize(st));
  s->n_records = n_rec;

  // 5. scatter + rank/gather into the set's record array
  if ((rc = ls_alloc(s, (void**)&s->records, sizeof(uint64_t) * (n_rec ? n_rec : 1)))) return rc;
  if (vattr && (rc = ls_alloc(s, (void**)&s->ends, sizeof(uint16_t) * (n_rec ? n_rec : 1))))
    return rc;
  DeviceBuf idx(st);
  if ((rc = idx.alloc(sizeof(uint64_t) * (n_rec ? n_rec : 1)))) return rc;
  if (n_slots > 0) {
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for((int64_t)n_slots)), dim3(kBlock), 0, st,
                       vox.as<uint32_t>(), rank.as<uint32_t>(), (int64_t)n_slots, s->offsets,
                       idx.as<uint64_t>());
    LS_HIP(hipGetLastError());
  }
  if (n_rec > 0) {
    hipLaunchKernelGGL(k_rank, dim3(blocks_for(n_rec)), dim3(kBlock), 0, st, idx.as<uint64_t>(),
                       rec.as<uint64_t>(), vattr ? ends_slots.as<uint16_t>() : nullptr,
                       (int64_t)n_rec, s->offsets, s->records, vattr ? s->ends : nullptr);
    LS_HIP(hipGetLastError());
  }

  // 6. macro-cell occupancy and list statistics
  if ((rc = vox_occupancy(s, st))) return rc;
  LS_HIP(hipStreamSynchronize(st));
  return LS_OK;
}

// Macro-cell occupancy words and list statistics of s->offsets; the
// statistics stay on the device after the occupancy words until
// lineset_info asks for them.
int vox_occupancy(ls_lineset* s, hipStream_t st) {
  GridArgs ga;
  for (int a = 0; a < 3; ++a) ga.g[a] = s->grid[a];
  ga.bins = s->bins;
  ga.bin_shift = 0;
  for (int a = 0; a < 3; ++a) s->macro[a] = (s->grid[a] + 3) / 4;
  int64_t nm = (int64_t)s->macro[0] * s->macro[1] * s->macro[2];
  int rc;
  if ((rc = ls_alloc(s, (void**)&s->occupancy, sizeof(uint64_t) * (nm + 2)))) return rc;
  char* stats = reinterpret_cast<char*>(s->occupancy + nm);
  LS_HIP(hipMemsetAsync(stats, 0, 16, st));
  hipLaunchKernelGGL(k_occupancy, dim3(blocks_for(nm)), dim3(kBlock), 0, st, s->offsets, ga,
                     s->macro[0], s->macro[1], s->macro[2], (unsigned long long*)s->occupancy,
                     reinterpret_cast<unsigned long long*>(stats),
                     reinterpret_cast<unsigned int*>(stats + 8));
  LS_HIP(hipGetLastError());
  s->stats_pending = true;
  return LS_OK;
}
