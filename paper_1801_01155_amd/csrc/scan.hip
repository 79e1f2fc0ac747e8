// Exclusive prefix sums (reduce-then-scan) and fill kernels for gfx950.
//
// A tile is 256 threads x 16 items. Pass 1 reduces each tile to one sum,
// pass 2 scans the tile sums in one workgroup, pass 3 rescans each tile with
// its offset. Tiles are staged through LDS so global loads and stores stay
// coalesced while each thread scans 16 consecutive items in registers.
#include "ls_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;
constexpr int kWaves = kThreads / 64;

template <typename T>
__device__ inline T wave_inclusive_scan(T x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

template <typename T>
__device__ inline T wave_reduce(T x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Loads a tile into `items` in blocked order (thread t owns elements
// t*kItems .. t*kItems + kItems - 1), via LDS, zero beyond n.
template <typename T>
__device__ inline void load_tile(const T* in, int64_t base, int64_t n, T (&items)[kItems],
                                 T* lds) {
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    lds[k * kThreads + threadIdx.x] = i < n ? in[i] : T(0);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kItems; ++k) items[k] = lds[threadIdx.x * kItems + k];
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_tile_reduce(const T* in, int64_t n, T* sums) {
  __shared__ T wsum[kWaves];
  int64_t base = (int64_t)blockIdx.x * kTile;
  T acc = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    if (i < n) acc += in[i];
  }
  acc = wave_reduce(acc);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T t = 0;
    for (int w = 0; w < kWaves; ++w) t += wsum[w];
    sums[blockIdx.x] = t;
  }
}

// One workgroup of 1024 threads scans `n` tile sums in place (exclusive) and
// writes the grand total to total[0].
template <typename T>
__global__ __launch_bounds__(1024) void k_scan_sums(T* sums, int64_t n, T* total) {
  __shared__ T wsum[16];
  __shared__ T carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += 1024) {
    int64_t i = base + threadIdx.x;
    T x = i < n ? sums[i] : T(0);
    T inc = wave_inclusive_scan(x);
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
    __syncthreads();
    T wpre = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wpre += wsum[w];
    T carry = carry_s;
    if (i < n) sums[i] = carry + wpre + inc - x;
    __syncthreads();
    if (threadIdx.x == 1023) carry_s = carry + wpre + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) total[0] = carry_s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_tile_scan(const T* in, T* out, int64_t n,
                                                        const T* tile_off) {
  __shared__ T lds[kTile];
  __shared__ T wsum[kWaves];
  int64_t base = (int64_t)blockIdx.x * kTile;
  T items[kItems];
  load_tile(in, base, n, items, lds);
  T tsum = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) tsum += items[k];
  T inc = wave_inclusive_scan(tsum);
  if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = inc;
  __syncthreads();
  T pre = tile_off[blockIdx.x];
  for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) pre += wsum[w];
  pre += inc - tsum;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    T x = items[k];
    lds[threadIdx.x * kItems + k] = pre;
    pre += x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    if (i < n) out[i] = lds[k * kThreads + threadIdx.x];
  }
}

template <typename T>
int scan_impl(const T* in, T* out, int64_t n, T* sums, hipStream_t st) {
  int64_t tiles = (n + kTile - 1) / kTile;
  if (tiles == 0) {
    // total of an empty range
    hipLaunchKernelGGL((k_scan_sums<T>), dim3(1), dim3(1024), 0, st, sums, (int64_t)0, out);
    LS_HIP(hipGetLastError());
    return LS_OK;
  }
  hipLaunchKernelGGL((k_tile_reduce<T>), dim3((unsigned)tiles), dim3(kThreads), 0, st, in, n, sums);
  LS_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_scan_sums<T>), dim3(1), dim3(1024), 0, st, sums, tiles, out + n);
  LS_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_tile_scan<T>), dim3((unsigned)tiles), dim3(kThreads), 0, st, in, out, n,
                     (const T*)sums);
  LS_HIP(hipGetLastError());
  return LS_OK;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

}  // namespace

int64_t scan_block_sums_len(int64_t n) { return (n + kTile - 1) / kTile + 1; }

int exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* sums,
                       hipStream_t st) {
  return scan_impl<uint32_t>(in, out, n, sums, st);
}

int exclusive_scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* sums,
                       hipStream_t st) {
  return scan_impl<uint64_t>(in, out, n, sums, st);
}

int fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return LS_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
  LS_HIP(hipGetLastError());
  return LS_OK;
}
