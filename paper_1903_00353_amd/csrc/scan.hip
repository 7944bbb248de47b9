// Exclusive prefix sum over int32 (tile sums, then either each tile's own
// offset from the sums before it, or a scan of the tile sums in one block
// followed by each tile's scan plus its offset).
#include "internal.h"

namespace csc {

constexpr int SB = 256;           // threads per block
constexpr int SITEMS = 8;         // items per thread
constexpr int STILE = SB * SITEMS;

__device__ inline int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// exclusive scan of one value per thread across the block; *tot gets the block total
template <int NT>
__device__ inline int block_excl_scan(int v, int* tot) {
  __shared__ int wsum[NT / 64 + 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int inc = wave_incl_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (w == 0) {
    int x = lane < NT / 64 ? wsum[lane] : 0;
    int xi = wave_incl_scan(x);
    if (lane < NT / 64) wsum[lane] = xi - x;
    if (lane == NT / 64 - 1) wsum[NT / 64] = xi;
  }
  __syncthreads();
  int res = inc - v + wsum[w];
  *tot = wsum[NT / 64];
  __syncthreads();
  return res;
}

__global__ __launch_bounds__(SB) void k_tile_sums(const int32_t* __restrict__ in, int64_t n, int32_t* sums) {
  int64_t base = (int64_t)blockIdx.x * STILE;
  int s = 0;
  for (int i = threadIdx.x; i < STILE; i += SB) {
    int64_t idx = base + i;
    if (idx < n) s += in[idx];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  __shared__ int ws[SB / 64];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < SB / 64; w++) t += ws[w];
    sums[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(1024) void k_scan_sums(int32_t* sums, int64_t nb, int64_t* total_i64, int32_t* total_i32) {
  __shared__ int carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += 1024) {
    int64_t idx = base + threadIdx.x;
    int v = idx < nb ? sums[idx] : 0;
    int tot;
    int ex = block_excl_scan<1024>(v, &tot);
    int carry = carry_s;
    if (idx < nb) sums[idx] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry_s = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (total_i64) *total_i64 = carry_s;
    if (total_i32) *total_i32 = carry_s;
  }
}

__global__ __launch_bounds__(SB) void k_scan_tiles(const int32_t* in, int32_t* out, int64_t n, const int32_t* sums) {
  __shared__ int tile[STILE];
  int64_t base = (int64_t)blockIdx.x * STILE;
  for (int i = threadIdx.x; i < STILE; i += SB) {
    int64_t idx = base + i;
    tile[i] = idx < n ? in[idx] : 0;
  }
  __syncthreads();
  int loc[SITEMS];
  int s = 0;
#pragma unroll
  for (int k = 0; k < SITEMS; k++) {
    loc[k] = s;
    s += tile[threadIdx.x * SITEMS + k];
  }
  int tot;
  int ex = block_excl_scan<SB>(s, &tot) + sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SITEMS; k++) tile[threadIdx.x * SITEMS + k] = ex + loc[k];
  __syncthreads();
  for (int i = threadIdx.x; i < STILE; i += SB) {
    int64_t idx = base + i;
    if (idx < n) out[idx] = tile[i];
  }
}

// With few tiles each block adds up the sums of the tiles before it itself (at
// most SHORT_TILES ints, coalesced), which saves the launch that scans the tile
// sums; the last block stores the total.
constexpr int64_t SHORT_TILES = 4096;

__global__ __launch_bounds__(SB) void k_scan_tiles_short(const int32_t* in, int32_t* out, int64_t n,
                                                         const int32_t* __restrict__ sums, int64_t* total_i64,
                                                         int32_t* total_i32) {
  __shared__ int tile[STILE];
  __shared__ int ws[SB / 64];
  const int64_t base = (int64_t)blockIdx.x * STILE;
  int pre = 0;
  for (int j = threadIdx.x; j < (int)blockIdx.x; j += SB) pre += sums[j];
  for (int i = threadIdx.x; i < STILE; i += SB) {
    const int64_t idx = base + i;
    tile[i] = idx < n ? in[idx] : 0;
  }
  for (int o = 32; o > 0; o >>= 1) pre += __shfl_down(pre, o, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = pre;
  __syncthreads();
  int offset = 0;
#pragma unroll
  for (int w = 0; w < SB / 64; w++) offset += ws[w];
  int loc[SITEMS];
  int s = 0;
#pragma unroll
  for (int k = 0; k < SITEMS; k++) {
    loc[k] = s;
    s += tile[threadIdx.x * SITEMS + k];
  }
  int tot;
  const int ex = block_excl_scan<SB>(s, &tot) + offset;
#pragma unroll
  for (int k = 0; k < SITEMS; k++) tile[threadIdx.x * SITEMS + k] = ex + loc[k];
  __syncthreads();
  for (int i = threadIdx.x; i < STILE; i += SB) {
    const int64_t idx = base + i;
    if (idx < n) out[idx] = tile[i];
  }
  if (threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) {
    if (total_i64) *total_i64 = offset + tot;
    if (total_i32) *total_i32 = offset + tot;
  }
}

int64_t scan_tmp_ints(int64_t n) { return (n + STILE - 1) / STILE + 1; }

hipError_t scan_sums_inplace(int32_t* sums, int64_t nb, int64_t* total_i64, hipStream_t s) {
  k_scan_sums<<<1, 1024, 0, s>>>(sums, nb, total_i64, nullptr);
  return hipGetLastError();
}

hipError_t exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, int64_t* total_i64,
                          int32_t* total_i32, hipStream_t s) {
  int64_t nb = (n + STILE - 1) / STILE;
  if (nb < 1) nb = 1;
  k_tile_sums<<<(unsigned)nb, SB, 0, s>>>(in, n, tmp);
  if (nb <= SHORT_TILES) {
    k_scan_tiles_short<<<(unsigned)nb, SB, 0, s>>>(in, out, n, tmp, total_i64, total_i32);
  } else {
    k_scan_sums<<<1, 1024, 0, s>>>(tmp, nb, total_i64, total_i32);
    k_scan_tiles<<<(unsigned)nb, SB, 0, s>>>(in, out, n, tmp);
  }
  return hipGetLastError();
}

}  // namespace csc
