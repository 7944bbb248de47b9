// Stable LSD radix sort of (key, value) pairs on the low `bits` key bits, 8 bits
// per pass (wider digits make the digit-major histogram as long as the data:
// 11-bit digits in tiles of 2048 pairs doubled the sort time). It groups
// triangle corners by vertex (stable, so each vertex's corners come out in
// ascending order) and orders soup corners by coordinate.
//
// Each pass runs three launches over tiles of RsCfg::TILE pairs (16 pairs per
// thread: 4096 pairs in blocks of 256 threads, or 8192 in blocks of 512 once
// the input fills at least 1536 such tiles, three for each block slot of the
// device at two 75 KB blocks per CU; below that the longer tiles leave slots
// idle and the shorter ones win):
//  * k_rs_hist: the digit histogram of every tile, stored digit-major
//    (hist[d * ntiles + tile]), counted with LDS integer atomics;
//  * an exclusive scan of that array: the output offset of (digit, tile);
//  * k_rs_scatter: every tile ranks its pairs stably per digit, stages them in
//    LDS in digit order and writes each digit's run to its offset, so that
//    consecutive threads write consecutive addresses.
// Tile item (w, r, lane) is pair (w * ROUNDS + r) * 64 + lane of the tile: wave
// w takes its pairs in ROUNDS rounds of 64 consecutive ones, so the order of
// (w, r, lane) is the input order and ranks follow it. Inside a round the lanes
// holding the same digit are found with one ballot per digit bit; each wave
// keeps running per-digit counts in LDS, advanced by the last lane of each
// digit group. No memset and no host synchronisation: safe to capture in a
// graph.
#include "internal.h"

namespace csc {

// digit width RB and block size TH: the tile is 16 pairs per thread
template <int RB, int TH>
struct RsCfg {
  static constexpr int BINS = 1 << RB;
  static constexpr int THREADS = TH;
  static constexpr int WAVES = TH / 64;
  static constexpr int ROUNDS = 16;
  static constexpr int TILE = TH * ROUNDS;
  // digits per thread in the per-tile tables (threads past the digits hold none)
  static constexpr int PER = BINS >= TH ? BINS / TH : 1;
  static_assert(BINS % TH == 0 || TH % BINS == 0, "whole digits per thread");
};

template <int RB, int TH>
__global__ __launch_bounds__(TH) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                int64_t ntiles, int32_t* hist) {
  using C = RsCfg<RB, TH>;
  __shared__ int s_h[C::BINS];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int b = t; b < C::BINS; b += TH) s_h[b] = 0;
  __syncthreads();
  const int64_t base = blockIdx.x * (int64_t)C::TILE + w * (C::ROUNDS * 64) + lane;
#pragma unroll 8
  for (int r = 0; r < C::ROUNDS; r++)
    if (base + r * 64 < n) atomicAdd(&s_h[(keys[base + r * 64] >> shift) & (C::BINS - 1)], 1);
  __syncthreads();
  for (int b = t; b < C::BINS; b += TH) hist[(int64_t)b * ntiles + blockIdx.x] = s_h[b];
}

// exclusive scan of one value per thread across the block of WAVES wavefronts
template <int WAVES>
__device__ inline int rs_block_excl(int v, int* s_w) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  int before = 0;
#pragma unroll
  for (int u = 0; u < WAVES; u++) before += u < w ? s_w[u] : 0;
  return before + inc - v;
}

// vin may be null: the values are then the input positions
template <int RB, int TH>
__global__ __launch_bounds__(TH) void k_rs_scatter(const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                                   uint32_t* kout, int32_t* vout, int64_t n, int shift,
                                                   int64_t ntiles, const int32_t* __restrict__ off) {
  using C = RsCfg<RB, TH>;
  __shared__ int s_cnt[C::WAVES][C::BINS];  // running, then starting, tile position of each digit per wave
  __shared__ int s_delta[C::BINS];          // output offset of each digit's run minus its tile start
  __shared__ int s_w[C::WAVES];
  __shared__ uint32_t s_k[C::TILE];
  __shared__ int32_t s_v[C::TILE];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int b = t; b < C::BINS; b += TH) {
#pragma unroll
    for (int u = 0; u < C::WAVES; u++) s_cnt[u][b] = 0;
  }
  __syncthreads();
  const int64_t tile0 = blockIdx.x * (int64_t)C::TILE;
  const int64_t base = tile0 + w * (C::ROUNDS * 64) + lane;
  uint32_t k[C::ROUNDS];
  int32_t v[C::ROUNDS];
#pragma unroll
  for (int r = 0; r < C::ROUNDS; r++) {
    const int64_t i = base + r * 64;
    const bool ok = i < n;
    k[r] = ok ? kin[i] : 0u;
    v[r] = ok ? (vin ? vin[i] : (int32_t)i) : 0;
  }
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const unsigned long long above = lane == 63 ? 0ull : (~0ull << (lane + 1));
  int pos[C::ROUNDS];
#pragma unroll
  for (int r = 0; r < C::ROUNDS; r++) {
    const bool ok = base + r * 64 < n;
    const int d = (int)((k[r] >> shift) & (C::BINS - 1));
    unsigned long long peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < RB; b++) {
      const unsigned long long m = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? m : ~m;
    }
    // all lanes read the digit's count before its last lane advances it; LDS
    // executes a wavefront's operations in order
    const int prev = ok ? s_cnt[w][d] : 0;
    pos[r] = prev + __popcll(peers & below);
    if (ok && (peers & above) == 0) s_cnt[w][d] = prev + __popcll(peers);
  }
  __syncthreads();
  {
    // digits t * PER .. t * PER + PER - 1: their starts in the tile (digit
    // order), each wave's start, and where their runs go
    const bool holds = t * C::PER < C::BINS;
    int tot[C::PER], sum = 0;
#pragma unroll
    for (int q = 0; q < C::PER; q++) {
      tot[q] = 0;
#pragma unroll
      for (int u = 0; u < C::WAVES; u++) tot[q] += holds ? s_cnt[u][t * C::PER + q] : 0;
      sum += tot[q];
    }
    int acc = rs_block_excl<C::WAVES>(sum, s_w);
#pragma unroll
    for (int q = 0; q < C::PER; q++) {
      const int d = t * C::PER + q;
      if (!holds) break;
      s_delta[d] = off[(int64_t)d * ntiles + blockIdx.x] - acc;
#pragma unroll
      for (int u = 0; u < C::WAVES; u++) {
        const int c = s_cnt[u][d];
        s_cnt[u][d] = acc;
        acc += c;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < C::ROUNDS; r++) {
    if (base + r * 64 < n) {
      const int p = s_cnt[w][(k[r] >> shift) & (C::BINS - 1)] + pos[r];
      s_k[p] = k[r];
      s_v[p] = v[r];
    }
  }
  __syncthreads();
  // the tile in digit order: position j of digit d goes to that digit's run
  const int tn = (int)(n - tile0 < C::TILE ? n - tile0 : C::TILE);
  for (int j = t; j < tn; j += TH) {
    const uint32_t key = s_k[j];
    const int64_t p = (int64_t)s_delta[(key >> shift) & (C::BINS - 1)] + j;
    kout[p] = key;
    vout[p] = s_v[j];
  }
}

namespace {
size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int RS_RB = 8;  // digit bits per pass

void rs_plan(int bits, int& passes, int& rb) {
  rb = RS_RB;
  passes = (bits + RS_RB - 1) / RS_RB;
}

using RsNarrow = RsCfg<RS_RB, 256>;
using RsWide = RsCfg<RS_RB, 512>;
constexpr int64_t RS_WIDE_MIN_TILES = 1536;

// the tile length used for n pairs
int64_t rs_tile(int64_t n) {
  return n >= RS_WIDE_MIN_TILES * RsWide::TILE ? RsWide::TILE : RsNarrow::TILE;
}
}  // namespace

// temporary storage: the other key and value buffers, the digit-major tile
// histogram and its scan's temporaries
size_t sort_pairs_tmp_bytes(int64_t n, int bits) {
  if (n < 0 || bits <= 0 || bits > 32) return 0;
  int passes, rb;
  rs_plan(bits, passes, rb);
  const int64_t h = ((int64_t)1 << rb) * ((n + rs_tile(n) - 1) / rs_tile(n));
  return al(sizeof(uint32_t) * (size_t)n) + al(sizeof(int32_t) * (size_t)n) + al(sizeof(int32_t) * (size_t)h) +
         al(sizeof(int32_t) * (size_t)scan_tmp_ints(h)) + 256;
}

// keys_in/vals_in are read only (vals_in null: the values are 0, 1, ..., n-1);
// the result lands in keys_out/vals_out, which must not overlap the inputs.
// Offsets are int32: n < 2^31.
hipError_t sort_pairs(void* tmp, size_t tmp_bytes, const uint32_t* keys_in, uint32_t* keys_out,
                      const int32_t* vals_in, int32_t* vals_out, int64_t n, int bits, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (n < 0 || n >= INT32_MAX || bits <= 0 || bits > 32 || !tmp || tmp_bytes < sort_pairs_tmp_bytes(n, bits))
    return hipErrorInvalidValue;
  int passes, rb;
  rs_plan(bits, passes, rb);
  const bool wide = rs_tile(n) == RsWide::TILE;
  const int64_t ntiles = (n + rs_tile(n) - 1) / rs_tile(n), h = ((int64_t)1 << rb) * ntiles;
  char* p = (char*)tmp;
  uint32_t* kalt = (uint32_t*)p;
  p += al(sizeof(uint32_t) * (size_t)n);
  int32_t* valt = (int32_t*)p;
  p += al(sizeof(int32_t) * (size_t)n);
  int32_t* hist = (int32_t*)p;
  p += al(sizeof(int32_t) * (size_t)h);
  int32_t* scan_tmp = (int32_t*)p;
  const uint32_t* ks = keys_in;
  const int32_t* vs = vals_in;
  for (int q = 0; q < passes; q++) {
    // the last pass writes the output; before it, passes alternate so that
    // they do too: ... -> alt -> out -> alt -> out
    const bool to_out = ((passes - 1 - q) & 1) == 0;
    uint32_t* kd = to_out ? keys_out : kalt;
    int32_t* vd = to_out ? vals_out : valt;
    const int shift = rb * q;
    const unsigned g = (unsigned)ntiles;
    if (wide) k_rs_hist<RS_RB, RsWide::THREADS><<<g, RsWide::THREADS, 0, s>>>(ks, n, shift, ntiles, hist);
    else k_rs_hist<RS_RB, RsNarrow::THREADS><<<g, RsNarrow::THREADS, 0, s>>>(ks, n, shift, ntiles, hist);
    hipError_t e = exclusive_scan(hist, hist, h, scan_tmp, nullptr, nullptr, s);
    if (e != hipSuccess) return e;
    if (wide)
      k_rs_scatter<RS_RB, RsWide::THREADS><<<g, RsWide::THREADS, 0, s>>>(ks, vs, kd, vd, n, shift, ntiles, hist);
    else
      k_rs_scatter<RS_RB, RsNarrow::THREADS><<<g, RsNarrow::THREADS, 0, s>>>(ks, vs, kd, vd, n, shift, ntiles,
                                                                             hist);
    ks = kd;
    vs = vd;
  }
  return hipGetLastError();
}

}  // namespace csc
