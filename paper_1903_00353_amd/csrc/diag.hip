// Diagnostics: replay of a logged stream of packed 64-bit atomicMin
// instructions (csc_scan_record_atomics), with nothing else in the kernel, to
// measure the atomic rate at exactly the scan's own locality; and a scattered
// float atomicAdd rate on a vertex-gradient-shaped target.
#include "internal.h"

namespace csc {

// one wavefront per logged round: lane l issues the round's atomicMin on key
// log[64 r + l] if bit l of the round's mask is set (mode 0, device scope, as
// the scan issues it), or only reads the log (mode 1, the cost of the replay's
// own reads), or issues the atomicMin at workgroup scope (mode 2: performed in
// the issuing XCD's L2, without cross-XCD coherence; a rate measurement only),
// or a plain store instead (mode 3), or (mode 4) the rounds in blocks of
// REPLAY_BATCH per wavefront: every address of the block loaded first, then the
// block's atomics issued back to back. Vector memory operations complete in
// order on this ISA (stores and atomics without return count in the same
// counter as loads), so in modes 0-3 each round's load also waits for the
// previous round's atomics; mode 4 waits once per block.
constexpr int REPLAY_BATCH = 8;
__global__ __launch_bounds__(256) void k_atomic_replay(const uint32_t* __restrict__ log,
                                                       const unsigned long long* __restrict__ mask, int64_t rounds,
                                                       unsigned long long* keys, int64_t n_keys, int mode,
                                                       unsigned* sink) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  unsigned acc = 0;
  if (mode == 4) {
    for (int64_t r0 = (blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6)) * REPLAY_BATCH; r0 < rounds;
         r0 += nw * REPLAY_BATCH) {
      uint32_t a[REPLAY_BATCH];
      bool on[REPLAY_BATCH];
#pragma unroll
      for (int b = 0; b < REPLAY_BATCH; b++) {
        const int64_t r = r0 + b;
        on[b] = r < rounds && ((mask[r < rounds ? r : 0] >> lane) & 1ull);
        a[b] = on[b] ? log[r * 64 + lane] : 0u;
      }
#pragma unroll
      for (int b = 0; b < REPLAY_BATCH; b++)
        if (on[b] && (int64_t)a[b] < n_keys) atomicMin(&keys[a[b]], (unsigned long long)((r0 + b) * 64 + lane));
    }
    return;
  }
  for (int64_t r = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); r < rounds; r += nw) {
    const unsigned long long m = mask[r];
    if ((m >> lane) & 1ull) {
      const uint32_t a = log[r * 64 + lane];
      const unsigned long long v = (unsigned long long)(r * 64 + lane);
      if (mode == 1) {
        acc += a;
      } else if ((int64_t)a < n_keys) {
        if (mode == 0) atomicMin(&keys[a], v);
        else if (mode == 2) __hip_atomic_fetch_min(&keys[a], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else keys[a] = v;
      }
    }
  }
  if (mode == 1 && acc == 0xffffffffu) sink[0] = acc;  // keeps the reads
}

// n float atomicAdds of three consecutive floats each (a vertex's x, y, z) at
// pseudo-random vertices among nv: the adjoint's flush pattern with no reuse
__global__ __launch_bounds__(256) void k_fadd_rate(float* g, int64_t nv, int64_t n, unsigned seed) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    uint64_t x = (uint64_t)i * 0x9E3779B97F4A7C15ull + seed;  // splitmix64 finaliser
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    const int64_t v = (int64_t)(x % (uint64_t)nv);
    atomicAdd(&g[3 * v], 1.f);
    atomicAdd(&g[3 * v + 1], 1.f);
    atomicAdd(&g[3 * v + 2], 1.f);
  }
}

}  // namespace csc

using namespace csc;

extern "C" int csc_atomic_replay(const uint32_t* log_d, const unsigned long long* mask_d, int64_t rounds,
                                 unsigned long long* keys_d, int64_t n_keys, int32_t mode, void* stream) {
  if (!log_d || !mask_d || !keys_d || rounds < 0 || n_keys <= 0 || mode < 0 || mode > 4)
    return CSC_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  k_atomic_replay<<<2048, 256, 0, s>>>(log_d, mask_d, rounds, keys_d, n_keys, mode, (unsigned*)keys_d);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CSC_OK : fail_hip(e);
}

extern "C" int csc_fadd_rate(float* grad_d, int64_t nv, int64_t n, void* stream) {
  if (!grad_d || nv <= 0 || n < 0) return CSC_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  k_fadd_rate<<<2048, 256, 0, s>>>(grad_d, nv, n, 12345u);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CSC_OK : fail_hip(e);
}
