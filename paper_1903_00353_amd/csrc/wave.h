// Cross-lane helpers for 64-lane wavefronts (gfx950), shared by the scan and
// adjoint kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>

namespace csc {

// DPP lane moves (gfx9 encodings): lane l reads lane l + 1 (wave_shl:1), l - 1
// (wave_shr:1), l - k within its row of 16 (row_shr:k), or lane 15 / 31 (the last
// of the row before, row_bcast). Lanes without a source keep `id`.
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118;
constexpr int DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138, DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143;

template <int CTRL, int ROWS = 0xf>
__device__ inline int dpp_i(int id, int x) {
  return __builtin_amdgcn_update_dpp(id, x, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS = 0xf>
__device__ inline float dpp_f(float id, float x) {
  return __int_as_float(dpp_i<CTRL, ROWS>(__float_as_int(id), __float_as_int(x)));
}

// inclusive prefix sum / maximum over the 64 lanes: shifts by 1, 2, 4, 8 inside
// each row of 16, then row 0's last lane into row 1 and row 2's into row 3, then
// lane 31 into rows 2-3 (every lane must be active)
__device__ inline int wave_prefix_sum(int x) {
  x += dpp_i<DPP_ROW_SHR1>(0, x);
  x += dpp_i<DPP_ROW_SHR2>(0, x);
  x += dpp_i<DPP_ROW_SHR4>(0, x);
  x += dpp_i<DPP_ROW_SHR8>(0, x);
  x += dpp_i<DPP_ROW_BCAST15, 0xa>(0, x);
  x += dpp_i<DPP_ROW_BCAST31, 0xc>(0, x);
  return x;
}
__device__ inline int wave_prefix_max(int x) {
  x = max(x, dpp_i<DPP_ROW_SHR1>(INT_MIN, x));
  x = max(x, dpp_i<DPP_ROW_SHR2>(INT_MIN, x));
  x = max(x, dpp_i<DPP_ROW_SHR4>(INT_MIN, x));
  x = max(x, dpp_i<DPP_ROW_SHR8>(INT_MIN, x));
  x = max(x, dpp_i<DPP_ROW_BCAST15, 0xa>(INT_MIN, x));
  x = max(x, dpp_i<DPP_ROW_BCAST31, 0xc>(INT_MIN, x));
  return x;
}

// memory ordering of a wavefront's own LDS writes before its reads of them
__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace csc
