// Interior fill of the dense field (Section 11.3): the band leaves every cell
// farther than band*h from the surface at +infinity, so the field jumps from its
// negative limit back to +infinity inside the solid (a second zero crossing).
// Sweeping along one grid axis and giving the unset cells inside the solid the
// value -infinity removes it.
//
// Where a step between two neighbouring cell centres of a column crosses the
// surface, both cells lie within one cell of the crossing, so both are band
// cells whenever band_cells > 1 (the band is strict: d < band_cells * h). Every
// run of unset cells therefore lies on the side of the band cells next to it:
// the one before it in the column, or, for the cells before the column's first
// band cell, the one after. A column without band cells does not meet the
// surface and is taken as outside. With band_cells <= 1 only the nearer cell of
// such a step is sure to be in the band, and the farther one, on the other
// side, would inherit the wrong side: the call rejects those bands.
#include "internal.h"

namespace csc {

// one thread per (x, y) column of the [n2][n1][n0] grid, walking z: consecutive
// threads read consecutive cells of each z-plane
__global__ __launch_bounds__(256) void k_interior_fill(float* dense, int n0, int n1, int n2) {
  const int64_t plane = (int64_t)n0 * n1;
  const int64_t col = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (col >= plane) return;
  float* p = dense + col;
  const float inf = __builtin_inff();
  int first = -1;       // first band cell of the column
  bool inside = false;  // side of the last band cell seen
  constexpr int U = 8;  // z steps loaded together
  for (int k0 = 0; k0 < n2; k0 += U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; u++) v[u] = k0 + u < n2 ? p[(k0 + u) * plane] : inf;
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (v[u] != inf) {
        inside = signbit(v[u]);
        if (first < 0) first = k0 + u;
      } else if (inside && k0 + u < n2) {
        p[(k0 + u) * plane] = -inf;
      }
    }
  }
  if (first > 0 && signbit(p[first * plane])) {  // the column starts inside the solid
    for (int k = 0; k < first; k++) p[k * plane] = -inf;
  }
}

}  // namespace csc

using namespace csc;

extern "C" int csc_interior_fill(const csc_features* f, float* dense_d, void* stream) {
  if (!f || !f->built || !dense_d || f->n_meshes != 1 || f->mesh.empty()) return CSC_INVALID_ARG;
  const MeshDesc& G = f->mesh[0];
  if (!(G.band > 1.f)) return CSC_INVALID_ARG;
  const int64_t cols = (int64_t)G.n[0] * G.n[1];
  hipStream_t s = (hipStream_t)stream;
  StageTimer t(TS_FILL, s);
  k_interior_fill<<<grid_1d(cols, 256), 256, 0, s>>>(dense_d, G.n[0], G.n[1], G.n[2]);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CSC_OK : fail_hip(e);
}
