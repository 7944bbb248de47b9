// Triangle-soup ingestion (Section 7, Section 7.1-7.2): an STL file lists every
// triangle with its own three corner positions, so a vertex shared by k
// triangles appears k times. Welding gives every distinct position one vertex
// index, turning the soup into the indexed mesh the feature build reads; the
// edge pairs then follow from the indexed mesh (twins around each vertex).
//
// The paper orders corners by 30-bit Morton codes, which can map different
// positions to the same code and leave a per-group sequential pass to separate
// them. Here the corners are ordered by their exact coordinates instead (three
// stable 32-bit radix sorts: z, then y, then x), so equal positions are adjacent
// and nothing is left to sort out per group. -0 is taken as +0 first (equal as
// positions). Vertices are numbered in order of first appearance in the soup:
// the sorts are stable, so the first corner of every group of equal positions
// is the earliest one in the soup.
#include <cmath>

#include "internal.h"

namespace csc {

// corner keys: the coordinate bits with -0 mapped to +0; non-finite input flagged
__global__ void k_soup_keys(const float* __restrict__ soup, int64_t n, uint32_t* kx, uint32_t* ky, uint32_t* kz,
                            int32_t* idx, int32_t* bad) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= n) return;
  float x = soup[3 * c], y = soup[3 * c + 1], z = soup[3 * c + 2];
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) *bad = 1;
  x = x == 0.f ? 0.f : x;
  y = y == 0.f ? 0.f : y;
  z = z == 0.f ? 0.f : z;
  kx[c] = __float_as_uint(x);
  ky[c] = __float_as_uint(y);
  kz[c] = __float_as_uint(z);
  idx[c] = (int32_t)c;
}

// next sort key in the current order: out[p] = key[order[p]]
__global__ void k_gather_u32(const uint32_t* __restrict__ key, const int32_t* __restrict__ order, int64_t n,
                             uint32_t* out) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < n) out[p] = key[order[p]];
}

// group heads in sorted order: a corner whose position differs from the previous one
__global__ void k_soup_heads(const uint32_t* __restrict__ kx, const uint32_t* __restrict__ ky,
                             const uint32_t* __restrict__ kz, const int32_t* __restrict__ order, int64_t n,
                             int32_t* head_sorted, int32_t* head_corner) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t c = order[p];
  bool h = p == 0;
  if (!h) {
    const int32_t b = order[p - 1];
    h = kx[c] != kx[b] || ky[c] != ky[b] || kz[c] != kz[b];
  }
  head_sorted[p] = h ? 1 : 0;
  head_corner[c] = h ? 1 : 0;
}

// at every head: its group's first corner, and that vertex's position
__global__ void k_soup_vertices(const float* __restrict__ soup, const int32_t* __restrict__ order,
                                const int32_t* __restrict__ head_sorted, const int32_t* __restrict__ group,
                                const int32_t* __restrict__ vid, int64_t n, int32_t* group_corner, float* verts) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n || !head_sorted[p]) return;
  const int32_t c = order[p];
  group_corner[group[p]] = c;
  const int64_t v = vid[c];
  verts[3 * v] = soup[3 * (int64_t)c];
  verts[3 * v + 1] = soup[3 * (int64_t)c + 1];
  verts[3 * v + 2] = soup[3 * (int64_t)c + 2];
}

// every corner gets the vertex of its group; group[p] is the exclusive count of
// heads before p, so the group of p is group[p] + head[p] - 1
__global__ void k_soup_tris(const int32_t* __restrict__ order, const int32_t* __restrict__ head_sorted,
                            const int32_t* __restrict__ group, const int32_t* __restrict__ group_corner,
                            const int32_t* __restrict__ vid, int64_t n, int32_t* tris) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t g = group[p] + head_sorted[p] - 1;
  tris[order[p]] = vid[group_corner[g]];
}

}  // namespace csc

using namespace csc;

extern "C" int csc_weld_soup(const float* soup_d, int64_t nf, float* verts_d, int32_t* tris_d, int64_t* nv,
                             void* stream) {
  if (!soup_d || !verts_d || !tris_d || !nv || nf <= 0 || 3 * nf >= INT32_MAX) return CSC_INVALID_ARG;
  int rc = check_device();
  if (rc != CSC_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = 3 * nf;
  const size_t sort_bytes = sort_pairs_tmp_bytes(n, 32);
  if (sort_bytes == 0) return fail_hip(hipErrorInvalidValue);
  // one scratch allocation: 4 key arrays, 2 orders, 5 int arrays, scan and sort temporaries
  const size_t a = (sizeof(int32_t) * (size_t)n + 255) & ~(size_t)255;
  const size_t scan_b = (sizeof(int32_t) * (size_t)scan_tmp_ints(n) + 255) & ~(size_t)255;
  const size_t total = 11 * a + scan_b + 256 + sort_bytes;
  char* W = nullptr;
  hipError_t e = hipMallocAsync((void**)&W, total, s);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? CSC_OUT_OF_MEMORY : fail_hip(e);
  uint32_t *kx = (uint32_t*)W, *ky = (uint32_t*)(W + a), *kz = (uint32_t*)(W + 2 * a), *kt = (uint32_t*)(W + 3 * a),
           *ko = (uint32_t*)(W + 4 * a);
  int32_t *oa = (int32_t*)(W + 5 * a), *ob = (int32_t*)(W + 6 * a), *hs = (int32_t*)(W + 7 * a),
          *hc = (int32_t*)(W + 8 * a), *vid = (int32_t*)(W + 9 * a), *grp = (int32_t*)(W + 10 * a);
  int32_t* scan_tmp = (int32_t*)(W + 11 * a);
  int32_t* bad = (int32_t*)(W + 11 * a + scan_b);
  void* sort_tmp = W + 11 * a + scan_b + 256;
  int64_t* nv_d = (int64_t*)(W + 11 * a + scan_b + 8);
  const unsigned B = 256, G = grid_1d(n, B);
#define CK(x)                            \
  do {                                   \
    hipError_t ee = (x);                 \
    if (ee != hipSuccess) {              \
      (void)hipFreeAsync(W, s);          \
      return fail_hip(ee);               \
    }                                    \
  } while (0)
  CK(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
  k_soup_keys<<<G, B, 0, s>>>(soup_d, n, kx, ky, kz, oa, bad);
  // z, then y, then x: stable, so the result is lexicographic in (x, y, z)
  CK(sort_pairs(sort_tmp, sort_bytes, kz, ko, oa, ob, n, 32, s));
  k_gather_u32<<<G, B, 0, s>>>(ky, ob, n, kt);
  CK(sort_pairs(sort_tmp, sort_bytes, kt, ko, ob, oa, n, 32, s));
  k_gather_u32<<<G, B, 0, s>>>(kx, oa, n, kt);
  CK(sort_pairs(sort_tmp, sort_bytes, kt, ko, oa, ob, n, 32, s));
  k_soup_heads<<<G, B, 0, s>>>(kx, ky, kz, ob, n, hs, hc);
  CK(exclusive_scan(hc, vid, n, scan_tmp, nv_d, nullptr, s));
  CK(exclusive_scan(hs, grp, n, scan_tmp, nullptr, nullptr, s));
  k_soup_vertices<<<G, B, 0, s>>>(soup_d, ob, hs, grp, vid, n, hc, verts_d);  // hc reused: group -> first corner
  k_soup_tris<<<G, B, 0, s>>>(ob, hs, grp, hc, vid, n, tris_d);
  CK(hipGetLastError());
  int64_t h_nv = 0;
  int32_t h_bad = 0;
  CK(hipMemcpyAsync(&h_nv, nv_d, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  CK(hipMemcpyAsync(&h_bad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  CK(hipFreeAsync(W, s));
  CK(hipStreamSynchronize(s));
#undef CK
  if (h_bad) return CSC_INVALID_ARG;
  *nv = h_nv;
  return CSC_OK;
}
