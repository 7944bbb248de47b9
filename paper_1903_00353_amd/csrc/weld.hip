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
#include <mutex>

#include "internal.h"

namespace csc {

__global__ void k_clear_flag(int32_t* p) { *p = 0; }

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

namespace {

// scratch bytes of a weld of n corners: 4 key arrays, 2 orders, 5 int arrays,
// scan temporaries, the flag and count words, the radix sort's temporaries
struct WeldLayout {
  size_t a, scan_b, sort_bytes, total;
};

WeldLayout weld_layout(int64_t n) {
  WeldLayout L;
  L.sort_bytes = sort_pairs_tmp_bytes(n, 32);
  L.a = (sizeof(int32_t) * (size_t)n + 255) & ~(size_t)255;
  L.scan_b = (sizeof(int32_t) * (size_t)scan_tmp_ints(n) + 255) & ~(size_t)255;
  L.total = 11 * L.a + L.scan_b + 256 + L.sort_bytes;
  return L;
}

// the weld on scratch memory W (weld_layout(3 nf).total bytes); queues the
// kernels and the two count copies on s, without synchronising
hipError_t weld_queue(const float* soup_d, int64_t nf, float* verts_d, int32_t* tris_d, char* W, const WeldLayout& L,
                      int64_t* h_nv, int32_t* h_bad, hipStream_t s) {
  const int64_t n = 3 * nf;
  const size_t a = L.a;
  uint32_t *kx = (uint32_t*)W, *ky = (uint32_t*)(W + a), *kz = (uint32_t*)(W + 2 * a), *kt = (uint32_t*)(W + 3 * a),
           *ko = (uint32_t*)(W + 4 * a);
  int32_t *oa = (int32_t*)(W + 5 * a), *ob = (int32_t*)(W + 6 * a), *hs = (int32_t*)(W + 7 * a),
          *hc = (int32_t*)(W + 8 * a), *vid = (int32_t*)(W + 9 * a), *grp = (int32_t*)(W + 10 * a);
  int32_t* scan_tmp = (int32_t*)(W + 11 * a);
  int32_t* bad = (int32_t*)(W + 11 * a + L.scan_b);
  void* sort_tmp = W + 11 * a + L.scan_b + 256;
  int64_t* nv_d = (int64_t*)(W + 11 * a + L.scan_b + 8);
  const unsigned B = 256, G = grid_1d(n, B);
  hipError_t e;
  k_clear_flag<<<1, 1, 0, s>>>(bad);
  k_soup_keys<<<G, B, 0, s>>>(soup_d, n, kx, ky, kz, oa, bad);
  // z, then y, then x: stable, so the result is lexicographic in (x, y, z)
  if ((e = sort_pairs(sort_tmp, L.sort_bytes, kz, ko, oa, ob, n, 32, s)) != hipSuccess) return e;
  k_gather_u32<<<G, B, 0, s>>>(ky, ob, n, kt);
  if ((e = sort_pairs(sort_tmp, L.sort_bytes, kt, ko, ob, oa, n, 32, s)) != hipSuccess) return e;
  k_gather_u32<<<G, B, 0, s>>>(kx, oa, n, kt);
  if ((e = sort_pairs(sort_tmp, L.sort_bytes, kt, ko, oa, ob, n, 32, s)) != hipSuccess) return e;
  k_soup_heads<<<G, B, 0, s>>>(kx, ky, kz, ob, n, hs, hc);
  if ((e = exclusive_scan(hc, vid, n, scan_tmp, nv_d, nullptr, s)) != hipSuccess) return e;
  if ((e = exclusive_scan(hs, grp, n, scan_tmp, nullptr, nullptr, s)) != hipSuccess) return e;
  k_soup_vertices<<<G, B, 0, s>>>(soup_d, ob, hs, grp, vid, n, hc, verts_d);  // hc reused: group -> first corner
  k_soup_tris<<<G, B, 0, s>>>(ob, hs, grp, hc, vid, n, tris_d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(h_nv, nv_d, sizeof(int64_t), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  return hipMemcpyAsync(h_bad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
}

bool weld_args_ok(const float* soup_d, int64_t nf, const float* verts_d, const int32_t* tris_d, const int64_t* nv) {
  return soup_d && verts_d && tris_d && nv && nf > 0 && 3 * nf < INT32_MAX;
}

}  // namespace

extern "C" int csc_weld_soup(const float* soup_d, int64_t nf, float* verts_d, int32_t* tris_d, int64_t* nv,
                             void* stream) {
  if (!weld_args_ok(soup_d, nf, verts_d, tris_d, nv)) return CSC_INVALID_ARG;
  int rc = check_device();
  if (rc != CSC_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  const WeldLayout L = weld_layout(3 * nf);
  if (L.sort_bytes == 0) return fail_hip(hipErrorInvalidValue);
  char* W = nullptr;
  hipError_t e = hipMallocAsync((void**)&W, L.total, s);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? CSC_OUT_OF_MEMORY : fail_hip(e);
  int64_t h_nv = 0;
  int32_t h_bad = 0;
  e = weld_queue(soup_d, nf, verts_d, tris_d, W, L, &h_nv, &h_bad, s);
  const hipError_t ef = hipFreeAsync(W, s);
  if (e == hipSuccess) e = ef;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e);
  if (h_bad) return CSC_INVALID_ARG;
  *nv = h_nv;
  return CSC_OK;
}

// ------------------------------------------------------------ allocation-free
// csc_weld_soup_noalloc keeps its scratch in this file-scope device array, one
// copy per GPU, held until the process ends. Host code never passes the array's
// name to a kernel (on the host it only names the symbol): each device's
// address comes from hipGetSymbolAddress on the first call with that device
// current, and is kept per device.
constexpr size_t WELD_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) char scratch[WELD_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[MAX_DEVICES] = {};

int scratch_for_current_device(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e);
  if (dev < 0 || dev >= MAX_DEVICES) return CSC_UNSUPPORTED_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail_hip(e != hipSuccess ? e : hipErrorInvalidSymbol);
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return CSC_OK;
}
}  // namespace

extern "C" int csc_weld_soup_noalloc(const float* soup_d, int64_t nf, float* verts_d, int32_t* tris_d, int64_t* nv,
                                     void* stream) {
  if (!weld_args_ok(soup_d, nf, verts_d, tris_d, nv)) return CSC_INVALID_ARG;
  const WeldLayout L = weld_layout(3 * nf);
  if (L.sort_bytes == 0) return CSC_INVALID_ARG;
  if (L.total > WELD_SCRATCH_BYTES) return CSC_WORKSPACE_TOO_SMALL;
  int rc = check_device();
  if (rc != CSC_OK) return rc;
  char* W = nullptr;
  rc = scratch_for_current_device(&W);
  if (rc != CSC_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  int64_t h_nv = 0;
  int32_t h_bad = 0;
  hipError_t e = weld_queue(soup_d, nf, verts_d, tris_d, W, L, &h_nv, &h_bad, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e);
  if (h_bad) return CSC_INVALID_ARG;
  *nv = h_nv;
  return CSC_OK;
}

extern "C" int64_t csc_weld_soup_noalloc_max_faces(void) {
  int64_t lo = 0, hi = (INT32_MAX - 1) / 3;
  while (lo < hi) {  // the largest nf whose scratch fits
    const int64_t mid = (lo + hi + 1) / 2;
    if (weld_layout(3 * mid).total <= WELD_SCRATCH_BYTES) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
