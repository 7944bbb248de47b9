// Feature construction (Section 7, Section 8): adjacency, normals, edge and
// vertex classes, polyhedron lists and the band bricks.
//
// Unlike the paper's Morton-code sort of a triangle soup (Section 7.1, 7.2) the
// input here is already indexed, so twins are found through a vertex -> face
// table and edges are numbered by a prefix sum over the half-edges that own
// them (start index < end index), which makes every id deterministic.
#include <string.h>

#include "geometry.h"
#include "internal.h"

namespace csc {

__device__ inline d3 vload_d(const float* V, int64_t i) {
  return mkd((double)V[3 * i], (double)V[3 * i + 1], (double)V[3 * i + 2]);
}
__device__ inline f3 vload_f(const float* V, int64_t i) { return mk(V[3 * i], V[3 * i + 1], V[3 * i + 2]); }

// corner c = 3f + j (32-bit: 3F < 2^31): vertex after / before it in its face, and
// the half-edge entering it (prev -> corner)
__device__ inline int32_t next_corner(int32_t c) { int32_t j = c % 3; return c - j + (j == 2 ? 0 : j + 1); }
__device__ inline int32_t prev_corner(int32_t c) { int32_t j = c % 3; return c - j + (j == 0 ? 2 : j - 1); }

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_check_verts(const float* __restrict__ V, int64_t nv, uint32_t* err) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= 3 * nv) return;
  if (!isfinite(V[i])) atomicOr(err, ERR_NONFINITE);
}

// index range and repeated-corner checks
__global__ void k_validate_faces(const int32_t* __restrict__ T, int64_t nf, int64_t nv, uint32_t* err) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int32_t a = T[3 * f], b = T[3 * f + 1], c = T[3 * f + 2];
  if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv) atomicOr(err, ERR_INDEX);
  else if (a == b || b == c || a == c) atomicOr(err, ERR_REPEAT);
}

__global__ void k_iota(int32_t* p, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

// Segment offsets of the corners sorted by vertex: off[v] = first position whose
// vertex is >= v (vertices without corners get empty segments), off[nv] = nh.
__global__ void k_offsets(const uint32_t* __restrict__ key, int64_t nh, int64_t nv, int32_t* off) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nh) return;
  const int64_t k = key[i], kp = i > 0 ? (int64_t)key[i - 1] : -1;
  for (int64_t v = kp + 1; v <= k; v++) off[v] = (int32_t)i;
  if (i == nh - 1)
    for (int64_t v = k + 1; v <= nv; v++) off[v] = (int32_t)nh;
}

constexpr int VK_THREADS = 128;
constexpr int VK_MAXD = 16;  // fans up to this degree are staged in LDS

// Per vertex u, over its fan of corners (staged in LDS):
//  * twins: the out-edge u -> w of corner c (half-edge c) pairs with the unique
//    in-edge w -> u of another corner around u; none or several: not a closed
//    2-manifold; two out-edges to the same w: inconsistent orientation;
//  * pseudonormal N = sum alpha_i n_i (Eq. 8), class from the side of each
//    neighbour against the plane through u with normal N (Section 3.1-3.2,
//    Section 8.3), cone aperture and ruff test from the normals (Section 3.3,
//    Section 4.2), all in double precision; number of vertex polyhedra.
__global__ __launch_bounds__(VK_THREADS) void k_vertex(const float* __restrict__ V, const int32_t* __restrict__ T,
                                                      int64_t nv, const int32_t* __restrict__ off,
                                                      const int32_t* __restrict__ vc, int ruff_mode, int saddle_mode,
                                                      int force_both, int32_t* twin, float4* vinfo, uint32_t* vbits,
                                                      int32_t* count, uint32_t* err) {
  __shared__ int32_t s_c[VK_MAXD][VK_THREADS], s_n[VK_MAXD][VK_THREADS], s_p[VK_MAXD][VK_THREADS];
  const int t = threadIdx.x;
  const int64_t v = blockIdx.x * (int64_t)VK_THREADS + t;
  if (v >= nv) return;
  const int32_t s0 = off[v], d = off[v + 1] - s0;
  const bool staged = d <= VK_MAXD;
  if (staged) {
    for (int k = 0; k < d; k++) {
      int32_t c = vc[s0 + k];
      s_c[k][t] = c;
      s_n[k][t] = T[next_corner(c)];
      s_p[k][t] = T[prev_corner(c)];
    }
  }
  auto C_ = [&](int k) { return staged ? s_c[k][t] : vc[s0 + k]; };
  auto N_ = [&](int k) { return staged ? s_n[k][t] : T[next_corner(vc[s0 + k])]; };
  auto P_ = [&](int k) { return staged ? s_p[k][t] : T[prev_corner(vc[s0 + k])]; };
  uint32_t e = 0;
  for (int i = 0; i < d; i++) {
    const int32_t w = N_(i);
    int32_t match = -1, nmatch = 0;
    for (int k = 0; k < d; k++) {
      if (k != i && N_(k) == w) e |= ERR_ORIENT;
      if (P_(k) == w) {
        nmatch++;
        match = prev_corner(C_(k));
      }
    }
    if (nmatch != 1) e |= ERR_NONMANIFOLD;
    twin[C_(i)] = nmatch == 1 ? match : -1;
  }
  if (e) atomicOr(err, e);
  const d3 pv = vload_d(V, v);
  VertexAccum acc;
  for (int k = 0; k < d; k++) acc.add_face(pv, vload_d(V, N_(k)), vload_d(V, P_(k)));
  VertexTest vt;
  vt.init(acc.n_alpha);
  for (int k = 0; k < d; k++) {
    const d3 p1 = vload_d(V, N_(k)), p2 = vload_d(V, P_(k));
    vt.neighbour(pv, p1);
    vt.normal(pv, p1, p2);
  }
  VertexClass cl = vt.finish(ruff_mode, saddle_mode, force_both);
  if (d == 0) cl.bits = 0;  // isolated vertex: no feature
  float cf = (float)cl.cos_t;
  if ((double)cf > cl.cos_t) cf = nextafterf(cf, -2.f);  // the stored cone contains the exact one
  vinfo[v] = make_float4((float)cl.axis.x, (float)cl.axis.y, (float)cl.axis.z, cf);
  vbits[v] = cl.bits;
  count[v] = ((cl.bits & V_POS) ? 1 : 0) + ((cl.bits & V_NEG) ? 1 : 0);
}

__global__ void k_owned(const int32_t* __restrict__ T, int64_t nh, int32_t* flag) {
  int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (h >= nh) return;
  flag[h] = T[h] < T[next_corner((int32_t)h)] ? 1 : 0;
}

// (an open or non-manifold surface can own more or fewer than 3F/2 half-edges: such
// a build is rejected after the final readback, and nothing is written past ne)
__global__ void k_edges(const int32_t* __restrict__ T, int64_t nh, int64_t ne, const int32_t* __restrict__ twin,
                        const int32_t* __restrict__ eid, int4* edges, int32_t* face_edges) {
  int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (h >= nh) return;
  int32_t u = T[h], w = T[next_corner((int32_t)h)];
  int32_t t = twin[h];
  if (u < w) {
    int32_t e = eid[h];
    if (e < ne) edges[e] = make_int4(u, w, (int)(h / 3), t >= 0 ? t / 3 : -1);
    face_edges[h] = e < ne ? e : -1;
  } else {
    int32_t e = t >= 0 ? eid[t] : -1;
    face_edges[h] = e < ne ? e : -1;
  }
}

// Unit face normal (double precision, stored in single) and the band bricks near
// the face: every brick within band*h (+ one cell) of its bounding box. A face
// whose dilated box stays within the 3x3x3 bricks around the brick of its
// centroid only seeds that brick (k_dilate_bricks covers the rest); larger ones
// mark every brick of their box directly.
__global__ void k_face_geom(const float* __restrict__ V, const int32_t* __restrict__ T, int64_t nf, float4* fn,
                            csc_grid g, int nbx, int nby, int nbz, uint8_t* seed, int32_t* flag, uint32_t* err) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const d3 a = vload_d(V, T[3 * f]), b = vload_d(V, T[3 * f + 1]), c = vload_d(V, T[3 * f + 2]);
  const d3 n = cross(b - a, c - a);
  const double l = len(n);
  if (!(l > 0)) {
    atomicOr(err, ERR_DEGENERATE);
    fn[f] = make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    fn[f] = make_float4((float)(n.x / l), (float)(n.y / l), (float)(n.z / l), 0.f);
  }
  const double r = (double)g.band_cells * g.h + g.h, ih = 1.0 / g.h;
  const double X[3][3] = {{a.x, b.x, c.x}, {a.y, b.y, c.y}, {a.z, b.z, c.z}};
  const int nbk[3] = {nbx, nby, nbz};
  int lo[3], hi[3], cb[3];
  bool small = true;
  for (int ax = 0; ax < 3; ax++) {
    const double x0 = X[ax][0], x1 = X[ax][1], x2 = X[ax][2];
    const double mn = fmin(x0, fmin(x1, x2)) - r, mx = fmax(x0, fmax(x1, x2)) + r;
    double lo_c = floor((mn - g.origin[ax]) * ih - 0.5), hi_c = ceil((mx - g.origin[ax]) * ih - 0.5);
    lo_c = fmax(lo_c, 0.0);
    hi_c = fmin(hi_c, (double)(g.n[ax] - 1));
    if (lo_c > hi_c) return;
    lo[ax] = (int)lo_c / BRICK;
    hi[ax] = (int)hi_c / BRICK;
    const double cc = floor(floor(((x0 + x1 + x2) / 3.0 - g.origin[ax]) * ih) / BRICK);  // centroid's brick
    cb[ax] = (int)fmax(-2.0, fmin(cc, (double)nbk[ax] + 1));
    small = small && cb[ax] >= 0 && cb[ax] < nbk[ax] && lo[ax] >= cb[ax] - 1 && hi[ax] <= cb[ax] + 1;
  }
  if (small) {
    uint8_t* p = &seed[cb[0] + (int64_t)nbx * (cb[1] + (int64_t)nby * cb[2])];
    if (*p == 0) *p = 1;
    return;
  }
  for (int z = lo[2]; z <= hi[2]; z++)
    for (int y = lo[1]; y <= hi[1]; y++)
      for (int x = lo[0]; x <= hi[0]; x++) {
        int32_t* p = &flag[x + (int64_t)nbx * (y + (int64_t)nby * z)];
        if (*p == 0) *p = 1;
      }
}

__device__ inline int32_t third_vertex(const int32_t* T, int64_t f, int32_t a, int32_t b) {
  int32_t x = T[3 * f], y = T[3 * f + 1], z = T[3 * f + 2];
  return (x != a && x != b) ? x : ((y != a && y != b) ? y : z);
}

// edge class (exact orientation of the four float corners) and the sides to extrude
__global__ void k_edge_class(const float* __restrict__ V, const int32_t* __restrict__ T, const int4* __restrict__ edges,
                             int64_t ne, int force_both, uint8_t* cls, int32_t* count) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int c = 0, sides = 0;
  int4 E = edges[e];
  if (E.x >= 0 && E.z >= 0 && E.w >= 0) {
    int32_t c1 = third_vertex(T, E.z, E.x, E.y), c2 = third_vertex(T, E.w, E.x, E.y);
    c = classify_edge(vload_f(V, E.x), vload_f(V, E.y), vload_f(V, c1), vload_f(V, c2));
    if (c == EDGE_CONVEX) sides = 1;
    else if (c == EDGE_CONCAVE) sides = 2;
    else if (c == EDGE_UNKNOWN) sides = 3;
    if (force_both) sides = 3;
  }
  cls[e] = (uint8_t)(c | (sides << 2));
  count[e] = __popc(sides);
}

// class statistics: one LDS histogram per block, one global add per bin and block
__global__ __launch_bounds__(256) void k_class_stats(const uint8_t* __restrict__ ecls, int64_t ne,
                                                     const uint32_t* __restrict__ vbits, int64_t nv, int64_t* stats) {
  __shared__ int h[16];
  if (threadIdx.x < 16) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int loc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ne; i += stride) {
    int c = ecls[i] & 3;
    loc[0] += c == EDGE_CONVEX;
    loc[1] += c == EDGE_CONCAVE;
    loc[2] += c == EDGE_FLAT;
    loc[3] += c == EDGE_UNKNOWN;
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv; i += stride) {
    uint32_t b = vbits[i];
    loc[4] += (b & V_CONVEX) != 0;
    loc[5] += (b & V_CONCAVE) != 0;
    loc[6] += (b & V_FLAT) != 0;
    loc[7] += (b & V_SADDLE) != 0;
    loc[8] += (b & V_RUFF) != 0;
  }
#pragma unroll
  for (int k = 0; k < 9; k++) {
    int x = loc[k];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd(&h[k], x);
  }
  __syncthreads();
  const int map[9] = {ST_E_CONVEX, ST_E_CONCAVE, ST_E_FLAT, ST_E_UNKNOWN, ST_V_CONVEX,
                      ST_V_CONCAVE, ST_V_FLAT,   ST_V_SADDLE, ST_V_RUFF};
  if (threadIdx.x < 9 && h[threadIdx.x])
    atomicAdd((unsigned long long*)&stats[map[threadIdx.x]], (unsigned long long)h[threadIdx.x]);
}

__global__ void k_edge_queue(const uint8_t* __restrict__ cls, int64_t ne, const int32_t* __restrict__ off, int32_t* q) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int sides = cls[e] >> 2;
  int32_t p = off[e];
  if (sides & 1) q[p++] = (int32_t)(e << 1);
  if (sides & 2) q[p++] = (int32_t)((e << 1) | 1);
}

__global__ void k_vertex_queue(const uint32_t* __restrict__ vbits, int64_t nv, const int32_t* __restrict__ off, int32_t* q) {
  int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= nv) return;
  uint32_t b = vbits[v];
  int32_t p = off[v];
  if (b & V_POS) q[p++] = (int32_t)(v << 1);
  if (b & V_NEG) q[p++] = (int32_t)((v << 1) | 1);
}

// flag every brick with a seed among its 27 neighbours
__global__ void k_dilate_bricks(const uint8_t* __restrict__ seed, int nbx, int nby, int nbz, int32_t* flag) {
  int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= (int64_t)nbx * nby * nbz) return;
  if (flag[b]) return;
  const int x = (int)(b % nbx), y = (int)((b / nbx) % nby), z = (int)(b / ((int64_t)nbx * nby));
  for (int dz = -1; dz <= 1; dz++) {
    int zz = z + dz;
    if (zz < 0 || zz >= nbz) continue;
    for (int dy = -1; dy <= 1; dy++) {
      int yy = y + dy;
      if (yy < 0 || yy >= nby) continue;
      for (int dx = -1; dx <= 1; dx++) {
        int xx = x + dx;
        if (xx < 0 || xx >= nbx) continue;
        if (seed[xx + (int64_t)nbx * (yy + (int64_t)nby * zz)]) {
          flag[b] = 1;
          return;
        }
      }
    }
  }
}

__global__ void k_brick_fix(const int32_t* __restrict__ flag, int32_t* index, int32_t* list, int64_t n) {
  int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= n) return;
  if (flag[b]) list[index[b]] = (int32_t)b;
  else index[b] = -1;
}

}  // namespace csc

using namespace csc;

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t off[20];
  size_t total;
};

// arena layout for nv vertices, nf faces, nbt bricks
Layout layout(int64_t nv, int64_t nf, int64_t nbt, size_t sort_bytes) {
  int64_t ne = 3 * nf / 2;
  int64_t big = 3 * nf > nbt ? 3 * nf : nbt;
  big = big > nv + 1 ? big : nv + 1;
  size_t sz[20] = {
      sizeof(int32_t) * (size_t)(nv + 1),   // 0 vtx_off
      sizeof(int32_t) * (size_t)(3 * nf),   // 1 vtx_faces
      sizeof(int32_t) * (size_t)(3 * nf),   // 2 face_edges
      sizeof(int4) * (size_t)(ne + 1),      // 3 edges
      sizeof(float4) * (size_t)nf,          // 4 face_n
      (size_t)(ne + 1),                     // 5 edge_cls
      sizeof(float4) * (size_t)nv,          // 6 vinfo
      sizeof(uint32_t) * (size_t)nv,        // 7 vbits
      sizeof(int32_t) * (size_t)(2 * ne + 1),  // 8 epoly
      sizeof(int32_t) * (size_t)(2 * nv + 1),  // 9 vpoly
      sizeof(int32_t) * (size_t)nbt,        // 10 brick_index
      sizeof(int32_t) * (size_t)nbt,        // 11 brick_list
      sizeof(int32_t) * (size_t)(big + 1),  // 12 t_a
      sizeof(int32_t) * (size_t)(big + 1),  // 13 t_b
      sizeof(int32_t) * (size_t)(big + 1),  // 14 t_c
      sizeof(int32_t) * (size_t)scan_tmp_ints(big + 1),  // 15 t_scan
      sizeof(int64_t) * ST_COUNT,           // 16 stats
      sizeof(uint32_t) * 4,                 // 17 err
      sort_bytes,                           // 18 radix sort scratch
      0};
  Layout L;
  size_t o = 0;
  for (int i = 0; i < 20; i++) {
    L.off[i] = o;
    o += align_up(sz[i]);
  }
  L.total = o;
  return L;
}

bool finite_pos(double x) { return x > 0 && x < 1e300; }

}  // namespace

extern "C" int csc_build_features(const float* verts_d, int64_t nv, const int32_t* tris_d, int64_t nf,
                                  const csc_grid* grid, const csc_options* opt, void* stream, csc_features** out) {
  if (!verts_d || !tris_d || !grid || !out || nv <= 0 || nf <= 0) return CSC_INVALID_ARG;
  if (nv > INT32_MAX / 2 || nf > INT32_MAX / 4) return CSC_INVALID_ARG;
  if (nf % 2 != 0) return CSC_NONMANIFOLD;  // a closed triangle surface has 3F/2 edges
  for (int a = 0; a < 3; a++) {
    if (grid->n[a] <= 0 || !isfinite(grid->origin[a])) return CSC_INVALID_ARG;
  }
  if (!finite_pos(grid->h) || !(grid->band_cells > 0) || !isfinite(grid->band_cells)) return CSC_INVALID_ARG;
  if ((int64_t)grid->n[0] * grid->n[1] * grid->n[2] > INT32_MAX) return CSC_GRID_TOO_LARGE;
  csc_options o = {1e-3f, 0, 0, 0};
  if (opt) o = *opt;
  if (!(o.eps_rel >= 0) || !(o.eps_rel < 0.5f) || o.ruff_mode < 0 || o.ruff_mode > 1 || o.saddle_mode < 0 ||
      o.saddle_mode > 2)
    return CSC_INVALID_ARG;
  int nb[3];
  for (int a = 0; a < 3; a++) nb[a] = (grid->n[a] + BRICK - 1) / BRICK;
  int64_t nbt = (int64_t)nb[0] * nb[1] * nb[2];
  if (nbt > (1 << 24)) return CSC_GRID_TOO_LARGE;
  int dc = check_device();
  if (dc != CSC_OK) return dc;

  hipStream_t s = (hipStream_t)stream;
  csc_features* F = *out;
  bool fresh = F == nullptr;
  if (fresh) {
    F = new (std::nothrow) csc_features();
    if (!F) return CSC_OUT_OF_MEMORY;
  }
  F->valid = false;
  int sort_bits = 1;
  while (sort_bits < 31 && ((int64_t)1 << sort_bits) < nv) sort_bits++;
  const size_t sort_bytes = sort_pairs_tmp_bytes(3 * nf, sort_bits);
  if (sort_bytes == 0) {
    if (fresh) delete F;
    return fail_hip(hipErrorInvalidValue);
  }
  Layout L = layout(nv, nf, nbt, sort_bytes);
  hipError_t he;
  if (F->arena_bytes < L.total) {
    if (F->arena) {
      he = hipStreamSynchronize(s);
      (void)hipFree(F->arena);
      F->arena = nullptr;
      F->arena_bytes = 0;
    }
    he = hipMalloc((void**)&F->arena, L.total);
    if (he != hipSuccess) {
      F->arena = nullptr;
      if (fresh) { if (F->h_stats) (void)hipHostFree(F->h_stats); delete F; }
      return he == hipErrorOutOfMemory ? CSC_OUT_OF_MEMORY : fail_hip(he);
    }
    F->arena_bytes = L.total;
  }
  if (!F->h_stats) {
    he = hipHostMalloc((void**)&F->h_stats, sizeof(int64_t) * (ST_COUNT + 2), hipHostMallocDefault);
    if (he != hipSuccess) {
      F->h_stats = nullptr;
      if (fresh) { (void)hipFree(F->arena); delete F; }
      return fail_hip(he);
    }
  }
  char* A = F->arena;
  F->verts = verts_d;
  F->tris = tris_d;
  F->nv = nv;
  F->nf = nf;
  F->ne = 3 * nf / 2;
  F->grid = *grid;
  F->opt = o;
  for (int a = 0; a < 3; a++) F->nb[a] = nb[a];
  F->nbricks_total = nbt;
  F->vtx_off = (int32_t*)(A + L.off[0]);
  F->vtx_faces = (int32_t*)(A + L.off[1]);
  F->face_edges = (int32_t*)(A + L.off[2]);
  F->edges = (int4*)(A + L.off[3]);
  F->face_n = (float4*)(A + L.off[4]);
  F->edge_cls = (uint8_t*)(A + L.off[5]);
  F->vinfo = (float4*)(A + L.off[6]);
  F->vbits = (uint32_t*)(A + L.off[7]);
  F->epoly = (int32_t*)(A + L.off[8]);
  F->vpoly = (int32_t*)(A + L.off[9]);
  F->brick_index = (int32_t*)(A + L.off[10]);
  F->brick_list = (int32_t*)(A + L.off[11]);
  F->t_a = (int32_t*)(A + L.off[12]);
  F->t_b = (int32_t*)(A + L.off[13]);
  F->t_c = (int32_t*)(A + L.off[14]);
  F->t_scan = (int32_t*)(A + L.off[15]);
  F->d_stats = (int64_t*)(A + L.off[16]);
  F->d_err = (uint32_t*)(A + L.off[17]);
  F->t_sort = (void*)(A + L.off[18]);
  F->t_sort_bytes = sort_bytes;

  const int B = 256;
  const int64_t nh = 3 * nf, ne = F->ne;
  auto fail = [&](int code) {
    if (fresh) csc_features_free(F);
    return code;
  };
#define CK(x)                                   \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return fail(fail_hip(e_)); \
  } while (0)

  StageTimer timer(TS_BUILD, s);
  // 1. validation; the first readback guards every indexed access below
  CK(hipMemsetAsync(F->d_stats, 0, sizeof(int64_t) * ST_COUNT, s));
  CK(hipMemsetAsync(F->d_err, 0, sizeof(uint32_t), s));
  k_check_verts<<<grid_1d(3 * nv, B), B, 0, s>>>(verts_d, nv, F->d_err);
  k_validate_faces<<<grid_1d(nf, B), B, 0, s>>>(tris_d, nf, nv, F->d_err);
  CK(hipGetLastError());
  CK(hipMemcpyAsync(F->h_stats + ST_COUNT, F->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  uint32_t err0 = *(uint32_t*)(F->h_stats + ST_COUNT);
  if (err0 & (ERR_INDEX | ERR_REPEAT | ERR_NONFINITE)) return fail(CSC_INVALID_ARG);

  // 2. vertex -> corner table: corners 3f+j stably sorted by their vertex T[3f+j]
  k_iota<<<grid_1d(nh, B), B, 0, s>>>(F->t_a, nh);
  CK(sort_pairs(F->t_sort, F->t_sort_bytes, (const uint32_t*)tris_d, (uint32_t*)F->t_b, F->t_a, F->vtx_faces, nh,
                sort_bits, s));
  k_offsets<<<grid_1d(nh, B), B, 0, s>>>((const uint32_t*)F->t_b, nh, nv, F->vtx_off);
  // 3. per vertex: twins, pseudonormal, class, cone; then edge numbering
  k_vertex<<<grid_1d(nv, VK_THREADS), VK_THREADS, 0, s>>>(verts_d, tris_d, nv, F->vtx_off, F->vtx_faces, o.ruff_mode,
                                                        o.saddle_mode, o.force_both_sides, F->t_a, F->vinfo,
                                                        F->vbits, F->t_c, F->d_err);
  CK(exclusive_scan(F->t_c, F->t_c, nv, F->t_scan, &F->d_stats[ST_NVPOLY], nullptr, s));
  k_vertex_queue<<<grid_1d(nv, B), B, 0, s>>>(F->vbits, nv, F->t_c, F->vpoly);
  k_owned<<<grid_1d(nh, B), B, 0, s>>>(tris_d, nh, F->t_b);
  k_fill_i32<<<grid_1d(4 * (ne + 1), B), B, 0, s>>>((int32_t*)F->edges, 4 * (ne + 1), -1);
  CK(exclusive_scan(F->t_b, F->t_b, nh, F->t_scan, &F->d_stats[ST_NE], nullptr, s));
  k_edges<<<grid_1d(nh, B), B, 0, s>>>(tris_d, nh, ne, F->t_a, F->t_b, F->edges, F->face_edges);
  // 4. face normals with the band bricks near each face, edge classes
  k_fill_i32<<<grid_1d(nbt, B), B, 0, s>>>(F->t_b, nbt, 0);
  k_fill_i32<<<grid_1d((nbt + 3) / 4, B), B, 0, s>>>(F->t_a, (nbt + 3) / 4, 0);
  k_face_geom<<<grid_1d(nf, B), B, 0, s>>>(verts_d, tris_d, nf, F->face_n, *grid, nb[0], nb[1], nb[2],
                                           (uint8_t*)F->t_a, F->t_b, F->d_err);
  k_edge_class<<<grid_1d(ne, B), B, 0, s>>>(verts_d, tris_d, F->edges, ne, o.force_both_sides, F->edge_cls, F->t_c);
  CK(exclusive_scan(F->t_c, F->t_c, ne, F->t_scan, &F->d_stats[ST_NEPOLY], nullptr, s));
  k_edge_queue<<<grid_1d(ne, B), B, 0, s>>>(F->edge_cls, ne, F->t_c, F->epoly);
  k_class_stats<<<256, 256, 0, s>>>(F->edge_cls, ne, F->vbits, nv, F->d_stats);
  // 5. band bricks
  k_dilate_bricks<<<grid_1d(nbt, B), B, 0, s>>>((const uint8_t*)F->t_a, nb[0], nb[1], nb[2], F->t_b);
  CK(exclusive_scan(F->t_b, F->brick_index, nbt, F->t_scan, &F->d_stats[ST_NBRICKS], nullptr, s));
  k_brick_fix<<<grid_1d(nbt, B), B, 0, s>>>(F->t_b, F->brick_index, F->brick_list, nbt);
  CK(hipGetLastError());
  CK(hipMemcpyAsync(F->h_stats, F->d_stats, sizeof(int64_t) * ST_COUNT, hipMemcpyDeviceToHost, s));
  CK(hipMemcpyAsync(F->h_stats + ST_COUNT, F->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
#undef CK
  uint32_t err = *(uint32_t*)(F->h_stats + ST_COUNT);
  const int64_t* st = F->h_stats;
  if (err & ERR_ORIENT) return fail(CSC_INCONSISTENT_ORIENTATION);
  if (err & ERR_NONMANIFOLD) return fail(CSC_NONMANIFOLD);
  if (st[ST_NE] != ne) return fail(CSC_NONMANIFOLD);
  if (err & ERR_DEGENERATE) return fail(CSC_DEGENERATE_FACE);
  F->n_epoly = st[ST_NEPOLY];
  F->n_vpoly = st[ST_NVPOLY];
  F->n_bricks = st[ST_NBRICKS];
  csc_feature_info& I = F->info;
  I.n_vertices = nv;
  I.n_faces = nf;
  I.n_edges = ne;
  I.n_edge_polyhedra = F->n_epoly;
  I.n_vertex_polyhedra = F->n_vpoly;
  I.edges_convex = st[ST_E_CONVEX];
  I.edges_concave = st[ST_E_CONCAVE];
  I.edges_flat = st[ST_E_FLAT];
  I.edges_unknown = st[ST_E_UNKNOWN];
  I.vertices_convex = st[ST_V_CONVEX];
  I.vertices_concave = st[ST_V_CONCAVE];
  I.vertices_flat = st[ST_V_FLAT];
  I.vertices_saddle = st[ST_V_SADDLE];
  I.vertices_ruff = st[ST_V_RUFF];
  I.n_bricks = F->n_bricks;
  I.max_band_cells = F->n_bricks * BRICK_CELLS;
  F->valid = true;
  *out = F;
  return CSC_OK;
}
