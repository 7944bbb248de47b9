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

// wave-aggregated counter increment (one atomic per wave)
__device__ inline void count_if(bool c, int64_t* ctr) {
  unsigned long long m = __ballot(c);
  if ((threadIdx.x & 63) == __ffsll((long long)__ballot(1)) - 1 && m)
    atomicAdd((unsigned long long*)ctr, (unsigned long long)__popcll(m));
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_check_verts(const float* __restrict__ V, int64_t nv, uint32_t* err) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= 3 * nv) return;
  if (!isfinite(V[i])) atomicOr(err, ERR_NONFINITE);
}

// index range / repeated-corner checks and per-vertex corner counts
__global__ void k_count_corners(const int32_t* __restrict__ T, int64_t nf, int64_t nv, int32_t* cnt, uint32_t* err) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int32_t a = T[3 * f], b = T[3 * f + 1], c = T[3 * f + 2];
  if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv) { atomicOr(err, ERR_INDEX); return; }
  if (a == b || b == c || a == c) { atomicOr(err, ERR_REPEAT); return; }
  atomicAdd(&cnt[a], 1);
  atomicAdd(&cnt[b], 1);
  atomicAdd(&cnt[c], 1);
}

__global__ void k_scatter_faces(const int32_t* __restrict__ T, int64_t nf, const int32_t* __restrict__ off,
                                int32_t* cursor, int32_t* vf) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  for (int j = 0; j < 3; j++) {
    int32_t v = T[3 * f + j];
    int32_t p = atomicAdd(&cursor[v], 1);
    vf[off[v] + p] = (int32_t)f;
  }
}

// deterministic order of each vertex's incident faces (ascending index)
__global__ void k_sort_segments(const int32_t* __restrict__ off, int32_t* vf, int64_t nv) {
  int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= nv) return;
  int32_t s = off[v], e = off[v + 1];
  for (int32_t i = s + 1; i < e; i++) {
    int32_t x = vf[i], j = i - 1;
    while (j >= s && vf[j] > x) { vf[j + 1] = vf[j]; j--; }
    vf[j + 1] = x;
  }
}

// twin of half-edge h = 3f+j (u -> w): the unique half-edge w -> u in another face around u
__global__ void k_twins(const int32_t* __restrict__ T, int64_t nf, const int32_t* __restrict__ off,
                        const int32_t* __restrict__ vf, int32_t* twin, uint32_t* err) {
  int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (h >= 3 * nf) return;
  int64_t f = h / 3;
  int j = (int)(h - 3 * f);
  int32_t u = T[3 * f + j], w = T[3 * f + (j + 1) % 3];
  int32_t match = -1, nmatch = 0, dup = 0;
  for (int32_t s = off[u]; s < off[u + 1]; s++) {
    int32_t g = vf[s];
    if (g == f) continue;
    for (int jj = 0; jj < 3; jj++) {
      int32_t x = T[3 * (int64_t)g + jj], y = T[3 * (int64_t)g + (jj + 1) % 3];
      if (x == w && y == u) { nmatch++; match = 3 * g + jj; }
      if (x == u && y == w) dup++;
    }
  }
  if (dup) atomicOr(err, ERR_ORIENT);
  if (nmatch != 1) atomicOr(err, ERR_NONMANIFOLD);
  twin[h] = nmatch == 1 ? match : -1;
}

__global__ void k_owned(const int32_t* __restrict__ T, int64_t nf, int32_t* flag) {
  int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (h >= 3 * nf) return;
  int64_t f = h / 3;
  int j = (int)(h - 3 * f);
  flag[h] = T[3 * f + j] < T[3 * f + (j + 1) % 3] ? 1 : 0;
}

// (an open or non-manifold surface can own more or fewer than 3F/2 half-edges: such
// a build is rejected after the final readback, and nothing is written past ne)
__global__ void k_edges(const int32_t* __restrict__ T, int64_t nf, int64_t ne, const int32_t* __restrict__ twin,
                        const int32_t* __restrict__ eid, int4* edges, int32_t* face_edges) {
  int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (h >= 3 * nf) return;
  int64_t f = h / 3;
  int j = (int)(h - 3 * f);
  int32_t u = T[3 * f + j], w = T[3 * f + (j + 1) % 3];
  int32_t t = twin[h];
  if (u < w) {
    int32_t e = eid[h];
    if (e < ne) edges[e] = make_int4(u, w, (int)f, t >= 0 ? t / 3 : -1);
    face_edges[h] = e < ne ? e : -1;
  } else {
    int32_t e = t >= 0 ? eid[t] : -1;
    face_edges[h] = e < ne ? e : -1;
  }
}

__global__ void k_face_geom(const float* __restrict__ V, const int32_t* __restrict__ T, int64_t nf, float4* fn,
                            uint32_t* err) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  d3 a = vload_d(V, T[3 * f]), b = vload_d(V, T[3 * f + 1]), c = vload_d(V, T[3 * f + 2]);
  d3 n = cross(b - a, c - a);
  double l = len(n);
  if (!(l > 0)) {
    atomicOr(err, ERR_DEGENERATE);
    fn[f] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  fn[f] = make_float4((float)(n.x / l), (float)(n.y / l), (float)(n.z / l), 0.f);
}

__device__ inline int32_t third_vertex(const int32_t* T, int64_t f, int32_t a, int32_t b) {
  int32_t x = T[3 * f], y = T[3 * f + 1], z = T[3 * f + 2];
  return (x != a && x != b) ? x : ((y != a && y != b) ? y : z);
}

// edge class (exact orientation of the four float corners) and the sides to extrude
__global__ void k_edge_class(const float* __restrict__ V, const int32_t* __restrict__ T, const int4* __restrict__ edges,
                             int64_t ne, int force_both, uint8_t* cls, int32_t* count, int64_t* stats) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int c = -1, sides = 0;
  if (e < ne) {
    int4 E = edges[e];
    if (E.x >= 0 && E.z >= 0 && E.w >= 0) {
      int32_t c1 = third_vertex(T, E.z, E.x, E.y), c2 = third_vertex(T, E.w, E.x, E.y);
      c = classify_edge(vload_f(V, E.x), vload_f(V, E.y), vload_f(V, c1), vload_f(V, c2));
      if (c == EDGE_CONVEX) sides = 1;
      else if (c == EDGE_CONCAVE) sides = 2;
      else if (c == EDGE_UNKNOWN) sides = 3;
      if (force_both) sides = 3;
    }
    cls[e] = (uint8_t)((c < 0 ? 0 : c) | (sides << 2));
    count[e] = __popc(sides);
  }
  count_if(c == EDGE_CONVEX, &stats[ST_E_CONVEX]);
  count_if(c == EDGE_CONCAVE, &stats[ST_E_CONCAVE]);
  count_if(c == EDGE_FLAT, &stats[ST_E_FLAT]);
  count_if(c == EDGE_UNKNOWN, &stats[ST_E_UNKNOWN]);
}

__global__ void k_edge_queue(const uint8_t* __restrict__ cls, int64_t ne, const int32_t* __restrict__ off, int32_t* q) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int sides = cls[e] >> 2;
  int32_t p = off[e];
  if (sides & 1) q[p++] = (int32_t)(e << 1);
  if (sides & 2) q[p++] = (int32_t)((e << 1) | 1);
}

// vertex pseudonormal (Eq. 8), class (Section 3.1-3.3, Section 8.3) and cone aperture (Section 4.2)
__global__ void k_vertex_class(const float* __restrict__ V, const int32_t* __restrict__ T,
                               const int32_t* __restrict__ off, const int32_t* __restrict__ vf, int64_t nv,
                               int ruff_mode, int saddle_mode, int force_both, float4* vinfo, uint32_t* vbits,
                               int32_t* count, int64_t* stats) {
  int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  uint32_t bits = 0;
  if (v < nv) {
    d3 pv = vload_d(V, v);
    VertexAccum acc;
    int32_t s0 = off[v], s1 = off[v + 1];
    for (int32_t s = s0; s < s1; s++) {
      int64_t g = vf[s];
      int jj = T[3 * g] == v ? 0 : (T[3 * g + 1] == v ? 1 : 2);
      acc.add_face(pv, vload_d(V, T[3 * g + (jj + 1) % 3]), vload_d(V, T[3 * g + (jj + 2) % 3]));
    }
    VertexTest t;
    t.init(acc.n_alpha);
    for (int32_t s = s0; s < s1; s++) {
      int64_t g = vf[s];
      int jj = T[3 * g] == v ? 0 : (T[3 * g + 1] == v ? 1 : 2);
      d3 p1 = vload_d(V, T[3 * g + (jj + 1) % 3]), p2 = vload_d(V, T[3 * g + (jj + 2) % 3]);
      t.neighbour(pv, p1);
      t.normal(pv, p1, p2);
    }
    VertexClass vc = t.finish(ruff_mode, saddle_mode, force_both);
    if (s1 == s0) vc.bits = 0;  // isolated vertex: no feature
    float cf = (float)vc.cos_t;
    if ((double)cf > vc.cos_t) cf = nextafterf(cf, -2.f);  // the stored cone contains the exact one
    vinfo[v] = make_float4((float)vc.axis.x, (float)vc.axis.y, (float)vc.axis.z, cf);
    vbits[v] = vc.bits;
    bits = vc.bits;
    count[v] = ((bits & V_POS) ? 1 : 0) + ((bits & V_NEG) ? 1 : 0);
  }
  bool ok = v < nv;
  count_if(ok && (bits & V_CONVEX), &stats[ST_V_CONVEX]);
  count_if(ok && (bits & V_CONCAVE), &stats[ST_V_CONCAVE]);
  count_if(ok && (bits & V_FLAT), &stats[ST_V_FLAT]);
  count_if(ok && (bits & V_SADDLE), &stats[ST_V_SADDLE]);
  count_if(ok && (bits & V_RUFF), &stats[ST_V_RUFF]);
}

__global__ void k_vertex_queue(const uint32_t* __restrict__ vbits, int64_t nv, const int32_t* __restrict__ off, int32_t* q) {
  int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= nv) return;
  uint32_t b = vbits[v];
  int32_t p = off[v];
  if (b & V_POS) q[p++] = (int32_t)(v << 1);
  if (b & V_NEG) q[p++] = (int32_t)((v << 1) | 1);
}

// every brick within band*h (+ one cell of margin) of a triangle's bounding box
__global__ void k_mark_bricks(const float* __restrict__ V, const int32_t* __restrict__ T, int64_t nf, csc_grid g,
                              int nbx, int nby, int nbz, int32_t* flag) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double r = (double)g.band_cells * g.h + g.h;
  int lo[3], hi[3];
  const int nbk[3] = {nbx, nby, nbz};
  for (int ax = 0; ax < 3; ax++) {
    double x0 = V[3 * T[3 * f] + ax], x1 = V[3 * T[3 * f + 1] + ax], x2 = V[3 * T[3 * f + 2] + ax];
    double mn = fmin(x0, fmin(x1, x2)) - r, mx = fmax(x0, fmax(x1, x2)) + r;
    double a = floor((mn - g.origin[ax]) / g.h - 0.5), b = ceil((mx - g.origin[ax]) / g.h - 0.5);
    if (a < 0) a = 0;
    if (b > g.n[ax] - 1) b = g.n[ax] - 1;
    if (a > b) return;
    lo[ax] = (int)a / BRICK;
    hi[ax] = (int)b / BRICK;
    if (hi[ax] >= nbk[ax]) hi[ax] = nbk[ax] - 1;
  }
  for (int z = lo[2]; z <= hi[2]; z++)
    for (int y = lo[1]; y <= hi[1]; y++)
      for (int x = lo[0]; x <= hi[0]; x++) flag[x + (int64_t)nbx * (y + (int64_t)nby * z)] = 1;
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
Layout layout(int64_t nv, int64_t nf, int64_t nbt) {
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
      0, 0};
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
  Layout L = layout(nv, nf, nbt);
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

  // 1. validation and corner counts; the first readback guards every indexed access below
  CK(hipMemsetAsync(F->d_stats, 0, sizeof(int64_t) * ST_COUNT, s));
  CK(hipMemsetAsync(F->d_err, 0, sizeof(uint32_t), s));
  k_fill_i32<<<grid_1d(nv + 1, B), B, 0, s>>>(F->t_a, nv + 1, 0);
  k_check_verts<<<grid_1d(3 * nv, B), B, 0, s>>>(verts_d, nv, F->d_err);
  k_count_corners<<<grid_1d(nf, B), B, 0, s>>>(tris_d, nf, nv, F->t_a, F->d_err);
  CK(hipGetLastError());
  CK(hipMemcpyAsync(F->h_stats + ST_COUNT, F->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  uint32_t err0 = *(uint32_t*)(F->h_stats + ST_COUNT);
  if (err0 & (ERR_INDEX | ERR_REPEAT | ERR_NONFINITE)) return fail(CSC_INVALID_ARG);

  // 2. vertex -> face table (count, scan, scatter, sort)
  CK(exclusive_scan(F->t_a, F->vtx_off, nv + 1, F->t_scan, nullptr, nullptr, s));
  k_fill_i32<<<grid_1d(nv + 1, B), B, 0, s>>>(F->t_a, nv + 1, 0);
  k_scatter_faces<<<grid_1d(nf, B), B, 0, s>>>(tris_d, nf, F->vtx_off, F->t_a, F->vtx_faces);
  k_sort_segments<<<grid_1d(nv, B), B, 0, s>>>(F->vtx_off, F->vtx_faces, nv);
  // 3. twins and edge numbering
  k_twins<<<grid_1d(nh, B), B, 0, s>>>(tris_d, nf, F->vtx_off, F->vtx_faces, F->t_a, F->d_err);
  k_owned<<<grid_1d(nh, B), B, 0, s>>>(tris_d, nf, F->t_b);
  k_fill_i32<<<grid_1d(4 * (ne + 1), B), B, 0, s>>>((int32_t*)F->edges, 4 * (ne + 1), -1);
  CK(exclusive_scan(F->t_b, F->t_b, nh, F->t_scan, &F->d_stats[ST_NE], nullptr, s));
  k_edges<<<grid_1d(nh, B), B, 0, s>>>(tris_d, nf, ne, F->t_a, F->t_b, F->edges, F->face_edges);
  // 4. geometry and classes
  k_face_geom<<<grid_1d(nf, B), B, 0, s>>>(verts_d, tris_d, nf, F->face_n, F->d_err);
  k_edge_class<<<grid_1d(ne, B), B, 0, s>>>(verts_d, tris_d, F->edges, ne, o.force_both_sides, F->edge_cls, F->t_c,
                                             F->d_stats);
  CK(exclusive_scan(F->t_c, F->t_c, ne, F->t_scan, &F->d_stats[ST_NEPOLY], nullptr, s));
  k_edge_queue<<<grid_1d(ne, B), B, 0, s>>>(F->edge_cls, ne, F->t_c, F->epoly);
  k_vertex_class<<<grid_1d(nv, B), B, 0, s>>>(verts_d, tris_d, F->vtx_off, F->vtx_faces, nv, o.ruff_mode,
                                               o.saddle_mode, o.force_both_sides, F->vinfo, F->vbits, F->t_a,
                                               F->d_stats);
  CK(exclusive_scan(F->t_a, F->t_a, nv, F->t_scan, &F->d_stats[ST_NVPOLY], nullptr, s));
  k_vertex_queue<<<grid_1d(nv, B), B, 0, s>>>(F->vbits, nv, F->t_a, F->vpoly);
  // 5. band bricks
  k_fill_i32<<<grid_1d(nbt, B), B, 0, s>>>(F->t_b, nbt, 0);
  k_mark_bricks<<<grid_1d(nf, B), B, 0, s>>>(verts_d, tris_d, nf, *grid, nb[0], nb[1], nb[2], F->t_b);
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
