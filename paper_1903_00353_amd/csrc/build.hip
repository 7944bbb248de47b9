// Feature construction (Section 7, Section 8) for a batch of meshes: adjacency,
// normals, edge and vertex classes, polyhedron lists and the band bricks.
//
// Unlike the paper's Morton-code sort of a triangle soup (Section 7.1, 7.2) the
// input here is indexed, so the corners of all triangles are grouped by vertex
// (stable radix sort, or counting + scatter + per-vertex sort when the build is
// captured into a graph), twins are matched around each vertex, and edges are
// numbered by a prefix sum over the half-edges that own them (start index < end
// index). Every id is deterministic. The whole sequence is device work with no
// host synchronisation; csc_features_sync reads errors and counts back.
#include <string.h>

#include <new>

#include "geometry.h"
#include "internal.h"
#include "wave.h"

namespace csc {

__device__ inline d3 vload_d(const float* V, int64_t i) {
  return mkd((double)V[3 * i], (double)V[3 * i + 1], (double)V[3 * i + 2]);
}
__device__ inline f3 vload_f(const float* V, int64_t i) { return mk(V[3 * i], V[3 * i + 1], V[3 * i + 2]); }
__device__ inline uint32_t* err_word(int64_t* stats) { return (uint32_t*)&stats[ST_ERR]; }

// corner c = 3f + j (32-bit: 3F < 2^31): the corner after / before it in its face
__device__ inline int32_t next_corner(int32_t c) { int32_t j = c % 3; return c - j + (j == 2 ? 0 : j + 1); }
__device__ inline int32_t prev_corner(int32_t c) { int32_t j = c % 3; return c - j + (j == 0 ? 2 : j - 1); }
// corner c itself and the corners after / before it, from its face's record
__device__ inline float4 rec_at(const FaceRec* R, int32_t c) { return R[c / 3].c[c % 3]; }
__device__ inline float4 rec_next(const FaceRec* R, int32_t c) {
  const int32_t j = c % 3;
  return R[c / 3].c[j == 2 ? 0 : j + 1];
}
__device__ inline float4 rec_prev(const FaceRec* R, int32_t c) {
  const int32_t j = c % 3;
  return R[c / 3].c[j == 0 ? 2 : j - 1];
}
__device__ inline f3 rec_posf(float4 c) { return mk(c.x, c.y, c.z); }

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_zero_i64(int64_t* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// Per face: its mesh, index range and repeated-corner checks, global indices. A
// face with a bad index is replaced by three copies of its mesh's first vertex so
// that every later access stays in bounds (the build then reports the error).
__device__ inline void globalize_face(const int32_t* __restrict__ T, int64_t f, int m,
                                      const int32_t* __restrict__ v_off, int32_t* tg, int32_t* face_mesh,
                                      int32_t* owned, int64_t* stats) {
  const int32_t nvm = v_off[m + 1] - v_off[m], vo = v_off[m];
  int32_t a = T[3 * f], b = T[3 * f + 1], c = T[3 * f + 2];
  if (a < 0 || b < 0 || c < 0 || a >= nvm || b >= nvm || c >= nvm) {
    atomicOr(err_word(stats), ERR_INDEX);
    a = b = c = 0;
  } else if (a == b || b == c || a == c) {
    atomicOr(err_word(stats), ERR_REPEAT);
  }
  tg[3 * f] = a + vo;
  tg[3 * f + 1] = b + vo;
  tg[3 * f + 2] = c + vo;
  face_mesh[f] = m;
  // half-edge u -> w numbers its edge when u < w
  owned[3 * f] = a < b ? 1 : 0;
  owned[3 * f + 1] = b < c ? 1 : 0;
  owned[3 * f + 2] = c < a ? 1 : 0;
}

// the largest m with off[m] <= x (off ascending, off[n_meshes] > x), stepping up
// from m0 <= that m
__device__ inline int segment_from(const int32_t* __restrict__ off, int m0, int64_t x) {
  int m = m0;
  while ((int64_t)off[m + 1] <= x) m++;
  return m;
}

// the input passes in one launch: finite coordinates (thread i < 3 nv); global
// indices and owned half-edges of face i < nf; mesh of vertex i < nv. The meshes
// of the block's first face and vertex are searched once; each thread steps up
// from there (a block rarely crosses a mesh boundary).
__global__ void k_inputs(const float* __restrict__ V, int64_t nv, const int32_t* __restrict__ T, int64_t nf,
                         const int32_t* __restrict__ f_off, const int32_t* __restrict__ v_off, int n_meshes,
                         int32_t* tg, int32_t* face_mesh, int32_t* owned, int32_t* vert_mesh, int64_t* stats) {
  __shared__ int s_mf, s_mv;
  const int64_t b0 = blockIdx.x * (int64_t)blockDim.x, i = b0 + threadIdx.x;
  if (threadIdx.x == 0) {
    s_mf = b0 < nf ? find_segment(f_off, n_meshes + 1, b0) : 0;
    s_mv = b0 < nv ? find_segment(v_off, n_meshes + 1, b0) : 0;
  }
  __syncthreads();
  if (i < 3 * nv && !isfinite(V[i])) atomicOr(err_word(stats), ERR_NONFINITE);
  if (i < nf) globalize_face(T, i, segment_from(f_off, s_mf, i), v_off, tg, face_mesh, owned, stats);
  if (i < nv) vert_mesh[i] = segment_from(v_off, s_mv, i);
}

struct FillJob {
  int32_t* p;
  int64_t n;
  int32_t v;
};

// three fills in one launch, over the concatenated ranges
__global__ void k_fill3(FillJob a, FillJob b, FillJob c) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < a.n) {
    a.p[i] = a.v;
    return;
  }
  i -= a.n;
  if (i < b.n) {
    b.p[i] = b.v;
    return;
  }
  i -= b.n;
  if (i < c.n) c.p[i] = c.v;
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

// Absorbing nearly flat features into the face prisms. A cell whose closest
// point q lies inside edge e (faces f1, f2 with unit normals n1, n2 at angle
// theta) sees q along a unit direction u perpendicular to e within theta of n1
// (or of -n1, concave side), so its projection onto f1's plane lies within
// r sin(theta) <= band h sin(theta) of q, a point of f1: it is inside f1's prism
// once the prism's side planes are moved out by that much, and there its exact
// distance to f1 is its distance to e. Likewise a cell whose closest point is
// vertex v sees it along a direction within theta_v (the cone aperture, every
// incident normal within theta_v of the pseudonormal N) of +N or -N: every
// tangent direction of the fan lies within theta_v of the plane normal to N,
// and q = v minimises the distance only if u has no positive component along
// any of them. Such a u is within 2 theta_v of +-n_f for every incident face,
// so the cell is inside the prism of f with slack band h sin(2 theta_v). When
// that slack is at most `absorb` cells the feature gets no polyhedron of its
// own and every face holding it takes the slack (rounded up, in 1/1024 cells).
// Flat features (theta = 0) already get none. Ruff vertices and hemispheres,
// and edges of unknown class, keep their polyhedra. The vertex pass keeps its
// slack code in the vertex's class word, the edge pass in a byte per edge (both
// written by the thread that owns the feature), and k_face_slack gives every
// face the largest code of its three edges and three vertices.
constexpr float SLACK_UNIT = 1.f / 1024.f;  // cells per step of the stored slack

__device__ inline uint8_t slack_code(double cells, float absorb) {
  if (!(cells <= (double)absorb)) return 0;
  const double q = ceil(cells * 1024.0) + 1.0;  // one step more: never below the bound
  return (uint8_t)(q < 255.0 ? q : 255.0);
}

__device__ inline uint8_t edge_slack(d3 u, d3 w, d3 c1, d3 c2, float band, float absorb) {
  const d3 n1 = cross(w - u, c1 - u), n2 = cross(u - w, c2 - w);
  const double l = len(n1) * len(n2);
  if (!(l > 0) || !(dot(n1, n2) > 0)) return 0;  // theta >= 90 degrees
  return slack_code((double)band * len(cross(n1, n2)) / l, absorb);
}

__device__ inline uint8_t vertex_slack(const VertexClass& cl, float band, float absorb) {
  if (!(cl.bits & (V_POS | V_NEG)) || (cl.bits & (V_POS_HEMI | V_NEG_HEMI | V_RUFF))) return 0;
  const double c = cl.cos_t;
  if (!(c > 0.7071067811865476) || c > 1.0) return 0;  // 2 theta up to 90 degrees
  const double sn = sqrt(fmax(0.0, 1.0 - c * c));
  return slack_code((double)band * 2.0 * sn * c, absorb);  // band * sin(2 theta)
}

constexpr int VK_THREADS = 128;
constexpr int VK_MAXD = 12;  // fans up to this degree are staged in LDS (18 KB per block: 4 wavefronts per SIMD)

// Per vertex u, over its fan of corners (staged in LDS; positions gathered from
// the vertex array, which stays far better cached than the face records):
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
                                                      int force_both, const int32_t* __restrict__ vert_mesh,
                                                      const MeshDesc* __restrict__ md, float absorb, int32_t* twin,
                                                      float4* vinfo, uint32_t* vbits,
                                                      int64_t* stats) {
  __shared__ int32_t s_c[VK_MAXD][VK_THREADS], s_n[VK_MAXD][VK_THREADS], s_p[VK_MAXD][VK_THREADS];
  const int t = threadIdx.x;
  const int64_t v = xcd_block() * VK_THREADS + t;
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
  if (e) atomicOr(err_word(stats), e);
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
  // a nearly flat vertex hands its region to the prisms of its faces (side slack
  // band * sin(2 theta), theta the cone aperture): see vertex_slack
  const uint8_t q = absorb > 0.f && !force_both ? vertex_slack(cl, md[vert_mesh[v]].band, absorb) : 0;
  if (q) cl.bits = (cl.bits & ~(V_POS | V_NEG)) | V_ABSORBED | ((uint32_t)q << V_SLACK_SHIFT);
  float cf = (float)cl.cos_t;
  if ((double)cf > cl.cos_t) cf = nextafterf(cf, -2.f);  // the stored cone contains the exact one
  vinfo[v] = make_float4((float)cl.axis.x, (float)cl.axis.y, (float)cl.axis.z, cf);
  vbits[v] = cl.bits;
}

// Edge records from the owned half-edges (u -> w with u < w) and, for each edge,
// its class from the exact orientation of its four corners (Section 8.2: the
// discriminant of the two face normals, evaluated exactly) with the sides to
// extrude. The third corner of the owning face precedes u in that face; the
// third corner of the twin's face precedes the twin's start. (An open or
// non-manifold surface can own more or fewer than 3F/2 half-edges: such a build
// is rejected, and nothing is written past ne; cls is zero-filled
// beforehand, so edges no half-edge produced stay unclassified and empty.)
__global__ void k_edges(const FaceRec* __restrict__ R, int64_t nh, int64_t ne,
                        const int32_t* __restrict__ twin, const int32_t* __restrict__ eid, int force_both,
                        const int32_t* __restrict__ face_mesh, const MeshDesc* __restrict__ md, float absorb,
                        int4* edges, int32_t* face_edges, uint8_t* cls, uint8_t* eslack) {
  int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (h >= nh) return;
  // this face's record: the three threads of a face read one sector together
  const float4 cu = rec_at(R, (int32_t)h), cw = rec_next(R, (int32_t)h);
  int32_t u = rec_vertex(cu), w = rec_vertex(cw);
  int32_t t = twin[h];
  if (u < w) {
    int32_t e = eid[h];
    face_edges[h] = e < ne ? e : -1;
    if (e >= ne) return;
    edges[e] = make_int4(u, w, (int)(h / 3), t >= 0 ? t / 3 : -1);
    int c = 0, sides = 0;
    uint8_t q = 0;
    if (t >= 0) {
      const f3 fu = rec_posf(cu), fw = rec_posf(cw), f1 = rec_posf(rec_prev(R, (int32_t)h)),
               f2 = rec_posf(rec_prev(R, t));
      c = classify_edge(fu, fw, f1, f2);
      if (c == EDGE_CONVEX) sides = 1;
      else if (c == EDGE_CONCAVE) sides = 2;
      else if (c == EDGE_UNKNOWN) sides = 3;
      if (force_both) sides = 3;
      // a nearly flat edge hands its wedge to its two face prisms
      if (absorb > 0.f && !force_both && (c == EDGE_CONVEX || c == EDGE_CONCAVE)) {
        q = edge_slack(tod(fu), tod(fw), tod(f1), tod(f2), md[face_mesh[h / 3]].band, absorb);
        if (q) sides = 0;
      }
    }
    eslack[e] = q;
    cls[e] = (uint8_t)(c | (sides << 2) | (q ? EDGE_ABSORBED : 0));
  } else {
    int32_t e = t >= 0 ? eid[t] : -1;
    face_edges[h] = e < ne ? e : -1;
  }
}

// Unit face normal (double precision, stored in single) and the band bricks near
// the face: the bricks holding a cell centre within band*h + eps of the face's
// bounding box, less those whose centres all lie farther than that from the
// face's plane. Every polyhedron of the face, its edges and its vertices lies in
// that box (the face prism within band*h*|n_k| + eps of the face along each
// axis, edge wedges and vertex cones within band*h + eps of their feature), and
// a scan writes only cells within band*h of a feature, so every cell a scan can
// write has its brick marked by one of the faces holding its feature.
__device__ inline void face_geom_one(const float* __restrict__ V, const int32_t* __restrict__ T, int64_t f,
                                     const int32_t* __restrict__ face_mesh, const MeshDesc* __restrict__ md,
                                     FaceRec* rec, int32_t* flag, int64_t* stats) {
  const int32_t ia = T[3 * f], ib = T[3 * f + 1], ic = T[3 * f + 2];
  const f3 af = vload_f(V, ia), bf = vload_f(V, ib), cf = vload_f(V, ic);
  const d3 a = mkd(af.x, af.y, af.z), b = mkd(bf.x, bf.y, bf.z), c = mkd(cf.x, cf.y, cf.z);
  const d3 n = cross(b - a, c - a);
  const double l = len(n);
  float4 un4 = make_float4(0.f, 0.f, 0.f, 0.f);
  if (!(l > 0)) atomicOr(err_word(stats), ERR_DEGENERATE);
  else un4 = make_float4((float)(n.x / l), (float)(n.y / l), (float)(n.z / l), 0.f);
  // the face's record: later passes read one aligned sector per face instead of
  // three vertex gathers
  FaceRec& o = rec[f];
  o.c[0] = make_float4(af.x, af.y, af.z, __int_as_float(ia));
  o.c[1] = make_float4(bf.x, bf.y, bf.z, __int_as_float(ib));
  o.c[2] = make_float4(cf.x, cf.y, cf.z, __int_as_float(ic));
  o.n = un4;
  const MeshDesc& g = md[face_mesh[f]];
  const double r = g.whd + g.epsd;
  const double X[3][3] = {{a.x, b.x, c.x}, {a.y, b.y, c.y}, {a.z, b.z, c.z}};
  int lo[3], hi[3];
  for (int ax = 0; ax < 3; ax++) {
    const double x0 = X[ax][0], x1 = X[ax][1], x2 = X[ax][2];
    const double mn = fmin(x0, fmin(x1, x2)) - r, mx = fmax(x0, fmax(x1, x2)) + r;
    // cells whose centre lies in [mn, mx], widened by 1e-3 cells against rounding
    // (the scan's own boxes are widened by 1e-4 cells)
    double lo_c = ceil((mn - g.origin[ax]) * g.inv_h - 0.5 - 1e-3);
    double hi_c = floor((mx - g.origin[ax]) * g.inv_h - 0.5 + 1e-3);
    lo_c = fmax(lo_c, 0.0);
    hi_c = fmin(hi_c, (double)(g.n[ax] - 1));
    if (!(lo_c <= hi_c)) return;
    lo[ax] = (int)lo_c / BRICK;
    hi[ax] = (int)hi_c / BRICK;
  }
  // A brick is kept only if some cell centre in it can lie within r of the face's
  // plane: a cell within band*h of an edge or vertex is that close to a face
  // holding it, and no key is written farther out. The centres of brick (x, y, z)
  // fill a box of half-width (BRICK - 1) h / 2 around origin + (BRICK x + BRICK / 2) h,
  // whose distance to the plane is at least |n.(c - a)| - (BRICK - 1) h |n|_1 / 2.
  // The test gets 1e-3 h of slack over r against rounding; a degenerate face
  // keeps its whole box.
  const bool cull = l > 0;
  const d3 un = cull ? mkd(n.x / l, n.y / l, n.z / l) : mkd(0.0, 0.0, 0.0);
  const double ext = 0.5 * (BRICK - 1) * g.h * (fabs(un.x) + fabs(un.y) + fabs(un.z)), lim = r + 1e-3 * g.h;
  for (int z = lo[2]; z <= hi[2]; z++)
    for (int y = lo[1]; y <= hi[1]; y++)
      for (int x = lo[0]; x <= hi[0]; x++) {
        if (cull) {
          const d3 c = mkd(g.origin[0] + (BRICK * x + BRICK / 2) * g.h, g.origin[1] + (BRICK * y + BRICK / 2) * g.h,
                           g.origin[2] + (BRICK * z + BRICK / 2) * g.h);
          if (fabs(dot(un, c - a)) - ext > lim) continue;
        }
        flag[brick_pos(g, x, y, z)] = 1;  // plain stores: no read to wait for
      }
}

// a grid striding over the faces (geom_blocks: sized below the device, so
// that the corner sort, which it runs beside, keeps compute units of its own)
__global__ void k_face_geom(const float* __restrict__ V, const int32_t* __restrict__ T, int64_t nf,
                            const int32_t* __restrict__ face_mesh, const MeshDesc* __restrict__ md, FaceRec* rec,
                            int32_t* flag, int64_t* stats) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < nf; f += stride)
    face_geom_one(V, T, f, face_mesh, md, rec, flag, stats);
}

// class statistics (and absorbed features): each thread counts 16 edge-class bytes and 4 vertex words per
// 16-byte load (both arrays start 256-byte aligned), one LDS histogram per
// block, one global add per bin and block
__device__ inline void count_edge_class(int c, int (&loc)[11]) {
  loc[9] += (c & EDGE_ABSORBED) != 0;
  c &= 3;
  loc[0] += c == EDGE_CONVEX;
  loc[1] += c == EDGE_CONCAVE;
  loc[2] += c == EDGE_FLAT;
  loc[3] += c == EDGE_UNKNOWN;
}
__device__ inline void count_vertex_class(uint32_t b, int (&loc)[11]) {
  loc[4] += (b & V_CONVEX) != 0;
  loc[5] += (b & V_CONCAVE) != 0;
  loc[6] += (b & V_FLAT) != 0;
  loc[7] += (b & V_SADDLE) != 0;
  loc[8] += (b & V_RUFF) != 0;
  loc[10] += (b & V_ABSORBED) != 0;
}

__global__ __launch_bounds__(256) void k_class_stats(const uint8_t* __restrict__ ecls, int64_t ne,
                                                     const uint32_t* __restrict__ vbits, int64_t nv, int64_t* stats) {
  __shared__ int h[16];
  if (threadIdx.x < 16) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  int loc[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const uint4* e16 = reinterpret_cast<const uint4*>(ecls);
  for (int64_t i = t0; i < ne / 16; i += stride) {
    const uint4 x = e16[i];
    const uint32_t wv[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int q = 0; q < 4; q++)
#pragma unroll
      for (int k = 0; k < 4; k++) count_edge_class((int)((wv[q] >> (8 * k)) & 0xffu), loc);
  }
  for (int64_t i = ne / 16 * 16 + t0; i < ne; i += stride) count_edge_class(ecls[i], loc);
  const uint4* v4 = reinterpret_cast<const uint4*>(vbits);
  for (int64_t i = t0; i < nv / 4; i += stride) {
    const uint4 x = v4[i];
    count_vertex_class(x.x, loc);
    count_vertex_class(x.y, loc);
    count_vertex_class(x.z, loc);
    count_vertex_class(x.w, loc);
  }
  for (int64_t i = nv / 4 * 4 + t0; i < nv; i += stride) count_vertex_class(vbits[i], loc);
#pragma unroll
  for (int k = 0; k < 11; k++) {
    int x = loc[k];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd(&h[k], x);
  }
  __syncthreads();
  const int map[11] = {ST_E_CONVEX, ST_E_CONCAVE, ST_E_FLAT, ST_E_UNKNOWN, ST_V_CONVEX, ST_V_CONCAVE,
                       ST_V_FLAT,   ST_V_SADDLE,  ST_V_RUFF, ST_E_ABSORBED, ST_V_ABSORBED};
  if (threadIdx.x < 11 && h[threadIdx.x])
    atomicAdd((unsigned long long*)&stats[map[threadIdx.x]], (unsigned long long)h[threadIdx.x]);
}

// per face: the largest slack code of its edges and vertices (gathers of the
// coalesced per-feature codes instead of scattered byte writes per face side),
// and which of them are absorbed (the face scan signs their cells itself)
__global__ void k_face_slack(const int32_t* __restrict__ T, const int32_t* __restrict__ face_edges,
                             const uint32_t* __restrict__ vbits, const uint8_t* __restrict__ eslack, int64_t nf,
                             int64_t ne, uint8_t* fslack, uint8_t* fabsorbed) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  uint32_t q = 0, bits = 0;
#pragma unroll
  for (int j = 0; j < 3; j++) {
    const uint32_t qv = (vbits[T[3 * f + j]] >> V_SLACK_SHIFT) & 0xffu;
    q = max(q, qv);
    if (qv) bits |= 8u << j;
    const int32_t e = face_edges[3 * f + j];
    const uint32_t qe = e >= 0 && e < ne ? (uint32_t)eslack[e] : 0u;
    q = max(q, qe);
    if (qe) bits |= 1u << j;
  }
  fslack[f] = (uint8_t)q;
  fabsorbed[f] = (uint8_t)bits;
}

// The extrusion lists in one compaction: item i (an edge or a vertex) has 0-2
// polyhedra, bit 0 of its side mask the outward one (entry i << 1) and bit 1
// the inward one ((i << 1) | 1); the entries follow item order. Pass 1 counts
// the polyhedra of each tile of QTILE items; pass 2 gives every tile its offset
// (the sum of the tile counts before it, added up by the block itself when the
// tiles are few, else scanned beforehand) and writes its entries, ranked inside
// the tile by a block scan. The side masks come straight from the classes, so
// no count array and no separate queue launch are needed.
struct VertexSides {
  const uint32_t* bits;
  __device__ int operator()(int64_t i) const { return (int)(bits[i] & (V_POS | V_NEG)); }
};
struct EdgeSides {
  const uint8_t* cls;
  __device__ int operator()(int64_t i) const { return (cls[i] >> 2) & 3; }
};
constexpr int QB = 256, QITEMS = 8, QTILE = QB * QITEMS;
constexpr int64_t Q_SHORT_TILES = 4096;

template <class S>
__global__ __launch_bounds__(QB) void k_queue_sums(S sides, int64_t n, int32_t* sums) {
  const int64_t base = (int64_t)blockIdx.x * QTILE;
  int c = 0;
  for (int i = threadIdx.x; i < QTILE; i += QB) {
    const int64_t idx = base + i;
    if (idx < n) c += __popc(sides(idx));
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
  __shared__ int ws[QB / 64];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < QB / 64; w++) t += ws[w];
    sums[blockIdx.x] = t;
  }
}

template <class S>
__global__ __launch_bounds__(QB) void k_queue_write(S sides, int64_t n, const int32_t* __restrict__ sums, int scanned,
                                                    int32_t* q, int64_t* total) {
  __shared__ int ws[QB / 64];
  __shared__ int wx[QB / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // this tile's offset
  int pre = 0;
  if (!scanned)
    for (int j = threadIdx.x; j < (int)blockIdx.x; j += QB) pre += sums[j];
  for (int o = 32; o > 0; o >>= 1) pre += __shfl_down(pre, o, 64);
  if (lane == 0) ws[w] = pre;
  // this thread's QITEMS consecutive items
  const int64_t first = (int64_t)blockIdx.x * QTILE + (int64_t)threadIdx.x * QITEMS;
  int m[QITEMS], c = 0;
#pragma unroll
  for (int k = 0; k < QITEMS; k++) {
    m[k] = first + k < n ? sides(first + k) : 0;
    c += __popc(m[k]);
  }
  const int incl = wave_prefix_sum(c);
  if (lane == 63) wx[w] = incl;
  __syncthreads();
  int offset = scanned ? sums[blockIdx.x] : 0, before = 0, tile = 0;
#pragma unroll
  for (int u = 0; u < QB / 64; u++) {
    if (!scanned) offset += ws[u];
    before += u < w ? wx[u] : 0;
    tile += wx[u];
  }
  int p = offset + before + incl - c;
#pragma unroll
  for (int k = 0; k < QITEMS; k++) {
    const int32_t id = (int32_t)(first + k);
    if (m[k] & 1) q[p++] = id << 1;
    if (m[k] & 2) q[p++] = (id << 1) | 1;
  }
  if (!scanned && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = offset + tile;
}

template <class S>
hipError_t queue_compact(S sides, int64_t n, int32_t* q, int64_t* total, int32_t* tmp, hipStream_t s) {
  int64_t nb = (n + QTILE - 1) / QTILE;
  if (nb < 1) nb = 1;
  k_queue_sums<S><<<(unsigned)nb, QB, 0, s>>>(sides, n, tmp);
  const bool few = nb <= Q_SHORT_TILES;
  if (!few) {
    hipError_t e = scan_sums_inplace(tmp, nb, total, s);
    if (e != hipSuccess) return e;
  }
  k_queue_write<S><<<(unsigned)nb, QB, 0, s>>>(sides, n, tmp, few ? 0 : 1, q, total);
  return hipGetLastError();
}

// slots of the flagged bricks (index = exclusive prefix of the flags), their
// list and mesh, and the first slot of every mesh
__global__ void k_brick_fix(const int32_t* __restrict__ flag, int32_t* index, int32_t* list, int32_t* bmesh,
                            const int32_t* __restrict__ brick_base, int n_meshes, int32_t* first_slot,
                            const int64_t* __restrict__ stats, int64_t n) {
  int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= n) return;
  const int m = find_segment(brick_base, n_meshes + 1, b);
  if (b == brick_base[m]) first_slot[m] = index[b];
  if (b == n - 1) first_slot[n_meshes] = (int32_t)stats[ST_NBRICKS];
  if (flag[b]) {
    list[index[b]] = (int32_t)b;
    bmesh[index[b]] = m;
  } else {
    index[b] = -1;
  }
}

int status_from_errors(uint64_t err, int64_t ne_found, int64_t ne_expected) {
  if (err & (ERR_INDEX | ERR_REPEAT | ERR_NONFINITE)) return CSC_INVALID_ARG;
  if (err & ERR_OVERFLOW) return CSC_WORKSPACE_TOO_SMALL;
  if (err & ERR_ORIENT) return CSC_INCONSISTENT_ORIENTATION;
  if (err & ERR_NONMANIFOLD) return CSC_NONMANIFOLD;
  if (ne_found != ne_expected) return CSC_NONMANIFOLD;
  if (err & ERR_DEGENERATE) return CSC_DEGENERATE_FACE;
  return CSC_OK;
}

// Key of the spatial processing order of the faces: the Morton code of each
// face's centroid in its own grid, at `axis_bits` bits per axis, with its mesh
// above it (the paper orders its triangle soup by Morton code as well, Section
// 7.1; here the order only schedules the face pass and changes no result).
__global__ void k_face_order_keys(const FaceRec* __restrict__ R, const int32_t* __restrict__ face_mesh,
                                  const MeshDesc* __restrict__ md, int64_t nf, int axis_bits, uint32_t* key) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint32_t top = (1u << axis_bits) - 1u;
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < nf; f += stride) {
    const int m = face_mesh[f];
    const MeshDesc& G = md[m];
    const float4 a = R[f].c[0], b = R[f].c[1], c = R[f].c[2];
    const double x[3] = {((double)a.x + b.x + c.x) / 3.0, ((double)a.y + b.y + c.y) / 3.0,
                         ((double)a.z + b.z + c.z) / 3.0};
    uint32_t code = 0;
    for (int k = 0; k < 3; k++) {
      const double u = (x[k] - G.origin[k]) * G.inv_h / G.n[k] * (double)(1u << axis_bits);
      const uint32_t qk = u <= 0.0 ? 0u : (u >= (double)top ? top : (uint32_t)u);  // NaN-free: finite inputs
      for (int bit = 0; bit < axis_bits; bit++) code |= ((qk >> bit) & 1u) << (3 * bit + k);
    }
    key[f] = ((uint32_t)m << (3 * axis_bits)) | code;
  }
}

}  // namespace csc

using namespace csc;

extern "C" int csc_features_order_faces(csc_features* F, int32_t enable, void* stream) {
  if (!F || !F->built || (enable != 0 && enable != 1)) return CSC_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (!enable || F->nf == 0) {
    if (F->face_order) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(F->face_order);
      F->face_order = nullptr;
      F->face_order_n = 0;
    }
    return CSC_OK;
  }
  const int64_t nf = F->nf;
  int mesh_bits = 0;
  while ((1 << mesh_bits) < F->n_meshes) mesh_bits++;
  int axis_bits = (32 - mesh_bits) / 3;
  if (axis_bits > 10) axis_bits = 10;
  const int bits = mesh_bits + 3 * axis_bits;
  const size_t sort_bytes = sort_pairs_tmp_bytes(nf, bits);
  if (sort_bytes == 0) return CSC_INVALID_ARG;
  const size_t key_bytes = ((size_t)nf * sizeof(uint32_t) + 255) & ~(size_t)255;
  if (!F->face_order) {
    hipError_t he = hipMalloc((void**)&F->face_order, sizeof(int32_t) * (size_t)nf);
    if (he != hipSuccess) {
      F->face_order = nullptr;
      return he == hipErrorOutOfMemory ? CSC_OUT_OF_MEMORY : fail_hip(he);
    }
  }
  F->face_order_n = 0;  // not valid until the sort below has run
  char* tmp = nullptr;
  hipError_t he = hipMalloc((void**)&tmp, 2 * key_bytes + sort_bytes);
  if (he != hipSuccess) return he == hipErrorOutOfMemory ? CSC_OUT_OF_MEMORY : fail_hip(he);
  uint32_t* key = (uint32_t*)tmp;
  uint32_t* key_sorted = (uint32_t*)(tmp + key_bytes);
  k_face_order_keys<<<grid_1d(nf, 256), 256, 0, s>>>(F->face_rec, F->face_mesh, F->d_mesh, nf, axis_bits, key);
  he = hipGetLastError();
  if (he == hipSuccess)
    he = sort_pairs(tmp + 2 * key_bytes, sort_bytes, key, key_sorted, nullptr, F->face_order, nf, bits, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  (void)hipFree(tmp);
  if (he != hipSuccess) return fail_hip(he);
  F->face_order_n = nf;
  return CSC_OK;
}

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

enum {
  L_MESH, L_FOFF, L_VOFF, L_BBASE, L_TRIS, L_FMESH, L_VMESH, L_VTXOFF, L_VTXC, L_FEDGES, L_EDGES, L_FREC, L_ECLS,
  L_VINFO, L_VBITS, L_EPOLY, L_VPOLY, L_BINDEX, L_BLIST, L_BMESH, L_FIRST, L_TA, L_TB, L_TC, L_TSCAN, L_BFLAG,
  L_TSCAN2, L_STATS, L_SORT, L_FSLACK, L_ESLACK, L_FABS, L_EID, L_N
};

struct Layout {
  size_t off[L_N];
  size_t total;
};

Layout layout(int n_meshes, int64_t nv, int64_t nf, int64_t nbt, size_t sort_bytes) {
  const int64_t ne = 3 * nf / 2;
  int64_t big = 3 * nf;
  big = big > nbt ? big : nbt;
  big = big > nv + 1 ? big : nv + 1;
  big = big > ne + 1 ? big : ne + 1;
  size_t sz[L_N];
  sz[L_MESH] = sizeof(MeshDesc) * (size_t)n_meshes;
  sz[L_FOFF] = sz[L_VOFF] = sz[L_BBASE] = sizeof(int32_t) * (size_t)(n_meshes + 1);
  sz[L_TRIS] = sizeof(int32_t) * (size_t)(3 * nf);
  sz[L_FMESH] = sizeof(int32_t) * (size_t)nf;
  sz[L_VMESH] = sizeof(int32_t) * (size_t)nv;
  sz[L_VTXOFF] = sizeof(int32_t) * (size_t)(nv + 1);
  sz[L_VTXC] = sizeof(int32_t) * (size_t)(3 * nf);
  sz[L_FEDGES] = sizeof(int32_t) * (size_t)(3 * nf);
  sz[L_EDGES] = sizeof(int4) * (size_t)(ne + 1);
  sz[L_FREC] = sizeof(FaceRec) * (size_t)nf;
  sz[L_ECLS] = (size_t)((ne + 4) / 4 * 4);  // whole ints: zero-filled as ints
  sz[L_VINFO] = sizeof(float4) * (size_t)nv;
  sz[L_VBITS] = sizeof(uint32_t) * (size_t)nv;
  sz[L_EPOLY] = sizeof(int32_t) * (size_t)(2 * ne + 1);
  sz[L_VPOLY] = sizeof(int32_t) * (size_t)(2 * nv + 1);
  sz[L_BINDEX] = sz[L_BLIST] = sz[L_BMESH] = sizeof(int32_t) * (size_t)nbt;
  sz[L_FIRST] = sizeof(int32_t) * (size_t)(n_meshes + 1);
  sz[L_TA] = sz[L_TB] = sz[L_TC] = sizeof(int32_t) * (size_t)(big + 1);
  sz[L_TSCAN] = sizeof(int32_t) * (size_t)scan_tmp_ints(big + 1);
  sz[L_BFLAG] = sizeof(int32_t) * (size_t)(nbt + 1);
  sz[L_TSCAN2] = sizeof(int32_t) * (size_t)scan_tmp_ints(big + 1);  // the brick flags and the edge numbering
  sz[L_STATS] = sizeof(int64_t) * ST_COUNT;
  sz[L_SORT] = sort_bytes;
  sz[L_FSLACK] = (size_t)(nf + 8);
  sz[L_ESLACK] = (size_t)(ne + 8);
  sz[L_FABS] = (size_t)(nf + 8);
  sz[L_EID] = sizeof(int32_t) * (size_t)(3 * nf + 1);
  Layout L;
  size_t o = 0;
  for (int i = 0; i < L_N; i++) {
    L.off[i] = o;
    o += align_up(sz[i]);
  }
  L.total = o;
  return L;
}

bool finite_pos(double x) { return x > 0 && x < 1e300; }

int check_grid(const csc_grid& g) {
  for (int a = 0; a < 3; a++)
    if (g.n[a] <= 0 || !isfinite(g.origin[a])) return CSC_INVALID_ARG;
  if (!finite_pos(g.h) || !(g.band_cells > 0) || !isfinite(g.band_cells)) return CSC_INVALID_ARG;
  if ((int64_t)g.n[0] * g.n[1] * g.n[2] > INT32_MAX) return CSC_GRID_TOO_LARGE;
  for (int a = 0; a < 3; a++)  // cell offsets inside a polyhedron box are packed in 16 bits
    if (g.n[a] > 65535) return CSC_GRID_TOO_LARGE;
  return CSC_OK;
}

bool same_config(const csc_features* F, const std::vector<MeshDesc>& m, const csc_options& o) {
  if ((int)F->mesh.size() != (int)m.size()) return false;
  if (memcmp(&F->opt, &o, sizeof(o)) != 0) return false;
  return memcmp(F->mesh.data(), m.data(), sizeof(MeshDesc) * m.size()) == 0;
}

}  // namespace

// Shared implementation of the single-mesh and batched builds.
int build_impl(const float* verts_d, const int32_t* tris_d, const int64_t* nv, const int64_t* nf,
               const csc_grid* grids, int32_t n_meshes, const csc_options* opt, int32_t flags, void* stream,
               csc_features** out) {
  if (!verts_d || !tris_d || !nv || !nf || !grids || !out || n_meshes <= 0) return CSC_INVALID_ARG;
  csc_options o = {1e-3f, 0, 0, 0, {0, 0, 0}, 0, 0.f, 0, 0, 0};
  if (opt) o = *opt;
  if (o.scan_grid < 0 || o.scan_grid > 3 || o.geom_blocks < 0 || (o.keep_store_empty & ~1)) return CSC_INVALID_ARG;
  if (o.scan_grid == 0) o.scan_grid = 2;  // default: persistent grid striding over the groups
  if (!(o.absorb_cells <= 0.24f) || o.absorb_cells != o.absorb_cells) return CSC_INVALID_ARG;
  // 0: the default; negative: every non-flat feature keeps its own polyhedron
  if (o.absorb_cells == 0.f) o.absorb_cells = 0.05f;
  if (!(o.eps_rel >= 0) || !(o.eps_rel < 0.5f) || o.ruff_mode < 0 || o.ruff_mode > 1 || o.scan_mode < 0 || o.scan_mode > 1 || o.saddle_mode < 0 ||
      o.saddle_mode > 2)
    return CSC_INVALID_ARG;
  for (int k = 0; k < 3; k++) {
    if (o.small_rows[k] < 0) return CSC_INVALID_ARG;
    if (o.small_rows[k] == 0) o.small_rows[k] = 32;
    if (o.small_rows[k] > (1 << 24)) o.small_rows[k] = 1 << 24;  // row totals of a wavefront stay in 32 bits
  }
  std::vector<MeshDesc> mesh((size_t)n_meshes);
  int64_t tv = 0, tf = 0, te = 0, tb = 0;
  for (int m = 0; m < n_meshes; m++) {
    if (nv[m] <= 0 || nf[m] <= 0) return CSC_INVALID_ARG;
    int gc = check_grid(grids[m]);
    if (gc != CSC_OK) return gc;
    if (nf[m] % 2 != 0) return CSC_NONMANIFOLD;  // a closed triangle surface has 3F/2 edges
    MeshDesc& d = mesh[m];
    memset(&d, 0, sizeof(d));
    const csc_grid& g = grids[m];
    for (int a = 0; a < 3; a++) {
      d.origin[a] = g.origin[a];
      d.n[a] = g.n[a];
      d.nb[a] = (g.n[a] + BRICK - 1) / BRICK;
      d.nt[a] = (d.nb[a] + TILE - 1) / TILE;
    }
    d.h = g.h;
    d.inv_h = 1.0 / g.h;
    d.whd = (double)g.band_cells * g.h;
    d.epsd = (double)o.eps_rel * g.h;
    d.hf = (float)g.h;
    d.whf = (float)d.whd;
    d.eps = (float)d.epsd;
    d.band = g.band_cells;
    d.brick_base = (int32_t)tb;
    d.v_off = (int32_t)tv;
    d.f_off = (int32_t)tf;
    d.e_off = (int32_t)te;
    d.nv = (int32_t)nv[m];
    d.nf = (int32_t)nf[m];
    d.ne = (int32_t)(3 * nf[m] / 2);
    tb += (int64_t)d.nt[0] * d.nt[1] * d.nt[2] * (TILE * TILE * TILE);
    tv += nv[m];
    tf += nf[m];
    te += 3 * nf[m] / 2;
    // feature ids (faces + edges + vertices) must fit in 30 bits of the packed key
    if (tf + te + tv >= (1 << 30)) return CSC_INVALID_ARG;
    if (tb > (1 << 26)) return CSC_GRID_TOO_LARGE;
  }
  int dc = check_device();
  if (dc != CSC_OK) return dc;

  const bool no_sync = (flags & CSC_BUILD_NO_SYNC) != 0;
  hipStream_t s = (hipStream_t)stream;
  csc_features* F = *out;
  const bool fresh = F == nullptr;
  if (fresh) {
    F = new (std::nothrow) csc_features();
    if (!F) return CSC_OUT_OF_MEMORY;
  }
  auto fail = [&](int code) {
    if (fresh) csc_features_free(F);
    else F->built = F->synced = false;
    return code;
  };
  if (F->face_order && F->face_order_n != tf) {  // an order of another face count is dropped
    (void)hipStreamSynchronize(s);
    (void)hipFree(F->face_order);
    F->face_order = nullptr;
    F->face_order_n = 0;
  }
  int sort_bits = 1;
  while (sort_bits < 31 && ((int64_t)1 << sort_bits) < tv) sort_bits++;
  const size_t sort_bytes = sort_pairs_tmp_bytes(3 * tf, sort_bits);
  if (sort_bytes == 0) return fail(fail_hip(hipErrorInvalidValue));
  Layout L = layout(n_meshes, tv, tf, tb, sort_bytes);
  const bool config_changed = fresh || !same_config(F, mesh, o) || F->arena_bytes < L.total || F->nv != tv ||
                              F->nf != tf;
  hipError_t he;
  if (F->arena_bytes < L.total) {
    if (F->arena) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(F->arena);
      F->arena = nullptr;
      F->arena_bytes = 0;
    }
    he = hipMalloc((void**)&F->arena, L.total);
    if (he != hipSuccess) {
      F->arena = nullptr;
      return fail(he == hipErrorOutOfMemory ? CSC_OUT_OF_MEMORY : fail_hip(he));
    }
    F->arena_bytes = L.total;
  }
  if (!F->h_stats) {
    he = hipHostMalloc((void**)&F->h_stats, sizeof(int64_t) * ST_COUNT, hipHostMallocDefault);
    if (he != hipSuccess) {
      F->h_stats = nullptr;
      return fail(fail_hip(he));
    }
  }
  if (!F->side) {  // default priority, like every stream here
    he = hipStreamCreateWithFlags(&F->side, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&F->ev_fork, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&F->ev_join, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&F->ev_geom, hipEventDisableTiming);
    if (he != hipSuccess) return fail(fail_hip(he));
  }
  char* A = F->arena;
  F->n_meshes = n_meshes;
  F->verts = verts_d;
  F->nv = tv;
  F->nf = tf;
  F->ne = te;
  F->nbt = tb;
  F->opt = o;
  F->sort_bits = sort_bits;
  F->d_mesh = (MeshDesc*)(A + L.off[L_MESH]);
  F->f_off = (int32_t*)(A + L.off[L_FOFF]);
  F->v_off = (int32_t*)(A + L.off[L_VOFF]);
  F->brick_base = (int32_t*)(A + L.off[L_BBASE]);
  F->tris_g = (int32_t*)(A + L.off[L_TRIS]);
  F->face_mesh = (int32_t*)(A + L.off[L_FMESH]);
  F->vert_mesh = (int32_t*)(A + L.off[L_VMESH]);
  F->vtx_off = (int32_t*)(A + L.off[L_VTXOFF]);
  F->vtx_corners = (int32_t*)(A + L.off[L_VTXC]);
  F->face_edges = (int32_t*)(A + L.off[L_FEDGES]);
  F->edges = (int4*)(A + L.off[L_EDGES]);
  F->face_rec = (FaceRec*)(A + L.off[L_FREC]);
  F->edge_cls = (uint8_t*)(A + L.off[L_ECLS]);
  F->vinfo = (float4*)(A + L.off[L_VINFO]);
  F->vbits = (uint32_t*)(A + L.off[L_VBITS]);
  F->epoly = (int32_t*)(A + L.off[L_EPOLY]);
  F->vpoly = (int32_t*)(A + L.off[L_VPOLY]);
  F->brick_index = (int32_t*)(A + L.off[L_BINDEX]);
  F->brick_list = (int32_t*)(A + L.off[L_BLIST]);
  F->brick_mesh = (int32_t*)(A + L.off[L_BMESH]);
  F->first_slot = (int32_t*)(A + L.off[L_FIRST]);
  F->t_a = (int32_t*)(A + L.off[L_TA]);
  F->t_b = (int32_t*)(A + L.off[L_TB]);
  F->t_c = (int32_t*)(A + L.off[L_TC]);
  F->t_scan = (int32_t*)(A + L.off[L_TSCAN]);
  F->brick_flag = (int32_t*)(A + L.off[L_BFLAG]);
  F->t_scan2 = (int32_t*)(A + L.off[L_TSCAN2]);
  F->d_stats = (int64_t*)(A + L.off[L_STATS]);
  F->t_sort = (void*)(A + L.off[L_SORT]);
  F->t_sort_bytes = sort_bytes;
  F->fslack = (uint8_t*)(A + L.off[L_FSLACK]);
  F->eslack = (uint8_t*)(A + L.off[L_ESLACK]);
  F->fabsorbed = (uint8_t*)(A + L.off[L_FABS]);
  F->t_eid = (int32_t*)(A + L.off[L_EID]);
  F->built = F->synced = false;

#define CK(x)                                        \
  do {                                               \
    hipError_t e_ = (x);                             \
    if (e_ != hipSuccess) return fail(fail_hip(e_)); \
  } while (0)

  if (config_changed) {
    // descriptors and offset tables change only with the configuration (never
    // inside a captured replay of the same batch)
    std::vector<int32_t> tabs(3 * (size_t)(n_meshes + 1));
    for (int m = 0; m <= n_meshes; m++) {
      tabs[m] = m < n_meshes ? mesh[m].f_off : (int32_t)tf;
      tabs[(n_meshes + 1) + m] = m < n_meshes ? mesh[m].v_off : (int32_t)tv;
      tabs[2 * (n_meshes + 1) + m] = m < n_meshes ? mesh[m].brick_base : (int32_t)tb;
    }
    CK(hipMemcpy(F->d_mesh, mesh.data(), sizeof(MeshDesc) * n_meshes, hipMemcpyHostToDevice));
    CK(hipMemcpy(F->f_off, tabs.data(), sizeof(int32_t) * (n_meshes + 1), hipMemcpyHostToDevice));
    CK(hipMemcpy(F->v_off, tabs.data() + (n_meshes + 1), sizeof(int32_t) * (n_meshes + 1), hipMemcpyHostToDevice));
    CK(hipMemcpy(F->brick_base, tabs.data() + 2 * (n_meshes + 1), sizeof(int32_t) * (n_meshes + 1),
                 hipMemcpyHostToDevice));
    F->mesh = mesh;
  }

  StageTimer timer(TS_BUILD, s);
  const int B = 256;
  const int64_t nh = 3 * tf, ne = te;
  // 1. inputs: finite coordinates, per-mesh index ranges, global indices
  k_zero_i64<<<1, 64, 0, s>>>(F->d_stats, ST_COUNT);
  // (the owned half-edge flags wait in face_edges, which k_edges fills later)
  k_inputs<<<grid_1d(3 * tv > tf ? 3 * tv : tf, B), B, 0, s>>>(verts_d, tv, tris_d, tf, F->f_off, F->v_off, n_meshes,
                                                               F->tris_g, F->face_mesh, F->face_edges,
                                                               F->vert_mesh, F->d_stats);
  const int32_t* T = F->tris_g;
  // Face records (corners, vertex indices, normal) with the band bricks near each
  // face, the brick slots and lists, the cleared edge tables and the edge
  // numbering: they need only the inputs, so they run on the side stream while
  // the corner table is sorted and the vertices classified here; the edge pass
  // waits for the records, the tables and the numbering.
  CK(hipEventRecord(F->ev_fork, s));
  // 2. vertex -> corner table: corners sorted by vertex (stable: each vertex's
  // corners in ascending order), then the segment starts
  CK(sort_pairs(F->t_sort, F->t_sort_bytes, (const uint32_t*)T, (uint32_t*)F->t_b, nullptr, F->vtx_corners, nh,
                sort_bits, s));
  k_offsets<<<grid_1d(nh, B), B, 0, s>>>((const uint32_t*)F->t_b, nh, tv, F->vtx_off);
  // the side branch (forked right after the inputs, issued after the sort so
  // that the sort's launches reach the device first)
  CK(hipStreamWaitEvent(F->side, F->ev_fork, 0));
  {
    hipStream_t s2 = F->side;
    k_fill_i32<<<grid_1d(tb, B), B, 0, s2>>>(F->brick_flag, tb, 0);
    {
      const unsigned need = grid_1d(tf, B), cap = (unsigned)o.geom_blocks;
      k_face_geom<<<cap > 0 && need > cap ? cap : need, B, 0, s2>>>(verts_d, T, tf, F->face_mesh, F->d_mesh,
                                                                    F->face_rec, F->brick_flag, F->d_stats);
    }
    {
      const FillJob a = {(int32_t*)F->edges, 4 * (ne + 1), -1}, b = {nullptr, 0, 0},
                    c = {(int32_t*)F->edge_cls, (ne + 3) / 4, 0};
      k_fill3<<<grid_1d(a.n + b.n + c.n, B), B, 0, s2>>>(a, b, c);
    }
    // edge ids: a prefix sum over the owned half-edge flags that k_inputs left in face_edges
    CK(exclusive_scan(F->face_edges, F->t_eid, nh, F->t_scan2, &F->d_stats[ST_NE], nullptr, s2));
    CK(hipEventRecord(F->ev_geom, s2));
    CK(exclusive_scan(F->brick_flag, F->brick_index, tb, F->t_scan2, &F->d_stats[ST_NBRICKS], nullptr, s2));
    k_brick_fix<<<grid_1d(tb, B), B, 0, s2>>>(F->brick_flag, F->brick_index, F->brick_list, F->brick_mesh,
                                              F->brick_base, n_meshes, F->first_slot, F->d_stats, tb);
    CK(hipEventRecord(F->ev_join, s2));
  }
  // 3. per vertex: twins, pseudonormal, class, cone; then edge numbering
  const float absorb = o.absorb_cells > 0.f ? o.absorb_cells : 0.f;
  k_vertex<<<grid_1d(tv, VK_THREADS), VK_THREADS, 0, s>>>(verts_d, T, tv, F->vtx_off, F->vtx_corners, o.ruff_mode,
                                                        o.saddle_mode, o.force_both_sides, F->vert_mesh, F->d_mesh,
                                                        absorb, F->t_a, F->vinfo, F->vbits, F->d_stats);
  CK(queue_compact(VertexSides{F->vbits}, tv, F->vpoly, &F->d_stats[ST_NVPOLY], F->t_scan, s));
  // edges with their classes and extrusion sides
  CK(hipStreamWaitEvent(s, F->ev_geom, 0));  // the face records, cleared edge tables and edge ids
  k_edges<<<grid_1d(nh, B), B, 0, s>>>(F->face_rec, nh, ne, F->t_a, F->t_eid, o.force_both_sides, F->face_mesh,
                                       F->d_mesh, absorb, F->edges, F->face_edges, F->edge_cls, F->eslack);
  k_face_slack<<<grid_1d(tf, B), B, 0, s>>>(T, F->face_edges, F->vbits, F->eslack, tf, ne, F->fslack,
                                            F->fabsorbed);
  // 4. edge polyhedron queue (the class statistics, which only the feature
  // counts report, are taken by csc_features_sync when it reads them back)
  CK(queue_compact(EdgeSides{F->edge_cls}, ne, F->epoly, &F->d_stats[ST_NEPOLY], F->t_scan, s));
  F->classes_counted = false;
  // 5. join the side stream
  CK(hipStreamWaitEvent(s, F->ev_join, 0));
  CK(hipGetLastError());
#undef CK
  F->built = true;
  if (no_sync) return CSC_OK;
  int rc = csc_features_sync(F, stream);
  if (rc != CSC_OK) return fail(rc);
  *out = F;
  return CSC_OK;
}

extern "C" int csc_features_sync(csc_features* F, void* stream) {
  if (!F || !F->built || !F->h_stats) return CSC_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (!F->classes_counted) {  // once per build: the classes stay until the next one
    const int64_t items = (F->ne / 16 > F->nv / 4 ? F->ne / 16 : F->nv / 4) + 1;
    k_class_stats<<<grid_1d(items < 1024 * 256 ? items : 1024 * 256, 256), 256, 0, s>>>(F->edge_cls, F->ne,
                                                                                       F->vbits, F->nv, F->d_stats);
    F->classes_counted = true;
  }
  hipError_t he = hipMemcpyAsync(F->h_stats, F->d_stats, sizeof(int64_t) * ST_COUNT, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return fail_hip(he);
  const int64_t* st = F->h_stats;
  int rc = status_from_errors((uint64_t)(uint32_t)st[ST_ERR], st[ST_NE], F->ne);
  if (rc != CSC_OK) {
    F->synced = false;
    return rc;
  }
  F->n_epoly = st[ST_NEPOLY];
  F->n_vpoly = st[ST_NVPOLY];
  F->n_bricks = st[ST_NBRICKS];
  csc_feature_info& I = F->info;
  I.n_vertices = F->nv;
  I.n_faces = F->nf;
  I.n_edges = F->ne;
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
  I.edges_absorbed = st[ST_E_ABSORBED];
  I.vertices_absorbed = st[ST_V_ABSORBED];
  I.n_bricks = F->n_bricks;
  I.max_band_cells = F->n_bricks * BRICK_CELLS;
  F->synced = true;
  return CSC_OK;
}

extern "C" int csc_build_features(const float* verts_d, int64_t nv, const int32_t* tris_d, int64_t nf,
                                  const csc_grid* grid, const csc_options* opt, void* stream, csc_features** out) {
  if (!grid) return CSC_INVALID_ARG;
  return build_impl(verts_d, tris_d, &nv, &nf, grid, 1, opt, 0, stream, out);
}

extern "C" int csc_build_features_batched(const float* verts_d, const int32_t* tris_d, const int64_t* nv,
                                          const int64_t* nf, const csc_grid* grids, int32_t n_meshes,
                                          const csc_options* opt, int32_t flags, void* stream, csc_features** out) {
  if (flags & ~(CSC_BUILD_NO_SYNC | CSC_BUILD_GRAPH_SAFE)) return CSC_INVALID_ARG;
  if ((flags & CSC_BUILD_NO_SYNC) && (!out || !*out)) return CSC_INVALID_ARG;
  return build_impl(verts_d, tris_d, nv, nf, grids, n_meshes, opt, flags, stream, out);
}
