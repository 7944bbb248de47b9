// Scan conversion of the characteristic polyhedra (Section 5, Section 9,
// Section 10) and the sign pass (Section 4.1.3), for a batch of meshes.
//
// Each polyhedron is walked row by row along the grid axis closest to its main
// direction (face normal, edge bisector, vertex axis): for every row of its
// bounding box the cells inside are found at once by intersecting the row with
// the half-spaces (the half-space test with slack of Alg. 2 solved for the row
// parameter) and, for vertices, with the ball of radius band*h; cones test their
// discriminant (Eq. 10) per cell. Each candidate cell gets the exact clamped
// point-feature distance and one packed 64-bit atomicMin of (float bits of |d|,
// feature id) into the brick store, the order-free replacement of the paper's
// float compare-and-swap loop (Section 9).
// Small polyhedra take one thread each (the paper's per-extrusion scheme); those
// with more rows go to an overflow list that a second kernel walks with one
// wavefront per polyhedron, its lanes splitting the rows (the role of the
// dynamic-parallelism hybrid of Section 9.1). Item counts are read on the
// device, so the whole sequence runs without host synchronisation.
#include "geometry.h"
#include "internal.h"
#include "wave.h"

namespace csc {

enum { KIND_FACE = 0, KIND_EDGE = 1, KIND_VERT = 2 };

struct ScanArgs {
  const float* V;
  const int32_t* T;            // global vertex indices
  const FaceRec* frec;         // [nf] corners, vertex indices, unit normal
  const int4* edges;
  const int32_t* face_edges;   // [nf][3] edge of each face side (wide faces: boundary signs)
  const uint8_t* fslack;       // [nf] side slack of each face prism (absorbed edges and vertices, 1/1024 cells)
  const uint8_t* fabsorbed;    // [nf] the face's absorbed edges (bits 0-2) and vertices (bits 3-5)
  const uint8_t* ecls;
  const float4* vinfo;
  const uint32_t* vbits;
  const int32_t* items;        // edge / vertex polyhedron list (unused for faces)
  const int64_t* n_items_d;    // device count of items (null: n_items)
  const int32_t* face_mesh;
  const int32_t* vert_mesh;
  const MeshDesc* md;
  const int32_t* brick_index;
  unsigned long long* keys;
  unsigned long long* counter;  // optional: number of atomicMin issued (diagnostics)
  // overflow list: polyhedra of this kind (item indices) with more than small_rows
  // rows from the front, wide ones from the back; their rows are cut into
  // chunks of OV_CHUNK, numbered in list order (ov_chunk0: an entry's first)
  int32_t* ov_items;
  int32_t* ov_chunk0;
  unsigned long long* ov_ctr;   // [0] front: entries << 36 | chunks, [1] back (wide) the same
  int64_t ov_cap;               // entries the two ends share
  int64_t* stats;               // error word (brick capacity overflow)
  int64_t cap;                  // bricks the key store holds
  int64_t nf, ne, n_items;      // totals; n_items = launch bound
  int32_t small_rows;           // more rows: one wavefront per polyhedron
  int32_t per_cell;             // 1: test every box cell by itself (Alg. 2) instead of row intervals
  int32_t grid_mode;            // one-polyhedron-per-lane pass: SCAN_GRID_* (how waves get their polyhedra)
  unsigned long long* head;     // SCAN_GRID_QUEUE: next group of 64 polyhedra to hand out
  int32_t queue_chunk;          // SCAN_GRID_QUEUE: groups a wavefront takes per pop
  // diagnostics (null in normal runs): every packed atomicMin instruction of this
  // launch logged as one round, its lanes' key indices at log[64 r + lane] and
  // the mask of issuing lanes at log_mask[r]
  uint32_t* log;
  unsigned long long* log_mask;
  unsigned* log_rounds;
  int64_t log_cap;              // rounds the log holds (later rounds are counted only)
};

// Packed key of a candidate: float bits of |d| in the high word; the low word
// holds the global feature id in bits 0-29 and, in bits 30-31, the sign when
// this polyhedron alone decides it (0 outside, 1 inside) or 2 when the sign pass
// must decide it (a face whose closest point lies on its boundary). The minimum
// keeps the smallest (|d| bits, sign code, id).
constexpr uint32_t SIGN_POS = 0u, SIGN_NEG = 1u, SIGN_OPEN = 2u;
constexpr uint32_t ID_MASK = 0x3fffffffu;

struct I3 {
  int x, y, z;
};

struct Poly {
  float pl[5][4];   // inside: m . p + off >= -eps  (p relative to the anchor cell centre)
  float g[9];       // feature points relative to the anchor cell centre
  float cone[4];    // vertex: axis, aperture cosine (or -2 for a hemisphere); face: unit normal
  float side;       // +1 outward polyhedron, -1 inward (edges and vertices)
  I3 anc;           // anchor cell (lowest corner of the box)
  I3 dim;           // box extent in cells
  int ra, ua, va;   // row axis and the two axes across rows
  int nt, nu, nv;   // cells along ra, ua, va (resolved once: no runtime-indexed arrays)
  int id;           // global feature id
  int mesh;
  int wide;         // box longer than WIDE_CELLS along some axis: distances in FP64
  int absorbed;     // face: its absorbed edges (bits 0-2, from corner j) and vertices (bits 3-5)
};

// Local-frame FP32 distances carry a rounding error of about 1e-7 cells per cell
// of box extent (the feature points lie that far from the anchor); up to 32
// cells that stays near 3e-6 h, well inside the 1e-5 h tolerance. Polyhedra
// with a longer box go to the overflow pass, which computes their distances in
// FP64 from the feature's own coordinates and the cell centre.
constexpr int WIDE_CELLS = 32;

__device__ inline d3 vload_d(const float* V, int64_t i) {
  return mkd((double)V[3 * i], (double)V[3 * i + 1], (double)V[3 * i + 2]);
}

// unit vector of an FP64 direction, normalised in FP32 (plane normals only decide
// membership, which carries a slack of 1e-3 cells)
__device__ inline f3 unit_f(d3 v) {
  const f3 w = tof(v);
  const float l2 = dot(w, w);
  return l2 > 0.f ? w * __builtin_amdgcn_rsqf(l2) : mk(0.f, 0.f, 0.f);
}

// axis of the largest |component|
__device__ inline int major_axis(double x, double y, double z) {
  double ax = fabs(x), ay = fabs(y), az = fabs(z);
  return ax >= ay ? (ax >= az ? 0 : 2) : (ay >= az ? 1 : 2);
}
__device__ inline void set_axes(Poly& q, int ra) {
  q.ra = ra;
  q.ua = ra == 0 ? 1 : 0;
  q.va = ra == 2 ? 1 : 2;
  // arithmetic blends: a select over record fields would be turned into a load
  // from a selected address, which keeps the whole record in scratch memory
  q.nt = q.dim.x * (ra == 0) + q.dim.y * (ra == 1) + q.dim.z * (ra == 2);
  q.nu = q.dim.y * (ra == 0) + q.dim.x * (ra != 0);
  q.nv = q.dim.y * (ra == 2) + q.dim.z * (ra != 2);
}

// one axis of a box: first cell and number of cells whose centres lie in [lo, hi]
__device__ inline bool axis_cells(double lo, double hi, double o, double ih, int n, int& a0, int& cnt) {
  const double marg = 1e-4;
  double a = ceil((lo - o) * ih - 0.5 - marg), b = floor((hi - o) * ih - 0.5 + marg);
  if (a < 0) a = 0;
  if (b > n - 1) b = n - 1;
  if (!(a <= b)) return false;
  a0 = (int)a;
  cnt = (int)(b - a) + 1;
  return true;
}

// bounding box [lo, hi] (world) -> anchor and dimensions in cells; false if empty
__device__ inline bool box_cells(const MeshDesc& G, const double lo[3], const double hi[3], Poly& q) {
  return axis_cells(lo[0], hi[0], G.origin[0], G.inv_h, G.n[0], q.anc.x, q.dim.x) &&
         axis_cells(lo[1], hi[1], G.origin[1], G.inv_h, G.n[1], q.anc.y, q.dim.y) &&
         axis_cells(lo[2], hi[2], G.origin[2], G.inv_h, G.n[2], q.anc.z, q.dim.z);
}

__device__ inline d3 anchor_centre(const MeshDesc& G, const Poly& q) {
  return mkd(G.origin[0] + (q.anc.x + 0.5) * G.h, G.origin[1] + (q.anc.y + 0.5) * G.h,
             G.origin[2] + (q.anc.z + 0.5) * G.h);
}

__device__ inline void set_plane(Poly& q, int i, f3 m, f3 through) {
  q.pl[i][0] = m.x;
  q.pl[i][1] = m.y;
  q.pl[i][2] = m.z;
  q.pl[i][3] = -dot(m, through);
}

// Face prism (Section 8.1): three inward side planes through the edges and the two
// caps |n . (x - a)| <= band*h (both the outward and inward prism at once). The
// side planes move out by the largest slack of the absorbed edges and vertices
// of the face (the regions of those nearly flat features lie within it).
__device__ inline int build_face(const ScanArgs& P, const MeshDesc& G, int64_t f, Poly& q) {
  const FaceRec& R = P.frec[f];
  const float4 ra = R.c[0], rb = R.c[1], rc = R.c[2], nn = R.n;
  d3 a = mkd(ra.x, ra.y, ra.z), b = mkd(rb.x, rb.y, rb.z), c = mkd(rc.x, rc.y, rc.z);
  d3 n = mkd(nn.x, nn.y, nn.z);
  const float slack = (float)P.fslack[f] * (1.f / 1024.f) * G.hf;  // absorbed features' slack, length units
  double lo[3], hi[3];
  const double A3[3] = {a.x, a.y, a.z}, B3[3] = {b.x, b.y, b.z}, C3[3] = {c.x, c.y, c.z}, N3[3] = {n.x, n.y, n.z};
  for (int k = 0; k < 3; k++) {
    double r = G.whd * fabs(N3[k]) + G.epsd + (double)slack;
    lo[k] = fmin(A3[k], fmin(B3[k], C3[k])) - r;
    hi[k] = fmax(A3[k], fmax(B3[k], C3[k])) + r;
  }
  if (!box_cells(G, lo, hi, q)) return 0;
  d3 c0 = anchor_centre(G, q);
  f3 A = tof(a - c0), B = tof(b - c0), C = tof(c - c0), nf = mk(nn.x, nn.y, nn.z);
  const f3 W[3] = {A, B, C};
  for (int j = 0; j < 3; j++) {
    f3 m = cross(nf, W[(j + 1) % 3] - W[j]);
    set_plane(q, j, m * __builtin_amdgcn_rsqf(dot(m, m)), W[j]);
    q.pl[j][3] += slack;
  }
  float na = dot(nf, A);
  q.pl[3][0] = -nf.x; q.pl[3][1] = -nf.y; q.pl[3][2] = -nf.z; q.pl[3][3] = na + G.whf;
  q.pl[4][0] = nf.x;  q.pl[4][1] = nf.y;  q.pl[4][2] = nf.z;  q.pl[4][3] = G.whf - na;
  q.g[0] = A.x; q.g[1] = A.y; q.g[2] = A.z;
  q.g[3] = B.x; q.g[4] = B.y; q.g[5] = B.z;
  q.g[6] = C.x; q.g[7] = C.y; q.g[8] = C.z;
  q.cone[0] = nf.x; q.cone[1] = nf.y; q.cone[2] = nf.z;
  q.side = 1.f;
  q.id = (int)f;
  q.absorbed = P.fabsorbed[f];
  set_axes(q, major_axis(n.x, n.y, n.z));
  return q.dim.x * q.dim.y * q.dim.z;
}

// Edge wedge (Section 8.2): the dihedral region spanned by the two face normals
// (outward side) or their negatives (inward side), between the end caps, cut by
// the base plane through the edge with the summed normal (Section 8.2); the far
// side is the band distance itself (cells with |d| >= band*h are dropped).
__device__ inline int build_edge(const ScanArgs& P, const MeshDesc& G, int32_t ent, Poly& q) {
  int64_t e = ent >> 1;
  double sg = (ent & 1) ? -1.0 : 1.0;
  int4 E = P.edges[e];
  d3 a = vload_d(P.V, E.x), b = vload_d(P.V, E.y);
  float4 f1 = P.frec[E.z].n, f2 = P.frec[E.w].n;
  d3 n1 = mkd(f1.x, f1.y, f1.z), n2 = mkd(f2.x, f2.y, f2.z);
  d3 ed = b - a;
  int cls = P.ecls[e] & 3;
  double kap;
  if (cls == EDGE_CONVEX) kap = 1.0;
  else if (cls == EDGE_CONCAVE) kap = -1.0;
  else kap = dot(ed, cross(n1, n2)) < 0 ? -1.0 : 1.0;
  d3 u1 = n1 * sg, u2 = n2 * sg, us = u1 + u2;
  double us2 = dot(us, us);
  const double U1[3] = {u1.x, u1.y, u1.z}, U2[3] = {u2.x, u2.y, u2.z}, US[3] = {us.x, us.y, us.z};
  const double A3[3] = {a.x, a.y, a.z}, B3[3] = {b.x, b.y, b.z};
  double lo[3], hi[3];
  const double tsc = us2 > 1e-12 ? 2.0 * G.whd / us2 : 0.0;
  for (int k = 0; k < 3; k++) {
    double x1 = G.whd * U1[k], x2 = G.whd * U2[k];
    double alo = fmin(0.0, fmin(x1, x2)), ahi = fmax(0.0, fmax(x1, x2));
    if (us2 > 1e-12) {  // the arc lies inside the quadrilateral through the tangent intersection
      double t = US[k] * tsc;
      alo = fmin(alo, t);
      ahi = fmax(ahi, t);
    } else {
      alo = -G.whd;
      ahi = G.whd;
    }
    alo = fmax(alo, -G.whd);
    ahi = fmin(ahi, G.whd);
    lo[k] = fmin(A3[k], B3[k]) + alo - G.epsd;
    hi[k] = fmax(A3[k], B3[k]) + ahi + G.epsd;
  }
  if (!box_cells(G, lo, hi, q)) return 0;
  d3 c0 = anchor_centre(G, q);
  f3 A = tof(a - c0), B = tof(b - c0);
  set_plane(q, 0, unit_f(cross(ed, n1) * (sg * kap)), A);
  set_plane(q, 1, unit_f(cross(n2, ed) * (sg * kap)), A);
  f3 eh = unit_f(ed);
  set_plane(q, 2, eh, A);
  set_plane(q, 3, eh * -1.f, B);
  if (us2 > 1e-18) set_plane(q, 4, unit_f(us), A);
  else { q.pl[4][0] = 0; q.pl[4][1] = 0; q.pl[4][2] = 0; q.pl[4][3] = 0; }
  q.g[0] = A.x; q.g[1] = A.y; q.g[2] = A.z;
  q.g[3] = B.x; q.g[4] = B.y; q.g[5] = B.z;
  q.side = (float)sg;
  q.id = (int)(P.nf + e);
  q.absorbed = 0;
  set_axes(q, us2 > 1e-12 ? major_axis(us.x, us.y, us.z) : major_axis(ed.x, ed.y, ed.z));
  return q.dim.x * q.dim.y * q.dim.z;
}

// Vertex cone (Section 4.2, Section 8.3) about the (possibly reflected)
// pseudonormal with the most diverging positive-pointing normal on its side, or a
// hemisphere (Section 4.1.3); box = cone box intersected with the sphere box.
__device__ inline int build_vertex(const ScanArgs& P, const MeshDesc& G, int32_t ent, Poly& q) {
  int64_t v = ent >> 1;
  double sg = (ent & 1) ? -1.0 : 1.0;
  float4 vi = P.vinfo[v];
  uint32_t bits = P.vbits[v];
  bool hemi = (ent & 1) ? (bits & V_NEG_HEMI) : (bits & V_POS_HEMI);
  double ct = vi.w;
  if (!(ct > 0)) hemi = true;
  d3 ax = mkd(vi.x * sg, vi.y * sg, vi.z * sg);
  d3 p = vload_d(P.V, v);
  const double AX[3] = {ax.x, ax.y, ax.z}, P3[3] = {p.x, p.y, p.z};
  // box of the cone: FP32 suffices (a relative error near 1e-7 of band*h, far
  // inside the eps margin the box is grown by); a cone opening to nearly 90
  // degrees gets the box of its hemisphere, which contains it
  const float ctf = (float)ct;
  const bool wide = hemi || !(ctf > 1e-6f);
  double tn = wide ? 0.0 : (double)(sqrtf(fmaxf(0.f, 1.f - ctf * ctf)) * __builtin_amdgcn_rcpf(ctf));
  double lo[3], hi[3];
  for (int k = 0; k < 3; k++) {
    const float axk = (float)AX[k];
    double s = (double)sqrtf(fmaxf(0.f, 1.f - axk * axk));
    double l, u;
    if (wide) {
      l = AX[k] > 0 ? -G.whd * s : -G.whd;
      u = AX[k] < 0 ? G.whd * s : G.whd;
    } else {
      l = fmax(-G.whd, fmin(0.0, G.whd * (AX[k] - tn * s)));
      u = fmin(G.whd, fmax(0.0, G.whd * (AX[k] + tn * s)));
    }
    lo[k] = P3[k] + l - G.epsd;
    hi[k] = P3[k] + u + G.epsd;
  }
  if (!box_cells(G, lo, hi, q)) return 0;
  d3 c0 = anchor_centre(G, q);
  f3 A = tof(p - c0), axf = tof(ax);
  set_plane(q, 0, axf, A);
  q.cone[0] = axf.x; q.cone[1] = axf.y; q.cone[2] = axf.z;
  q.cone[3] = hemi ? -2.f : vi.w;
  q.g[0] = A.x; q.g[1] = A.y; q.g[2] = A.z;
  q.side = (float)sg;
  q.id = (int)(P.nf + P.ne + v);
  q.absorbed = 0;
  set_axes(q, major_axis(ax.x, ax.y, ax.z));
  return q.dim.x * q.dim.y * q.dim.z;
}

template <int KIND>
__device__ inline int build_poly(const ScanArgs& P, int64_t item, Poly& q) {
  int nc;
  if constexpr (KIND == KIND_FACE) {
    const int64_t f = P.items ? P.items[item] : item;  // the face order, if one is set
    q.mesh = P.face_mesh[f];
    nc = build_face(P, P.md[q.mesh], f, q);
  } else if constexpr (KIND == KIND_EDGE) {
    const int32_t ent = P.items[item];
    q.mesh = P.face_mesh[P.edges[ent >> 1].z];
    nc = build_edge(P, P.md[q.mesh], ent, q);
  } else {
    const int32_t ent = P.items[item];
    q.mesh = P.vert_mesh[ent >> 1];
    nc = build_vertex(P, P.md[q.mesh], ent, q);
  }
  q.wide = nc > 0 && max(q.dim.x, max(q.dim.y, q.dim.z)) > WIDE_CELLS;
  return nc;
}

__device__ inline int lanes_below(unsigned long long m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// component a of (x, y, z) by value (taking an array's address would force the
// polyhedron record out of registers)
__device__ inline float pick3(float x, float y, float z, int a) {
  return x * (float)(a == 0) + y * (float)(a == 1) + z * (float)(a == 2);
}

// Per-plane coefficients along a row: the slack-extended test m . p + off >= -eps at
// cell (t, du, dv) of the row reads  sl * t + su * du + sv * dv + k >= 0.
struct Rows {
  float sl[5], inv[5], su[5], sv[5], k[5];
  float A[3];       // vertex position (ball test)
  float R2;         // (band*h + eps)^2
  float hf, ihf, eps;  // cell size, its inverse and the slack of the polyhedron's grid
  int nt;           // cells along the row
};

template <int KIND, bool WIDE>
__device__ inline void setup_rows(const Poly& q, const MeshDesc& G, Rows& r) {
  constexpr int NPL = KIND == KIND_VERT ? 1 : 5;
  // a wide polyhedron's planes are rounded at the size of its box: its slack
  // grows by 1e-6 h per cell of extent (several times that rounding)
  const float eps = WIDE ? G.eps + 1e-6f * G.hf * (float)max(q.dim.x, max(q.dim.y, q.dim.z)) : G.eps;
#pragma unroll
  for (int i = 0; i < NPL; i++) {
    r.sl[i] = pick3(q.pl[i][0], q.pl[i][1], q.pl[i][2], q.ra) * G.hf;
    r.inv[i] = fabsf(r.sl[i]) > 1e-20f ? __builtin_amdgcn_rcpf(r.sl[i]) : 0.f;
    r.su[i] = pick3(q.pl[i][0], q.pl[i][1], q.pl[i][2], q.ua) * G.hf;
    r.sv[i] = pick3(q.pl[i][0], q.pl[i][1], q.pl[i][2], q.va) * G.hf;
    r.k[i] = q.pl[i][3] + eps;
  }
  r.A[0] = pick3(q.g[0], q.g[1], q.g[2], q.ra);
  r.A[1] = pick3(q.g[0], q.g[1], q.g[2], q.ua);
  r.A[2] = pick3(q.g[0], q.g[1], q.g[2], q.va);
  r.R2 = (G.whf + G.eps) * (G.whf + G.eps);
  r.hf = G.hf;
  r.ihf = (float)G.inv_h;
  r.eps = eps;
  r.nt = q.nt;
}

// cells [t0, t1] of row (du, dv) that can lie in the polyhedron (conservative)
template <int KIND>
__device__ inline bool row_range(const Rows& r, int du, int dv, int& t0, int& t1) {
  const float hf = r.hf;
  constexpr int NPL = KIND == KIND_VERT ? 1 : 5;
  float lo = 0.f, hi = (float)(r.nt - 1);
  bool dead = false;  // a plane parallel to the row with the row outside it
  // selects, not branches: every lane takes the same instructions
#pragma unroll
  for (int i = 0; i < NPL; i++) {
    const float v = r.su[i] * du + r.sv[i] * dv + r.k[i];
    const float x = -v * r.inv[i];
    lo = fmaxf(lo, r.inv[i] > 0.f ? x : -__builtin_inff());
    hi = fminf(hi, r.inv[i] < 0.f ? x : __builtin_inff());
    dead = dead || (r.inv[i] == 0.f && v < 0.f);
  }
  if (dead) return false;
  if constexpr (KIND == KIND_VERT) {  // the ball |p - v| < band*h (+ slack)
    const float qu = du * hf - r.A[1], qv = dv * hf - r.A[2];
    const float disc = r.R2 - qu * qu - qv * qv;
    if (disc < 0.f) return false;
    const float w = sqrtf(disc) * r.ihf, c = r.A[0] * r.ihf;
    lo = fmaxf(lo, c - w);
    hi = fminf(hi, c + w);
  }
  // the bounds carry relative rounding far below 1e-4 cells
  t0 = max(0, (int)ceilf(lo - 1e-4f));
  t1 = min(r.nt - 1, (int)floorf(hi + 1e-4f));
  return t0 <= t1;
}

// the brick slot of the last brick looked up (consecutive candidates of a lane
// mostly share a brick)
struct BrickCache {
  int64_t bl = -1;
  int32_t slot = -1;
};

// Candidate cells of a wavefront's polyhedra pass through a small ring in LDS:
// each lane searches the rows of its own polyhedron (cheap interval tests) and
// appends the cells it finds; every 64 queued candidates are then finished with
// all 64 lanes busy, each lane fetching the owning lane's polyhedron by lane
// permutation. This keeps the exact distance and the atomic, the expensive part,
// free of the imbalance between polyhedra of very different sizes.
constexpr int QCAP = 128;  // < 64 left after each drain, plus at most 64 appended per round

__device__ inline unsigned long long pack_cand(int lane, int t, int du, int dv) {
  return ((unsigned long long)lane << 48) | ((unsigned long long)t << 32) | ((unsigned long long)du << 16) |
         (unsigned long long)dv;
}

// a value of the polyhedron held by lane L. With UNI every lane holds the same
// polyhedron (the overflow pass): the value is read from the first active lane,
// a scalar broadcast instead of an LDS permutation. (Taking the lane's own value
// directly would let the compiler fuse the setup arithmetic into the distance
// arithmetic and round differently from the one-lane-per-polyhedron pass.)
__device__ inline int first_lane(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline float first_lane(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }

template <bool UNI, typename T>
__device__ inline T from_lane(T x, int L) {
  if constexpr (UNI) return first_lane(x);
  else return __shfl(x, L, 64);
}

// Distance and sign code of cell (i, j, k) to the feature of a wide polyhedron
// (global id), in FP64 relative to the cell centre: the feature's corners are
// read again from the face and vertex arrays. The sign is always decided here,
// with the pseudonormal of the feature holding the closest point (Section
// 4.1.3), so that it stays right next to the surface however far the corners
// lie. False when the cell lies outside the band.
template <int KIND>
__device__ inline bool dist_wide(const ScanArgs& P, const MeshDesc& G, int id, int i, int j, int k, float& d,
                                 uint32_t& code) {
  const d3 c = mkd(G.origin[0] + (i + 0.5) * G.h, G.origin[1] + (j + 0.5) * G.h, G.origin[2] + (k + 0.5) * G.h);
  const d3 o = mkd(0.0, 0.0, 0.0);
  double dd;
  if constexpr (KIND == KIND_FACE) {
    const FaceRec& R = P.frec[id];
    const float4 ra = R.c[0], rb = R.c[1], rc = R.c[2];
    d3 qq;
    double w[3];
    const int region = closest_triangle_t<d3, double>(o, mkd(ra.x, ra.y, ra.z) - c, mkd(rb.x, rb.y, rb.z) - c,
                                                      mkd(rc.x, rc.y, rc.z) - c, qq, w);
    dd = len(qq);
    float4 n4;
    if (region == 0) {
      n4 = R.n;
    } else if (region <= 3) {
      const int4 E = P.edges[P.face_edges[3 * (int64_t)id + region - 1]];
      const float4 f1 = P.frec[E.z].n, f2 = P.frec[E.w].n;
      n4 = make_float4(f1.x + f2.x, f1.y + f2.y, f1.z + f2.z, 0.f);
    } else {
      n4 = P.vinfo[P.T[3 * (int64_t)id + region - 4]];
    }
    // (c - q) . N >= 0: outside
    code = dot(qq, mkd(n4.x, n4.y, n4.z)) <= 0.0 ? SIGN_POS : SIGN_NEG;
  } else if constexpr (KIND == KIND_EDGE) {
    const int4 E = P.edges[id - P.nf];
    double tt;
    const d3 qq = closest_segment_t<d3, double>(o, vload_d(P.V, E.x) - c, vload_d(P.V, E.y) - c, tt);
    dd = len(qq);
    d3 N;
    if (tt <= 0.0 || tt >= 1.0) {
      const float4 vi = P.vinfo[tt <= 0.0 ? E.x : E.y];
      N = mkd(vi.x, vi.y, vi.z);
    } else {
      const float4 f1 = P.frec[E.z].n, f2 = P.frec[E.w].n;
      N = mkd((double)f1.x + f2.x, (double)f1.y + f2.y, (double)f1.z + f2.z);
    }
    code = dot(qq, N) <= 0.0 ? SIGN_POS : SIGN_NEG;
  } else {
    const int64_t v = id - P.nf - P.ne;
    const d3 qq = vload_d(P.V, v) - c;
    dd = len(qq);
    const float4 vi = P.vinfo[v];
    code = dot(qq, mkd(vi.x, vi.y, vi.z)) <= 0.0 ? SIGN_POS : SIGN_NEG;
  }
  d = (float)dd;
  return dd < G.whd;
}

// diagnostics: the lanes about to issue one atomicMin instruction record it as a
// round of the log (index and lane mask)
__device__ inline void log_atomic(const ScanArgs& P, uint32_t at) {
  const unsigned long long m = __ballot(true);
  const int lane = threadIdx.x & 63, leader = __ffsll((long long)m) - 1;
  unsigned r = 0;
  if (lane == leader) r = atomicAdd(P.log_rounds, 1u);
  r = __shfl(r, leader, 64);
  if ((int64_t)r < P.log_cap) {
    P.log[(int64_t)r * 64 + lane] = at;
    if (lane == leader) P.log_mask[r] = m;
  }
}

// exact distance of one queued candidate and its packed atomic minimum; called by
// all lanes of the wavefront together (lane permutations), `valid` per lane.
// WIDE (overflow pass only): the distance in FP64 (dist_wide). LOG: record the
// atomic instruction (diagnostic instantiation).
template <int KIND, bool UNI, bool WIDE, bool LOG>
__device__ inline void finish_cand(const ScanArgs& P, const Poly& q, unsigned long long ent, bool valid,
                                   BrickCache& bc, unsigned& issued) {
  const int L = valid ? (int)(ent >> 48) : 0;
  const int t = (int)((ent >> 32) & 0xffff), du = (int)((ent >> 16) & 0xffff), dv = (int)(ent & 0xffff);
  const int mesh = from_lane<UNI>(q.mesh, L), id = from_lane<UNI>(q.id, L);
  // row axes, with the face's absorbed features above them (one lane move).
  // Every pass decides the same cells: the packed key orders equal distances by
  // sign code before feature id, so a face whose boundary cell one pass decided
  // and another left open would win or lose a tie by schedule.
  const int axes = from_lane<UNI>(q.ra | (q.ua << 2) | (q.absorbed << 4), L);
  const int ax = from_lane<UNI>(q.anc.x, L), ay = from_lane<UNI>(q.anc.y, L), az = from_lane<UNI>(q.anc.z, L);
  const f3 g0 = mk(from_lane<UNI>(q.g[0], L), from_lane<UNI>(q.g[1], L), from_lane<UNI>(q.g[2], L));
  f3 g1 = mk(0.f, 0.f, 0.f), g2 = mk(0.f, 0.f, 0.f), nn = mk(0.f, 0.f, 0.f);
  float side = 1.f;
  if constexpr (KIND == KIND_FACE) {
    g1 = mk(from_lane<UNI>(q.g[3], L), from_lane<UNI>(q.g[4], L), from_lane<UNI>(q.g[5], L));
    g2 = mk(from_lane<UNI>(q.g[6], L), from_lane<UNI>(q.g[7], L), from_lane<UNI>(q.g[8], L));
    nn = mk(from_lane<UNI>(q.cone[0], L), from_lane<UNI>(q.cone[1], L), from_lane<UNI>(q.cone[2], L));
  } else if constexpr (KIND == KIND_EDGE) {
    g1 = mk(from_lane<UNI>(q.g[3], L), from_lane<UNI>(q.g[4], L), from_lane<UNI>(q.g[5], L));
    nn = mk(from_lane<UNI>(q.pl[4][0], L), from_lane<UNI>(q.pl[4][1], L), from_lane<UNI>(q.pl[4][2], L));
    side = from_lane<UNI>(q.side, L);
  } else {
    nn = mk(from_lane<UNI>(q.cone[0], L), from_lane<UNI>(q.cone[1], L), from_lane<UNI>(q.cone[2], L));
    side = from_lane<UNI>(q.side, L);
  }
  if (!valid) return;
  const MeshDesc& G = P.md[mesh];
  const int ra = axes & 3, ua = (axes >> 2) & 3;
  const int di = ra == 0 ? t : (ua == 0 ? du : dv);
  const int dj = ra == 1 ? t : (ua == 1 ? du : dv);
  const int dk = ra == 2 ? t : (ua == 2 ? du : dv);
  const int i = ax + di, j = ay + dj, k = az + dk;
  float d;
  uint32_t code;
  if constexpr (WIDE) {
    if (!dist_wide<KIND>(P, G, id, i, j, k, d, code)) return;
  } else {
  const float hf = G.hf;
  const f3 p = mk(di * hf, dj * hf, dk * hf);
  if constexpr (KIND == KIND_FACE) {
    f3 qq;
    float w[3];
    const int region = closest_triangle(p, g0, g1, g2, qq, w);
    d = norm3(p - qq);
    // Interior closest point: the face normal is the pseudonormal. On the
    // boundary, at an absorbed edge or vertex (region r: edge from corner r - 1,
    // or corner r - 4; bit r - 1 either way), the face normal gives the same
    // sign: such a cell sees the feature along a direction within 90 degrees of
    // every incident face normal (the absorption bound, an angle under 45
    // degrees, at most doubled), so its dot products with the face normal and
    // with the feature's pseudonormal share their sign. Other boundary points
    // are left to the sign pass.
    const bool own = region == 0 || ((axes >> (3 + region)) & 1);
    code = !own ? SIGN_OPEN : (dot(p - qq, nn) >= 0.f ? SIGN_POS : SIGN_NEG);
  } else if constexpr (KIND == KIND_EDGE) {
    float tt;
    const f3 qq = closest_segment(p, g0, g1, tt);
    d = norm3(p - qq);
    // interior of the edge: pseudonormal n1 + n2 = side * (base plane normal) * |n1 + n2|
    const bool ok = tt > 0.f && tt < 1.f && dot(nn, nn) > 0.f;
    code = !ok ? SIGN_OPEN : (dot(p - qq, nn) * side >= 0.f ? SIGN_POS : SIGN_NEG);
  } else {
    const f3 rr = p - g0;
    d = norm3(rr);
    // the vertex itself: its angle-weighted pseudonormal (axis = side * N)
    code = dot(rr, nn) * side >= 0.f ? SIGN_POS : SIGN_NEG;
  }
  if (!(d < G.whf)) return;
  }
  const int64_t bl = brick_pos(G, i >> BRICK_SHIFT, j >> BRICK_SHIFT, k >> BRICK_SHIFT);
  if (bl != bc.bl) {
    bc.bl = bl;
    bc.slot = P.brick_index[bl];
  }
  const int32_t slot = bc.slot;
  if (slot >= 0 && slot < P.cap) {
    const unsigned long long key = ((unsigned long long)__float_as_uint(d) << 32) | (code << 30) | (uint32_t)id;
    const int64_t at = (int64_t)slot * BRICK_CELLS + brick_local(i, j, k);
    if constexpr (LOG) log_atomic(P, (uint32_t)at);
    atomicMin(&P.keys[at], key);
    issued++;
  } else if (slot >= P.cap) {
    atomicOr((uint32_t*)&P.stats[ST_ERR], ERR_OVERFLOW);
  }
}


// the row coefficients of the polyhedron held by lane L, fetched by lane
// permutation (with the row-axis slopes when each cell is tested on its own);
// called by all lanes together
template <int KIND, bool UNI>
__device__ inline Rows rows_of(const Rows& r, int L, bool per_cell) {
  constexpr int NPL = KIND == KIND_VERT ? 1 : 5;
  Rows o;
#pragma unroll
  for (int i = 0; i < NPL; i++) {
    o.inv[i] = from_lane<UNI>(r.inv[i], L);
    o.su[i] = from_lane<UNI>(r.su[i], L);
    o.sv[i] = from_lane<UNI>(r.sv[i], L);
    o.k[i] = from_lane<UNI>(r.k[i], L);
  }
  if (per_cell) {
#pragma unroll
    for (int i = 0; i < NPL; i++) o.sl[i] = from_lane<UNI>(r.sl[i], L);
  }
  o.nt = from_lane<UNI>(r.nt, L);
  if constexpr (KIND == KIND_VERT) {
    o.A[0] = from_lane<UNI>(r.A[0], L);
    o.A[1] = from_lane<UNI>(r.A[1], L);
    o.A[2] = from_lane<UNI>(r.A[2], L);
    o.R2 = from_lane<UNI>(r.R2, L);
    o.hf = from_lane<UNI>(r.hf, L);
    o.ihf = from_lane<UNI>(r.ihf, L);
  }
  return o;
}

// Alg. 2 for one cell: every half-space with slack (and, for vertices, the
// ball of radius band*h); the per-cell alternative to the row interval
template <int KIND>
__device__ inline bool cell_in(const Rows& o, int t, int du, int dv) {
  constexpr int NPL = KIND == KIND_VERT ? 1 : 5;
  bool in = true;
#pragma unroll
  for (int i = 0; i < NPL; i++) in = in && o.sl[i] * t + o.su[i] * du + o.sv[i] * dv + o.k[i] >= 0.f;
  if constexpr (KIND == KIND_VERT) {
    const float qt = t * o.hf - o.A[0], qu = du * o.hf - o.A[1], qv = dv * o.hf - o.A[2];
    in = in && qt * qt + qu * qu + qv * qv <= o.R2;
  }
  return in;
}

// The rows of the wavefront's polyhedra (lane l holds `rows` rows of its own
// polyhedron q) are dealt out evenly: in each round lane j takes the j-th next
// row of the whole wavefront, finds the lane owning it (binary search over the
// prefix sums of the row counts), computes its interval with the owner's
// coefficients, and queues its candidate cells in ring `qb` (this wavefront's
// own) under the owner's lane number. Lanes with many rows thus no longer hold
// up the others. Must be called by all lanes of the wavefront.
template <int KIND, bool UNI, bool WIDE, bool LOG>
__device__ inline void scan_rows_wave(const ScanArgs& P, const Poly& q, const Rows& r, int rows, int row0,
                                      unsigned long long* qb, unsigned& issued) {
  const int lane = threadIdx.x & 63;
  const int incl = wave_prefix_sum(rows), excl = incl - rows;
  const int total = __builtin_amdgcn_readlane(incl, 63);
  uint32_t head = 0, tail = 0;  // the same in every lane
  BrickCache bc;
  for (int base = 0; base < total; base += 64) {
    const int g = base + lane;
    int lo = 0, hi = 63;  // the last lane whose rows start at or before g
    if constexpr (!UNI) {
#pragma unroll
      for (int s = 0; s < 6; s++) {
        const int mid = (lo + hi + 1) >> 1;
        if (__shfl(excl, mid, 64) <= g) lo = mid;
        else hi = mid - 1;
      }
    }
    const int L = lo;  // with UNI lane 0 owns every row
    const int rloc = UNI ? row0 + g : g - __shfl(excl, L, 64), nuL = from_lane<UNI>(q.nu, L);
    const int nud = nuL > 0 ? nuL : 1;  // past the last row L may hold no polyhedron
    const int dv = g < total ? rloc / nud : 0, du = g < total ? rloc - dv * nud : 0;
    int t = 0, t1 = -1;
    const Rows o = rows_of<KIND, UNI>(r, L, P.per_cell);
    if (P.per_cell) {  // every cell of the row, each tested by itself below
      t = 0;
      t1 = o.nt - 1;
    } else if (!row_range<KIND>(o, du, dv, t, t1)) {
      t1 = -1;
    }
    if (g >= total) t1 = -1;
    // vertices: the owner's cone for the per-cell discriminant
    [[maybe_unused]] f3 cg = mk(0.f, 0.f, 0.f), cax = mk(0.f, 0.f, 0.f);
    [[maybe_unused]] float cct = -2.f, chf = 0.f, ceps = 0.f;
    [[maybe_unused]] int cra = 0, cua = 0;
    if constexpr (KIND == KIND_VERT) {
      cg = mk(from_lane<UNI>(q.g[0], L), from_lane<UNI>(q.g[1], L), from_lane<UNI>(q.g[2], L));
      cax = mk(from_lane<UNI>(q.cone[0], L), from_lane<UNI>(q.cone[1], L), from_lane<UNI>(q.cone[2], L));
      cct = from_lane<UNI>(q.cone[3], L);
      chf = from_lane<UNI>(r.hf, L);
      ceps = from_lane<UNI>(r.eps, L);
      const int ax = from_lane<UNI>(q.ra | (q.ua << 2), L);
      cra = ax & 3;
      cua = (ax >> 2) & 3;
    }
    while (true) {
      const bool has = t <= t1;
      if (__ballot(has) == 0) break;
      bool push = has && (!P.per_cell || cell_in<KIND>(o, t, du, dv));
      if constexpr (KIND == KIND_VERT) {  // cone discriminant with slack (Eq. 10)
        if (push && cct > -1.f) {
          const int di = cra == 0 ? t : (cua == 0 ? du : dv);
          const int dj = cra == 1 ? t : (cua == 1 ? du : dv);
          const int dk = cra == 2 ? t : (cua == 2 ? du : dv);
          const f3 rr = mk(di * chf, dj * chf, dk * chf) - cg;
          const float te = dot(rr, cax) + ceps;
          push = te >= 0.f && te * te >= cct * cct * dot(rr, rr);
        }
      }
      const unsigned long long pm = __ballot(push);
      if (push) qb[(tail + lanes_below(pm)) & (QCAP - 1)] = pack_cand(L, t, du, dv);
      tail += (uint32_t)__popcll(pm);
      if (has) t++;
      if (tail - head >= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const unsigned long long e = qb[(head + lane) & (QCAP - 1)];
        finish_cand<KIND, UNI, WIDE, LOG>(P, q, e, true, bc, issued);
        head += 64;
      }
    }
  }
  if (tail != head) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool valid = (uint32_t)lane < tail - head;
    const unsigned long long e = valid ? qb[(head + lane) & (QCAP - 1)] : 0ull;
    finish_cand<KIND, UNI, WIDE, LOG>(P, q, e, valid, bc, issued);
  }
  // the ring is reused by the next call: finish its reads first
  __builtin_amdgcn_wave_barrier();
}

// The row coefficients of every lane's polyhedron, staged in LDS for the
// one-polyhedron-per-lane pass so that the lane taking a row reads its owner's
// with a few 16-byte loads: faces and edges inv, su, sv, k, sl of their five
// planes, then nt, the owner's first row in the wavefront's numbering and nu;
// vertices the same for their one plane, then the ball and cone data in (row,
// u, v) order.
template <int KIND>
struct RowSlot {
  static constexpr int F4 = KIND == KIND_VERT ? 5 : 7;  // float4 per lane
};

struct RowsOf {
  Rows o;
  int excl, nu;
  f3 cax;       // vertices: cone axis in (row, u, v) order
  float cct;    // vertices: aperture cosine, or below -1 for a hemisphere
};

template <int KIND>
__device__ inline void put_slot(float4* sl, const Rows& r, const Poly& q, int excl) {
  if constexpr (KIND != KIND_VERT) {
    sl[0] = make_float4(r.inv[0], r.inv[1], r.inv[2], r.inv[3]);
    sl[1] = make_float4(r.inv[4], r.su[0], r.su[1], r.su[2]);
    sl[2] = make_float4(r.su[3], r.su[4], r.sv[0], r.sv[1]);
    sl[3] = make_float4(r.sv[2], r.sv[3], r.sv[4], r.k[0]);
    sl[4] = make_float4(r.k[1], r.k[2], r.k[3], r.k[4]);
    sl[5] = make_float4(r.sl[0], r.sl[1], r.sl[2], r.sl[3]);
    sl[6] = make_float4(r.sl[4], __int_as_float(r.nt), __int_as_float(excl), __int_as_float(q.nu));
  } else {
    sl[0] = make_float4(r.inv[0], r.su[0], r.sv[0], r.k[0]);
    sl[1] = make_float4(r.sl[0], __int_as_float(r.nt), __int_as_float(excl), __int_as_float(q.nu));
    sl[2] = make_float4(r.A[0], r.A[1], r.A[2], r.R2);
    sl[3] = make_float4(r.hf, r.ihf, r.eps, q.cone[3]);
    sl[4] = make_float4(pick3(q.cone[0], q.cone[1], q.cone[2], q.ra), pick3(q.cone[0], q.cone[1], q.cone[2], q.ua),
                        pick3(q.cone[0], q.cone[1], q.cone[2], q.va), 0.f);
  }
}

template <int KIND>
__device__ inline RowsOf get_slot(const float4* sl) {
  RowsOf w;
  if constexpr (KIND != KIND_VERT) {
    const float4 a = sl[0], b = sl[1], c = sl[2], d = sl[3], e = sl[4], f = sl[5], g = sl[6];
    w.o.inv[0] = a.x; w.o.inv[1] = a.y; w.o.inv[2] = a.z; w.o.inv[3] = a.w; w.o.inv[4] = b.x;
    w.o.su[0] = b.y; w.o.su[1] = b.z; w.o.su[2] = b.w; w.o.su[3] = c.x; w.o.su[4] = c.y;
    w.o.sv[0] = c.z; w.o.sv[1] = c.w; w.o.sv[2] = d.x; w.o.sv[3] = d.y; w.o.sv[4] = d.z;
    w.o.k[0] = d.w; w.o.k[1] = e.x; w.o.k[2] = e.y; w.o.k[3] = e.z; w.o.k[4] = e.w;
    w.o.sl[0] = f.x; w.o.sl[1] = f.y; w.o.sl[2] = f.z; w.o.sl[3] = f.w; w.o.sl[4] = g.x;
    w.o.nt = __float_as_int(g.y);
    w.excl = __float_as_int(g.z);
    w.nu = __float_as_int(g.w);
    w.cct = -2.f;
  } else {
    const float4 a = sl[0], b = sl[1], c = sl[2], d = sl[3], e = sl[4];
    w.o.inv[0] = a.x; w.o.su[0] = a.y; w.o.sv[0] = a.z; w.o.k[0] = a.w;
    w.o.sl[0] = b.x;
    w.o.nt = __float_as_int(b.y);
    w.excl = __float_as_int(b.z);
    w.nu = __float_as_int(b.w);
    w.o.A[0] = c.x; w.o.A[1] = c.y; w.o.A[2] = c.z; w.o.R2 = c.w;
    w.o.hf = d.x; w.o.ihf = d.y; w.o.eps = d.z; w.cct = d.w;
    w.cax = mk(e.x, e.y, e.z);
  }
  return w;
}

// The one-polyhedron-per-lane pass: the rows of the wavefront's polyhedra (lane
// l holds `rows` rows of its own polyhedron q, coefficients r) are dealt out
// evenly, 64 per round, lane j taking the j-th. The owner of each row: every
// lane marks the round position where its rows start, and a prefix maximum over
// the positions (carrying the owner of the round's first row) gives the last
// start at or before each. The lane computes the row's interval from the
// owner's staged coefficients and queues its candidate cells in the
// wavefront's ring under the owner's lane number; every 64 queued cells are
// finished by all lanes together. Must be called by all lanes of the wavefront.
template <int KIND, bool LOG>
__device__ inline void scan_rows_lanes(const ScanArgs& P, const Poly& q, const Rows& r, int rows, float4* slots,
                                       int* marks, unsigned long long* qb, unsigned& issued) {
  constexpr int F4 = RowSlot<KIND>::F4;
  const int lane = threadIdx.x & 63;
  const int incl = wave_prefix_sum(rows), excl = incl - rows;
  const int total = __builtin_amdgcn_readlane(incl, 63);
  if (rows > 0) put_slot<KIND>(slots + lane * F4, r, q, excl);
  uint32_t head = 0, tail = 0;  // the same in every lane
  BrickCache bc;
  int carry = 0;
  for (int base = 0; base < total; base += 64) {
    marks[lane] = -1;
    wave_sync_lds();
    const int s0 = excl - base;
    if (rows > 0 && s0 >= 0 && s0 < 64) marks[s0] = lane;
    wave_sync_lds();
    const int L = wave_prefix_max(max(marks[lane], carry));
    carry = __builtin_amdgcn_readlane(L, 63);
    const int g = base + lane;
    const RowsOf w = get_slot<KIND>(slots + L * F4);
    const int rloc = g - w.excl;
    const int nud = w.nu > 0 ? w.nu : 1;
    const int dv = g < total ? rloc / nud : 0, du = g < total ? rloc - dv * nud : 0;
    int t = 0, t1 = -1;
    if (P.per_cell) {  // every cell of the row, each tested by itself below
      t = 0;
      t1 = w.o.nt - 1;
    } else if (!row_range<KIND>(w.o, du, dv, t, t1)) {
      t1 = -1;
    }
    if (g >= total) t1 = -1;
    while (true) {
      const bool has = t <= t1;
      if (__ballot(has) == 0) break;
      bool push = has && (!P.per_cell || cell_in<KIND>(w.o, t, du, dv));
      if constexpr (KIND == KIND_VERT) {  // cone discriminant with slack (Eq. 10)
        if (push && w.cct > -1.f) {
          const f3 rr = mk(t * w.o.hf - w.o.A[0], du * w.o.hf - w.o.A[1], dv * w.o.hf - w.o.A[2]);
          const float te = dot(rr, w.cax) + w.o.eps;
          push = te >= 0.f && te * te >= w.cct * w.cct * dot(rr, rr);
        }
      }
      const unsigned long long pm = __ballot(push);
      if (push) qb[(tail + lanes_below(pm)) & (QCAP - 1)] = pack_cand(L, t, du, dv);
      tail += (uint32_t)__popcll(pm);
      if (has) t++;
      if (tail - head >= 64) {
        wave_sync_lds();
        const unsigned long long e = qb[(head + lane) & (QCAP - 1)];
        finish_cand<KIND, false, false, LOG>(P, q, e, true, bc, issued);
        head += 64;
      }
    }
  }
  if (tail != head) {
    wave_sync_lds();
    const bool valid = (uint32_t)lane < tail - head;
    const unsigned long long e = valid ? qb[(head + lane) & (QCAP - 1)] : 0ull;
    finish_cand<KIND, false, false, LOG>(P, q, e, valid, bc, issued);
  }
  // the ring, slots and marks are reused by the next call: finish the reads first
  __builtin_amdgcn_wave_barrier();
}

// counter[0] counts the one-thread-per-polyhedron launch, counter[3] the overflow launch
__device__ inline void add_issued(const ScanArgs& P, unsigned issued, int slot) {
  if (!P.counter) return;
  unsigned long long c = issued;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(P.counter + slot, c);
}

__device__ inline int64_t item_count(const ScanArgs& P) {
  return P.n_items_d ? (*P.n_items_d < P.n_items ? *P.n_items_d : P.n_items) : P.n_items;
}

constexpr int OV_CHUNK = 256;  // rows of an overflow work item
constexpr unsigned long long OV_MASK = (1ull << 36) - 1;

// append this lane's polyhedron (if `mine`) to one end of the overflow list:
// one 64-bit atomic per wavefront adds the entries and their chunks at once, so
// entry order and chunk numbering agree
__device__ inline void ov_append(const ScanArgs& P, bool mine, int end, int64_t item, int rows) {
  const unsigned long long m = __ballot(mine);
  if (!m) return;
  const int c = mine ? (rows + OV_CHUNK - 1) / OV_CHUNK : 0;
  const int ci = wave_prefix_sum(c), tot = __builtin_amdgcn_readlane(ci, 63);
  const int lane = threadIdx.x & 63, leader = __ffsll((long long)m) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(&P.ov_ctr[end], ((unsigned long long)__popcll(m) << 36) | (unsigned)tot);
  const uint32_t blo = __shfl((uint32_t)base, leader, 64), bhi = __shfl((uint32_t)(base >> 32), leader, 64);
  base = ((unsigned long long)bhi << 32) | blo;
  if (mine) {
    const int64_t idx = (int64_t)(base >> 36) + lanes_below(m);
    const int64_t slot = end ? P.ov_cap - 1 - idx : idx;
    P.ov_items[slot] = (int32_t)item;
    P.ov_chunk0[slot] = (int32_t)((int64_t)(base & OV_MASK) + ci - c);
  }
}

// How the waves of the one-polyhedron-per-lane pass get their polyhedra (64
// consecutive items per group): one group per wave of a grid sized to the
// items; a persistent grid (as many waves as fit at once) striding over the
// groups; or that grid taking groups from a device counter in the order the
// waves ask (an atomic head over the kind's whole list, so waves that drew
// cheap groups take more).
enum { SCAN_GRID_LAUNCH = 1, SCAN_GRID_STRIDE = 2, SCAN_GRID_QUEUE = 3 };

// one polyhedron per lane, the rows of a wavefront's polyhedra shared by its
// lanes; polyhedra with more than small_rows rows go to the front of the
// overflow list, wide ones to its back
template <int KIND, bool LOG>
__device__ inline void scan_group(const ScanArgs& P, int64_t item, int64_t count, float4* slots, int* marks,
                                  unsigned long long* qb, unsigned& issued) {
  Poly q;  // not cleared: a lane without a polyhedron owns no row, so no lane reads it
  q.wide = 0;
  const int nc = item < count ? build_poly<KIND>(P, item, q) : 0;
  const int rows = nc > 0 ? q.nu * q.nv : 0;
  const bool big = nc > 0 && (rows > P.small_rows || q.wide);
  ov_append(P, big && !q.wide, 0, item, rows);
  ov_append(P, big && q.wide, 1, item, rows);
  Rows r;  // set only for lanes with rows to deal; rows past the end are dropped whatever it holds
  if (nc > 0 && !big) setup_rows<KIND, false>(q, P.md[q.mesh], r);
  scan_rows_lanes<KIND, LOG>(P, q, r, nc > 0 && !big ? rows : 0, slots, marks, qb, issued);
}

template <int KIND, bool LOG>
__global__ __launch_bounds__(256) void k_scan_small(ScanArgs P) {
  __shared__ unsigned long long s_q[256 / 64][QCAP];
  __shared__ float4 s_slot[256 / 64][64 * RowSlot<KIND>::F4];
  __shared__ int s_mark[256 / 64][64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t count = item_count(P), groups = (count + 63) >> 6;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  unsigned issued = 0;
  if (P.grid_mode == SCAN_GRID_QUEUE) {
    // Same-address atomics serialise (about 10 ns each here), so a wavefront
    // takes queue_chunk groups per pop: about two pops per wavefront in all.
    const int64_t k = P.queue_chunk;
    auto pop = [&]() -> int64_t {
      unsigned long long g = 0;
      if (lane == 0) g = atomicAdd(P.head, (unsigned long long)k);
      return (int64_t)__builtin_amdgcn_readfirstlane((int)g);
    };
    // every wave leaves once its next chunk starts past the last group
    for (int64_t g0 = pop(); g0 < groups; g0 = pop())
      for (int64_t g = g0; g < g0 + k && g < groups; g++)
        scan_group<KIND, LOG>(P, 64 * g + lane, count, s_slot[w], s_mark[w], s_q[w], issued);
  } else {
    for (int64_t g = blockIdx.x * (int64_t)(blockDim.x >> 6) + w; g < groups;
         g = P.grid_mode == SCAN_GRID_STRIDE ? g + nw : groups)
      scan_group<KIND, LOG>(P, 64 * g + lane, count, s_slot[w], s_mark[w], s_q[w], issued);
  }
  add_issued(P, issued, 0);
}

// first chunk of overflow entry e (list order; the wide list fills from the back)
template <bool WIDE>
__device__ inline int64_t ov_first_chunk(const ScanArgs& P, int64_t e) {
  return P.ov_chunk0[WIDE ? P.ov_cap - 1 - e : e];
}

// The overflow list in chunks of OV_CHUNK rows of one polyhedron per wavefront
// and step (a persistent grid striding over the chunks: the list follows face
// order, so neighbouring chunks are alike in cost), the chunk's rows dealt out
// to the lanes. WIDE: the back of the list (wide polyhedra), with FP64
// distances; otherwise the front. Every lane holds the same polyhedron. The
// chunk's entry is the last whose first chunk is at or before it, found by a
// 64-way search (lane j tests the j-th of 64 evenly spaced entries; chunk
// numbers grow along the list): a few vector loads in place of a chain of
// dependent ones, starting from the previous chunk's entry.
template <int KIND, bool WIDE, bool LOG>
__global__ __launch_bounds__(64) void k_scan_big(ScanArgs P) {
  __shared__ unsigned long long s_q[QCAP];
  const int lane = threadIdx.x;
  const unsigned long long ctr = P.ov_ctr[WIDE ? 1 : 0];
  const int64_t n = (int64_t)(ctr >> 36), total = (int64_t)(ctr & OV_MASK);
  unsigned issued = 0;
  int64_t lo = 0;  // entry 0 starts at chunk 0; later chunks lie at or after the previous one's entry
  for (int64_t ch = blockIdx.x; ch < total; ch += gridDim.x) {
    int64_t hi = n - 1;
    while (lo < hi) {
      const int64_t step = (hi - lo + 64) >> 6;  // ceil((hi - lo + 1) / 64)
      const int64_t at = lo + lane * step;
      const bool le = at <= hi && ov_first_chunk<WIDE>(P, at) <= ch;
      const int last = 63 - __clzll((long long)__ballot(le));  // lane 0 always holds
      const int64_t nlo = lo + last * step;
      hi = nlo + step - 1 < hi ? nlo + step - 1 : hi;
      lo = nlo;
    }
    const int64_t slot = WIDE ? P.ov_cap - 1 - lo : lo;
    Poly q = {};
    if (build_poly<KIND>(P, P.ov_items[slot], q) <= 0) continue;  // the same for every lane
    const int r0 = (int)(ch - P.ov_chunk0[slot]) * OV_CHUNK, rows = q.nu * q.nv;
    const int cnt = rows - r0 < OV_CHUNK ? rows - r0 : OV_CHUNK;
    if (cnt <= 0) continue;
    Rows r;
    setup_rows<KIND, WIDE>(q, P.md[q.mesh], r);
    scan_rows_wave<KIND, true, WIDE, LOG>(P, q, r, lane == 0 ? cnt : 0, r0, s_q, issued);  // lane 0: the rows
  }
  add_issued(P, issued, 3);
}

__global__ void k_zero_i32(int32_t* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// every key of the allocated bricks (device count, capped) set to empty; block 0
// also clears the zn counters at zero
__global__ void k_init_keys(unsigned long long* keys, const int64_t* __restrict__ stats, int64_t cap,
                            unsigned long long* zero, int zn) {
  if (blockIdx.x == 0 && (int)threadIdx.x < zn) zero[threadIdx.x] = 0;
  const int64_t nb = stats[ST_NBRICKS] < cap ? stats[ST_NBRICKS] : cap;
  const int64_t n = nb * BRICK_CELLS;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = EMPTY_KEY;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// number of set keys per brick slot (0 for slots past the allocated bricks): one
// wavefront per brick, every lane loading its BRICK_ROUNDS keys at once (lane + 64 r)
__global__ __launch_bounds__(256) void k_brick_count(const unsigned long long* __restrict__ keys,
                                                     const int64_t* __restrict__ stats, int64_t cap, int32_t* cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t nb = stats[ST_NBRICKS] < cap ? stats[ST_NBRICKS] : cap;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t s = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); s < cap; s += nw) {
    int c = 0;
    if (s < nb) {
      const unsigned long long* kp = keys + s * BRICK_CELLS + lane;
      unsigned long long k[BRICK_ROUNDS];
#pragma unroll
      for (int r = 0; r < BRICK_ROUNDS; r++) k[r] = kp[64 * r];
#pragma unroll
      for (int r = 0; r < BRICK_ROUNDS; r++) c += __popcll(__ballot(k[r] != EMPTY_KEY));
    }
    if (lane == 0) cnt[s] = c;
  }
}

// band offsets of every mesh from the per-brick offsets
__global__ void k_band_offsets(const int32_t* __restrict__ first_slot, const int32_t* __restrict__ boff, int n_meshes,
                               int64_t cap, int64_t* band_off) {
  for (int m = threadIdx.x; m <= n_meshes; m += blockDim.x) {
    int64_t s = first_slot[m];
    band_off[m] = boff[s < cap ? s : cap];
  }
}

struct SignArgs {
  const float* V;
  const int32_t* T;
  const FaceRec* frec;  // [nf] corners, vertex indices, unit normal
  const int4* edges;
  const int32_t* face_edges;
  const float4* vinfo;
  const int32_t* brick_list;
  const int32_t* brick_mesh;
  const MeshDesc* md;
  unsigned long long* keys;  // read; with RESET, every set key is returned to empty
  const int32_t* boff;
  const int64_t* stats;
  float* sdf;
  int32_t* feat;
  int32_t* cell;
  float* dense;
  int64_t cap;
  int64_t nf, ne;
};

// mesh-local feature id of a global one
__device__ inline int32_t local_id(const SignArgs& P, const MeshDesc& G, int32_t id) {
  return id < P.nf ? id - G.f_off
                   : (id < P.nf + P.ne ? G.nf + (int32_t)(id - P.nf - G.e_off)
                                       : G.nf + G.ne + (int32_t)(id - P.nf - P.ne - G.v_off));
}

__device__ inline void put_cell(const SignArgs& P, const MeshDesc& G, int64_t out, float sd, int32_t local, int i,
                                int j, int k) {
  const int32_t lin = i + G.n[0] * (j + G.n[1] * k);
  P.sdf[out] = sd;
  P.feat[out] = local;
  P.cell[out] = lin;
  if (P.dense) P.dense[lin] = sd;
}

__device__ inline f3 rel(const float* V, int64_t i, d3 c) { return tof(vload_d(V, i) - c); }
__device__ inline f3 xyz(float4 a) { return mk(a.x, a.y, a.z); }

// a cell whose winning face candidate had its closest point on the face boundary:
// recompute the closest point and take the pseudonormal of the feature holding
// it (only for polyhedra of at most WIDE_CELLS: wide ones decide every sign in
// the scan, in FP64)
__device__ inline void sign_open(const SignArgs& P, const MeshDesc& G, unsigned long long key, int i, int j,
                                       int k, int64_t out) {
  const float d = __uint_as_float((uint32_t)(key >> 32));
  const int32_t id = (int32_t)((uint32_t)key & ID_MASK);
  const d3 c = mkd(G.origin[0] + (i + 0.5) * G.h, G.origin[1] + (j + 0.5) * G.h, G.origin[2] + (k + 0.5) * G.h);
  f3 qq = mk(0.f, 0.f, 0.f), N = mk(0.f, 0.f, 0.f);
  if (id < P.nf) {
    const int64_t f = id;
    float wt[3];
    const FaceRec& R = P.frec[f];
    const float4 ra = R.c[0], rb = R.c[1], rc = R.c[2];
    int r = closest_triangle(mk(0.f, 0.f, 0.f), tof(mkd(ra.x, ra.y, ra.z) - c), tof(mkd(rb.x, rb.y, rb.z) - c),
                             tof(mkd(rc.x, rc.y, rc.z) - c), qq, wt);
    if (r == 0) N = xyz(R.n);
    else if (r <= 3) {
      int4 E = P.edges[P.face_edges[3 * f + r - 1]];
      N = xyz(P.frec[E.z].n) + xyz(P.frec[E.w].n);
    } else N = xyz(P.vinfo[P.T[3 * f + r - 4]]);
  } else if (id < P.nf + P.ne) {
    int4 E = P.edges[id - P.nf];
    float tt;
    qq = closest_segment(mk(0.f, 0.f, 0.f), rel(P.V, E.x, c), rel(P.V, E.y, c), tt);
    if (tt <= 0.f) N = xyz(P.vinfo[E.x]);
    else if (tt >= 1.f) N = xyz(P.vinfo[E.y]);
    else N = xyz(P.frec[E.z].n) + xyz(P.frec[E.w].n);
  } else {
    const int64_t v = id - P.nf - P.ne;
    qq = rel(P.V, v, c);
    N = xyz(P.vinfo[v]);
  }
  const float s = dot(mk(-qq.x, -qq.y, -qq.z), N) >= 0.f ? 1.f : -1.f;
  put_cell(P, G, out, s * d, local_id(P, G, id), i, j, k);
}

// Sign of every band cell (Section 4.1.3, Eq. 8) and the compact band list with
// each mesh's own feature ids and cell indices. One wavefront per brick: lane l
// holds the cells of in-brick position l + 64 r for r < BRICK_ROUNDS (Morton
// order, brick_local), loaded at once; the output position is the brick's
// offset plus the rank among the set cells in (r, lane) order, which is the
// in-brick position order. Most keys carry their sign from the scan; the rest
// (SIGN_OPEN) are finished after the brick's decided cells. With RESET each set
// key is stored back as empty once its cell is written, so that the store is
// empty for the next scan without a pass of its own (its stores take the pass
// from 70 to 74 registers, hence a kernel of its own).
template <bool RESET>
__global__ __launch_bounds__(256) void k_sign(SignArgs P) {
  const int lane = threadIdx.x & 63;
  const int64_t nb = P.stats[ST_NBRICKS] < P.cap ? P.stats[ST_NBRICKS] : P.cap;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t slot = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); slot < nb; slot += nw) {
    unsigned long long* kp = P.keys + slot * BRICK_CELLS + lane;
    unsigned long long key[BRICK_ROUNDS];
#pragma unroll
    for (int r = 0; r < BRICK_ROUNDS; r++) key[r] = kp[64 * r];
    const MeshDesc& G = P.md[P.brick_mesh[slot]];
    int bx, by, bz;
    brick_coords(G, P.brick_list[slot], bx, by, bz);
    // cell of round r: in-brick position lane + 64 r
    auto cell_i = [&](int r) { int i, j, k; brick_cell(lane + 64 * r, i, j, k); return bx * BRICK + i; };
    auto cell_j = [&](int r) { int i, j, k; brick_cell(lane + 64 * r, i, j, k); return by * BRICK + j; };
    auto cell_k = [&](int r) { int i, j, k; brick_cell(lane + 64 * r, i, j, k); return bz * BRICK + k; };
    const int64_t ob = P.boff[slot];
    int before = 0;
    unsigned open_bits = 0;
    unsigned long long open_pos = 0;  // 9-bit band ranks within the brick of open cells r = 0..6
    uint32_t open_pos7 = 0;
#pragma unroll
    for (int r = 0; r < BRICK_ROUNDS; r++) {
      const bool valid = key[r] != EMPTY_KEY;
      const unsigned long long msk = __ballot(valid);
      if (valid) {
        const uint32_t pos = (uint32_t)(before + lanes_below(msk));
        const uint32_t lo = (uint32_t)key[r];
        const uint32_t code = lo >> 30;
        if (code == SIGN_OPEN) {
          open_bits |= 1u << r;
          if (r < 7) open_pos |= (unsigned long long)pos << (9 * r);
          else open_pos7 = pos;
        } else {
          const float d = __uint_as_float((uint32_t)(key[r] >> 32));
          put_cell(P, G, ob + pos, code == SIGN_NEG ? -d : d, local_id(P, G, (int32_t)(lo & ID_MASK)), cell_i(r),
                   cell_j(r), cell_k(r));
          if (RESET) kp[64 * r] = EMPTY_KEY;
        }
      }
      before += __popcll(msk);
    }
    while (open_bits) {
      const int r = __ffs(open_bits) - 1;
      open_bits &= open_bits - 1;
      const uint32_t pos = r < 7 ? (uint32_t)(open_pos >> (9 * r)) & 511u : open_pos7;
      sign_open(P, G, kp[64 * r], cell_i(r), cell_j(r), cell_k(r), ob + pos);
      if (RESET) kp[64 * r] = EMPTY_KEY;
    }
  }
}

}  // namespace csc

using namespace csc;

namespace {
size_t au(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr int PERSIST_BLOCKS = 2048;

struct WsLayout {
  size_t keys, cnt, scan, big, boff, ctr, total;
  int64_t cap;
};

int64_t capacity(const csc_features* f) { return f->synced ? f->n_bricks : f->nbt; }

WsLayout ws_layout(const csc_features* f, int64_t cap) {
  WsLayout L;
  L.cap = cap;
  L.keys = 0;
  L.cnt = au(sizeof(unsigned long long) * (size_t)(cap * BRICK_CELLS + 1));
  L.scan = L.cnt + au(sizeof(int32_t) * (size_t)(cap + 1));
  L.big = L.scan + au(sizeof(int32_t) * (size_t)scan_tmp_ints(cap + 1));
  // the overflow lists: 6 counters (two per kind), then per kind its entries and
  // their first chunks (the kinds are scanned concurrently)
  L.boff = L.big + 256 + au(2 * sizeof(int32_t) * (size_t)(f->nf + 2 * f->ne + 2 * f->nv + 3));
  L.ctr = L.boff + au(sizeof(int64_t) * (size_t)(f->n_meshes + 1));
  L.total = L.ctr + au(8 * sizeof(unsigned long long));
  return L;
}

// cap from the workspace size: the largest brick count whose layout fits
bool cap_from_bytes(const csc_features* f, size_t bytes, WsLayout& L) {
  int64_t hi = f->nbt, lo = 0;
  if (ws_layout(f, 0).total > bytes) return false;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) / 2;
    if (ws_layout(f, mid).total <= bytes) lo = mid;
    else hi = mid - 1;
  }
  L = ws_layout(f, lo);
  return true;
}

ScanArgs scan_args(const csc_features* f, unsigned long long* keys, int64_t cap) {
  ScanArgs A;
  A.V = f->verts;
  A.T = f->tris_g;
  A.frec = f->face_rec;
  A.edges = f->edges;
  A.face_edges = f->face_edges;
  A.fslack = f->fslack;
  A.fabsorbed = f->fabsorbed;
  A.ecls = f->edge_cls;
  A.vinfo = f->vinfo;
  A.vbits = f->vbits;
  A.items = nullptr;
  A.n_items_d = nullptr;
  A.face_mesh = f->face_mesh;
  A.vert_mesh = f->vert_mesh;
  A.md = f->d_mesh;
  A.brick_index = f->brick_index;
  A.keys = keys;
  A.counter = nullptr;
  A.ov_items = nullptr;
  A.ov_chunk0 = nullptr;
  A.ov_ctr = nullptr;
  A.ov_cap = 0;
  A.stats = f->d_stats;
  A.cap = cap;
  A.nf = f->nf;
  A.ne = f->ne;
  A.n_items = 0;
  A.small_rows = 32;
  A.per_cell = 0;
  A.log = nullptr;
  A.log_mask = nullptr;
  A.log_rounds = nullptr;
  A.log_cap = 0;
  A.grid_mode = SCAN_GRID_STRIDE;
  A.head = nullptr;
  A.queue_chunk = 1;
  return A;
}

// diagnostics: which launches log their atomics (csc_scan_record_atomics)
struct AtomicLog {
  uint32_t* log;
  unsigned long long* mask;
  unsigned* rounds;
  int64_t cap;
  int select;  // launch tag to log (kind, 3 + kind overflow, 6 + kind wide), -1 all
};

bool logged(const AtomicLog* lg, int tag) { return lg && (lg->select < 0 || lg->select == tag); }

ScanArgs with_log(ScanArgs A, const AtomicLog* lg) {
  A.log = lg->log;
  A.log_mask = lg->mask;
  A.log_rounds = lg->rounds;
  A.log_cap = lg->cap;
  return A;
}

// blocks of a kernel resident at once on the whole device (queried once)
template <typename K>
unsigned resident_blocks(K kernel, int threads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1 || cus < 1)
    return 1024;
  return (unsigned)(per_cu * cus);
}

template <int KIND, bool LOG>
unsigned small_grid(const ScanArgs& A) {
  const unsigned need = grid_1d(A.n_items, 256);
  if (A.grid_mode == SCAN_GRID_LAUNCH) return need;
  static const unsigned resident = resident_blocks(k_scan_small<KIND, LOG>, 256);
  return need < resident ? need : resident;
}

// the chunked overflow pass: every wavefront the device holds at once (a few
// thousand; an empty list costs one load and exit per wavefront)
template <int KIND, bool LOG>
unsigned big_grid() {
  static const unsigned resident = resident_blocks(k_scan_big<KIND, false, LOG>, 64);
  return resident;
}

// groups per pop of the group queue: about two pops per wavefront of the grid
// (from the launch bound of the item count), at least 1, at most 64
inline int32_t queue_chunk(const ScanArgs& A, unsigned blocks) {
  const int64_t groups = (A.n_items + 63) / 64, waves = 4 * (int64_t)blocks;
  const int64_t k = groups / (2 * waves);
  return (int32_t)(k < 1 ? 1 : (k > 64 ? 64 : k));
}

template <int KIND>
void launch_kind(ScanArgs A, int stage, int stage_big, hipStream_t s, const AtomicLog* lg) {
  {
    StageTimer t(stage, s);
    if (logged(lg, KIND)) {
      const unsigned g = small_grid<KIND, true>(A);
      A.queue_chunk = queue_chunk(A, g);
      k_scan_small<KIND, true><<<g, 256, 0, s>>>(with_log(A, lg));
    } else {
      const unsigned g = small_grid<KIND, false>(A);
      A.queue_chunk = queue_chunk(A, g);
      k_scan_small<KIND, false><<<g, 256, 0, s>>>(A);
    }
  }
  {
    StageTimer t(stage_big, s);
    if (logged(lg, 3 + KIND)) k_scan_big<KIND, false, true><<<big_grid<KIND, true>(), 64, 0, s>>>(with_log(A, lg));
    else k_scan_big<KIND, false, false><<<big_grid<KIND, false>(), 64, 0, s>>>(A);
  }
  // wide polyhedra (boxes over WIDE_CELLS): rare, FP64, in chunks of rows
  StageTimer t(TS_SCAN_WIDE, s);
  if (logged(lg, 6 + KIND)) k_scan_big<KIND, true, true><<<PERSIST_BLOCKS / 8, 64, 0, s>>>(with_log(A, lg));
  else k_scan_big<KIND, true, false><<<PERSIST_BLOCKS / 8, 64, 0, s>>>(A);
}

// key initialisation and the scan launches of the three kinds; counters
// (3 slots) may be null; big: the overflow lists (6 counters in 256 bytes, then
// each kind's entries and first chunks). For a batch, faces run on
// the caller's stream and edges, then vertices, on the side stream, forked
// after the key initialisation and joined at the end (their atomic minima
// commute): the batch's mix of polyhedron sizes leaves idle slots in each
// kind's passes (batch of 64: 1.875 -> 1.792 ms per step). One large mesh
// fills the GPU with each kind alone, and there the overlap only adds
// contention (1024^3 sphere: 3.43 -> 3.47 ms), so it stays on one stream.
// With stage timing on, the kinds also run one after another, so that each
// timed stage is one kernel running alone.
// fill_store: every key of the allocated bricks set to empty first; else the
// caller keeps the store empty between scans (csc_options.keep_store_empty).
void run_scans(const csc_features* f, unsigned long long* keys, int64_t cap, unsigned long long* counters,
               int32_t* big, hipStream_t s, bool fill_store, const AtomicLog* lg = nullptr) {
  unsigned long long* ov_ctr = (unsigned long long*)big;
  int32_t* ov = big + 64;  // past the 256 bytes of counters
  {
    StageTimer t(TS_INIT, s);
    // with the overflow lists' two counters and group head per kind
    if (fill_store) k_init_keys<<<PERSIST_BLOCKS * 4, 256, 0, s>>>(keys, f->d_stats, cap, ov_ctr, 9);
    else k_init_keys<<<1, 64, 0, s>>>(keys, f->d_stats, 0, ov_ctr, 9);
  }
  // a fork that cannot be set up leaves everything on the caller's stream
  bool fork = f->n_meshes > 1 && !stage_timing_on() && f->side && !lg;
  if (fork)
    fork = hipEventRecord(f->ev_fork, s) == hipSuccess && hipStreamWaitEvent(f->side, f->ev_fork, 0) == hipSuccess;
  hipStream_t s2 = fork ? f->side : s;
  ScanArgs A = scan_args(f, keys, cap);
  A.grid_mode = f->opt.scan_grid;
  A.head = ov_ctr + 6;
  A.ov_ctr = ov_ctr;
  A.ov_cap = f->nf;
  A.ov_items = ov;
  A.ov_chunk0 = ov + f->nf;
  A.counter = counters;
  A.n_items = f->nf;
  A.items = f->face_order_n == f->nf ? f->face_order : nullptr;
  A.small_rows = f->opt.small_rows[0];
  A.per_cell = f->opt.scan_mode == 1;
  launch_kind<KIND_FACE>(A, TS_SCAN_FACE, TS_SCAN_FACE_BIG, s, lg);
  ov += 2 * f->nf;
  A.head = ov_ctr + 7;
  A.ov_ctr = ov_ctr + 2;
  A.ov_cap = 2 * f->ne;
  A.ov_items = ov;
  A.ov_chunk0 = ov + 2 * f->ne;
  A.small_rows = f->opt.small_rows[1];
  A.per_cell = f->opt.scan_mode == 1;
  A.items = f->epoly;
  A.n_items = 2 * f->ne;
  A.n_items_d = &f->d_stats[ST_NEPOLY];
  A.counter = counters ? counters + 1 : nullptr;
  launch_kind<KIND_EDGE>(A, TS_SCAN_EDGE, TS_SCAN_EDGE_BIG, s2, lg);
  ov += 4 * f->ne;
  A.head = ov_ctr + 8;
  A.ov_ctr = ov_ctr + 4;
  A.ov_cap = 2 * f->nv;
  A.ov_items = ov;
  A.ov_chunk0 = ov + 2 * f->nv;
  A.small_rows = f->opt.small_rows[2];
  A.per_cell = f->opt.scan_mode == 1;
  A.items = f->vpoly;
  A.n_items = 2 * f->nv;
  A.n_items_d = &f->d_stats[ST_NVPOLY];
  A.counter = counters ? counters + 2 : nullptr;
  launch_kind<KIND_VERT>(A, TS_SCAN_VERT, TS_SCAN_VERT_BIG, s2, lg);
  if (fork && (hipEventRecord(f->ev_join, s2) != hipSuccess || hipStreamWaitEvent(s, f->ev_join, 0) != hipSuccess))
    (void)hipStreamSynchronize(s2);  // no join on the device: finish the side branch from the host
}

// after scans with no sign pass: the store left empty again for a caller that
// keeps it so
void empty_store_again(const csc_features* f, unsigned long long* keys, int64_t cap, hipStream_t s) {
  if (f->opt.keep_store_empty) k_init_keys<<<PERSIST_BLOCKS * 4, 256, 0, s>>>(keys, f->d_stats, cap, nullptr, 0);
}

int scan_convert_impl(const csc_features* f, void* workspace_d, size_t ws_bytes, float* sdf_d, int32_t* feat_d,
                      int32_t* cell_d, int64_t* n_band_d, int64_t* band_off_d, float* dense_d, hipStream_t s) {
  WsLayout L;
  if (!cap_from_bytes(f, ws_bytes, L)) return CSC_WORKSPACE_TOO_SMALL;
  const int64_t cap = L.cap;
  char* W = (char*)workspace_d;
  unsigned long long* keys = (unsigned long long*)(W + L.keys);
  int32_t* cnt = (int32_t*)(W + L.cnt);
  int32_t* tmp = (int32_t*)(W + L.scan);
  int64_t* boff64 = band_off_d ? band_off_d : (int64_t*)(W + L.boff);
  if (dense_d) {
    const MeshDesc& G = f->mesh[0];
    int64_t nd = (int64_t)G.n[0] * G.n[1] * G.n[2];
    k_fill_f32<<<PERSIST_BLOCKS * 4, 256, 0, s>>>(dense_d, nd, __builtin_inff());
  }
  run_scans(f, keys, cap, nullptr, (int32_t*)(W + L.big), s, !f->opt.keep_store_empty);
  hipError_t e;
  {
    StageTimer t(TS_COUNT, s);
    static const unsigned count_blocks = resident_blocks(k_brick_count, 256);
    if (cap > 0) k_brick_count<<<count_blocks, 256, 0, s>>>(keys, f->d_stats, cap, cnt);
    e = exclusive_scan(cnt, cnt, cap, tmp, n_band_d, cnt + cap, s);
    k_band_offsets<<<1, 64, 0, s>>>(f->first_slot, cnt, f->n_meshes, cap, boff64);
  }
  if (e != hipSuccess) return fail_hip(e);
  if (cap > 0) {
    StageTimer t(TS_SIGN, s);
    SignArgs S;
    S.V = f->verts;
    S.T = f->tris_g;
    S.frec = f->face_rec;
    S.edges = f->edges;
    S.face_edges = f->face_edges;
    S.vinfo = f->vinfo;
    S.brick_list = f->brick_list;
    S.brick_mesh = f->brick_mesh;
    S.md = f->d_mesh;
    S.keys = keys;
    S.boff = cnt;
    S.stats = f->d_stats;
    S.sdf = sdf_d;
    S.feat = feat_d;
    S.cell = cell_d;
    S.dense = dense_d;
    S.cap = cap;
    S.nf = f->nf;
    S.ne = f->ne;
    // every block resident at once (the persistent loop strides over the bricks)
    if (f->opt.keep_store_empty) {
      static const unsigned sign_blocks = resident_blocks(k_sign<true>, 256);
      k_sign<true><<<sign_blocks, 256, 0, s>>>(S);
    } else {
      static const unsigned sign_blocks = resident_blocks(k_sign<false>, 256);
      k_sign<false><<<sign_blocks, 256, 0, s>>>(S);
    }
  }
  e = hipGetLastError();
  return e == hipSuccess ? CSC_OK : fail_hip(e);
}

}  // namespace

extern "C" int csc_scan_convert_workspace(const csc_features* f, size_t* bytes, int64_t* max_band_cells) {
  if (!f || !f->built || !bytes) return CSC_INVALID_ARG;
  const int64_t cap = capacity(f);
  *bytes = ws_layout(f, cap).total;
  if (max_band_cells) *max_band_cells = cap * BRICK_CELLS;
  return CSC_OK;
}

extern "C" int csc_scan_convert_workspace_for(const csc_features* f, int64_t n_bricks, size_t* bytes,
                                              int64_t* max_band_cells) {
  if (!f || !f->built || !bytes || n_bricks < 0) return CSC_INVALID_ARG;
  const int64_t cap = n_bricks < f->nbt ? n_bricks : f->nbt;
  *bytes = ws_layout(f, cap).total;
  if (max_band_cells) *max_band_cells = cap * BRICK_CELLS;
  return CSC_OK;
}

extern "C" int csc_scan_convert(const csc_features* f, void* workspace_d, size_t ws_bytes, float* sdf_d,
                                int32_t* feat_d, int32_t* cell_d, int64_t* n_band_d, float* dense_d, void* stream) {
  if (!f || !f->built || !workspace_d || !sdf_d || !feat_d || !cell_d || !n_band_d) return CSC_INVALID_ARG;
  if (dense_d && f->n_meshes != 1) return CSC_INVALID_ARG;
  return scan_convert_impl(f, workspace_d, ws_bytes, sdf_d, feat_d, cell_d, n_band_d, nullptr, dense_d,
                           (hipStream_t)stream);
}

extern "C" int csc_scan_convert_batched(const csc_features* f, void* workspace_d, size_t ws_bytes, float* sdf_d,
                                        int32_t* feat_d, int32_t* cell_d, int64_t* band_off_d, void* stream) {
  if (!f || !f->built || !workspace_d || !sdf_d || !feat_d || !cell_d || !band_off_d) return CSC_INVALID_ARG;
  return scan_convert_impl(f, workspace_d, ws_bytes, sdf_d, feat_d, cell_d, nullptr, band_off_d, nullptr,
                           (hipStream_t)stream);
}

extern "C" int csc_scan_convert_count(const csc_features* f, void* workspace_d, size_t ws_bytes, int64_t counts[6],
                                      void* stream) {
  if (!f || !f->built || !workspace_d || !counts) return CSC_INVALID_ARG;
  WsLayout L;
  if (!cap_from_bytes(f, ws_bytes, L)) return CSC_WORKSPACE_TOO_SMALL;
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)workspace_d;
  unsigned long long* ctr = (unsigned long long*)(W + L.ctr);
  k_zero_u64<<<1, 64, 0, s>>>(ctr, 6);
  run_scans(f, (unsigned long long*)(W + L.keys), L.cap, ctr, (int32_t*)(W + L.big), s, true);
  empty_store_again(f, (unsigned long long*)(W + L.keys), L.cap, s);
  unsigned long long h[6];
  hipError_t e = hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e);
  for (int i = 0; i < 6; i++) counts[i] = (int64_t)h[i];
  return CSC_OK;
}

extern "C" int csc_scan_record_atomics(const csc_features* f, void* workspace_d, size_t ws_bytes, int32_t launch,
                                       uint32_t* log_d, unsigned long long* mask_d, int64_t max_rounds,
                                       int64_t* rounds, void* stream) {
  if (!f || !f->built || !workspace_d || !rounds || launch < -1 || launch > 8 || max_rounds < 0 ||
      (max_rounds > 0 && (!log_d || !mask_d)))
    return CSC_INVALID_ARG;
  WsLayout L;
  if (!cap_from_bytes(f, ws_bytes, L)) return CSC_WORKSPACE_TOO_SMALL;
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)workspace_d;
  unsigned long long* ctr = (unsigned long long*)(W + L.ctr);
  k_zero_u64<<<1, 64, 0, s>>>(ctr, 8);
  AtomicLog lg;
  lg.log = log_d;
  lg.mask = mask_d;
  lg.rounds = (unsigned*)(ctr + 7);
  lg.cap = max_rounds;
  lg.select = launch;
  run_scans(f, (unsigned long long*)(W + L.keys), L.cap, nullptr, (int32_t*)(W + L.big), s, true, &lg);
  empty_store_again(f, (unsigned long long*)(W + L.keys), L.cap, s);
  unsigned h = 0;
  hipError_t e = hipMemcpyAsync(&h, ctr + 7, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e);
  *rounds = (int64_t)h;
  return CSC_OK;
}
