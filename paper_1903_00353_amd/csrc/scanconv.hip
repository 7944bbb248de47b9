// Scan conversion of the characteristic polyhedra (Section 5, Section 9,
// Section 10) and the sign pass (Section 4.1.3).
//
// One wavefront takes 64 polyhedra of one kind (one per lane), builds their
// planes, bounding boxes and local frames into LDS, then walks the union of
// their bounding-box cells 64 at a time: every lane tests one cell against its
// polyhedron (half-space test with slack, Alg. 2; cone/hemisphere discriminant,
// Eq. 10), the cells inside are compacted into an LDS queue, and each full queue
// of 64 candidates gets the exact clamped point-feature distance and one packed
// 64-bit atomicMin of (float bits of |d|, feature id) into the brick store.
// The paper's per-extrusion thread (Section 9) becomes this load-balanced wave;
// its float compare-and-swap loop becomes a single order-free integer min.
#include "geometry.h"
#include "internal.h"

namespace csc {

enum { KIND_FACE = 0, KIND_EDGE = 1, KIND_VERT = 2 };

struct ScanArgs {
  const float* V;
  const int32_t* T;
  const float4* fn;
  const int4* edges;
  const uint8_t* ecls;
  const float4* vinfo;
  const uint32_t* vbits;
  const int32_t* items;       // edge / vertex polyhedron list (unused for faces)
  const int32_t* brick_index;
  unsigned long long* keys;
  unsigned long long* counter;  // optional: number of atomicMin issued (diagnostics)
  int64_t nf, ne, n_items;
  double o[3];
  double h, whd, epsd;
  int n[3];
  int nb[3];
  float hf, whf, eps;
};

struct Poly {
  float pl[5][4];   // inside: m . p + off >= -eps  (p relative to the anchor cell centre)
  float g[9];       // feature points relative to the anchor cell centre
  float cone[4];    // vertex: axis, aperture cosine (or -2 for a hemisphere)
  int anc[3];
  int dim[3];
  int id;
};

__device__ inline d3 vload_d(const float* V, int64_t i) {
  return mkd((double)V[3 * i], (double)V[3 * i + 1], (double)V[3 * i + 2]);
}

__device__ inline f3 unit_f(d3 v) {
  double l = len(v);
  return l > 0 ? tof(v * (1.0 / l)) : mk(0.f, 0.f, 0.f);
}

// bounding box [lo, hi] (world) -> anchor and dimensions in cells; false if empty
__device__ inline bool box_cells(const ScanArgs& P, const double lo[3], const double hi[3], Poly& q) {
  const double marg = 1e-4;
  for (int k = 0; k < 3; k++) {
    double a = ceil((lo[k] - P.o[k]) / P.h - 0.5 - marg), b = floor((hi[k] - P.o[k]) / P.h - 0.5 + marg);
    if (a < 0) a = 0;
    if (b > P.n[k] - 1) b = P.n[k] - 1;
    if (!(a <= b)) return false;
    q.anc[k] = (int)a;
    q.dim[k] = (int)(b - a) + 1;
  }
  return true;
}

__device__ inline d3 anchor_centre(const ScanArgs& P, const Poly& q) {
  return mkd(P.o[0] + (q.anc[0] + 0.5) * P.h, P.o[1] + (q.anc[1] + 0.5) * P.h, P.o[2] + (q.anc[2] + 0.5) * P.h);
}

__device__ inline void set_plane(Poly& q, int i, f3 m, f3 through) {
  q.pl[i][0] = m.x;
  q.pl[i][1] = m.y;
  q.pl[i][2] = m.z;
  q.pl[i][3] = -dot(m, through);
}

// Face prism (Section 8.1): three inward side planes through the edges and the two
// caps |n . (x - a)| <= band*h (both the outward and inward prism at once).
__device__ inline int build_face(const ScanArgs& P, int64_t f, Poly& q) {
  d3 a = vload_d(P.V, P.T[3 * f]), b = vload_d(P.V, P.T[3 * f + 1]), c = vload_d(P.V, P.T[3 * f + 2]);
  float4 nn = P.fn[f];
  d3 n = mkd(nn.x, nn.y, nn.z);
  double lo[3], hi[3];
  const double A3[3] = {a.x, a.y, a.z}, B3[3] = {b.x, b.y, b.z}, C3[3] = {c.x, c.y, c.z}, N3[3] = {n.x, n.y, n.z};
  for (int k = 0; k < 3; k++) {
    double r = P.whd * fabs(N3[k]) + P.epsd;
    lo[k] = fmin(A3[k], fmin(B3[k], C3[k])) - r;
    hi[k] = fmax(A3[k], fmax(B3[k], C3[k])) + r;
  }
  if (!box_cells(P, lo, hi, q)) return 0;
  d3 c0 = anchor_centre(P, q);
  f3 A = tof(a - c0), B = tof(b - c0), C = tof(c - c0), nf = mk(nn.x, nn.y, nn.z);
  const f3 W[3] = {A, B, C};
  for (int j = 0; j < 3; j++) {
    f3 m = cross(nf, W[(j + 1) % 3] - W[j]);
    float l = norm3(m);
    set_plane(q, j, m * (1.f / l), W[j]);
  }
  float na = dot(nf, A);
  q.pl[3][0] = -nf.x; q.pl[3][1] = -nf.y; q.pl[3][2] = -nf.z; q.pl[3][3] = na + P.whf;
  q.pl[4][0] = nf.x;  q.pl[4][1] = nf.y;  q.pl[4][2] = nf.z;  q.pl[4][3] = P.whf - na;
  q.g[0] = A.x; q.g[1] = A.y; q.g[2] = A.z;
  q.g[3] = B.x; q.g[4] = B.y; q.g[5] = B.z;
  q.g[6] = C.x; q.g[7] = C.y; q.g[8] = C.z;
  q.id = (int)f;
  return q.dim[0] * q.dim[1] * q.dim[2];
}

// Edge wedge (Section 8.2): the dihedral region spanned by the two face normals
// (outward side) or their negatives (inward side), between the end caps, cut by
// the base plane through the edge with the summed normal (Section 8.2); the far
// side is the band distance itself (cells with |d| >= band*h are dropped).
__device__ inline int build_edge(const ScanArgs& P, int64_t item, Poly& q) {
  int32_t ent = P.items[item];
  int64_t e = ent >> 1;
  double sg = (ent & 1) ? -1.0 : 1.0;
  int4 E = P.edges[e];
  d3 a = vload_d(P.V, E.x), b = vload_d(P.V, E.y);
  float4 f1 = P.fn[E.z], f2 = P.fn[E.w];
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
  for (int k = 0; k < 3; k++) {
    double x1 = P.whd * U1[k], x2 = P.whd * U2[k];
    double alo = fmin(0.0, fmin(x1, x2)), ahi = fmax(0.0, fmax(x1, x2));
    if (us2 > 1e-12) {  // the arc lies inside the quadrilateral through the tangent intersection
      double t = P.whd * 2.0 * US[k] / us2;
      alo = fmin(alo, t);
      ahi = fmax(ahi, t);
    } else {
      alo = -P.whd;
      ahi = P.whd;
    }
    alo = fmax(alo, -P.whd);
    ahi = fmin(ahi, P.whd);
    lo[k] = fmin(A3[k], B3[k]) + alo - P.epsd;
    hi[k] = fmax(A3[k], B3[k]) + ahi + P.epsd;
  }
  if (!box_cells(P, lo, hi, q)) return 0;
  d3 c0 = anchor_centre(P, q);
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
  q.id = (int)(P.nf + e);
  return q.dim[0] * q.dim[1] * q.dim[2];
}

// Vertex cone (Section 4.2, Section 8.3) about the (possibly reflected)
// pseudonormal with the most diverging positive-pointing normal on its side, or a
// hemisphere (Section 4.1.3); box = cone box intersected with the sphere box.
__device__ inline int build_vertex(const ScanArgs& P, int64_t item, Poly& q) {
  int32_t ent = P.items[item];
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
  double tn = hemi ? 0.0 : sqrt(fmax(0.0, 1.0 - ct * ct)) / ct;
  double lo[3], hi[3];
  for (int k = 0; k < 3; k++) {
    double s = sqrt(fmax(0.0, 1.0 - AX[k] * AX[k]));
    double l, u;
    if (hemi) {
      l = AX[k] > 0 ? -P.whd * s : -P.whd;
      u = AX[k] < 0 ? P.whd * s : P.whd;
    } else {
      l = fmax(-P.whd, fmin(0.0, P.whd * (AX[k] - tn * s)));
      u = fmin(P.whd, fmax(0.0, P.whd * (AX[k] + tn * s)));
    }
    lo[k] = P3[k] + l - P.epsd;
    hi[k] = P3[k] + u + P.epsd;
  }
  if (!box_cells(P, lo, hi, q)) return 0;
  d3 c0 = anchor_centre(P, q);
  f3 A = tof(p - c0), axf = tof(ax);
  set_plane(q, 0, axf, A);
  q.cone[0] = axf.x; q.cone[1] = axf.y; q.cone[2] = axf.z;
  q.cone[3] = hemi ? -2.f : vi.w;
  q.g[0] = A.x; q.g[1] = A.y; q.g[2] = A.z;
  q.id = (int)(P.nf + P.ne + v);
  return q.dim[0] * q.dim[1] * q.dim[2];
}

__device__ inline long long wave_incl_scan_ll(long long v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    long long t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ inline int lanes_below(unsigned long long m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// a / b for a >= 0, b >= 1: float reciprocal estimate, then exact correction
// (one step suffices while a < 2^24, which covers ordinary polyhedra)
__device__ inline int idiv(int a, int b) {
  int qq = (int)((float)a * __builtin_amdgcn_rcpf((float)b));
  int r = a - qq * b;
  while (r < 0) { qq--; r += b; }
  while (r >= b) { qq++; r -= b; }
  return qq;
}

template <int KIND>
__global__ __launch_bounds__(64) void k_scan(ScanArgs P) {
  constexpr int NPL = KIND == KIND_VERT ? 1 : 5;
  constexpr int NG = KIND == KIND_FACE ? 9 : (KIND == KIND_EDGE ? 6 : 3);
  __shared__ float s_pl[NPL * 4][64];
  __shared__ float s_g[NG][64];
  __shared__ float s_cone[4][64];
  __shared__ int s_anc[3][64];
  __shared__ int s_nx[64], s_nxy[64], s_id[64];
  __shared__ long long s_start[65];
  __shared__ int s_qs[128], s_qi[128], s_qj[128], s_qk[128];

  const int lane = threadIdx.x;
  const int64_t item = (int64_t)blockIdx.x * 64 + lane;
  Poly q;
  int nc = 0;
  if (item < P.n_items) {
    if constexpr (KIND == KIND_FACE) nc = build_face(P, item, q);
    else if constexpr (KIND == KIND_EDGE) nc = build_edge(P, item, q);
    else nc = build_vertex(P, item, q);
  }
  if (nc > 0) {
#pragma unroll
    for (int i = 0; i < NPL; i++)
#pragma unroll
      for (int c = 0; c < 4; c++) s_pl[i * 4 + c][lane] = q.pl[i][c];
#pragma unroll
    for (int i = 0; i < NG; i++) s_g[i][lane] = q.g[i];
    if constexpr (KIND == KIND_VERT)
#pragma unroll
      for (int c = 0; c < 4; c++) s_cone[c][lane] = q.cone[c];
    s_anc[0][lane] = q.anc[0];
    s_anc[1][lane] = q.anc[1];
    s_anc[2][lane] = q.anc[2];
    s_nx[lane] = q.dim[0];
    s_nxy[lane] = q.dim[0] * q.dim[1];
    s_id[lane] = q.id;
  }
  long long inc = wave_incl_scan_ll(nc);
  s_start[lane] = inc - nc;
  if (lane == 63) s_start[64] = inc;
  __syncthreads();
  const long long total = s_start[64];
  const float hf = P.hf, eps = P.eps;
  unsigned issued = 0;

  auto process = [&](int sl, int di, int dj, int dk) {
    f3 p = mk(di * hf, dj * hf, dk * hf);
    float d;
    if constexpr (KIND == KIND_FACE) {
      f3 A = mk(s_g[0][sl], s_g[1][sl], s_g[2][sl]);
      f3 B = mk(s_g[3][sl], s_g[4][sl], s_g[5][sl]);
      f3 C = mk(s_g[6][sl], s_g[7][sl], s_g[8][sl]);
      f3 qq;
      float w[3];
      closest_triangle(p, A, B, C, qq, w);
      d = norm3(p - qq);
    } else if constexpr (KIND == KIND_EDGE) {
      f3 A = mk(s_g[0][sl], s_g[1][sl], s_g[2][sl]);
      f3 B = mk(s_g[3][sl], s_g[4][sl], s_g[5][sl]);
      float t;
      d = norm3(p - closest_segment(p, A, B, t));
    } else {
      d = norm3(p - mk(s_g[0][sl], s_g[1][sl], s_g[2][sl]));
    }
    if (d < P.whf) {
      int i = s_anc[0][sl] + di, j = s_anc[1][sl] + dj, k = s_anc[2][sl] + dk;
      int64_t bl = (int64_t)(i >> 3) + (int64_t)P.nb[0] * ((j >> 3) + (int64_t)P.nb[1] * (k >> 3));
      int32_t slot = P.brick_index[bl];
      if (slot >= 0) {
        unsigned long long key = ((unsigned long long)__float_as_uint(d) << 32) | (unsigned int)s_id[sl];
        atomicMin(&P.keys[(int64_t)slot * BRICK_CELLS + (i & 7) + 8 * (j & 7) + 64 * (k & 7)], key);
        issued++;
      }
    }
  };

  int qn = 0;
  for (long long base = 0; base < total; base += 64) {
    const long long g = base + lane;
    bool in = false;
    int sl = 0, di = 0, dj = 0, dk = 0;
    if (g < total) {
      int lo = 0, hi = 63;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (s_start[mid] <= g) lo = mid;
        else hi = mid - 1;
      }
      sl = lo;
      int loc = (int)(g - s_start[sl]);
      int nx = s_nx[sl], nxy = s_nxy[sl];
      dk = idiv(loc, nxy);
      int rem = loc - dk * nxy;
      dj = idiv(rem, nx);
      di = rem - dj * nx;
      f3 p = mk(di * hf, dj * hf, dk * hf);
      in = true;
#pragma unroll
      for (int i = 0; i < NPL; i++) {
        float v = s_pl[4 * i][sl] * p.x + s_pl[4 * i + 1][sl] * p.y + s_pl[4 * i + 2][sl] * p.z + s_pl[4 * i + 3][sl];
        in = in && (v >= -eps);
      }
      if constexpr (KIND == KIND_VERT) if (in) {
        f3 r = p - mk(s_g[0][sl], s_g[1][sl], s_g[2][sl]);
        float rr = dot(r, r);
        float lim = P.whf + eps;
        in = rr < lim * lim;
        float ct = s_cone[3][sl];
        if (in && ct > -1.f) {
          float te = dot(r, mk(s_cone[0][sl], s_cone[1][sl], s_cone[2][sl])) + eps;
          in = te >= 0.f && te * te >= ct * ct * rr;
        }
      }
    }
    unsigned long long m = __ballot(in);
    int pos = qn + lanes_below(m);
    if (in) {
      s_qs[pos] = sl;
      s_qi[pos] = di;
      s_qj[pos] = dj;
      s_qk[pos] = dk;
    }
    qn += __popcll(m);
    __syncthreads();
    if (qn >= 64) {
      process(s_qs[lane], s_qi[lane], s_qj[lane], s_qk[lane]);
      __syncthreads();
      if (lane < qn - 64) {
        int a0 = s_qs[64 + lane], a1 = s_qi[64 + lane], a2 = s_qj[64 + lane], a3 = s_qk[64 + lane];
        s_qs[lane] = a0;
        s_qi[lane] = a1;
        s_qj[lane] = a2;
        s_qk[lane] = a3;
      }
      qn -= 64;
      __syncthreads();
    }
  }
  if (lane < qn) process(s_qs[lane], s_qi[lane], s_qj[lane], s_qk[lane]);
  if (P.counter) {
    unsigned long long c = issued;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if (lane == 0 && c) atomicAdd(P.counter, c);
  }
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// number of set keys per brick
__global__ __launch_bounds__(512) void k_brick_count(const unsigned long long* __restrict__ keys, int32_t* cnt) {
  __shared__ int ws[8];
  unsigned long long k = keys[(int64_t)blockIdx.x * BRICK_CELLS + threadIdx.x];
  unsigned long long m = __ballot(k != EMPTY_KEY);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < 8; w++) t += ws[w];
    cnt[blockIdx.x] = t;
  }
}

struct SignArgs {
  const float* V;
  const int32_t* T;
  const float4* fn;
  const int4* edges;
  const int32_t* face_edges;
  const float4* vinfo;
  const int32_t* brick_list;
  const unsigned long long* keys;
  const int32_t* boff;
  float* sdf;
  int32_t* feat;
  int32_t* cell;
  float* dense;
  int64_t nf, ne;
  double o[3];
  double h;
  int n[3];
  int nb[3];
};

__device__ inline f3 rel(const float* V, int64_t i, d3 c) { return tof(vload_d(V, i) - c); }
__device__ inline f3 xyz(float4 a) { return mk(a.x, a.y, a.z); }

// Sign of a band cell from the pseudonormal of the lowest-dimensional feature
// holding its closest point (face normal; edge: sum of the two face normals;
// vertex: angle-weighted pseudonormal), Section 4.1.3 and Eq. 8.
__global__ __launch_bounds__(512) void k_sign(SignArgs P) {
  __shared__ int ws[9];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t slot = blockIdx.x;
  unsigned long long key = P.keys[slot * BRICK_CELLS + t];
  bool valid = key != EMPTY_KEY;
  unsigned long long m = __ballot(valid);
  if (lane == 0) ws[w] = __popcll(m);
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int i = 0; i < 8; i++) {
      int c = ws[i];
      ws[i] = acc;
      acc += c;
    }
  }
  __syncthreads();
  if (!valid) return;
  const int64_t out = P.boff[slot] + ws[w] + lanes_below(m);
  const int32_t b = P.brick_list[slot];
  const int bx = b % P.nb[0], by = (b / P.nb[0]) % P.nb[1], bz = b / (P.nb[0] * P.nb[1]);
  const int i = bx * 8 + (t & 7), j = by * 8 + ((t >> 3) & 7), k = bz * 8 + (t >> 6);
  const float d = __uint_as_float((uint32_t)(key >> 32));
  const int32_t id = (int32_t)(key & 0xffffffffu);
  const d3 c = mkd(P.o[0] + (i + 0.5) * P.h, P.o[1] + (j + 0.5) * P.h, P.o[2] + (k + 0.5) * P.h);
  f3 qq, N;
  if (id < P.nf) {
    const int64_t f = id;
    float wt[3];
    int r = closest_triangle(mk(0.f, 0.f, 0.f), rel(P.V, P.T[3 * f], c), rel(P.V, P.T[3 * f + 1], c),
                             rel(P.V, P.T[3 * f + 2], c), qq, wt);
    if (r == 0) N = xyz(P.fn[f]);
    else if (r <= 3) {
      int4 E = P.edges[P.face_edges[3 * f + r - 1]];
      N = xyz(P.fn[E.z]) + xyz(P.fn[E.w]);
    } else N = xyz(P.vinfo[P.T[3 * f + r - 4]]);
  } else if (id < P.nf + P.ne) {
    int4 E = P.edges[id - P.nf];
    float tt;
    qq = closest_segment(mk(0.f, 0.f, 0.f), rel(P.V, E.x, c), rel(P.V, E.y, c), tt);
    if (tt <= 0.f) N = xyz(P.vinfo[E.x]);
    else if (tt >= 1.f) N = xyz(P.vinfo[E.y]);
    else N = xyz(P.fn[E.z]) + xyz(P.fn[E.w]);
  } else {
    const int64_t v = id - P.nf - P.ne;
    qq = rel(P.V, v, c);
    N = xyz(P.vinfo[v]);
  }
  const float s = dot(mk(-qq.x, -qq.y, -qq.z), N) >= 0.f ? 1.f : -1.f;
  const int32_t lin = i + P.n[0] * (j + P.n[1] * k);
  P.sdf[out] = s * d;
  P.feat[out] = id;
  P.cell[out] = lin;
  if (P.dense) P.dense[lin] = s * d;
}

}  // namespace csc

using namespace csc;

namespace {
size_t au(size_t x) { return (x + 255) & ~(size_t)255; }
struct WsLayout {
  size_t keys, cnt, scan, total;
};
WsLayout ws_layout(const csc_features* f) {
  WsLayout L;
  int64_t nb = f->n_bricks;
  L.keys = 0;
  L.cnt = au(sizeof(unsigned long long) * (size_t)(nb * BRICK_CELLS + 1));
  L.scan = L.cnt + au(sizeof(int32_t) * (size_t)(nb + 1));
  L.total = L.scan + au(sizeof(int32_t) * (size_t)scan_tmp_ints(nb + 1) + 3 * sizeof(unsigned long long));
  return L;
}
}  // namespace

extern "C" int csc_scan_convert_workspace(const csc_features* f, size_t* bytes, int64_t* max_band_cells) {
  if (!f || !f->valid || !bytes) return CSC_INVALID_ARG;
  *bytes = ws_layout(f).total;
  if (max_band_cells) *max_band_cells = f->n_bricks * BRICK_CELLS;
  return CSC_OK;
}

namespace {

ScanArgs scan_args(const csc_features* f, unsigned long long* keys, unsigned long long* counter) {
  ScanArgs A;
  A.V = f->verts;
  A.T = f->tris;
  A.fn = f->face_n;
  A.edges = f->edges;
  A.ecls = f->edge_cls;
  A.vinfo = f->vinfo;
  A.vbits = f->vbits;
  A.items = nullptr;
  A.brick_index = f->brick_index;
  A.keys = keys;
  A.counter = counter;
  A.nf = f->nf;
  A.ne = f->ne;
  A.n_items = 0;
  for (int k = 0; k < 3; k++) {
    A.o[k] = f->grid.origin[k];
    A.n[k] = f->grid.n[k];
    A.nb[k] = f->nb[k];
  }
  A.h = f->grid.h;
  A.whd = (double)f->grid.band_cells * f->grid.h;
  A.epsd = (double)f->opt.eps_rel * f->grid.h;
  A.hf = (float)f->grid.h;
  A.whf = (float)A.whd;
  A.eps = (float)A.epsd;
  return A;
}

// key init and the three scan launches; counters (3 slots) may be null
void run_scans(const csc_features* f, unsigned long long* keys, unsigned long long* counters, hipStream_t s) {
  const int64_t nk = f->n_bricks * BRICK_CELLS;
  {
    StageTimer t(TS_INIT, s);
    k_fill_u64<<<grid_1d(nk, 256), 256, 0, s>>>(keys, nk, EMPTY_KEY);
  }
  ScanArgs A = scan_args(f, keys, counters);
  {
    StageTimer t(TS_SCAN_FACE, s);
    A.n_items = f->nf;
    k_scan<KIND_FACE><<<grid_1d(f->nf, 64), 64, 0, s>>>(A);
  }
  if (f->n_epoly > 0) {
    StageTimer t(TS_SCAN_EDGE, s);
    A.items = f->epoly;
    A.n_items = f->n_epoly;
    A.counter = counters ? counters + 1 : nullptr;
    k_scan<KIND_EDGE><<<grid_1d(f->n_epoly, 64), 64, 0, s>>>(A);
  }
  if (f->n_vpoly > 0) {
    StageTimer t(TS_SCAN_VERT, s);
    A.items = f->vpoly;
    A.n_items = f->n_vpoly;
    A.counter = counters ? counters + 2 : nullptr;
    k_scan<KIND_VERT><<<grid_1d(f->n_vpoly, 64), 64, 0, s>>>(A);
  }
}

}  // namespace

extern "C" int csc_scan_convert(const csc_features* f, void* workspace_d, size_t ws_bytes, float* sdf_d,
                                int32_t* feat_d, int32_t* cell_d, int64_t* n_band_d, float* dense_d, void* stream) {
  if (!f || !f->valid || !workspace_d || !sdf_d || !feat_d || !cell_d || !n_band_d) return CSC_INVALID_ARG;
  WsLayout L = ws_layout(f);
  if (ws_bytes < L.total) return CSC_WORKSPACE_TOO_SMALL;
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)workspace_d;
  unsigned long long* keys = (unsigned long long*)(W + L.keys);
  int32_t* cnt = (int32_t*)(W + L.cnt);
  int32_t* tmp = (int32_t*)(W + L.scan);
  const int64_t nk = f->n_bricks * BRICK_CELLS;

  if (dense_d) {
    int64_t nd = (int64_t)f->grid.n[0] * f->grid.n[1] * f->grid.n[2];
    k_fill_f32<<<grid_1d(nd, 256), 256, 0, s>>>(dense_d, nd, __builtin_inff());
  }
  if (nk > 0) run_scans(f, keys, nullptr, s);
  hipError_t e;
  {
    StageTimer t(TS_COUNT, s);
    if (nk > 0) k_brick_count<<<(unsigned)f->n_bricks, 512, 0, s>>>(keys, cnt);
    e = exclusive_scan(cnt, cnt, f->n_bricks, tmp, n_band_d, nullptr, s);
  }
  if (e != hipSuccess) return fail_hip(e);
  if (nk > 0) {
    StageTimer t(TS_SIGN, s);
    SignArgs S;
    S.V = f->verts;
    S.T = f->tris;
    S.fn = f->face_n;
    S.edges = f->edges;
    S.face_edges = f->face_edges;
    S.vinfo = f->vinfo;
    S.brick_list = f->brick_list;
    S.keys = keys;
    S.boff = cnt;
    S.sdf = sdf_d;
    S.feat = feat_d;
    S.cell = cell_d;
    S.dense = dense_d;
    S.nf = f->nf;
    S.ne = f->ne;
    for (int k = 0; k < 3; k++) {
      S.o[k] = f->grid.origin[k];
      S.n[k] = f->grid.n[k];
      S.nb[k] = f->nb[k];
    }
    S.h = f->grid.h;
    k_sign<<<(unsigned)f->n_bricks, 512, 0, s>>>(S);
  }
  e = hipGetLastError();
  return e == hipSuccess ? CSC_OK : fail_hip(e);
}

extern "C" int csc_scan_convert_count(const csc_features* f, void* workspace_d, size_t ws_bytes, int64_t counts[3],
                                      void* stream) {
  if (!f || !f->valid || !workspace_d || !counts) return CSC_INVALID_ARG;
  WsLayout L = ws_layout(f);
  if (ws_bytes < L.total) return CSC_WORKSPACE_TOO_SMALL;
  hipStream_t s = (hipStream_t)stream;
  char* W = (char*)workspace_d;
  unsigned long long* keys = (unsigned long long*)(W + L.keys);
  unsigned long long* ctr = (unsigned long long*)(W + L.scan);  // reuses the scan scratch
  hipError_t e = hipMemsetAsync(ctr, 0, 3 * sizeof(unsigned long long), s);
  if (e != hipSuccess) return fail_hip(e);
  if (f->n_bricks > 0) run_scans(f, keys, ctr, s);
  unsigned long long h[3];
  e = hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e);
  for (int i = 0; i < 3; i++) counts[i] = (int64_t)h[i];
  return CSC_OK;
}
