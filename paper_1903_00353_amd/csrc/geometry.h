// Geometry and predicates shared by the device kernels (and evaluated on the host
// by the diagnostic entry points). Everything here is __host__ __device__.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace csc {

struct f3 { float x, y, z; };
struct d3 { double x, y, z; };

__host__ __device__ inline f3 mk(float x, float y, float z) { f3 r = {x, y, z}; return r; }
__host__ __device__ inline f3 operator+(f3 a, f3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__host__ __device__ inline f3 operator-(f3 a, f3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__host__ __device__ inline f3 operator*(f3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
__host__ __device__ inline float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ inline f3 cross(f3 a, f3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

__host__ __device__ inline d3 mkd(double x, double y, double z) { d3 r = {x, y, z}; return r; }
__host__ __device__ inline d3 operator+(d3 a, d3 b) { return mkd(a.x + b.x, a.y + b.y, a.z + b.z); }
__host__ __device__ inline d3 operator-(d3 a, d3 b) { return mkd(a.x - b.x, a.y - b.y, a.z - b.z); }
__host__ __device__ inline d3 operator*(d3 a, double s) { return mkd(a.x * s, a.y * s, a.z * s); }
__host__ __device__ inline double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ inline d3 cross(d3 a, d3 b) {
  return mkd(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double len(d3 a) { return sqrt(dot(a, a)); }
__host__ __device__ inline d3 tod(f3 a) { return mkd(a.x, a.y, a.z); }
__host__ __device__ inline f3 tof(d3 a) { return mk((float)a.x, (float)a.y, (float)a.z); }

// ---------------------------------------------------------------- exact sign
// Error-free transformations (Knuth's two-sum, fused-multiply-add two-product)
// and Shewchuk's growing of a non-overlapping expansion (Shewchuk, "Adaptive
// Precision Floating-Point Arithmetic and Fast Robust Geometric Predicates",
// 1997): the components sum exactly to the value, the last non-zero one carries
// its sign.
__host__ __device__ inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bv = s - a;
  double av = s - bv;
  e = (a - av) + (b - bv);
}
__host__ __device__ inline void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = fma(a, b, -p);
}
__host__ __device__ inline int grow_expansion(int n, double* e, double b) {
  double q = b;
  int m = 0;
  for (int i = 0; i < n; i++) {
    double s, t;
    two_sum(q, e[i], s, t);
    q = s;
    if (t != 0.0) e[m++] = t;
  }
  if (q != 0.0 || m == 0) e[m++] = q;
  return m;
}

// Exact sign of w . (u x v) for double vectors whose components are exact
// (differences of floats): each of the six cofactor products is split into four
// doubles by two_prod, and all 24 are summed into one expansion. Kept out of line:
// it runs only when the filter below cannot decide.
__host__ __device__ __attribute__((noinline)) inline int orient3d_exact(double ux, double uy, double uz, double vx,
                                                                      double vy, double vz, double wx, double wy,
                                                                      double wz) {
  const double P[6][3] = {{wx, uy, vz}, {-wx, uz, vy}, {wy, uz, vx}, {-wy, ux, vz}, {wz, ux, vy}, {-wz, uy, vx}};
  double e[32];
  int n = 0;
  for (int t = 0; t < 6; t++) {
    double p, pe, p1, e1, p2, e2;
    two_prod(P[t][0], P[t][1], p, pe);
    two_prod(p, P[t][2], p1, e1);
    two_prod(pe, P[t][2], p2, e2);
    n = grow_expansion(n, e, p1);
    n = grow_expansion(n, e, e1);
    n = grow_expansion(n, e, p2);
    n = grow_expansion(n, e, e2);
  }
  double top = e[n - 1];
  return top > 0 ? 1 : (top < 0 ? -1 : 0);
}

// Sign of (d - a) . ((b - a) x (c - a)) for single-precision points, evaluated
// exactly: +1, -1 or 0. Returns 2 if a coordinate difference is not exact in
// double precision (coordinates more than 2^29 apart in magnitude); callers
// treat that as "unknown".
__host__ __device__ inline int orient3d_sign(f3 a, f3 b, f3 c, f3 d) {
  double ux, uy, uz, vx, vy, vz, wx, wy, wz, e0, e1, e2, e3, e4, e5, e6, e7, e8;
  two_sum((double)b.x, -(double)a.x, ux, e0);
  two_sum((double)b.y, -(double)a.y, uy, e1);
  two_sum((double)b.z, -(double)a.z, uz, e2);
  two_sum((double)c.x, -(double)a.x, vx, e3);
  two_sum((double)c.y, -(double)a.y, vy, e4);
  two_sum((double)c.z, -(double)a.z, vz, e5);
  two_sum((double)d.x, -(double)a.x, wx, e6);
  two_sum((double)d.y, -(double)a.y, wy, e7);
  two_sum((double)d.z, -(double)a.z, wz, e8);
  if (e0 != 0.0 || e1 != 0.0 || e2 != 0.0 || e3 != 0.0 || e4 != 0.0 || e5 != 0.0 || e6 != 0.0 || e7 != 0.0 ||
      e8 != 0.0)
    return 2;
  const double t0 = wx * uy * vz, t1 = -(wx * uz * vy), t2 = wy * uz * vx, t3 = -(wy * ux * vz),
               t4 = wz * ux * vy, t5 = -(wz * uy * vx);
  const double det = ((t0 + t1) + (t2 + t3)) + (t4 + t5);
  const double perm = fabs(t0) + fabs(t1) + fabs(t2) + fabs(t3) + fabs(t4) + fabs(t5);
  // static filter: the rounding error of the sum above is far below 1e-12 * perm
  if (det > 1e-12 * perm) return 1;
  if (det < -1e-12 * perm) return -1;
  if (perm == 0.0) return 0;
  return orient3d_exact(ux, uy, uz, vx, vy, vz, wx, wy, wz);
}

// -------------------------------------------------------- feature classes
// Edge a->b runs counter-clockwise in its left face (third vertex c1); the right
// face has third vertex c2. The edge is convex when c2 lies below the left face's
// plane (Section 3.1: convex edges only need the outward extrusion, concave ones
// the inward one, flat ones none; Section 8.2).
enum { EDGE_FLAT = 0, EDGE_CONVEX = 1, EDGE_CONCAVE = 2, EDGE_UNKNOWN = 3 };
constexpr int EDGE_ABSORBED = 16;  // class byte: bits 0-1 class, 2-3 extruded sides, 4 absorbed by its faces
__host__ __device__ inline int classify_edge(f3 a, f3 b, f3 c1, f3 c2) {
  int s = orient3d_sign(a, b, c1, c2);
  if (s == 2) return EDGE_UNKNOWN;
  return s < 0 ? EDGE_CONVEX : (s > 0 ? EDGE_CONCAVE : EDGE_FLAT);
}

// Vertex record bits.
enum : uint32_t {
  V_POS = 1u,        // extrusion on the outward side
  V_NEG = 2u,        // extrusion on the inward side
  V_POS_HEMI = 4u,   // outward extrusion is a hemisphere (else a cone)
  V_NEG_HEMI = 8u,   // inward extrusion is a hemisphere
  V_CONVEX = 16u, V_CONCAVE = 32u, V_FLAT = 64u, V_SADDLE = 128u, V_RUFF = 256u,
  V_ABSORBED = 512u  // nearly flat: its region handed to the prisms of its faces
};
constexpr int V_SLACK_SHIFT = 16;  // bits 16-23 of the class word: the absorbed vertex's slack code

struct VertexClass {
  d3 axis;        // unit angle-weighted pseudonormal
  double cos_t;   // cone aperture: least n_i . axis over normals with n_i . axis > 0
  uint32_t bits;
};

// Running classification of one vertex from its incident faces, in double
// precision. Pass 1 accumulates N = sum_i alpha_i n_i (Eq. 8; alpha_i the corner
// angle, n_i the unit normal); pass 2 tests each one-ring neighbour against the
// plane through the vertex with normal N (Section 3.1, Section 3.2) and each
// normal against N (Section 3.3, Section 4.2).
struct VertexAccum {
  d3 n_alpha = {0, 0, 0};
  // corner at v of a triangle (v, p1, p2): alpha = atan2(|e1 x e2|, e1 . e2)
  __host__ __device__ inline void add_face(d3 v, d3 p1, d3 p2) {
    d3 e1 = p1 - v, e2 = p2 - v;
    d3 n = cross(e1, e2);
    double ln = len(n);
    if (!(ln > 0)) return;
    n_alpha = n_alpha + n * (atan2(ln, dot(e1, e2)) / ln);
  }
};

struct VertexTest {
  d3 axis;
  double nlen;
  int pos = 0, neg = 0, unc = 0, nonpos_normal = 0;
  double cos_t = 2.0;
  __host__ __device__ inline void init(d3 n_alpha) {
    nlen = len(n_alpha);
    axis = nlen > 0 ? n_alpha * (1.0 / nlen) : mkd(0, 0, 1);
  }
  // neighbour p of vertex v: which side of the pseudonormal plane
  __host__ __device__ inline void neighbour(d3 v, d3 p) {
    d3 r = p - v;
    double s = dot(r, axis);
    double tol = 1e-12 * len(r);
    if (s > tol) pos++;
    else if (s < -tol) neg++;
    else unc++;
  }
  // incident face normal (unnormalised cross product of the two corner edges)
  __host__ __device__ inline void normal(d3 v, d3 p1, d3 p2) {
    d3 n = cross(p1 - v, p2 - v);
    double ln = len(n);
    if (!(ln > 0)) return;
    double c = dot(n, axis) / ln;
    if (c > 0) { if (c < cos_t) cos_t = c; }
    else nonpos_normal = 1;
  }
  // ruff_mode 0: hemisphere where some normal points away from the axis, else cone
  // saddle_mode 0: cone and its reflection; 1: hemispheres on both sides; 2: none
  __host__ __device__ inline VertexClass finish(int ruff_mode, int saddle_mode, int force_both) const {
    VertexClass vc;
    vc.axis = axis;
    vc.cos_t = cos_t > 1.0 ? 1.0 : cos_t;
    uint32_t b = 0;
    if (!(nlen > 0)) {
      b = V_SADDLE | V_POS | V_NEG | V_POS_HEMI | V_NEG_HEMI;  // no usable axis: cover all
    } else if (pos == 0 && neg == 0) {
      b = V_FLAT;
    } else if (neg > 0 && pos == 0 && unc == 0) {
      b = V_CONVEX | V_POS;
    } else if (pos > 0 && neg == 0 && unc == 0) {
      b = V_CONCAVE | V_NEG;
    } else {
      b = V_SADDLE;
      if (saddle_mode == 0) b |= V_POS | V_NEG;
      else if (saddle_mode == 1) b |= V_POS | V_NEG | V_POS_HEMI | V_NEG_HEMI;
    }
    if (force_both) b |= V_POS | V_NEG;
    if (nonpos_normal) {
      b |= V_RUFF;
      if (ruff_mode == 0) b |= V_POS_HEMI | V_NEG_HEMI;
    }
    if (cos_t > 1.0) b |= V_POS_HEMI | V_NEG_HEMI;  // no normal points along the axis
    vc.bits = b;
    return vc;
  }
};

// ------------------------------------------------------------ distances
// Closest point of the closed triangle (a, b, c) to p by the Voronoi-region tests
// of Ericson, Real-Time Collision Detection (2005), section 5.1.5. Returns the
// region: 0 face, 1..3 local edge j-1 (corner j-1 to corner j mod 3), 4..6
// corner j-4; writes the barycentric weights of q. V3 / S: f3 / float on the
// scan path, d3 / double where the operands span many cells. RCP (float only):
// quotients through the hardware reciprocal (about 1 ulp) instead of a correctly
// rounded division, where weights feed a gradient rather than a distance.
template <typename S, bool RCP>
__host__ __device__ inline S tri_div(S a, S b) {
  if constexpr (RCP) return a * __builtin_amdgcn_rcpf(b);  // instantiated in device code only
  else return a / b;
}
template <typename V3, typename S, bool RCP = false>
__host__ __device__ inline int closest_triangle_t(V3 p, V3 a, V3 b, V3 c, V3& q, S w[3]) {
  const S zero = 0, one = 1;
  V3 ab = b - a, ac = c - a, ap = p - a;
  S d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= zero && d2 <= zero) { w[0] = one; w[1] = zero; w[2] = zero; q = a; return 4; }
  V3 bp = p - b;
  S d3v = dot(ab, bp), d4 = dot(ac, bp);
  if (d3v >= zero && d4 <= d3v) { w[0] = zero; w[1] = one; w[2] = zero; q = b; return 5; }
  S vc = d1 * d4 - d3v * d2;
  if (vc <= zero && d1 >= zero && d3v <= zero) {
    S t = tri_div<S, RCP>(d1, d1 - d3v);
    w[0] = one - t; w[1] = t; w[2] = zero; q = a + ab * t; return 1;
  }
  V3 cp = p - c;
  S d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= zero && d5 <= d6) { w[0] = zero; w[1] = zero; w[2] = one; q = c; return 6; }
  S vb = d5 * d2 - d1 * d6;
  if (vb <= zero && d2 >= zero && d6 <= zero) {
    S t = tri_div<S, RCP>(d2, d2 - d6);
    w[0] = one - t; w[1] = zero; w[2] = t; q = a + ac * t; return 3;
  }
  S va = d3v * d6 - d5 * d4;
  if (va <= zero && (d4 - d3v) >= zero && (d5 - d6) >= zero) {
    S t = tri_div<S, RCP>(d4 - d3v, (d4 - d3v) + (d5 - d6));
    w[0] = zero; w[1] = one - t; w[2] = t; q = b + (c - b) * t; return 2;
  }
  S den = tri_div<S, RCP>(one, va + vb + vc);
  S v = vb * den, ww = vc * den;
  w[0] = one - v - ww; w[1] = v; w[2] = ww;
  q = a + ab * v + ac * ww;
  return 0;
}

__host__ __device__ inline int closest_triangle(f3 p, f3 a, f3 b, f3 c, f3& q, float w[3]) {
  return closest_triangle_t<f3, float>(p, a, b, c, q, w);
}

// Closest point of the closed segment [a, b]; t is the weight of b.
template <typename V3, typename S>
__host__ __device__ inline V3 closest_segment_t(V3 p, V3 a, V3 b, S& t) {
  const S zero = 0, one = 1;
  V3 ab = b - a;
  S den = dot(ab, ab);
  S s = den > zero ? dot(p - a, ab) / den : zero;
  s = s < zero ? zero : (s > one ? one : s);
  t = s;
  return a + ab * s;
}

__host__ __device__ inline f3 closest_segment(f3 p, f3 a, f3 b, float& t) {
  return closest_segment_t<f3, float>(p, a, b, t);
}

__host__ __device__ inline float norm3(f3 a) { return sqrtf(dot(a, a)); }

}  // namespace csc
