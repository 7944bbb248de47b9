// Adjoint of the band values with respect to the vertex positions.
//
// With the closest feature of each band cell held fixed (the minimum over
// features is attained there: envelope theorem), SDF(c) = s |c - q| with
// q = sum_k w_k x_k on the feature, so dSDF/dx_k = -s w_k (c - q) / |c - q|.
// Each band cell scatters grad_sdf(c) * dSDF/dx_k into its 1-3 vertices.
#include "geometry.h"
#include "internal.h"
#include "wave.h"

namespace csc {

struct BwdArgs {
  const float* V;
  const FaceRec* frec;       // [nf] corners, vertex indices, unit normal
  const int4* edges;
  const MeshDesc* md;
  const float* sdf;
  const int32_t* feat;       // each mesh's own feature ids
  const int32_t* cell;       // each mesh's own linear cell index
  const float* gsdf;         // dL/dSDF per band cell; null: L = sum of SDF^2, so 2 SDF
  const int64_t* band_off;   // [n_meshes+1] band offsets, or null (one mesh)
  const int64_t* n_dev;      // one mesh: optional device band size
  float* grad;
  int64_t n;                 // launch bound (and band size if nothing is on the device)
  int n_meshes;
};

__device__ inline f3 relb(const float* V, int64_t i, d3 c) {
  return tof(mkd((double)V[3 * i] - c.x, (double)V[3 * i + 1] - c.y, (double)V[3 * i + 2] - c.z));
}
__device__ inline f3 relv(float4 p, d3 c) {
  return tof(mkd((double)p.x - c.x, (double)p.y - c.y, (double)p.z - c.z));
}

// the per-cell inputs of one band cell; gs = 0 past the end of the run
struct BwCell {
  float gs, sd;
  int32_t lin, lf;
};

__device__ inline BwCell load_cell(const BwdArgs& P, int64_t i, int64_t end) {
  BwCell c = {0.f, 0.f, 0, 0};
  if (i < end) {
    c.sd = P.sdf[i];
    c.gs = P.gsdf ? P.gsdf[i] : 2.f * c.sd;  // fused loss: exactly torch's 2 * sdf
    c.lin = P.cell[i];
    c.lf = P.feat[i];
  }
  return c;
}

// what a thread needs of the mesh its cells belong to, kept in registers until
// its cells reach the next mesh
struct BwMesh {
  double ox, oy, oz, h, inv_n0, inv_n1;
  int n0, n1, nf, ne, f_off, e_off, v_off;
  int64_t end;  // first band cell past this mesh
};

__device__ inline BwMesh load_mesh(const BwdArgs& P, int m) {
  const MeshDesc& G = P.md[m];
  BwMesh M;
  M.ox = G.origin[0];
  M.oy = G.origin[1];
  M.oz = G.origin[2];
  M.h = G.h;
  M.n0 = G.n[0];
  M.n1 = G.n[1];
  M.inv_n0 = 1.0 / G.n[0];
  M.inv_n1 = 1.0 / G.n[1];
  M.nf = G.nf;
  M.ne = G.ne;
  M.f_off = G.f_off;
  M.e_off = G.e_off;
  M.v_off = G.v_off;
  M.end = P.band_off ? P.band_off[m + 1] : INT64_MAX;
  return M;
}

// floor(a / d) for 0 <= a < 2^31 and 0 < d < 2^16, with inv = 1 / d rounded: the
// product is within one of the quotient, and the remainder puts it right
__device__ inline int div_floor(int a, int d, double inv) {
  int q = (int)((double)a * inv);
  const int64_t r = (int64_t)a - (int64_t)q * d;
  q += r >= d ? 1 : 0;
  q -= r < 0 ? 1 : 0;
  return q;
}

// one step of the segmented inclusive scan over the lanes: add the partial sums
// of the source lane where it lies in the same run. Row shifts 1, 2, 4, 8 scan
// each row of 16; the two broadcasts carry row 0 into row 1 and row 2 into
// row 3, then rows 0-1 into rows 2-3.
template <int CTRL, int ROWS>
__device__ inline void seg_step(int run, f3 (&con)[3]) {
  const bool take = dpp_i<CTRL, ROWS>(-1, run) == run;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const float ux = dpp_f<CTRL, ROWS>(0.f, con[k].x), uy = dpp_f<CTRL, ROWS>(0.f, con[k].y),
                uz = dpp_f<CTRL, ROWS>(0.f, con[k].z);
    if (take) con[k] = con[k] + mk(ux, uy, uz);
  }
}

// The pass is bound by the latency of its loads and of the table's LDS round
// trips, so occupancy comes first: a 16 KB table per block of 256 lets 8 blocks
// share a CU, and the register budget is held to 64 for 8 wavefronts per SIMD.
constexpr int BW_THREADS = 256;
constexpr int BW_WAVES_PER_SIMD = 8;
constexpr int BW_SLOTS = 512;                 // hash table of (vertex, 3 partial sums) per block
constexpr int BW_FLUSH = 256;                 // flush once more slots than this are taken
constexpr int BW_PROBES = 16;                 // a vertex not placed within this many slots goes to HBM
constexpr int BW_BLOCKS = 2048;               // persistent grid: 8 resident blocks of 256 per CU
// LDS adds of floats are slow on this chip where 64-bit integer adds are not,
// so the table sums in fixed point: c * 2^fx, rounded to an integer, when its
// magnitude is below 2^42 (no overflow; the rounding is at most 2^-41 of the
// block's largest term), otherwise (a term far larger than the block's first
// chunk's, or not finite) c goes straight to the gradient. Terms that round to
// zero add nothing.
__device__ inline void add_fixed(unsigned long long* slot, float c, int fx, float* direct) {
  const float v = ldexpf(c, fx);
  if (fabsf(v) < 4398046511104.f) {  // |v| < 2^42
    const long long iv = (long long)rintf(v);
    if (iv != 0) atomicAdd(slot, (unsigned long long)iv);
  } else if (c != 0.f) {
    atomicAdd(direct, c);
  }
}

// max(m, |a|) over finite a only
__device__ inline float fmax_finite(float m, float a) {
  const float b = fabsf(a);
  return b <= __FLT_MAX__ ? fmaxf(m, b) : m;
}

__device__ inline float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

constexpr int log2i(int x) { return x <= 1 ? 0 : 1 + log2i(x >> 1); }
constexpr int BW_HASH_SHIFT = 32 - log2i(BW_SLOTS);
static_assert((BW_SLOTS & (BW_SLOTS - 1)) == 0 && BW_FLUSH < BW_SLOTS, "table size");

// Each block takes one contiguous run of band cells (band cells follow the
// tile-ordered bricks, so a run covers a compact piece of surface and shares most
// of its vertices) in chunks of one cell per thread. Contributions are summed per
// vertex in an LDS hash table (linear probing) that is added to the global
// gradient once it is more than BW_FLUSH slots full, and at the end: one global
// add per vertex, axis and flush instead of one per band cell. Probing stops
// after BW_PROBES slots; such a vertex's contribution goes to the gradient
// directly, so a full table costs time, never correctness.
__global__ __launch_bounds__(BW_THREADS, BW_WAVES_PER_SIMD) void k_backward(BwdArgs P) {
  __shared__ int s_key[BW_SLOTS];
  __shared__ unsigned long long s_acc[3][BW_SLOTS];  // fixed-point sums, two's complement
  __shared__ int s_used;
  __shared__ float s_gmax[BW_THREADS / 64];
  int64_t lim = P.n;
  if (P.band_off) lim = P.band_off[P.n_meshes] < lim ? P.band_off[P.n_meshes] : lim;
  else if (P.n_dev && *P.n_dev < lim) lim = *P.n_dev;
  // this block's run [c0, c1), a whole number of chunks
  const int64_t chunks = (lim + BW_THREADS - 1) / BW_THREADS;
  const int64_t per = (chunks + gridDim.x - 1) / gridDim.x;
  const int64_t c0 = blockIdx.x * per * BW_THREADS;
  const int64_t c1 = min(lim, c0 + per * BW_THREADS);
  if (c0 >= c1) return;  // block-uniform
  for (int k = threadIdx.x; k < BW_SLOTS; k += BW_THREADS) {
    s_key[k] = -1;
    s_acc[0][k] = s_acc[1][k] = s_acc[2][k] = 0ull;
  }
  if (threadIdx.x == 0) s_used = 0;
  // Fixed-point scale of this block: 2^fx, with fx such that the largest finite
  // |dL/dSDF| of the block's first chunk scales to just below 2^40. Every term is
  // bounded by its cell's |dL/dSDF| (|g| = 1, 0 <= w <= 1). A scaled term of
  // magnitude below 2^42 is rounded to an integer (at most 2^-41 of the largest
  // term; exact from 2^23 up, where the float is integer-valued) and summed
  // exactly in 64-bit integers (a slot gets fewer than 2^20 terms between
  // flushes: no overflow), in any order. Larger terms (much larger than the first
  // chunk's, or non-finite) are added to the gradient as floats: the scale decides
  // how fast the sum goes, not whether it is right.
  float gmax = 0.f;
  if (c0 + threadIdx.x < c1)
    gmax = fmax_finite(0.f, P.gsdf ? P.gsdf[c0 + threadIdx.x] : 2.f * P.sdf[c0 + threadIdx.x]);
  gmax = wave_max(gmax);
  if ((threadIdx.x & 63) == 0) s_gmax[threadIdx.x >> 6] = gmax;
  __syncthreads();
#pragma unroll
  for (int w = 0; w < BW_THREADS / 64; w++) gmax = fmaxf(gmax, s_gmax[w]);
  int gexp = 0;
  (void)frexpf(gmax, &gexp);  // gmax < 2^gexp
  const int fx = 40 - gexp;
  // the mesh of this thread's first cell; a thread past the end of the band
  // (whose cells are never used) takes the last mesh, so that every descriptor
  // and offset it reads exists
  int m = P.band_off ? find_segment(P.band_off, P.n_meshes + 1, c0 + threadIdx.x) : 0;
  if (m > P.n_meshes - 1) m = P.n_meshes - 1;
  BwMesh M = load_mesh(P, m);
  for (int64_t base = c0; base < c1; base += BW_THREADS) {
    const int64_t i = base + threadIdx.x;
    const BwCell cur = load_cell(P, i, c1);
    const float gs = cur.gs;
    // this cell's contribution to each vertex k of its feature: f_k * g
    int32_t vid[3] = {-1, -1, -1};
    f3 con[3] = {mk(0.f, 0.f, 0.f), mk(0.f, 0.f, 0.f), mk(0.f, 0.f, 0.f)};
    int64_t fkey = -1 - (int64_t)threadIdx.x;  // unique unless the cell contributes
    if (gs != 0.f) {
      if (i >= M.end) {  // cells only move forward through the meshes
        while (i >= P.band_off[m + 1]) m++;
        M = load_mesh(P, m);
      }
      const int32_t lin = cur.lin, lf = cur.lf;
      const int row = div_floor(lin, M.n0, M.inv_n0), ck = div_floor(row, M.n1, M.inv_n1);
      const int ci = lin - row * M.n0, cj = row - ck * M.n1;
      const d3 c = mkd(M.ox + (ci + 0.5) * M.h, M.oy + (cj + 0.5) * M.h, M.oz + (ck + 0.5) * M.h);
      const f3 zero = mk(0.f, 0.f, 0.f);
      f3 q;
      float w[3] = {0.f, 0.f, 0.f};
      int mcount;
      int32_t v3[3];
      if (lf < M.nf) {
        const int64_t f = (int64_t)M.f_off + lf;
        const FaceRec& R = P.frec[f];  // one sector: corners and vertex indices
        const float4 ra = R.c[0], rb = R.c[1], rc = R.c[2];
        v3[0] = rec_vertex(ra);
        v3[1] = rec_vertex(rb);
        v3[2] = rec_vertex(rc);
        closest_triangle_t<f3, float, true>(zero, relv(ra, c), relv(rb, c), relv(rc, c), q, w);
        mcount = 3;
      } else if (lf < M.nf + M.ne) {
        int4 E = P.edges[(int64_t)M.e_off + (lf - M.nf)];
        v3[0] = E.x;
        v3[1] = E.y;
        float t;
        q = closest_segment(zero, relb(P.V, E.x, c), relb(P.V, E.y, c), t);
        w[0] = 1.f - t;
        w[1] = t;
        mcount = 2;
      } else {
        v3[0] = M.v_off + (lf - M.nf - M.ne);
        q = relb(P.V, v3[0], c);
        w[0] = 1.f;
        mcount = 1;
      }
      const float dd = dot(q, q);
      if (dd > 0.f) {
        const float s = cur.sd < 0.f ? -1.f : 1.f;
        // c - q = -q in this frame; g = s (c - q) / |c - q| (hardware reciprocal
        // square root, about 1 ulp: the pass is bound by its vector instructions)
        const f3 g = q * (-s * rsqrtf(dd));
        for (int k = 0; k < 3; k++) {
          if (k < mcount) {
            vid[k] = v3[k];
            con[k] = g * (-gs * w[k]);
          }
        }
        fkey = ((int64_t)m << 32) | (uint32_t)lf;
      }
    }
    // Consecutive band cells often share their feature (large triangles cover many
    // cells). When a wavefront holds enough such runs of equal feature in
    // consecutive lanes, each run is first summed across its lanes (segmented
    // inclusive scan) and only its last lane touches the table: far fewer
    // conflicting LDS atomics on the same few slots. A feature can come back in
    // a later, separate run of the same wavefront, so runs are told apart by a
    // run number (count of run heads up to the lane), not by the feature. All
    // lane moves are DPP operands of vector instructions, which leaves the LDS
    // to the table.
    const int lane = threadIdx.x & 63;
    const int klo = (int)fkey, khi = (int)(fkey >> 32);
    // every lane moves both halves before anything is compared: a DPP read from a
    // lane switched off by a branch would return the fallback
    const int nlo = dpp_i<DPP_WAVE_SHL1>(~klo, klo), nhi = dpp_i<DPP_WAVE_SHL1>(~khi, khi);
    const int plo = dpp_i<DPP_WAVE_SHR1>(~klo, klo), phi = dpp_i<DPP_WAVE_SHR1>(~khi, khi);
    const bool same_next = (nlo == klo) & (nhi == khi);
    const bool same_prev = (plo == klo) & (phi == khi);
    bool owner = fkey >= 0;
    if (__popcll(__ballot(same_next)) >= 8) {
      const unsigned long long heads = __ballot(!same_prev);
      const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
      const int run = __popcll(heads & upto);
      seg_step<DPP_ROW_SHR1, 0xf>(run, con);
      seg_step<DPP_ROW_SHR2, 0xf>(run, con);
      seg_step<DPP_ROW_SHR4, 0xf>(run, con);
      seg_step<DPP_ROW_SHR8, 0xf>(run, con);
      seg_step<DPP_ROW_BCAST15, 0xa>(run, con);
      seg_step<DPP_ROW_BCAST31, 0xc>(run, con);
      owner = owner && !same_next;
    }
    int n_new = 0;
    if (owner) {
      unsigned h[3];
      int old[3];
#pragma unroll
      for (int k = 0; k < 3; k++) {
        h[k] = ((unsigned)vid[k] * 2654435761u) >> BW_HASH_SHIFT;
        old[k] = vid[k] >= 0 ? atomicCAS(&s_key[h[k]], -1, vid[k]) : vid[k];
      }
#pragma unroll
      for (int k = 0; k < 3; k++) {
        if (vid[k] < 0) continue;
        for (int probe = 1; old[k] != -1 && old[k] != vid[k] && probe < BW_PROBES; probe++) {
          h[k] = (h[k] + 1) & (BW_SLOTS - 1);
          old[k] = atomicCAS(&s_key[h[k]], -1, vid[k]);
        }
        if (old[k] == -1 || old[k] == vid[k]) {
          if (old[k] == -1) n_new++;
          add_fixed(&s_acc[0][h[k]], con[k].x, fx, P.grad + 3 * (int64_t)vid[k]);
          add_fixed(&s_acc[1][h[k]], con[k].y, fx, P.grad + 3 * (int64_t)vid[k] + 1);
          add_fixed(&s_acc[2][h[k]], con[k].z, fx, P.grad + 3 * (int64_t)vid[k] + 2);
        } else {  // crowded neighbourhood: straight to the gradient
          atomicAdd(P.grad + 3 * (int64_t)vid[k], con[k].x);
          atomicAdd(P.grad + 3 * (int64_t)vid[k] + 1, con[k].y);
          atomicAdd(P.grad + 3 * (int64_t)vid[k] + 2, con[k].z);
        }
      }
    }
    {
      // new slots of the wavefront, counted with ballots: one add to s_used
      const int c = __popcll(__ballot(n_new >= 1)) + __popcll(__ballot(n_new >= 2)) + __popcll(__ballot(n_new >= 3));
      if (lane == 0 && c) atomicAdd(&s_used, c);
    }
    __syncthreads();
    const int used = s_used;
    const bool last = base + BW_THREADS >= c1;
    __syncthreads();  // every thread has read s_used before the next chunk changes it
    if (!last && used <= BW_FLUSH) continue;  // block-uniform: room for another chunk
    // flush: consecutive lanes add the three components of one vertex (a wave
    // instruction covers about 21 slots in 12-byte runs); the table is then
    // more than BW_FLUSH / BW_SLOTS full, except at the end of the run
    for (int k = threadIdx.x; k < 3 * BW_SLOTS; k += BW_THREADS) {
      const int slot = k / 3, cmp = k - 3 * slot;
      const int v = s_key[slot];
      const long long q = (long long)s_acc[cmp][slot];
      if (v >= 0 && q != 0) atomicAdd(P.grad + 3 * (int64_t)v + cmp, (float)ldexp((double)q, -fx));
    }
    __syncthreads();
    if (last) break;
    for (int k = threadIdx.x; k < BW_SLOTS; k += BW_THREADS) {
      s_key[k] = -1;
      s_acc[0][k] = s_acc[1][k] = s_acc[2][k] = 0ull;
    }
    if (threadIdx.x == 0) s_used = 0;
    __syncthreads();
  }
}

}  // namespace csc

using namespace csc;

namespace {

int backward_impl(const csc_features* f, const float* sdf_d, const int32_t* feat_d, const int32_t* cell_d, int64_t n,
                  const int64_t* n_dev, const int64_t* band_off, const float* grad_sdf_d, float* grad_verts_d,
                  hipStream_t s) {
  BwdArgs A;
  A.V = f->verts;
  A.frec = f->face_rec;
  A.edges = f->edges;
  A.md = f->d_mesh;
  A.sdf = sdf_d;
  A.feat = feat_d;
  A.cell = cell_d;
  A.gsdf = grad_sdf_d;
  A.band_off = band_off;
  A.n_dev = n_dev;
  A.grad = grad_verts_d;
  A.n = n;
  A.n_meshes = f->n_meshes;
  StageTimer t(TS_BACKWARD, s);
  const int64_t chunks = (n + BW_THREADS - 1) / BW_THREADS;
  k_backward<<<(int)(chunks < BW_BLOCKS ? chunks : BW_BLOCKS), BW_THREADS, 0, s>>>(A);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CSC_OK : fail_hip(e);
}

}  // namespace

extern "C" int csc_sdf_backward(const csc_features* f, const float* sdf_d, const int32_t* feat_d,
                                const int32_t* cell_d, int64_t n_band, const int64_t* n_band_d,
                                const float* grad_sdf_d, float* grad_verts_d, void* stream) {
  if (!f || !f->built || n_band < 0 || !grad_verts_d || f->n_meshes != 1) return CSC_INVALID_ARG;
  if (n_band > 0 && (!sdf_d || !feat_d || !cell_d)) return CSC_INVALID_ARG;
  if (n_band == 0) return CSC_OK;
  return backward_impl(f, sdf_d, feat_d, cell_d, n_band, n_band_d, nullptr, grad_sdf_d, grad_verts_d,
                       (hipStream_t)stream);
}

extern "C" int csc_sdf_backward_batched(const csc_features* f, const float* sdf_d, const int32_t* feat_d,
                                        const int32_t* cell_d, int64_t max_band, const int64_t* band_off_d,
                                        const float* grad_sdf_d, float* grad_verts_d, void* stream) {
  if (!f || !f->built || max_band < 0 || !grad_verts_d || !band_off_d) return CSC_INVALID_ARG;
  if (max_band > 0 && (!sdf_d || !feat_d || !cell_d)) return CSC_INVALID_ARG;
  if (max_band == 0) return CSC_OK;
  return backward_impl(f, sdf_d, feat_d, cell_d, max_band, nullptr, band_off_d, grad_sdf_d, grad_verts_d,
                       (hipStream_t)stream);
}
