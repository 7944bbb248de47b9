// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/csc.h"

namespace csc {

// The band store is allocated in bricks of BRICK^3 cells (BRICK a power of two,
// 4 or 8). A band about 2*band cells thick fills a brick of edge b to roughly
// 2 band / (2 band + b): 4-cell bricks hold more set keys, which shrinks the key
// initialisation and the brick count (-35%, -25% measured), but each small
// triangle then marks about 8 times as many bricks (the face pass ran 2-3 times
// longer, its scattered stores slowing the sort beside it) and the sign pass
// holds one key per lane instead of eight (+75%): 8-cell bricks stay the default.
#ifndef CSC_BRICK_SHIFT
#define CSC_BRICK_SHIFT 3
#endif
constexpr int BRICK_SHIFT = CSC_BRICK_SHIFT;
constexpr int BRICK = 1 << BRICK_SHIFT;            // band store brick edge (cells)
constexpr int BRICK_CELLS = BRICK * BRICK * BRICK;
constexpr int BRICK_ROUNDS = BRICK_CELLS / 64;     // keys per lane when one wavefront holds a brick
static_assert(BRICK_CELLS % 64 == 0 && BRICK_ROUNDS <= 8, "a brick fills whole wavefronts, at most 8 keys a lane");
// Position of cell (i, j, k) inside its brick: Morton order, the bits of the
// three in-brick coordinates interleaved (x lowest), so that 8 consecutive keys
// (64 bytes) hold a 2x2x2 block of cells and 16 (128 bytes) a 4x2x2 block. The
// cells one wavefront's atomics reach lie close together in all three axes: in
// this order they touch fewer cache lines than with rows of x (26 -> 19 lines
// of 64 bytes per instruction on a batch of 64 meshes, whose logged atomics
// then replay 31% faster).
__host__ __device__ inline int brick_local(int i, int j, int k) {
  int l = 0;
#pragma unroll
  for (int b = 0; b < BRICK_SHIFT; b++)
    l |= (((i >> b) & 1) << (3 * b)) | (((j >> b) & 1) << (3 * b + 1)) | (((k >> b) & 1) << (3 * b + 2));
  return l;
}
// the in-brick coordinates of position l (inverse of brick_local)
__host__ __device__ inline void brick_cell(int l, int& i, int& j, int& k) {
  i = j = k = 0;
#pragma unroll
  for (int b = 0; b < BRICK_SHIFT; b++) {
    i |= ((l >> (3 * b)) & 1) << b;
    j |= ((l >> (3 * b + 1)) & 1) << b;
    k |= ((l >> (3 * b + 2)) & 1) << b;
  }
}
constexpr unsigned long long EMPTY_KEY = ~0ull;

// device error bits gathered during a build or scan
enum : uint32_t {
  ERR_INDEX = 1u, ERR_REPEAT = 2u, ERR_NONFINITE = 4u, ERR_NONMANIFOLD = 8u, ERR_ORIENT = 16u,
  ERR_DEGENERATE = 32u, ERR_OVERFLOW = 64u
};

// device counters and statistics (int64 slots)
enum {
  ST_NE = 0, ST_NEPOLY, ST_NVPOLY, ST_NBRICKS,
  ST_E_CONVEX, ST_E_CONCAVE, ST_E_FLAT, ST_E_UNKNOWN,
  ST_V_CONVEX, ST_V_CONCAVE, ST_V_FLAT, ST_V_SADDLE, ST_V_RUFF,
  ST_ERR, ST_E_ABSORBED, ST_V_ABSORBED, ST_COUNT = 16
};

// One mesh of a batch: its grid, band and slice of the concatenated arrays.
struct MeshDesc {
  double origin[3];
  double h, inv_h, whd, epsd;
  float hf, whf, eps, band;
  int32_t n[3];
  int32_t nb[3];                // bricks per axis
  int32_t nt[3];                // tiles of 4x4x4 bricks per axis
  int32_t brick_base;           // first brick position of this mesh in the batch's brick space
  int32_t v_off, f_off, e_off;  // first vertex / face / edge of this mesh
  int32_t nv, nf, ne;
};

// Position of brick (bx, by, bz) in the batch's brick space: bricks are numbered
// tile by tile (tiles of 4x4x4 bricks, x fastest), and linearly inside a tile, so
// that consecutive brick slots (and the band list that follows their order) stay
// spatially compact.
constexpr int TILE = 4;
__host__ __device__ inline int64_t brick_pos(const MeshDesc& G, int bx, int by, int bz) {
  const int64_t tile = (bx >> 2) + (int64_t)G.nt[0] * ((by >> 2) + (int64_t)G.nt[1] * (bz >> 2));
  return G.brick_base + (tile << 6) + (bx & 3) + ((by & 3) << 2) + ((bz & 3) << 4);
}
__host__ __device__ inline void brick_coords(const MeshDesc& G, int64_t pos, int& bx, int& by, int& bz) {
  const int64_t p = pos - G.brick_base, tile = p >> 6;
  const int l = (int)(p & 63);
  const int tx = (int)(tile % G.nt[0]), ty = (int)((tile / G.nt[0]) % G.nt[1]);
  const int tz = (int)(tile / ((int64_t)G.nt[0] * G.nt[1]));
  bx = tx * 4 + (l & 3);
  by = ty * 4 + ((l >> 2) & 3);
  bz = tz * 4 + (l >> 4);
}

// Exclusive prefix sum of in[0..n) into out (may alias in). If total_i64 is not
// null the sum is stored there; if total_i32 is not null, also there. tmp must
// hold scan_tmp_ints(n) ints. Kernels only (safe inside a captured graph).
int64_t scan_tmp_ints(int64_t n);
// exclusive scan, in place, of nb tile sums by one block; *total_i64 gets the total
hipError_t scan_sums_inplace(int32_t* sums, int64_t nb, int64_t* total_i64, hipStream_t s);
hipError_t exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, int64_t* total_i64,
                          int32_t* total_i32, hipStream_t s);

// stable radix sort of n (key, value) pairs on the low `bits` key bits; vals_in
// null: the values are 0, 1, ..., n-1
size_t sort_pairs_tmp_bytes(int64_t n, int bits);
hipError_t sort_pairs(void* tmp, size_t tmp_bytes, const uint32_t* keys_in, uint32_t* keys_out,
                      const int32_t* vals_in, int32_t* vals_out, int64_t n, int bits, hipStream_t s);

int fail_hip(hipError_t e);  // records the HIP error text, returns CSC_HIP_ERROR
int check_device();          // CSC_OK or CSC_UNSUPPORTED_DEVICE / CSC_HIP_ERROR

// timed stages (csc_timing_*)
enum {
  TS_BUILD = 0, TS_INIT, TS_SCAN_FACE, TS_SCAN_EDGE, TS_SCAN_VERT, TS_COUNT, TS_SIGN, TS_BACKWARD,
  TS_SCAN_FACE_BIG, TS_SCAN_EDGE_BIG, TS_SCAN_VERT_BIG, TS_FILL, TS_SCAN_WIDE, N_STAGES
};

// whether stage timing is on (csc_timing_enable)
bool stage_timing_on();

// Records a pair of events around its scope on stream s when timing is enabled
// and the stream is not being captured into a graph.
class StageTimer {
 public:
  StageTimer(int stage, hipStream_t s);
  ~StageTimer();
  StageTimer(const StageTimer&) = delete;
  StageTimer& operator=(const StageTimer&) = delete;

 private:
  int stage_;
  hipStream_t s_;
  void* a_ = nullptr;
  void* b_ = nullptr;
  bool active_ = false;
};

// MI355X deals the workgroups of a launch to its 8 XCDs in turn (workgroup b to
// XCD b mod 8), and each XCD has an L2 of its own. xcd_block renumbers the
// workgroups so that each XCD takes one contiguous slice of the grid, so that
// neighbouring items that gather the same data meet in one L2. A bijection on
// [0, gridDim.x) for any grid size; a different dealing order costs locality,
// never correctness. Measured, it pays only in the vertex pass (fans of
// neighbouring vertices share corners and positions: -11%); where the work per
// item is uneven along the grid (polyhedron queues) a contiguous slice per XCD
// unbalances the XCDs, and the face and edge passes ran 10% slower with it.
#ifndef CSC_N_XCD
#define CSC_N_XCD 8
#endif
__device__ inline int64_t xcd_block() {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t per = nb / CSC_N_XCD, r = nb % CSC_N_XCD, x = b % CSC_N_XCD;
  return x * per + (x < r ? x : r) + b / CSC_N_XCD;
}

inline unsigned grid_1d(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

// largest m with table[m] <= x over table[0..n] (ascending, table[0] = 0 <= x)
template <typename T>
__host__ __device__ inline int find_segment(const T* table, int n, int64_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if ((int64_t)table[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace csc

// The handle: a batch of one or more meshes. Device arrays live in one arena.
// One 64-byte record per face, written by the build: corner j as (x, y, z, its
// global vertex index as the bits of w) for j = 0..2, then the unit normal
// (w = 0). A pass that needs a face's corners, vertex indices or normal reads
// one aligned 64-byte sector instead of gathering from the vertex array: faces
// near each other in space are often far apart in the input's order, and each
// scattered 12-byte gather costs a whole sector.
struct FaceRec {
  float4 c[3];
  float4 n;
};
static_assert(sizeof(FaceRec) == 64, "one sector per face");
__device__ inline int32_t rec_vertex(const float4& c) { return __float_as_int(c.w); }

struct csc_features {
  int32_t n_meshes = 0;
  std::vector<csc::MeshDesc> mesh;  // host copy of the descriptors
  const float* verts = nullptr;     // caller's vertices, all meshes concatenated
  int64_t nv = 0, nf = 0, ne = 0;   // totals over the batch
  int64_t nbt = 0;                  // bricks of all grids
  csc_options opt{};
  int sort_bits = 1;

  char* arena = nullptr;
  size_t arena_bytes = 0;

  csc::MeshDesc* d_mesh = nullptr;  // [n_meshes]
  int32_t* f_off = nullptr;         // [n_meshes+1] first face of each mesh
  int32_t* v_off = nullptr;         // [n_meshes+1] first vertex
  int32_t* brick_base = nullptr;    // [n_meshes+1] first brick
  int32_t* tris_g = nullptr;        // [nf][3] global vertex indices (sanitised)
  int32_t* face_mesh = nullptr;     // [nf]
  int32_t* vert_mesh = nullptr;     // [nv]
  int32_t* vtx_off = nullptr;       // [nv+1]
  int32_t* vtx_corners = nullptr;   // [3nf] per vertex its corners 3f+j, ascending
  int32_t* face_edges = nullptr;    // [3nf]
  int4* edges = nullptr;            // [ne] (a, b, f_left, f_right), global indices
  FaceRec* face_rec = nullptr;      // [nf] corners, vertex ids and unit normal of each face
  uint8_t* edge_cls = nullptr;      // [ne] class | side bits << 2
  float4* vinfo = nullptr;          // [nv] unit pseudonormal, cone aperture cosine
  uint32_t* vbits = nullptr;        // [nv] class bits
  int32_t* epoly = nullptr;         // [<= 2ne] (e << 1) | inward
  int32_t* vpoly = nullptr;         // [<= 2nv] (v << 1) | inward
  int32_t* brick_index = nullptr;   // [nbt] -> slot or -1
  int32_t* brick_list = nullptr;    // [nbt] slot -> brick
  int32_t* brick_mesh = nullptr;    // [nbt] slot -> mesh
  int32_t* first_slot = nullptr;    // [n_meshes+1] first slot of each mesh's bricks
  int32_t* t_a = nullptr;           // temporaries
  int32_t* t_b = nullptr;
  int32_t* t_c = nullptr;
  int32_t* t_scan = nullptr;
  void* t_sort = nullptr;           // radix sort scratch
  size_t t_sort_bytes = 0;
  int64_t* d_stats = nullptr;       // [ST_COUNT] counters; ST_ERR holds the error bits
  int64_t* h_stats = nullptr;       // pinned host mirror [ST_COUNT]
  // the build's brick marking runs on `side`, forked from and joined back into
  // the caller's stream with the two events (capturable: a parallel branch)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_geom = nullptr;     // the face records are written (the vertex and edge passes read them)
  int32_t* brick_flag = nullptr;    // [nbt + 1] brick marks of the build
  int32_t* t_scan2 = nullptr;       // scan temporaries of the side branch
  int32_t* t_eid = nullptr;         // [3nf + 1] edge id of each owned half-edge (prefix sum, side branch)
  uint8_t* fslack = nullptr;        // [nf] side slack of the face prism: the largest code of its absorbed
                                    // edges and vertices (1/1024 cells)
  uint8_t* eslack = nullptr;        // [ne] slack code of each absorbed edge (0: not absorbed)
  uint8_t* fabsorbed = nullptr;     // [nf] bit j: the edge from corner j absorbed; bit 3 + j: corner j's vertex
  int32_t* face_order = nullptr;    // [face_order_n] optional processing order of the face pass (own allocation)
  int64_t face_order_n = 0;

  bool built = false;               // device work queued for the current inputs
  bool synced = false;              // counts below read back since the last build
  bool classes_counted = false;     // the class statistics of the last build are in d_stats
  int64_t n_epoly = 0, n_vpoly = 0, n_bricks = 0;
  csc_feature_info info{};
};

namespace csc {
// status of a device-side error word
int status_from_errors(uint64_t err, int64_t ne_found, int64_t ne_expected);
}  // namespace csc
