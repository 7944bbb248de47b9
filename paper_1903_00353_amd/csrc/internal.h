// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/csc.h"

namespace csc {

constexpr int BRICK = 8;          // band store brick edge (cells)
constexpr int BRICK_CELLS = 512;  // BRICK^3
constexpr unsigned long long EMPTY_KEY = ~0ull;

// device error bits gathered during the build
enum : uint32_t {
  ERR_INDEX = 1u, ERR_REPEAT = 2u, ERR_NONFINITE = 4u, ERR_NONMANIFOLD = 8u, ERR_ORIENT = 16u,
  ERR_DEGENERATE = 32u, ERR_EDGECOUNT = 64u
};

// device statistics slots
enum {
  ST_NE = 0, ST_NEPOLY, ST_NVPOLY, ST_NBRICKS,
  ST_E_CONVEX, ST_E_CONCAVE, ST_E_FLAT, ST_E_UNKNOWN,
  ST_V_CONVEX, ST_V_CONCAVE, ST_V_FLAT, ST_V_SADDLE, ST_V_RUFF,
  ST_COUNT = 16
};

// Exclusive prefix sum of in[0..n) into out (may alias in). If total_i64 is not
// null the sum is stored there; if total_i32 is not null, also there. tmp must
// hold scan_tmp_ints(n) ints.
int64_t scan_tmp_ints(int64_t n);
hipError_t exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, int64_t* total_i64,
                          int32_t* total_i32, hipStream_t s);

// stable radix sort of n (key, value) pairs on the low `bits` key bits
size_t sort_pairs_tmp_bytes(int64_t n, int bits);
hipError_t sort_pairs(void* tmp, size_t tmp_bytes, const uint32_t* keys_in, uint32_t* keys_out,
                      const int32_t* vals_in, int32_t* vals_out, int64_t n, int bits, hipStream_t s);

int fail_hip(hipError_t e);  // records the HIP error text, returns CSC_HIP_ERROR

// timed stages (csc_timing_*)
enum { TS_BUILD = 0, TS_INIT, TS_SCAN_FACE, TS_SCAN_EDGE, TS_SCAN_VERT, TS_COUNT, TS_SIGN, TS_BACKWARD, N_STAGES };

// Records a pair of events around its scope on stream s when timing is enabled.
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
int check_device();          // CSC_OK or CSC_UNSUPPORTED_DEVICE / CSC_HIP_ERROR

inline unsigned grid_1d(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace csc

// The handle. Device arrays live in one arena allocation.
struct csc_features {
  const float* verts = nullptr;
  const int32_t* tris = nullptr;
  int64_t nv = 0, nf = 0, ne = 0;
  csc_grid grid{};
  csc_options opt{};
  int32_t nb[3] = {0, 0, 0};   // bricks per axis
  int64_t nbricks_total = 0;   // nb[0]*nb[1]*nb[2]

  char* arena = nullptr;
  size_t arena_bytes = 0;

  int32_t* vtx_off = nullptr;     // [nv+1]
  int32_t* vtx_faces = nullptr;   // [3nf], per vertex its corners 3f+j, ascending
  int32_t* face_edges = nullptr;  // [3nf]
  int4* edges = nullptr;          // [ne] (a, b, f_left, f_right)
  float4* face_n = nullptr;       // [nf] unit normal
  uint8_t* edge_cls = nullptr;    // [ne] class | side bits << 2
  float4* vinfo = nullptr;        // [nv] unit pseudonormal, cone aperture cosine
  uint32_t* vbits = nullptr;      // [nv] class bits
  int32_t* epoly = nullptr;       // [<= 2ne] (e << 1) | inward
  int32_t* vpoly = nullptr;       // [<= 2nv] (v << 1) | inward
  int32_t* brick_index = nullptr; // [nbricks_total] -> slot or -1
  int32_t* brick_list = nullptr;  // [nbricks_total] slot -> brick
  int32_t* t_a = nullptr;         // temporaries
  int32_t* t_b = nullptr;
  int32_t* t_c = nullptr;
  int32_t* t_scan = nullptr;
  void* t_sort = nullptr;         // radix sort scratch
  size_t t_sort_bytes = 0;
  int64_t* d_stats = nullptr;     // [ST_COUNT]
  uint32_t* d_err = nullptr;
  int64_t* h_stats = nullptr;     // pinned host mirror [ST_COUNT + 1]

  int64_t n_epoly = 0, n_vpoly = 0, n_bricks = 0;
  csc_feature_info info{};
  bool valid = false;
};
