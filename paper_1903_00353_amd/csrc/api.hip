// Error reporting, device check, handle bookkeeping and the host-side
// evaluation of the classification predicates.
#include <string.h>

#include <mutex>

#include "geometry.h"
#include "internal.h"

namespace {
thread_local char g_last_hip[256] = "";
std::mutex g_dev_mu;
int g_dev_ok[64];  // 0 unknown, 1 gfx950, 2 other
}  // namespace

namespace csc {

int fail_hip(hipError_t e) {
  const char* s = hipGetErrorString(e);
  strncpy(g_last_hip, s ? s : "unknown HIP error", sizeof(g_last_hip) - 1);
  g_last_hip[sizeof(g_last_hip) - 1] = 0;
  return CSC_HIP_ERROR;
}

int check_device() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e);
  if (dev < 0 || dev >= 64) return CSC_UNSUPPORTED_DEVICE;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if (g_dev_ok[dev] == 0) {
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return fail_hip(e);
    g_dev_ok[dev] = strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
  }
  return g_dev_ok[dev] == 1 ? CSC_OK : CSC_UNSUPPORTED_DEVICE;
}

}  // namespace csc

using namespace csc;

extern "C" const char* csc_error_string(int code) {
  switch (code) {
    case CSC_OK: return "ok";
    case CSC_INVALID_ARG: return "invalid argument";
    case CSC_NONMANIFOLD: return "surface is open or non-manifold (an edge without exactly two triangles)";
    case CSC_INCONSISTENT_ORIENTATION: return "inconsistent orientation (a directed edge occurs twice)";
    case CSC_DEGENERATE_FACE: return "degenerate (zero-area) triangle";
    case CSC_GRID_TOO_LARGE: return "grid too large";
    case CSC_OUT_OF_MEMORY: return "out of device memory";
    case CSC_HIP_ERROR: return "HIP runtime error";
    case CSC_WORKSPACE_TOO_SMALL: return "workspace too small";
    case CSC_UNSUPPORTED_DEVICE: return "unsupported device (gfx950 required)";
    default: return "unknown status";
  }
}

extern "C" const char* csc_last_hip_error(void) { return g_last_hip; }

extern "C" int csc_features_info(const csc_features* f, csc_feature_info* info) {
  if (!f || !f->synced || !info) return CSC_INVALID_ARG;
  *info = f->info;
  return CSC_OK;
}

extern "C" void csc_features_free(csc_features* f) {
  if (!f) return;
  if (f->side) (void)hipStreamSynchronize(f->side);
  if (f->arena) (void)hipFree(f->arena);
  if (f->face_order) (void)hipFree(f->face_order);
  if (f->h_stats) (void)hipHostFree(f->h_stats);
  if (f->ev_fork) (void)hipEventDestroy(f->ev_fork);
  if (f->ev_join) (void)hipEventDestroy(f->ev_join);
  if (f->ev_geom) (void)hipEventDestroy(f->ev_geom);
  if (f->side) (void)hipStreamDestroy(f->side);
  delete f;
}

extern "C" int csc_classify_edge(const float a[3], const float b[3], const float c1[3], const float c2[3]) {
  if (!a || !b || !c1 || !c2) return -CSC_INVALID_ARG;
  return classify_edge(mk(a[0], a[1], a[2]), mk(b[0], b[1], b[2]), mk(c1[0], c1[1], c1[2]), mk(c2[0], c2[1], c2[2]));
}

extern "C" int csc_classify_vertex(const float v[3], const float* ring, int32_t n_faces, const csc_options* opt,
                                   double axis[3], double* cos_t) {
  if (!v || !ring || n_faces <= 0 || !axis || !cos_t) return -CSC_INVALID_ARG;
  csc_options o = {1e-3f, 0, 0, 0, {0, 0, 0}, 0, 0.f, 0, 0, 0};
  if (opt) o = *opt;
  d3 pv = mkd(v[0], v[1], v[2]);
  VertexAccum acc;
  for (int i = 0; i < n_faces; i++) {
    const float* p = ring + 6 * i;
    acc.add_face(pv, mkd(p[0], p[1], p[2]), mkd(p[3], p[4], p[5]));
  }
  VertexTest t;
  t.init(acc.n_alpha);
  for (int i = 0; i < n_faces; i++) {
    const float* p = ring + 6 * i;
    d3 p1 = mkd(p[0], p[1], p[2]), p2 = mkd(p[3], p[4], p[5]);
    t.neighbour(pv, p1);
    t.normal(pv, p1, p2);
  }
  VertexClass vc = t.finish(o.ruff_mode, o.saddle_mode, o.force_both_sides);
  axis[0] = vc.axis.x;
  axis[1] = vc.axis.y;
  axis[2] = vc.axis.z;
  *cos_t = vc.cos_t;
  return (int)vc.bits;
}
