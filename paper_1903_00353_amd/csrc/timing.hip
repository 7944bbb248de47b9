// Optional per-stage timing with HIP events recorded on the caller's stream.
#include <mutex>
#include <vector>

#include "internal.h"

namespace {
struct Rec {
  int stage;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_pending;
double g_ms[csc::N_STAGES];
int64_t g_calls[csc::N_STAGES];
const char* g_names[csc::N_STAGES] = {"build_features", "init_keys",      "scan_faces",     "scan_edges",
                                      "scan_vertices",  "brick_count",    "sign",           "backward",
                                      "scan_faces_big", "scan_edges_big", "scan_vertices_big",
                                      "interior_fill",  "scan_wide"};

void drain_locked() {
  for (Rec& r : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      g_ms[r.stage] += ms;
      g_calls[r.stage] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_pending.clear();
}
}  // namespace

namespace csc {

bool stage_timing_on() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_on;
}

StageTimer::StageTimer(int stage, hipStream_t s) : stage_(stage), s_(s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  if (hipEventCreate((hipEvent_t*)&a_) != hipSuccess) return;
  if (hipEventCreate((hipEvent_t*)&b_) != hipSuccess) {
    (void)hipEventDestroy((hipEvent_t)a_);
    return;
  }
  active_ = hipEventRecord((hipEvent_t)a_, s_) == hipSuccess;
}

StageTimer::~StageTimer() {
  if (!active_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipEventRecord((hipEvent_t)b_, s_);
  g_pending.push_back(Rec{stage_, (hipEvent_t)a_, (hipEvent_t)b_});
}

}  // namespace csc

extern "C" int csc_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  return CSC_OK;
}

extern "C" int csc_timing_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  for (int i = 0; i < csc::N_STAGES; i++) {
    g_ms[i] = 0;
    g_calls[i] = 0;
  }
  return CSC_OK;
}

extern "C" int csc_timing_read(double* ms, int64_t* calls, int32_t n) {
  if (!ms || !calls || n < 0) return CSC_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  for (int i = 0; i < n && i < csc::N_STAGES; i++) {
    ms[i] = g_ms[i];
    calls[i] = g_calls[i];
  }
  return CSC_OK;
}

extern "C" const char* csc_timing_stage_name(int32_t stage) {
  return stage >= 0 && stage < csc::N_STAGES ? g_names[stage] : "";
}
