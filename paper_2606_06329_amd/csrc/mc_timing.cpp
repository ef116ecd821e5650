// Stage timers: hipEvent pairs around every kernel launch while enabled.
#include <mutex>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/mecuco.h"
#include "mc_internal.h"

namespace {

struct Rec {
  int stage;
  hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_open;          // recorded, not yet read
std::vector<hipEvent_t> g_pool;   // reusable events
hipEvent_t g_pending[MC_STAGE_COUNT];
bool g_has_pending[MC_STAGE_COUNT] = {};

const char* kNames[MC_STAGE_COUNT] = {"knn_colsum", "knn_mean", "knn_center", "knn_stats",
                                       "knn_gemm_topk", "knn_rerank", "curv_fast", "curv_exact",
                                       "curv_backward", "knn_column_topk", "knn_rescan",
                                       "curv_gram", "curv_eigen", "curv_range"};

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

namespace mc {

void timing_begin(int stage, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on || stage < 0 || stage >= MC_STAGE_COUNT) return;
  hipEvent_t e = take();
  if (!e) return;
  if (hipEventRecord(e, s) != hipSuccess) {   // no timing for this launch; leave no error behind
    (void)hipGetLastError();
    g_pool.push_back(e);
    return;
  }
  g_pending[stage] = e;
  g_has_pending[stage] = true;
}

void timing_end(int stage, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on || stage < 0 || stage >= MC_STAGE_COUNT || !g_has_pending[stage]) return;
  hipEvent_t e = take();
  g_has_pending[stage] = false;
  if (!e) {
    g_pool.push_back(g_pending[stage]);
    return;
  }
  if (hipEventRecord(e, s) != hipSuccess) {
    (void)hipGetLastError();
    g_pool.push_back(g_pending[stage]);
    g_pool.push_back(e);
    return;
  }
  g_open.push_back(Rec{stage, g_pending[stage], e});
}

}  // namespace mc

extern "C" {

int mc_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  return MC_OK;
}

int mc_timing_read(int32_t stage, double* total_ms, int64_t* launches) {
  if (stage < 0 || stage >= MC_STAGE_COUNT || !total_ms || !launches) return MC_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  double tot = 0.0;
  int64_t cnt = 0;
  std::vector<Rec> keep;
  for (const Rec& r : g_open) {
    if (r.stage != stage) {
      keep.push_back(r);
      continue;
    }
    if (hipEventSynchronize(r.b) != hipSuccess) return MC_ELAUNCH;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return MC_ELAUNCH;
    tot += ms;
    ++cnt;
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_open.swap(keep);
  *total_ms = tot;
  *launches = cnt;
  return MC_OK;
}

const char* mc_stage_name(int32_t stage) {
  if (stage < 0 || stage >= MC_STAGE_COUNT) return "unknown";
  return kNames[stage];
}

}  // extern "C"
