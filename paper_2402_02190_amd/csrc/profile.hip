// Per-kernel timing with HIP events, for roofline measurement.
//
// While profiling is on, every kernel launch of the library is bracketed by
// two events recorded on the launch's own stream, and tagged with a short
// kernel-family name and its algorithmic work (FLOPs for GEMMs, compulsory
// HBM bytes for the memory-bound kernels).  Launches on a stream being
// captured are not recorded.
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace cpra {

namespace {

struct Rec {
  std::string name;
  hipEvent_t a, b;
  double flops, bytes, gather;
};

struct Summary {
  std::string name;
  int64_t launches = 0;
  double total_ms = 0, flops = 0, bytes = 0, gather = 0;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::vector<Summary> g_summary;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

thread_local int t_suspended = 0;

}  // namespace

ProfSuspend::ProfSuspend() { ++t_suspended; }
ProfSuspend::~ProfSuspend() { --t_suspended; }

ProfScope::ProfScope(const char* name, hipStream_t stream, double flops, double bytes, double gather)
    : active_(false), stream_(stream) {
  if (!g_on || t_suspended) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t a = get_event(), b = get_event();
  if (!a || !b) return;
  hipEventRecord(a, stream);
  g_recs.push_back(Rec{name, a, b, flops, bytes, gather});
  idx_ = g_recs.size() - 1;
  active_ = true;
}

ProfScope::~ProfScope() {
  if (!active_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEventRecord(g_recs[idx_].b, stream_);
}

}  // namespace cpra

extern "C" {

cpra_status cpra_profile_begin(void) {
  using namespace cpra;
  std::lock_guard<std::mutex> lk(g_mu);
  for (Rec& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  g_summary.clear();
  g_on = true;
  return CPRA_OK;
}

cpra_status cpra_profile_stop(void) {
  std::lock_guard<std::mutex> lk(cpra::g_mu);
  cpra::g_on = false;
  return CPRA_OK;
}

cpra_status cpra_profile_collect(void) {
  using namespace cpra;
  std::lock_guard<std::mutex> lk(g_mu);
  std::unordered_map<std::string, size_t> where;
  for (size_t i = 0; i < g_summary.size(); ++i) where[g_summary[i].name] = i;
  for (Rec& r : g_recs) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "profile_collect: %s", hipGetErrorString(e));
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "profile_collect: %s", hipGetErrorString(e));
    auto it = where.find(r.name);
    if (it == where.end()) {
      where[r.name] = g_summary.size();
      g_summary.push_back(Summary{r.name});
      it = where.find(r.name);
    }
    Summary& s = g_summary[it->second];
    s.launches += 1;
    s.total_ms += ms;
    s.flops += r.flops;
    s.bytes += r.bytes;
    s.gather += r.gather;
  }
  return CPRA_OK;
}

cpra_status cpra_profile_end(int32_t* n_kernels) {
  using namespace cpra;
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = false;
  for (Rec& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  if (n_kernels) *n_kernels = (int32_t)g_summary.size();
  return CPRA_OK;
}

cpra_status cpra_profile_get(int32_t i, char* name, size_t name_len, int64_t* launches,
                             double* total_ms, double* flops, double* bytes, double* gather) {
  using namespace cpra;
  std::lock_guard<std::mutex> lk(g_mu);
  if (i < 0 || i >= (int32_t)g_summary.size()) CPRA_FAIL(CPRA_ERR_PARAM, "profile_get: index out of range");
  const Summary& s = g_summary[i];
  if (name && name_len) {
    snprintf(name, name_len, "%s", s.name.c_str());
  }
  if (launches) *launches = s.launches;
  if (total_ms) *total_ms = s.total_ms;
  if (flops) *flops = s.flops;
  if (bytes) *bytes = s.bytes;
  if (gather) *gather = s.gather;
  return CPRA_OK;
}

}  // extern "C"
