// A second stream per device for work that can overlap the main chain of a
// training step (the weight-gradient GEMMs, the loss-term reduction), plus the
// events that fork it from and join it back into the caller's stream.  The
// fork/join events make the overlap valid both for eager execution and inside
// a captured graph (the side stream joins the capture through the fork event).
// Created on first use per device, kept for the life of the process, at the
// default priority.  CPRA_OVERLAP=0 in the environment keeps all work on the
// caller's stream.
#include <cstdlib>
#include <map>
#include <mutex>

#include "common.hpp"

namespace cpra {

namespace {
std::mutex g_side_mu;
std::map<int, SideStream> g_side;
}  // namespace

// Read at every call (a host getenv per training step), so that a caller can
// time the kernels of eager steps alone and still capture overlapped steps.
bool overlap_enabled() {
  const char* e = getenv("CPRA_OVERLAP");
  return !(e != nullptr && e[0] == '0');
}

cpra_status get_side_stream(SideStream** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "side stream: hipGetDevice: %s", hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_side_mu);
  auto it = g_side.find(dev);
  if (it == g_side.end()) {
    SideStream s{};
    e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "side stream: create: %s", hipGetErrorString(e));
    for (int i = 0; i < 2; ++i) {
      e = hipEventCreateWithFlags(&s.ev[i], hipEventDisableTiming);
      if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "side stream: event: %s", hipGetErrorString(e));
    }
    it = g_side.emplace(dev, s).first;
  }
  *out = &it->second;
  return CPRA_OK;
}

cpra_status fork_to(SideStream* s, hipStream_t main) {
  hipError_t e = hipEventRecord(s->ev[0], main);
  if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, s->ev[0], 0);
  if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "fork: %s", hipGetErrorString(e));
  return CPRA_OK;
}

cpra_status fork_mark(SideStream* s, hipStream_t main) {
  const hipError_t e = hipEventRecord(s->ev[0], main);
  if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "fork mark: %s", hipGetErrorString(e));
  return CPRA_OK;
}

cpra_status fork_wait(SideStream* s) {
  const hipError_t e = hipStreamWaitEvent(s->stream, s->ev[0], 0);
  if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "fork wait: %s", hipGetErrorString(e));
  return CPRA_OK;
}

cpra_status join_from(SideStream* s, hipStream_t main) {
  hipError_t e = hipEventRecord(s->ev[1], s->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(main, s->ev[1], 0);
  if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "join: %s", hipGetErrorString(e));
  return CPRA_OK;
}

}  // namespace cpra
