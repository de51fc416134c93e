// Captured step graphs: record the enqueued work of one training step once
// and replay it with a single launch per step (the step reads gamma and
// Adam's t from a device counter, so the recorded work is step-invariant).
#include "common.hpp"

struct cpra_graph_s {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" {

cpra_status cpra_capture_begin(cpra_stream_t stream) {
  if (stream == nullptr) CPRA_FAIL(CPRA_ERR_PARAM, "capture_begin: the null stream cannot be captured");
  hipError_t e = hipStreamBeginCapture(cpra::as_stream(stream), hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "capture_begin: %s", hipGetErrorString(e));
  return CPRA_OK;
}

cpra_status cpra_capture_end(cpra_stream_t stream, cpra_graph* out) {
  if (out == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "capture_end: out is NULL");
  *out = nullptr;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(cpra::as_stream(stream), &graph);
  if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "capture_end: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(graph);
    CPRA_FAIL(CPRA_ERR_HIP, "capture_end: instantiate: %s", hipGetErrorString(e));
  }
  cpra_graph g = new cpra_graph_s{graph, exec};
  *out = g;
  return CPRA_OK;
}

cpra_status cpra_graph_launch(cpra_graph graph, cpra_stream_t stream) {
  if (graph == nullptr) CPRA_FAIL(CPRA_ERR_NULL, "graph_launch: graph is NULL");
  hipError_t e = hipGraphLaunch(graph->exec, cpra::as_stream(stream));
  if (e != hipSuccess) CPRA_FAIL(CPRA_ERR_HIP, "graph_launch: %s", hipGetErrorString(e));
  return CPRA_OK;
}

cpra_status cpra_graph_destroy(cpra_graph graph) {
  if (graph == nullptr) return CPRA_OK;
  hipGraphExecDestroy(graph->exec);
  hipGraphDestroy(graph->graph);
  delete graph;
  return CPRA_OK;
}

}  // extern "C"
