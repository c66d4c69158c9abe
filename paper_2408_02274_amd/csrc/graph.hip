// Batching by graph capture: the N-Mueller applies of several operators
// (bodies, or copies of one operator holding different right-hand sides)
// recorded once into one hipGraph and replayed with a single launch (project
// addition; the paper runs one forward map at a time).  Each operator's
// applies form one branch of the graph, so small bodies that leave most of
// the GPU idle run side by side.  Nothing in the apply path allocates, copies
// between host and device or synchronises, so the captured work is exactly
// the eager work.
#include <hip/hip_runtime.h>

#include <new>
#include <vector>

#include "../../include/ifgf.h"
#include "device.hpp"
#include "util.hpp"

using namespace ifgf;

struct ifgf_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t nodes = 0;
  int branches = 0;
  ~ifgf_graph_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

extern "C" {

int nmuller_graph_capture(ifgf_graph_t* out, int nops, const nmuller_t* ops, const void* const* y,
                          const int* nrhs, void* const* Ay) {
  clear_error();
  if (!out || !ops || !y || !nrhs || !Ay) return set_error(IFGF_EINVAL, "null argument");
  *out = nullptr;
  if (nops < 1) return set_error(IFGF_EINVAL, "nops must be >= 1");
  for (int i = 0; i < nops; ++i) {
    if (!ops[i] || !y[i] || !Ay[i]) return set_error(IFGF_EINVAL, "null operator or buffer");
    if (timing_on(nmuller_ifgf(ops[i])))
      return set_error(IFGF_EINVAL, "switch per-kernel timing off before capturing");
  }
  // One branch per distinct operator: applies of one operator share its
  // workspaces and stay in order on their branch; different operators share
  // nothing and run side by side.  The branches fork from and join into the
  // capture stream.
  std::vector<nmuller_t> distinct;
  std::vector<int> branch(nops);
  for (int i = 0; i < nops; ++i) {
    int b = 0;
    while (b < (int)distinct.size() && distinct[b] != ops[i]) ++b;
    if (b == (int)distinct.size()) distinct.push_back(ops[i]);
    branch[i] = b;
  }
  const int nb = (int)distinct.size();
  ifgf_graph_s* g = new (std::nothrow) ifgf_graph_s();
  if (!g) return set_error(IFGF_ENOMEM, "host allocation failed");
  std::vector<hipStream_t> bs(nb, nullptr);
  std::vector<hipEvent_t> ev(nb + 1, nullptr);
  hipStream_t cs = nullptr;
  auto cleanup = [&]() {
    for (hipStream_t s2 : bs)
      if (s2) (void)hipStreamDestroy(s2);
    for (hipEvent_t e2 : ev)
      if (e2) (void)hipEventDestroy(e2);
    if (cs) (void)hipStreamDestroy(cs);
  };
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  for (int b = 0; b < nb && e == hipSuccess; ++b) e = hipStreamCreateWithFlags(&bs[b], hipStreamNonBlocking);
  for (int b = 0; b <= nb && e == hipSuccess; ++b) e = hipEventCreateWithFlags(&ev[b], hipEventDisableTiming);
  if (e != hipSuccess) {
    cleanup();
    delete g;
    return set_hip_error(e, "capture streams");
  }
  if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    cleanup();
    delete g;
    return set_hip_error(e, "hipStreamBeginCapture");
  }
  int rc = IFGF_OK;
  if ((e = hipEventRecord(ev[nb], cs)) != hipSuccess) rc = set_hip_error(e, "fork event");
  for (int b = 0; b < nb && rc == IFGF_OK; ++b)
    if ((e = hipStreamWaitEvent(bs[b], ev[nb], 0)) != hipSuccess) rc = set_hip_error(e, "fork");
  for (int i = 0; i < nops && rc == IFGF_OK; ++i) rc = nmuller_apply(ops[i], y[i], nrhs[i], Ay[i], bs[branch[i]]);
  for (int b = 0; b < nb && rc == IFGF_OK; ++b) {
    if ((e = hipEventRecord(ev[b], bs[b])) != hipSuccess || (e = hipStreamWaitEvent(cs, ev[b], 0)) != hipSuccess)
      rc = set_hip_error(e, "join");
  }
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(cs, &graph);
  cleanup();
  g->graph = graph;
  if (rc != IFGF_OK) {
    delete g;
    return rc;   // the apply's own message stands
  }
  if (e2 != hipSuccess) {
    delete g;
    return set_hip_error(e2, "hipStreamEndCapture");
  }
  size_t nn = 0;
  (void)hipGraphGetNodes(graph, nullptr, &nn);
  g->nodes = (int64_t)nn;
  g->branches = nb;
  if ((e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
    delete g;
    return set_hip_error(e, "hipGraphInstantiate");
  }
  *out = g;
  return IFGF_OK;
}

int ifgf_graph_launch(ifgf_graph_t g, void* stream) {
  clear_error();
  if (!g || !g->exec) return set_error(IFGF_EINVAL, "graph is NULL");
  hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? IFGF_OK : set_hip_error(e, "hipGraphLaunch");
}

int ifgf_graph_nodes(ifgf_graph_t g, int64_t* nodes) {
  clear_error();
  if (!g || !nodes) return set_error(IFGF_EINVAL, "null argument");
  *nodes = g->nodes;
  return IFGF_OK;
}

void ifgf_graph_destroy(ifgf_graph_t g) { delete g; }

}  // extern "C"
