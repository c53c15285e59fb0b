// Replaying a captured HIP graph for long runs of launch-bound steps.
#pragma once
#include <map>
#include <mutex>

#include "common.hpp"

namespace mpf {

// A stream per device for stream capture (created once, default priority,
// not synchronising with the null stream: capture executes nothing).
inline int capture_stream(hipStream_t* out) {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  MPF_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find(dev);
  if (it == streams.end()) {
    hipStream_t s = nullptr;
    MPF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    it = streams.emplace(dev, s).first;
  }
  *out = it->second;
  return MPF_OK;
}

// Runs launch(k, stream), which enqueues k steps on stream, for n_steps steps
// on st.  With at least two graphs' worth of steps, graph_steps steps are
// captured once into a graph that is then launched n_steps / graph_steps
// times, and the rest is enqueued directly: the same kernels with the same
// arguments in the same order, so the results are the same bit for bit; what
// changes is the host's launch overhead, which bounds the steps of small
// cells.  The call then waits for st before it frees the graph.  A caller's
// stream that is itself being captured gets direct launches (no nested
// capture, no wait), and so does any run whose capture cannot be set up
// (nothing has been enqueued on st at that point).
template <typename L>
int run_steps(int n_steps, int graph_steps, L&& launch, hipStream_t st) {
  if (graph_steps < 1 || n_steps < 2 * graph_steps) return launch(n_steps, st);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
    return launch(n_steps, st);
  hipStream_t cs = nullptr;
  if (capture_stream(&cs) != MPF_OK) return launch(n_steps, st);
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return launch(n_steps, st);
  int rc = launch(graph_steps, cs);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &g);
  hipGraphExec_t ex = nullptr;
  if (rc || ec != hipSuccess || !g || hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();  // a failed capture leaves no work behind: launch directly
    return launch(n_steps, st);
  }
  const int reps = n_steps / graph_steps;
  for (int r = 0; r < reps && rc == MPF_OK; ++r)
    if (hipGraphLaunch(ex, st) != hipSuccess) rc = MPF_ERR_HIP;
  if (rc == MPF_OK && n_steps > reps * graph_steps) rc = launch(n_steps - reps * graph_steps, st);
  const hipError_t es = hipStreamSynchronize(st);
  (void)hipGraphExecDestroy(ex);
  (void)hipGraphDestroy(g);
  if (rc == MPF_OK && es != hipSuccess) rc = MPF_ERR_HIP;
  return rc;
}

}  // namespace mpf
