// Optional per-launch timing: while a Trace is installed on the calling host
// thread, every launch made through LOD_LAUNCH is bracketed by two hipEvents
// recorded on the launch stream.  Used only by the *_timed entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace lodh {

struct TraceRec {
  const char *name;
  hipEvent_t a, b;
};

struct Trace {
  std::vector<TraceRec> recs;
};

Trace *&current_trace();

struct TraceScope {
  Trace *t;
  size_t idx;
  hipStream_t st;
  TraceScope(const char *name, hipStream_t s) : t(current_trace()), idx(0), st(s) {
    if (!t) return;
    TraceRec r{name, nullptr, nullptr};
    // a launch whose events cannot be made or recorded is left out of the trace
    if (hipEventCreate(&r.a) != hipSuccess) { t = nullptr; return; }
    if (hipEventCreate(&r.b) != hipSuccess || hipEventRecord(r.a, st) != hipSuccess) {
      (void)hipEventDestroy(r.a);
      if (r.b) (void)hipEventDestroy(r.b);
      t = nullptr;
      return;
    }
    idx = t->recs.size();
    t->recs.push_back(r);
  }
  ~TraceScope() {
    // a failed record shows up as a failed elapsed-time query in lod_trace_end
    if (t) (void)hipEventRecord(t->recs[idx].b, st);
  }
};

}  // namespace lodh

#define LOD_LAUNCH(kernel, grid, block, shmem, stream, ...)              \
  do {                                                                    \
    ::lodh::TraceScope lod_trace_scope_(#kernel, (stream));               \
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);  \
  } while (0)
