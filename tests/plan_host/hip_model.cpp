// Host-only model of the HIP runtime for the plan executor's sanitizer test (test
// infrastructure; no GPU).  It keeps what matters for the executor's memory safety:
//   * device work is asynchronous: launches and stream-ordered frees are queued and run
//     in submission order at the next synchronising call, so a buffer freed (for real)
//     or a graph destroyed while work that uses it is still queued is caught by
//     AddressSanitizer when the work runs;
//   * stream capture follows the documented rules: launches on a capturing stream become
//     graph nodes; an event recorded during a capture carries that capture's nodes; a
//     stream that waits on such an event joins the capture; an event recorded in one
//     capture cannot be waited on outside it or in another one; every stream that joined
//     must be joined back into the origin before the capture ends;
//   * an executable graph runs its nodes' work through the graph object, so destroying
//     either while a replay is queued is a use after free.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <set>
#include <vector>

#include "model.h"

struct ihipGraph;
struct hipGraphNode {
  int id;
  std::function<void()> work;
  std::vector<hipGraphNode *> deps;
};
struct ihipGraph {
  int id;
  bool live = true;  // capture in progress
  hipStream_t origin = nullptr;
  std::vector<hipGraphNode *> nodes;
  std::set<hipStream_t> joined;
};
struct ihipStream_t {
  ihipGraph *graph = nullptr;                 // capture this stream takes part in
  std::vector<hipGraphNode *> last;           // capture: nodes the next node depends on
  unsigned long long seq = 0;                 // capture: work recorded on this stream
  std::map<hipStream_t, unsigned long long> covers;  // capture: work of other streams joined into this one
};
struct ihipEvent_t {
  ihipGraph *graph = nullptr;  // capture the last record happened in
  std::vector<hipGraphNode *> nodes;
  hipStream_t stream = nullptr;
  unsigned long long seq = 0;
  std::map<hipStream_t, unsigned long long> covers;
  unsigned long long when = 0;  // eager: queue position
  bool in_capture = false, outside = false;  // ever recorded inside / outside a capture
};

namespace {
// The executor keeps capture events and eager events apart; an event used both ways is
// reported (the runtime's handling of such reuse is not something the executor relies on).
void check_event_use(hipEvent_t e) {
  if (e->in_capture && e->outside) {
    std::fprintf(stderr, "model: event %p recorded both inside and outside a stream capture\n", (void *)e);
    std::abort();
  }
}
}  // namespace
struct hipGraphExec {
  std::vector<std::function<void()>> work;
};

namespace {
std::vector<std::function<void()>> g_queue;  // device work in submission order
int g_graph_ids = 0;
unsigned long long g_clock = 0;

void drain() {
  // work may enqueue nothing; run in order
  std::vector<std::function<void()>> q;
  q.swap(g_queue);
  for (auto &w : q) w();
}

void touch_nodes(const std::vector<hipGraphNode *> &v) {
  volatile int sink = 0;
  for (hipGraphNode *n : v) sink += n->id;  // a node of a destroyed graph is a use after free
  (void)sink;
}
}  // namespace

namespace model {
void submit(hipStream_t s, std::function<void()> work) {
  if (s && s->graph) {
    auto *n = new hipGraphNode{(int)s->graph->nodes.size(), std::move(work), s->last};
    touch_nodes(n->deps);
    s->graph->nodes.push_back(n);
    s->last.assign(1, n);
    s->seq++;
  } else {
    g_queue.push_back(std::move(work));
    g_clock++;
  }
}
bool capturing(hipStream_t s) { return s && s->graph; }
void synchronize() { drain(); }
}  // namespace model

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  *s = new ihipStream_t();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  if (!s) return hipErrorInvalidResourceHandle;
  if (s->graph) return hipErrorIllegalState;
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  if (s && s->graph) return hipErrorStreamCaptureUnsupported;
  drain();
  return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) {
  drain();
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
  *e = new ihipEvent_t();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  if (!e) return hipErrorInvalidResourceHandle;
  if (s && s->graph) {
    e->graph = s->graph;
    e->nodes = s->last;
    touch_nodes(e->nodes);
    e->stream = s;
    e->seq = s->seq;
    e->covers = s->covers;
    e->in_capture = true;
  } else {
    e->graph = nullptr;
    e->nodes.clear();
    e->stream = s;
    e->when = g_clock;
    e->outside = true;
  }
  check_event_use(e);
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  if (!e) return hipErrorInvalidResourceHandle;
  if (e->graph) {
    if (!e->graph->live) return hipErrorStreamCaptureIsolation;  // recorded in a finished capture
    if (s && s->graph && s->graph != e->graph) return hipErrorStreamCaptureIsolation;
    if (!s) return hipErrorStreamCaptureIsolation;
    touch_nodes(e->nodes);
    if (!s->graph) {  // s joins the capture
      s->graph = e->graph;
      s->last = e->nodes;
      s->seq = 0;
      s->covers.clear();
      e->graph->joined.insert(s);
    } else {
      for (hipGraphNode *n : e->nodes)
        if (std::find(s->last.begin(), s->last.end(), n) == s->last.end()) s->last.push_back(n);
    }
    auto &c = s->covers[e->stream];
    if (e->seq > c) c = e->seq;
    for (auto &kv : e->covers)
      if (kv.second > s->covers[kv.first]) s->covers[kv.first] = kv.second;
    return hipSuccess;
  }
  if (s && s->graph) return hipErrorStreamCaptureIsolation;  // an outside event into a capture
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  if (!e) return hipErrorInvalidResourceHandle;
  if (e->graph) return hipErrorStreamCaptureUnsupported;
  drain();
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  if (!a || !b || a->graph || b->graph) return hipErrorInvalidResourceHandle;
  // plus a deterministic jitter, so that searches over timings take every branch
  static unsigned long long calls = 0;
  unsigned long long z = ++calls * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 31)) * 0xBF58476D1CE4E5B9ull;
  *ms = 0.001f * (float)(b->when >= a->when ? b->when - a->when : 0) + 0.5f + 0.01f * (float)((z >> 40) % 100);
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (!s) return hipErrorStreamCaptureUnsupported;  // the null stream cannot capture
  if (s->graph) return hipErrorIllegalState;
  auto *g = new ihipGraph();
  g->id = ++g_graph_ids;
  g->origin = s;
  s->graph = g;
  s->last.clear();
  s->seq = 0;
  s->covers.clear();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *out) {
  *out = nullptr;
  if (!s || !s->graph) return hipErrorIllegalState;
  ihipGraph *g = s->graph;
  if (g->origin != s) return hipErrorStreamCaptureUnmatched;
  hipError_t st = hipSuccess;
  for (hipStream_t j : g->joined) {
    auto it = s->covers.find(j);
    if (j->seq > 0 && (it == s->covers.end() || it->second < j->seq)) st = hipErrorStreamCaptureUnjoined;
    j->graph = nullptr;
    j->last.clear();
    j->covers.clear();
    j->seq = 0;
  }
  s->graph = nullptr;
  s->last.clear();
  s->covers.clear();
  s->seq = 0;
  g->live = false;
  if (st != hipSuccess) {
    for (auto *n : g->nodes) delete n;
    delete g;
    return st;
  }
  *out = g;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
  if (!g) return hipErrorInvalidValue;
  auto *e = new hipGraphExec();
  for (auto *n : g->nodes) {
    touch_nodes(n->deps);
    e->work.push_back(n->work);
  }
  *x = e;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  if (!x) return hipErrorInvalidValue;
  if (s && s->graph) return hipErrorStreamCaptureUnsupported;
  g_queue.push_back([x]() {
    for (auto &w : x->work) w();  // through the executable graph: destroyed early = use after free
  });
  g_clock += x->work.size();
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete x;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  if (!g) return hipErrorInvalidValue;
  for (auto *n : g->nodes) delete n;
  delete g;
  return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind) {
  drain();
  std::memcpy(dst, src, bytes);
  return hipSuccess;
}
const char *hipGetErrorString(hipError_t e) {
  static char buf[32];
  std::snprintf(buf, sizeof(buf), "model error %d", e);
  return buf;
}

// ----------------------------------------------------------- calls of the column library's host unit
hipError_t hipGetDevice(int *device) {
  *device = 0;
  return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t *prop, int) {
  prop->multiProcessorCount = 256;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void **ptr, const void *symbol) {
  *ptr = const_cast<void *>(symbol);
  return hipSuccess;
}
hipError_t hipMallocAsync(void **ptr, size_t bytes, hipStream_t s) {
  if (s && s->graph) return hipErrorStreamCaptureUnsupported;
  *ptr = std::calloc(1, bytes ? bytes : 1);
  return *ptr ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipFreeAsync(void *ptr, hipStream_t s) {
  if (s && s->graph) return hipErrorStreamCaptureUnsupported;
  model::submit(nullptr, [ptr]() { std::free(ptr); });  // after the work queued before it
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  model::submit(s, [dst, src, bytes]() { std::memcpy(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }

