// ms_plan.hip -- the plan executor of libmorphgpu.so: a plan is an ordered list of
// operator steps over input columns (section 3.3).  It runs eagerly, one launch sequence
// per step, or as one captured HIP graph replayed with no allocation and no host work
// per step; independent steps may go to parallel branches; an autotuner picks the
// launch shape per plan and caches it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/morphgpu.h"
#include "ms_batch.h"
#include "ms_kernels.h"
#include "ms_runtime.h"

using namespace ms;

namespace {

enum ResKind { R_COLUMN, R_BITMAP, R_BYTES };

struct Result {
  ms_column *col = nullptr;
  void *ptr = nullptr;
  uint64_t bytes = 0;
  void *stream = nullptr;
};

constexpr uint32_t kMaxBranches = 16;
constexpr uint32_t kMaxWgPerCu = 32;
constexpr uint32_t kMaxChunksPerWg = 64;

ms_status fail(ms_status st, const char *msg) {
  rt::set_error(msg);
  return st;
}
ms_status hip_fail(hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  rt::set_error(m.c_str());
  return MS_ERR_HIP;
}

ResKind result_kind(uint32_t op) {
  switch (op) {
    case MS_OP_BITMAP: return R_BITMAP;
    case MS_OP_SUM:
    case MS_OP_GROUP_SUM:
    case MS_OP_FOOTPRINTS:
    case MS_OP_STATS: return R_BYTES;
    default: return R_COLUMN;
  }
}

// Operands each step reads: 'c' column, 'm' bitmap step, '-' unused.
const char *operand_kinds(uint32_t op) {
  switch (op) {
    case MS_OP_SEMIJOIN: return "cm";
    case MS_OP_PROJECT:
    case MS_OP_INTERSECT:
    case MS_OP_GROUP_SUM: return "cc";
    default: return "c-";
  }
}

uint64_t result_bytes(const ms_step &s) {
  switch (s.op) {
    case MS_OP_BITMAP: return 4 * ((s.param + 31) / 32) + 4;
    case MS_OP_SUM: return 8;
    case MS_OP_GROUP_SUM: return 8 * (s.param ? s.param : 1);
    case MS_OP_FOOTPRINTS: return 48;
    case MS_OP_STATS: return 128;
    default: return 0;
  }
}

uint64_t fnv(uint64_t h, const void *p, size_t n) {
  const unsigned char *b = static_cast<const unsigned char *>(p);
  for (size_t i = 0; i < n; i++) {
    h ^= b[i];
    h *= 0x100000001B3ull;
  }
  return h;
}

}  // namespace

// Events that fork a run onto the branch streams, order steps across branches and join
// the branches back.  Eager runs use the plan's own set; every capture gets a fresh set
// that lives and dies with the captured graph, so no event is ever recorded both in a
// capture and outside one.
struct EventSet {
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join, step;
};

struct ms_plan {
  std::vector<ms_step> steps;
  std::vector<const ms_column *> inputs;
  ms_tune tune{1, 0, 0, 0};
  std::vector<int> branch_of;
  std::vector<Result> eager, graph_res;
  bool last_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void *arena = nullptr;
  uint64_t arena_bytes = 0;
  void *arena_stream = nullptr;
  hipStream_t cap = nullptr;              // capture origin (captures need a non-null stream)
  std::vector<hipStream_t> br;            // branch streams
  EventSet eager_ev;                      // events of eager runs
  EventSet graph_ev;                      // events recorded in the captured graph
  std::vector<batch::Upload> uploads;     // batched task tables: kept until a sync (eager) or copied after a capture
};

namespace {

void assign_branches(ms_plan *p) {
  const uint32_t B = p->tune.branches;
  p->branch_of.assign(p->steps.size(), 0);
  uint32_t rr = 0;
  for (size_t i = 0; i < p->steps.size(); i++) {
    const ms_step &s = p->steps[i];
    const char *ok = operand_kinds(s.op);
    int dep = -1;
    if (ok[0] != '-' && s.a >= 0) dep = s.a;
    else if (ok[1] != '-' && s.b >= 0) dep = s.b;
    p->branch_of[i] = dep >= 0 ? p->branch_of[dep] : (int)(rr++ % B);
  }
}

void destroy_events(EventSet &ev) {
  if (ev.fork) (void)hipEventDestroy(ev.fork);
  for (auto e : ev.join) (void)hipEventDestroy(e);
  for (auto e : ev.step) (void)hipEventDestroy(e);
  ev = EventSet();
}

// Sizes an event set for the plan's steps and branches.
ms_status ensure_events(ms_plan *p, EventSet &ev) {
  auto make = [](hipEvent_t &e) { return hipEventCreateWithFlags(&e, hipEventDisableTiming); };
  if (!ev.fork) {
    hipError_t e = make(ev.fork);
    if (e != hipSuccess) return hip_fail(e, "event create");
  }
  while (ev.join.size() < p->tune.branches) {
    hipEvent_t x;
    hipError_t e = make(x);
    if (e != hipSuccess) return hip_fail(e, "event create");
    ev.join.push_back(x);
  }
  while (ev.step.size() < p->steps.size()) {
    hipEvent_t x;
    hipError_t e = make(x);
    if (e != hipSuccess) return hip_fail(e, "event create");
    ev.step.push_back(x);
  }
  return MS_OK;
}

ms_status ensure_streams(ms_plan *p) {
  if (!p->cap) {
    hipError_t e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "stream create");
  }
  while (p->br.size() < p->tune.branches) {
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "stream create");
    p->br.push_back(s);
  }
  return ensure_events(p, p->eager_ev);
}

const ms_column *column_of(const ms_plan *p, const std::vector<Result> &r, int32_t ref) {
  return ref >= 0 ? r[ref].col : p->inputs[-1 - ref];
}

void free_results(std::vector<Result> &r) {
  for (auto &x : r) {
    if (x.col) ms_column_free(x.col);
    if (x.ptr) rt::free(x.ptr, x.bytes, x.stream);
    x = Result();
  }
}

// Launch one step on stream s; its result goes to r[i].
ms_status exec_step(ms_plan *p, size_t i, void *s, std::vector<Result> &r) {
  const ms_step &st = p->steps[i];
  Result &out = r[i];
  const ms_column *A = (operand_kinds(st.op)[0] == 'c') ? column_of(p, r, st.a) : nullptr;
  const ms_column *B = (operand_kinds(st.op)[1] == 'c') ? column_of(p, r, st.b) : nullptr;
  if (result_kind(st.op) != R_COLUMN) {
    out.bytes = result_bytes(st);
    out.stream = s;
    out.ptr = rt::alloc(out.bytes, s);
    if (!out.ptr) return fail(MS_ERR_OOM, "result allocation failed");
  }
  switch (st.op) {
    case MS_OP_MORPH: return ms_morph(A, st.out, s, &out.col);
    case MS_OP_SELECT: return ms_select(A, (ms_cmp)st.cmp, st.c0, st.c1, st.out, s, &out.col);
    case MS_OP_BITMAP: return ms_bitmap_from_positions(A, st.param, static_cast<uint32_t *>(out.ptr), s);
    case MS_OP_SEMIJOIN:
      return ms_semijoin(A, static_cast<const uint32_t *>(r[st.b].ptr), st.param, st.out, s, &out.col);
    case MS_OP_PROJECT: return ms_project(A, B, st.out, s, &out.col);
    case MS_OP_INTERSECT: return ms_intersect(A, B, st.param, st.out, s, &out.col);
    case MS_OP_SUM: return ms_sum(A, static_cast<uint64_t *>(out.ptr), s);
    case MS_OP_GROUP_SUM: return ms_group_sum(A, B, (uint32_t)st.param, static_cast<uint64_t *>(out.ptr), s);
    case MS_OP_FOOTPRINTS: return ms_footprints(A, static_cast<uint64_t *>(out.ptr), s);
    case MS_OP_STATS: return ms_stats(A, static_cast<float *>(out.ptr), s);
    default: return fail(MS_ERR_INVALID_ARG, "unknown step");
  }
}

// Batched: level by level; the operators of a level (steps whose operands all come from
// earlier levels) are recorded and issued as batched launches on `origin`, their other
// kernels spread over the branch streams.
ms_status run_levels(ms_plan *p, hipStream_t origin, std::vector<Result> &r, EventSet &ev) {
  const size_t n = p->steps.size();
  std::vector<uint32_t> level(n, 0);
  uint32_t levels = 0;
  for (size_t i = 0; i < n; i++) {
    const ms_step &s = p->steps[i];
    const char *ok = operand_kinds(s.op);
    const int32_t refs[2] = {ok[0] != '-' ? s.a : -1, ok[1] != '-' ? s.b : -1};
    for (int32_t ref : refs)
      if (ref >= 0) level[i] = std::max(level[i], level[ref] + 1);
    levels = std::max(levels, level[i] + 1);
  }
  ms_status st = MS_OK;
  batch::Streams bs;
  bs.origin = origin;
  bs.branches = reinterpret_cast<void *const *>(p->br.data());
  bs.n_branches = p->tune.branches;
  bs.fork = ev.fork;
  bs.join = ev.join.data();
  for (uint32_t l = 0; l < levels && st == MS_OK; l++) {
    batch::begin();
    for (size_t i = 0; i < n && st == MS_OK; i++) {
      if (level[i] != l) continue;
      batch::next_op();
      st = exec_step(p, i, origin, r);
    }
    const hipError_t e = batch::flush(bs, p->uploads);  // also after an error: frees run, recording stops
    if (st == MS_OK && e != hipSuccess) st = hip_fail(e, "batched launch");
  }
  return st;
}

// All steps, forked from and joined back into `origin`, ordered across branches by `ev`.
ms_status run_steps(ms_plan *p, hipStream_t origin, std::vector<Result> &r, EventSet &ev) {
  r.assign(p->steps.size(), Result());
  const uint32_t B = p->tune.branches;
  rt::set_thread_wg_per_cu(p->tune.wg_per_cu);
  rt::set_thread_chunks_per_wg(p->tune.chunks_per_wg);
  ms_status st = MS_OK;
  hipError_t e = hipSuccess;
  if (p->tune.batch) {
    st = run_levels(p, origin, r, ev);
  } else if (B == 1) {
    for (size_t i = 0; i < p->steps.size() && st == MS_OK; i++) st = exec_step(p, i, origin, r);
  } else {
    e = hipEventRecord(ev.fork, origin);
    for (uint32_t b = 0; b < B && e == hipSuccess; b++) e = hipStreamWaitEvent(p->br[b], ev.fork, 0);
    for (size_t i = 0; i < p->steps.size() && st == MS_OK && e == hipSuccess; i++) {
      const ms_step &s = p->steps[i];
      const int b = p->branch_of[i];
      const char *ok = operand_kinds(s.op);
      const int32_t refs[2] = {ok[0] != '-' ? s.a : -1, ok[1] != '-' ? s.b : -1};
      for (int32_t ref : refs)
        if (ref >= 0 && p->branch_of[ref] != b && e == hipSuccess) e = hipStreamWaitEvent(p->br[b], ev.step[ref], 0);
      if (e != hipSuccess) break;
      st = exec_step(p, i, p->br[b], r);
      if (st == MS_OK) e = hipEventRecord(ev.step[i], p->br[b]);
    }
    // always join every branch back, also after an error (a capture must end joined)
    for (uint32_t b = 0; b < B; b++) {
      hipError_t e2 = hipEventRecord(ev.join[b], p->br[b]);
      if (e2 == hipSuccess) e2 = hipStreamWaitEvent(origin, ev.join[b], 0);
      if (e == hipSuccess) e = e2;
    }
  }
  rt::set_thread_wg_per_cu(0);
  rt::set_thread_chunks_per_wg(0);
  if (st != MS_OK) return st;
  return e == hipSuccess ? MS_OK : hip_fail(e, "branch fork/join");
}

void drop_graph(ms_plan *p) {
  // Replays may still be queued on any stream the caller launched them on: wait for the
  // device before the executable graph, its kernel arguments and the arena go away.
  if (p->exec || p->graph || p->arena || !p->graph_res.empty()) (void)hipDeviceSynchronize();
  p->uploads.clear();
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  destroy_events(p->graph_ev);  // after the graph that recorded them
  for (auto &x : p->graph_res)
    if (x.col) ms_column_free(x.col);  // arena columns: frees only the handle
  p->graph_res.clear();
  if (p->arena) rt::free(p->arena, p->arena_bytes, p->arena_stream);
  p->arena = nullptr;
  p->arena_bytes = 0;
  if (p->last_graph) p->last_graph = false;
}

// One capture of the plan on the plan's capture stream with arena `a`, recording the
// events of `ev` (which must not be used outside this capture's graph).
ms_status capture(ms_plan *p, rt::Arena *a, std::vector<Result> &r, hipGraph_t *g, EventSet &ev) {
  *g = nullptr;
  ms_status st = ensure_events(p, ev);
  if (st != MS_OK) return st;
  hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "begin capture");
  rt::set_thread_arena(a);
  prof_suspend(true);  // no timing events inside a graph
  st = run_steps(p, p->cap, r, ev);
  prof_suspend(false);
  rt::set_thread_arena(nullptr);
  e = hipStreamEndCapture(p->cap, g);
  if (st != MS_OK) {
    if (*g) (void)hipGraphDestroy(*g);
    *g = nullptr;
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  return MS_OK;
}

}  // namespace

extern "C" {

ms_status ms_plan_create(const ms_step *steps, uint32_t n_steps, const ms_column *const *inputs, uint32_t n_inputs,
                         ms_plan **out) {
  if (!out) return fail(MS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!rt::initialized()) return fail(MS_ERR_NOT_INITIALIZED, "ms_init not called");
  if (n_steps && !steps) return fail(MS_ERR_INVALID_ARG, "steps is NULL");
  if (n_inputs && !inputs) return fail(MS_ERR_INVALID_ARG, "inputs is NULL");
  for (uint32_t j = 0; j < n_inputs; j++)
    if (!inputs[j]) return fail(MS_ERR_INVALID_ARG, "input column is NULL");
  for (uint32_t i = 0; i < n_steps; i++) {
    const ms_step &s = steps[i];
    if (s.op > MS_OP_STATS) return fail(MS_ERR_INVALID_ARG, "unknown step kind");
    const char *ok = operand_kinds(s.op);
    const int32_t refs[2] = {s.a, s.b};
    for (int k = 0; k < 2; k++) {
      if (ok[k] == '-') continue;
      const int32_t ref = refs[k];
      if (ref >= 0) {
        if ((uint32_t)ref >= i) return fail(MS_ERR_INVALID_ARG, "a step may only read earlier steps");
        const ResKind rk = result_kind(steps[ref].op);
        if (ok[k] == 'c' && rk != R_COLUMN) return fail(MS_ERR_INVALID_ARG, "operand is not a column");
        if (ok[k] == 'm' && steps[ref].op != MS_OP_BITMAP) return fail(MS_ERR_INVALID_ARG, "operand is not a bitmap");
        if (ok[k] == 'm' && s.param > steps[ref].param)
          return fail(MS_ERR_INVALID_ARG, "semi-join domain exceeds the bitmap's");
      } else {
        if (ok[k] == 'm') return fail(MS_ERR_INVALID_ARG, "a bitmap operand must be a bitmap step");
        if ((uint64_t)(-(int64_t)ref - 1) >= n_inputs) return fail(MS_ERR_INVALID_ARG, "input index out of range");
      }
    }
    if ((s.op == MS_OP_BITMAP || s.op == MS_OP_SEMIJOIN || s.op == MS_OP_INTERSECT) && s.param > (1ull << 32))
      return fail(MS_ERR_INVALID_ARG, "domain exceeds 2^32");
    if (s.op == MS_OP_GROUP_SUM && s.param >= (1ull << 32)) return fail(MS_ERR_INVALID_ARG, "too many groups");
    if (result_kind(s.op) == R_COLUMN) {
      if (s.out.kind > MS_RLE) return fail(MS_ERR_INVALID_ARG, "unknown output format");
      if (s.out.kind == MS_STATIC_BP && s.out.bit_width != MS_BW_AUTO && s.out.bit_width > 32)
        return fail(MS_ERR_INVALID_ARG, "static BP width must be 0..32 or auto");
    }
  }
  ms_plan *p = new ms_plan();
  p->steps.assign(steps, steps + n_steps);
  p->inputs.assign(inputs, inputs + n_inputs);
  assign_branches(p);
  *out = p;
  return MS_OK;
}

ms_status ms_plan_destroy(ms_plan *p) {
  if (!p) return MS_OK;
  (void)hipDeviceSynchronize();
  drop_graph(p);
  free_results(p->eager);
  for (auto s : p->br) (void)hipStreamDestroy(s);
  destroy_events(p->eager_ev);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  delete p;
  return MS_OK;
}

ms_status ms_plan_set_format(ms_plan *p, uint32_t step, ms_format fmt) {
  if (!p) return fail(MS_ERR_INVALID_ARG, "plan is NULL");
  if (step >= p->steps.size()) return fail(MS_ERR_INVALID_ARG, "step out of range");
  if (result_kind(p->steps[step].op) != R_COLUMN) return fail(MS_ERR_INVALID_ARG, "step produces no column");
  if (fmt.kind > MS_RLE) return fail(MS_ERR_INVALID_ARG, "unknown output format");
  if (fmt.kind == MS_STATIC_BP && fmt.bit_width != MS_BW_AUTO && fmt.bit_width > 32)
    return fail(MS_ERR_INVALID_ARG, "static BP width must be 0..32 or auto");
  ms_format &f = p->steps[step].out;
  if (f.kind != fmt.kind || f.bit_width != fmt.bit_width) {
    drop_graph(p);
    f = fmt;
  }
  return MS_OK;
}

ms_status ms_plan_get_format(const ms_plan *p, uint32_t step, ms_format *fmt) {
  if (!p || !fmt) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  if (step >= p->steps.size()) return fail(MS_ERR_INVALID_ARG, "step out of range");
  *fmt = p->steps[step].out;
  return MS_OK;
}

ms_status ms_plan_set_tune(ms_plan *p, const ms_tune *t) {
  if (!p || !t) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  if (t->branches < 1 || t->branches > kMaxBranches) return fail(MS_ERR_INVALID_ARG, "branches must be 1..16");
  if (t->wg_per_cu > kMaxWgPerCu) return fail(MS_ERR_INVALID_ARG, "wg_per_cu must be 0..32");
  if (t->chunks_per_wg > kMaxChunksPerWg) return fail(MS_ERR_INVALID_ARG, "chunks_per_wg must be 0..64");
  if (t->batch > 1) return fail(MS_ERR_INVALID_ARG, "batch must be 0 or 1");
  if (t->branches != p->tune.branches || t->wg_per_cu != p->tune.wg_per_cu ||
      t->chunks_per_wg != p->tune.chunks_per_wg || t->batch != p->tune.batch) {
    drop_graph(p);
    p->tune = *t;
    assign_branches(p);
  }
  return MS_OK;
}

ms_status ms_plan_get_tune(const ms_plan *p, ms_tune *t) {
  if (!p || !t) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  *t = p->tune;
  return MS_OK;
}

ms_status ms_plan_run(ms_plan *p, void *stream) {
  if (!p) return fail(MS_ERR_INVALID_ARG, "plan is NULL");
  ms_status st = ensure_streams(p);
  if (st != MS_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!p->eager.empty() || !p->uploads.empty()) {
    (void)hipStreamSynchronize(s);
    for (auto b : p->br) (void)hipStreamSynchronize(b);
    free_results(p->eager);
    p->uploads.clear();
  }
  st = run_steps(p, s, p->eager, p->eager_ev);
  p->last_graph = false;
  if (st != MS_OK) {  // no partial results survive a failed run
    (void)hipStreamSynchronize(s);
    for (auto b : p->br) (void)hipStreamSynchronize(b);
    free_results(p->eager);
    p->eager.clear();
    p->uploads.clear();
  }
  return st;
}

ms_status ms_plan_launch(ms_plan *p, void *stream) {
  if (!p) return fail(MS_ERR_INVALID_ARG, "plan is NULL");
  if (rt::thread_arena()) return fail(MS_ERR_INVALID_ARG, "plans do not nest");
  if (!p->exec) {
    ms_status st = ensure_streams(p);
    if (st != MS_OK) return st;
    // nothing of an earlier eager run or replay is in flight on the plan's streams when
    // a capture starts
    hipError_t se = hipDeviceSynchronize();
    if (se != hipSuccess) return hip_fail(se, "device sync");
    p->uploads.clear();
    // 1) size the arena with a capture that is never instantiated (its own events)
    rt::Arena m;
    m.measure = true;
    std::vector<Result> tmp;
    hipGraph_t g = nullptr;
    EventSet mev;
    st = capture(p, &m, tmp, &g, mev);
    for (auto &x : tmp)
      if (x.col) ms_column_free(x.col);
    if (g) (void)hipGraphDestroy(g);
    destroy_events(mev);
    if (st != MS_OK) return st;
    // 2) back it and capture for real
    p->arena_bytes = m.used + 256;
    p->arena_stream = stream;
    p->arena = rt::alloc(p->arena_bytes, stream);
    if (!p->arena) return fail(MS_ERR_OOM, "arena allocation failed");
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));  // arena ready before replays
    if (e != hipSuccess) return hip_fail(e, "stream sync");
    rt::Arena a;
    a.base = static_cast<char *>(p->arena);
    a.size = p->arena_bytes;
    st = capture(p, &a, p->graph_res, &p->graph, p->graph_ev);
    if (st != MS_OK) {
      drop_graph(p);
      return st;
    }
    // task tables of batched launches: into the arena once the capture has ended
    for (const batch::Upload &u : p->uploads) {
      e = hipMemcpy(u.dev, u.host.data(), u.host.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        drop_graph(p);
        return hip_fail(e, "batch table copy");
      }
    }
    p->uploads.clear();
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_graph(p);
      return hip_fail(e, "graph instantiate");
    }
  }
  hipError_t e = hipGraphLaunch(p->exec, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  p->last_graph = true;
  return MS_OK;
}

ms_status ms_plan_result(const ms_plan *p, uint32_t step, const ms_column **col, void **dev_ptr) {
  if (!p) return fail(MS_ERR_INVALID_ARG, "plan is NULL");
  if (step >= p->steps.size()) return fail(MS_ERR_INVALID_ARG, "step out of range");
  const std::vector<Result> &r = p->last_graph ? p->graph_res : p->eager;
  if (col) *col = r.empty() ? nullptr : r[step].col;
  if (dev_ptr) *dev_ptr = r.empty() ? nullptr : r[step].ptr;
  return MS_OK;
}

ms_status ms_plan_read_result(const ms_plan *p, uint32_t step, void *host_dst, uint64_t bytes, void *stream,
                              uint64_t *copied) {
  if (!p) return fail(MS_ERR_INVALID_ARG, "plan is NULL");
  if (step >= p->steps.size()) return fail(MS_ERR_INVALID_ARG, "step out of range");
  if (result_kind(p->steps[step].op) == R_COLUMN) return fail(MS_ERR_INVALID_ARG, "step produces a column");
  const std::vector<Result> &r = p->last_graph ? p->graph_res : p->eager;
  if (r.empty() || !r[step].ptr) return fail(MS_ERR_INVALID_ARG, "plan has not run");
  const uint64_t n = std::min<uint64_t>(bytes, result_bytes(p->steps[step]));
  if (n && !host_dst) return fail(MS_ERR_INVALID_ARG, "destination is NULL");
  hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  if (e == hipSuccess && n) e = hipMemcpy(host_dst, r[step].ptr, n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "result copy");
  if (copied) *copied = n;
  return MS_OK;
}

uint64_t ms_plan_arena_bytes(const ms_plan *p) { return p ? p->arena_bytes : 0; }

static ms_status time_replays(ms_plan *p, void *stream, uint32_t reps, hipEvent_t e0, hipEvent_t e1, float *ms);

ms_status ms_plan_autotune(ms_plan *p, void *stream, uint32_t reps, const char *cache_path, ms_tune *best,
                           float *best_ms) {
  if (!p) return fail(MS_ERR_INVALID_ARG, "plan is NULL");
  if (reps == 0) reps = 3;
  // plan signature: steps and the shapes of the inputs
  uint64_t h = 0xCBF29CE484222325ull;
  for (const ms_step &s : p->steps) h = fnv(h, &s, sizeof(s));
  for (const ms_column *c : p->inputs) {
    ms_column_info ci;
    ms_status st = ms_column_info_get(c, stream, &ci);
    if (st != MS_OK) return st;
    const uint64_t key[3] = {ci.kind, ci.bit_width, ci.n};
    h = fnv(h, key, sizeof(key));
  }
  char sig[32];
  std::snprintf(sig, sizeof(sig), "%016llx", (unsigned long long)h);
  if (cache_path) {
    if (FILE *f = std::fopen(cache_path, "r")) {
      char line[256];
      ms_tune found{0, 0, 0, 0};
      float fms = 0.f;
      while (std::fgets(line, sizeof(line), f)) {
        char k[64];
        unsigned b = 0, w = 0, c = 0, bat = 0;
        float t = 0.f;
        if (std::sscanf(line, "%63s %u %u %u %u %f", k, &b, &w, &c, &bat, &t) == 6 && std::strcmp(k, sig) == 0) {
          found = ms_tune{b, w, c, bat};
          fms = t;
        }
      }
      std::fclose(f);
      if (found.branches) {
        ms_status st = ms_plan_set_tune(p, &found);
        if (st != MS_OK) return st;
        if (best) *best = found;
        if (best_ms) *best_ms = fms;
        return MS_OK;
      }
    }
  }
  // branches x workgroups per CU, then chunks per workgroup at the best of those, then the
  // batched level-by-level launches at that grid
  static const uint32_t kBranches[] = {1, 2, 4, 8};
  static const uint32_t kWg[] = {0, 2, 4, 8, 16};  // 0: each operator's default
  static const uint32_t kChunks[] = {1, 2, 8, 16};  // besides the default of four
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(MS_ERR_HIP, "event create failed");
  ms_tune bt{1, 0, 0, 0};
  float bms = 1e30f;
  ms_status st = MS_OK;
  auto trial = [&](const ms_tune &t) {
    st = ms_plan_set_tune(p, &t);
    float ms = 0.f;
    if (st == MS_OK) st = time_replays(p, stream, reps, e0, e1, &ms);
    if (st == MS_OK && ms < bms) {
      bms = ms;
      bt = t;
    }
  };
  for (uint32_t b : kBranches)
    for (uint32_t w : kWg)
      if (st == MS_OK) trial(ms_tune{b, w, 0, 0});
  const ms_tune base = bt;
  for (uint32_t c : kChunks)
    if (st == MS_OK) trial(ms_tune{base.branches, base.wg_per_cu, c, 0});
  if (st == MS_OK) trial(ms_tune{bt.branches, bt.wg_per_cu, bt.chunks_per_wg, 1});
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != MS_OK) return st;
  st = ms_plan_set_tune(p, &bt);
  if (st != MS_OK) return st;
  if (cache_path) {
    if (FILE *f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "%s %u %u %u %u %.4f\n", sig, bt.branches, bt.wg_per_cu, bt.chunks_per_wg, bt.batch, bms);
      std::fclose(f);
    }
  }
  if (best) *best = bt;
  if (best_ms) *best_ms = bms;
  return MS_OK;
}


// Mean time (ms) of `reps` graph replays of the plan as it stands (captures first if needed).
static ms_status time_replays(ms_plan *p, void *stream, uint32_t reps, hipEvent_t e0, hipEvent_t e1, float *ms) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ms_status st = ms_plan_launch(p, stream);  // capture + warm replay
  if (st != MS_OK) return st;
  hipError_t e = hipEventRecord(e0, s);
  for (uint32_t r = 0; r < reps && st == MS_OK; r++) st = ms_plan_launch(p, stream);
  if (st != MS_OK) return st;
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  if (e != hipSuccess) return hip_fail(e, "timing");
  *ms /= (float)reps;
  return MS_OK;
}

}  // extern "C"
