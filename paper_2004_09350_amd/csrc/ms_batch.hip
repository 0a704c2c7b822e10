// ms_batch.hip -- the recorder behind batched persistent launches (declarations and rules
// in ms_batch.h).  A plan level's operators record their launches; the flush issues them
// phase by phase, one persistent launch per batched kernel kind and phase, with the
// level's task tables (argument blocks, segment prefix, ticket) in one device block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ms_batch.h"
#include "ms_kernels.h"
#include "ms_runtime.h"

namespace ms {
namespace batch {
namespace {

struct Entry {
  unsigned phase = 0;
  int kind = -1;  // BatchKind, or -1 for a recorded plain launch
  std::function<hipError_t(void *)> launch;
  std::vector<unsigned char> args;
  unsigned segs = 0;
  size_t shm = 0;
};
struct Free {
  void *p;
  uint64_t bytes;
  void *stream;
};
struct Recorder {
  std::vector<Entry> entries;
  std::vector<Free> frees;
  unsigned phase = 0;
};

thread_local Recorder *t_rec = nullptr;
constexpr unsigned kBatchWgPerCu = 4;  // persistent grid (workgroups per CU) unless the plan's tune sets one

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

}  // namespace

bool recording() { return t_rec != nullptr; }

hipError_t record_task(unsigned kind, const void *args, size_t bytes, unsigned segs, size_t shm) {
  Entry e;
  e.phase = t_rec->phase++;
  e.kind = (int)kind;
  const unsigned char *a = static_cast<const unsigned char *>(args);
  e.args.assign(a, a + bytes);
  e.segs = segs;
  e.shm = shm;
  t_rec->entries.push_back(std::move(e));
  return hipSuccess;
}

void record_launch(std::function<hipError_t(void *)> launch) {
  Entry e;
  e.phase = t_rec->phase++;
  e.launch = std::move(launch);
  t_rec->entries.push_back(std::move(e));
}

bool defer_free(void *p, uint64_t bytes, void *stream) {
  if (!t_rec) return false;
  t_rec->frees.push_back({p, bytes, stream});
  return true;
}

void begin() {
  delete t_rec;
  t_rec = new Recorder();
}

void next_op() {
  if (t_rec) t_rec->phase = 0;
}

hipError_t flush(const Streams &st, std::vector<Upload> &uploads) {
  void *const stream = st.origin;
  const bool fan = st.n_branches > 1;
  Recorder *r = t_rec;
  t_rec = nullptr;  // from here on launches and frees are issued at once
  if (!r) return hipSuccess;
  hipError_t e = hipSuccess;
  unsigned phases = 0;
  for (const Entry &x : r->entries) phases = std::max(phases, x.phase + 1);
  const rt::Arena *arena = rt::thread_arena();
  const unsigned wg = rt::thread_wg_per_cu() ? rt::thread_wg_per_cu() : kBatchWgPerCu;
  const uint64_t cap = (uint64_t)rt::cus() * wg;
  for (unsigned ph = 0; ph < phases && e == hipSuccess; ph++) {
    // the phase's launches (plain ones and one per batched kind) go round-robin over the
    // branches, which fork from the origin here and join it at the end of the phase
    unsigned count = 0;
    std::vector<bool> kinds(BK_COUNT, false);
    for (const Entry &x : r->entries) {
      if (x.phase != ph) continue;
      if (x.kind < 0) count++;
      else if (!kinds[x.kind]) kinds[x.kind] = true, count++;
    }
    const unsigned nb = fan ? std::min(count, st.n_branches) : 1u;  // branches with work in this phase
    const bool forked = nb > 1;
    if (forked) {
      e = hipEventRecord(st.fork, reinterpret_cast<hipStream_t>(stream));
      for (unsigned b = 0; b < nb && e == hipSuccess; b++)
        e = hipStreamWaitEvent(reinterpret_cast<hipStream_t>(st.branches[b]), st.fork, 0);
    }
    unsigned rr = 0;
    auto next_stream = [&]() { return forked ? st.branches[rr++ % nb] : stream; };
    for (const Entry &x : r->entries)
      if (x.phase == ph && x.kind < 0 && e == hipSuccess) e = x.launch(next_stream());
    for (unsigned kind = 0; kind < BK_COUNT && e == hipSuccess; kind++) {
      std::vector<const Entry *> tasks;
      for (const Entry &x : r->entries)
        if (x.phase == ph && x.kind == (int)kind && x.segs > 0) tasks.push_back(&x);
      if (tasks.empty()) continue;
      // longest first: big tasks' segments start early, small ones fill in behind them
      std::stable_sort(tasks.begin(), tasks.end(), [](const Entry *a, const Entry *b) { return a->segs > b->segs; });
      const uint64_t n = tasks.size(), asz = tasks[0]->args.size();
      const uint64_t off_prefix = align256(asz * n), off_ticket = off_prefix + align256(4 * (n + 1));
      const uint64_t bytes = off_ticket + 256;
      Upload up;
      up.host.assign(off_ticket, 0);
      unsigned *prefix = reinterpret_cast<unsigned *>(up.host.data() + off_prefix);
      size_t shm = 0;
      uint64_t total = 0;
      for (uint64_t i = 0; i < n; i++) {
        std::memcpy(up.host.data() + i * asz, tasks[i]->args.data(), asz);
        prefix[i] = (unsigned)total;
        total += tasks[i]->segs;
        shm = std::max(shm, tasks[i]->shm);
      }
      if (total >= (1ull << 32)) {
        e = hipErrorInvalidValue;
        break;
      }
      prefix[n] = (unsigned)total;
      void *const ks = next_stream();
      char *dev = static_cast<char *>(rt::alloc(bytes, ks));
      if (!dev) {
        e = hipErrorOutOfMemory;
        break;
      }
      up.dev = dev;
      if (!arena) {  // eager: copy now, keep the host bytes until the caller synchronises
        e = hipMemcpyAsync(dev, up.host.data(), off_ticket, hipMemcpyHostToDevice, reinterpret_cast<hipStream_t>(ks));
        uploads.push_back(std::move(up));
      } else if (!arena->measure) {  // capture: the caller copies once the capture has ended
        uploads.push_back(std::move(up));
      }
      unsigned *ticket = reinterpret_cast<unsigned *>(dev + off_ticket);
      if (e == hipSuccess) e = launch_fill_u32(ticket, 1, 0u, ks);
      const BatchQueue q{reinterpret_cast<const unsigned *>(dev + off_prefix), (unsigned)n, ticket};
      const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(total, cap));
      if (e == hipSuccess) e = launch_batch(kind, dev, q, grid, shm, ks);
      rt::free(dev, bytes, ks);
    }
    if (forked) {  // always join back (a capture must end joined)
      for (unsigned b = 0; b < nb; b++) {
        hipError_t e2 = hipEventRecord(st.join[b], reinterpret_cast<hipStream_t>(st.branches[b]));
        if (e2 == hipSuccess) e2 = hipStreamWaitEvent(reinterpret_cast<hipStream_t>(stream), st.join[b], 0);
        if (e == hipSuccess) e = e2;
      }
    }
  }
  for (const Free &f : r->frees) rt::free(f.p, f.bytes, f.stream);
  delete r;
  return e;
}

}  // namespace batch
}  // namespace ms
