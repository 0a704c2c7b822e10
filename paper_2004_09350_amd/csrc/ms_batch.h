// ms_batch.h -- recording a plan level's kernel launches and issuing them as batched
// persistent launches (host side; the device side is batch_run in ms_kcommon.h).
//
// While a thread records, every kernel launch of the library is held back: launchers with
// a batched kernel (BatchKind) record their argument block and workgroup count, any other
// launch records itself as a closure, and frees of device memory wait for the flush.
// Launch i of an operator (counted from next_op) belongs to phase i.  flush issues the
// phases in order; within a phase, the tasks of one batched kind become one launch of that
// kind's persistent kernel (tasks in decreasing size, workgroups taking tickets), and these
// launches and the closures are spread round-robin over the branch streams, which fork from
// the origin before the phase and join it after.  Operators recorded together
// must be independent of each other: only an operator's own earlier launches (earlier
// phases) order its work.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <vector>

namespace ms {
namespace batch {

bool recording();
hipError_t record_task(unsigned kind, const void *args, size_t bytes, unsigned segs, size_t shm);
void record_launch(std::function<hipError_t(void *stream)> launch);
// Queues a free until the flush while recording (returns false when not recording).
bool defer_free(void *p, uint64_t bytes, void *stream);

// A task table for the device: copied by the flush itself on an eager run (`host` is then
// kept until the caller synchronises), by the caller after the capture on a real capture,
// not at all on a measuring capture.
struct Upload {
  void *dev = nullptr;
  std::vector<unsigned char> host;
};

void begin();    // start recording on this thread
void next_op();  // the next launches start a new operator (phase 0)
// Streams of a flush: the n_branches branch streams (origin itself when n_branches < 2),
// forked from `origin` with `fork` and joined back with join[b].
struct Streams {
  void *origin = nullptr;
  void *const *branches = nullptr;
  unsigned n_branches = 0;
  hipEvent_t fork = nullptr;
  const hipEvent_t *join = nullptr;
};
// Issues everything recorded since begin, runs the deferred frees and stops recording
// (also after an error).
hipError_t flush(const Streams &st, std::vector<Upload> &uploads);

}  // namespace batch
}  // namespace ms
