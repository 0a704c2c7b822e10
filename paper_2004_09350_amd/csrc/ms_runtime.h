// ms_runtime.h -- host-side hooks of the column library used by the plan executor:
// per-thread allocation arena (for graph capture) and launch-shape override.
#pragma once
#include <cstdint>

struct ms_column;

namespace ms {
namespace rt {

// A bump arena.  While set for a thread, every device allocation of the library on that
// thread is carved from it and frees are no-ops.  measure = true hands out addresses
// from kMeasureBase without backing memory: only for sizing a capture that is never run.
struct Arena {
  char *base = nullptr;
  uint64_t size = 0;
  uint64_t used = 0;
  bool measure = false;
};
constexpr uint64_t kMeasureBase = 1ull << 44;

void set_thread_arena(Arena *a);
Arena *thread_arena();
// Persistent-grid cap in workgroups per compute unit for launches from this thread.
void set_thread_wg_per_cu(unsigned w);
unsigned thread_wg_per_cu();
// Chunks per workgroup that size the persistent grid (0: the default of four).
void set_thread_chunks_per_wg(unsigned c);
void *alloc(uint64_t bytes, void *stream);
void free(void *p, uint64_t bytes, void *stream);
unsigned cus();
bool initialized();
void set_error(const char *msg);
uint64_t column_rows_cap(const ms_column *c);

}  // namespace rt
}  // namespace ms
