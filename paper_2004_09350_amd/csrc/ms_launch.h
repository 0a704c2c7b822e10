// ms_launch.h -- host-side launch helpers for the kernel translation units.
//
// The kernels are split over several translation units so that they compile in
// parallel; every unit that launches kernels includes this header.
#pragma once
#include <hip/hip_runtime.h>

#include "ms_batch.h"
#include "ms_device.h"
#include "ms_kernels.h"

namespace ms {

// Per-launch timing, recorded with two events on the launch's stream when enabled.
int prof_begin(const char *name, void *stream);  // record index, or -1 when not timing
void prof_end(int rec, void *stream);
struct ProfScope {
  int rec;
  void *s;
  ProfScope(const char *name, void *stream) : rec(prof_begin(name, stream)), s(stream) {}
  ~ProfScope() {
    if (rec >= 0) prof_end(rec, s);
  }
};

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Dynamic LDS of the kernels that stage RLE input runs (kRing * 512 words per wave):
// only an RLE input needs it, so other inputs keep the occupancy of the static buffers.
constexpr size_t kRingBytes = sizeof(unsigned) * kWaves * kRing * kBlk;
constexpr unsigned long long kLdsBitmapBits = 32ull * kWaves * kRing * kBlk;
inline size_t ring_shm(const ColView &c) { return c.kind == RLE ? kRingBytes : 0; }

// While the thread records a batch (ms_batch.h) the launch is held back as a closure over
// copies of its arguments and issued by the flush, on the stream the flush gives it.
#define MS_LAUNCH_SHM(name, kern, grid, block, shm, stream, ...)                          \
  do {                                                                                    \
    if (::ms::batch::recording()) {                                                       \
      ::ms::batch::record_launch([=](void *st_) {                                         \
        ProfScope ps_(name, st_);                                                         \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), shm, S(st_), __VA_ARGS__);      \
        return hipGetLastError();                                                         \
      });                                                                                 \
    } else {                                                                              \
      ProfScope ps_(name, stream);                                                        \
      hipLaunchKernelGGL(kern, dim3(grid), dim3(block), shm, S(stream), __VA_ARGS__);     \
    }                                                                                     \
  } while (0)
#define MS_LAUNCH_NAMED(name, kern, grid, block, stream, ...) \
  MS_LAUNCH_SHM(name, kern, grid, block, 0, stream, __VA_ARGS__)
#define MS_LAUNCH(kern, grid, block, stream, ...) MS_LAUNCH_NAMED(#kern, kern, grid, block, stream, __VA_ARGS__)

// The device error word: init_err_word allocates it and points every unit's copy of
// g_err_word at it (each unit registers its setter from a static initialiser).
using ErrWordSetter = bool (*)(unsigned *word);
void register_err_word_setter(ErrWordSetter f);
namespace {
bool set_unit_err_word(unsigned *word) {
  unsigned *back = nullptr;  // read back: a unit whose pointer is not set must fail here, not in a kernel
  return hipMemcpyToSymbol(HIP_SYMBOL(g_err_word), &word, sizeof(word)) == hipSuccess &&
         hipMemcpyFromSymbol(&back, HIP_SYMBOL(g_err_word), sizeof(back)) == hipSuccess && back == word;
}
const bool g_err_setter_registered = (register_err_word_setter(set_unit_err_word), true);
}  // namespace

inline const char *out_kind_suffix(unsigned k) {
  static const char *const n[] = {"UNCOMPR", "STATIC_BP", "DYN_BP", "DELTA_DYN_BP", "FOR_DYN_BP"};
  return k < 5 ? n[k] : "?";
}

}  // namespace ms
