// ms_api.hip -- the C ABI of libmorphgpu.so: columns, allocation, operator entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/morphgpu.h"
#include "ms_batch.h"
#include "ms_kernels.h"
#include "ms_runtime.h"

using namespace ms;

struct ms_column {
  uint32_t kind;
  uint32_t width;          // static BP: explicit width, or the widest possible (32) for auto
  uint64_t n_cap;          // capacity in values
  uint64_t n_host;         // element count known on the host, or UINT64_MAX
  uint64_t nb_cap;         // DynBP-family block capacity
  uint64_t payload_cap;    // payload words the buffer holds (without slack)
  void *buf;               // owned device buffer
  uint64_t buf_bytes;
  void *stream;            // stream the buffer was allocated on
  ColView v;
  uint32_t sorted;
  bool arena;              // buffer lives in a plan's arena (never freed on its own)
};

namespace {

constexpr uint64_t kUnknown = ~0ull;
constexpr uint64_t kGroupByMaxDomain = 1ull << 28;  // presence bitmap of at most 32 MB

ms_alloc_fn g_alloc = nullptr;
ms_free_fn g_free = nullptr;
void *g_ctx = nullptr;
bool g_init = false;
int g_cus = 256;
thread_local std::string t_err;

ms_status fail(ms_status st, const std::string &msg) {
  t_err = msg;
  return st;
}

ms_status hip_fail(hipError_t e, const char *what) {
  return fail(MS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Allocation goes to the calling thread's arena while one is set (plan capture), else to
// the registered callbacks, else to hipMallocAsync.
thread_local rt::Arena *t_arena = nullptr;
thread_local unsigned t_wg_per_cu = 0;  // 0: each operator's default
thread_local unsigned t_chunks_per_wg = 0;  // 0: the default of four

void *dev_alloc(uint64_t bytes, void *stream) {
  if (bytes == 0) bytes = 256;
  if (t_arena) {
    const uint64_t at = (t_arena->used + 255) & ~255ull;
    t_arena->used = at + bytes;
    if (t_arena->measure) return reinterpret_cast<void *>(rt::kMeasureBase + at);
    if (t_arena->used > t_arena->size) return nullptr;
    return t_arena->base + at;
  }
  if (g_alloc) return g_alloc(bytes, stream, g_ctx);
  void *p = nullptr;
  if (hipMallocAsync(&p, bytes, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return nullptr;
  return p;
}

void dev_free(void *p, uint64_t bytes, void *stream) {
  if (!p || t_arena) return;
  if (bytes == 0) bytes = 256;
  if (batch::defer_free(p, bytes, stream)) return;  // its users are recorded, not yet issued
  if (g_free)
    g_free(p, bytes, stream, g_ctx);
  else
    (void)hipFreeAsync(p, reinterpret_cast<hipStream_t>(stream));
}

struct Scratch {
  void *stream;
  std::vector<std::pair<void *, uint64_t>> blocks;
  bool ok = true;
  explicit Scratch(void *s) : stream(s) {}
  template <class T>
  T *get(uint64_t count) {
    uint64_t bytes = std::max<uint64_t>(count * sizeof(T), 256);
    void *p = dev_alloc(bytes, stream);
    if (!p) {
      ok = false;
      return nullptr;
    }
    blocks.push_back({p, bytes});
    return reinterpret_cast<T *>(p);
  }
  ~Scratch() {
    for (auto &b : blocks) dev_free(b.first, b.second, stream);
  }
};

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// Persistent grid: one workgroup per four chunks (or the plan's chunks_per_wg), capped at
// wg_per_cu workgroups per CU (the plan's tune, else the operator's default: a multiple of
// the workgroups one CU holds at once, so that the last round of workgroups is not a
// partial one).
constexpr unsigned kWgPerCuDefault = 4;
constexpr unsigned kWgPerCuProject = 3;  // the gather kernels hold three workgroups per CU
constexpr unsigned kChunksPerWgDefault = 4;
unsigned grid_for(uint64_t chunks, unsigned dflt = kWgPerCuDefault) {
  uint64_t max_wg = (uint64_t)g_cus * (t_wg_per_cu ? t_wg_per_cu : dflt);
  const uint64_t cpw = t_chunks_per_wg ? t_chunks_per_wg : kChunksPerWgDefault;
  uint64_t g = (chunks + cpw - 1) / cpw;
  if (g < 1) g = 1;
  if (g > max_wg) g = max_wg;
  return (unsigned)g;
}

uint64_t chunks_of(uint64_t n) { return (n + kBlk - 1) / kBlk; }

bool valid_kind(uint32_t k) { return k <= MS_RLE; }

// Allocate a column of `kind` with room for n_cap values (payload_words: explicit
// payload size for canonical layouts, or kUnknown for the worst case).
ms_status alloc_column(uint32_t kind, uint32_t width, uint64_t n_cap, uint64_t nb_exact, uint64_t payload_words,
                       void *stream, ms_column **out) {
  *out = nullptr;
  ms_column *c = new ms_column();
  c->kind = kind;
  c->width = width;
  c->n_cap = n_cap;
  c->n_host = kUnknown;
  c->stream = stream;
  c->sorted = 0;
  c->arena = t_arena != nullptr;
  std::memset(&c->v, 0, sizeof(c->v));
  c->v.kind = kind;
  c->v.width = width;
  c->v.n_cap = n_cap;
  uint64_t off = align256(sizeof(ColHdr));
  uint64_t o_widths = 0, o_offsets = 0, o_bases = 0, o_rem = 0, o_payload = 0, o_rv = 0, o_rs = 0;
  switch (kind) {
    case MS_UNCOMPR:
      o_payload = off;
      c->payload_cap = n_cap;
      off += align256(4 * n_cap + 64);
      break;
    case MS_STATIC_BP: {
      o_rem = off;
      off += align256(4 * 32);
      o_payload = off;
      uint64_t w = (width > 32) ? 32 : width;
      c->payload_cap = (payload_words != kUnknown) ? payload_words : (n_cap * w + 31) / 32;
      off += align256(4 * (c->payload_cap + kPayloadSlackWords));
      break;
    }
    case MS_DYN_BP:
    case MS_DELTA_DYN_BP:
    case MS_FOR_DYN_BP: {
      uint64_t nb = (nb_exact != kUnknown) ? nb_exact : n_cap / kBlk;
      c->nb_cap = nb;
      o_widths = off;
      off += align256(nb + 16);
      o_offsets = off;
      off += align256(4 * nb + 16);
      o_bases = off;
      off += align256(4 * nb + 16);
      o_rem = off;
      off += align256(4 * kBlk);
      o_payload = off;
      c->payload_cap = (payload_words != kUnknown) ? payload_words : nb * kBlk;
      off += align256(4 * (c->payload_cap + kPayloadSlackWords));
      break;
    }
    case MS_RLE:
      o_rv = off;
      off += align256(4 * n_cap + 16);
      o_rs = off;
      off += align256(4 * n_cap + 16);
      c->payload_cap = 0;
      break;
    default: delete c; return fail(MS_ERR_INVALID_ARG, "bad format kind");
  }
  c->v.payload_cap = c->payload_cap;
  c->buf_bytes = off;
  c->buf = dev_alloc(off, stream);
  if (!c->buf) {
    delete c;
    return fail(MS_ERR_OOM, "device allocation failed");
  }
  char *b = reinterpret_cast<char *>(c->buf);
  c->v.hdr = reinterpret_cast<ColHdr *>(b);
  if (o_widths) c->v.widths = reinterpret_cast<unsigned char *>(b + o_widths);
  if (o_offsets) c->v.offsets = reinterpret_cast<unsigned *>(b + o_offsets);
  if (o_bases) c->v.bases = reinterpret_cast<unsigned *>(b + o_bases);
  if (o_rem) c->v.rem = reinterpret_cast<unsigned *>(b + o_rem);
  if (o_payload) c->v.payload = reinterpret_cast<unsigned *>(b + o_payload);
  if (o_rv) c->v.rvalues = reinterpret_cast<unsigned *>(b + o_rv);
  if (o_rs) c->v.rstarts = reinterpret_cast<unsigned *>(b + o_rs);
  *out = c;
  return MS_OK;
}

void free_column(ms_column *c) {
  if (!c) return;
  if (!c->arena) dev_free(c->buf, c->buf_bytes, c->stream);
  delete c;
}

ms_status check_fmt(ms_format f) {
  if (!valid_kind(f.kind)) return fail(MS_ERR_INVALID_ARG, "unknown output format");
  if (f.kind == MS_STATIC_BP && f.bit_width != MS_BW_AUTO && f.bit_width > 32)
    return fail(MS_ERR_INVALID_ARG, "static BP width must be 0..32 or auto");
  return MS_OK;
}

ms_status check_init() { return g_init ? MS_OK : fail(MS_ERR_NOT_INITIALIZED, "ms_init not called"); }

// Output column for a producer of at most n_cap values.
ms_status make_output(ms_format fmt, uint64_t n_cap, void *stream, ms_column **out, unsigned &auto_w) {
  auto_w = (fmt.kind == MS_STATIC_BP && fmt.bit_width == MS_BW_AUTO) ? 1u : 0u;
  uint32_t w = (fmt.kind == MS_STATIC_BP) ? (auto_w ? 32u : fmt.bit_width) : 0u;
  ms_status st = alloc_column(fmt.kind, w, n_cap, kUnknown, kUnknown, stream, out);
  if (st != MS_OK) return st;
  (*out)->v.width = w;
  return MS_OK;
}

ms_status launched(hipError_t e, ms_column **out) {
  if (e != hipSuccess) {
    if (out && *out) {
      free_column(*out);
      *out = nullptr;
    }
    return hip_fail(e, "kernel launch");
  }
  return MS_OK;
}

// Header of a count-known producer's output: count from `n_src`, ORs from the partials,
// auto-width static BP narrowed to its main part.
hipError_t finish_produced(const ColView &out, const ColHdr *n_src, const unsigned *partials, unsigned G,
                           unsigned auto_w, unsigned sorted, unsigned *narrow_tmp, void *stream) {
  FinishArgs f{};
  f.out = out;
  f.n_src = n_src;
  f.partials = partials;
  f.G = G;
  f.Wp = out.width;
  f.auto_w = auto_w;
  f.sorted = sorted;
  f.mode = 0;
  hipError_t e = hipSuccess;
  if (out.kind == MS_STATIC_BP && auto_w) e = launch_narrow(f, narrow_tmp, G, stream);
  if (e == hipSuccess) e = launch_finish(f, stream);
  return e;
}

ms_status read_hdr(const ms_column *c, void *stream, ColHdr &h) {
  hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "stream sync");
  e = hipMemcpy(&h, c->v.hdr, sizeof(ColHdr), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "header copy");
  return MS_OK;
}

// Two-phase compaction shared by select, semi-join and intersect.
ms_status compaction(const ms_column *in, const PredArgs &pa_in, bool emit_values, bool check_sorted, ms_format fmt,
                     void *stream, ms_column **out) {
  *out = nullptr;
  ms_status st = check_fmt(fmt);
  if (st != MS_OK) return st;
  const uint64_t n_cap = in->n_host != kUnknown ? in->n_host : in->n_cap;
  const uint64_t C = chunks_of(n_cap);
  const unsigned G = grid_for(C);
  unsigned auto_w = 0;
  st = make_output(fmt, n_cap, stream, out, auto_w);
  if (st != MS_OK) return st;
  Scratch sc(stream);
  const bool blocky = fmt.kind != MS_UNCOMPR && fmt.kind != MS_RLE;
  PredArgs pa = pa_in;
  pa.in = in->v;
  pa.bitmask = sc.get<unsigned char>(C * 64 + 64);
  pa.seg_count = sc.get<unsigned>(G);
  pa.seg_or = sc.get<unsigned>(G);
  pa.chunk_first = check_sorted ? sc.get<unsigned>(C + 1) : nullptr;
  pa.chunk_last = check_sorted ? sc.get<unsigned>(C + 1) : nullptr;
  EmitArgs ea;
  std::memset(&ea, 0, sizeof(ea));
  ea.in = in->v;
  ea.out = (*out)->v;
  ea.auto_w = auto_w;
  ea.emit_values = emit_values ? 1u : 0u;
  ea.check_sorted = check_sorted ? 1u : 0u;
  ea.bitmask = pa.bitmask;
  ea.seg_count = pa.seg_count;
  ea.seg_or = pa.seg_or;
  ea.chunk_first = pa.chunk_first;
  ea.chunk_last = pa.chunk_last;
  ea.stage_g = blocky ? sc.get<unsigned>(n_cap + 1) : nullptr;
  ea.wave_count = sc.get<unsigned>(2ull * kWaves * G);
  ea.partials = sc.get<unsigned>(2 * G);
  unsigned *narrow_tmp = (fmt.kind == MS_STATIC_BP && auto_w) ? sc.get<unsigned>(n_cap + kPayloadSlackWords) : nullptr;
  if (!sc.ok) {
    free_column(*out);
    *out = nullptr;
    return fail(MS_ERR_OOM, "scratch allocation failed");
  }
  hipError_t e = launch_pred(pa, G, stream);
  if (e == hipSuccess) e = launch_emit(ea, G, stream);
  if (e == hipSuccess && fmt.kind == MS_STATIC_BP && auto_w)
    e = finish_produced((*out)->v, nullptr, ea.partials, G, 1, 1, narrow_tmp, stream);
  st = launched(e, out);
  if (st == MS_OK) (*out)->sorted = 1;
  return st;
}

// ---------------------------------------------------------------------------------------------
// Group-sum shared by ms_group_sum and ms_group_sum_noalloc.
constexpr uint32_t kMaxLdsGroupsHost = 4096;  // the kernel's LDS histogram holds this many groups

ms_status group_sum_check(const ms_column *groups, const ms_column *vals, uint32_t G_groups, const uint64_t *dev_out) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!groups || !vals) return fail(MS_ERR_INVALID_ARG, "input is NULL");
  if (G_groups && !dev_out) return fail(MS_ERR_INVALID_ARG, "output is NULL");
  if (groups->n_host != kUnknown && vals->n_host != kUnknown && groups->n_host != vals->n_host)
    return fail(MS_ERR_LENGTH_MISMATCH, "groups and values differ in length");
  return MS_OK;
}

// Workgroups of the group-sum kernel: the persistent grid, at most one per CU (the
// partials are G x groups), and at most what max_partials partial sums allow.
unsigned group_sum_grid(const ms_column *groups, const ms_column *vals, uint32_t G_groups, uint64_t max_partials) {
  const uint64_t n_cap = std::min(groups->n_host != kUnknown ? groups->n_host : groups->n_cap,
                                  vals->n_host != kUnknown ? vals->n_host : vals->n_cap);
  uint64_t G = grid_for(chunks_of(n_cap));
  if (G > (uint64_t)g_cus) G = (uint64_t)g_cus;
  if (G_groups <= kMaxLdsGroupsHost) G = std::min<uint64_t>(G, std::max<uint64_t>(max_partials / G_groups, 1));
  return (unsigned)G;
}

// partials: G x G_groups sums (LDS path) or G_groups sums that must start at zero.
ms_status group_sum_launch(const ms_column *groups, const ms_column *vals, uint32_t G_groups, uint64_t *dev_out,
                           unsigned G, unsigned long long *partials, void *stream) {
  hipError_t e = hipSuccess;
  if (G_groups > kMaxLdsGroupsHost) e = launch_fill_u64(partials, G_groups, 0ull, stream);  // a kernel, not a memset
  if (e == hipSuccess)
    e = launch_group_sum(groups->v, vals->v, G_groups, reinterpret_cast<unsigned long long *>(dev_out), G, partials,
                         stream);
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

// ---------------------------------------------------------------------------------------------
// Static scratch of the allocation-free entry point: 2 MiB of partial sums in the library's
// own device memory (each device holds its copy until the process ends).  In host code the
// name `scratch` is a host-side stand-in, never a device address: the device address is
// looked up once per device and kept in g_scratch_dev.
constexpr uint64_t kNoAllocScratchU64 = 1ull << 18;
constexpr uint32_t kNoAllocMaxGroups = (uint32_t)kNoAllocScratchU64;
static __device__ __align__(256) unsigned long long scratch[kNoAllocScratchU64];
constexpr int kMaxDevices = 64;
unsigned long long *g_scratch_dev[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on the first use on that device
// when ms_init ran on another one).
ms_status noalloc_scratch(unsigned long long **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(MS_ERR_UNSUPPORTED, "device index beyond the scratch table");
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_scratch_dev[dev] = static_cast<unsigned long long *>(ptr);
  }
  *out = g_scratch_dev[dev];
  return MS_OK;
}

}  // namespace

namespace ms {
namespace rt {
void set_thread_arena(Arena *a) { t_arena = a; }
Arena *thread_arena() { return t_arena; }
void set_thread_wg_per_cu(unsigned w) { t_wg_per_cu = w; }
unsigned thread_wg_per_cu() { return t_wg_per_cu; }
void set_thread_chunks_per_wg(unsigned c) { t_chunks_per_wg = c; }
void *alloc(uint64_t bytes, void *stream) { return dev_alloc(bytes, stream); }
void free(void *p, uint64_t bytes, void *stream) { dev_free(p, bytes, stream); }
unsigned cus() { return (unsigned)g_cus; }
bool initialized() { return g_init; }
void set_error(const char *msg) { t_err = msg; }
uint64_t column_rows_cap(const ms_column *c) { return c->n_host != kUnknown ? c->n_host : c->n_cap; }
}  // namespace rt
}  // namespace ms

extern "C" {

ms_status ms_init(ms_alloc_fn alloc, ms_free_fn free_fn, void *ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr)) return fail(MS_ERR_INVALID_ARG, "give both callbacks or neither");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  g_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  e = init_err_word();
  if (e != hipSuccess) return hip_fail(e, "device error word");
  unsigned long long *scratch_dev = nullptr;
  ms_status sst = noalloc_scratch(&scratch_dev);
  if (sst != MS_OK) return sst;
  g_alloc = alloc;
  g_free = free_fn;
  g_ctx = ctx;
  g_init = true;
  return MS_OK;
}

const char *ms_last_error(void) { return t_err.c_str(); }

ms_status ms_column_free(ms_column *col) {
  free_column(col);
  return MS_OK;
}

ms_status ms_column_wrap_uncompr(const uint32_t *dev_vals, uint64_t n, void *stream, ms_column **out) {
  if (!out) return fail(MS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (n >= (1ull << 32)) return fail(MS_ERR_INVALID_ARG, "columns hold fewer than 2^32 values");
  if (n > 0 && (!dev_vals || (reinterpret_cast<uintptr_t>(dev_vals) & 15)))
    return fail(MS_ERR_INVALID_ARG, "values must be a 16-byte aligned device pointer");
  ms_column *c = new ms_column();
  c->kind = MS_UNCOMPR;
  c->width = 0;
  c->n_cap = n;
  c->n_host = n;
  c->nb_cap = 0;
  c->payload_cap = n;
  c->stream = stream;
  c->sorted = 0;
  c->buf_bytes = align256(sizeof(ColHdr));
  c->buf = dev_alloc(c->buf_bytes, stream);
  if (!c->buf) {
    delete c;
    return fail(MS_ERR_OOM, "device allocation failed");
  }
  std::memset(&c->v, 0, sizeof(c->v));
  c->v.kind = MS_UNCOMPR;
  c->v.hdr = reinterpret_cast<ColHdr *>(c->buf);
  c->v.payload = const_cast<unsigned *>(dev_vals);
  c->v.n_cap = n;
  c->v.payload_cap = n;
  hipError_t e = launch_set_hdr(c->v.hdr, n, 0, 0, 0, 0, 0, stream);
  Scratch sc(stream);
  const unsigned G = grid_for(chunks_of(n));
  unsigned *partials = sc.get<unsigned>(2 * G);
  if (!sc.ok) {
    free_column(c);
    return fail(MS_ERR_OOM, "scratch allocation failed");
  }
  if (e == hipSuccess) e = launch_colstats(c->v, G, partials, stream);
  if (e != hipSuccess) {
    free_column(c);
    return hip_fail(e, "kernel launch");
  }
  *out = c;
  return MS_OK;
}

ms_status ms_morph(const ms_column *in, ms_format fmt, void *stream, ms_column **out) {
  if (!out) return fail(MS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!in) return fail(MS_ERR_INVALID_ARG, "input is NULL");
  st = check_fmt(fmt);
  if (st != MS_OK) return st;
  const uint64_t n_cap = in->n_host != kUnknown ? in->n_host : in->n_cap;
  const unsigned G = grid_for(chunks_of(n_cap));
  unsigned auto_w = 0;
  st = make_output(fmt, n_cap, stream, out, auto_w);
  if (st != MS_OK) return st;
  Scratch sc(stream);
  unsigned *partials = sc.get<unsigned>(2 * G);
  unsigned *seg = (fmt.kind == MS_RLE) ? sc.get<unsigned>(kWaves * G) : nullptr;  // runs per wave
  unsigned *narrow_tmp = (fmt.kind == MS_STATIC_BP && auto_w) ? sc.get<unsigned>(n_cap + kPayloadSlackWords) : nullptr;
  if (!sc.ok) {
    free_column(*out);
    *out = nullptr;
    return fail(MS_ERR_OOM, "scratch allocation failed");
  }
  hipError_t e;
  if (fmt.kind == MS_RLE)
    e = launch_rle(0, in->v, in->v, (*out)->v, G, seg, partials, stream);
  else
    e = launch_morph(in->v, (*out)->v, auto_w, G, partials, stream);
  if (e == hipSuccess)
    e = finish_produced((*out)->v, in->v.hdr, partials, G, auto_w, in->sorted, narrow_tmp, stream);
  st = launched(e, out);
  if (st == MS_OK) {
    (*out)->n_host = in->n_host;
    (*out)->sorted = in->sorted;
  }
  return st;
}

ms_status ms_column_shrink(ms_column *col, void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!col) return fail(MS_ERR_INVALID_ARG, "column is NULL");
  if (col->arena) return fail(MS_ERR_INVALID_ARG, "a plan's result column cannot be shrunk");
  ColHdr h;
  st = read_hdr(col, stream, h);
  if (st != MS_OK) return st;
  const uint64_t n = h.n;
  ms_column *nc = nullptr;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  switch (col->kind) {
    case MS_UNCOMPR: {
      if (col->buf_bytes <= align256(sizeof(ColHdr))) {  // wrapped: nothing owned to shrink
        col->n_host = n;
        return MS_OK;
      }
      st = alloc_column(MS_UNCOMPR, 0, n, kUnknown, kUnknown, stream, &nc);
      if (st != MS_OK) return st;
      if (n) e = hipMemcpyAsync(nc->v.payload, col->v.payload, 4 * n, hipMemcpyDeviceToDevice, s);
      break;
    }
    case MS_STATIC_BP: {
      const uint64_t n_main = n & ~31ull;
      const uint64_t words = n_main * h.sbp_width / 32;
      st = alloc_column(MS_STATIC_BP, h.sbp_width, n, kUnknown, words, stream, &nc);
      if (st != MS_OK) return st;
      if (words) e = hipMemcpyAsync(nc->v.payload, col->v.payload, 4 * words, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess && n > n_main)
        e = hipMemcpyAsync(nc->v.rem, col->v.rem, 4 * (n - n_main), hipMemcpyDeviceToDevice, s);
      break;
    }
    case MS_DYN_BP:
    case MS_DELTA_DYN_BP:
    case MS_FOR_DYN_BP: {
      const uint64_t n_main = n & ~511ull, nb = n_main / kBlk;
      std::vector<unsigned char> widths(nb);
      if (nb) {
        e = hipMemcpy(widths.data(), col->v.widths, nb, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "widths copy");
      }
      std::vector<unsigned> noff(nb + 1);
      uint64_t words = 0;
      for (uint64_t k = 0; k < nb; k++) {
        noff[k] = (unsigned)words;
        words += 16ull * widths[k];
      }
      st = alloc_column(col->kind, 0, n, nb, words, stream, &nc);
      if (st != MS_OK) return st;
      Scratch sc(stream);
      unsigned *d_noff = sc.get<unsigned>(nb + 1);
      if (!sc.ok) {
        free_column(nc);
        return fail(MS_ERR_OOM, "scratch allocation failed");
      }
      if (nb) {
        e = hipMemcpyAsync(nc->v.widths, col->v.widths, nb, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(nc->v.bases, col->v.bases, 4 * nb, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(nc->v.offsets, noff.data(), 4 * nb, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_noff, noff.data(), 4 * nb, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
          e = launch_shrink_payload(col->v.payload, col->v.offsets, col->v.widths, d_noff, nc->v.payload, nb, stream);
      }
      if (e == hipSuccess && n > n_main)
        e = hipMemcpyAsync(nc->v.rem, col->v.rem, 4 * (n - n_main), hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);  // noff lives on the host stack
      break;
    }
    case MS_RLE: {
      st = alloc_column(MS_RLE, 0, h.runs, kUnknown, kUnknown, stream, &nc);
      if (st != MS_OK) return st;
      if (h.runs) {
        e = hipMemcpyAsync(nc->v.rvalues, col->v.rvalues, 4 * h.runs, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
          e = hipMemcpyAsync(nc->v.rstarts, col->v.rstarts, 4 * h.runs, hipMemcpyDeviceToDevice, s);
      }
      nc->n_cap = n;
      nc->v.n_cap = h.runs;
      break;
    }
    default: return fail(MS_ERR_INVALID_ARG, "bad column");
  }
  if (e == hipSuccess) e = hipMemcpyAsync(nc->v.hdr, col->v.hdr, sizeof(ColHdr), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) {
    free_column(nc);
    return hip_fail(e, "shrink copy");
  }
  // swap the new buffer into the caller's handle
  dev_free(col->buf, col->buf_bytes, col->stream);
  col->buf = nc->buf;
  col->buf_bytes = nc->buf_bytes;
  col->stream = stream;
  col->v = nc->v;
  col->v.n_cap = (col->kind == MS_RLE) ? h.runs : n;
  col->n_cap = n;
  col->nb_cap = nc->nb_cap;
  col->payload_cap = nc->payload_cap;
  col->width = (col->kind == MS_STATIC_BP) ? h.sbp_width : 0;
  col->v.width = col->width;
  col->n_host = n;
  delete nc;
  return MS_OK;
}

ms_status ms_column_encode(const uint32_t *dev_vals, uint64_t n, ms_format fmt, void *stream, ms_column **out) {
  if (!out) return fail(MS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ms_column *raw = nullptr;
  ms_status st = ms_column_wrap_uncompr(dev_vals, n, stream, &raw);
  if (st != MS_OK) return st;
  st = ms_morph(raw, fmt, stream, out);
  if (st == MS_OK) {
    st = ms_column_shrink(*out, stream);
    if (st != MS_OK) {
      free_column(*out);
      *out = nullptr;
    }
  }
  (void)hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  free_column(raw);
  return st;
}

ms_status ms_column_decode(const ms_column *col, uint32_t *dev_out, void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!col) return fail(MS_ERR_INVALID_ARG, "column is NULL");
  const uint64_t n_cap = col->n_host != kUnknown ? col->n_host : col->n_cap;
  if (n_cap && !dev_out) return fail(MS_ERR_INVALID_ARG, "output is NULL");
  if (reinterpret_cast<uintptr_t>(dev_out) & 15) return fail(MS_ERR_INVALID_ARG, "output must be 16-byte aligned");
  hipError_t e = launch_decode(col->v, dev_out, grid_for(chunks_of(n_cap)), stream);
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

ms_status ms_column_info_get(const ms_column *col, void *stream, ms_column_info *out) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!col || !out) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  ColHdr h;
  st = read_hdr(col, stream, h);
  if (st != MS_OK) return st;
  std::memset(out, 0, sizeof(*out));
  out->n = h.n;
  out->kind = col->kind;
  out->or_all = h.or_all;
  out->sorted = h.sorted | col->sorted;
  out->capacity_bytes = col->buf_bytes;
  const uint64_t n = h.n;
  switch (col->kind) {
    case MS_UNCOMPR:
      out->n_main = n;
      out->payload_words = n;
      out->payload_extent = n;
      out->footprint = 4 * n;
      break;
    case MS_STATIC_BP:
      out->bit_width = h.sbp_width;
      out->n_main = n & ~31ull;
      out->n_rem = n - out->n_main;
      out->payload_words = out->n_main * h.sbp_width / 32;
      out->payload_extent = out->payload_words;
      out->footprint = 4 * out->payload_words + 4 * out->n_rem;
      break;
    case MS_RLE:
      out->n_main = n;
      out->runs = h.runs;
      out->footprint = 8 * h.runs;
      break;
    default: {
      out->n_main = n & ~511ull;
      out->n_rem = n - out->n_main;
      const uint64_t nb = out->n_main / kBlk;
      out->n_blocks = nb;
      std::vector<unsigned char> w(nb);
      std::vector<unsigned> o(nb);
      if (nb) {
        hipError_t e = hipMemcpy(w.data(), col->v.widths, nb, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(o.data(), col->v.offsets, 4 * nb, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "metadata copy");
      }
      uint64_t words = 0, extent = 0;
      for (uint64_t k = 0; k < nb; k++) {
        words += 16ull * w[k];
        extent = std::max<uint64_t>(extent, (uint64_t)o[k] + 16ull * w[k]);
      }
      out->payload_words = words;
      out->payload_extent = extent;
      out->footprint = (col->kind == MS_DYN_BP ? 5 : 9) * nb + 4 * words + 4 * out->n_rem;
    }
  }
  return MS_OK;
}

ms_status ms_column_read_section(const ms_column *col, ms_section sec, void *host_dst, uint64_t bytes, void *stream,
                                 uint64_t *copied) {
  ms_column_info info;
  ms_status st = ms_column_info_get(col, stream, &info);
  if (st != MS_OK) return st;
  const void *src = nullptr;
  uint64_t size = 0;
  switch (sec) {
    case MS_SEC_WIDTHS: src = col->v.widths; size = info.n_blocks; break;
    case MS_SEC_OFFSETS: src = col->v.offsets; size = 4 * info.n_blocks; break;
    case MS_SEC_BASES: src = col->v.bases; size = 4 * info.n_blocks; break;
    case MS_SEC_PAYLOAD: src = col->v.payload; size = 4 * info.payload_extent; break;
    case MS_SEC_REM: src = col->v.rem; size = 4 * info.n_rem; break;
    case MS_SEC_RVALUES: src = col->v.rvalues; size = 4 * info.runs; break;
    case MS_SEC_RSTARTS: src = col->v.rstarts; size = 4 * info.runs; break;
    default: return fail(MS_ERR_INVALID_ARG, "bad section");
  }
  const uint64_t nbytes = std::min(bytes, size);
  if (nbytes && (!src || !host_dst)) return fail(MS_ERR_INVALID_ARG, "section not present");
  if (nbytes) {
    hipError_t e = hipMemcpy(host_dst, src, nbytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "section copy");
  }
  if (copied) *copied = nbytes;
  return MS_OK;
}

ms_status ms_select(const ms_column *in, ms_cmp cmp, uint32_t c0, uint32_t c1, ms_format fmt, void *stream,
                    ms_column **out) {
  if (!out) return fail(MS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!in) return fail(MS_ERR_INVALID_ARG, "input is NULL");
  PredArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.mode = 0;
  // every comparison becomes "v - lo <= span" (unsigned), possibly negated
  unsigned lo = 0, span = 0, neg = 0;
  bool never = false;
  switch (cmp) {
    case MS_EQ: lo = c0; span = 0; break;
    case MS_NE: lo = c0; span = 0; neg = 1; break;
    case MS_LT: if (c0 == 0) never = true; else { lo = 0; span = c0 - 1; } break;
    case MS_LE: lo = 0; span = c0; break;
    case MS_GT: if (c0 == 0xFFFFFFFFu) never = true; else { lo = c0 + 1; span = 0xFFFFFFFFu - c0 - 1; } break;
    case MS_GE: lo = c0; span = 0xFFFFFFFFu - c0; break;
    case MS_BETWEEN: if (c0 > c1) never = true; else { lo = c0; span = c1 - c0; } break;
    default: return fail(MS_ERR_INVALID_ARG, "unknown comparison");
  }
  if (never) {
    lo = 0;
    span = 0xFFFFFFFFu;
    neg = 1;
  }
  pa.lo = lo;
  pa.span = span;
  pa.neg = neg;
  return compaction(in, pa, false, false, fmt, stream, out);
}

ms_status ms_bitmap_from_positions(const ms_column *pos, uint64_t domain, uint32_t *dev_bitmap, void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!pos) return fail(MS_ERR_INVALID_ARG, "input is NULL");
  if (domain > (1ull << 32)) return fail(MS_ERR_INVALID_ARG, "domain exceeds 2^32");
  const uint64_t words = (domain + 31) / 32;
  if (words && !dev_bitmap) return fail(MS_ERR_INVALID_ARG, "bitmap is NULL");
  const uint64_t n_cap = pos->n_host != kUnknown ? pos->n_host : pos->n_cap;
  Scratch sc(stream);
  unsigned *ends = sc.get<unsigned>(4 * chunks_of(n_cap) + 4);
  if (!sc.ok) return fail(MS_ERR_OOM, "scratch allocation failed");
  hipError_t e = launch_fill_u32(dev_bitmap, words, 0u, stream);
  if (e == hipSuccess)
    e = launch_bitmap(pos->v, domain, dev_bitmap, ends, nullptr, nullptr, grid_for(chunks_of(n_cap)), stream);
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

ms_status ms_semijoin(const ms_column *keys, const uint32_t *dev_bitmap, uint64_t domain, ms_format fmt,
                      void *stream, ms_column **out) {
  if (!out) return fail(MS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!keys) return fail(MS_ERR_INVALID_ARG, "input is NULL");
  if (domain > (1ull << 32)) return fail(MS_ERR_INVALID_ARG, "domain exceeds 2^32");
  if (domain && !dev_bitmap) return fail(MS_ERR_INVALID_ARG, "bitmap is NULL");
  PredArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.mode = 1;
  pa.bitmap = dev_bitmap;
  pa.domain = domain;
  return compaction(keys, pa, false, false, fmt, stream, out);
}

ms_status ms_intersect(const ms_column *a, const ms_column *b, uint64_t domain, ms_format fmt, void *stream,
                       ms_column **out) {
  if (!out) return fail(MS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!a || !b) return fail(MS_ERR_INVALID_ARG, "input is NULL");
  if (domain > (1ull << 32)) return fail(MS_ERR_INVALID_ARG, "domain exceeds 2^32");
  // probe the list with the smaller capacity against a bitmap of the other one
  const ms_column *probe = a, *build = b;
  const uint64_t ca = a->n_host != kUnknown ? a->n_host : a->n_cap;
  const uint64_t cb = b->n_host != kUnknown ? b->n_host : b->n_cap;
  if (cb < ca) std::swap(probe, build);
  Scratch sc(stream);
  const uint64_t words = (domain + 31) / 32;
  unsigned *bm = sc.get<unsigned>(words + 1);
  const uint64_t ncb = std::max(ca, cb);
  const uint64_t Cb = chunks_of(ncb);
  unsigned *first = sc.get<unsigned>(Cb + 1), *last = sc.get<unsigned>(Cb + 1);
  unsigned *ends = sc.get<unsigned>(4 * Cb + 4);
  if (!sc.ok) return fail(MS_ERR_OOM, "scratch allocation failed");
  {
    hipError_t e = launch_fill_u32(bm, words, 0u, stream);
    if (e == hipSuccess) e = launch_bitmap(build->v, domain, bm, ends, first, last, grid_for(Cb), stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
  }
  PredArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.mode = 2;
  pa.bitmap = bm;
  pa.domain = domain;
  return compaction(probe, pa, true, true, fmt, stream, out);
}

ms_status ms_project(const ms_column *data, const ms_column *pos, ms_format fmt, void *stream, ms_column **out) {
  if (!out) return fail(MS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!data || !pos) return fail(MS_ERR_INVALID_ARG, "input is NULL");
  st = check_fmt(fmt);
  if (st != MS_OK) return st;
  const uint64_t n_cap = pos->n_host != kUnknown ? pos->n_host : pos->n_cap;
  const unsigned G = grid_for(chunks_of(n_cap), kWgPerCuProject);
  unsigned auto_w = 0;
  st = make_output(fmt, n_cap, stream, out, auto_w);
  if (st != MS_OK) return st;
  Scratch sc(stream);
  unsigned *partials = sc.get<unsigned>(2 * G);
  unsigned *seg = (fmt.kind == MS_RLE) ? sc.get<unsigned>(kWaves * G) : nullptr;  // runs per wave
  unsigned *narrow_tmp = (fmt.kind == MS_STATIC_BP && auto_w) ? sc.get<unsigned>(n_cap + kPayloadSlackWords) : nullptr;
  if (!sc.ok) {
    free_column(*out);
    *out = nullptr;
    return fail(MS_ERR_OOM, "scratch allocation failed");
  }
  hipError_t e;
  if (fmt.kind == MS_RLE)
    e = launch_rle(1, pos->v, data->v, (*out)->v, G, seg, partials, stream);
  else
    e = launch_project(pos->v, data->v, (*out)->v, auto_w, G, partials, stream);
  if (e == hipSuccess) e = finish_produced((*out)->v, pos->v.hdr, partials, G, auto_w, 0, narrow_tmp, stream);
  st = launched(e, out);
  if (st == MS_OK) (*out)->n_host = pos->n_host;
  return st;
}

ms_status ms_sum(const ms_column *in, uint64_t *dev_result, void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!in || !dev_result) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  const uint64_t n_cap = in->n_host != kUnknown ? in->n_host : in->n_cap;
  const unsigned G = grid_for(chunks_of(n_cap));
  Scratch sc(stream);
  unsigned long long *partials = sc.get<unsigned long long>(G);
  if (!sc.ok) return fail(MS_ERR_OOM, "scratch allocation failed");
  hipError_t e = launch_sum(in->v, reinterpret_cast<unsigned long long *>(dev_result), G, partials, stream);
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

ms_status ms_group_sum(const ms_column *groups, const ms_column *vals, uint32_t G_groups, uint64_t *dev_out,
                       void *stream) {
  ms_status st = group_sum_check(groups, vals, G_groups, dev_out);
  if (st != MS_OK || G_groups == 0) return st;
  const unsigned G = group_sum_grid(groups, vals, G_groups, ~0ull);
  const bool lds = G_groups <= kMaxLdsGroupsHost;
  Scratch sc(stream);
  unsigned long long *partials = sc.get<unsigned long long>(lds ? (uint64_t)G * G_groups : G_groups);
  if (!sc.ok) return fail(MS_ERR_OOM, "scratch allocation failed");
  return group_sum_launch(groups, vals, G_groups, dev_out, G, partials, stream);
}

ms_status ms_group_sum_noalloc(const ms_column *groups, const ms_column *vals, uint32_t G_groups, uint64_t *dev_out,
                               void *stream) {
  ms_status st = group_sum_check(groups, vals, G_groups, dev_out);
  if (st != MS_OK || G_groups == 0) return st;
  if (G_groups > kNoAllocMaxGroups)
    return fail(MS_ERR_INVALID_ARG, "ms_group_sum_noalloc takes at most 262144 groups (its static scratch holds "
                                    "262144 partial sums)");
  unsigned long long *partials = nullptr;
  st = noalloc_scratch(&partials);
  if (st != MS_OK) return st;
  const unsigned G = group_sum_grid(groups, vals, G_groups, kNoAllocScratchU64);
  const bool was_suspended = prof_suspended();
  prof_suspend(true);  // per-launch timing creates events: none from this entry point
  st = group_sum_launch(groups, vals, G_groups, dev_out, G, partials, stream);
  prof_suspend(was_suspended);
  return st;
}

// ---------------------------------------------------------------------------------------------
// The wider operator set: calc, join with position pairs, group-by with its own group ids.

// A count-known transform of one or two columns into fmt (RLE outputs go through an
// uncompressed column that is then morphed).
static ms_status transform_out(uint64_t n_cap, const ColHdr *n_src, ms_format fmt, void *stream, ms_column **out,
                               const std::function<hipError_t(const ColView &, unsigned, unsigned *)> &launch) {
  *out = nullptr;
  ms_status st = check_fmt(fmt);
  if (st != MS_OK) return st;
  const ms_format direct = fmt.kind == MS_RLE ? ms_format{MS_UNCOMPR, 0} : fmt;
  const unsigned G = grid_for(chunks_of(n_cap));
  unsigned auto_w = 0;
  ms_column *o = nullptr;
  st = make_output(direct, n_cap, stream, &o, auto_w);
  if (st != MS_OK) return st;
  Scratch sc(stream);
  unsigned *partials = sc.get<unsigned>(2 * G);
  unsigned *narrow_tmp = (direct.kind == MS_STATIC_BP && auto_w) ? sc.get<unsigned>(n_cap + kPayloadSlackWords) : nullptr;
  if (!sc.ok) {
    free_column(o);
    return fail(MS_ERR_OOM, "scratch allocation failed");
  }
  hipError_t e = launch(o->v, G, partials);
  if (e == hipSuccess) e = finish_produced(o->v, n_src, partials, G, auto_w, 0, narrow_tmp, stream);
  st = launched(e, &o);
  if (st != MS_OK) return st;
  if (fmt.kind != MS_RLE) {
    *out = o;
    return MS_OK;
  }
  st = ms_morph(o, fmt, stream, out);
  free_column(o);
  return st;
}

ms_status ms_calc(const ms_column *a, const ms_column *b, uint32_t op, ms_format fmt, void *stream, ms_column **out) {
  if (!out) return fail(MS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!a || !b) return fail(MS_ERR_INVALID_ARG, "input is NULL");
  if (op > MS_CALC_MUL) return fail(MS_ERR_INVALID_ARG, "unknown calc operation");
  if (a->n_host != kUnknown && b->n_host != kUnknown && a->n_host != b->n_host)
    return fail(MS_ERR_LENGTH_MISMATCH, "calc inputs differ in length");
  const uint64_t n_cap = a->n_host != kUnknown ? a->n_host : a->n_cap;
  st = transform_out(n_cap, a->v.hdr, fmt, stream, out, [&](const ColView &o, unsigned G, unsigned *partials) {
    return launch_calc(a->v, b->v, op, o, G, partials, stream);
  });
  if (st == MS_OK) (*out)->n_host = a->n_host;
  return st;
}

ms_status ms_join(const ms_column *keys, const uint32_t *dev_bitmap, uint64_t domain, ms_format fmt_left,
                  ms_format fmt_right, void *stream, ms_column **left, ms_column **right) {
  if (!left || !right) return fail(MS_ERR_INVALID_ARG, "out is NULL");
  *left = *right = nullptr;
  ms_status st = ms_semijoin(keys, dev_bitmap, domain, fmt_left, stream, left);
  if (st != MS_OK) return st;
  st = ms_project(keys, *left, fmt_right, stream, right);
  if (st != MS_OK) {
    free_column(*left);
    *left = nullptr;
  }
  return st;
}

ms_status ms_group_by(const ms_column *keys, uint64_t domain, ms_format fmt_ids, ms_format fmt_keys, void *stream,
                      ms_column **ids, ms_column **distinct) {
  if (!ids || !distinct) return fail(MS_ERR_INVALID_ARG, "out is NULL");
  *ids = *distinct = nullptr;
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!keys) return fail(MS_ERR_INVALID_ARG, "input is NULL");
  if (domain == 0 || domain > kGroupByMaxDomain)
    return fail(MS_ERR_INVALID_ARG, "group-by domain must be in [1, 2^28]");
  st = check_fmt(fmt_ids);
  if (st == MS_OK) st = check_fmt(fmt_keys);
  if (st != MS_OK) return st;
  const uint64_t n_cap = keys->n_host != kUnknown ? keys->n_host : keys->n_cap;
  const uint64_t C = chunks_of(domain), words = (domain + 31) / 32;
  Scratch sc(stream);
  // the bitmap doubles as the emit phase's row-order bitmask: 64 bytes per chunk and one more
  unsigned *bitmap = reinterpret_cast<unsigned *>(sc.get<unsigned char>(C * 64 + 64));
  unsigned *block_sums = sc.get<unsigned>((words + 1023) / 1024 + 1);
  unsigned *wprefix = sc.get<unsigned>(words + 1);
  if (!sc.ok) return fail(MS_ERR_OOM, "scratch allocation failed");
  hipError_t e = launch_fill_u32(bitmap, (C * 64 + 64) / 4, 0u, stream);
  if (e == hipSuccess) e = launch_mark_keys(keys->v, domain, bitmap, grid_for(chunks_of(n_cap)), stream);
  if (e == hipSuccess) e = launch_word_prefix(bitmap, words, block_sums, wprefix, stream);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  // ids: the rank of every key
  st = transform_out(n_cap, keys->v.hdr, fmt_ids, stream, ids, [&](const ColView &o, unsigned G, unsigned *partials) {
    return launch_rank(keys->v, domain, bitmap, wprefix, o, G, partials, stream);
  });
  if (st != MS_OK) return st;
  (*ids)->n_host = keys->n_host;
  // distinct keys: the set positions of the bitmap, through the compaction's emit phase
  const unsigned G = grid_for(C);
  unsigned auto_w = 0;
  st = make_output(fmt_keys, domain, stream, distinct, auto_w);
  if (st != MS_OK) {
    free_column(*ids);
    *ids = nullptr;
    return st;
  }
  const bool blocky = fmt_keys.kind != MS_UNCOMPR && fmt_keys.kind != MS_RLE;
  Scratch se(stream);
  ColHdr *hdr = reinterpret_cast<ColHdr *>(se.get<unsigned char>(sizeof(ColHdr)));
  EmitArgs ea;
  std::memset(&ea, 0, sizeof(ea));
  ea.in.kind = MS_UNCOMPR;
  ea.in.hdr = hdr;
  ea.in.n_cap = domain;
  ea.out = (*distinct)->v;
  ea.auto_w = auto_w;
  ea.bitmask = reinterpret_cast<const unsigned char *>(bitmap);
  unsigned *seg_count = se.get<unsigned>(G);
  unsigned *seg_or = se.get<unsigned>(G);
  ea.seg_count = seg_count;
  ea.seg_or = seg_or;
  ea.stage_g = blocky ? se.get<unsigned>(domain + 1) : nullptr;
  ea.wave_count = se.get<unsigned>(2ull * kWaves * G);
  ea.partials = se.get<unsigned>(2 * G);
  unsigned *narrow_tmp = (fmt_keys.kind == MS_STATIC_BP && auto_w) ? se.get<unsigned>(domain + kPayloadSlackWords)
                                                                  : nullptr;
  if (!se.ok) {
    free_column(*ids);
    free_column(*distinct);
    *ids = *distinct = nullptr;
    return fail(MS_ERR_OOM, "scratch allocation failed");
  }
  e = launch_set_hdr(hdr, domain, 0, 0, 0, 0, 0, stream);
  if (e == hipSuccess) e = launch_bitmask_segments(bitmap, domain, G, seg_count, seg_or, stream);
  if (e == hipSuccess) e = launch_emit(ea, G, stream);
  if (e == hipSuccess && fmt_keys.kind == MS_STATIC_BP && auto_w)
    e = finish_produced((*distinct)->v, nullptr, ea.partials, G, 1, 1, narrow_tmp, stream);
  st = launched(e, distinct);
  if (st != MS_OK) {
    free_column(*ids);
    *ids = nullptr;
    return st;
  }
  (*distinct)->sorted = 1;
  return MS_OK;
}

ms_status ms_footprints(const ms_column *in, uint64_t *dev_bytes6, void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!in || !dev_bytes6) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  const uint64_t n_cap = in->n_host != kUnknown ? in->n_host : in->n_cap;
  const uint64_t C = chunks_of(n_cap);
  const unsigned G = grid_for(C);
  const unsigned G2 = (unsigned)std::min<uint64_t>(std::max<uint64_t>((C + kWG - 1) / kWG, 1), 1024);
  Scratch sc(stream);
  unsigned long long *part = sc.get<unsigned long long>(5ull * G);
  unsigned long long *bpart = sc.get<unsigned long long>(G2);
  unsigned *first = sc.get<unsigned>(C);
  unsigned *last = sc.get<unsigned>(C);
  if (!sc.ok) return fail(MS_ERR_OOM, "scratch allocation failed");
  hipError_t e = launch_footprints(in->v, G, part, first, last, bpart, G2,
                                   reinterpret_cast<unsigned long long *>(dev_bytes6), stream);
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

ms_status ms_stats(const ms_column *in, float *dev_features32, void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!in || !dev_features32) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  Scratch sc(stream);
  void *chunks = sc.get<unsigned char>(stats_scratch_bytes());
  if (!sc.ok) return fail(MS_ERR_OOM, "scratch allocation failed");
  hipError_t e = launch_stats(in->v, chunks, dev_features32, stream);
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

uint32_t ms_mlp_nparam(void) { return mlp_nparam(); }

ms_status ms_mlp_forward(const float *params, const float *x, uint64_t n, float *y, uint32_t *pick, void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (n && (!params || !x || (!y && !pick))) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  if (n >= (1ull << 31)) return fail(MS_ERR_INVALID_ARG, "batch too large");
  hipError_t e = launch_mlp_forward(params, x, (unsigned)n, y, pick, stream);
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

ms_status ms_mlp_grad(const float *params, const float *x, const float *t, uint64_t n, float *grad, float *loss,
                      void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!params || !grad || (n && (!x || !t))) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  if (n == 0) return fail(MS_ERR_INVALID_ARG, "empty batch");
  if (n >= (1ull << 26)) return fail(MS_ERR_INVALID_ARG, "batch too large");
  const unsigned nwg = mlp_grad_workgroups((unsigned)n);
  Scratch sc(stream);
  float *gpart = sc.get<float>((uint64_t)nwg * mlp_nparam());
  float *lpart = sc.get<float>(nwg);
  if (!sc.ok) return fail(MS_ERR_OOM, "scratch allocation failed");
  hipError_t e = launch_mlp_grad(params, x, t, (unsigned)n, gpart, lpart, grad, loss, stream);
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

ms_status ms_adam_step(float *params, const float *grad, float *m, float *v, uint64_t step, float lr, float beta1,
                       float beta2, float eps, void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!params || !grad || !m || !v) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  if (step == 0) return fail(MS_ERR_INVALID_ARG, "step counts from 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f)) return fail(MS_ERR_INVALID_ARG, "beta out of range");
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  hipError_t e = launch_adam(params, grad, m, v, lr, beta1, beta2, eps, c1, c2, stream);
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

void ms_prof_enable(int on) { prof_enable(on != 0); }
uint64_t ms_prof_count(void) { return prof_count(); }
ms_status ms_prof_get(uint64_t i, const char **name, float *ms) {
  if (!name || !ms) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  return prof_get(i, name, ms) ? MS_OK : fail(MS_ERR_INVALID_ARG, "no such record");
}
void ms_prof_reset(void) { prof_reset(); }

ms_status ms_sync(void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "stream sync");
  unsigned code = read_and_clear_err(stream);
  if (code) {
    static const char *names[] = {"ok", "invalid argument", "unsupported", "value too wide for the static BP width",
                                  "position or group out of range", "input not strictly increasing",
                                  "length mismatch"};
    return fail((ms_status)code, std::string("device-side error: ") + (code < 7 ? names[code] : "unknown"));
  }
  return MS_OK;
}

}  // extern "C"
