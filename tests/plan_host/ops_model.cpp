// Host-only stand-ins for the column library under the plan executor (test
// infrastructure).  Columns own heap buffers ("device memory" of the model) obtained
// through the same allocation rules as the library: a thread's arena while one is set
// (measure mode hands out addresses that must never be touched), else the allocator,
// whose frees are stream ordered.  Every operator queues work that reads its inputs'
// buffers and writes its output and scratch buffers, so a buffer freed or an arena
// released while work that uses it is queued or captured is caught by AddressSanitizer.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "../../include/morphgpu.h"
#include "../../paper_2004_09350_amd/csrc/ms_batch.h"
#include "../../paper_2004_09350_amd/csrc/ms_kernels.h"
#include "../../paper_2004_09350_amd/csrc/ms_runtime.h"
#include "model.h"

struct ms_column {
  uint32_t magic;
  uint32_t kind;
  uint64_t n;
  unsigned char *buf;
  uint64_t bytes;
  bool arena;
  hipStream_t stream;
};

namespace {
constexpr uint32_t kMagic = 0xC011C011u;
thread_local ms::rt::Arena *t_arena = nullptr;
thread_local unsigned t_wg = 0;
thread_local bool t_prof_suspended = false;
thread_local std::string t_err;
int g_fail_arena_alloc_after = -1;  // >= 0: the arena allocation with this index fails (tests error paths)
int g_arena_allocs = 0;

void touch_read(const unsigned char *p, uint64_t bytes) {
  volatile unsigned char s = 0;
  s ^= p[0];
  s ^= p[bytes - 1];
  (void)s;
}
void touch_write(unsigned char *p, uint64_t bytes) {
  p[0] = 1;
  p[bytes - 1] = 2;
}

const ms_column *valid(const ms_column *c) {
  if (c && c->magic != kMagic) {
    std::fprintf(stderr, "model: column handle %p is not a live column\n", (const void *)c);
    std::abort();
  }
  return c;
}

ms_status new_column(uint32_t kind, uint64_t n, void *stream, ms_column **out) {
  *out = nullptr;
  auto *c = new ms_column();
  c->magic = kMagic;
  c->kind = kind;
  c->n = n;
  c->bytes = 256 + 4 * n;
  c->arena = t_arena != nullptr;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->buf = static_cast<unsigned char *>(ms::rt::alloc(c->bytes, stream));
  if (!c->buf) {
    delete c;
    return MS_ERR_OOM;
  }
  *out = c;
  return MS_OK;
}

// One "kernel": reads the inputs' buffers, writes the output's and a scratch buffer.
ms_status launch(void *stream, std::initializer_list<const ms_column *> ins, ms_column *out, void *dev_out,
                 uint64_t dev_bytes) {
  for (const ms_column *c : ins)
    if (!valid(c)) return MS_ERR_INVALID_ARG;
  unsigned char *scratch = static_cast<unsigned char *>(ms::rt::alloc(512, stream));
  if (!scratch) return MS_ERR_OOM;
  struct Buf {
    const unsigned char *p;
    uint64_t n;
  };
  std::vector<Buf> rd;
  for (const ms_column *c : ins) rd.push_back({c->buf, c->bytes});
  unsigned char *wp = out ? out->buf : static_cast<unsigned char *>(dev_out);
  const uint64_t wn = out ? out->bytes : dev_bytes;
  model::submit(reinterpret_cast<hipStream_t>(stream), [rd, wp, wn, scratch]() {
    for (const Buf &b : rd) touch_read(b.p, b.n);
    if (wp && wn) touch_write(wp, wn);
    touch_write(scratch, 512);
  });
  ms::rt::free(scratch, 512, stream);
  return MS_OK;
}

ms_status produce(uint32_t kind, uint64_t n, void *s, ms_column **out, std::initializer_list<const ms_column *> ins) {
  if (!out) return MS_ERR_INVALID_ARG;
  *out = nullptr;
  for (const ms_column *c : ins)
    if (!valid(c)) return MS_ERR_INVALID_ARG;
  ms_status st = new_column(kind, n, s, out);
  if (st != MS_OK) return st;
  st = launch(s, ins, *out, nullptr, 0);
  if (st != MS_OK) {
    ms_column_free(*out);
    *out = nullptr;
  }
  return st;
}
}  // namespace

// ------------------------------------------------------------------- runtime hooks
namespace ms {
namespace rt {
void set_thread_arena(Arena *a) { t_arena = a; }
Arena *thread_arena() { return t_arena; }
void set_thread_wg_per_cu(unsigned w) { t_wg = w; }
unsigned thread_wg_per_cu() { return t_wg; }
void set_thread_chunks_per_wg(unsigned c) { (void)c; }
void *alloc(uint64_t bytes, void *stream) {
  (void)stream;
  if (bytes == 0) bytes = 256;
  if (t_arena) {
    if (g_fail_arena_alloc_after >= 0 && !t_arena->measure && g_arena_allocs++ == g_fail_arena_alloc_after)
      return nullptr;
    const uint64_t at = (t_arena->used + 255) & ~255ull;
    t_arena->used = at + bytes;
    if (t_arena->measure) return reinterpret_cast<void *>(kMeasureBase + at);
    if (t_arena->used > t_arena->size) return nullptr;
    return t_arena->base + at;
  }
  return std::malloc(bytes);
}
void free(void *p, uint64_t bytes, void *stream) {
  (void)bytes;
  if (!p || t_arena) return;
  model::submit(nullptr, [p]() { std::free(p); });  // stream ordered, like the caching allocator
  (void)stream;
}
unsigned cus() { return 256; }
bool initialized() { return true; }
void set_error(const char *msg) { t_err = msg; }
uint64_t column_rows_cap(const ms_column *c) { return c->n; }
}  // namespace rt
void prof_suspend(bool on) { t_prof_suspended = on; }
bool prof_suspended() { return t_prof_suspended; }
}  // namespace ms

// The executor's batched mode: operators here queue their work directly, so nothing is
// recorded and a flush has nothing to issue.
namespace ms {
namespace batch {
bool recording() { return false; }
void begin() {}
void next_op() {}
hipError_t flush(const Streams &, std::vector<Upload> &) { return hipSuccess; }
}  // namespace batch
}  // namespace ms

void model_fail_arena_alloc(int index) {
  g_fail_arena_alloc_after = index;
  g_arena_allocs = 0;
}

// ------------------------------------------------------------------- columns and operators
extern "C" {
const char *ms_last_error(void) { return t_err.c_str(); }

ms_status ms_column_free(ms_column *c) {
  if (!c) return MS_OK;
  valid(c);
  if (!c->arena) ms::rt::free(c->buf, c->bytes, c->stream);
  c->magic = 0;
  delete c;
  return MS_OK;
}
ms_status ms_column_info_get(const ms_column *c, void *stream, ms_column_info *out) {
  if (!valid(c) || !out) return MS_ERR_INVALID_ARG;
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return MS_ERR_HIP;
  std::memset(out, 0, sizeof(*out));
  out->n = c->n;
  out->kind = c->kind;
  return MS_OK;
}
ms_status ms_morph(const ms_column *in, ms_format f, void *s, ms_column **out) {
  return produce(f.kind, valid(in) ? in->n : 0, s, out, {in});
}
ms_status ms_select(const ms_column *in, ms_cmp, uint32_t, uint32_t, ms_format f, void *s, ms_column **out) {
  return produce(f.kind, valid(in) ? in->n : 0, s, out, {in});
}
ms_status ms_bitmap_from_positions(const ms_column *pos, uint64_t domain, uint32_t *bm, void *s) {
  if (!valid(pos)) return MS_ERR_INVALID_ARG;
  return launch(s, {pos}, nullptr, bm, 4 * ((domain + 31) / 32));
}
ms_status ms_semijoin(const ms_column *keys, const uint32_t *bm, uint64_t domain, ms_format f, void *s,
                      ms_column **out) {
  (void)bm;
  (void)domain;
  return produce(f.kind, valid(keys) ? keys->n : 0, s, out, {keys});
}
ms_status ms_project(const ms_column *data, const ms_column *pos, ms_format f, void *s, ms_column **out) {
  return produce(f.kind, valid(pos) ? pos->n : 0, s, out, {data, pos});
}
ms_status ms_intersect(const ms_column *a, const ms_column *b, uint64_t, ms_format f, void *s, ms_column **out) {
  return produce(f.kind, valid(a) && valid(b) ? (a->n < b->n ? a->n : b->n) : 0, s, out, {a, b});
}
ms_status ms_sum(const ms_column *in, uint64_t *r, void *s) { return launch(s, {in}, nullptr, r, 8); }
ms_status ms_group_sum(const ms_column *g, const ms_column *v, uint32_t G, uint64_t *out, void *s) {
  return launch(s, {g, v}, nullptr, out, 8ull * (G ? G : 1));
}
ms_status ms_footprints(const ms_column *in, uint64_t *out6, void *s) { return launch(s, {in}, nullptr, out6, 48); }
ms_status ms_stats(const ms_column *in, float *f, void *s) { return launch(s, {in}, nullptr, f, 128); }
}  // extern "C"

// A base column owned by the test driver (not an arena column).
ms_column *model_input(uint64_t n) {
  ms_column *c = nullptr;
  new_column(0, n, nullptr, &c);
  return c;
}
