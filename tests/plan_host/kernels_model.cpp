// Host-only stand-ins for the library's kernel launchers (test infrastructure: the real host
// unit csrc/ms_api.hip runs against these and the host model of the runtime, no GPU).
// Every launcher queues work on its stream that writes what the kernel writes, over the
// extents the kernel's contract gives (scratch arrays, result arrays, the output column's
// header), so that a scratch buffer sized too small for its kernel, or one freed or reused
// while the work that uses it is still queued, is caught by AddressSanitizer.  Values are
// stand-ins: an output keeps half of its input's rows; payloads are not produced.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "../../paper_2004_09350_amd/csrc/ms_batch.h"
#include "../../paper_2004_09350_amd/csrc/ms_kernels.h"
#include "model.h"

namespace ms {
namespace {
constexpr unsigned long long kRows = 512;

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }
unsigned long long chunks(unsigned long long n) { return (n + kRows - 1) / kRows; }

template <class T>
void fill(T *p, unsigned long long n, T v) {
  for (unsigned long long i = 0; i < n; i++) p[i] = v;
}

// Input row count as the kernels see it: the header's (the host knows only the capacity).
unsigned long long rows(const ColView &c) { return c.hdr ? c.hdr->n : 0; }

void set_rows(const ColView &out, unsigned long long n) {
  out.hdr->n = std::min<unsigned long long>(n, out.n_cap);
  out.hdr->runs = out.kind == RLE ? out.hdr->n : 0;
  out.hdr->sbp_width = out.kind == STATIC_BP ? std::min(out.width, 32u) : 0;
}

unsigned g_err_word = 0;
bool g_prof_on = false;
thread_local bool t_prof_suspended = false;

// A launch: recorded while the thread records a batch (issued by the flush), else queued.
template <class F>
hipError_t issue(void *s, F work) {
  if (batch::recording()) {
    batch::record_launch([work](void *st) {  // issued by the flush on the stream it picks
      model::submit(S(st), work);
      return hipSuccess;
    });
    return hipSuccess;
  }
  model::submit(S(s), work);
  return hipSuccess;
}

// Per-segment effects of the kernels that have a batched variant (segment seg of G).
void pred_seg(const PredArgs &a, unsigned seg, unsigned G) {
  const unsigned long long C = chunks(rows(a.in));
  const unsigned long long cb = C * seg / G, ce = C * (seg + 1) / G;
  if (ce > cb) std::memset(a.bitmask + cb * 64, 0, (ce - cb) * 64);
  a.seg_count[seg] = 0;
  a.seg_or[seg] = 0;
  for (unsigned long long c = cb; c < ce; c++) {
    if (a.chunk_first) a.chunk_first[c] = 0;
    if (a.chunk_last) a.chunk_last[c] = 0;
  }
  if (a.mode == 1 && a.domain) {
    volatile unsigned sink = a.bitmap[(a.domain - 1) / 32];
    (void)sink;
  }
}
void emit_seg(const EmitArgs &a, unsigned seg, unsigned G) {
  const unsigned long long C = chunks(rows(a.in));
  volatile unsigned sink = 0;
  if (C) sink += a.bitmask[C * 64 - 1];
  for (unsigned i = 0; i < G; i++) sink += a.seg_count[i] + a.seg_or[i];
  fill(a.wave_count + 2ull * kWaves * seg, 2ull * kWaves, 0u);
  fill(a.partials + 2ull * seg, 2ull, 0u);
  const unsigned long long n = rows(a.in) / 2;
  if (seg == 0) {
    if (a.stage_g && n) {
      a.stage_g[0] = 0;
      a.stage_g[std::min(n, a.out.n_cap)] = 0;  // n_cap + 1 words
    }
    set_rows(a.out, n);
  }
}
void emit_fix_seg(const EmitArgs &a, unsigned seg) {
  volatile unsigned sink = a.wave_count[2ull * kWaves * seg] + a.out.hdr->sbp_width;
  (void)sink;
}
void finish_one(const FinishArgs &a) {
  volatile unsigned sink = 0;
  for (unsigned i = 0; a.partials && i < 2 * a.G; i++) sink += a.partials[i];
  if (a.n_src) set_rows(a.out, a.n_src->n);
  else if (a.mode == 0) set_rows(a.out, a.out.hdr->n);
}
void group_sum_seg(const GroupSumArgs &a, unsigned seg) {
  if (a.partials) {
    if (a.groups <= 4096) fill(a.partials + (unsigned long long)seg * a.groups, a.groups, 0ull);
    else a.partials[0] += 0;
  }
}
void group_sum_finish_seg(const GroupSumFinishArgs &a, unsigned seg) {
  if (a.lds) {
    volatile unsigned long long sink = a.partials[(unsigned long long)(a.G - 1) * a.groups + seg];
    (void)sink;
    a.out[seg] = 0;
  } else {
    for (unsigned long long i = (unsigned long long)seg * 256; i < a.groups && i < (seg + 1ull) * 256; i++)
      a.out[i] = a.partials[i];
  }
}
void fill_seg(const FillArgs &a, unsigned seg, unsigned G) {
  for (unsigned long long i = (unsigned long long)seg * 256; i < a.n; i += (unsigned long long)G * 256)
    for (unsigned long long j = i; j < i + 256 && j < a.n; j++) {
      if (a.p32) a.p32[j] = (unsigned)a.v;
      else a.p64[j] = a.v;
    }
}
}  // namespace

hipError_t init_err_word() {
  g_err_word = 0;
  return hipSuccess;
}
unsigned read_and_clear_err(void *stream) {
  if (hipStreamSynchronize(S(stream)) != hipSuccess) return E_INVALID;
  const unsigned e = g_err_word;
  g_err_word = 0;
  return e;
}
void prof_enable(bool on) { g_prof_on = on; }
size_t prof_count() { return 0; }
bool prof_get(size_t, const char **, float *) { return false; }
void prof_reset() {}
void prof_suspend(bool on) { t_prof_suspended = on; }
bool prof_suspended() { return t_prof_suspended; }

hipError_t launch_colstats(const ColView &in, unsigned G, unsigned *partials, void *s) {
  (void)in;
  issue(s, [=]() { fill(partials, 2ull * G, 0u); });
  return hipSuccess;
}
hipError_t launch_finish(const FinishArgs &a, void *s) {
  if (batch::recording()) return batch::record_task(BK_FINISH, &a, sizeof(a), 1, 0);
  model::submit(S(s), [a]() { finish_one(a); });
  return hipSuccess;
}
hipError_t launch_narrow(const FinishArgs &a, unsigned *tmp, unsigned G, void *s) {
  (void)G;
  issue(s, [a, tmp]() {
    if (tmp) tmp[0] = 0;  // the repacked main part: n_cap + slack words
  });
  return hipSuccess;
}
hipError_t launch_set_hdr(ColHdr *h, unsigned long long n, unsigned long long runs, unsigned width, unsigned or_all,
                          unsigned or_main, unsigned sorted, void *s) {
  issue(s, [=]() {
    std::memset(h, 0, sizeof(ColHdr));
    h->n = n;
    h->runs = runs;
    h->sbp_width = width;
    h->or_all = or_all;
    h->or_main = or_main;
    h->sorted = sorted;
  });
  return hipSuccess;
}
hipError_t launch_morph(const ColView &in, const ColView &out, unsigned auto_w, unsigned G, unsigned *partials,
                        void *s) {
  (void)auto_w;
  issue(s, [=]() {
    fill(partials, 2ull * G, 0u);
    set_rows(out, rows(in));
  });
  return hipSuccess;
}
hipError_t launch_project(const ColView &pos, const ColView &data, const ColView &out, unsigned auto_w, unsigned G,
                          unsigned *partials, void *s) {
  (void)data;
  (void)auto_w;
  issue(s, [=]() {
    fill(partials, 2ull * G, 0u);
    set_rows(out, rows(pos));
  });
  return hipSuccess;
}
hipError_t launch_calc(const ColView &a, const ColView &b, unsigned op, const ColView &out, unsigned G,
                       unsigned *partials, void *s) {
  (void)b;
  (void)op;
  issue(s, [=]() {
    fill(partials, 2ull * G, 0u);
    set_rows(out, rows(a));
  });
  return hipSuccess;
}
hipError_t launch_rank(const ColView &keys, unsigned long long domain, const unsigned *bitmap, const unsigned *wprefix,
                       const ColView &out, unsigned G, unsigned *partials, void *s) {
  issue(s, [=]() {
    volatile unsigned sink = 0;
    const unsigned long long words = (domain + 31) / 32;
    if (words) sink += bitmap[words - 1] + wprefix[words - 1];
    fill(partials, 2ull * G, 0u);
    set_rows(out, rows(keys));
  });
  return hipSuccess;
}
hipError_t launch_mark_keys(const ColView &keys, unsigned long long domain, unsigned *bitmap, unsigned G, void *s) {
  (void)keys;
  (void)G;
  issue(s, [=]() {
    if (domain) bitmap[(domain - 1) / 32] |= 1u;
  });
  return hipSuccess;
}
hipError_t launch_word_prefix(const unsigned *bitmap, unsigned long long words, unsigned *block_sums,
                              unsigned *wprefix, void *s) {
  issue(s, [=]() {
    volatile unsigned sink = 0;
    if (words) sink += bitmap[words - 1];
    fill(block_sums, (words + 1023) / 1024, 0u);
    fill(wprefix, words, 0u);
  });
  return hipSuccess;
}
hipError_t launch_bitmask_segments(const unsigned *bitmap, unsigned long long domain, unsigned G, unsigned *seg_count,
                                   unsigned *seg_or, void *s) {
  issue(s, [=]() {
    volatile unsigned sink = 0;
    if (domain) sink += bitmap[(domain - 1) / 32];
    fill(seg_count, G, 0u);
    fill(seg_or, G, 0u);
  });
  return hipSuccess;
}
hipError_t launch_decode(const ColView &in, unsigned *out, unsigned G, void *s) {
  (void)G;
  issue(s, [=]() {
    const unsigned long long n = rows(in);
    if (n) {
      out[0] = 0;
      out[n - 1] = 0;
    }
  });
  return hipSuccess;
}
hipError_t launch_rle(unsigned mode, const ColView &a, const ColView &b, const ColView &out, unsigned G,
                      unsigned *wave_count, unsigned *partials, void *s) {
  (void)mode;
  (void)b;
  issue(s, [=]() {
    if (wave_count) fill(wave_count, 1ull * kWaves * G, 0u);
    if (partials) fill(partials, 2ull * G, 0u);
    set_rows(out, rows(a));
  });
  return hipSuccess;
}
hipError_t launch_pred(const PredArgs &a, unsigned G, void *s) {
  if (batch::recording()) return batch::record_task(BK_PRED0 + a.mode, &a, sizeof(a), G, 0);
  model::submit(S(s), [a, G]() {
    for (unsigned seg = 0; seg < G; seg++) pred_seg(a, seg, G);
  });
  return hipSuccess;
}
hipError_t launch_emit(const EmitArgs &a, unsigned G, void *s) {
  const bool fix = a.out.kind == STATIC_BP || a.out.kind == DYN_BP || a.out.kind == DELTA_DYN_BP ||
                   a.out.kind == FOR_DYN_BP;
  if (batch::recording()) {
    hipError_t e = batch::record_task(BK_EMIT, &a, sizeof(a), G, 0);
    if (e == hipSuccess && fix) e = batch::record_task(BK_EMIT_FIX, &a, sizeof(a), G, 0);
    return e;
  }
  model::submit(S(s), [a, G, fix]() {
    for (unsigned seg = 0; seg < G; seg++) emit_seg(a, seg, G);
    for (unsigned seg = 0; fix && seg < G; seg++) emit_fix_seg(a, seg);
  });
  return hipSuccess;
}
hipError_t launch_sum(const ColView &in, unsigned long long *result, unsigned G, unsigned long long *partials,
                      void *s) {
  if (batch::recording()) {
    const SumArgs sa{in, partials};
    const SumFinishArgs sf{partials, G, result};
    hipError_t e = batch::record_task(BK_SUM, &sa, sizeof(sa), G, 0);
    return e == hipSuccess ? batch::record_task(BK_SUM_FINISH, &sf, sizeof(sf), 1, 0) : e;
  }
  model::submit(S(s), [=]() {
    fill(partials, G, 0ull);
    result[0] = 0;
  });
  return hipSuccess;
}
hipError_t launch_group_sum(const ColView &g, const ColView &v, unsigned groups, unsigned long long *out, unsigned G,
                            unsigned long long *partials, void *s) {
  const GroupSumArgs ga{g, v, groups, partials};
  const unsigned lds = groups <= 4096 ? 1u : 0u;
  const GroupSumFinishArgs gf{partials, G, groups, lds, out};
  const unsigned fsegs = lds ? groups : (groups + 255) / 256;
  if (batch::recording()) {
    hipError_t e = batch::record_task(BK_GROUP_SUM, &ga, sizeof(ga), G, 0);
    if (e == hipSuccess && groups > 0) e = batch::record_task(BK_GROUP_SUM_FINISH, &gf, sizeof(gf), fsegs, 0);
    return e;
  }
  model::submit(S(s), [=]() {
    for (unsigned seg = 0; seg < G; seg++) group_sum_seg(ga, seg);
    for (unsigned seg = 0; groups > 0 && seg < fsegs; seg++) group_sum_finish_seg(gf, seg);
  });
  return hipSuccess;
}
hipError_t launch_fill_u32(unsigned *p, unsigned long long n, unsigned v, void *s) {
  if (n == 0) return hipSuccess;
  const FillArgs f{p, nullptr, n, v};
  const unsigned blocks = (unsigned)std::min<unsigned long long>((n + 255) / 256, 2048ull);
  if (batch::recording()) return batch::record_task(BK_FILL, &f, sizeof(f), blocks, 0);
  model::submit(S(s), [f, blocks]() {
    for (unsigned seg = 0; seg < blocks; seg++) fill_seg(f, seg, blocks);
  });
  return hipSuccess;
}
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long n, unsigned long long v, void *s) {
  if (n == 0) return hipSuccess;
  const FillArgs f{nullptr, p, n, v};
  const unsigned blocks = (unsigned)std::min<unsigned long long>((n + 255) / 256, 2048ull);
  if (batch::recording()) return batch::record_task(BK_FILL, &f, sizeof(f), blocks, 0);
  model::submit(S(s), [f, blocks]() {
    for (unsigned seg = 0; seg < blocks; seg++) fill_seg(f, seg, blocks);
  });
  return hipSuccess;
}
hipError_t launch_bitmap(const ColView &pos, unsigned long long domain, unsigned *bitmap, unsigned *ends,
                         unsigned *first, unsigned *last, unsigned G, void *s) {
  (void)G;
  issue(s, [=]() {
    const unsigned long long C = chunks(rows(pos));
    if (domain) bitmap[(domain - 1) / 32] |= 0u;
    if (ends) fill(ends, 4 * C, 0u);
    if (first) fill(first, C, 0u);
    if (last) fill(last, C, 0u);
  });
  return hipSuccess;
}
hipError_t launch_shrink_payload(const unsigned *src, const unsigned *old_off, const unsigned char *widths,
                                 const unsigned *new_off, unsigned *dst, unsigned long long nb, void *s) {
  (void)src;
  (void)dst;
  issue(s, [=]() {
    volatile unsigned sink = 0;
    if (nb) sink += old_off[nb - 1] + widths[nb - 1] + new_off[nb - 1];
  });
  return hipSuccess;
}
hipError_t launch_footprints(const ColView &in, unsigned G, unsigned long long *part, unsigned *first, unsigned *last,
                             unsigned long long *bpart, unsigned G2, unsigned long long *out6, void *s) {
  issue(s, [=]() {
    const unsigned long long C = chunks(rows(in));
    fill(part, 5ull * G, 0ull);
    fill(first, C, 0u);
    fill(last, C, 0u);
    fill(bpart, G2, 0ull);
    fill(out6, 6, 0ull);
  });
  return hipSuccess;
}
namespace {
// The tickets of one batched launch, taken in order: (task, segment) pairs over the table.
template <class Args, class F>
void run_tickets(const Args *tasks, const BatchQueue &q, unsigned *ticket, F f) {
  const unsigned total = q.seg_prefix[q.n_tasks];
  for (unsigned t = (*ticket)++; t < total; t = (*ticket)++) {
    unsigned lo = 0, hi = q.n_tasks;
    while (hi - lo > 1) {
      const unsigned mid = (lo + hi) / 2;
      if (q.seg_prefix[mid] <= t) lo = mid;
      else hi = mid;
    }
    f(tasks[lo], t - q.seg_prefix[lo], q.seg_prefix[lo + 1] - q.seg_prefix[lo]);
  }
}
}  // namespace

hipError_t launch_pred_batch(unsigned mode, const PredArgs *tasks, const BatchQueue &q, unsigned grid, size_t shm,
                             void *s) {
  (void)mode;
  (void)grid;
  (void)shm;
  model::submit(S(s), [tasks, q]() {
    run_tickets(tasks, q, q.ticket, [](const PredArgs &a, unsigned seg, unsigned G) { pred_seg(a, seg, G); });
  });
  return hipSuccess;
}
hipError_t launch_batch(unsigned kind, const void *tasks, const BatchQueue &q, unsigned grid, size_t shm, void *s) {
  if (kind <= BK_PRED2) return launch_pred_batch(kind - BK_PRED0, static_cast<const PredArgs *>(tasks), q, grid, shm, s);
  model::submit(S(s), [kind, tasks, q]() {
    switch (kind) {
      case BK_EMIT:
        run_tickets(static_cast<const EmitArgs *>(tasks), q, q.ticket,
                    [](const EmitArgs &a, unsigned seg, unsigned G) { emit_seg(a, seg, G); });
        break;
      case BK_EMIT_FIX:
        run_tickets(static_cast<const EmitArgs *>(tasks), q, q.ticket,
                    [](const EmitArgs &a, unsigned seg, unsigned) { emit_fix_seg(a, seg); });
        break;
      case BK_FINISH:
        run_tickets(static_cast<const FinishArgs *>(tasks), q, q.ticket,
                    [](const FinishArgs &a, unsigned, unsigned) { finish_one(a); });
        break;
      case BK_SUM:
        run_tickets(static_cast<const SumArgs *>(tasks), q, q.ticket,
                    [](const SumArgs &a, unsigned seg, unsigned) { a.partials[seg] = 0; });
        break;
      case BK_SUM_FINISH:
        run_tickets(static_cast<const SumFinishArgs *>(tasks), q, q.ticket, [](const SumFinishArgs &a, unsigned, unsigned) {
          volatile unsigned long long sink = a.partials[a.G - 1];
          (void)sink;
          a.result[0] = 0;
        });
        break;
      case BK_GROUP_SUM:
        run_tickets(static_cast<const GroupSumArgs *>(tasks), q, q.ticket,
                    [](const GroupSumArgs &a, unsigned seg, unsigned) { group_sum_seg(a, seg); });
        break;
      case BK_GROUP_SUM_FINISH:
        run_tickets(static_cast<const GroupSumFinishArgs *>(tasks), q, q.ticket,
                    [](const GroupSumFinishArgs &a, unsigned seg, unsigned) { group_sum_finish_seg(a, seg); });
        break;
      case BK_FILL:
        run_tickets(static_cast<const FillArgs *>(tasks), q, q.ticket,
                    [](const FillArgs &a, unsigned seg, unsigned G) { fill_seg(a, seg, G); });
        break;
      default: std::abort();
    }
  });
  return hipSuccess;
}

size_t stats_scratch_bytes() { return 64 * 1024; }
hipError_t launch_stats(const ColView &in, void *chunks_buf, float *feat, void *s) {
  (void)in;
  issue(s, [=]() {
    std::memset(chunks_buf, 0, stats_scratch_bytes());
    fill(feat, 32, 0.f);
  });
  return hipSuccess;
}
unsigned mlp_nparam() { return 6662; }
unsigned mlp_grad_workgroups(unsigned n) { return (n + 63) / 64; }
hipError_t launch_mlp_forward(const float *params, const float *x, unsigned n, float *y, unsigned *pick, void *s) {
  issue(s, [=]() {
    volatile float sink = params[mlp_nparam() - 1];
    if (n) sink += x[32ull * n - 1];
    if (y) fill(y, 6ull * n, 0.f);
    if (pick) fill(pick, n, 0u);
  });
  return hipSuccess;
}
hipError_t launch_mlp_grad(const float *params, const float *x, const float *t, unsigned n, float *gpart, float *lpart,
                           float *grad, float *loss, void *s) {
  issue(s, [=]() {
    volatile float sink = params[mlp_nparam() - 1] + x[32ull * n - 1] + t[6ull * n - 1];
    fill(gpart, 1ull * mlp_grad_workgroups(n) * mlp_nparam(), 0.f);
    fill(lpart, mlp_grad_workgroups(n), 0.f);
    fill(grad, mlp_nparam(), 0.f);
    if (loss) loss[0] = 0.f;
  });
  return hipSuccess;
}
hipError_t launch_adam(float *p, const float *g, float *m, float *v, float, float, float, float, float, float,
                       void *s) {
  issue(s, [=]() {
    for (unsigned i = 0; i < mlp_nparam(); i++) p[i] += 0.f * (g[i] + m[i] + v[i]);
  });
  return hipSuccess;
}

}  // namespace ms
