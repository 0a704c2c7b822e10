// ms_kernels.h -- kernel argument blocks and host launchers (implemented in ms_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "ms_internal.h"

namespace ms {

struct PredArgs {
  ColView in;
  unsigned mode;              // 0 range predicate, 1 bitmap on keys, 2 bitmap on values (intersect)
  unsigned lo, span, neg;     // range predicate: ((v - lo) <= span) != neg
  const unsigned *bitmap;
  unsigned long long domain;
  unsigned char *bitmask;     // one byte per lane per chunk = one bit per row
  unsigned *seg_count;
  unsigned *seg_or;
  unsigned *chunk_first, *chunk_last;
};

struct FinishArgs {
  ColView out;
  const ColHdr *n_src;        // element count to record (NULL: keep out's header count)
  const unsigned *partials;   // {OR of all values, OR of the main part} per workgroup
  unsigned G;
  unsigned Wp;                // static BP packing width used by the producer
  unsigned auto_w;            // static BP auto width: narrow to the main part's width
  unsigned sorted;
  unsigned mode;              // 0 finish a produced column, 1 record OR statistics only
};

struct EmitArgs {
  ColView in;                 // the phase-1 input (decoded again when emitting values)
  ColView out;
  unsigned auto_w;
  unsigned emit_values;
  unsigned check_sorted;
  const unsigned char *bitmask;
  const unsigned *seg_count;
  const unsigned *seg_or;
  const unsigned *chunk_first, *chunk_last;
  unsigned *stage_g;          // global staging for blocks shared by several waves
  unsigned *wave_count;       // (first output, count) of each wave (kWaves per workgroup), for the fix phase
  unsigned *partials;
};

// Batched persistent launches: one launch runs the same kernel for many operators of a plan
// level.  Task i (in decreasing size) has seg_prefix[i+1] - seg_prefix[i] segments, the
// workgroups of its ordinary launch; workgroups take tickets t = 0, 1, ... from *ticket
// (zeroed before the launch), ticket t being segment t - seg_prefix[i] of the last task i
// with seg_prefix[i] <= t.
struct BatchQueue {
  const unsigned *seg_prefix;  // n_tasks + 1 entries, seg_prefix[0] = 0
  unsigned n_tasks;
  unsigned *ticket;
};
struct SumArgs {
  ColView in;
  unsigned long long *partials;
};
struct SumFinishArgs {
  const unsigned long long *partials;
  unsigned G;
  unsigned long long *result;
};
struct GroupSumArgs {
  ColView g, v;
  unsigned groups;
  unsigned long long *partials;
};
struct GroupSumFinishArgs {
  const unsigned long long *partials;
  unsigned G, groups, lds;
  unsigned long long *out;
};
struct FillArgs {
  unsigned *p32;               // one of p32, p64
  unsigned long long *p64;
  unsigned long long n, v;
};
struct MorphArgs {
  ColView in, out;
  unsigned auto_w;
  unsigned *partials;
};
struct ProjectArgs {
  ColView pos, data, out;
  unsigned auto_w;
  unsigned *partials;
};
struct NarrowArgs {
  FinishArgs f;
  unsigned *tmp;
};
// Kernels with a batched variant (morph and project: one kind per output kind 0..4).
enum BatchKind : unsigned {
  BK_PRED0, BK_PRED1, BK_PRED2, BK_EMIT, BK_EMIT_VALS, BK_EMIT_FIX, BK_FINISH, BK_SUM, BK_SUM_FINISH, BK_GROUP_SUM,
  BK_GROUP_SUM_FINISH, BK_FILL, BK_NARROW, BK_NARROW_COPY, BK_MORPH0, BK_PROJECT0 = BK_MORPH0 + 5,
  BK_PROJECT_RLE0 = BK_PROJECT0 + 5, BK_COUNT = BK_PROJECT_RLE0 + 5
};
// Launch of kind's batched kernel over tasks (device array of that kind's argument struct).
hipError_t launch_batch(unsigned kind, const void *tasks, const BatchQueue &q, unsigned grid, size_t shm, void *s);
hipError_t launch_pred_batch(unsigned mode, const PredArgs *tasks, const BatchQueue &q, unsigned grid, size_t shm,
                             void *s);
template <unsigned OK>
hipError_t launch_morph_batch_ok(const MorphArgs *tasks, const BatchQueue &q, unsigned grid, size_t shm, void *s);
template <unsigned OK>
hipError_t launch_project_batch_ok(const ProjectArgs *tasks, bool data_rle, const BatchQueue &q, unsigned grid,
                                   size_t shm, void *s);

hipError_t init_err_word();  // once, at library initialisation (the current device)
unsigned read_and_clear_err(void *stream);
void prof_enable(bool on);
size_t prof_count();
bool prof_get(size_t i, const char **name, float *ms);
void prof_reset();
void prof_suspend(bool on);  // this thread's launches are not timed while set
bool prof_suspended();
hipError_t launch_colstats(const ColView &in, unsigned G, unsigned *partials, void *s);
hipError_t launch_finish(const FinishArgs &a, void *s);
hipError_t launch_narrow(const FinishArgs &a, unsigned *tmp, unsigned G, void *s);
hipError_t launch_set_hdr(ColHdr *h, unsigned long long n, unsigned long long runs, unsigned width, unsigned or_all,
                          unsigned or_main, unsigned sorted, void *s);
// One translation unit per output kind holds each of these.
template <unsigned OK>
hipError_t launch_morph_ok(const ColView &in, const ColView &out, unsigned auto_w, unsigned G, unsigned *partials,
                           void *s);
template <unsigned OK>
hipError_t launch_project_ok(const ColView &pos, const ColView &data, const ColView &out, unsigned auto_w, unsigned G,
                             unsigned *partials, void *s);
hipError_t launch_morph(const ColView &in, const ColView &out, unsigned auto_w, unsigned G, unsigned *partials,
                        void *s);
// calc and group-by ids into a block or uncompressed output kind (one unit per kind)
template <unsigned OK>
hipError_t launch_calc_ok(const ColView &a, const ColView &b, unsigned op, const ColView &out, unsigned G,
                          unsigned *partials, void *s);
template <unsigned OK>
hipError_t launch_rank_ok(const ColView &keys, unsigned long long domain, const unsigned *bitmap,
                          const unsigned *wprefix, const ColView &out, unsigned G, unsigned *partials, void *s);
hipError_t launch_calc(const ColView &a, const ColView &b, unsigned op, const ColView &out, unsigned G,
                       unsigned *partials, void *s);
hipError_t launch_rank(const ColView &keys, unsigned long long domain, const unsigned *bitmap,
                       const unsigned *wprefix, const ColView &out, unsigned G, unsigned *partials, void *s);
// Group-by support: presence bitmap of the keys (domain bits, zeroed first; keys >= domain
// raise E_RANGE), per-word exclusive prefix counts of its set bits (block_sums: one word
// per 1024 bitmap words), and the per-segment counts / position ORs of a row-order bitmap
// for the compaction's emit phase.
hipError_t launch_mark_keys(const ColView &keys, unsigned long long domain, unsigned *bitmap, unsigned G, void *s);
hipError_t launch_word_prefix(const unsigned *bitmap, unsigned long long words, unsigned *block_sums,
                              unsigned *wprefix, void *s);
hipError_t launch_bitmask_segments(const unsigned *bitmap, unsigned long long domain, unsigned G, unsigned *seg_count,
                                   unsigned *seg_or, void *s);
hipError_t launch_decode(const ColView &in, unsigned *out, unsigned G, void *s);
hipError_t launch_rle(unsigned mode, const ColView &a, const ColView &b, const ColView &out, unsigned G,
                      unsigned *wave_count, unsigned *partials, void *s);  // wave_count: kWaves * G words
hipError_t launch_project(const ColView &pos, const ColView &data, const ColView &out, unsigned auto_w, unsigned G,
                          unsigned *partials, void *s);
hipError_t launch_pred(const PredArgs &a, unsigned G, void *s);
hipError_t launch_emit(const EmitArgs &a, unsigned G, void *s);
hipError_t launch_sum(const ColView &in, unsigned long long *result, unsigned G, unsigned long long *partials,
                      void *s);
hipError_t launch_group_sum(const ColView &g, const ColView &v, unsigned groups, unsigned long long *out, unsigned G,
                            unsigned long long *partials, void *s);
hipError_t launch_fill_u32(unsigned *p, unsigned long long n, unsigned v, void *s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long n, unsigned long long v, void *s);
// Bitmap of a position list (fill it with zeros first).  ends: 4 words per chunk of the
// list.  first/last (one word per chunk, or both NULL): check that the list increases.
hipError_t launch_bitmap(const ColView &pos, unsigned long long domain, unsigned *bitmap, unsigned *ends,
                         unsigned *first, unsigned *last, unsigned G, void *s);
hipError_t launch_shrink_payload(const unsigned *src, const unsigned *old_off, const unsigned char *widths,
                                 const unsigned *new_off, unsigned *dst, unsigned long long nb, void *s);

hipError_t launch_footprints(const ColView &in, unsigned G, unsigned long long *part, unsigned *first, unsigned *last,
                             unsigned long long *bpart, unsigned G2, unsigned long long *out6, void *s);
size_t stats_scratch_bytes();
hipError_t launch_stats(const ColView &in, void *chunks, float *feat, void *s);
unsigned mlp_nparam();
unsigned mlp_grad_workgroups(unsigned n);
hipError_t launch_mlp_forward(const float *params, const float *x, unsigned n, float *y, unsigned *pick, void *s);
hipError_t launch_mlp_grad(const float *params, const float *x, const float *t, unsigned n, float *gpart,
                           float *lpart, float *grad, float *loss, void *s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps, float c1,
                       float c2, void *s);

}  // namespace ms
