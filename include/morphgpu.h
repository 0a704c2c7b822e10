/*
 * morphgpu.h -- C ABI of libmorphgpu.so, compression-enabled columnar operators
 * for AMD Instinct MI355X (gfx950).
 *
 * Model (MorphStore, Damme et al., PVLDB 13, 2020):
 *   - every base column and every intermediate is a sequence of unsigned integers
 *     held in exactly one format, possibly uncompressed (section 3.1);
 *   - operators take columns and return columns (headless BATs, section 3.1);
 *   - each operator decompresses its inputs on the fly and recompresses its output
 *     into a format chosen per intermediate, independently of the input formats
 *     ("on-the-fly de/re-compression", section 3.2);
 *   - a plan must be consistent and its final results are uncompressed (section 3.3).
 *
 * Conventions for every call:
 *   - Pointers named dev_* are device pointers (HBM of the current HIP device);
 *     host_* are host pointers.  `stream` is a hipStream_t (NULL = default stream).
 *   - Inputs are borrowed and never modified.  Every ms_column** output is a new
 *     column owned by the caller and released with ms_column_free.  On any error
 *     *out is set to NULL and nothing is leaked.
 *   - Calls are asynchronous on `stream`; only ms_column_info, ms_column_read_section,
 *     ms_column_shrink, ms_sync and the selector's save/load/get calls synchronise.
 *   - Element counts of data-dependent outputs live on the device.  Errors that
 *     depend on data (a position out of range, an unsorted intersect input, a group
 *     id >= G, a value too wide for a fixed static-BP width) raise a sticky device
 *     flag that the next ms_sync returns and clears.  Argument errors are returned
 *     at once.  ms_last_error() gives a message for the last failing call of the
 *     calling thread.
 *   - Values and positions are uint32 (columns hold fewer than 2^32 values); sums
 *     are uint64 and wrap modulo 2^64.
 *
 * Formats (block size bs; a column of n values keeps its first floor(n/bs)*bs
 * values compressed and the n mod bs rest uncompressed, section 4.1):
 *   MS_UNCOMPR       bs 1    the values
 *   MS_STATIC_BP     bs 32   all values packed at one width b (section 4.1's static BP)
 *   MS_DYN_BP        bs 512  per-block width w_k = bw(OR of the block) (binary packing,
 *                            section 2.1, with SIMD-BP512's block size)
 *   MS_DELTA_DYN_BP  bs 512  DELTA inside each block (base = first value, modular
 *                            differences), then per-block packing (a section 2.1 cascade)
 *   MS_FOR_DYN_BP    bs 512  FOR with the block minimum as reference, then packing
 *   MS_RLE           runs as (value, start) pairs (section 2.1)
 * Packing is least-significant-bit first into little-endian 32-bit words.
 * Footprint = widths 1 B/block + directory 4 B/block + bases/references 4 B/block +
 * payload + 4 B per remainder value; RLE 8 B per run; uncompressed 4 B per value.
 */
#ifndef MORPHGPU_H
#define MORPHGPU_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MS_UNCOMPR = 0, MS_STATIC_BP = 1, MS_DYN_BP = 2, MS_DELTA_DYN_BP = 3, MS_FOR_DYN_BP = 4, MS_RLE = 5
} ms_kind;
#define MS_NUM_KINDS 6
#define MS_BW_AUTO 0xFFFFFFFFu

/* Output format of an operator: kind plus, for MS_STATIC_BP, the width (0..32) or
 * MS_BW_AUTO for the narrowest width that holds every compressed value. */
typedef struct { uint32_t kind; uint32_t bit_width; } ms_format;

/* Unsigned comparisons of select (section 5.1's selection; BETWEEN is c0 <= v <= c1). */
typedef enum { MS_EQ = 0, MS_NE, MS_LT, MS_LE, MS_GT, MS_GE, MS_BETWEEN } ms_cmp;

typedef enum {
  MS_OK = 0, MS_ERR_INVALID_ARG = 1, MS_ERR_UNSUPPORTED = 2, MS_ERR_VALUE_TOO_WIDE = 3,
  MS_ERR_OUT_OF_RANGE = 4, MS_ERR_NOT_SORTED = 5, MS_ERR_LENGTH_MISMATCH = 6, MS_ERR_OOM = 7,
  MS_ERR_HIP = 8, MS_ERR_NOT_INITIALIZED = 9
} ms_status;

typedef struct ms_column ms_column;

/* Device memory provider.  alloc returns device memory usable in stream order on
 * `stream` (NULL on failure); free releases it in stream order.  Passing NULL
 * callbacks to ms_init selects HIP's stream-ordered pool (hipMallocAsync). */
typedef void *(*ms_alloc_fn)(uint64_t bytes, void *stream, void *ctx);
typedef void (*ms_free_fn)(void *ptr, uint64_t bytes, void *stream, void *ctx);

/* Initialise the library on the current device.  Must be called once per process
 * before any other call; may be called again to swap the allocator. */
ms_status ms_init(ms_alloc_fn alloc, ms_free_fn free_fn, void *ctx);
const char *ms_last_error(void);

/* Column construction (section 4.1: a column is one buffer holding its first
 * floor(n/bs) values in its format and the n mod bs rest uncompressed, with the sizes of
 * both parts kept as metadata).  ms_column_encode compresses n device values into fmt
 * (static BP with an explicit width raises MS_ERR_VALUE_TOO_WIDE through ms_sync
 * when a main-part value needs more bits).  The result has the canonical layout:
 * blocks in order, directory offsets = running sums of 16*w_k words. */
ms_status ms_column_encode(const uint32_t *dev_vals, uint64_t n, ms_format fmt, void *stream, ms_column **out);
/* Wrap n uncompressed device values without copying (uncompressed is one of the formats,
 * section 4.1); the memory stays owned by the caller and must outlive the column.
 * dev_vals must be 16-byte aligned. */
ms_status ms_column_wrap_uncompr(const uint32_t *dev_vals, uint64_t n, void *stream, ms_column **out);
/* Decode into dev_out (room for the column's element count): the decompression half of
 * section 3.2's morph into the uncompressed format. */
ms_status ms_column_decode(const ms_column *col, uint32_t *dev_out, void *stream);
ms_status ms_column_free(ms_column *col);

typedef struct {
  uint64_t n;               /* element count */
  uint32_t kind;
  uint32_t bit_width;       /* static BP width, else 0 */
  uint64_t n_main, n_rem;   /* compressed main part and uncompressed remainder */
  uint64_t n_blocks;        /* 512-blocks of the DynBP family */
  uint64_t runs;            /* RLE runs */
  uint64_t payload_words;   /* packed words in use */
  uint64_t payload_extent;  /* words of the payload region a reader may address */
  uint64_t footprint;       /* bytes by the section rule above */
  uint64_t capacity_bytes;  /* device bytes held by the column */
  uint32_t or_all;          /* OR of all values */
  uint32_t sorted;          /* 1 when known strictly increasing (position lists) */
} ms_column_info;
/* Synchronises `stream`, then reports the column's layout and footprint (the metadata of
 * section 4.1: sizes of the compressed main part and the remainder, plus format fields). */
ms_status ms_column_info_get(const ms_column *col, void *stream, ms_column_info *out);

/* Sections of the column buffer of section 4.1, for inspection and parity checks; copied
 * to host after a sync. */
typedef enum {
  MS_SEC_WIDTHS = 0, MS_SEC_OFFSETS = 1, MS_SEC_BASES = 2, MS_SEC_PAYLOAD = 3, MS_SEC_REM = 4,
  MS_SEC_RVALUES = 5, MS_SEC_RSTARTS = 6
} ms_section;
/* Copies min(bytes, section size) bytes of `sec` to host_dst; *copied gets the count.
 * Section sizes: widths n_blocks B; offsets and bases 4*n_blocks B; payload
 * 4*payload_extent B; rem 4*n_rem B; rvalues and rstarts 4*runs B. */
ms_status ms_column_read_section(const ms_column *col, ms_section sec, void *host_dst, uint64_t bytes,
                                 void *stream, uint64_t *copied);
/* Rewrite the column into an exactly sized buffer with the canonical layout (DynBP
 * payload blocks contiguous and in order; section 4.1's continuous buffer).  Operator
 * outputs are allocated for their worst case; this returns the unused capacity.
 * Synchronises `stream`. */
ms_status ms_column_shrink(ms_column *col, void *stream);

/* Format change, section 3.2 "direct morphing": out = encode_fmt(decode(in)). */
ms_status ms_morph(const ms_column *in, ms_format fmt, void *stream, ms_column **out);

/* select (section 5.1): ascending positions i with cmp(v_i, c0[, c1]), as a column in fmt. */
ms_status ms_select(const ms_column *in, ms_cmp cmp, uint32_t c0, uint32_t c1, ms_format fmt, void *stream,
                    ms_column **out);
/* Bitmap with bit p set for every position p (domain bits, 32-bit words, bit p in word
 * p/32 at position p%32): the build side of the semi-join below, i.e. the qualifying
 * dimension rows of one filter of the star-schema plans of section 5.2 (section 4.2 keeps
 * to the operators those plans need).  dev_bitmap must hold ceil(domain/32) words; it is
 * fully written.  A position >= domain raises MS_ERR_OUT_OF_RANGE. */
ms_status ms_bitmap_from_positions(const ms_column *pos, uint64_t domain, uint32_t *dev_bitmap, void *stream);
/* semi-join of a foreign-key column against a dimension bitmap (the star plans of
 * section 5.2): ascending i with keys_i < domain and bit keys_i set. */
ms_status ms_semijoin(const ms_column *keys, const uint32_t *dev_bitmap, uint64_t domain, ms_format fmt,
                      void *stream, ms_column **out);
/* project (section 4.2): out_j = data[pos_j] in pos's order; a position >= |data|
 * raises MS_ERR_OUT_OF_RANGE (that element reads 0). */
ms_status ms_project(const ms_column *data, const ms_column *pos, ms_format fmt, void *stream, ms_column **out);
/* intersect of two strictly increasing position lists: combines the fact-table rows that
 * pass the filters of two dimensions in the star-schema plans of section 5.2 (the
 * conjunction of their semi-joins); unsorted input raises MS_ERR_NOT_SORTED.  `domain`
 * bounds every position (positions < domain). */
ms_status ms_intersect(const ms_column *a, const ms_column *b, uint64_t domain, ms_format fmt, void *stream,
                       ms_column **out);
/* sum (section 5.1): *dev_result = sum of all values mod 2^64. */
ms_status ms_sum(const ms_column *in, uint64_t *dev_result, void *stream);
/* group-based aggregation (section 4.2): dev_out[g] = sum of vals_i with groups_i = g,
 * for g < G (empty groups 0; result uncompressed).  Unequal lengths return
 * MS_ERR_LENGTH_MISMATCH when both are known on the host, else raise it on the device. */
ms_status ms_group_sum(const ms_column *groups, const ms_column *vals, uint32_t G, uint64_t *dev_out,
                       void *stream);
/* ms_group_sum for callers that cannot allocate device memory: code being captured into a
 * HIP graph, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, result
 * and errors as ms_group_sum, but the per-workgroup partial sums live in a static 2 MiB
 * device array of the library (262144 uint64, held by each device the library runs on
 * until the process ends) instead of memory from the allocator: nothing is allocated or
 * freed, no allocator callback runs and no timing event is created.  G must be at most
 * 262144 (else MS_ERR_INVALID_ARG); with G <= 4096 the grid is capped so that
 * workgroups x G partial sums fit the array.  Every call on a device shares that device's
 * array: calls that overlap in time on one device (different streams, or host threads)
 * race and give wrong sums; calls ordered on one stream are safe.  Partial sums that must
 * start at zero are cleared by a fill kernel inside the call. */
ms_status ms_group_sum_noalloc(const ms_column *groups, const ms_column *vals, uint32_t G, uint64_t *dev_out,
                               void *stream);

/* Element-wise arithmetic on two columns of equal length (section 4.2 lists calc among
 * the operators; the star-schema plans of section 5.2 compute measures from two columns):
 * out_i = a_i op b_i in unsigned 32-bit arithmetic modulo 2^32.  Lengths that differ raise
 * MS_ERR_LENGTH_MISMATCH (at once when both are known on the host, else on the device). */
typedef enum { MS_CALC_ADD = 0, MS_CALC_SUB = 1, MS_CALC_MUL = 2 } ms_calc_op;
ms_status ms_calc(const ms_column *a, const ms_column *b, uint32_t op, ms_format fmt, void *stream, ms_column **out);
/* Join of a foreign-key column with a dimension whose qualifying rows are marked in
 * dev_bitmap (as ms_semijoin; the star plans of section 5.2 join fact and dimension tables
 * on dense surrogate keys, i.e. dimension row positions), emitting position pairs: *left =
 * the ascending fact positions i with keys_i < domain and bit keys_i set, in fmt_left;
 * *right = the dimension positions keys_i of those rows, in the same order, in fmt_right.
 * Both columns are owned by the caller. */
ms_status ms_join(const ms_column *keys, const uint32_t *dev_bitmap, uint64_t domain, ms_format fmt_left,
                  ms_format fmt_right, void *stream, ms_column **left, ms_column **right);
/* Group-by with group ids assigned from the data (section 4.2's grouping, whose ids the
 * group-based aggregation consumes): *distinct = the distinct keys in ascending order, in
 * fmt_keys; *ids = for every row the rank of its key among them (0 .. #groups - 1), in
 * fmt_ids, ready for ms_group_sum with G >= #groups (the count is *distinct's element
 * count).  Every key must be below `domain` (1 .. 2^28; the presence bitmap takes domain / 8
 * bytes of scratch), else MS_ERR_OUT_OF_RANGE is raised on the device. */
ms_status ms_group_by(const ms_column *keys, uint64_t domain, ms_format fmt_ids, ms_format fmt_keys, void *stream,
                      ms_column **ids, ms_column **distinct);

/* Exact footprint in bytes of the column in each of the six formats (section 5.2:
 * exhaustive format selection tries every format; footprints are what it compares).
 * dev_bytes6[kind] (device, 6 x uint64, indexed by ms_kind) receives the size that
 * ms_column_encode / ms_morph would give the column in that format, by the section
 * rule used for ms_column_info.footprint: UNCOMPR 4 B/value; STATIC_BP at its
 * automatic width (bit width of the OR of the main part) plus 4 B per remainder value;
 * DynBP family 1 B width + 4 B directory (+ 4 B base for DELTA/FOR) per 512-block,
 * 64 x width B of payload per block, 4 B per remainder value; RLE 8 B per run.
 * One pass over the column; nothing is encoded. */
ms_status ms_footprints(const ms_column *in, uint64_t *dev_bytes6, void *stream);

/* Data characteristics for format selection (section 5.2 names the number of values,
 * the bit-width histogram and the sort order among them).  dev_features32 (device,
 * 32 floats) receives, over a sample of at most 128 chunks of 512 consecutive values
 * (all values when n <= 65536; otherwise chunk floor(s * floor(n/512) / 128), s < 128):
 *   [0..11]  fraction of values whose bit width b falls in class 0 (b = 0) or
 *            1 + (b - 1) / 3;
 *   [12..19] fraction of neighbouring pairs inside a chunk whose difference (mod 2^32)
 *            has bit width class 0 or 1 + (b - 1) / 5;
 *   [20] fraction of pairs in non-decreasing order (1 if there are none);
 *   [21] log2(mean run length) / 32, runs counted inside chunks;
 *   [22] log2(1 + HyperLogLog distinct estimate) / 32 (256 registers, SplitMix64
 *        finaliser of v + 0x9E3779B97F4A7C15, small-range correction);
 *   [23] log2(max - min + 1) / 32; [24] log2(n + 1) / 32;
 *   [25..27] mean per-chunk bit width of the OR, of the chunk-minimum residuals and of
 *        the neighbour differences, / 32;
 *   [28] bw(min) / 32; [29] bw(max) / 32; [30] bw(floor(mean)) / 32;
 *   [31] fraction of sampled chunks holding one distinct value.
 * An empty column gives all zeros except [20] = 1.  Computed in double, stored as float. */
ms_status ms_stats(const ms_column *in, float *dev_features32, void *stream);

/* Learned format selection (section 5.2 selects formats with a cost model over data
 * characteristics that estimates the compression rate and the (de)compression performance
 * of each algorithm).  The model here is a 32-64-64-6 perceptron with ReLU hidden layers
 * that maps the 32 features to one cost per format (index = ms_kind); the selection is the
 * smallest output.  The library trains two of them (ms_selector below): a size network,
 * whose targets are t_k = log2(1 + 8 * footprint_k / n) / 6 (log-scaled bits per value),
 * and a decode-cost network, whose targets are t_k = log2(1 + 1000 * ns_k / n) / 16
 * (log-scaled picoseconds per value of decoding format k).
 * Parameters: one device float vector of ms_mlp_nparam() = 6662 values, row-major
 * W1[64][32], b1[64], W2[64][64], b2[64], W3[6][64], b3[6].  All buffers device,
 * float, batch-major (x: n x 32, y and targets: n x 6). */
uint32_t ms_mlp_nparam(void);
/* y (may be NULL) receives the outputs, pick (may be NULL) the argmin (ties to the
 * lower kind).  n = 0 is a no-op. */
ms_status ms_mlp_forward(const float *params, const float *x, uint64_t n, float *y, uint32_t *pick, void *stream);
/* Gradient of the mean squared error over the n x 6 outputs into grad (6662 floats);
 * loss (device float, may be NULL) receives the loss.  Deterministic: partial sums in a
 * fixed order.  n must be in [1, 2^26). */
ms_status ms_mlp_grad(const float *params, const float *x, const float *t, uint64_t n, float *grad, float *loss,
                      void *stream);
/* One Adam step (Kingma & Ba 2015) with bias correction for step number `step` >= 1:
 * m, v are the moment vectors (6662 floats each, zero before step 1), updated in place
 * with params. */
ms_status ms_adam_step(float *params, const float *grad, float *m, float *v, uint64_t step, float lr, float beta1,
                       float beta2, float eps, void *stream);

/* Selector: the size network and the decode-cost network with their parameters on the
 * device (section 5.2's cost model covers both the compression rate and the (de)compression
 * performance).  ms_selector_create copies the initial parameters (host, 6662 floats each,
 * drawn by the caller) to the device.  Every call below is asynchronous on `stream` unless
 * it says otherwise. */
typedef struct ms_selector ms_selector;
enum { MS_NET_SIZE = 0, MS_NET_COST = 1 };
enum { MS_OBJ_FOOTPRINT = 0, MS_OBJ_DECODE = 1 };  /* which network's costs a pick minimises */
ms_status ms_selector_create(const float *host_init_size, const float *host_init_cost, ms_selector **out);
/* Waits for the device, then frees the selector. */
ms_status ms_selector_destroy(ms_selector *sel);
/* Copies network `net`'s 6662 parameters to dev_dst (device, 6662 floats). */
ms_status ms_selector_params(const ms_selector *sel, uint32_t net, float *dev_dst, void *stream);
/* Bit k set: network k was trained by ms_selector_train or loaded as trained. */
uint32_t ms_selector_trained(const ms_selector *sel);
/* File format: 8 bytes "MSSEL001", uint32 6662, uint32 2, uint32 trained bits, then the
 * size network's and the decode-cost network's parameters (float32, little-endian).  Both
 * calls synchronise the device; a file of any other shape is MS_ERR_INVALID_ARG. */
ms_status ms_selector_save(const ms_selector *sel, const char *path);
ms_status ms_selector_load(const char *path, ms_selector **out);
/* Training targets on the device from the engine's labels, for `count` columns:
 * size: dev_bytes6 (count x 6 uint64 footprints, as ms_footprints writes them) and dev_n
 * (count uint64 element counts; 0 counts as 1) -> dev_t6[i][k] = log2(1 + 8 * bytes / n) / 6;
 * cost: dev_ns6 (count x 6 float decode times in ns, as ms_decode_cost measures them) ->
 * dev_t6[i][k] = log2(1 + 1000 * ns / n) / 16.  Computed in double, stored as float. */
ms_status ms_selector_size_targets(const uint64_t *dev_bytes6, const uint64_t *dev_n, uint64_t count, float *dev_t6,
                                   void *stream);
ms_status ms_selector_cost_targets(const float *dev_ns6, const uint64_t *dev_n, uint64_t count, float *dev_t6,
                                   void *stream);
/* Mini-batch Adam on network `net` over `count` samples (dev_x count x 32, dev_t count x 6):
 * `epochs` passes; pass e visits the rows in the order j -> (a_e * j + b_e) mod count, a
 * permutation drawn from SplitMix64 (Steele, Lea and Flood 2014; mix64 its output function,
 * gamma = 0x9E3779B97F4A7C15): key = mix64(seed), x = mix64(key + (2e + 1) * gamma),
 * y = mix64(key + (2e + 2) * gamma), a_e = 1 + x mod (count - 1), then a_e + 1 (after
 * count - 1 comes 1) until gcd(a_e, count) = 1, b_e = y mod count (a = 1, b = 0 when
 * count = 1).  Consecutive `batch` positions form a batch (the last one may be short); each
 * batch takes the gradient ms_mlp_grad computes on its rows and one Adam step (Adam starts
 * from zero moments at step 1 in every call).
 * host_last_loss (may be NULL; else the call synchronises `stream`) receives the mean batch
 * loss of the last pass.  count must be in [1, 2^31), batch in [1, 2^26). */
typedef struct {
  uint32_t epochs, batch;
  float lr, beta1, beta2, eps;
  uint64_t seed;
} ms_train_cfg;
ms_status ms_selector_train(ms_selector *sel, uint32_t net, const float *dev_x, const float *dev_t, uint64_t count,
                            const ms_train_cfg *cfg, float *host_last_loss, void *stream);
/* Inference: dev_kinds[i] (may be NULL) = the format of least predicted cost under
 * `objective` (MS_OBJ_FOOTPRINT: the size network, MS_OBJ_DECODE: the decode-cost network),
 * ties to the lower kind; dev_pred6 (may be NULL) = that network's count x 6 outputs. */
ms_status ms_selector_pick(const ms_selector *sel, uint32_t objective, const float *dev_x, uint64_t count,
                           uint32_t *dev_kinds, float *dev_pred6, void *stream);
/* Exhaustive selection (section 5.2: every format is tried per column and the smallest
 * physical size kept; column footprints add up, so the per-column choice is the plan's
 * optimum).  ms_select_exhaustive writes the column's six exact footprints (as
 * ms_footprints) to dev_bytes6 and the least one's kind, ties to the lower kind, to
 * *dev_kind (device uint32).  ms_select_argmin does the choice for `count` footprint rows
 * already on the device (count x 6 uint64 -> count uint32). */
ms_status ms_select_exhaustive(const ms_column *in, uint64_t *dev_bytes6, uint32_t *dev_kind, void *stream);
ms_status ms_select_argmin(const uint64_t *dev_bytes6, uint64_t count, uint32_t *dev_kinds, void *stream);
/* Decode-cost labels: morphs the column into each of the six formats (static BP at the
 * automatic width) and times `reps` decodes of each (ms_column_decode, HIP events on
 * `stream`, after one untimed decode); host_ns6[k] receives the mean nanoseconds per decode
 * of format k.  Allocates the six trial columns and a decode buffer through the allocator;
 * synchronises `stream`. */
ms_status ms_decode_cost(const ms_column *in, uint32_t reps, float *host_ns6, void *stream);

/* ------------------------------------------------------------------------------------
 * Plans (section 3.3: a query is a plan of operators; every intermediate is materialised
 * in the format chosen for it; the plan must be consistent, i.e. each operator reads its
 * inputs in the formats their producers wrote).  A plan is an ordered list of steps over
 * input columns; it runs eagerly (one launch sequence per step) or as one captured HIP
 * graph that is replayed.  Independent steps may run on parallel branches (streams).
 * ---------------------------------------------------------------------------------- */
typedef enum {
  MS_OP_MORPH = 0,      /* a -> column in `out`                                        */
  MS_OP_SELECT = 1,     /* a, cmp, c0, c1 -> position column                           */
  MS_OP_BITMAP = 2,     /* a (positions), param = domain -> device bitmap              */
  MS_OP_SEMIJOIN = 3,   /* a (keys), b (a BITMAP step), param = domain -> positions    */
  MS_OP_PROJECT = 4,    /* a (data), b (positions) -> column                           */
  MS_OP_INTERSECT = 5,  /* a, b (positions), param = domain -> positions               */
  MS_OP_SUM = 6,        /* a -> uint64[1]                                              */
  MS_OP_GROUP_SUM = 7,  /* a (groups), b (values), param = G -> uint64[G]              */
  MS_OP_FOOTPRINTS = 8, /* a -> uint64[6] (ms_footprints)                              */
  MS_OP_STATS = 9       /* a -> float[32] (ms_stats)                                   */
} ms_op_kind;

/* Operand references: k >= 0 is the result of step k (k < this step); -1 - j is input
 * column j.  Unused operands are ignored. */
typedef struct {
  uint32_t op;          /* ms_op_kind */
  int32_t a, b;
  uint32_t cmp, c0, c1; /* MS_OP_SELECT */
  uint64_t param;       /* domain (BITMAP, SEMIJOIN, INTERSECT) or group count (GROUP_SUM) */
  ms_format out;        /* output format of column-producing steps */
} ms_step;

/* Launch shape: parallel branches (1..16), the persistent-grid cap in workgroups per
 * compute unit (1..32, or 0 for each operator's default: 4, and 3 for project) and the
 * chunks of 512 values per workgroup that size the grid below that cap (1..64, or 0 for
 * the default of 4): grid = min(ceil(chunks / chunks_per_wg), CUs x wg_per_cu).
 * batch = 1 runs the plan level by level: the operators of a level (steps whose operands
 * all come from earlier levels) share one persistent launch per kernel and phase for
 * select, semi-join and intersect (predicate, emit, fix-up, finish), sum and group-sum
 * (and the fills they need); a launch's workgroups take (operator, segment) tickets,
 * largest operator first.  The level's other kernels are issued in the same phase order,
 * spread over the branches. */
typedef struct {
  uint32_t branches;
  uint32_t wg_per_cu;
  uint32_t chunks_per_wg;
  uint32_t batch;
} ms_tune;

typedef struct ms_plan ms_plan;

/* Validates the steps (operand kinds and order) and borrows the input columns, which
 * must outlive the plan.  Default tune: 1 branch, each operator's default grid. */
ms_status ms_plan_create(const ms_step *steps, uint32_t n_steps, const ms_column *const *inputs, uint32_t n_inputs,
                         ms_plan **out);
ms_status ms_plan_destroy(ms_plan *plan);
/* Change a step's output format or the launch shape (drops a captured graph). */
ms_status ms_plan_set_format(ms_plan *plan, uint32_t step, ms_format fmt);
ms_status ms_plan_set_tune(ms_plan *plan, const ms_tune *tune);
/* The output format a step currently has (as set at creation or by ms_plan_set_format). */
ms_status ms_plan_get_format(const ms_plan *plan, uint32_t step, ms_format *fmt);
ms_status ms_plan_get_tune(const ms_plan *plan, ms_tune *tune);
/* Eager run on `stream`: frees the previous run's results (after synchronising), then
 * launches step by step through the allocator given to ms_init. */
ms_status ms_plan_run(ms_plan *plan, void *stream);
/* Graph run: the first call (or the first after a change) captures the plan into a HIP
 * graph whose intermediates live in one arena owned by the plan, then every call
 * replays it on `stream`.  Results stay valid until the next capture or destroy.
 * Nothing is allocated on replay. */
ms_status ms_plan_launch(ms_plan *plan, void *stream);
/* Result of a step of the last run (borrowed): the column for column steps, else the
 * device pointer of the bitmap / uint64 / float output.  NULL before the first run. */
ms_status ms_plan_result(const ms_plan *plan, uint32_t step, const ms_column **col, void **dev_ptr);
/* Copy up to `bytes` of a non-column result of the last run to host memory (synchronises
 * `stream`); *copied (may be NULL) receives the byte count. */
ms_status ms_plan_read_result(const ms_plan *plan, uint32_t step, void *host_dst, uint64_t bytes, void *stream,
                              uint64_t *copied);
/* Arena bytes of the captured graph (0 before the first ms_plan_launch). */
uint64_t ms_plan_arena_bytes(const ms_plan *plan);
/* Autotuner: times ms_plan_launch for every (branches in {1, 2, 4, 8}, wg_per_cu in {0, 2,
 * 4, 8, 16}) candidate over `reps` replays, then chunks_per_wg in {1, 2, 8, 16} at the best
 * of those, then the batched level-by-level launches (batch = 1) at the best shape, and
 * keeps the fastest.  With cache_path, a tune recorded there for the same
 * plan signature (steps and input shapes) is applied without timing, and new results are
 * appended.  best (may be NULL) receives the tune; best_ms (may be NULL) its time. */
ms_status ms_plan_autotune(ms_plan *plan, void *stream, uint32_t reps, const char *cache_path, ms_tune *best,
                           float *best_ms);

/* Launch timing.  While enabled, every kernel launch is bracketed by two HIP events
 * recorded on its own stream.  Records are kept in launch order until ms_prof_reset.
 * ms_prof_get needs the launches to have finished (call ms_sync first); *name points
 * to a static string (the kernel's name). */
void ms_prof_enable(int on);
uint64_t ms_prof_count(void);
ms_status ms_prof_get(uint64_t i, const char **name, float *ms);
void ms_prof_reset(void);

/* Synchronise `stream` and return (then clear) the first data-dependent error. */
ms_status ms_sync(void *stream);

#ifdef __cplusplus
}
#endif
#endif
