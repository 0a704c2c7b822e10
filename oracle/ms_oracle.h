/*
 * ms_oracle.h -- plain, slow CPU oracle for the compression-enabled operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke() check and the
 * bench's cpu_baseline leg may link or call this library.  It shares no code,
 * header, table or constant with the GPU library; both follow the same format
 * definitions independently.
 *
 * Paper: MorphStore (Damme et al., PVLDB 13, 2020).
 *   Formats follow section 2.1 (FOR, DELTA, RLE, binary packing) and section 4.1
 *   (compressed main part of floor(n/bs)*bs values followed by an uncompressed
 *   remainder).  Operators follow their plain definitions on decoded sequences:
 *   select (section 5.1, "sorted column containing the positions"), project
 *   (section 4.2), sum (section 5.1), group-based aggregation (section 4.2), set
 *   intersection and semi-join as used by the star-schema plans (section 5.2).
 *
 * All values and positions are uint32, sums are uint64 (wrapping mod 2^64).
 */
#ifndef MS_ORACLE_H
#define MS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_UNCOMPR = 0, OR_STATIC_BP = 1, OR_DYN_BP = 2, OR_DELTA_DYN_BP = 3, OR_FOR_DYN_BP = 4, OR_RLE = 5 };
enum { OR_EQ = 0, OR_NE, OR_LT, OR_LE, OR_GT, OR_GE, OR_BETWEEN };
enum {
  OR_OK = 0, OR_ERR_INVALID_ARG = 1, OR_ERR_UNSUPPORTED = 2, OR_ERR_VALUE_TOO_WIDE = 3,
  OR_ERR_OUT_OF_RANGE = 4, OR_ERR_NOT_SORTED = 5, OR_ERR_LENGTH_MISMATCH = 6
};
#define OR_BW_AUTO 0xFFFFFFFFu

/* An encoded column as separate sections.  The caller owns every array and must
 * size them: widths/offsets/bases >= n/512 + 1 entries, payload >= n + 16 words,
 * rem >= 512 words, rvalues/rstarts >= n entries. */
typedef struct {
  uint32_t kind;
  uint32_t bit_width;       /* static BP width; 0 otherwise */
  uint64_t n, n_main, n_rem;
  uint64_t nb;              /* blocks of 512 (DynBP family) */
  uint64_t payload_words;   /* words of payload actually used */
  uint64_t runs;            /* RLE run count */
  uint8_t *widths;
  uint32_t *offsets;        /* payload word offset of each block (block directory) */
  uint32_t *bases;          /* DELTA: first value of the block; FOR: block minimum */
  uint32_t *payload;        /* UNCOMPR values, or packed words */
  uint32_t *rem;            /* uncompressed remainder */
  uint32_t *rvalues, *rstarts;
} or_column;

uint32_t or_bw(uint32_t x);
int or_encode(const uint32_t *v, uint64_t n, uint32_t kind, uint32_t bw_req, or_column *c);
int or_decode(const or_column *c, uint32_t *out);
uint64_t or_footprint(const or_column *c);

uint64_t or_select(const uint32_t *v, uint64_t n, uint32_t cmp, uint32_t c0, uint32_t c1, uint32_t *out);
int or_bitmap_from_positions(const uint32_t *p, uint64_t np, uint64_t domain, uint32_t *bitmap);
uint64_t or_semijoin(const uint32_t *keys, uint64_t n, const uint32_t *bitmap, uint64_t domain, uint32_t *out);
int or_project(const uint32_t *data, uint64_t n, const uint32_t *pos, uint64_t np, uint32_t *out);
int or_intersect(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb, uint32_t *out, uint64_t *nout);
uint64_t or_sum(const uint32_t *v, uint64_t n);
int or_group_sum(const uint32_t *g, uint64_t ng, const uint32_t *v, uint64_t nv, uint32_t G, uint64_t *out);

/* 32 column statistics (double precision); definitions in ms_oracle.c. */
void or_stats(const uint32_t *v, uint64_t n, double *feat32);
/* Exact footprint in bytes of v in each of the six formats (static BP at auto width). */
void or_footprints(const uint32_t *v, uint64_t n, uint64_t *bytes6);

/* MLP 32-64-64-6 with ReLU, double precision.  Parameter vector layout:
 * W1[64][32], b1[64], W2[64][64], b2[64], W3[6][64], b3[6]  (row-major, out x in). */
#define OR_MLP_NPARAM (64 * 32 + 64 + 64 * 64 + 64 + 6 * 64 + 6)
void or_mlp_forward(const double *p, const double *x, uint64_t batch, double *y);
double or_mlp_loss_grad(const double *p, const double *x, const double *t, uint64_t batch, double *grad);
void or_adam_step(double *p, const double *g, double *m, double *v, uint64_t step, double lr,
                  double beta1, double beta2, double eps, uint64_t count);

#ifdef __cplusplus
}
#endif
#endif
