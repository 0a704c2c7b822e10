/* Drives every oracle function over block-boundary sizes and value widths so that the
 * oracle can run under AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure).  Arrays are sized exactly as ms_oracle.h documents, so an access
 * past a documented bound is a sanitizer report.  Exit status 0: every round trip held. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/ms_oracle.h"

static uint64_t state = 0x1234567ull;
static uint32_t next_u32(uint32_t bits) {
  state = state * 6364136223846793005ull + 1442695040888963407ull;
  uint32_t x = (uint32_t)(state >> 32);
  return bits >= 32 ? x : (x & ((1u << bits) - 1u));
}

static int fails = 0;
#define EXPECT(c)                                             \
  do {                                                        \
    if (!(c)) {                                               \
      fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #c); \
      fails++;                                                \
    }                                                         \
  } while (0)

static void round_trip(const uint32_t *v, uint64_t n) {
  uint64_t nbk = n / 512 + 1;
  for (uint32_t kind = 0; kind < 6; kind++) {
    or_column c;
    memset(&c, 0, sizeof c);
    c.widths = malloc(nbk);
    c.offsets = malloc(4 * nbk);
    c.bases = malloc(4 * nbk);
    c.payload = malloc(4 * (n + 16));
    c.rem = malloc(4 * 512);
    c.rvalues = malloc(4 * (n ? n : 1));
    c.rstarts = malloc(4 * (n ? n : 1));
    EXPECT(or_encode(v, n, kind, OR_BW_AUTO, &c) == OR_OK);
    uint32_t *out = malloc(4 * (n ? n : 1));
    EXPECT(or_decode(&c, out) == OR_OK);
    EXPECT(n == 0 || memcmp(out, v, 4 * n) == 0);
    (void)or_footprint(&c);
    free(out);
    free(c.widths);
    free(c.offsets);
    free(c.bases);
    free(c.payload);
    free(c.rem);
    free(c.rvalues);
    free(c.rstarts);
  }
  uint64_t fp[6];
  or_footprints(v, n, fp);
  double f[32];
  or_stats(v, n, f);
}

static void operators(const uint32_t *v, uint64_t n) {
  uint32_t *pos = malloc(4 * (n ? n : 1)), *pos2 = malloc(4 * (n ? n : 1)), *out = malloc(4 * (n ? n : 1));
  uint64_t np = or_select(v, n, OR_LT, 1u << 11, 0, pos);
  uint64_t np2 = or_select(v, n, OR_BETWEEN, 100, 1u << 13, pos2);
  EXPECT(or_project(v, n, pos, np, out) == OR_OK);
  uint64_t k = 0;
  EXPECT(or_intersect(pos, np, pos2, np2, out, &k) == OR_OK);
  uint64_t domain = n ? n : 1;
  uint32_t *bm = calloc((domain + 31) / 32, 4);
  EXPECT(or_bitmap_from_positions(pos, np, domain, bm) == OR_OK);
  (void)or_semijoin(v, n, bm, domain, out);
  (void)or_sum(v, n);
  uint32_t *g = malloc(4 * (n ? n : 1));
  for (uint64_t i = 0; i < n; i++) g[i] = v[i] % 250;
  uint64_t gs[250];
  EXPECT(or_group_sum(g, n, v, n, 250, gs) == OR_OK);
  free(g);
  free(bm);
  free(pos);
  free(pos2);
  free(out);
}

static void network(void) {
  double *p = malloc(sizeof(double) * OR_MLP_NPARAM), *g = malloc(sizeof(double) * OR_MLP_NPARAM);
  double *m = calloc(OR_MLP_NPARAM, sizeof(double)), *vv = calloc(OR_MLP_NPARAM, sizeof(double));
  for (int i = 0; i < OR_MLP_NPARAM; i++) p[i] = (double)next_u32(16) / 65536.0 - 0.5;
  double x[7 * 32], t[7 * 6], y[7 * 6];
  for (int i = 0; i < 7 * 32; i++) x[i] = (double)next_u32(16) / 65536.0;
  for (int i = 0; i < 7 * 6; i++) t[i] = (double)next_u32(16) / 65536.0;
  or_mlp_forward(p, x, 7, y);
  (void)or_mlp_loss_grad(p, x, t, 7, g);
  or_adam_step(p, g, m, vv, 1, 1e-3, 0.9, 0.999, 1e-8, OR_MLP_NPARAM);
  free(p);
  free(g);
  free(m);
  free(vv);
}

int main(void) {
  static const uint64_t sizes[] = {0, 1, 2, 31, 32, 33, 511, 512, 513, 1023, 1024, 1025, 65536, 65537, 70001};
  static const uint32_t widths[] = {0, 1, 3, 7, 12, 20, 31, 32};
  for (size_t a = 0; a < sizeof sizes / sizeof *sizes; a++) {
    uint64_t n = sizes[a];
    uint32_t *v = malloc(4 * (n ? n : 1));
    for (size_t b = 0; b < sizeof widths / sizeof *widths; b++) {
      for (uint64_t i = 0; i < n; i++) v[i] = next_u32(widths[b]);
      round_trip(v, n);
      operators(v, n);
      for (uint64_t i = 1; i < n; i++) v[i] = v[i - 1] + next_u32(3);  /* sorted */
      round_trip(v, n);
      for (uint64_t i = 0; i < n; i++) v[i] = (uint32_t)(i / 64) * 7u;  /* runs */
      round_trip(v, n);
    }
    free(v);
  }
  network();
  if (fails) {
    fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  printf("oracle sanitize ok\n");
  return 0;
}
