/*
 * ms_oracle.c -- plain, slow CPU oracle (TEST INFRASTRUCTURE ONLY: used by the
 * tests, by smoke() and by the bench's cpu_baseline leg; never by the product).
 *
 * Every routine is the plain definition written out: bit packing goes one bit
 * at a time, operators loop over decoded values.  No blocking, no SIMD, no
 * reordering beyond what the definitions state.
 *
 * Format definitions (paper section 2.1 for the techniques, section 4.1 for the
 * main-part/remainder split):
 *   bw(x)      = 0 for x = 0, else the position of the highest set bit plus one
 *                (the "effective bit width" used by binary packing, section 2.1).
 *   Pack(v, b) = value j occupies stream bits [j*b, j*b + b); stream bit k is bit
 *                (k mod 32) of 32-bit word floor(k / 32) (least significant first).
 *   UNCOMPR        block size 1, values stored as they are.
 *   STATIC_BP(b)   block size 32, all main-part values packed at one width b
 *                  ("static BP", section 4.1).
 *   DYN_BP         block size 512, block k packed at w_k = bw(OR of the block)
 *                  (binary packing, section 2.1, with SIMD-BP512's block size).
 *   DELTA_DYN_BP   DELTA (difference to the predecessor, section 2.1) inside each
 *                  512-block, base_k = first value, r_0 = 0, r_j = v_j - v_{j-1}
 *                  mod 2^32, then DYN_BP on the residuals.
 *   FOR_DYN_BP     FOR (difference to a reference, section 2.1) with the block
 *                  minimum as reference, then DYN_BP on the residuals.
 *   RLE            maximal runs as (value, start position) pairs (section 2.1).
 * The compressed main part holds floor(n/bs)*bs values, the remaining n mod bs
 * values follow uncompressed (section 4.1).
 */
#include "ms_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

uint32_t or_bw(uint32_t x) {
  uint32_t b = 0;
  while (x) {
    b++;
    x >>= 1;
  }
  return b;
}

/* Pack: put the low b bits of v at stream bits [bitpos, bitpos + b), one bit at a time. */
static void put_bits(uint32_t *words, uint64_t bitpos, uint32_t b, uint32_t v) {
  for (uint32_t t = 0; t < b; t++) {
    uint64_t k = bitpos + t;
    if ((v >> t) & 1u) words[k >> 5] |= 1u << (k & 31);
  }
}

static uint32_t get_bits(const uint32_t *words, uint64_t bitpos, uint32_t b) {
  uint32_t v = 0;
  for (uint32_t t = 0; t < b; t++) {
    uint64_t k = bitpos + t;
    v |= ((words[k >> 5] >> (k & 31)) & 1u) << t;
  }
  return v;
}

static uint64_t block_size(uint32_t kind) {
  switch (kind) {
    case OR_STATIC_BP: return 32;
    case OR_DYN_BP:
    case OR_DELTA_DYN_BP:
    case OR_FOR_DYN_BP: return 512;
    default: return 1;
  }
}

int or_encode(const uint32_t *v, uint64_t n, uint32_t kind, uint32_t bw_req, or_column *c) {
  if (kind > OR_RLE) return OR_ERR_INVALID_ARG;
  if (n >= (1ull << 32)) return OR_ERR_INVALID_ARG;
  c->kind = kind;
  c->n = n;
  c->bit_width = 0;
  c->nb = 0;
  c->payload_words = 0;
  c->runs = 0;
  if (kind == OR_UNCOMPR) {
    c->n_main = n;
    c->n_rem = 0;
    for (uint64_t i = 0; i < n; i++) c->payload[i] = v[i];
    c->payload_words = n;
    return OR_OK;
  }
  if (kind == OR_RLE) {
    /* A run starts at 0 and wherever the value differs from its predecessor. */
    uint64_t r = 0;
    for (uint64_t i = 0; i < n; i++) {
      if (i == 0 || v[i] != v[i - 1]) {
        c->rvalues[r] = v[i];
        c->rstarts[r] = (uint32_t)i;
        r++;
      }
    }
    c->runs = r;
    c->n_main = n;
    c->n_rem = 0;
    return OR_OK;
  }
  uint64_t bs = block_size(kind);
  c->n_main = (n / bs) * bs;
  c->n_rem = n - c->n_main;
  for (uint64_t i = 0; i < c->n_rem; i++) c->rem[i] = v[c->n_main + i];

  if (kind == OR_STATIC_BP) {
    uint32_t orv = 0;
    for (uint64_t i = 0; i < c->n_main; i++) orv |= v[i];
    uint32_t b;
    if (bw_req == OR_BW_AUTO) {
      b = or_bw(orv);
    } else {
      if (bw_req > 32) return OR_ERR_INVALID_ARG;
      b = bw_req;
      if (or_bw(orv) > b) return OR_ERR_VALUE_TOO_WIDE;
    }
    c->bit_width = b;
    uint64_t words = c->n_main * b / 32;
    for (uint64_t w = 0; w < words; w++) c->payload[w] = 0;
    for (uint64_t i = 0; i < c->n_main; i++) put_bits(c->payload, i * b, b, v[i]);
    c->payload_words = words;
    return OR_OK;
  }

  /* DynBP family: blocks of 512. */
  uint64_t nb = c->n_main / 512;
  c->nb = nb;
  uint64_t off = 0;
  uint32_t r[512];
  for (uint64_t k = 0; k < nb; k++) {
    const uint32_t *blk = v + 512 * k;
    uint32_t base = 0;
    if (kind == OR_DYN_BP) {
      for (int j = 0; j < 512; j++) r[j] = blk[j];
    } else if (kind == OR_DELTA_DYN_BP) {
      base = blk[0];
      r[0] = 0;
      for (int j = 1; j < 512; j++) r[j] = blk[j] - blk[j - 1]; /* modular difference */
    } else { /* FOR */
      base = blk[0];
      for (int j = 1; j < 512; j++)
        if (blk[j] < base) base = blk[j];
      for (int j = 0; j < 512; j++) r[j] = blk[j] - base;
    }
    uint32_t orv = 0;
    for (int j = 0; j < 512; j++) orv |= r[j];
    uint32_t w = or_bw(orv);
    c->widths[k] = (uint8_t)w;
    c->offsets[k] = (uint32_t)off;
    c->bases[k] = base;
    for (uint64_t q = 0; q < 16ull * w; q++) c->payload[off + q] = 0;
    for (int j = 0; j < 512; j++) put_bits(c->payload + off, (uint64_t)j * w, w, r[j]);
    off += 16ull * w;
  }
  c->payload_words = off;
  return OR_OK;
}

int or_decode(const or_column *c, uint32_t *out) {
  uint64_t n = c->n;
  switch (c->kind) {
    case OR_UNCOMPR:
      for (uint64_t i = 0; i < n; i++) out[i] = c->payload[i];
      return OR_OK;
    case OR_RLE: {
      if (n == 0) return c->runs == 0 ? OR_OK : OR_ERR_INVALID_ARG;
      if (c->runs == 0 || c->rstarts[0] != 0) return OR_ERR_INVALID_ARG;
      for (uint64_t r = 0; r < c->runs; r++) {
        uint64_t s = c->rstarts[r];
        uint64_t e = (r + 1 < c->runs) ? c->rstarts[r + 1] : n;
        if (e <= s || e > n) return OR_ERR_INVALID_ARG;
        for (uint64_t i = s; i < e; i++) out[i] = c->rvalues[r];
      }
      return OR_OK;
    }
    case OR_STATIC_BP: {
      uint32_t b = c->bit_width;
      if (b > 32 || c->n_main % 32 || c->n_main + c->n_rem != n) return OR_ERR_INVALID_ARG;
      for (uint64_t i = 0; i < c->n_main; i++) out[i] = get_bits(c->payload, i * b, b);
      for (uint64_t i = 0; i < c->n_rem; i++) out[c->n_main + i] = c->rem[i];
      return OR_OK;
    }
    case OR_DYN_BP:
    case OR_DELTA_DYN_BP:
    case OR_FOR_DYN_BP: {
      if (c->n_main % 512 || c->n_main + c->n_rem != n || c->nb * 512 != c->n_main) return OR_ERR_INVALID_ARG;
      for (uint64_t k = 0; k < c->nb; k++) {
        uint32_t w = c->widths[k];
        if (w > 32) return OR_ERR_INVALID_ARG;
        const uint32_t *p = c->payload + c->offsets[k];
        uint32_t *o = out + 512 * k;
        for (int j = 0; j < 512; j++) {
          uint32_t r = get_bits(p, (uint64_t)j * w, w);
          if (c->kind == OR_DYN_BP)
            o[j] = r;
          else if (c->kind == OR_FOR_DYN_BP)
            o[j] = c->bases[k] + r;
          else
            o[j] = (j == 0) ? c->bases[k] + r : o[j - 1] + r;
        }
      }
      for (uint64_t i = 0; i < c->n_rem; i++) out[c->n_main + i] = c->rem[i];
      return OR_OK;
    }
    default: return OR_ERR_INVALID_ARG;
  }
}

/* Footprint: sum of the section sizes.  Widths 1 B per block, block directory
 * 4 B per block, bases/refs 4 B per block, payload 4 B per word, remainder 4 B
 * per value, RLE 8 B per run. */
uint64_t or_footprint(const or_column *c) {
  switch (c->kind) {
    case OR_UNCOMPR: return 4 * c->n;
    case OR_RLE: return 8 * c->runs;
    case OR_STATIC_BP: return 4 * c->payload_words + 4 * c->n_rem;
    case OR_DYN_BP: return 5 * c->nb + 4 * c->payload_words + 4 * c->n_rem;
    default: return 9 * c->nb + 4 * c->payload_words + 4 * c->n_rem;
  }
}

static int pred(uint32_t v, uint32_t cmp, uint32_t c0, uint32_t c1) {
  switch (cmp) {
    case OR_EQ: return v == c0;
    case OR_NE: return v != c0;
    case OR_LT: return v < c0;
    case OR_LE: return v <= c0;
    case OR_GT: return v > c0;
    case OR_GE: return v >= c0;
    case OR_BETWEEN: return c0 <= v && v <= c1;
    default: return 0;
  }
}

/* select: ascending positions i with pred(v_i).  Returns the count. */
uint64_t or_select(const uint32_t *v, uint64_t n, uint32_t cmp, uint32_t c0, uint32_t c1, uint32_t *out) {
  uint64_t k = 0;
  for (uint64_t i = 0; i < n; i++)
    if (pred(v[i], cmp, c0, c1)) out[k++] = (uint32_t)i;
  return k;
}

int or_bitmap_from_positions(const uint32_t *p, uint64_t np, uint64_t domain, uint32_t *bitmap) {
  uint64_t words = (domain + 31) / 32;
  for (uint64_t w = 0; w < words; w++) bitmap[w] = 0;
  for (uint64_t i = 0; i < np; i++) {
    if (p[i] >= domain) return OR_ERR_OUT_OF_RANGE;
    bitmap[p[i] >> 5] |= 1u << (p[i] & 31);
  }
  return OR_OK;
}

/* semi-join: ascending positions i whose key lies in the domain and has its bit set. */
uint64_t or_semijoin(const uint32_t *keys, uint64_t n, const uint32_t *bitmap, uint64_t domain, uint32_t *out) {
  uint64_t k = 0;
  for (uint64_t i = 0; i < n; i++) {
    uint32_t key = keys[i];
    if (key < domain && ((bitmap[key >> 5] >> (key & 31)) & 1u)) out[k++] = (uint32_t)i;
  }
  return k;
}

int or_project(const uint32_t *data, uint64_t n, const uint32_t *pos, uint64_t np, uint32_t *out) {
  for (uint64_t j = 0; j < np; j++) {
    if (pos[j] >= n) return OR_ERR_OUT_OF_RANGE;
    out[j] = data[pos[j]];
  }
  return OR_OK;
}

/* intersect of strictly increasing lists, by a plain merge. */
int or_intersect(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb, uint32_t *out, uint64_t *nout) {
  for (uint64_t i = 1; i < na; i++)
    if (a[i] <= a[i - 1]) return OR_ERR_NOT_SORTED;
  for (uint64_t i = 1; i < nb; i++)
    if (b[i] <= b[i - 1]) return OR_ERR_NOT_SORTED;
  uint64_t i = 0, j = 0, k = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j])
      i++;
    else if (b[j] < a[i])
      j++;
    else {
      out[k++] = a[i];
      i++;
      j++;
    }
  }
  *nout = k;
  return OR_OK;
}

uint64_t or_sum(const uint32_t *v, uint64_t n) {
  uint64_t s = 0;
  for (uint64_t i = 0; i < n; i++) s += v[i];
  return s;
}

int or_group_sum(const uint32_t *g, uint64_t ng, const uint32_t *v, uint64_t nv, uint32_t G, uint64_t *out) {
  if (ng != nv) return OR_ERR_LENGTH_MISMATCH;
  for (uint32_t q = 0; q < G; q++) out[q] = 0;
  for (uint64_t i = 0; i < ng; i++)
    if (g[i] >= G) return OR_ERR_OUT_OF_RANGE;
  for (uint64_t i = 0; i < ng; i++) out[g[i]] += v[i];
  return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Column statistics: 32 features of a column, computed on a fixed sample.
 * Sample: n <= 65536 takes every value, split into consecutive pieces of 512
 * ("chunks", the last one possibly shorter).  Larger columns take 128 full
 * chunks, chunk s being the floor(s * C / 128)-th of the C = floor(n / 512) full
 * 512-value chunks.  "Pairs" are neighbours inside one chunk.
 *   f[0..11]  fraction of sampled values with bw in {0},{1-3},{4-6},...,{31-32}
 *   f[12..19] fraction of pairs whose modular difference has bw in
 *             {0},{1-5},{6-10},...,{26-30},{31-32}
 *   f[20]     fraction of pairs with v_j >= v_{j-1} (1 when there are no pairs)
 *   f[21]     log2(mean run length) / 32, runs counted inside chunks
 *   f[22]     log2(1 + E) / 32, E the HyperLogLog distinct-count estimate with 256
 *             registers over SplitMix64 hashes of the sampled values
 *   f[23]     log2(max - min + 1) / 32 over the sample
 *   f[24]     log2(n + 1) / 32 (exact n)
 *   f[25]     mean over chunks of bw(OR of the chunk) / 32
 *   f[26]     mean over chunks of bw(OR of v - chunk minimum) / 32
 *   f[27]     mean over chunks of bw(OR of in-chunk differences) / 32
 *   f[28..30] bw(min) / 32, bw(max) / 32, bw(floor(mean)) / 32
 *   f[31]     fraction of chunks whose values are all equal
 * ------------------------------------------------------------------------- */
static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void or_stats(const uint32_t *v, uint64_t n, double *f) {
  for (int i = 0; i < 32; i++) f[i] = 0.0;
  uint64_t nchunks, C = n / 512;
  int all = n <= 65536;
  nchunks = all ? (n + 511) / 512 : 128;
  uint64_t m = 0, pairs = 0, sorted = 0, changes = 0, const_chunks = 0;
  uint64_t vb[12] = {0}, db[8] = {0};
  uint32_t mn = 0xFFFFFFFFu, mx = 0;
  uint64_t sum = 0;
  double w_or = 0, w_for = 0, w_delta = 0;
  uint8_t reg[256];
  memset(reg, 0, sizeof reg);
  for (uint64_t s = 0; s < nchunks; s++) {
    uint64_t start = all ? 512 * s : 512 * ((s * C) / 128);
    uint64_t len = all ? ((n - start) < 512 ? (n - start) : 512) : 512;
    const uint32_t *ch = v + start;
    uint32_t c_or = 0, c_min = 0xFFFFFFFFu, d_or = 0;
    int is_const = 1;
    for (uint64_t j = 0; j < len; j++) {
      uint32_t x = ch[j];
      uint32_t b = or_bw(x);
      vb[b == 0 ? 0 : 1 + (b - 1) / 3]++;
      c_or |= x;
      if (x < c_min) c_min = x;
      if (x < mn) mn = x;
      if (x > mx) mx = x;
      sum += x;
      uint64_t h = mix64((uint64_t)x + 0x9E3779B97F4A7C15ull);
      uint32_t idx = (uint32_t)(h >> 56);
      uint64_t rest = h << 8;
      uint32_t rank = 1;
      while (rank <= 56 && !(rest & 0x8000000000000000ull)) {
        rank++;
        rest <<= 1;
      }
      if (rank > reg[idx]) reg[idx] = (uint8_t)rank;
      if (j > 0) {
        uint32_t d = x - ch[j - 1];
        uint32_t db_w = or_bw(d);
        db[db_w == 0 ? 0 : 1 + (db_w - 1) / 5]++;
        d_or |= d;
        pairs++;
        if (x >= ch[j - 1]) sorted++;
        if (x != ch[j - 1]) {
          changes++;
          is_const = 0;
        }
      }
    }
    uint32_t f_or = 0;
    for (uint64_t j = 0; j < len; j++) f_or |= ch[j] - c_min;
    w_or += or_bw(c_or);
    w_for += or_bw(f_or);
    w_delta += or_bw(d_or);
    const_chunks += is_const;
    m += len;
  }
  if (m == 0) {
    f[20] = 1.0;
    return;
  }
  for (int i = 0; i < 12; i++) f[i] = (double)vb[i] / (double)m;
  for (int i = 0; i < 8; i++) f[12 + i] = pairs ? (double)db[i] / (double)pairs : 0.0;
  f[20] = pairs ? (double)sorted / (double)pairs : 1.0;
  uint64_t runs = nchunks + changes;
  f[21] = log2((double)m / (double)runs) / 32.0;
  double z = 0.0;
  uint32_t zeros = 0;
  for (int j = 0; j < 256; j++) {
    z += ldexp(1.0, -(int)reg[j]);
    if (reg[j] == 0) zeros++;
  }
  double E = (0.7213 / (1.0 + 1.079 / 256.0)) * 256.0 * 256.0 / z;
  if (E <= 2.5 * 256.0 && zeros > 0) E = 256.0 * log(256.0 / (double)zeros);
  f[22] = log2(1.0 + E) / 32.0;
  f[23] = log2((double)(mx - mn) + 1.0) / 32.0;
  f[24] = log2((double)n + 1.0) / 32.0;
  f[25] = w_or / (double)nchunks / 32.0;
  f[26] = w_for / (double)nchunks / 32.0;
  f[27] = w_delta / (double)nchunks / 32.0;
  f[28] = or_bw(mn) / 32.0;
  f[29] = or_bw(mx) / 32.0;
  f[30] = or_bw((uint32_t)(sum / m)) / 32.0;
  f[31] = (double)const_chunks / (double)nchunks;
}

/* Footprint of each format: encode into it and measure (static BP at auto width). */
void or_footprints(const uint32_t *v, uint64_t n, uint64_t *bytes6) {
  uint64_t nbk = n / 512 + 1;
  or_column c;
  c.widths = (uint8_t *)malloc(nbk);
  c.offsets = (uint32_t *)malloc(4 * nbk);
  c.bases = (uint32_t *)malloc(4 * nbk);
  c.payload = (uint32_t *)malloc(4 * (n + 16));
  c.rem = (uint32_t *)malloc(4 * 512);
  c.rvalues = (uint32_t *)malloc(4 * (n + 1));
  c.rstarts = (uint32_t *)malloc(4 * (n + 1));
  for (uint32_t kind = 0; kind < 6; kind++) {
    or_encode(v, n, kind, OR_BW_AUTO, &c);
    bytes6[kind] = or_footprint(&c);
  }
  free(c.widths);
  free(c.offsets);
  free(c.bases);
  free(c.payload);
  free(c.rem);
  free(c.rvalues);
  free(c.rstarts);
}

/* ---------------------------------------------------------------------------
 * Format-selector network: 32 -> 64 (ReLU) -> 64 (ReLU) -> 6, mean squared
 * error over batch x 6 outputs, Adam (Kingma & Ba, 2015).  Double precision.
 * ------------------------------------------------------------------------- */
#define W1_OFF 0
#define B1_OFF (W1_OFF + 64 * 32)
#define W2_OFF (B1_OFF + 64)
#define B2_OFF (W2_OFF + 64 * 64)
#define W3_OFF (B2_OFF + 64)
#define B3_OFF (W3_OFF + 6 * 64)

static void layer(const double *W, const double *b, const double *x, int nin, int nout, double *z) {
  for (int o = 0; o < nout; o++) {
    double s = b[o];
    for (int i = 0; i < nin; i++) s += W[o * nin + i] * x[i];
    z[o] = s;
  }
}

void or_mlp_forward(const double *p, const double *x, uint64_t batch, double *y) {
  double z1[64], h1[64], z2[64], h2[64];
  for (uint64_t s = 0; s < batch; s++) {
    layer(p + W1_OFF, p + B1_OFF, x + 32 * s, 32, 64, z1);
    for (int i = 0; i < 64; i++) h1[i] = z1[i] > 0 ? z1[i] : 0;
    layer(p + W2_OFF, p + B2_OFF, h1, 64, 64, z2);
    for (int i = 0; i < 64; i++) h2[i] = z2[i] > 0 ? z2[i] : 0;
    layer(p + W3_OFF, p + B3_OFF, h2, 64, 6, y + 6 * s);
  }
}

double or_mlp_loss_grad(const double *p, const double *x, const double *t, uint64_t batch, double *g) {
  for (int i = 0; i < OR_MLP_NPARAM; i++) g[i] = 0;
  double loss = 0;
  double scale = 1.0 / (double)(batch * 6);
  double z1[64], h1[64], z2[64], h2[64], y[6], dy[6], dh2[64], dz2[64], dh1[64], dz1[64];
  for (uint64_t s = 0; s < batch; s++) {
    const double *xs = x + 32 * s;
    layer(p + W1_OFF, p + B1_OFF, xs, 32, 64, z1);
    for (int i = 0; i < 64; i++) h1[i] = z1[i] > 0 ? z1[i] : 0;
    layer(p + W2_OFF, p + B2_OFF, h1, 64, 64, z2);
    for (int i = 0; i < 64; i++) h2[i] = z2[i] > 0 ? z2[i] : 0;
    layer(p + W3_OFF, p + B3_OFF, h2, 64, 6, y);
    for (int o = 0; o < 6; o++) {
      double e = y[o] - t[6 * s + o];
      loss += e * e * scale;
      dy[o] = 2.0 * e * scale;
    }
    for (int o = 0; o < 6; o++) {
      g[B3_OFF + o] += dy[o];
      for (int i = 0; i < 64; i++) g[W3_OFF + o * 64 + i] += dy[o] * h2[i];
    }
    for (int i = 0; i < 64; i++) {
      double a = 0;
      for (int o = 0; o < 6; o++) a += p[W3_OFF + o * 64 + i] * dy[o];
      dh2[i] = a;
      dz2[i] = z2[i] > 0 ? a : 0;
    }
    for (int o = 0; o < 64; o++) {
      g[B2_OFF + o] += dz2[o];
      for (int i = 0; i < 64; i++) g[W2_OFF + o * 64 + i] += dz2[o] * h1[i];
    }
    for (int i = 0; i < 64; i++) {
      double a = 0;
      for (int o = 0; o < 64; o++) a += p[W2_OFF + o * 64 + i] * dz2[o];
      dh1[i] = a;
      dz1[i] = z1[i] > 0 ? a : 0;
    }
    for (int o = 0; o < 64; o++) {
      g[B1_OFF + o] += dz1[o];
      for (int i = 0; i < 32; i++) g[W1_OFF + o * 32 + i] += dz1[o] * xs[i];
    }
  }
  (void)dh2;
  (void)dh1;
  return loss;
}

void or_adam_step(double *p, const double *g, double *m, double *v, uint64_t step, double lr, double beta1,
                  double beta2, double eps, uint64_t count) {
  double c1 = 1.0 - pow(beta1, (double)step);
  double c2 = 1.0 - pow(beta2, (double)step);
  for (uint64_t i = 0; i < count; i++) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}
