// ms_ops2.hip -- kernels of the wider operator set (section 4.2's operator list beyond the
// scans: calc, a join emitting position pairs, a group-by assigning its own group ids):
// the group-by's presence bitmap of the keys, its per-word prefix counts, and the
// per-segment counts that let the compaction's emit phase write the distinct keys; plus
// the dispatch of calc and the group ids to their per-output-kind units.
#include <hip/hip_runtime.h>

#include "ms_kcommon.h"
#include "ms_launch.h"

namespace ms {

// Presence bitmap: bit k of word k / 32 set for every key k (keys >= domain raise E_RANGE).
__global__ __launch_bounds__(kWG) void k_mark_keys(ColView kv, unsigned long long domain, unsigned *bitmap) {
  extern __shared__ __attribute__((aligned(16))) unsigned ring[];  // ring_shm() bytes
  const InCol k = load_in(kv);
  const unsigned lane = lane_id(), w = wave_id();
  const unsigned long long C = (k.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, gridDim.x, cb, ce);
  bool bad = false;
  stream_chunks(k, cb, ce, w, lane, ring + w * kRing * kBlk, kv.hdr, [&](unsigned long long c, const unsigned (&v)[8]) {
    const unsigned valid = chunk_valid(c, lane, k.n);
#pragma unroll
    for (int i = 0; i < 8; i++) {
      if (!((valid >> i) & 1u)) continue;
      const unsigned x = v[i];
      if ((unsigned long long)x >= domain) {
        bad = true;
        continue;
      }
      const unsigned bit = 1u << (x & 31u);
      if (!(bitmap[x >> 5] & bit)) atomicOr(bitmap + (x >> 5), bit);  // skip the atomic once set
    }
  });
  if (bad) raise_err(E_RANGE);
}

constexpr unsigned kPrefixBlock = 1024;  // bitmap words per workgroup of the prefix kernels

__global__ __launch_bounds__(kWG) void k_block_popc(const unsigned *bitmap, unsigned long long words,
                                                    unsigned *block_sums) {
  __shared__ unsigned long long red[kWaves];
  const unsigned long long w0 = (unsigned long long)blockIdx.x * kPrefixBlock;
  unsigned c = 0;
  for (unsigned i = threadIdx.x; i < kPrefixBlock; i += kWG)
    if (w0 + i < words) c += __popc(bitmap[w0 + i]);
  const unsigned long long t = wg_add64(c, red);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = (unsigned)t;
}

// Exclusive scan of the block sums in place (one workgroup, 256 at a time with a carry).
__global__ __launch_bounds__(kWG) void k_scan_block_sums(unsigned *block_sums, unsigned n) {
  __shared__ unsigned wsum[kWaves];
  __shared__ unsigned carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const unsigned lane = lane_id(), w = wave_id();
  for (unsigned base = 0; base < n; base += kWG) {
    const unsigned i = base + threadIdx.x;
    const unsigned x = i < n ? block_sums[i] : 0u;
    unsigned tot;
    const unsigned incl = wave_incl_scan(x, 0u, OpAdd(), tot);
    if (lane == 0) wsum[w] = tot;
    __syncthreads();
    unsigned before = carry;
    for (unsigned j = 0; j < w; j++) before += wsum[j];
    if (i < n) block_sums[i] = before + incl - x;
    __syncthreads();
    if (threadIdx.x == 0) carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
}

// wprefix[w] = set bits in words [0, w): the block's offset plus a scan inside the block
// (each thread takes four consecutive words).
__global__ __launch_bounds__(kWG) void k_word_prefix(const unsigned *bitmap, unsigned long long words,
                                                     const unsigned *block_off, unsigned *wprefix) {
  __shared__ unsigned wsum[kWaves];
  const unsigned lane = lane_id(), w = wave_id();
  const unsigned long long w0 = (unsigned long long)blockIdx.x * kPrefixBlock + 4ull * threadIdx.x;
  unsigned c[4], s = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    c[k] = (w0 + k < words) ? __popc(bitmap[w0 + k]) : 0u;
    s += c[k];
  }
  unsigned tot;
  const unsigned incl = wave_incl_scan(s, 0u, OpAdd(), tot);
  if (lane == 0) wsum[w] = tot;
  __syncthreads();
  unsigned run = block_off[blockIdx.x] + incl - s;
  for (unsigned j = 0; j < w; j++) run += wsum[j];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    if (w0 + k < words) wprefix[w0 + k] = run;
    run += c[k];
  }
}

// Counts and position ORs per workgroup segment of a row-order bitmap of `domain` rows,
// as the predicate phase leaves them for the emit phase (segment s of G over its 512-row
// chunks; the OR has the bit width of the segment's largest set position).
__global__ __launch_bounds__(kWG) void k_bitmask_segments(const unsigned *bitmap, unsigned long long domain,
                                                          unsigned *seg_count, unsigned *seg_or) {
  __shared__ unsigned long long red[kWaves];
  __shared__ unsigned redo[kWaves];
  const unsigned long long C = (domain + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, gridDim.x, cb, ce);
  const unsigned long long words = (domain + 31) / 32;
  unsigned cnt = 0, orv = 0;
  for (unsigned long long q = cb * 16 + threadIdx.x; q < ce * 16 && q < words; q += kWG) {
    const unsigned x = bitmap[q];
    cnt += __popc(x);
    if (x) orv |= (unsigned)(q * 32) | (31u - __clz(x));
  }
  const unsigned long long t = wg_add64(cnt, red);
  orv = wg_or(orv, redo);
  if (threadIdx.x == 0) {
    seg_count[blockIdx.x] = (unsigned)t;
    seg_or[blockIdx.x] = orv;
  }
}

hipError_t launch_mark_keys(const ColView &keys, unsigned long long domain, unsigned *bitmap, unsigned G, void *s) {
  MS_LAUNCH_SHM("k_mark_keys", k_mark_keys, G, kWG, ring_shm(keys), s, keys, domain, bitmap);
  return hipGetLastError();
}

hipError_t launch_word_prefix(const unsigned *bitmap, unsigned long long words, unsigned *block_sums,
                              unsigned *wprefix, void *s) {
  if (words == 0) return hipSuccess;
  const unsigned nb = (unsigned)((words + kPrefixBlock - 1) / kPrefixBlock);
  MS_LAUNCH(k_block_popc, nb, kWG, s, bitmap, words, block_sums);
  MS_LAUNCH(k_scan_block_sums, 1, kWG, s, block_sums, nb);
  MS_LAUNCH(k_word_prefix, nb, kWG, s, bitmap, words, block_sums, wprefix);
  return hipGetLastError();
}

hipError_t launch_bitmask_segments(const unsigned *bitmap, unsigned long long domain, unsigned G, unsigned *seg_count,
                                   unsigned *seg_or, void *s) {
  MS_LAUNCH(k_bitmask_segments, G, kWG, s, bitmap, domain, seg_count, seg_or);
  return hipGetLastError();
}

#define MS_BY_BLOCK_KIND(K, LAUNCH)                 \
  switch (K) {                                     \
    case UNCOMPR: LAUNCH(UNCOMPR); break;          \
    case STATIC_BP: LAUNCH(STATIC_BP); break;      \
    case DYN_BP: LAUNCH(DYN_BP); break;            \
    case DELTA_DYN_BP: LAUNCH(DELTA_DYN_BP); break; \
    case FOR_DYN_BP: LAUNCH(FOR_DYN_BP); break;    \
    default: return hipErrorInvalidValue;          \
  }

hipError_t launch_calc(const ColView &a, const ColView &b, unsigned op, const ColView &out, unsigned G,
                       unsigned *partials, void *s) {
#define MS_L(K) return launch_calc_ok<K>(a, b, op, out, G, partials, s)
  MS_BY_BLOCK_KIND(out.kind, MS_L)
#undef MS_L
}

hipError_t launch_rank(const ColView &keys, unsigned long long domain, const unsigned *bitmap,
                       const unsigned *wprefix, const ColView &out, unsigned G, unsigned *partials, void *s) {
#define MS_L(K) return launch_rank_ok<K>(keys, domain, bitmap, wprefix, out, G, partials, s)
  MS_BY_BLOCK_KIND(out.kind, MS_L)
#undef MS_L
}

}  // namespace ms
