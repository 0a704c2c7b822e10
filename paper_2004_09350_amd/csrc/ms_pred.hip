// ms_pred.hip -- compaction phase 1 of select, semi-join and intersect: the predicate
// over the input's rows as a row-order bitmask plus per-segment counts and ORs (its own
// translation unit so that it compiles in parallel with the other kernels).
#include <hip/hip_runtime.h>

#include "ms_kcommon.h"
#include "ms_launch.h"

namespace ms {

// ---------------------------------------------------------------------------------------------
// Narrow static BP select: the predicate on packed words (section 2.2's bit-parallel scans).
//
// A wave takes four consecutive full chunks at a time: lane l reads the W words holding
// rows 32l .. 32l+31 of those 2048 rows (one coalesced load of 256*W bytes per wave) and
// writes the 32 predicate bits of its rows as one word of the row-order bitmask (bytes
// 4l .. 4l+3 of the four chunks' 256 mask bytes).  For W in {1, 2, 4, 8} no field crosses
// a word: the comparison runs on all 32/W fields of a word at once (SWAR): per field,
// d = (v - A) mod 2^W by a borrow-free subtraction, then the flag "S < d" from the top-bit
// rule of unsigned comparison, then the flags are gathered into 32/W consecutive bits.
// Other widths extract the 32 fields with compile-time shifts.  Values are W bits wide, so
// the predicate "(v - lo) <= span" (lo + span < 2^32) restricted to [0, 2^W) is the field
// interval [A, A + S] (or nothing, as "not everything").
struct NarrowPred {
  unsigned A, S, keep;  // field interval start and length - 1, replicated; keep: H, or 0 to negate
};

__device__ __forceinline__ unsigned replicate(unsigned x, unsigned W) {
  unsigned r = 0;
  for (unsigned b = 0; b < 32; b += W) r |= x << b;
  return r;
}

__device__ __forceinline__ NarrowPred narrow_pred(unsigned lo, unsigned span, bool neg, unsigned W) {
  const unsigned top = (1u << W) - 1u;  // W <= 8
  unsigned a = 0, sl = top;
  bool ng = neg;
  if (lo > top) {
    ng = !neg;  // no W-bit value qualifies: "not (every value)"
  } else {
    a = lo;
    const unsigned long long e = (unsigned long long)lo + span;
    sl = (unsigned)min(e, (unsigned long long)top) - lo;
  }
  const unsigned H = replicate(1u << (W - 1), W);
  return NarrowPred{replicate(a, W), replicate(sl, W), ng ? 0u : H};
}

// Flags (bit W-1 of each field) of "field in [A, A + S]", xor-ed with keep's complement.
template <int W>
__device__ __forceinline__ unsigned swar_flags(unsigned x, const NarrowPred &p, bool a_zero) {
  constexpr unsigned H = W == 2 ? 0xAAAAAAAAu : W == 4 ? 0x88888888u : 0x80808080u;
  constexpr unsigned L = ~H;
  unsigned d = x;
  if (!a_zero) {  // d = x - A per field: borrow-free, the top bit fixed up by xor
    const unsigned z = (x | H) - (p.A & L);
    d = z ^ ((x ^ ~p.A) & H);
  }
  // S < d per field: where the top bits differ it is d's top bit, else the borrow out of
  // the lower bits, i.e. the complement of the top bit of (S | H) - (d & L)
  const unsigned t = (p.S | H) - (d & L);
  const unsigned m = p.S ^ d;
  const unsigned gt = (m & d) | (~m & ~t);
  return (gt ^ p.keep) & H;  // keep = H: in range = not (S < d); keep = 0: negated
}

// Gather the flags of one word into its 32/W low bits (field order).
template <int W>
__device__ __forceinline__ unsigned swar_gather(unsigned f) {
  if constexpr (W == 2) {
    f >>= 1;
    f = (f | (f >> 1)) & 0x33333333u;
    f = (f | (f >> 2)) & 0x0F0F0F0Fu;
    f = (f | (f >> 4)) & 0x00FF00FFu;
    return (f | (f >> 8)) & 0xFFFFu;
  } else if constexpr (W == 4) {
    f >>= 3;
    f = (f | (f >> 3)) & 0x03030303u;
    f = (f | (f >> 6)) & 0x000F000Fu;
    return (f | (f >> 12)) & 0xFFu;
  } else {
    f >>= 7;
    f = (f | (f >> 7)) & 0x00030003u;
    return (f | (f >> 14)) & 0xFu;
  }
}

template <int W>
__device__ __forceinline__ void narrow_load(const unsigned *__restrict__ p, unsigned (&x)[8]) {
  if constexpr (W == 4 || W == 8) {
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
#pragma unroll
    for (int k = 0; k < W / 4; k++) {
      const uint4 a = q[k];
      x[4 * k] = a.x; x[4 * k + 1] = a.y; x[4 * k + 2] = a.z; x[4 * k + 3] = a.w;
    }
  } else if constexpr (W == 2 || W == 6) {
    const uint2 *q = reinterpret_cast<const uint2 *>(p);
#pragma unroll
    for (int k = 0; k < W / 2; k++) {
      const uint2 a = q[k];
      x[2 * k] = a.x; x[2 * k + 1] = a.y;
    }
  } else {
#pragma unroll
    for (int k = 0; k < W; k++) x[k] = p[k];
  }
}

// Predicate bits of the lane's 32 consecutive values held in W words.
template <int W>
__device__ __forceinline__ unsigned narrow_mask(const unsigned (&x)[8], const NarrowPred &p, bool a_zero,
                                                unsigned lo, unsigned span, bool neg) {
  unsigned mask = 0;
  if constexpr (W == 1) {
    // v in {0, 1}: each bit qualifies by its own value
    const unsigned q0 = ((0u - lo) <= span) != neg ? 0xFFFFFFFFu : 0u;
    const unsigned q1 = ((1u - lo) <= span) != neg ? 0xFFFFFFFFu : 0u;
    mask = (x[0] & q1) | (~x[0] & q0);
  } else if constexpr (W == 2 || W == 4 || W == 8) {
#pragma unroll
    for (int k = 0; k < W; k++) mask |= swar_gather<W>(swar_flags<W>(x[k], p, a_zero)) << (k * (32 / W));
  } else {
#pragma unroll
    for (int i = 0; i < 32; i++) {
      const int bit = i * W, q = bit >> 5, sh = bit & 31;
      unsigned v;
      if (sh + W <= 32)
        v = (x[q] >> sh) & ((1u << W) - 1u);
      else
        v = __builtin_amdgcn_alignbit(x[q + 1], x[q], sh) & ((1u << W) - 1u);
      if (((v - lo) <= span) != neg) mask |= 1u << i;
    }
  }
  return mask;
}

// Full chunks [cb, ce) of a static BP column of width W (1..8), four per wave step
// (the step's lanes past ce are masked), four steps of loads in flight.
template <int W>
__device__ __forceinline__ void pred_narrow_sbp(const InCol &in, unsigned long long cb, unsigned long long ce,
                                                unsigned w, unsigned lane, unsigned lo, unsigned span, bool neg,
                                                unsigned char *bitmask, unsigned &cnt, unsigned &orv) {
  if (ce <= cb) return;
  const NarrowPred p = narrow_pred(lo, span, neg, W);
  const bool a_zero = p.A == 0;
  const unsigned long long nq = (ce - cb + 3) / 4;  // steps of four chunks over the segment
  const unsigned long long nj = w < nq ? (nq - w + kWaves - 1) / kWaves : 0ull;  // this wave's steps
  if (nj == 0) return;
  const unsigned sub = lane >> 4;  // the lane's chunk within a step
  // lane's load address for step j (clamped to the last full chunk of the segment)
  auto addr = [&](unsigned long long j) {
    unsigned long long c = cb + 4ull * (w + kWaves * j) + sub;
    c = min(c, ce - 1);
    return in.payload + c * 16ull * W + (lane & 15u) * W;
  };
  unsigned x[4][8];
#pragma unroll
  for (int s = 0; s < 4; s++) narrow_load<W>(addr(min((unsigned long long)s, nj - 1)), x[s]);
  for (unsigned long long g = 0; 4 * g < nj; g++) {
    auto slot = [&](auto S) {
      constexpr int s = decltype(S)::value;
      const unsigned long long j = 4 * g + s;
      unsigned mask = 0;
      const unsigned long long c = cb + 4ull * (w + kWaves * j) + sub;
      const bool live = j < nj;
      if (live) mask = narrow_mask<W>(x[s], p, a_zero, lo, span, neg);
      narrow_load<W>(addr(min(j + 4, nj - 1)), x[s]);  // reload on every path (see stream_blocks)
      __builtin_amdgcn_sched_barrier(0);
      if (live && c < ce) {
        const unsigned long long row0 = c * kBlk + 32ull * (lane & 15u);
        reinterpret_cast<unsigned *>(bitmask + c * 64)[lane & 15u] = mask;
        cnt += __popc(mask);
        if (mask) orv |= (unsigned)row0 | (31u - __clz(mask));
      }
    };
    slot(std::integral_constant<int, 0>{});
    slot(std::integral_constant<int, 1>{});
    slot(std::integral_constant<int, 2>{});
    slot(std::integral_constant<int, 3>{});
  }
}

// RLE select evaluated per run (section 3.2's specialised operators on compressed data):
// the predicate is tested once per run and every qualifying run sets the bits of its rows.
// A wave walks its contiguous chunk range [c_begin, c_end) in steps of four chunks (2048
// rows; lane l owns the mask word of rows 32l .. 32l+31 of the step, in the wave's LDS).
// The runs overlapping the step are loaded 64 at a time (run k's end is run k+1's start);
// each lane ORs the bits of its run's rows into the step's words with LDS atomics, then
// every lane stores its word to the row-order bitmask.
__device__ __forceinline__ void pred_rle_direct(const InCol &in, unsigned long long c_begin,
                                                unsigned long long c_end, unsigned lane, unsigned *words,
                                                unsigned lo, unsigned span, bool neg, unsigned char *bitmask,
                                                unsigned &cnt, unsigned &orv) {
  if (c_begin >= c_end || in.runs == 0) return;
  const unsigned long long n = in.n;
  unsigned long long r = rle_find_wave(in, c_begin * kBlk, lane, 0);  // run holding the first row
  for (unsigned long long c0 = c_begin; c0 < c_end; c0 += 4) {
    const unsigned long long R0 = c0 * kBlk;
    const unsigned long long R1 = min(min(c_end, c0 + 4) * kBlk, n);  // rows of this step: [R0, R1)
    words[lane] = 0u;
    wave_sync();
    while (true) {
      const unsigned long long q = r + lane;
      const bool have = q < in.runs;
      const unsigned long long s = have ? in.rstarts[q] : n;
      const unsigned long long e = (q + 1 < in.runs) ? in.rstarts[q + 1] : n;
      const unsigned val = have ? in.rvalues[q] : 0u;
      const bool qual = have && (((val - lo) <= span) != neg);
      const unsigned long long a = max(s, R0), b = min(e, R1);  // the run's rows inside the step
      if (qual && a < b) {
        for (unsigned long long x = a; x < b;) {
          const unsigned wi = (unsigned)((x - R0) >> 5);
          const unsigned long long wend = min(R0 + 32ull * (wi + 1), b);
          const unsigned lo_bit = (unsigned)((x - R0) & 31u), nb = (unsigned)(wend - x);
          const unsigned bits = (nb >= 32 ? 0xFFFFFFFFu : ((1u << nb) - 1u)) << lo_bit;
          atomicOr(words + wi, bits);
          x = wend;
        }
      }
      // runs are consecutive: stop once a loaded run reaches past the step (or the last run)
      const unsigned long long reach = __ballot(!have || e >= R1);
      if (reach) {
        r += (unsigned long long)__builtin_ctzll(reach);  // first run ending at or past R1
        break;
      }
      r += 64;
    }
    wave_sync();
    // the run holding R1 starts the next step: the one found above unless it ends exactly at R1
    {
      const unsigned long long e = (r + 1 < in.runs) ? in.rstarts[r + 1] : n;
      if (e <= R1 && r + 1 < in.runs) r++;
    }
    const unsigned long long c = c0 + (lane >> 4);
    const unsigned mask = words[lane];
    wave_sync();
    if (c < min(c_end, c0 + 4)) {
      reinterpret_cast<unsigned *>(bitmask + c * 64)[lane & 15u] = mask;
      cnt += __popc(mask);
      if (mask) orv |= (unsigned)(R0 + 32ull * lane) | (31u - __clz(mask));
    }
  }
}

// Whether the RLE runs of chunks [cb, ce) average at least kRleDirectRun rows: then the
// per-run walk above does less work than decoding every row (the chunk stream below
// handles one row per value, whatever the run lengths).
constexpr unsigned long long kRleDirectRun = 16;
__device__ __forceinline__ bool rle_long_runs(const InCol &in, unsigned long long cb, unsigned long long ce,
                                              unsigned lane) {
  if (ce <= cb || in.runs == 0) return false;
  const unsigned long long r0 = cb * kBlk, r1 = min(ce * kBlk, in.n);
  if (r1 <= r0) return false;
  const unsigned long long a = rle_find_wave(in, r0, lane, 0), b = rle_find_wave(in, r1 - 1, lane, a);
  return r1 - r0 >= kRleDirectRun * (b - a + 1);
}

// ---------------------------------------------------------------------------------------------
// Compaction phase 1: predicate -> one bit per row, count and OR per segment.
// mode 0: range predicate ((v - lo) <= span) != neg, emits positions
// mode 1: bitmap predicate v < domain && bit(v), emits positions (semi-join)
// mode 2: bitmap predicate on values, emits values, checks strict increase (intersect)
template <unsigned MODE>
__device__ __forceinline__ void pred_body(const PredArgs &a, const unsigned seg, const unsigned G) {
  extern __shared__ __attribute__((aligned(16))) unsigned ring[];  // ring_shm() bytes
  __shared__ unsigned long long red[kWaves];
  __shared__ unsigned redo[kWaves];
  const InCol in = load_in(a.in);
  const unsigned lane = lane_id(), w = wave_id();
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, seg, G, cb, ce);
  unsigned cnt = 0, orv = 0;
  bool unsorted = false;
  constexpr unsigned mode = MODE;
  const unsigned lo = a.lo, span = a.span;
  const bool neg = a.neg != 0;
  const unsigned long long domain = a.domain;
  const unsigned *bitmap = a.bitmap;
  unsigned char *bitmask = a.bitmask;
  unsigned *chunk_first = a.chunk_first, *chunk_last = a.chunk_last;
  // A semi-join bitmap that fits the workgroup's dynamic LDS (kLdsBitmapBits, the size
  // of the ring that RLE input uses otherwise) is probed there instead of through the
  // caches; a larger one keeps its first kLdsBitmapBits bits there, which spares the
  // caches the probes of the keys below that bound.
  const bool lds_bm = mode == 1 && in.kind != RLE;
  const unsigned long long lds_bits = min(domain, kLdsBitmapBits);
  if (lds_bm) {
    const unsigned nw = (unsigned)((lds_bits + 31) / 32);
    for (unsigned t = threadIdx.x; t < nw; t += kWG) ring[t] = bitmap[t];
    __syncthreads();
  }
  unsigned long long c_rest = cb;  // chunks [cb, c_rest) done by the narrow path
  if constexpr (MODE == 0) {
    if (in.kind == RLE && rle_long_runs(in, cb, ce, lane)) {  // a contiguous quarter of the segment per wave
      const unsigned long long nseg = ce - cb;
      pred_rle_direct(in, cb + nseg * w / kWaves, cb + nseg * (w + 1) / kWaves, lane, ring + w * kRing * kBlk, lo,
                      span, neg, bitmask, cnt, orv);
      c_rest = ce;
    } else if (in.kind == STATIC_BP && in.W >= 1 && in.W <= 8) {
      c_rest = max(cb, min(ce, in.n_main / kBlk));
      switch (in.W) {
#define MS_NARROW_CASE(WW) \
  case WW: pred_narrow_sbp<WW>(in, cb, c_rest, w, lane, lo, span, neg, bitmask, cnt, orv); break;
        MS_NARROW_CASE(1) MS_NARROW_CASE(2) MS_NARROW_CASE(3) MS_NARROW_CASE(4)
        MS_NARROW_CASE(5) MS_NARROW_CASE(6) MS_NARROW_CASE(7) MS_NARROW_CASE(8)
#undef MS_NARROW_CASE
        default: break;
      }
    }
  }
  stream_chunks(in, c_rest, ce, w, lane, ring + w * kRing * kBlk, a.in.hdr, [&](unsigned long long c, const unsigned (&v)[8]) {
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
    const unsigned valid = chunk_valid(c, lane, in.n);
    unsigned mask = 0;
    if constexpr (mode == 0) {
#pragma unroll
      for (int i = 0; i < 8; i++)
        if (((v[i] - lo) <= span) != neg) mask |= 1u << i;
    } else if (mode == 1 && lds_bm && domain <= kLdsBitmapBits) {
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const unsigned x = v[i];
        if ((unsigned long long)x < domain && ((ring[x >> 5] >> (x & 31)) & 1u)) mask |= 1u << i;
      }
    } else if (mode == 1 && lds_bm) {
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const unsigned x = v[i];
        if ((unsigned long long)x < domain) {
          const unsigned word = (unsigned long long)x < lds_bits ? ring[x >> 5] : bitmap[x >> 5];
          if ((word >> (x & 31)) & 1u) mask |= 1u << i;
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const unsigned x = v[i];
        if ((unsigned long long)x < domain && ((bitmap[x >> 5] >> (x & 31)) & 1u)) mask |= 1u << i;
      }
    }
    mask &= valid;
    bitmask[c * 64 + lane] = (unsigned char)mask;
    cnt += __popc(mask);
    if constexpr (mode == 2) {
#pragma unroll
      for (int i = 0; i < 8; i++)
        if (mask & (1u << i)) orv |= v[i];
      // strictly increasing inside the chunk; chunk ends are checked by the emit phase
      const unsigned prev = lane_prev(v[7]);
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const unsigned pv = i ? v[i - 1] : prev;
        if (((valid >> i) & 1u) && (i > 0 || lane > 0) && v[i] <= pv) unsorted = true;
      }
      const unsigned long long last_idx = min(in.n, (c + 1) * kBlk) - 1;
      if (lane == 0) chunk_first[c] = v[0];
      if (idx0 <= last_idx && last_idx < idx0 + 8) chunk_last[c] = select8(v, (unsigned)(last_idx - idx0));
    } else if (mask) {
      orv |= (unsigned)idx0 | (31u - __clz(mask));  // positions: bit width of the largest
    }
  });
  if (unsorted) raise_err(E_NOT_SORTED);
  const unsigned long long t = wg_add64(cnt, red);
  orv = wg_or(orv, redo);
  if (threadIdx.x == 0) {
    a.seg_count[seg] = (unsigned)t;
    a.seg_or[seg] = orv;
  }
}

template <unsigned MODE>
__global__ __launch_bounds__(kWG) void k_pred(PredArgs a) {
  pred_body<MODE>(a, blockIdx.x, gridDim.x);
}

// The same for a batch of operators (one plan level): workgroups take (task, segment) tickets.
template <unsigned MODE>
__global__ __launch_bounds__(kWG) void k_pred_batch(const PredArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const PredArgs &a, unsigned seg, unsigned G) { pred_body<MODE>(a, seg, G); });
}


// Semi-join against a bitmap larger than the 256-thread kernel's LDS part: one workgroup of
// 1024 threads per CU keeps the first kWideLdsBits bits (nearly all of the 160 KB a
// workgroup may hold) in LDS and probes only the keys above them through the caches.  Its four quarters do exactly the work of four
// consecutive workgroups of k_pred<1> (segments 4b .. 4b+3 of the same G, four waves each),
// so the emit phase sees the same segments and counts.  Keys in any format but RLE.
constexpr unsigned kWideWG = 1024;
constexpr unsigned kWideLdsWords = 40896;
constexpr unsigned long long kWideLdsBits = 32ull * kWideLdsWords;

__global__ __launch_bounds__(kWideWG) void k_semijoin_wide(PredArgs a, unsigned G) {
  __shared__ unsigned bm[kWideLdsWords];
  __shared__ unsigned s_cnt[kWideWG / 64], s_or[kWideWG / 64];
  const InCol in = load_in(a.in);
  const unsigned lane = lane_id(), w = wave_id(), q = w >> 2, w4 = w & 3u;
  const unsigned seg = 4u * blockIdx.x + q;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb = 0, ce = 0;
  if (seg < G) segment(C, seg, G, cb, ce);
  const unsigned long long domain = a.domain;
  const unsigned *bitmap = a.bitmap;
  unsigned char *bitmask = a.bitmask;
  const unsigned long long lds_bits = min(domain, kWideLdsBits);
  const unsigned nw = (unsigned)((lds_bits + 31) / 32);
  for (unsigned t = threadIdx.x; t < nw; t += kWideWG) bm[t] = bitmap[t];
  __syncthreads();
  unsigned cnt = 0, orv = 0;
  stream_chunks(in, cb, ce, w4, lane, nullptr, a.in.hdr, [&](unsigned long long c, const unsigned (&v)[8]) {
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
    const unsigned valid = chunk_valid(c, lane, in.n);
    unsigned mask = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const unsigned x = v[i];
      if ((unsigned long long)x < domain) {
        const unsigned word = (unsigned long long)x < lds_bits ? bm[x >> 5] : bitmap[x >> 5];
        if ((word >> (x & 31)) & 1u) mask |= 1u << i;
      }
    }
    mask &= valid;
    bitmask[c * 64 + lane] = (unsigned char)mask;
    cnt += __popc(mask);
    if (mask) orv |= (unsigned)idx0 | (31u - __clz(mask));
  });
  cnt = wave_add(cnt);
  orv = wave_or(orv);
  if (lane == 0) {
    s_cnt[w] = cnt;
    s_or[w] = orv;
  }
  __syncthreads();
  if (w4 == 0 && lane == 0 && seg < G) {
    a.seg_count[seg] = s_cnt[w] + s_cnt[w + 1] + s_cnt[w + 2] + s_cnt[w + 3];
    a.seg_or[seg] = s_or[w] | s_or[w + 1] | s_or[w + 2] | s_or[w + 3];
  }
}

hipError_t launch_pred(const PredArgs &a, unsigned G, void *s) {
  // the semi-join probes (the first kLdsBitmapBits bits of) its bitmap in LDS
  const size_t shm = a.mode == 1 ? kRingBytes : ring_shm(a.in);
  const bool wide = a.mode == 1 && a.in.kind != RLE && a.domain > kLdsBitmapBits;
  if (!wide && batch::recording()) return batch::record_task(BK_PRED0 + a.mode, &a, sizeof(a), G, shm);
  if (a.mode == 0)
    MS_LAUNCH_SHM("k_pred<0>", k_pred<0>, G, kWG, shm, s, a);
  else if (a.mode == 1 && a.in.kind != RLE && a.domain > kLdsBitmapBits)
    MS_LAUNCH(k_semijoin_wide, (G + 3) / 4, kWideWG, s, a, G);
  else if (a.mode == 1)
    MS_LAUNCH_SHM("k_pred<1>", k_pred<1>, G, kWG, shm, s, a);
  else
    MS_LAUNCH_SHM("k_pred<2>", k_pred<2>, G, kWG, shm, s, a);
  return hipGetLastError();
}

hipError_t launch_pred_batch(unsigned mode, const PredArgs *tasks, const BatchQueue &q, unsigned grid, size_t shm,
                             void *s) {
  if (mode == 0)
    MS_LAUNCH_SHM("k_pred_batch<0>", k_pred_batch<0>, grid, kWG, shm, s, tasks, q);
  else if (mode == 1)
    MS_LAUNCH_SHM("k_pred_batch<1>", k_pred_batch<1>, grid, kWG, shm, s, tasks, q);
  else
    MS_LAUNCH_SHM("k_pred_batch<2>", k_pred_batch<2>, grid, kWG, shm, s, tasks, q);
  return hipGetLastError();
}
}  // namespace ms
