// ms_device.h -- device primitives for CDNA4 (gfx950, wave64).
//
// Unit of work: a wave handles one 512-value chunk at a time, lane l holding the
// 8 consecutive values 8l..8l+7 of the chunk.  Packed at width W those 8 values
// are the W bytes starting at byte l*W of the chunk's packed block, so every lane
// reads one short contiguous window and unpacks it with compile-time shifts
// (one instantiation per width 0..32).  Packing runs the other way: each lane
// ORs its window into a zeroed per-wave LDS block, then the wave writes the
// block out with 16-byte stores.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>

#include "ms_internal.h"

namespace ms {

#define MS_WIDTH_CASES(X)                                                                                        \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
  X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

// Address of the library's device error word (the first data-dependent error since the
// last sync).  Every translation unit has its own copy of this pointer; all of them are
// set to the same word when the library is initialised.
namespace {
__constant__ unsigned *g_err_word;
}

__device__ __forceinline__ void raise_err(unsigned code) { atomicCAS(g_err_word, 0u, code); }

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }
// Values the whole wave shares, moved to scalar registers: branches on them become
// scalar branches and their loads scalar work.
__device__ __forceinline__ unsigned uni(unsigned x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ unsigned long long uni(unsigned long long x) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)x);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
__device__ __forceinline__ unsigned bw(unsigned x) { return x ? 32u - __clz(x) : 0u; }
__device__ __forceinline__ unsigned lowmask(unsigned w) { return w >= 32 ? 0xFFFFFFFFu : ((1u << w) - 1u); }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cross-lane operations through DPP (data-parallel primitives inside the VALU: no LDS
// round trip).  An inclusive scan runs as four row shifts (1, 2, 4, 8 lanes inside each
// row of 16; lanes whose source lies outside the row keep the operation's identity), then
// the totals of rows 0..2, read into scalar registers, are folded into the later rows.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned dpp(unsigned ident, unsigned x) {
  return (unsigned)__builtin_amdgcn_update_dpp((int)ident, (int)x, CTRL, ROW_MASK, 0xF, false);
}
template <class Op>
__device__ __forceinline__ unsigned wave_incl_scan(unsigned x, unsigned ident, Op op, unsigned &total) {
  x = op(x, dpp<0x111, 0xF>(ident, x));  // row_shr:1
  x = op(x, dpp<0x112, 0xF>(ident, x));  // row_shr:2
  x = op(x, dpp<0x114, 0xF>(ident, x));  // row_shr:4
  x = op(x, dpp<0x118, 0xF>(ident, x));  // row_shr:8
  const unsigned t0 = __builtin_amdgcn_readlane(x, 15), t1 = __builtin_amdgcn_readlane(x, 31);
  const unsigned t2 = __builtin_amdgcn_readlane(x, 47), t3 = __builtin_amdgcn_readlane(x, 63);
  const unsigned p1 = t0, p2 = op(t0, t1), p3 = op(p2, t2);
  total = op(p3, t3);
  const unsigned row = __lane_id() >> 4;
  return op(x, row == 0 ? ident : row == 1 ? p1 : row == 2 ? p2 : p3);
}
template <class Op>
__device__ __forceinline__ unsigned wave_incl_scan(unsigned x, unsigned ident, Op op) {
  unsigned total;
  return wave_incl_scan(x, ident, op, total);
}
struct OpAdd {
  __device__ unsigned operator()(unsigned a, unsigned b) const { return a + b; }
};
struct OpOr {
  __device__ unsigned operator()(unsigned a, unsigned b) const { return a | b; }
};
struct OpMin {
  __device__ unsigned operator()(unsigned a, unsigned b) const { return a < b ? a : b; }
};
struct OpMax {
  __device__ unsigned operator()(unsigned a, unsigned b) const { return a > b ? a : b; }
};
// Reductions, as wave-uniform values.
template <class Op>
__device__ __forceinline__ unsigned wave_reduce(unsigned x, unsigned ident, Op op) {
  x = op(x, dpp<0x111, 0xF>(ident, x));  // row_shr:1
  x = op(x, dpp<0x112, 0xF>(ident, x));  // row_shr:2
  x = op(x, dpp<0x114, 0xF>(ident, x));  // row_shr:4
  x = op(x, dpp<0x118, 0xF>(ident, x));  // row_shr:8: lane 15 of each row holds the row's total
  return op(op(__builtin_amdgcn_readlane(x, 15), __builtin_amdgcn_readlane(x, 31)),
            op(__builtin_amdgcn_readlane(x, 47), __builtin_amdgcn_readlane(x, 63)));
}
__device__ __forceinline__ unsigned wave_or(unsigned x) { return wave_reduce(x, 0u, OpOr()); }
__device__ __forceinline__ unsigned wave_min(unsigned x) { return wave_reduce(x, 0xFFFFFFFFu, OpMin()); }
__device__ __forceinline__ unsigned wave_add(unsigned x) { return wave_reduce(x, 0u, OpAdd()); }
__device__ __forceinline__ unsigned wave_max(unsigned x) { return wave_reduce(x, 0u, OpMax()); }
__device__ __forceinline__ unsigned long long wave_add64(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
  return x;
}
// Exclusive prefix sum over the 64 lanes (wrapping uint32 arithmetic).
__device__ __forceinline__ unsigned wave_excl_scan(unsigned x, unsigned lane) {
  (void)lane;
  return wave_incl_scan(x, 0u, OpAdd()) - x;
}
// The value of the previous lane (lane 0 gets 0): a row shift, and the last lane of the
// previous row for the first lane of rows 1..3.
__device__ __forceinline__ unsigned lane_prev(unsigned x) {
  const unsigned y = dpp<0x111, 0xF>(0u, x);  // row_shr:1
  const unsigned l = __lane_id();
  const unsigned e15 = __builtin_amdgcn_readlane(x, 15), e31 = __builtin_amdgcn_readlane(x, 31);
  const unsigned e47 = __builtin_amdgcn_readlane(x, 47);
  return l == 16 ? e15 : l == 32 ? e31 : l == 48 ? e47 : y;
}
// if_set where bit `lane` of the wave-uniform mask w is set, else if_clear: one VALU select
// whose lane condition is w itself (held in a scalar register pair).
__device__ __forceinline__ unsigned lane_bit_select(unsigned long long w, unsigned if_set, unsigned if_clear) {
  unsigned r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(if_clear), "v"(if_set), "s"(w));
  return r;
}
// Set bits of the wave-uniform mask w in lanes below this one, plus acc.
__device__ __forceinline__ unsigned lanes_below(unsigned long long w, unsigned acc) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(w >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)w, acc));
}
// OR of the indices (0..63) of the set bits of w.
__device__ __forceinline__ unsigned bit_index_or(unsigned long long w) {
  return ((w & 0xAAAAAAAAAAAAAAAAull) ? 1u : 0u) | ((w & 0xCCCCCCCCCCCCCCCCull) ? 2u : 0u) |
         ((w & 0xF0F0F0F0F0F0F0F0ull) ? 4u : 0u) | ((w & 0xFF00FF00FF00FF00ull) ? 8u : 0u) |
         ((w & 0xFFFF0000FFFF0000ull) ? 16u : 0u) | ((w & 0xFFFFFFFF00000000ull) ? 32u : 0u);
}
// The value of lane 63 / lane 0, wave-uniform.
__device__ __forceinline__ unsigned lane_last(unsigned x) { return __builtin_amdgcn_readlane(x, 63); }
__device__ __forceinline__ unsigned lane_first(unsigned x) { return __builtin_amdgcn_readlane(x, 0); }

// ---------------------------------------------------------------------------------------------
// Unpack: lane's 8 values of a block packed at width W (block 64-byte aligned).
template <int W>
__device__ __forceinline__ void extract8(const unsigned *w, unsigned (&v)[8]) {
#pragma unroll
  for (int i = 0; i < 8; i++) {
    constexpr unsigned mask = (W >= 32) ? 0xFFFFFFFFu : ((1u << W) - 1u);
    const int bit = i * W;
    const int q = bit >> 5, sh = bit & 31;
    if (sh + W <= 32)
      v[i] = (w[q] >> sh) & mask;
    else
      v[i] = __builtin_amdgcn_alignbit(w[q + 1], w[q], sh) & mask;
  }
}

// The lane's window: byte offset lane*W of the block, i.e. word (lane*W)/4 at bit
// shift 8*((lane*W) mod 4).  Computed once at run time so that nothing per width is
// hoisted out of the callers' loops.
struct Window {
  unsigned word;  // first word of the lane's window
  unsigned s;     // bit shift of the first value inside that word (0, 8, 16 or 24)
};
__device__ __forceinline__ Window lane_window(unsigned W, unsigned lane) {
  unsigned byte = lane * W;
  asm volatile("" : "+v"(byte));  // keep the window per iteration, not per width
  return Window{byte >> 2, (byte & 3u) * 8u};
}

template <int W>
__device__ __forceinline__ void unpack8(const unsigned *__restrict__ p, unsigned s, unsigned lane, unsigned (&v)[8]) {
  if constexpr (W == 0) {
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = 0;
  } else if constexpr (W == 32) {
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
    uint4 a = q[0], b = q[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else if constexpr (W % 4 == 0) {
    constexpr int NW = W / 4;  // the lane's window is word aligned (s == 0)
    unsigned w[NW];
#pragma unroll
    for (int k = 0; k < NW; k++) w[k] = p[k];
    extract8<W>(w, v);
  } else {
    constexpr int NW = (W + 3) / 4;
    unsigned raw[NW + 1], w[NW];
#pragma unroll
    for (int k = 0; k <= NW; k++) raw[k] = p[k];
#pragma unroll
    for (int k = 0; k < NW; k++) w[k] = __builtin_amdgcn_alignbit(raw[k + 1], raw[k], s);
    extract8<W>(w, v);
  }
}

__device__ __forceinline__ void unpack8_rt(unsigned W, const unsigned *__restrict__ blk, unsigned lane,
                                           unsigned (&v)[8]) {
  const Window win = lane_window(W, lane);
  const unsigned *p = blk + win.word;
  switch (W) {
#define MS_UNPACK_CASE(w) \
  case w: unpack8<w>(p, win.s, lane, v); break;
    MS_WIDTH_CASES(MS_UNPACK_CASE)
#undef MS_UNPACK_CASE
    default:
#pragma unroll
      for (int i = 0; i < 8; i++) v[i] = 0;
  }
}

// Random access: the value at bit offset `bit` of width W in a packed stream.
__device__ __forceinline__ unsigned extract_at(const unsigned *__restrict__ words, unsigned long long bit, unsigned W) {
  if (W == 0) return 0;
  const unsigned long long q = bit >> 5;
  const unsigned sh = (unsigned)(bit & 31);
  const unsigned lo = words[q];
  const unsigned hi = (sh + W > 32) ? words[q + 1] : 0u;
  return __builtin_amdgcn_alignbit(hi, lo, sh) & lowmask(W);
}

// ---------------------------------------------------------------------------------------------
// Pack: OR the lane's 8 W-bit values into a zeroed LDS block (16*W words).
template <int W>
__device__ __forceinline__ void pack8_lds(unsigned *dst, unsigned s, const unsigned (&r)[8]) {
  if constexpr (W == 0) {
    return;
  } else if constexpr (W == 32) {
#pragma unroll
    for (int i = 0; i < 8; i++) dst[i] = r[i];
  } else {
    constexpr int NW = (W + 3) / 4;
    unsigned w[NW + 1];
#pragma unroll
    for (int k = 0; k <= NW; k++) w[k] = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const int bit = i * W;
      const int q = bit >> 5, sh = bit & 31;
      w[q] |= r[i] << sh;
      if (sh + W > 32) w[q + 1] |= r[i] >> (32 - sh);
    }
    if constexpr (W % 4 == 0) {
#pragma unroll
      for (int k = 0; k < NW; k++) dst[k] = w[k];  // word-aligned, owned by this lane alone
    } else if constexpr (W > 4) {
      // 8W > 32 bits per lane: a word holds bits of at most two neighbouring lanes.  The
      // lane writes every word it touches except a partial last one, which the next lane
      // writes with this lane's part brought over by a lane shift; every word of the
      // block is written exactly once, so the buffer needs no clearing and no atomics.
      unsigned g[NW + 1];  // the lane's bits of words 0..NW of its window
#pragma unroll
      for (int k = 0; k <= NW; k++) {
        const unsigned hi = k < NW ? w[k] : 0u, lo = k > 0 ? w[k - 1] : 0u;
        g[k] = (unsigned)(((((unsigned long long)hi) << 32) | lo) >> (32u - s));
      }
      const unsigned e = s + 8u * W;          // end bit relative to the window's first word
      const unsigned nspan = (e + 31u) >> 5;  // NW or NW + 1 words
      const bool last_partial = (e & 31u) != 0u;
      const unsigned last = (nspan == (unsigned)NW + 1u) ? g[NW] : g[NW - 1];
      const unsigned from_prev = lane_prev(last_partial ? last : 0u);
      if (s != 0u) g[0] |= from_prev;  // the previous lane ended inside this word
      const unsigned nwrite = last_partial ? nspan - 1u : nspan;
#pragma unroll
      for (int k = 0; k <= NW; k++)
        if ((unsigned)k < nwrite) dst[k] = g[k];
    } else {
      unsigned prev = 0;
#pragma unroll
      for (int k = 0; k <= NW; k++) {
        const unsigned cur = w[k];
        const unsigned g = (unsigned)(((((unsigned long long)cur) << 32) | prev) << s >> 32);
        if (g) atomicOr(dst + k, g);
        prev = cur;
      }
    }
  }
}

__device__ __forceinline__ void pack8_lds_rt(unsigned W, unsigned *lds, unsigned lane, const unsigned (&r)[8]) {
  const Window win = lane_window(W, lane);
  unsigned *dst = lds + win.word;
  switch (W) {
#define MS_PACK_CASE(w) \
  case w: pack8_lds<w>(dst, win.s, r); break;
    MS_WIDTH_CASES(MS_PACK_CASE)
#undef MS_PACK_CASE
    default: break;
  }
}

// Pack one 512-value block held by the wave (8 values per lane, each < 2^W) and
// write its 16*W words to dst (64-byte aligned).  lds: the wave's 512-word buffer.
__device__ __forceinline__ void pack_block(unsigned W, const unsigned (&r)[8], unsigned lane, unsigned *lds,
                                           unsigned *__restrict__ dst) {
  if (W == 0) return;
  const unsigned words = 16u * W;
  if (W < 4) {  // several lanes share a word: OR-ed in with LDS atomics
    for (unsigned q = lane; q < words; q += 64) lds[q] = 0;
    wave_sync();
  }
  pack8_lds_rt(W, lds, lane, r);
  wave_sync();
  const uint4 *s4 = reinterpret_cast<const uint4 *>(lds);
  uint4 *d4 = reinterpret_cast<uint4 *>(dst);
  for (unsigned q = lane; q < 4u * W; q += 64) d4[q] = s4[q];
  wave_sync();
}

// ---------------------------------------------------------------------------------------------
// Input column as seen by a kernel, with the sizes read from its device header.
struct InCol {
  unsigned kind, W;
  unsigned long long n, n_main, nb, runs, payload_cap;
  const unsigned char *widths;
  const unsigned *offsets, *bases, *payload, *rem, *rvalues, *rstarts;
};

__device__ __forceinline__ InCol load_in(const ColView &c) {
  InCol in;
  in.kind = c.kind;
  in.n = uni(c.hdr->n);
  in.W = uni(c.hdr->sbp_width);
  in.runs = uni(min(c.hdr->runs, c.n_cap));
  in.payload_cap = c.payload_cap;
  in.widths = c.widths;
  in.offsets = c.offsets;
  in.bases = c.bases;
  in.payload = c.payload;
  in.rem = c.rem;
  in.rvalues = c.rvalues;
  in.rstarts = c.rstarts;
  if (c.kind == STATIC_BP)
    in.n_main = in.n & ~31ull;
  else if (c.kind == DYN_BP || c.kind == DELTA_DYN_BP || c.kind == FOR_DYN_BP)
    in.n_main = in.n & ~511ull;
  else
    in.n_main = in.n;
  in.nb = in.n_main >> 9;
  return in;
}

// Last run r with rstarts[r] <= idx (runs are sorted by start, rstarts[0] = 0), searched
// in [lo, hi) where the caller knows rstarts[lo] <= idx.
__device__ __forceinline__ unsigned long long rle_find_in(const InCol &in, unsigned long long idx,
                                                         unsigned long long lo, unsigned long long hi) {
  while (hi - lo > 1) {
    unsigned long long mid = (lo + hi) >> 1;
    if (in.rstarts[mid] <= idx)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Run holding value idx, found by the whole wave: each step probes 64 evenly spaced
// runs at once.  Bounds: the run index of value idx lies in [idx - (n - R), idx].
__device__ __forceinline__ unsigned long long rle_find_wave(const InCol &in, unsigned long long idx, unsigned lane,
                                                           unsigned long long hint) {
  const unsigned long long slack = in.n - in.runs;
  unsigned long long lo = idx > slack ? idx - slack : 0ull;
  unsigned long long hi = min(in.runs, idx + 1);
  // hint: the run of an earlier value; the run of idx is at or after it
  if (hint < hi && hint > lo) {
    const unsigned sh = in.rstarts[hint];
    if (sh <= idx) {
      lo = hint;
      hi = min(hi, hint + (idx - sh) + 1);  // at most one new run per value after run `hint` starts
    }
  }
  if (lo >= hi) lo = hi ? hi - 1 : 0;
  while (hi - lo > 1) {
    const unsigned long long step = (hi - lo + 63) / 64;
    const unsigned long long probe = lo + lane * step;
    const bool ok = probe < hi && in.rstarts[probe] <= idx;
    const unsigned long long m = __ballot(ok);
    const unsigned j = m ? 63u - __clzll(m) : 0u;
    lo = lo + j * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

__device__ __forceinline__ unsigned long long rle_find(const InCol &in, unsigned long long idx) {
  unsigned long long lo = 0, hi = in.runs;  // invariant: rstarts[lo] <= idx, answer in [lo, hi)
  while (hi - lo > 1) {
    unsigned long long mid = (lo + hi) >> 1;
    if (in.rstarts[mid] <= idx)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Decode chunk c (values 512c .. 512c+511); lane gets 8 consecutive values.  Values
// at indices >= n are unspecified (callers mask them out).
__device__ __forceinline__ void decode_chunk(const InCol &in, unsigned long long c, unsigned lane, unsigned (&v)[8],
                                             unsigned long long &rle_hint) {
  const unsigned long long idx0 = c * kBlk + 8ull * lane;
  switch (in.kind) {
    case UNCOMPR: {
      if (idx0 + 8 <= in.n) {
        const uint4 *p = reinterpret_cast<const uint4 *>(in.payload + idx0);
        uint4 a = p[0], b = p[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
      } else {
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = (idx0 + i < in.n) ? in.payload[idx0 + i] : 0u;
      }
      break;
    }
    case STATIC_BP: {
      if (c * kBlk < in.n_main && in.W <= 32 && (c + 1) * 16ull * in.W <= in.payload_cap + 512) {
        unpack8_rt(in.W, in.payload + c * 16ull * in.W, lane, v);  // lanes past n_main read slack
      }
      if (idx0 >= in.n_main) {
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = (idx0 + i < in.n) ? in.rem[idx0 + i - in.n_main] : 0u;
      }
      break;
    }
    case DYN_BP:
    case DELTA_DYN_BP:
    case FOR_DYN_BP: {
      if (c < in.nb) {
        unsigned W = uni((unsigned)in.widths[c]);
        unsigned long long off = uni((unsigned long long)in.offsets[c]);
        if (W > 32 || off + 16ull * W > in.payload_cap) {  // a corrupt directory never reads out of bounds
          raise_err(E_INVALID);
          W = 0;
          off = 0;
        }
        unpack8_rt(W, in.payload + off, lane, v);
        if (in.kind == FOR_DYN_BP) {
          const unsigned ref = uni(in.bases[c]);
#pragma unroll
          for (int i = 0; i < 8; i++) v[i] += ref;
        } else if (in.kind == DELTA_DYN_BP) {
#pragma unroll
          for (int i = 1; i < 8; i++) v[i] += v[i - 1];
          const unsigned excl = wave_excl_scan(v[7], lane) + uni(in.bases[c]);
#pragma unroll
          for (int i = 0; i < 8; i++) v[i] += excl;
        }
      } else {
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = (idx0 + i < in.n) ? in.rem[idx0 + i - in.n_main] : 0u;
      }
      break;
    }
    case RLE: {
      // run of the chunk's first value by a 64-way search of the whole wave (bounded by
      // the wave's previous chunk), then each lane finds its own run among the at most
      // 8*lane + 1 runs that follow and reads the next 8 run starts at once
      const unsigned long long c0 = c * kBlk;
      unsigned long long r0 = 0;
      if (c0 < in.n) {
        r0 = rle_find_wave(in, c0, lane, rle_hint);
        rle_hint = r0;
      }
      if (idx0 < in.n) {
        const unsigned long long hi = min(in.runs, r0 + 8ull * lane + 1);
        unsigned long long r;
        if (in.rstarts[hi - 1] <= idx0) {  // dense runs: the upper bound itself
          r = hi - 1;
        } else {
          unsigned long long lo = r0, step = 1;
          while (lo + step < hi && in.rstarts[lo + step] <= idx0) {
            lo += step;
            step <<= 1;
          }
          r = rle_find_in(in, idx0, lo, min(hi, lo + step));
        }
        unsigned st[7], val[8];
#pragma unroll
        for (int k = 0; k < 7; k++) st[k] = (r + 1 + k < in.runs) ? in.rstarts[r + 1 + k] : 0xFFFFFFFFu;
#pragma unroll
        for (int k = 0; k < 8; k++) val[k] = (r + k < in.runs) ? in.rvalues[r + k] : 0u;
        // value i is in run r + (number of run starts in (idx0, idx0 + i])
#pragma unroll
        for (int i = 0; i < 8; i++) {
          unsigned x = val[0];
#pragma unroll
          for (int k = 0; k < 7; k++)
            if (k < i && st[k] <= idx0 + i) x = val[k + 1];
          v[i] = x;
        }
      } else {
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = 0;
      }
      break;
    }
    default:
#pragma unroll
      for (int i = 0; i < 8; i++) v[i] = 0;
  }
}

__device__ __forceinline__ void decode_chunk(const InCol &in, unsigned long long c, unsigned lane, unsigned (&v)[8]) {
  unsigned long long hint = 0;
  decode_chunk(in, c, lane, v, hint);
}

// ---------------------------------------------------------------------------------------------
// Pipelined chunk decode.  issue() starts the global loads of one chunk (coalesced
// 16-byte loads of the packed block, or the lane's own 8 values when uncompressed)
// without waiting for them; finish() stages a packed block through the wave's LDS
// buffer, unpacks the lane's window and applies FOR / DELTA.  Callers issue chunk
// c + kWaves before finishing chunk c, so two chunks per wave are in flight.
// Partial chunks, remainders and RLE take the direct path (decode_chunk).
struct Raw {
  uint4 q0, q1;
  unsigned W, base;
  unsigned mode;  // 0 packed block, 1 uncompressed lane data, 2 direct path
};

__device__ __forceinline__ Raw issue_chunk(const InCol &in, unsigned long long c, unsigned lane) {
  Raw r;
  r.q0 = make_uint4(0, 0, 0, 0);
  r.q1 = r.q0;
  r.W = 0;
  r.base = 0;
  r.mode = 2;
  const unsigned long long c0 = c * kBlk;
  const unsigned *blk = nullptr;
  switch (in.kind) {
    case UNCOMPR:
      if (c0 + kBlk <= in.n) {
        const uint4 *p = reinterpret_cast<const uint4 *>(in.payload + c0) + 2 * lane;
        r.q0 = p[0];
        r.q1 = p[1];
        r.mode = 1;
      }
      return r;
    case STATIC_BP:
      if (c0 + kBlk <= in.n_main && in.W <= 32) {
        r.W = in.W;
        blk = in.payload + c * 16ull * in.W;
        r.mode = 0;
      }
      break;
    case DYN_BP:
    case DELTA_DYN_BP:
    case FOR_DYN_BP:
      if (c < in.nb) {
        unsigned W = in.widths[c];
        unsigned long long off = in.offsets[c];
        if (W > 32 || off + 16ull * W > in.payload_cap) {  // a corrupt directory never reads out of bounds
          raise_err(E_INVALID);
          W = 0;
          off = 0;
        }
        r.W = W;
        r.base = (in.kind == DYN_BP) ? 0u : uni(in.bases[c]);
        blk = in.payload + off;
        r.mode = 0;
      }
      break;
    default: return r;
  }
  if (r.mode == 0) {
    const uint4 *b4 = reinterpret_cast<const uint4 *>(blk);
    const unsigned nq = 4u * r.W;  // 16-byte pieces of the block
    if (lane < nq) r.q0 = b4[lane];
    if (lane + 64 < nq) r.q1 = b4[lane + 64];
  }
  return r;
}

__device__ __forceinline__ void finish_chunk(const InCol &in, const Raw &r, unsigned long long c, unsigned lane,
                                             unsigned *lds, unsigned (&v)[8]) {
  if (r.mode == 1) {
    v[0] = r.q0.x; v[1] = r.q0.y; v[2] = r.q0.z; v[3] = r.q0.w;
    v[4] = r.q1.x; v[5] = r.q1.y; v[6] = r.q1.z; v[7] = r.q1.w;
    return;
  }
  if (r.mode == 2) {
    decode_chunk(in, c, lane, v);
    return;
  }
  uint4 *l4 = reinterpret_cast<uint4 *>(lds);
  const unsigned nq = 4u * r.W;
  if (lane < nq) l4[lane] = r.q0;
  if (lane + 64 < nq) l4[lane + 64] = r.q1;
  wave_sync();
  unpack8_rt(r.W, lds, lane, v);
  wave_sync();
  if (in.kind == FOR_DYN_BP) {
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] += r.base;
  } else if (in.kind == DELTA_DYN_BP) {
#pragma unroll
    for (int i = 1; i < 8; i++) v[i] += v[i - 1];
    const unsigned excl = wave_excl_scan(v[7], lane) + r.base;
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] += excl;
  }
}

// v[k] for a lane-varying k in 0..7, as a chain of selects (an indexed read of the
// register array would go through scratch memory).
__device__ __forceinline__ unsigned select8(const unsigned (&v)[8], unsigned k) {
  unsigned x = v[0];
#pragma unroll
  for (int i = 1; i < 8; i++) {
    x = k == (unsigned)i ? v[i] : x;
    asm volatile("" : "+v"(x));
  }
  return x;
}

constexpr int kRing = 4;  // the kernels' per-wave LDS buffer holds kRing * 512 words

// ---------------------------------------------------------------------------------------------
// Direct window loads.  A packed 512-value block (uncompressed = width 32) is read by
// each lane straight into registers: its 8 values are W bytes at byte lane * W, a window
// of at most 9 words.  Loads of kPre chunks are in flight per wave; every width has its
// own load and unpack code, picked by a scalar branch per chunk.
constexpr int kPre = 4;
constexpr int kWin = 9;
struct Win {
  unsigned x[kWin];
};

template <int W>
__device__ __forceinline__ void win_issue(const unsigned *__restrict__ blk, unsigned lane, Win &r) {
  if constexpr (W == 0) {
    return;
  } else if constexpr (W % 16 == 0) {  // 16-byte aligned window of W/4 words
    const uint4 *q = reinterpret_cast<const uint4 *>(blk + lane * (W / 4));
#pragma unroll
    for (int k = 0; k < W / 16; k++) {
      const uint4 a = q[k];
      r.x[4 * k] = a.x; r.x[4 * k + 1] = a.y; r.x[4 * k + 2] = a.z; r.x[4 * k + 3] = a.w;
    }
  } else if constexpr (W % 8 == 0) {  // 8-byte aligned window of W/4 words
    const uint2 *q = reinterpret_cast<const uint2 *>(blk + lane * (W / 4));
#pragma unroll
    for (int k = 0; k < W / 8; k++) {
      const uint2 a = q[k];
      r.x[2 * k] = a.x; r.x[2 * k + 1] = a.y;
    }
  } else if constexpr (W % 4 == 0) {
    const unsigned *q = blk + lane * (W / 4);
#pragma unroll
    for (int k = 0; k < W / 4; k++) r.x[k] = q[k];
  } else {  // window at byte lane * W: (W + 3) / 4 words and one more for the shift
    const unsigned *q = blk + ((lane * W) >> 2);
#pragma unroll
    for (int k = 0; k <= (W + 3) / 4; k++) r.x[k] = q[k];
  }
}

template <int W>
__device__ __forceinline__ void win_unpack(const Win &r, unsigned lane, unsigned (&v)[8]) {
  if constexpr (W == 0) {
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = 0;
  } else if constexpr (W == 32) {
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = r.x[i];
  } else if constexpr (W % 4 == 0) {
    extract8<W>(r.x, v);
  } else {
    constexpr int NW = (W + 3) / 4;
    const unsigned sh = ((lane * W) & 3u) * 8u;
    unsigned w[NW];
#pragma unroll
    for (int k = 0; k < NW; k++) w[k] = __builtin_amdgcn_alignbit(r.x[k + 1], r.x[k], sh);
    extract8<W>(w, v);
  }
}

// Fixed-count window loads (the same loads for every width, so that the compiler can
// count them and wait only for the chunk it consumes): 9 words from word (lane*W)/4 of a
// packed block, or a lane's 8 words of an uncompressed chunk.
__device__ __forceinline__ void win_issue9(const unsigned *__restrict__ blk, unsigned W, unsigned lane, Win &r) {
  const unsigned *q = blk + ((lane * W) >> 2);
#pragma unroll
  for (int k = 0; k < kWin; k++) r.x[k] = q[k];
}
__device__ __forceinline__ void win_issue_unc(const unsigned *__restrict__ blk, unsigned lane, Win &r) {
  const uint4 *q = reinterpret_cast<const uint4 *>(blk + 8u * lane);
  const uint4 a = q[0], b = q[1];
  r.x[0] = a.x; r.x[1] = a.y; r.x[2] = a.z; r.x[3] = a.w;
  r.x[4] = b.x; r.x[5] = b.y; r.x[6] = b.z; r.x[7] = b.w;
}

__device__ __forceinline__ void win_issue_rt(unsigned W, const unsigned *__restrict__ blk, unsigned lane, Win &r) {
  switch (W) {
#define MS_ISSUE_CASE(w) \
  case w: win_issue<w>(blk, lane, r); break;
    MS_WIDTH_CASES(MS_ISSUE_CASE)
#undef MS_ISSUE_CASE
    default: break;
  }
}

__device__ __forceinline__ void win_unpack_rt(unsigned W, const Win &r, unsigned lane, unsigned (&v)[8]) {
  switch (W) {
#define MS_WUNPACK_CASE(w) \
  case w: win_unpack<w>(r, lane, v); break;
    MS_WIDTH_CASES(MS_WUNPACK_CASE)
#undef MS_WUNPACK_CASE
    default:
      __builtin_unreachable();  // widths come from locate(), which maps a corrupt one to 0
  }
}

// RLE input walked run by run over the chunks [c_begin, c_end).  The runs [r, whi) it needs are staged in a ring of kRunCap (start, value)
// pairs in its LDS (run q in slot q mod kRunCap); each lane finds its 8 values there.
// While a chunk's body runs, the runs the next chunks will need are already being
// loaded (coalesced) into registers, so sparse and dense runs both stream without a
// load round trip per chunk.  lds: 2 * kRunCap words.
constexpr unsigned kRunCap = 1024;
constexpr unsigned kRunMask = kRunCap - 1;
constexpr unsigned kRunPre = 9;  // prefetch rounds of 64 runs (576 runs at most)
static_assert(2 * kRunCap <= kRing * kBlk, "run staging fits the wave's ring buffer");
static_assert((kRunCap & kRunMask) == 0, "ring size is a power of two");

template <class Body>
__device__ __forceinline__ void rle_stream(const InCol &in, unsigned long long c_begin, unsigned long long c_end,
                                           unsigned lane, unsigned *lds, Body &&body) {
  if (c_begin >= c_end) return;
  unsigned *S = lds, *V = lds + kRunCap;
  unsigned long long r = (in.runs > 0) ? rle_find_wave(in, c_begin * kBlk, lane, 0) : 0ull;
  unsigned long long whi = r;  // runs [r, whi) are staged
  unsigned est = 64;           // runs per chunk, as the last chunk had
  unsigned pst[kRunPre], pval[kRunPre];
  unsigned npre = 0;           // rounds of 64 in flight in pst/pval, for runs [whi, whi + 64 * npre)

  auto issue = [&](unsigned rounds) {
#pragma unroll
    for (unsigned k = 0; k < kRunPre; k++) {
      if (k < rounds) {
        const unsigned long long q = whi + 64ull * k + lane;
        pst[k] = (q < in.runs) ? in.rstarts[q] : 0xFFFFFFFFu;
        pval[k] = (q < in.runs) ? in.rvalues[q] : 0u;
      }
    }
    npre = rounds;
  };
  auto land = [&]() {
#pragma unroll
    for (unsigned k = 0; k < kRunPre; k++) {
      if (k < npre) {
        const unsigned slot = (unsigned)((whi + 64ull * k + lane) & kRunMask);
        S[slot] = pst[k];
        V[slot] = pval[k];
      }
    }
    whi += 64ull * npre;
    npre = 0;
    wave_sync();
  };

  for (unsigned long long c = c_begin; c < c_end; c++) {
    const unsigned long long c0 = c * kBlk;
    const unsigned long long c1 = min(c0 + kBlk, in.n);
    // make sure the staged runs reach past c1 (or the last run)
    while (true) {
      const bool covered = whi >= in.runs || (whi > r && (unsigned long long)S[(whi - 1) & kRunMask] >= c1);
      if (covered || whi - r + 64 > kRunCap) break;
      const unsigned room = (unsigned)(kRunCap - (whi - r)) / 64;
      issue(min(min(room, kRunPre), max(1u, (est + 63) / 64 + 1)));
      land();
    }
    const unsigned long long nst = whi - r;  // staged runs from r
    const unsigned long long idx0 = c0 + 8ull * lane;
    unsigned v[8];
    unsigned j = 0;  // staged index relative to r
    // Runs of one value each across a full chunk: run r holds c0, and the run 511 later
    // starting at c0 + 511 forces runs r + k to start at c0 + k, so value k is run r + k.
    const bool unit_runs = c1 - c0 == kBlk && nst >= kBlk && S[(r + kBlk - 1) & kRunMask] == (unsigned)(c0 + kBlk - 1);
    if (unit_runs) {
#pragma unroll
      for (int i = 0; i < 8; i++) v[i] = V[(r + 8ull * lane + i) & kRunMask];
      j = 8u * lane + 7u;
    } else if (idx0 < c1) {
      const unsigned x0 = (unsigned)idx0;
      unsigned lo = 0, hi = (unsigned)nst;  // last staged run starting at or before idx0
      while (hi - lo > 1) {
        const unsigned mid = (lo + hi) >> 1;
        if (S[(r + mid) & kRunMask] <= x0)
          lo = mid;
        else
          hi = mid;
      }
      j = lo;
      v[0] = V[(r + j) & kRunMask];
#pragma unroll
      for (int i = 1; i < 8; i++) {
        const unsigned nxt = (j + 1 < nst) ? S[(r + j + 1) & kRunMask] : 0xFFFFFFFFu;
        if (nxt <= x0 + (unsigned)i) j++;  // runs start at distinct indices: at most one per step
        v[i] = V[(r + j) & kRunMask];
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; i++) v[i] = 0u;
    }
    // the run holding c1, the first value of the next chunk
    const unsigned jl = lane_last(j);
    const unsigned nxt = (jl + 1 < nst) ? S[(r + jl + 1) & kRunMask] : 0xFFFFFFFFu;
    wave_sync();
    est = jl + 1;
    r += jl + (((unsigned long long)nxt == c1) ? 1u : 0u);
    // keep about two chunks of runs ahead: start their loads now, land them after the body
    if (c + 1 < c_end && whi < in.runs) {
      const unsigned long long ahead = whi - r;
      const unsigned long long want = min(2ull * est + 64ull, (unsigned long long)(kRunCap - 64));
      if (ahead < want) {
        const unsigned room = (unsigned)((kRunCap - ahead) / 64);
        const unsigned rounds = min(min(room, kRunPre), (unsigned)((want - ahead + 63) / 64));
        if (rounds > 0) issue(rounds);
      }
    }
    body(c, v);
    if (npre) land();
  }
}

// The chunks c = first + STRIDE * j, j < nj, of an uncompressed (MODE 0), static BP
// (MODE 1) or DynBP-family (MODE 2) column: full blocks stream through direct window
// loads, kPre chunks ahead, with the block directory of the next group of chunks loaded
// one group earlier (lane s holds chunk s's entry); the remaining chunks take the direct
// path.  In the steady-state loop every load is issued on every path, so that the
// compiler's wait counts let the kPre windows stay in flight: only the first group
// needs the window it consumes.
template <int MODE, int STRIDE, class Body>
__device__ __forceinline__ void stream_blocks(const InCol &in, unsigned long long first, unsigned long long nj,
                                              unsigned lane, Body &&body) {
  constexpr bool UNC = MODE == 0, DYN = MODE == 2;
  if (nj == 0) return;
  unsigned long long cmain;  // chunks [0, cmain) are full packed blocks
  unsigned Wfix = 32;
  if (UNC) {
    cmain = in.n / kBlk;
  } else if (!DYN) {
    cmain = (in.W <= 32) ? in.n_main / kBlk : 0ull;
    Wfix = in.W;
  } else {
    cmain = in.nb;
  }
  const unsigned long long njm = (first < cmain) ? min(nj, (cmain - first + STRIDE - 1) / STRIDE) : 0ull;
  if (njm > 0) {
    // directory of group g (chunks kPre*g .. kPre*g+3 of this wave) in lanes 0..3; every
    // lane loads (lane & 3)'s entry, clamped to the wave's last full block
    auto dir_load = [&](unsigned long long g, unsigned &dw, unsigned &doff, unsigned &dbase) {
      if (DYN) {
        const unsigned long long j = min(kPre * g + (lane & (unsigned)(kPre - 1)), njm - 1);
        const unsigned long long c = first + STRIDE * j;
        dw = in.widths[c];
        doff = in.offsets[c];
        dbase = in.bases[c];
      } else {
        dw = doff = dbase = 0;
      }
    };
    // width and payload offset of chunk j, whose directory entry is in lane s of (dw, doff)
    auto locate = [&](unsigned long long j, unsigned s, unsigned dw, unsigned doff, unsigned &W,
                      unsigned long long &off) {
      const unsigned long long c = first + STRIDE * j;
      if (DYN) {
        W = __builtin_amdgcn_readlane(dw, s);
        off = __builtin_amdgcn_readlane(doff, s);
        if (W > 32 || off + 16ull * W > in.payload_cap) {  // a corrupt directory never reads out of bounds
          raise_err(E_INVALID);
          W = 0;
          off = 0;
        }
      } else {
        W = Wfix;
        off = c * 16ull * Wfix;
      }
    };
    Win win[kPre];
    unsigned dwA, doA, dbA, dwB, doB, dbB;
    dir_load(0, dwA, doA, dbA);
    dir_load(1, dwB, doB, dbB);
    auto issue = [&](const unsigned *blk, unsigned W, Win &r) {
      if (UNC)
        win_issue_unc(blk, lane, r);
      else
        win_issue9(blk, W, lane, r);
    };
    // the first windows are loaded on every path (slots past the wave's last full block
    // load that block again and are never consumed), so that the wait counts inside the
    // steady-state loop do not have to allow for a path with fewer loads in flight
    auto prime = [&](auto S) {
      constexpr int s = decltype(S)::value;
      const unsigned long long js = min((unsigned long long)s, njm - 1);
      unsigned W;
      unsigned long long off;
      locate(js, (unsigned)js, dwA, doA, W, off);
      issue(in.payload + off, W, win[s]);
    };
    prime(std::integral_constant<int, 0>{});
    prime(std::integral_constant<int, 1>{});
    prime(std::integral_constant<int, 2>{});
    prime(std::integral_constant<int, 3>{});
    // group g: one chunk per slot (the slot index is a compile-time constant so that the
    // windows stay in registers).  Every slot reloads its window on every path (past the
    // wave's last full block it loads that block again, never consumed), so the wait
    // before a window counts the other slots' loads as still in flight.
    for (unsigned long long g = 0; kPre * g < njm; g++) {
      unsigned dwC, doC, dbC;
      dir_load(g + 2, dwC, doC, dbC);
      auto slot = [&](auto S) {
        constexpr int s = decltype(S)::value;
        const unsigned long long j = kPre * g + s;
        const bool live = j < njm;
        const unsigned long long c = first + STRIDE * j;
        unsigned v[8];
        if (live) {
          unsigned W;
          unsigned long long off;
          locate(j, s, dwA, doA, W, off);
          if (UNC) {
#pragma unroll
            for (int i = 0; i < 8; i++) v[i] = win[s].x[i];
          } else {
            win_unpack_rt(W, win[s], lane, v);
          }
          if (DYN && in.kind == FOR_DYN_BP) {
            const unsigned ref = __builtin_amdgcn_readlane(dbA, s);
#pragma unroll
            for (int i = 0; i < 8; i++) v[i] += ref;
          } else if (DYN && in.kind == DELTA_DYN_BP) {
#pragma unroll
            for (int i = 1; i < 8; i++) v[i] += v[i - 1];
            const unsigned excl = wave_excl_scan(v[7], lane) + __builtin_amdgcn_readlane(dbA, s);
#pragma unroll
            for (int i = 0; i < 8; i++) v[i] += excl;
          }
        }
        // the reload, outside any branch: chunk j + kPre, or the wave's last full block again
        {
          unsigned Wn;
          unsigned long long offn;
          locate(min(j + kPre, njm - 1), s, dwB, doB, Wn, offn);
          issue(in.payload + offn, Wn, win[s]);
        }
        // keep the reload ahead of the body: the scheduler would otherwise sink the
        // loads of all four slots to the end of the group
        __builtin_amdgcn_sched_barrier(0);
        if (live) body(c, v);
      };
      static_assert(kPre == 4, "four slots below");
      slot(std::integral_constant<int, 0>{});
      slot(std::integral_constant<int, 1>{});
      slot(std::integral_constant<int, 2>{});
      slot(std::integral_constant<int, 3>{});
      dwA = dwB; doA = doB; dbA = dbB;
      dwB = dwC; doB = doC; dbB = dbC;
    }
  }
  unsigned long long rle_hint = 0;
  for (unsigned long long j = njm; j < nj; j++) {
    const unsigned long long c = first + STRIDE * j;
    unsigned v[8];
    decode_chunk(in, c, lane, v, rle_hint);
    body(c, v);
  }
}

// Walk the wave's chunks c = cb + w + kWaves * j < ce.  Full packed blocks (the main
// part of UNCOMPR, STATIC_BP and the DynBP family) stream through direct window loads,
// kPre chunks ahead, with the block directory of the next group of chunks loaded one
// group earlier (lane s holds chunk s's entry); the remaining chunks take the direct
// path.  RLE columns are walked run by run.  ring: the wave's kRing * 512 LDS words.
template <class Body>
__device__ __forceinline__ void stream_chunks(const InCol &in, unsigned long long cb, unsigned long long ce,
                                              unsigned w, unsigned lane, unsigned *ring, const void *dummy,
                                              Body &&body) {
  (void)dummy;
  if (in.kind == RLE) {  // a contiguous quarter of the segment per wave
    const unsigned long long nseg = ce - cb;
    rle_stream(in, cb + nseg * w / kWaves, cb + nseg * (w + 1) / kWaves, lane, ring, body);
    return;
  }
  const unsigned long long first = cb + w;
  const unsigned long long nj = first < ce ? (ce - first + kWaves - 1) / kWaves : 0ull;
  if (in.kind == UNCOMPR)
    stream_blocks<0, kWaves>(in, first, nj, lane, body);
  else if (in.kind == STATIC_BP)
    stream_blocks<1, kWaves>(in, first, nj, lane, body);
  else
    stream_blocks<2, kWaves>(in, first, nj, lane, body);
}

// Walk the chunks [c_begin, c_end) in order (one wave; used where a chunk needs the
// value before it).  ring: the wave's kRing * 512 LDS words (RLE input only).
template <class Body>
__device__ __forceinline__ void stream_range(const InCol &in, unsigned long long c_begin, unsigned long long c_end,
                                             unsigned lane, unsigned *ring, Body &&body) {
  if (c_begin >= c_end) return;
  if (in.kind == RLE)
    rle_stream(in, c_begin, c_end, lane, ring, body);
  else if (in.kind == UNCOMPR)
    stream_blocks<0, 1>(in, c_begin, c_end - c_begin, lane, body);
  else if (in.kind == STATIC_BP)
    stream_blocks<1, 1>(in, c_begin, c_end - c_begin, lane, body);
  else
    stream_blocks<2, 1>(in, c_begin, c_end - c_begin, lane, body);
}

// Walk chunks cb + w, cb + w + kWaves, ... < ce with one chunk of look-ahead;
// body(c, v) gets the decoded values.  lds: the wave's 512-word buffer.
template <class Body>
__device__ __forceinline__ void for_chunks(const InCol &in, unsigned long long cb, unsigned long long ce, unsigned w,
                                           unsigned lane, unsigned *lds, Body &&body) {
  unsigned long long c = cb + w;
  if (c >= ce) return;
  Raw cur = issue_chunk(in, c, lane);
  while (true) {
    const unsigned long long cn = c + kWaves;
    const bool more = cn < ce;
    Raw nxt;
    if (more) nxt = issue_chunk(in, cn, lane);
    unsigned v[8];
    finish_chunk(in, cur, c, lane, lds, v);
    body(c, v);
    if (!more) break;
    cur = nxt;
    c = cn;
  }
}

// Random access to value idx (< n) of a column (used by project).
__device__ __forceinline__ unsigned value_at(const InCol &in, unsigned long long idx) {
  switch (in.kind) {
    case UNCOMPR: return in.payload[idx];
    case STATIC_BP:
      if (idx < in.n_main) return in.W <= 32 ? extract_at(in.payload, idx * in.W, in.W) : 0u;
      return in.rem[idx - in.n_main];
    case DYN_BP:
    case FOR_DYN_BP: {
      if (idx >= in.n_main) return in.rem[idx - in.n_main];
      const unsigned long long k = idx >> 9;
      unsigned W = in.widths[k];
      unsigned long long off = in.offsets[k];
      if (W > 32 || off + 16ull * W > in.payload_cap) {
        raise_err(E_INVALID);
        return 0;
      }
      unsigned x = extract_at(in.payload + off, (idx & 511) * W, W);
      return in.kind == FOR_DYN_BP ? x + in.bases[k] : x;
    }
    case DELTA_DYN_BP: {
      if (idx >= in.n_main) return in.rem[idx - in.n_main];
      const unsigned long long k = idx >> 9;
      const unsigned W = in.widths[k];
      const unsigned long long off = in.offsets[k];
      if (W > 32 || off + 16ull * W > in.payload_cap) {
        raise_err(E_INVALID);
        return 0;
      }
      const unsigned *p = in.payload + off;
      unsigned x = in.bases[k];
      const unsigned j = (unsigned)(idx & 511);
      for (unsigned t = 1; t <= j; t++) x += extract_at(p, (unsigned long long)t * W, W);
      return x;
    }
    case RLE: return in.rvalues[rle_find(in, idx)];
    default: return 0;
  }
}

// Gather: v[i] <- data[v[i]] for the lane's 8 positions (bit i of `valid` set), with the
// format switch outside the per-value loop so each case unrolls.  Positions >= n read 0
// and set *bad.
template <int KIND>
__device__ __forceinline__ void gather8_kind(const InCol &d, unsigned (&v)[8], unsigned valid, bool &bad) {
  InCol dk = d;
  dk.kind = KIND;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    unsigned x = 0;
    if (valid & (1u << i)) {
      if (v[i] < d.n)
        x = value_at(dk, v[i]);
      else
        bad = true;
    }
    v[i] = x;
  }
}

__device__ __forceinline__ unsigned long long wave_min64(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const unsigned long long y = __shfl_xor(x, d);
    x = y < x ? y : x;
  }
  return x;
}

// Block-wise gather for formats without cheap random access (DELTA needs the prefix of
// its block, RLE a run search): the wave decodes each touched 512-block once into
// `blk` and serves every lane's positions inside it.  Up to 16 blocks per call (enough
// for sorted positions); positions left over take the per-value path.
__device__ __forceinline__ void gather8_blocks(const InCol &d, unsigned (&v)[8], unsigned valid, bool &bad,
                                               unsigned lane, unsigned *blk, unsigned *stage) {
  unsigned pend = 0, res[8];
#pragma unroll
  for (int i = 0; i < 8; i++) {
    res[i] = 0;
    if ((valid >> i) & 1u) {
      if (v[i] < d.n)
        pend |= 1u << i;
      else
        bad = true;
    }
  }
  for (int it = 0; it < 16; it++) {
    unsigned long long mine = ~0ull;
#pragma unroll
    for (int i = 0; i < 8; i++)
      if ((pend >> i) & 1u) mine = min(mine, (unsigned long long)(v[i] >> 9));
    const unsigned long long k = wave_min64(mine);
    if (k == ~0ull) break;
    const Raw r = issue_chunk(d, k, lane);
    unsigned x[8];
    finish_chunk(d, r, k, lane, stage, x);
#pragma unroll
    for (int i = 0; i < 8; i++) blk[8 * lane + i] = x[i];
    wave_sync();
#pragma unroll
    for (int i = 0; i < 8; i++) {
      if (((pend >> i) & 1u) && (v[i] >> 9) == k) {
        res[i] = blk[v[i] & 511];
        pend &= ~(1u << i);
      }
    }
    wave_sync();
  }
#pragma unroll
  for (int i = 0; i < 8; i++)
    if ((pend >> i) & 1u) res[i] = value_at(d, v[i]);
#pragma unroll
  for (int i = 0; i < 8; i++) v[i] = res[i];
}

// blk, stage: the wave's two 512-word LDS buffers (used for DELTA and RLE data only).
// Gather from an RLE column.  When the wave's positions ascend (select outputs do), the
// runs spanning them are staged window by window in LDS (512 runs, 511 of them
// resolvable, per window; S: starts, V: values) and every position is found by binary
// search there; each window starts at the run of the smallest pending position.  Other
// position orders search each position on its own.
__device__ __forceinline__ void gather8_rle(const InCol &d, unsigned (&v)[8], unsigned valid, bool &bad,
                                            unsigned lane, unsigned *S, unsigned *V) {
  unsigned pend = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    if ((valid >> i) & 1u) {
      if (v[i] < d.n)
        pend |= 1u << i;
      else
        bad = true;
    }
  }
  bool ok = true;
#pragma unroll
  for (int i = 1; i < 8; i++)
    if ((valid >> i) & 1u) ok = ok && v[i - 1] <= v[i];
  const unsigned pl = lane_prev(v[7]);
  if (lane > 0 && (valid & 1u)) ok = ok && pl <= v[0];
  if (__ballot(!ok) != 0ull || d.runs == 0) {
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = ((pend >> i) & 1u) ? value_at(d, v[i]) : 0u;
    return;
  }
  unsigned long long r = 0;
  bool first = true;
  unsigned res_init[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (__ballot(pend != 0) != 0ull) {
    // Runs of one value each: position p then lies in run r0 + (p - pmin), where r0 holds
    // the wave's smallest position pmin; a run found to start at p holds p.  Both arrays
    // are gathered at once; the misses go on through the staged windows below.
    unsigned mine = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < 8; i++)
      if ((pend >> i) & 1u) mine = min(mine, v[i]);
    const unsigned pmin = wave_min(mine);
    const unsigned long long r0 = rle_find_wave(d, pmin, lane, 0ull);
    unsigned cand[8];
    unsigned hitm = 0;  // values resolved here
#pragma unroll
    for (int i = 0; i < 8; i++) {
      cand[i] = 0u;
      if ((pend >> i) & 1u) {
        const unsigned long long q = r0 + (v[i] - pmin);
        if (q < d.runs) {
          const unsigned s = d.rstarts[q];
          cand[i] = d.rvalues[q];
          if (s == v[i] || v[i] == pmin) hitm |= 1u << i;
        }
      }
    }
    pend &= ~hitm;
    if (__ballot(pend != 0) == 0ull) {
#pragma unroll
      for (int i = 0; i < 8; i++) v[i] = cand[i];
      return;
    }
#pragma unroll
    for (int i = 0; i < 8; i++) cand[i] = ((hitm >> i) & 1u) ? cand[i] : 0u;
    r = r0;
    first = false;
    // the misses continue through the staged windows, starting at their own smallest position
#pragma unroll
    for (int i = 0; i < 8; i++) res_init[i] = cand[i];
  }
  unsigned res[8];
#pragma unroll
  for (int i = 0; i < 8; i++) res[i] = res_init[i];
  while (__ballot(pend != 0) != 0ull) {
    unsigned mine = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < 8; i++)
      if ((pend >> i) & 1u) mine = min(mine, v[i]);
    const unsigned pmin = wave_min(mine);
    r = rle_find_wave(d, pmin, lane, first ? 0ull : r);
    first = false;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const unsigned long long q = r + 64ull * k + lane;
      S[64 * k + lane] = (q < d.runs) ? d.rstarts[q] : 0xFFFFFFFFu;
      V[64 * k + lane] = (q < d.runs) ? d.rvalues[q] : 0u;
    }
    wave_sync();
    const unsigned s_end = S[511];  // positions below the start of the last staged run resolve here
#pragma unroll
    for (int i = 0; i < 8; i++) {
      if (((pend >> i) & 1u) && v[i] < s_end) {
        unsigned lo = 0;  // last staged run starting at or before v[i] (S[0] <= v[i] < S[511])
#pragma unroll
        for (unsigned step = 256; step > 0; step >>= 1)
          if (lo + step < 511u && S[lo + step] <= v[i]) lo += step;
        res[i] = V[lo];
        pend &= ~(1u << i);
      }
    }
    wave_sync();
    r += 511;
  }
#pragma unroll
  for (int i = 0; i < 8; i++) v[i] = res[i];
}

template <bool WITH_RLE = true>
__device__ __forceinline__ void gather8(const InCol &d, unsigned (&v)[8], unsigned valid, bool &bad, unsigned lane,
                                        unsigned *blk, unsigned *stage) {
  switch (d.kind) {
    case UNCOMPR: gather8_kind<UNCOMPR>(d, v, valid, bad); break;
    case STATIC_BP: gather8_kind<STATIC_BP>(d, v, valid, bad); break;
    case DYN_BP: gather8_kind<DYN_BP>(d, v, valid, bad); break;
    case DELTA_DYN_BP: gather8_blocks(d, v, valid, bad, lane, blk, stage); break;
    case RLE:
      if constexpr (WITH_RLE) gather8_rle(d, v, valid, bad, lane, blk, stage);
      break;
    case FOR_DYN_BP: gather8_kind<FOR_DYN_BP>(d, v, valid, bad); break;
    default: break;
  }
}

}  // namespace ms
