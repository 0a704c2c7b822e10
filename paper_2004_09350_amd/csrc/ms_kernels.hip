// ms_kernels.hip -- the operator kernels and their host-side launchers.
//
// Every operator decodes its inputs in registers and writes its output directly in
// the requested format (the paper's on-the-fly de/re-compression, section 3.2, with
// the input side at register granularity and the output side at block granularity,
// section 4.2).  Kernels use persistent workgroups; workgroup s owns a contiguous
// segment of 512-value chunks.
//
// Operators with a data-dependent output count (select, semi-join, intersect) run
// in two phases: the predicate phase writes one bit per input row plus a count per
// segment; the emit phase derives each segment's output offset from the counts,
// turns set bits back into positions (or values) and packs complete 512-blocks
// from LDS.  An output block whose values come from several segments is gathered
// in a global staging array and packed by the segment that completes it.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ms_device.h"
#include "ms_kernels.h"

namespace ms {


// Segment s of G over C chunks.
__device__ __forceinline__ void segment(unsigned long long C, unsigned s, unsigned G, unsigned long long &cb,
                                        unsigned long long &ce) {
  cb = C * s / G;
  ce = C * (s + 1) / G;
}

// Workgroup reductions (256 threads).
__device__ __forceinline__ unsigned long long wg_add64(unsigned long long x, unsigned long long *sh) {
  x = wave_add64(x);
  const unsigned w = threadIdx.x >> 6;
  __syncthreads();
  if (lane_id() == 0) sh[w] = x;
  __syncthreads();
  unsigned long long t = 0;
  for (int i = 0; i < kWaves; i++) t += sh[i];
  __syncthreads();
  return t;
}
__device__ __forceinline__ unsigned wg_or(unsigned x, unsigned *sh) {
  x = wave_or(x);
  const unsigned w = threadIdx.x >> 6;
  __syncthreads();
  if (lane_id() == 0) sh[w] = x;
  __syncthreads();
  unsigned t = 0;
  for (int i = 0; i < kWaves; i++) t |= sh[i];
  __syncthreads();
  return t;
}

// Arrive at the end of a kernel; returns true in every thread of the last workgroup.
__device__ __forceinline__ bool fin_arrive(unsigned slot, unsigned G) {
  __shared__ unsigned s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(&g_ring[slot], 1u);
    s_last = (prev == G - 1) ? 1u : 0u;
    if (s_last) atomicExch(&g_ring[slot], 0u);
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) __threadfence();
  return last;
}

// ---------------------------------------------------------------------------------------------
// Output side.
struct OutCol {
  ColView c;
  unsigned W;                       // static BP packing width (provisional for auto)
  unsigned long long n;             // output element count
  unsigned long long n_main;        // compressed main part
  unsigned long long nb;            // full 512-blocks of the DynBP family
};

__device__ __forceinline__ OutCol make_out(const ColView &c, unsigned long long n, unsigned W) {
  OutCol o;
  o.c = c;
  o.W = W;
  o.n = n;
  if (c.kind == STATIC_BP)
    o.n_main = n & ~31ull;
  else if (c.kind == DYN_BP || c.kind == DELTA_DYN_BP || c.kind == FOR_DYN_BP)
    o.n_main = n & ~511ull;
  else
    o.n_main = n;
  o.nb = o.n_main >> 9;
  return o;
}

// Encode output block k (a full 512-block of a DynBP-family column) from the wave's
// registers into its 512-word payload slot.
__device__ __forceinline__ void encode_dyn_block(const OutCol &o, unsigned long long k, const unsigned (&v)[8],
                                                 unsigned lane, unsigned *lds) {
  unsigned r[8];
  unsigned base = 0;
  if (o.c.kind == DELTA_DYN_BP) {
    const unsigned prev = __shfl_up(v[7], 1);
    base = __shfl(v[0], 0);
    r[0] = lane ? v[0] - prev : 0u;
#pragma unroll
    for (int i = 1; i < 8; i++) r[i] = v[i] - v[i - 1];
  } else if (o.c.kind == FOR_DYN_BP) {
    unsigned m = v[0];
#pragma unroll
    for (int i = 1; i < 8; i++) m = min(m, v[i]);
    base = wave_min(m);
#pragma unroll
    for (int i = 0; i < 8; i++) r[i] = v[i] - base;
  } else {
#pragma unroll
    for (int i = 0; i < 8; i++) r[i] = v[i];
  }
  unsigned orr = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) orr |= r[i];
  const unsigned W = bw(wave_or(orr));
  const unsigned long long off = k * (unsigned long long)kBlk;
  if (lane == 0) {
    o.c.widths[k] = (unsigned char)W;
    o.c.offsets[k] = (unsigned)off;
    o.c.bases[k] = base;
  }
  pack_block(W, r, lane, lds, o.c.payload + off);
}

// Encode output chunk c of a static BP column: `valid` values of the chunk are
// defined (valid = 512 except for the last chunk); values of the main part are
// packed at o.W, values past n_main go to the remainder.
__device__ __forceinline__ void encode_sbp_chunk(const OutCol &o, unsigned long long c, const unsigned (&v)[8],
                                                 unsigned lane, unsigned *lds, unsigned &or_main) {
  const unsigned long long idx0 = c * kBlk + 8ull * lane;
  const bool in_main = idx0 + 8 <= o.n_main;
  unsigned r[8];
  unsigned orr = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    r[i] = in_main ? v[i] : 0u;
    orr |= r[i];
  }
  or_main |= orr;
  if (o.W < 32 && (orr >> o.W) != 0) raise_err(E_TOO_WIDE);
  if (c * kBlk < o.n_main) {
#pragma unroll
    for (int i = 0; i < 8; i++) r[i] &= lowmask(o.W);
    pack_block(o.W, r, lane, lds, o.c.payload + c * 16ull * o.W);
  }
  if (!in_main) {
#pragma unroll
    for (int i = 0; i < 8; i++)
      if (idx0 + i < o.n && idx0 + i >= o.n_main) o.c.rem[idx0 + i - o.n_main] = v[i];
  }
}

// Write output chunk c of a count-known operator (output index = chunk position).
// Handles UNCOMPR, STATIC_BP and the DynBP family (RLE outputs take the two-phase path).
__device__ __forceinline__ void write_chunk_known(const OutCol &o, unsigned long long c, const unsigned (&v)[8],
                                                  unsigned lane, unsigned *lds, unsigned &or_all,
                                                  unsigned &or_main) {
  const unsigned long long idx0 = c * kBlk + 8ull * lane;
#pragma unroll
  for (int i = 0; i < 8; i++)
    if (idx0 + i < o.n) or_all |= v[i];
  switch (o.c.kind) {
    case UNCOMPR: {
      if (idx0 + 8 <= o.n) {
        uint4 *p = reinterpret_cast<uint4 *>(o.c.payload + idx0);
        p[0] = make_uint4(v[0], v[1], v[2], v[3]);
        p[1] = make_uint4(v[4], v[5], v[6], v[7]);
      } else {
#pragma unroll
        for (int i = 0; i < 8; i++)
          if (idx0 + i < o.n) o.c.payload[idx0 + i] = v[i];
      }
      break;
    }
    case STATIC_BP: encode_sbp_chunk(o, c, v, lane, lds, or_main); break;
    case DYN_BP:
    case DELTA_DYN_BP:
    case FOR_DYN_BP: {
      if (c < o.nb) {
        encode_dyn_block(o, c, v, lane, lds);
      } else {
#pragma unroll
        for (int i = 0; i < 8; i++)
          if (idx0 + i < o.n) o.c.rem[idx0 + i - o.n_main] = v[i];
      }
      break;
    }
    default: break;
  }
}

// Narrow a static BP payload in place from width Wf to Wt < Wf (one workgroup,
// chunk by chunk in increasing order: output chunk c only overlaps input chunks <= c).
__device__ void narrow_sbp(const ColView &c, unsigned long long n_main, unsigned Wf, unsigned Wt, unsigned *lds_all) {
  const unsigned lane = lane_id(), w = threadIdx.x >> 6;
  unsigned *lds = lds_all + w * kBlk;
  const unsigned long long C = (n_main + kBlk - 1) / kBlk;
  for (unsigned long long c0 = 0; c0 < C; c0 += kWaves) {
    const unsigned long long cc = c0 + w;
    unsigned v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (cc < C) unpack8_rt(Wf, c.payload + cc * 16ull * Wf, lane, v);
    __syncthreads();
    if (cc < C) {
      const unsigned long long idx0 = cc * kBlk + 8ull * lane;
#pragma unroll
      for (int i = 0; i < 8; i++) v[i] = (idx0 + i < n_main) ? v[i] : 0u;
      pack_block(Wt, v, lane, lds, c.payload + cc * 16ull * Wt);
    }
    __syncthreads();
  }
}

// Last-workgroup epilogue of every column-producing kernel: reduce per-workgroup
// partials {or_all, or_main}, write the header, narrow an auto-width static BP column.
__device__ void finish_column(const ColView &oc, unsigned long long n, unsigned Wp, bool auto_w,
                              const unsigned *partials, unsigned G, unsigned *lds_all) {
  __shared__ unsigned s_or[2];
  unsigned a = 0, m = 0;
  for (unsigned i = threadIdx.x; i < G; i += kWG) {
    a |= partials[2 * i];
    m |= partials[2 * i + 1];
  }
  __shared__ unsigned red[kWaves];
  a = wg_or(a, red);
  m = wg_or(m, red);
  if (threadIdx.x == 0) {
    s_or[0] = a;
    s_or[1] = m;
  }
  __syncthreads();
  unsigned W = Wp;
  if (oc.kind == STATIC_BP && auto_w) {
    const unsigned Wt = bw(s_or[1]);
    const unsigned long long n_main = n & ~31ull;
    if (Wt < Wp && n_main > 0) narrow_sbp(oc, n_main, Wp, Wt, lds_all);
    W = Wt;
  }
  if (threadIdx.x == 0) {
    oc.hdr->n = n;
    oc.hdr->or_all = s_or[0];
    oc.hdr->or_main = s_or[1];
    oc.hdr->sbp_width = (oc.kind == STATIC_BP) ? W : 0u;
    if (oc.kind != RLE) oc.hdr->runs = 0;
  }
}

// ---------------------------------------------------------------------------------------------
// Column statistics needed by later operators: OR of all values (width bound).
__global__ __launch_bounds__(kWG) void k_colstats(ColView inv, unsigned *partials, unsigned slot) {
  const InCol in = load_in(inv);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6, G = gridDim.x;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned a = 0, m = 0;
  const unsigned long long nm32 = in.n & ~31ull;
  for (unsigned long long c = cb + w; c < ce; c += kWaves) {
    unsigned v[8];
    decode_chunk(in, c, lane, v);
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      if (idx0 + i < in.n) a |= v[i];
      if (idx0 + i < nm32) m |= v[i];
    }
  }
  __shared__ unsigned red[kWaves];
  a = wg_or(a, red);
  m = wg_or(m, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = m;
  }
  if (fin_arrive(slot, G)) {
    unsigned aa = 0, mm = 0;
    for (unsigned i = threadIdx.x; i < G; i += kWG) {
      aa |= partials[2 * i];
      mm |= partials[2 * i + 1];
    }
    aa = wg_or(aa, red);
    mm = wg_or(mm, red);
    if (threadIdx.x == 0) {
      inv.hdr->or_all = aa;
      inv.hdr->or_main = mm;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Morph (and encode / decode): out = encode_fmt(decode(in)), count known.
// W_src: 0 = explicit width in out.width; 1 = auto from the input's OR of all values.
__global__ __launch_bounds__(kWG) void k_morph(ColView inv, ColView outv, unsigned auto_w, unsigned *partials,
                                               unsigned slot) {
  __shared__ unsigned lds_all[kWaves * kBlk];
  const InCol in = load_in(inv);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6, G = gridDim.x;
  unsigned Wp = outv.width;
  if (outv.kind == STATIC_BP && auto_w) Wp = bw(inv.hdr->or_all);
  const OutCol o = make_out(outv, in.n, Wp);
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned or_all = 0, or_main = 0;
  unsigned *lds = lds_all + w * kBlk;
  for (unsigned long long c = cb + w; c < ce; c += kWaves) {
    unsigned v[8];
    decode_chunk(in, c, lane, v);
    write_chunk_known(o, c, v, lane, lds, or_all, or_main);
  }
  __shared__ unsigned red[kWaves];
  or_all = wg_or(or_all, red);
  or_main = wg_or(or_main, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = or_all;
    partials[2 * blockIdx.x + 1] = or_main;
  }
  if (fin_arrive(slot, G)) finish_column(outv, in.n, Wp, auto_w != 0, partials, G, lds_all);
}

// Decode into a plain device array.
__global__ __launch_bounds__(kWG) void k_decode(ColView inv, unsigned *__restrict__ out) {
  const InCol in = load_in(inv);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6, G = gridDim.x;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  for (unsigned long long c = cb + w; c < ce; c += kWaves) {
    unsigned v[8];
    decode_chunk(in, c, lane, v);
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
    if (idx0 + 8 <= in.n) {
      uint4 *p = reinterpret_cast<uint4 *>(out + idx0);
      p[0] = make_uint4(v[0], v[1], v[2], v[3]);
      p[1] = make_uint4(v[4], v[5], v[6], v[7]);
    } else {
#pragma unroll
      for (int i = 0; i < 8; i++)
        if (idx0 + i < in.n) out[idx0 + i] = v[i];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// RLE output for count-known producers (morph, project): phase 1 counts run starts per
// segment, phase 2 writes (value, start) pairs.  `src` yields chunk values.
struct ChunkSrc {
  unsigned mode;   // 0 = decode column `a`; 1 = project: a = positions, b = data
  ColView a, b;
};

__device__ __forceinline__ unsigned long long src_n(const ChunkSrc &s) { return s.a.hdr->n; }

__device__ __forceinline__ void src_chunk(const ChunkSrc &s, const InCol &ia, const InCol &ib, unsigned long long c,
                                          unsigned lane, unsigned (&v)[8]) {
  decode_chunk(ia, c, lane, v);
  if (s.mode == 1) {
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      if (idx0 + i < ia.n) {
        const unsigned p = v[i];
        if (p < ib.n) {
          v[i] = value_at(ib, p);
        } else {
          raise_err(E_RANGE);
          v[i] = 0;
        }
      }
    }
  }
}

__device__ __forceinline__ unsigned src_value(const ChunkSrc &s, const InCol &ia, const InCol &ib,
                                              unsigned long long idx) {
  unsigned x = value_at(ia, idx);
  if (s.mode == 1) x = x < ib.n ? value_at(ib, x) : 0u;
  return x;
}

__global__ __launch_bounds__(kWG) void k_rle_count(ChunkSrc s, unsigned *seg_count) {
  const InCol ia = load_in(s.a);
  InCol ib = ia;
  if (s.mode == 1) ib = load_in(s.b);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6, G = gridDim.x;
  const unsigned long long n = ia.n;
  const unsigned long long C = (n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned cnt = 0;
  for (unsigned long long c = cb + w; c < ce; c += kWaves) {
    unsigned v[8];
    src_chunk(s, ia, ib, c, lane, v);
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
    unsigned prev = __shfl_up(v[7], 1);
    if (lane == 0) prev = (c > 0) ? src_value(s, ia, ib, c * kBlk - 1) : ~v[0];
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const unsigned pv = i ? v[i - 1] : prev;
      if (idx0 + i < n && (idx0 + i == 0 || v[i] != pv)) cnt++;
    }
  }
  __shared__ unsigned long long red[kWaves];
  const unsigned long long t = wg_add64(cnt, red);
  if (threadIdx.x == 0) seg_count[blockIdx.x] = (unsigned)t;
}

__global__ __launch_bounds__(kWG) void k_rle_emit(ChunkSrc s, ColView outv, const unsigned *seg_count,
                                                  unsigned *partials, unsigned slot) {
  __shared__ unsigned lds_all[kWaves * kBlk];
  __shared__ unsigned long long red[kWaves];
  __shared__ unsigned s_chunk_runs[kWaves];
  const InCol ia = load_in(s.a);
  InCol ib = ia;
  if (s.mode == 1) ib = load_in(s.b);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6, G = gridDim.x;
  const unsigned long long n = ia.n;
  const unsigned long long C = (n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned long long before = 0, total = 0;
  for (unsigned i = threadIdx.x; i < G; i += kWG) {
    total += seg_count[i];
    if (i < blockIdx.x) before += seg_count[i];
  }
  before = wg_add64(before, red);
  total = wg_add64(total, red);
  unsigned or_all = 0;
  // Chunks are taken in order, kWaves at a time, so run indices stay ordered.
  unsigned long long base = before;
  for (unsigned long long c0 = cb; c0 < ce; c0 += kWaves) {
    const unsigned long long c = c0 + w;
    unsigned v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned flags = 0;
    if (c < ce) {
      src_chunk(s, ia, ib, c, lane, v);
      const unsigned long long idx0 = c * kBlk + 8ull * lane;
      unsigned prev = __shfl_up(v[7], 1);
      if (lane == 0) prev = (c > 0) ? src_value(s, ia, ib, c * kBlk - 1) : ~v[0];
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const unsigned pv = i ? v[i - 1] : prev;
        if (idx0 + i < n) {
          or_all |= v[i];
          if (idx0 + i == 0 || v[i] != pv) flags |= 1u << i;
        }
      }
    }
    const unsigned cnt = __popc(flags);
    const unsigned off = wave_excl_scan(cnt, lane);
    const unsigned chunk_total = __shfl(off + cnt, 63);
    if (lane == 0) s_chunk_runs[w] = chunk_total;
    __syncthreads();
    unsigned long long my = base;
    for (unsigned j = 0; j < w; j++) my += s_chunk_runs[j];
    unsigned long long all = base;
    for (unsigned j = 0; j < kWaves; j++) all += s_chunk_runs[j];
    __syncthreads();
    if (c < ce) {
      unsigned long long r = my + off;
      const unsigned long long idx0 = c * kBlk + 8ull * lane;
#pragma unroll
      for (int i = 0; i < 8; i++) {
        if (flags & (1u << i)) {
          if (r < outv.n_cap) {
            outv.rvalues[r] = v[i];
            outv.rstarts[r] = (unsigned)(idx0 + i);
          } else {
            raise_err(E_INVALID);
          }
          r++;
        }
      }
    }
    base = all;
  }
  __shared__ unsigned redu[kWaves];
  or_all = wg_or(or_all, redu);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = or_all;
    partials[2 * blockIdx.x + 1] = 0;
  }
  if (fin_arrive(slot, G)) {
    finish_column(outv, n, 0, false, partials, G, lds_all);
    if (threadIdx.x == 0) outv.hdr->runs = total;
  }
}

// ---------------------------------------------------------------------------------------------
// Project: out_j = data[pos_j].
__global__ __launch_bounds__(kWG) void k_project(ColView posv, ColView datav, ColView outv, unsigned auto_w,
                                                 unsigned *partials, unsigned slot) {
  __shared__ unsigned lds_all[kWaves * kBlk];
  const InCol ip = load_in(posv);
  const InCol id = load_in(datav);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6, G = gridDim.x;
  unsigned Wp = outv.width;
  if (outv.kind == STATIC_BP && auto_w) Wp = bw(datav.hdr->or_all);
  const OutCol o = make_out(outv, ip.n, Wp);
  const unsigned long long C = (ip.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned or_all = 0, or_main = 0;
  unsigned *lds = lds_all + w * kBlk;
  for (unsigned long long c = cb + w; c < ce; c += kWaves) {
    unsigned v[8];
    decode_chunk(ip, c, lane, v);
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      unsigned x = 0;
      if (idx0 + i < ip.n) {
        if (v[i] < id.n)
          x = value_at(id, v[i]);
        else
          raise_err(E_RANGE);
      }
      v[i] = x;
    }
    write_chunk_known(o, c, v, lane, lds, or_all, or_main);
  }
  __shared__ unsigned red[kWaves];
  or_all = wg_or(or_all, red);
  or_main = wg_or(or_main, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = or_all;
    partials[2 * blockIdx.x + 1] = or_main;
  }
  if (fin_arrive(slot, G)) finish_column(outv, ip.n, Wp, auto_w != 0, partials, G, lds_all);
}

// ---------------------------------------------------------------------------------------------
// Compaction phase 1: predicate -> one bit per row, count and OR per segment.
// mode 0: range predicate ((v - lo) <= span) != neg, emits positions
// mode 1: bitmap predicate v < domain && bit(v), emits positions (semi-join)
// mode 2: bitmap predicate on values, emits values, checks strict increase (intersect)
__global__ __launch_bounds__(kWG) void k_pred(PredArgs a) {
  const InCol in = load_in(a.in);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6, G = gridDim.x;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  // zero the staging counters of the emit phase
  for (unsigned long long i = (unsigned long long)blockIdx.x * kWG + threadIdx.x; i < a.n_counters;
       i += (unsigned long long)G * kWG)
    a.counters[i] = 0;
  unsigned cnt = 0, orv = 0;
  for (unsigned long long c = cb + w; c < ce; c += kWaves) {
    unsigned v[8];
    decode_chunk(in, c, lane, v);
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
    unsigned mask = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      bool p;
      if (a.mode == 0) {
        p = ((v[i] - a.lo) <= a.span) != (a.neg != 0);
      } else {
        const unsigned x = v[i];
        p = (unsigned long long)x < a.domain && ((a.bitmap[x >> 5] >> (x & 31)) & 1u);
      }
      if (idx0 + i < in.n && p) mask |= 1u << i;
    }
    a.bitmask[c * 64 + lane] = (unsigned char)mask;
    cnt += __popc(mask);
    if (a.mode == 2) {
#pragma unroll
      for (int i = 0; i < 8; i++)
        if (mask & (1u << i)) orv |= v[i];
      // strictly increasing inside the chunk; chunk ends are checked by the emit phase
      const unsigned prev = __shfl_up(v[7], 1);
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const unsigned pv = i ? v[i - 1] : prev;
        if (idx0 + i < in.n && (i > 0 || lane > 0) && v[i] <= pv) raise_err(E_NOT_SORTED);
      }
      const unsigned long long last_idx = min(in.n, (c + 1) * kBlk) - 1;
      if (lane == 0) a.chunk_first[c] = v[0];
      if (idx0 <= last_idx && last_idx < idx0 + 8) a.chunk_last[c] = v[last_idx - idx0];
    } else if (mask) {
      unsigned bits = 0;
#pragma unroll
      for (int i = 0; i < 8; i++)
        if (mask & (1u << i)) bits |= (unsigned)i;
      orv |= (unsigned)idx0 | bits;
    }
  }
  __shared__ unsigned long long red[kWaves];
  __shared__ unsigned redo[kWaves];
  const unsigned long long t = wg_add64(cnt, red);
  orv = wg_or(orv, redo);
  if (threadIdx.x == 0) {
    a.seg_count[blockIdx.x] = (unsigned)t;
    a.seg_or[blockIdx.x] = orv;
  }
}

// ---------------------------------------------------------------------------------------------
// Compaction phase 2: emit.
constexpr int kEmitChunks = 8;                 // chunks per emit tile (2 per wave)
constexpr int kStage = kEmitChunks * kBlk + kBlk;

// Block structure of a compaction output: blocks of 512 over [0, Nb) where Nb = n_main
// for the DynBP family (the rest is remainder) and N for static BP (last block partial).
__device__ __forceinline__ unsigned long long blk_end(unsigned long long k, unsigned long long Nb) {
  return min((k + 1) * (unsigned long long)kBlk, Nb);
}

// Encode block k of a compaction output from v (8 per lane); `len` values valid.
__device__ __forceinline__ void encode_out_block(const OutCol &o, unsigned long long k, const unsigned (&v)[8],
                                                 unsigned lane, unsigned *lds, unsigned &or_main) {
  if (o.c.kind == STATIC_BP) {
    encode_sbp_chunk(o, k, v, lane, lds, or_main);
  } else {
    encode_dyn_block(o, k, v, lane, lds);
  }
}

__global__ __launch_bounds__(kWG) void k_emit(EmitArgs a) {
  __shared__ unsigned stage[kStage];
  __shared__ unsigned lds_all[kWaves * kBlk];
  __shared__ unsigned s_ctot[kEmitChunks];
  __shared__ unsigned long long red[kWaves];
  __shared__ unsigned redo[kWaves];
  __shared__ unsigned s_flag;
  const InCol in = load_in(a.in);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6, G = gridDim.x, seg = blockIdx.x;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, seg, G, cb, ce);

  // Offsets from the phase-1 counts.
  unsigned long long before = 0, total = 0;
  unsigned orv = 0;
  for (unsigned i = threadIdx.x; i < G; i += kWG) {
    total += a.seg_count[i];
    if (i < seg) before += a.seg_count[i];
    orv |= a.seg_or[i];
  }
  before = wg_add64(before, red);
  total = wg_add64(total, red);
  orv = wg_or(orv, redo);
  const unsigned long long O = before, N = total;
  unsigned Wp = a.out.width;
  if (a.out.kind == STATIC_BP && a.auto_w) Wp = bw(orv);
  const OutCol o = make_out(a.out, N, Wp);
  const unsigned kind = a.out.kind;
  const bool blocky = (kind == STATIC_BP || kind == DYN_BP || kind == DELTA_DYN_BP || kind == FOR_DYN_BP);
  const unsigned long long Nb = (kind == STATIC_BP) ? N : o.n_main;   // block elements are [0, Nb)

  const unsigned long long mycnt = a.seg_count[seg];
  const unsigned long long E = O + mycnt;       // end (exclusive) of this segment's outputs
  // Owned blocks: fully inside [O, E) and below Nb.
  unsigned long long A = 0, B = 0;
  if (blocky) {
    const unsigned long long Eb = min(E, Nb);
    const unsigned long long kA = (O + kBlk - 1) / kBlk;
    unsigned long long kB1;  // one past the last owned block
    if (Eb == Nb && Nb > 0)
      kB1 = (Nb + kBlk - 1) / kBlk;
    else
      kB1 = Eb / kBlk;
    if (O >= Nb || kA >= kB1) {
      A = B = (O < Nb) ? O : Nb;  // nothing owned
    } else {
      A = kA * kBlk;
      B = blk_end(kB1 - 1, Nb);
    }
  }
  // sortedness across chunk ends (intersect inputs)
  if (a.check_sorted) {
    for (unsigned long long c = cb + threadIdx.x; c < ce; c += kWG)
      if (c > 0 && a.chunk_first[c] <= a.chunk_last[c - 1]) raise_err(E_NOT_SORTED);
  }

  unsigned or_all = 0, or_main = 0;
  unsigned long long emitted = 0;   // outputs of this segment so far
  unsigned long long Lbase = A;     // global index of stage[0] (owned elements only)
  unsigned *lds = lds_all + w * kBlk;
  const unsigned long long n_main_o = o.n_main;

  for (unsigned long long t0 = cb; t0 < ce; t0 += kEmitChunks) {
    unsigned v[2][8];
    unsigned msk[2], off[2];
#pragma unroll
    for (int j = 0; j < 2; j++) {
      const unsigned lc = 2 * w + j;
      const unsigned long long c = t0 + lc;
      msk[j] = 0;
      if (c < ce) {
        msk[j] = a.bitmask[c * 64 + lane];
        if (a.emit_values) decode_chunk(in, c, lane, v[j]);
      }
      const unsigned cntl = __popc(msk[j]);
      off[j] = wave_excl_scan(cntl, lane);
      if (lane == 63) s_ctot[lc] = off[j] + cntl;
    }
    __syncthreads();
    unsigned long long tile_base = 0, tile_total = 0, cbase[2] = {0, 0};
    for (unsigned lc = 0; lc < kEmitChunks; lc++) {
      if (lc == 2 * w) cbase[0] = tile_total;
      if (lc == 2 * w + 1) cbase[1] = tile_total;
      tile_total += s_ctot[lc];
    }
    (void)tile_base;
#pragma unroll
    for (int j = 0; j < 2; j++) {
      const unsigned long long c = t0 + 2 * w + j;
      if (c >= ce || !msk[j]) continue;
      unsigned long long g = O + emitted + cbase[j] + off[j];
      const unsigned long long idx0 = c * kBlk + 8ull * lane;
#pragma unroll
      for (int i = 0; i < 8; i++) {
        if (!(msk[j] & (1u << i))) continue;
        const unsigned val = a.emit_values ? v[j][i] : (unsigned)(idx0 + i);
        or_all |= val;
        if (g < n_main_o) or_main |= val;
        if (g >= a.out.n_cap) {
          raise_err(E_INVALID);
        } else if (kind == UNCOMPR) {
          a.out.payload[g] = val;
        } else if (kind == RLE) {
          a.out.rvalues[g] = val;
          a.out.rstarts[g] = (unsigned)g;
        } else if (g >= Nb) {
          a.out.rem[g - Nb] = val;             // DynBP-family remainder
        } else if (g < A || g >= B) {
          a.stage_g[g] = val;                  // shared block
        } else {
          const unsigned long long li = g - Lbase;
          if (li < (unsigned long long)kStage)
            stage[li] = val;
          else
            raise_err(E_INVALID);
        }
        g++;
      }
    }
    __syncthreads();
    emitted += tile_total;
    if (blocky && B > A) {
      const unsigned long long have_end = min(O + emitted, B);
      if (have_end > Lbase) {
        const unsigned long long have = have_end - Lbase;
        unsigned long long nfull = have / kBlk;
        // the final block of the output may be partial and ends at B
        const bool final_partial = (have_end == B) && (have % kBlk != 0);
        const unsigned long long nenc = nfull + (final_partial ? 1 : 0);
        for (unsigned long long j = w; j < nenc; j += kWaves) {
          unsigned x[8];
#pragma unroll
          for (int i = 0; i < 8; i++) {
            const unsigned long long li = j * kBlk + 8ull * lane + i;
            x[i] = (li < have) ? stage[li] : 0u;
          }
          encode_out_block(o, (Lbase / kBlk) + j, x, lane, lds, or_main);
        }
        __syncthreads();
        const unsigned long long keep = final_partial ? 0 : have - nfull * kBlk;
        if (nfull > 0) {
          for (unsigned long long i = threadIdx.x; i < keep; i += kWG) stage[i] = stage[nfull * kBlk + i];
        }
        __syncthreads();
        Lbase += nenc * kBlk;
        if (final_partial) Lbase = B;
      }
    }
  }
  // Shared blocks: contribute counts; the contributor that completes a block packs it.
  if (blocky) {
    const unsigned long long Eb = min(E, Nb);
    unsigned long long ks[2];
    unsigned long long kc[2];
    int nk = 0;
    if (O < Nb) {
      if (A == B) {  // no owned block: [O, Eb) spans at most two blocks
        unsigned long long k = O / kBlk;
        while (k * kBlk < Eb && nk < 2) {
          const unsigned long long lo = max(O, k * kBlk), hi = min(Eb, blk_end(k, Nb));
          ks[nk] = k;
          kc[nk] = hi - lo;
          nk++;
          k++;
        }
      } else {
        if (O < A) {
          ks[nk] = O / kBlk;
          kc[nk] = A - O;
          nk++;
        }
        if (B < Eb) {
          ks[nk] = B / kBlk;
          kc[nk] = Eb - B;
          nk++;
        }
      }
    }
    for (int q = 0; q < nk; q++) {
      const unsigned long long k = ks[q];
      const unsigned long long target = blk_end(k, Nb) - k * kBlk;
      __threadfence();
      __syncthreads();
      if (threadIdx.x == 0) {
        const unsigned prev = atomicAdd(&a.counters[k], (unsigned)kc[q]);
        s_flag = (prev + kc[q] == target) ? 1u : 0u;
      }
      __syncthreads();
      if (s_flag) {
        __threadfence();
        if (w == 0) {
          unsigned x[8];
#pragma unroll
          for (int i = 0; i < 8; i++) {
            const unsigned long long li = 8ull * lane + i;
            x[i] = (li < target) ? __hip_atomic_load(&a.stage_g[k * kBlk + li], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)
                                 : 0u;
          }
          encode_out_block(o, k, x, lane, lds, or_main);
        }
      }
      __syncthreads();
    }
  }
  or_all = wg_or(or_all, redo);
  or_main = wg_or(or_main, redo);
  if (threadIdx.x == 0) {
    a.partials[2 * seg] = or_all;
    a.partials[2 * seg + 1] = or_main;
  }
  if (fin_arrive(a.slot, G)) {
    finish_column(a.out, N, Wp, a.auto_w != 0, a.partials, G, lds_all);
    if (threadIdx.x == 0) {
      if (kind == RLE) a.out.hdr->runs = N;
      a.out.hdr->sorted = 1;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Sum and group-sum.
__global__ __launch_bounds__(kWG) void k_sum(ColView inv, unsigned long long *result,
                                             unsigned long long *partials, unsigned slot) {
  const InCol in = load_in(inv);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6, G = gridDim.x;
  __shared__ unsigned long long red[kWaves];
  unsigned long long s = 0;
  if (in.kind == RLE) {
    // sum over runs: value * run length (section 2.2)
    unsigned long long rb, re;
    segment(in.runs, blockIdx.x, G, rb, re);
    for (unsigned long long r = rb + threadIdx.x; r < re; r += kWG) {
      const unsigned long long st = in.rstarts[r];
      const unsigned long long en = (r + 1 < in.runs) ? in.rstarts[r + 1] : in.n;
      s += (unsigned long long)in.rvalues[r] * (en - st);
    }
  } else {
    const unsigned long long C = (in.n + kBlk - 1) / kBlk;
    unsigned long long cb, ce;
    segment(C, blockIdx.x, G, cb, ce);
    for (unsigned long long c = cb + w; c < ce; c += kWaves) {
      unsigned v[8];
      decode_chunk(in, c, lane, v);
      const unsigned long long idx0 = c * kBlk + 8ull * lane;
      if (idx0 + 8 <= in.n) {
#pragma unroll
        for (int i = 0; i < 8; i++) s += v[i];
      } else {
#pragma unroll
        for (int i = 0; i < 8; i++)
          if (idx0 + i < in.n) s += v[i];
      }
    }
  }
  s = wg_add64(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  if (fin_arrive(slot, G)) {
    unsigned long long t = 0;
    for (unsigned i = threadIdx.x; i < G; i += kWG) t += partials[i];
    t = wg_add64(t, red);
    if (threadIdx.x == 0) *result = t;
  }
}

constexpr unsigned kMaxLdsGroups = 4096;

__global__ __launch_bounds__(kWG) void k_group_sum(ColView gv, ColView vv, unsigned G_groups,
                                                   unsigned long long *out, unsigned long long *partials,
                                                   unsigned slot) {
  __shared__ unsigned long long hist[kMaxLdsGroups];
  const InCol ig = load_in(gv);
  const InCol iv = load_in(vv);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6, G = gridDim.x;
  if (ig.n != iv.n) {
    if (blockIdx.x == 0 && threadIdx.x == 0) raise_err(E_LENGTH);
  }
  const unsigned long long n = min(ig.n, iv.n);
  const bool use_lds = G_groups <= kMaxLdsGroups;
  for (unsigned i = threadIdx.x; i < kMaxLdsGroups; i += kWG) hist[i] = 0;
  __syncthreads();
  const unsigned long long C = (n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  for (unsigned long long c = cb + w; c < ce; c += kWaves) {
    unsigned g[8], v[8];
    decode_chunk(ig, c, lane, g);
    decode_chunk(iv, c, lane, v);
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      if (idx0 + i < n) {
        if (g[i] >= G_groups) {
          raise_err(E_RANGE);
        } else if (use_lds) {
          atomicAdd(&hist[g[i]], (unsigned long long)v[i]);
        } else {
          atomicAdd(&partials[g[i]], (unsigned long long)v[i]);
        }
      }
    }
  }
  __syncthreads();
  if (use_lds) {
    for (unsigned q = threadIdx.x; q < G_groups; q += kWG)
      partials[(unsigned long long)blockIdx.x * G_groups + q] = hist[q];
  }
  if (fin_arrive(slot, G)) {
    if (use_lds) {
      for (unsigned q = threadIdx.x; q < G_groups; q += kWG) {
        unsigned long long t = 0;
        for (unsigned b = 0; b < G; b++) t += partials[(unsigned long long)b * G_groups + q];
        out[q] = t;
      }
    } else {
      for (unsigned q = threadIdx.x; q < G_groups; q += kWG) out[q] = partials[q];
    }
  }
}

__global__ void k_set_hdr(ColHdr *h, unsigned long long n, unsigned long long runs, unsigned width,
                          unsigned or_all, unsigned or_main, unsigned sorted) {
  if (threadIdx.x == 0) {
    h->n = n;
    h->runs = runs;
    h->sbp_width = width;
    h->or_all = or_all;
    h->or_main = or_main;
    h->sorted = sorted;
  }
}

__global__ void k_fill_u32(unsigned *p, unsigned long long n, unsigned v) {
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long n, unsigned long long v) {
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// Bitmap from positions: bit p of the (zeroed) bitmap for every position p.  With
// chunk_first/chunk_last set it also checks that the positions strictly increase
// (inside chunks here, across chunk ends in k_check_order).
__global__ __launch_bounds__(kWG) void k_bitmap(ColView posv, unsigned long long domain, unsigned *bitmap,
                                                unsigned *chunk_first, unsigned *chunk_last) {
  const InCol in = load_in(posv);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6, G = gridDim.x;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  for (unsigned long long c = cb + w; c < ce; c += kWaves) {
    unsigned v[8];
    decode_chunk(in, c, lane, v);
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
    if (chunk_first) {
      const unsigned prev = __shfl_up(v[7], 1);
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const unsigned pv = i ? v[i - 1] : prev;
        if (idx0 + i < in.n && (i > 0 || lane > 0) && v[i] <= pv) raise_err(E_NOT_SORTED);
      }
      const unsigned long long last_idx = min(in.n, (c + 1) * kBlk) - 1;
      if (lane == 0) chunk_first[c] = v[0];
      if (idx0 <= last_idx && last_idx < idx0 + 8) chunk_last[c] = v[last_idx - idx0];
    }
    // combine bits that land in the same word before the atomic
    unsigned cur_word = 0xFFFFFFFFu, bits = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      if (idx0 + i < in.n) {
        const unsigned p = v[i];
        if ((unsigned long long)p >= domain) {
          raise_err(E_RANGE);
        } else {
          const unsigned wd = p >> 5;
          if (wd != cur_word) {
            if (bits) atomicOr(&bitmap[cur_word], bits);
            cur_word = wd;
            bits = 0;
          }
          bits |= 1u << (p & 31);
        }
      }
    }
    if (bits) atomicOr(&bitmap[cur_word], bits);
  }
}

__global__ void k_check_order(const unsigned *chunk_first, const unsigned *chunk_last, ColView posv) {
  const unsigned long long n = posv.hdr->n;
  const unsigned long long C = (n + kBlk - 1) / kBlk;
  for (unsigned long long c = 1 + (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; c < C;
       c += (unsigned long long)gridDim.x * blockDim.x)
    if (chunk_first[c] <= chunk_last[c - 1]) raise_err(E_NOT_SORTED);
}

// Canonical copy of a DynBP-family payload: block k moves from old_off[k] to new_off[k].
__global__ __launch_bounds__(kWG) void k_shrink_payload(const unsigned *src, const unsigned *old_off,
                                                        const unsigned char *widths, const unsigned *new_off,
                                                        unsigned *dst, unsigned long long nb) {
  const unsigned lane = lane_id(), w = threadIdx.x >> 6;
  for (unsigned long long k = (unsigned long long)blockIdx.x * kWaves + w; k < nb;
       k += (unsigned long long)gridDim.x * kWaves) {
    const unsigned words = 16u * widths[k];
    const uint4 *s4 = reinterpret_cast<const uint4 *>(src + old_off[k]);
    uint4 *d4 = reinterpret_cast<uint4 *>(dst + new_off[k]);
    for (unsigned q = lane; q < words / 4; q += 64) d4[q] = s4[q];
  }
}

// ---------------------------------------------------------------------------------------------
// Host-side launchers.
static hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

unsigned read_and_clear_err(void *stream) {
  unsigned e = 0, z = 0;
  if (hipMemcpyFromSymbolAsync(&e, HIP_SYMBOL(g_err), sizeof(e), 0, hipMemcpyDeviceToHost, S(stream)) != hipSuccess ||
      hipMemcpyToSymbolAsync(HIP_SYMBOL(g_err), &z, sizeof(z), 0, hipMemcpyHostToDevice, S(stream)) != hipSuccess ||
      hipStreamSynchronize(S(stream)) != hipSuccess)
    return E_INVALID;
  return e;
}

hipError_t launch_set_hdr(ColHdr *h, unsigned long long n, unsigned long long runs, unsigned width, unsigned or_all,
                          unsigned or_main, unsigned sorted, void *s) {
  hipLaunchKernelGGL(k_set_hdr, dim3(1), dim3(64), 0, S(s), h, n, runs, width, or_all, or_main, sorted);
  return hipGetLastError();
}
hipError_t launch_colstats(const ColView &in, unsigned G, unsigned *partials, unsigned slot, void *s) {
  hipLaunchKernelGGL(k_colstats, dim3(G), dim3(kWG), 0, S(s), in, partials, slot);
  return hipGetLastError();
}
hipError_t launch_morph(const ColView &in, const ColView &out, unsigned auto_w, unsigned G, unsigned *partials,
                        unsigned slot, void *s) {
  hipLaunchKernelGGL(k_morph, dim3(G), dim3(kWG), 0, S(s), in, out, auto_w, partials, slot);
  return hipGetLastError();
}
hipError_t launch_decode(const ColView &in, unsigned *out, unsigned G, void *s) {
  hipLaunchKernelGGL(k_decode, dim3(G), dim3(kWG), 0, S(s), in, out);
  return hipGetLastError();
}
hipError_t launch_rle(unsigned mode, const ColView &a, const ColView &b, const ColView &out, unsigned G,
                      unsigned *seg_count, unsigned *partials, unsigned slot, void *s) {
  ChunkSrc src;
  src.mode = mode;
  src.a = a;
  src.b = b;
  hipLaunchKernelGGL(k_rle_count, dim3(G), dim3(kWG), 0, S(s), src, seg_count);
  hipLaunchKernelGGL(k_rle_emit, dim3(G), dim3(kWG), 0, S(s), src, out, seg_count, partials, slot);
  return hipGetLastError();
}
hipError_t launch_project(const ColView &pos, const ColView &data, const ColView &out, unsigned auto_w, unsigned G,
                          unsigned *partials, unsigned slot, void *s) {
  hipLaunchKernelGGL(k_project, dim3(G), dim3(kWG), 0, S(s), pos, data, out, auto_w, partials, slot);
  return hipGetLastError();
}
hipError_t launch_pred(const PredArgs &a, unsigned G, void *s) {
  hipLaunchKernelGGL(k_pred, dim3(G), dim3(kWG), 0, S(s), a);
  return hipGetLastError();
}
hipError_t launch_emit(const EmitArgs &a, unsigned G, void *s) {
  hipLaunchKernelGGL(k_emit, dim3(G), dim3(kWG), 0, S(s), a);
  return hipGetLastError();
}
hipError_t launch_sum(const ColView &in, unsigned long long *result, unsigned G, unsigned long long *partials,
                      unsigned slot, void *s) {
  hipLaunchKernelGGL(k_sum, dim3(G), dim3(kWG), 0, S(s), in, result, partials, slot);
  return hipGetLastError();
}
hipError_t launch_group_sum(const ColView &g, const ColView &v, unsigned groups, unsigned long long *out, unsigned G,
                            unsigned long long *partials, unsigned slot, void *s) {
  hipLaunchKernelGGL(k_group_sum, dim3(G), dim3(kWG), 0, S(s), g, v, groups, out, partials, slot);
  return hipGetLastError();
}
hipError_t launch_fill_u32(unsigned *p, unsigned long long n, unsigned v, void *s) {
  if (n == 0) return hipSuccess;
  unsigned blocks = (unsigned)std::min<unsigned long long>((n + 255) / 256, 2048ull);
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, S(s), p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long n, unsigned long long v, void *s) {
  if (n == 0) return hipSuccess;
  unsigned blocks = (unsigned)std::min<unsigned long long>((n + 255) / 256, 2048ull);
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks), dim3(256), 0, S(s), p, n, v);
  return hipGetLastError();
}
hipError_t launch_bitmap(const ColView &pos, unsigned long long domain, unsigned *bitmap, unsigned G, void *s) {
  hipLaunchKernelGGL(k_bitmap, dim3(G), dim3(kWG), 0, S(s), pos, domain, bitmap, (unsigned *)nullptr,
                     (unsigned *)nullptr);
  return hipGetLastError();
}
hipError_t launch_bitmap_checked(const ColView &pos, unsigned long long domain, unsigned *bitmap, unsigned *first,
                                 unsigned *last, unsigned G, void *s) {
  hipLaunchKernelGGL(k_bitmap, dim3(G), dim3(kWG), 0, S(s), pos, domain, bitmap, first, last);
  return hipGetLastError();
}
hipError_t launch_check_order(const unsigned *first, const unsigned *last, const ColView &pos, void *s) {
  hipLaunchKernelGGL(k_check_order, dim3(256), dim3(256), 0, S(s), first, last, pos);
  return hipGetLastError();
}
hipError_t launch_shrink_payload(const unsigned *src, const unsigned *old_off, const unsigned char *widths,
                                 const unsigned *new_off, unsigned *dst, unsigned long long nb, void *s) {
  if (nb == 0) return hipSuccess;
  unsigned blocks = (unsigned)std::min<unsigned long long>((nb + kWaves - 1) / kWaves, 4096ull);
  hipLaunchKernelGGL(k_shrink_payload, dim3(blocks), dim3(kWG), 0, S(s), src, old_off, widths, new_off, dst, nb);
  return hipGetLastError();
}

}  // namespace ms
