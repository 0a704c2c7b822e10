// ms_kernels.hip -- the operator kernels and their host-side launchers.
//
// Every operator decodes its inputs in registers and writes its output directly in
// the requested format (the paper's on-the-fly de/re-compression, section 3.2, with
// the input side at register granularity and the output side at block granularity,
// section 4.2).  Workgroup s of G owns a contiguous segment of 512-value chunks;
// its four waves walk the segment's chunks with one chunk of look-ahead.
//
// Operators with a data-dependent output count (select, semi-join, intersect) run
// in phases: the predicate phase writes one bit per input row plus a count per
// segment; the emit phase derives each segment's output offset from the counts,
// turns set bits back into positions (or values) and packs the output blocks that
// lie inside the segment from LDS; blocks shared by neighbouring segments are
// gathered in a staging array and packed by a fix-up kernel.  No kernel waits on
// another workgroup: every cross-workgroup dependency is a kernel boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

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
  const unsigned w = wave_id();
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
  const unsigned w = wave_id();
  __syncthreads();
  if (lane_id() == 0) sh[w] = x;
  __syncthreads();
  unsigned t = 0;
  for (int i = 0; i < kWaves; i++) t |= sh[i];
  __syncthreads();
  return t;
}

__device__ __forceinline__ unsigned valid_mask(unsigned long long idx0, unsigned long long n) {
  return idx0 >= n ? 0u : (idx0 + 8 <= n ? 0xFFu : ((1u << (unsigned)(n - idx0)) - 1u));
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
    const unsigned prev = lane_prev(v[7]);
    base = lane_first(v[0]);
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

// Encode output chunk c of a static BP column; values of the main part are packed at
// o.W, values past n_main go to the remainder.
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
template <unsigned OK>
__device__ __forceinline__ void write_chunk_known(const OutCol &o, unsigned long long c, const unsigned (&v)[8],
                                                  unsigned lane, unsigned *lds, unsigned &or_all,
                                                  unsigned &or_main) {
  const unsigned long long idx0 = c * kBlk + 8ull * lane;
#pragma unroll
  for (int i = 0; i < 8; i++)
    if (idx0 + i < o.n) or_all |= v[i];
  switch (OK) {
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

// ---------------------------------------------------------------------------------------------
// Finish: one workgroup after a column-producing kernel.  Reduces the per-workgroup
// {OR of all values, OR of the main part} and writes the header.
__global__ __launch_bounds__(kWG) void k_finish(FinishArgs a) {
  __shared__ unsigned red[kWaves];
  __shared__ unsigned long long s_n;
  unsigned ao = 0, mo = 0;
  for (unsigned i = threadIdx.x; i < a.G; i += kWG) {
    ao |= a.partials[2 * i];
    mo |= a.partials[2 * i + 1];
  }
  ao = wg_or(ao, red);
  mo = wg_or(mo, red);
  if (threadIdx.x == 0) s_n = a.n_src ? a.n_src->n : a.out.hdr->n;
  __syncthreads();
  const unsigned long long n = s_n;
  if (a.mode == 1) {  // statistics of an existing column
    if (threadIdx.x == 0) {
      a.out.hdr->or_all = ao;
      a.out.hdr->or_main = mo;
    }
    return;
  }
  __shared__ unsigned s_wp;
  if (threadIdx.x == 0) s_wp = (a.out.kind == STATIC_BP && a.auto_w) ? a.out.hdr->sbp_width : a.Wp;
  __syncthreads();
  const unsigned Wprov = s_wp;  // the width the producer packed at
  unsigned W = Wprov;
  if (a.out.kind == STATIC_BP && a.auto_w) W = min(bw(mo), Wprov);  // k_narrow repacked when smaller
  if (threadIdx.x == 0) {
    a.out.hdr->n = n;
    a.out.hdr->or_all = ao;
    a.out.hdr->or_main = mo;
    a.out.hdr->sbp_width = (a.out.kind == STATIC_BP) ? W : 0u;
    if (a.out.kind != RLE) a.out.hdr->runs = 0;
    a.out.hdr->sorted = a.sorted;
  }
}

// Narrowing of an auto-width static BP column whose main part needs fewer bits than
// the width it was packed at: k_narrow repacks every chunk into `tmp` at the narrow
// width, k_narrow_copy copies it back.  Both exit at once when nothing narrows.
__device__ __forceinline__ bool narrow_plan(const FinishArgs &a, unsigned long long &n_main, unsigned &Wf,
                                            unsigned &Wt, unsigned *red) {
  unsigned mo = 0;
  for (unsigned i = threadIdx.x; i < a.G; i += kWG) mo |= a.partials[2 * i + 1];
  mo = wg_or(mo, red);
  const unsigned long long n = a.n_src ? a.n_src->n : a.out.hdr->n;
  n_main = n & ~31ull;
  Wf = a.out.hdr->sbp_width;
  Wt = bw(mo);
  return Wf <= 32 && Wt < Wf && n_main > 0;
}

__global__ __launch_bounds__(kWG) void k_narrow(FinishArgs a, unsigned *tmp) {
  __shared__ __attribute__((aligned(16))) unsigned lds_all[kWaves * kBlk];
  __shared__ unsigned red[kWaves];
  unsigned long long n_main;
  unsigned Wf, Wt;
  if (!narrow_plan(a, n_main, Wf, Wt, red)) return;
  const unsigned lane = lane_id(), w = wave_id();
  unsigned *lds = lds_all + w * kBlk;
  const unsigned long long C = (n_main + kBlk - 1) / kBlk;
  for (unsigned long long c = (unsigned long long)blockIdx.x * kWaves + w; c < C;
       c += (unsigned long long)gridDim.x * kWaves) {
    unsigned v[8];
    unpack8_rt(Wf, a.out.payload + c * 16ull * Wf, lane, v);
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = (idx0 + i < n_main) ? v[i] : 0u;
    pack_block(Wt, v, lane, lds, tmp + c * 16ull * Wt);
  }
}

__global__ __launch_bounds__(kWG) void k_narrow_copy(FinishArgs a, const unsigned *tmp) {
  __shared__ unsigned red[kWaves];
  unsigned long long n_main;
  unsigned Wf, Wt;
  if (!narrow_plan(a, n_main, Wf, Wt, red)) return;
  const unsigned long long words = n_main * Wt / 32;  // n_main is a multiple of 32
  for (unsigned long long q = (unsigned long long)blockIdx.x * kWG + threadIdx.x; q < words;
       q += (unsigned long long)gridDim.x * kWG)
    a.out.payload[q] = tmp[q];
}

// ---------------------------------------------------------------------------------------------
// Column statistics needed by later operators: OR of all values (width bound).
__global__ __launch_bounds__(kWG) void k_colstats(ColView inv, unsigned *partials) {
  __shared__ __attribute__((aligned(16))) unsigned ring[kWaves * kRing * kBlk];
  __shared__ unsigned red[kWaves];
  const InCol in = load_in(inv);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned a = 0, m = 0;
  const unsigned long long nm32 = in.n & ~31ull;
  stream_chunks(in, cb, ce, w, lane, ring + w * kRing * kBlk, inv.hdr, [&](unsigned long long c, const unsigned (&v)[8]) {
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      if (idx0 + i < in.n) a |= v[i];
      if (idx0 + i < nm32) m |= v[i];
    }
  });
  a = wg_or(a, red);
  m = wg_or(m, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = m;
  }
}

// ---------------------------------------------------------------------------------------------
// Morph (and encode): out = encode_fmt(decode(in)), count known.
template <unsigned OK>
__global__ __launch_bounds__(kWG) void k_morph(ColView inv, ColView outv, unsigned auto_w, unsigned *partials) {
  __shared__ __attribute__((aligned(16))) unsigned ring[kWaves * kRing * kBlk];
  __shared__ __attribute__((aligned(16))) unsigned lds_all[kWaves * kBlk];
  __shared__ unsigned red[kWaves];
  const InCol in = load_in(inv);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x;
  unsigned Wp = outv.width;
  if (outv.kind == STATIC_BP && auto_w) Wp = bw(inv.hdr->or_all);
  const OutCol o = make_out(outv, in.n, Wp);
  if (blockIdx.x == 0 && threadIdx.x == 0) outv.hdr->sbp_width = Wp;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned or_all = 0, or_main = 0;
  unsigned *lds = lds_all + w * kBlk;
  stream_chunks(in, cb, ce, w, lane, ring + w * kRing * kBlk, inv.hdr, [&](unsigned long long c, const unsigned (&v)[8]) {
    write_chunk_known<OK>(o, c, v, lane, lds, or_all, or_main);
  });
  or_all = wg_or(or_all, red);
  or_main = wg_or(or_main, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = or_all;
    partials[2 * blockIdx.x + 1] = or_main;
  }
}

// Decode into a plain device array.
__global__ __launch_bounds__(kWG) void k_decode(ColView inv, unsigned *__restrict__ out) {
  __shared__ __attribute__((aligned(16))) unsigned ring[kWaves * kRing * kBlk];
  const InCol in = load_in(inv);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  stream_chunks(in, cb, ce, w, lane, ring + w * kRing * kBlk, inv.hdr, [&](unsigned long long c, const unsigned (&v)[8]) {
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
  });
}

// ---------------------------------------------------------------------------------------------
// Project: out_j = data[pos_j].
// Project: gather the data column at the positions streamed from posv and encode the
// values into the output format.  RLE data columns have their own kernel (their gather
// stages runs in LDS and needs its own registers).
template <unsigned OK, bool DRLE>
__device__ __forceinline__ void project_body(const ColView &posv, const ColView &datav, const ColView &outv,
                                             unsigned auto_w, unsigned *partials) {
  __shared__ __attribute__((aligned(16))) unsigned ring[kWaves * kRing * kBlk];
  __shared__ __attribute__((aligned(16))) unsigned gblk[kWaves * kBlk];
  __shared__ __attribute__((aligned(16))) unsigned lds_all[kWaves * kBlk];
  __shared__ unsigned red[kWaves];
  const InCol ip = load_in(posv);
  const InCol id = load_in(datav);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6, G = gridDim.x;  // w kept in a VGPR: SGPRs run short here
  unsigned Wp = outv.width;
  if (outv.kind == STATIC_BP && auto_w) Wp = bw(datav.hdr->or_all);
  const OutCol o = make_out(outv, ip.n, Wp);
  if (blockIdx.x == 0 && threadIdx.x == 0) outv.hdr->sbp_width = Wp;
  const unsigned long long C = (ip.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned or_all = 0, or_main = 0;
  unsigned *lds = lds_all + w * kBlk;
  bool bad = false;
  stream_chunks(ip, cb, ce, w, lane, ring + w * kRing * kBlk, posv.hdr, [&](unsigned long long c, const unsigned (&pv)[8]) {
    unsigned v[8];
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = pv[i];
    const unsigned valid = valid_mask(c * kBlk + 8ull * lane, ip.n);
    if constexpr (DRLE)
      gather8_rle(id, v, valid, bad, lane, gblk + w * kBlk, lds);
    else
      gather8<false>(id, v, valid, bad, lane, gblk + w * kBlk, lds);
    write_chunk_known<OK>(o, c, v, lane, lds, or_all, or_main);
  });
  if (bad) raise_err(E_RANGE);
  or_all = wg_or(or_all, red);
  or_main = wg_or(or_main, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = or_all;
    partials[2 * blockIdx.x + 1] = or_main;
  }
}

template <unsigned OK>
__global__ __launch_bounds__(kWG, 3) void k_project(ColView posv, ColView datav, ColView outv, unsigned auto_w,
                                                 unsigned *partials) {
  project_body<OK, false>(posv, datav, outv, auto_w, partials);
}
template <unsigned OK>
__global__ __launch_bounds__(kWG) void k_project_rle(ColView posv, ColView datav, ColView outv, unsigned auto_w,
                                                     unsigned *partials) {
  project_body<OK, true>(posv, datav, outv, auto_w, partials);
}

// ---------------------------------------------------------------------------------------------
// RLE output for count-known producers (morph, project): phase 1 counts run starts per
// segment, phase 2 writes (value, start) pairs.
struct ChunkSrc {
  unsigned mode;   // 0 = decode column `a`; 1 = project: a = positions, b = data
  ColView a, b;
};

__device__ __forceinline__ unsigned src_value(const ChunkSrc &s, const InCol &ia, const InCol &ib,
                                              unsigned long long idx) {
  unsigned x = value_at(ia, idx);
  if (s.mode == 1) x = x < ib.n ? value_at(ib, x) : 0u;
  return x;
}

// Both RLE phases walk the segment's chunks in lockstep, kWaves at a time, so that the
// value before a chunk (needed to see whether the chunk starts a new run) is the last
// value of the neighbouring wave's chunk, passed through LDS.  The emit phase stages a
// chunk's runs in LDS and writes them with coalesced stores.  MODE 0 decodes column a
// (morph), MODE 1 gathers b at the positions in a (project).
template <unsigned MODE, bool EMIT>
__device__ __forceinline__ void rle_walk(const ChunkSrc &s, const ColView &outv, const unsigned *seg_count,
                                         unsigned *seg_out, unsigned *partials) {
  __shared__ __attribute__((aligned(16))) unsigned lds_all[kWaves * kBlk];
  __shared__ __attribute__((aligned(16))) unsigned gblk[MODE == 1 ? kWaves * kBlk : 1];
  __shared__ unsigned gstage[MODE == 1 ? kWaves * kBlk : 1];
  __shared__ unsigned rstage[EMIT ? 2 * kWaves * kBlk : 1];
  __shared__ unsigned long long red[kWaves];
  __shared__ unsigned s_chunk_runs[kWaves];
  __shared__ unsigned s_last[kWaves];
  __shared__ unsigned s_first_prev;
  __shared__ unsigned redu[kWaves];
  const InCol ia = load_in(s.a);
  InCol ib = ia;
  if (MODE == 1) ib = load_in(s.b);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x;
  const unsigned long long n = ia.n;
  const unsigned long long C = (n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned long long base = 0, total = 0;
  if (EMIT) {
    unsigned long long before = 0;
    for (unsigned i = threadIdx.x; i < G; i += kWG) {
      total += seg_count[i];
      if (i < blockIdx.x) before += seg_count[i];
    }
    base = wg_add64(before, red);
    total = wg_add64(total, red);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      outv.hdr->n = n;
      outv.hdr->runs = total;
    }
  }
  if (threadIdx.x == 0 && cb > 0 && cb < ce) s_first_prev = src_value(s, ia, ib, cb * kBlk - 1);
  __syncthreads();
  unsigned carry = s_first_prev;  // last value before the current round's first chunk
  unsigned or_all = 0, cnt_all = 0;
  bool bad = false;
  unsigned *lds = lds_all + w * kBlk;
  unsigned *rv = rstage + (EMIT ? 2 * w * kBlk : 0), *rs = rv + kBlk;
  Raw cur;
  if (cb + w < ce) cur = issue_chunk(ia, cb + w, lane);
  for (unsigned long long c0 = cb; c0 < ce; c0 += kWaves) {
    const unsigned long long c = c0 + w;
    Raw nxt;
    if (c + kWaves < ce) nxt = issue_chunk(ia, c + kWaves, lane);
    unsigned v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (c < ce) {
      finish_chunk(ia, cur, c, lane, lds, v);
      if (MODE == 1)
        gather8(ib, v, valid_mask(c * kBlk + 8ull * lane, n), bad, lane, gblk + w * kBlk, gstage + w * kBlk);
      if (lane == 63) s_last[w] = v[7];
    }
    __syncthreads();
    const unsigned before_chunk = (w > 0) ? s_last[w - 1] : carry;
    const unsigned next_carry = s_last[kWaves - 1];
    unsigned flags = 0;
    if (c < ce) {
      const unsigned long long idx0 = c * kBlk + 8ull * lane;
      unsigned prev = lane_prev(v[7]);
      if (lane == 0) prev = before_chunk;
      const unsigned valid = valid_mask(idx0, n);
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const unsigned pv = i ? v[i - 1] : prev;
        if ((valid >> i) & 1u) {
          or_all |= v[i];
          if (idx0 + i == 0 || v[i] != pv) flags |= 1u << i;
        }
      }
    }
    const unsigned cnt = __popc(flags);
    cnt_all += cnt;
    if (EMIT) {
      const unsigned off = wave_excl_scan(cnt, lane);
      const unsigned chunk_total = lane_last(off + cnt);
      if (lane == 0) s_chunk_runs[w] = chunk_total;
      __syncthreads();
      unsigned long long my = base;
      for (unsigned j = 0; j < w; j++) my += s_chunk_runs[j];
      unsigned long long all = base;
      for (unsigned j = 0; j < kWaves; j++) all += s_chunk_runs[j];
      if (c < ce) {
        const unsigned idx0 = (unsigned)(c * kBlk) + 8u * lane;
        unsigned q = off;
#pragma unroll
        for (int i = 0; i < 8; i++) {
          if (flags & (1u << i)) {
            rv[q] = v[i];
            rs[q] = idx0 + i;
            q++;
          }
        }
        wave_sync();
        if (my + chunk_total <= outv.n_cap) {
          for (unsigned t = lane; t < chunk_total; t += 64) {  // consecutive lanes, consecutive runs
            outv.rvalues[my + t] = rv[t];
            outv.rstarts[my + t] = rs[t];
          }
        } else if (chunk_total > 0) {
          raise_err(E_INVALID);
        }
        wave_sync();
      }
      base = all;
    }
    __syncthreads();  // s_last and s_chunk_runs are rewritten next round
    carry = next_carry;
    cur = nxt;
  }
  if (bad) raise_err(E_RANGE);
  if (EMIT) {
    or_all = wg_or(or_all, redu);
    if (threadIdx.x == 0) {
      partials[2 * blockIdx.x] = or_all;
      partials[2 * blockIdx.x + 1] = 0;
    }
  } else {
    const unsigned long long t = wg_add64(cnt_all, red);
    if (threadIdx.x == 0) seg_out[blockIdx.x] = (unsigned)t;
  }
}

__global__ __launch_bounds__(kWG) void k_rle_count(ChunkSrc s, unsigned *seg_count) {
  rle_walk<0, false>(s, s.a, nullptr, seg_count, nullptr);
}
__global__ __launch_bounds__(kWG) void k_rle_emit(ChunkSrc s, ColView outv, const unsigned *seg_count,
                                                  unsigned *partials) {
  rle_walk<0, true>(s, outv, seg_count, nullptr, partials);
}
__global__ __launch_bounds__(kWG) void k_rle_count_proj(ChunkSrc s, unsigned *seg_count) {
  rle_walk<1, false>(s, s.a, nullptr, seg_count, nullptr);
}
__global__ __launch_bounds__(kWG) void k_rle_emit_proj(ChunkSrc s, ColView outv, const unsigned *seg_count,
                                                       unsigned *partials) {
  rle_walk<1, true>(s, outv, seg_count, nullptr, partials);
}

// ---------------------------------------------------------------------------------------------
// Compaction phase 1: predicate -> one bit per row, count and OR per segment.
// mode 0: range predicate ((v - lo) <= span) != neg, emits positions
// mode 1: bitmap predicate v < domain && bit(v), emits positions (semi-join)
// mode 2: bitmap predicate on values, emits values, checks strict increase (intersect)
template <unsigned MODE>
__global__ __launch_bounds__(kWG) void k_pred(PredArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned ring[kWaves * kRing * kBlk];
  __shared__ unsigned long long red[kWaves];
  __shared__ unsigned redo[kWaves];
  const InCol in = load_in(a.in);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned cnt = 0, orv = 0;
  bool unsorted = false;
  constexpr unsigned mode = MODE;
  const unsigned lo = a.lo, span = a.span;
  const bool neg = a.neg != 0;
  const unsigned long long domain = a.domain;
  const unsigned *bitmap = a.bitmap;
  unsigned char *bitmask = a.bitmask;
  unsigned *chunk_first = a.chunk_first, *chunk_last = a.chunk_last;
  stream_chunks(in, cb, ce, w, lane, ring + w * kRing * kBlk, a.in.hdr, [&](unsigned long long c, const unsigned (&v)[8]) {
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
    const unsigned valid = valid_mask(idx0, in.n);
    unsigned mask = 0;
    if constexpr (mode == 0) {
#pragma unroll
      for (int i = 0; i < 8; i++)
        if (((v[i] - lo) <= span) != neg) mask |= 1u << i;
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
    a.seg_count[blockIdx.x] = (unsigned)t;
    a.seg_or[blockIdx.x] = orv;
  }
}

// ---------------------------------------------------------------------------------------------
// Compaction phase 2: emit.

// Output blocks of a compaction: 512-blocks over [0, Nb), Nb = n_main for the DynBP
// family (the rest is remainder) and N for static BP (the last block may be partial).
__device__ __forceinline__ unsigned long long blk_end(unsigned long long k, unsigned long long Nb) {
  return min((k + 1) * (unsigned long long)kBlk, Nb);
}

__device__ __forceinline__ void encode_out_block(const OutCol &o, unsigned long long k, const unsigned (&v)[8],
                                                 unsigned lane, unsigned *lds, unsigned &or_main) {
  if (o.c.kind == STATIC_BP)
    encode_sbp_chunk(o, k, v, lane, lds, or_main);
  else
    encode_dyn_block(o, k, v, lane, lds);
}

// Offsets of segment `seg` from the phase-1 counts: O (outputs before it), N (total),
// OR of every segment's OR.
__device__ __forceinline__ void seg_offsets(const unsigned *seg_count, const unsigned *seg_or, unsigned seg,
                                            unsigned G, unsigned long long &O, unsigned long long &N, unsigned &orv,
                                            unsigned long long *red, unsigned *redo) {
  unsigned long long before = 0, total = 0;
  unsigned o = 0;
  for (unsigned i = threadIdx.x; i < G; i += kWG) {
    total += seg_count[i];
    if (i < seg) before += seg_count[i];
    o |= seg_or[i];
  }
  O = wg_add64(before, red);
  N = wg_add64(total, red);
  orv = wg_or(o, redo);
}

__device__ __forceinline__ unsigned emit_width(const EmitArgs &a, unsigned orv) {
  return (a.out.kind == STATIC_BP && a.auto_w) ? bw(orv) : a.out.width;
}

// Output range of wave w of workgroup seg: [Ow, Ew), from the workgroup's offset O and
// the per-wave counts.
__device__ __forceinline__ void wave_range(const unsigned *cnt4, unsigned w, unsigned long long O,
                                           unsigned long long &Ow, unsigned long long &Ew) {
  unsigned long long before = 0;
  for (unsigned j = 0; j < w; j++) before += cnt4[j];
  Ow = O + before;
  Ew = Ow + cnt4[w];
}

// Blocks owned by the output range [Ow, Ew): those lying entirely inside it and below Nb
// are packed by the wave from LDS; the other block elements go to the global stage.
__device__ __forceinline__ void owned_blocks(unsigned long long Ow, unsigned long long Ew, unsigned long long Nb,
                                             unsigned long long &A, unsigned long long &B) {
  const unsigned long long Eb = min(Ew, Nb);
  const unsigned long long kA = (Ow + kBlk - 1) / kBlk;
  const unsigned long long kB1 = (Eb == Nb && Nb > 0) ? (Nb + kBlk - 1) / kBlk : Eb / kBlk;
  if (Ow >= Nb || kA >= kB1) {
    A = B = (Ow < Nb) ? Ow : Nb;
  } else {
    A = kA * kBlk;
    B = blk_end(kB1 - 1, Nb);
  }
}

// Compaction phase 2.  Each wave emits a contiguous quarter of its workgroup's chunks on
// its own: it counts its outputs from the bitmask, learns its output offset through
// LDS, then streams its chunks, appending outputs of owned blocks to a two-block ring
// in its LDS and packing each block as soon as it is complete.  No workgroup barrier
// inside the loop.
constexpr unsigned kEmitRing = 2 * kBlk;

__global__ __launch_bounds__(kWG) void k_emit(EmitArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned ring_all[kWaves * kEmitRing];
  __shared__ __attribute__((aligned(16))) unsigned lds_all[kWaves * kBlk];
  __shared__ unsigned s_wcnt[kWaves];
  __shared__ unsigned long long red[kWaves];
  __shared__ unsigned redo[kWaves];
  const InCol in = load_in(a.in);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x, seg = blockIdx.x;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, seg, G, cb, ce);
  unsigned long long O, N;
  unsigned orv;
  seg_offsets(a.seg_count, a.seg_or, seg, G, O, N, orv, red, redo);
  const unsigned Wp = emit_width(a, orv);
  const OutCol o = make_out(a.out, N, Wp);
  const unsigned kind = a.out.kind;
  const bool blocky = (kind == STATIC_BP || kind == DYN_BP || kind == DELTA_DYN_BP || kind == FOR_DYN_BP);
  const unsigned long long Nb = (kind == STATIC_BP) ? N : o.n_main;   // block elements are [0, Nb)
  if (seg == 0 && threadIdx.x == 0) {
    a.out.hdr->n = N;
    a.out.hdr->or_all = orv;
    a.out.hdr->sorted = 1;
    a.out.hdr->runs = (kind == RLE) ? N : 0ull;
    a.out.hdr->sbp_width = (kind == STATIC_BP) ? Wp : 0u;
  }
  if (a.check_sorted) {
    for (unsigned long long c = cb + threadIdx.x; c < ce; c += kWG)
      if (c > 0 && a.chunk_first[c] <= a.chunk_last[c - 1]) raise_err(E_NOT_SORTED);
  }
  // this wave's chunks and its output count
  const unsigned long long nseg = ce - cb;
  const unsigned long long cw0 = cb + nseg * w / kWaves, cw1 = cb + nseg * (w + 1) / kWaves;
  unsigned cnt = 0;
#pragma unroll 4
  for (unsigned long long c = cw0; c < cw1; c++) cnt += __popc((unsigned)a.bitmask[c * 64 + lane]);
  cnt = wave_add(cnt);
  if (lane == 0) s_wcnt[w] = cnt;
  __syncthreads();
  unsigned long long Ow, Ew;
  wave_range(s_wcnt, w, O, Ow, Ew);
  if (lane == 0) {  // the fix phase reads each wave's output range from here
    a.wave_count[2ull * (kWaves * seg + w)] = (unsigned)Ow;
    a.wave_count[2ull * (kWaves * seg + w) + 1] = cnt;
  }
  unsigned long long A = 0, B = 0;
  if (blocky) owned_blocks(Ow, Ew, Nb, A, B);

  unsigned or_main = 0;
  const bool cap_ok = N <= a.out.n_cap;
  // Output indices are below 2^32 (columns hold fewer than 2^32 values): 32-bit from here.
  const unsigned n_main_o = (unsigned)o.n_main, A32 = (unsigned)A, B32 = (unsigned)B, Nb32 = (unsigned)Nb;
  const unsigned cap32 = (unsigned)min(a.out.n_cap, 0xFFFFFFFFull);
  unsigned *ring = ring_all + w * kEmitRing;
  unsigned *lds = lds_all + w * kBlk;
  unsigned g_done = A32;          // owned outputs below g_done are packed
  unsigned g = (unsigned)Ow;      // next output index of this wave
  const unsigned char *bm = a.bitmask + lane;
  // bitmask bytes four chunks ahead
  unsigned q0 = (cw0 < cw1) ? bm[cw0 * 64] : 0u;
  unsigned q1 = (cw0 + 1 < cw1) ? bm[(cw0 + 1) * 64] : 0u;
  unsigned q2 = (cw0 + 2 < cw1) ? bm[(cw0 + 2) * 64] : 0u;
  unsigned q3 = (cw0 + 3 < cw1) ? bm[(cw0 + 3) * 64] : 0u;
  for (unsigned long long c = cw0; c < cw1; c++) {
    unsigned m = q0;
    q0 = q1;
    q1 = q2;
    q2 = q3;
    q3 = (c + 4 < cw1) ? bm[(c + 4) * 64] : 0u;
    unsigned v[8];
    if (a.emit_values) decode_chunk(in, c, lane, v);
    const unsigned cntl = __popc(m);
    const unsigned off = wave_excl_scan(cntl, lane);
    const unsigned tot = lane_last(off + cntl);
    const unsigned idx0 = (unsigned)(c * kBlk) + 8u * lane;
    unsigned gl = g + off;   // this lane's first output
    const unsigned gend = gl + cntl;
    if (blocky) {
      if (cap_ok && gend <= n_main_o && gl >= A32 && gend <= B32) {
        // owned, staged block elements: append to the ring
        unsigned k = gl - A32, orl = 0;
        while (m) {
          const unsigned i = __ffs(m) - 1;
          m &= m - 1;
          const unsigned val = a.emit_values ? select8(v, i) : idx0 + i;
          ring[k & (kEmitRing - 1)] = val;
          orl |= val;
          k++;
        }
        or_main |= orl;
      }
    } else if (cap_ok && tot > 0) {
      // uncompressed and RLE outputs: stage the chunk's outputs, then coalesced stores
      unsigned k = off, orl = 0;
      while (m) {
        const unsigned i = __ffs(m) - 1;
        m &= m - 1;
        const unsigned val = a.emit_values ? select8(v, i) : idx0 + i;
        lds[k++] = val;
        orl |= val;
      }
      or_main |= orl;  // n_main = N for these kinds
      wave_sync();
      if (kind == UNCOMPR) {
        for (unsigned t = lane; t < tot; t += 64) a.out.payload[g + t] = lds[t];
      } else {
        for (unsigned t = lane; t < tot; t += 64) {
          a.out.rvalues[g + t] = lds[t];
          a.out.rstarts[g + t] = g + t;
        }
      }
      wave_sync();
    }
    while (m) {  // elements outside the fast paths
      const unsigned i = __ffs(m) - 1;
      m &= m - 1;
      const unsigned val = a.emit_values ? select8(v, i) : idx0 + i;
      if (gl < n_main_o) or_main |= val;
      if (gl >= cap32) {
        raise_err(E_INVALID);
      } else if (kind == UNCOMPR) {
        a.out.payload[gl] = val;
      } else if (kind == RLE) {
        a.out.rvalues[gl] = val;
        a.out.rstarts[gl] = gl;
      } else if (gl >= Nb32) {
        a.out.rem[gl - Nb32] = val;           // DynBP-family remainder
      } else if (gl < A32 || gl >= B32) {
        a.stage_g[gl] = val;                  // block shared with a neighbouring wave
      } else {
        ring[(gl - A32) & (kEmitRing - 1)] = val;
      }
      gl++;
    }
    g += tot;
    if (blocky && B32 > A32) {
      wave_sync();
      // pack every owned block that is now complete (the last block of the output may be partial)
      const unsigned have_end = min(g, B32);
      while (g_done < have_end) {
        const unsigned bend = (unsigned)blk_end(g_done / kBlk, Nb);
        if (bend > have_end) break;
        const unsigned len = bend - g_done;
        const unsigned *src = ring + ((g_done - A32) & (kEmitRing - 1));
        unsigned x[8];
        const unsigned l0 = 8u * lane;
        if (l0 + 8 <= len) {  // two 16-byte reads: no bank conflicts between lanes
          const uint4 *s4 = reinterpret_cast<const uint4 *>(src + l0);
          const uint4 p = s4[0], q = s4[1];
          x[0] = p.x; x[1] = p.y; x[2] = p.z; x[3] = p.w;
          x[4] = q.x; x[5] = q.y; x[6] = q.z; x[7] = q.w;
        } else {
#pragma unroll
          for (int i = 0; i < 8; i++) x[i] = (l0 + i < len) ? src[l0 + i] : 0u;
        }
        encode_out_block(o, g_done / kBlk, x, lane, lds, or_main);
        g_done = bend;
      }
      wave_sync();
    }
  }
  or_main = wg_or(or_main, redo);
  if (threadIdx.x == 0) {
    a.partials[2 * seg] = orv;
    a.partials[2 * seg + 1] = or_main;
  }
}

// Compaction phase 3 (block formats): a block that started before a wave's output range
// is packed from the global stage by the wave whose range holds its last element.
__global__ __launch_bounds__(kWG) void k_emit_fix(EmitArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned lds_all[kWaves * kBlk];
  const unsigned lane = lane_id(), w = wave_id(), seg = blockIdx.x;
  // the emit phase recorded the output count and width in the header, and each wave's range
  const unsigned long long N = a.out.hdr->n;
  const unsigned Wp = (a.out.kind == STATIC_BP) ? a.out.hdr->sbp_width : a.out.width;
  const OutCol o = make_out(a.out, N, Wp);
  const unsigned long long Nb = (a.out.kind == STATIC_BP) ? N : o.n_main;
  const unsigned long long Ow = a.wave_count[2ull * (kWaves * seg + w)];
  const unsigned long long Ew = Ow + a.wave_count[2ull * (kWaves * seg + w) + 1];
  const unsigned long long Eb = min(Ew, Nb);
  if (Eb <= Ow) return;  // no block element in this wave's range
  // Only the block holding the range's first output can have started before it; it is
  // packed here when it also ends inside the range.
  const unsigned long long k = Ow / kBlk;
  const unsigned long long end = blk_end(k, Nb);
  if (k * kBlk == Ow || end > Eb) return;
  const unsigned long long len = end - k * kBlk;
  unsigned x[8];
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const unsigned long long li = 8ull * lane + i;
    x[i] = (li < len) ? a.stage_g[k * kBlk + li] : 0u;
  }
  unsigned om = 0;
  encode_out_block(o, k, x, lane, lds_all + w * kBlk, om);
}

// ---------------------------------------------------------------------------------------------
// Sum and group-sum.
__global__ __launch_bounds__(kWG) void k_sum(ColView inv, unsigned long long *partials) {
  __shared__ __attribute__((aligned(16))) unsigned ring[kWaves * kRing * kBlk];
  __shared__ unsigned long long red[kWaves];
  const InCol in = load_in(inv);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x;
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
    stream_chunks(in, cb, ce, w, lane, ring + w * kRing * kBlk, inv.hdr, [&](unsigned long long c, const unsigned (&v)[8]) {
      const unsigned valid = valid_mask(c * kBlk + 8ull * lane, in.n);
      unsigned long long t = 0;
#pragma unroll
      for (int i = 0; i < 8; i++) t += ((valid >> i) & 1u) ? v[i] : 0u;
      s += t;
    });
  }
  s = wg_add64(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kWG) void k_sum_finish(const unsigned long long *partials, unsigned G,
                                                    unsigned long long *result) {
  __shared__ unsigned long long red[kWaves];
  unsigned long long t = 0;
  for (unsigned i = threadIdx.x; i < G; i += kWG) t += partials[i];
  t = wg_add64(t, red);
  if (threadIdx.x == 0) *result = t;
}

constexpr unsigned kMaxLdsGroups = 4096;

__global__ __launch_bounds__(kWG) void k_group_sum(ColView gv, ColView vv, unsigned G_groups,
                                                   unsigned long long *partials) {
  __shared__ unsigned long long hist[kMaxLdsGroups];
  __shared__ __attribute__((aligned(16))) unsigned lds_all[2 * kWaves * kBlk];
  const InCol ig = load_in(gv);
  const InCol iv = load_in(vv);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x;
  if (ig.n != iv.n && blockIdx.x == 0 && threadIdx.x == 0) raise_err(E_LENGTH);
  const unsigned long long n = min(ig.n, iv.n);
  const bool use_lds = G_groups <= kMaxLdsGroups;
  for (unsigned i = threadIdx.x; i < kMaxLdsGroups; i += kWG) hist[i] = 0;
  __syncthreads();
  const unsigned long long C = (n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned *ldg = lds_all + w * kBlk, *ldv = lds_all + (kWaves + w) * kBlk;
  bool bad = false;
  unsigned long long c = cb + w;
  if (c < ce) {
    Raw rg = issue_chunk(ig, c, lane), rv = issue_chunk(iv, c, lane);
    while (true) {
      const unsigned long long cn = c + kWaves;
      const bool more = cn < ce;
      Raw ng, nv;
      if (more) {
        ng = issue_chunk(ig, cn, lane);
        nv = issue_chunk(iv, cn, lane);
      }
      unsigned g[8], v[8];
      finish_chunk(ig, rg, c, lane, ldg, g);
      finish_chunk(iv, rv, c, lane, ldv, v);
      const unsigned valid = valid_mask(c * kBlk + 8ull * lane, n);
#pragma unroll
      for (int i = 0; i < 8; i++) {
        if ((valid >> i) & 1u) {
          if (g[i] >= G_groups)
            bad = true;
          else if (use_lds)
            atomicAdd(&hist[g[i]], (unsigned long long)v[i]);
          else
            atomicAdd(&partials[g[i]], (unsigned long long)v[i]);
        }
      }
      if (!more) break;
      rg = ng;
      rv = nv;
      c = cn;
    }
  }
  if (bad) raise_err(E_RANGE);
  __syncthreads();
  if (use_lds) {
    for (unsigned q = threadIdx.x; q < G_groups; q += kWG)
      partials[(unsigned long long)blockIdx.x * G_groups + q] = hist[q];
  }
}

__global__ void k_group_sum_finish(const unsigned long long *partials, unsigned G, unsigned G_groups, unsigned lds,
                                   unsigned long long *out) {
  const unsigned q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= G_groups) return;
  if (!lds) {
    out[q] = partials[q];
    return;
  }
  unsigned long long t = 0;
  for (unsigned b = 0; b < G; b++) t += partials[(unsigned long long)b * G_groups + q];
  out[q] = t;
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
  __shared__ __attribute__((aligned(16))) unsigned ring[kWaves * kRing * kBlk];
  const InCol in = load_in(posv);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  bool bad_range = false, bad_order = false;
  stream_chunks(in, cb, ce, w, lane, ring + w * kRing * kBlk, posv.hdr, [&](unsigned long long c, const unsigned (&v)[8]) {
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
    const unsigned valid = valid_mask(idx0, in.n);
    if (chunk_first) {
      const unsigned prev = lane_prev(v[7]);
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const unsigned pv = i ? v[i - 1] : prev;
        if (((valid >> i) & 1u) && (i > 0 || lane > 0) && v[i] <= pv) bad_order = true;
      }
      const unsigned long long last_idx = min(in.n, (c + 1) * kBlk) - 1;
      if (lane == 0) chunk_first[c] = v[0];
      if (idx0 <= last_idx && last_idx < idx0 + 8) chunk_last[c] = select8(v, (unsigned)(last_idx - idx0));
    }
    // combine bits that land in the same word before the atomic
    unsigned cur_word = 0xFFFFFFFFu, bits = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      if ((valid >> i) & 1u) {
        const unsigned p = v[i];
        if ((unsigned long long)p >= domain) {
          bad_range = true;
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
  });
  if (bad_range) raise_err(E_RANGE);
  if (bad_order) raise_err(E_NOT_SORTED);
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
  const unsigned lane = lane_id(), w = wave_id();
  for (unsigned long long k = (unsigned long long)blockIdx.x * kWaves + w; k < nb;
       k += (unsigned long long)gridDim.x * kWaves) {
    const unsigned words = 16u * widths[k];
    const uint4 *s4 = reinterpret_cast<const uint4 *>(src + old_off[k]);
    uint4 *d4 = reinterpret_cast<uint4 *>(dst + new_off[k]);
    for (unsigned q = lane; q < words / 4; q += 64) d4[q] = s4[q];
  }
}

#include "ms_stats.inc"
#include "ms_mlp.inc"

// Per-launch timing: when enabled, every launch is bracketed by two events on its stream.
namespace {
struct ProfRec {
  const char *name;
  hipEvent_t a, b;
};
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_ev_pool;
std::mutex g_prof_mu;
bool g_prof_on = false;
thread_local bool t_prof_suspended = false;

hipEvent_t ev_get() {
  if (!g_ev_pool.empty()) {
    hipEvent_t e = g_ev_pool.back();
    g_ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  ProfRec r{nullptr, nullptr, nullptr};
  hipStream_t s;
  ProfScope(const char *name, void *stream) : s(reinterpret_cast<hipStream_t>(stream)) {
    if (!g_prof_on || t_prof_suspended) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    r.name = name;
    r.a = ev_get();
    r.b = ev_get();
    if (r.a) (void)hipEventRecord(r.a, s);
  }
  ~ProfScope() {
    if (!r.name) return;
    if (r.b) (void)hipEventRecord(r.b, s);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.push_back(r);
  }
};
}  // namespace

void prof_enable(bool on) { g_prof_on = on; }
void prof_suspend(bool on) { t_prof_suspended = on; }
size_t prof_count() {
  std::lock_guard<std::mutex> g(g_prof_mu);
  return g_prof.size();
}
// name and duration (ms) of record i; the caller synchronises first.
bool prof_get(size_t i, const char **name, float *ms) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (i >= g_prof.size()) return false;
  *name = g_prof[i].name;
  *ms = 0.f;
  if (g_prof[i].a && g_prof[i].b) (void)hipEventElapsedTime(ms, g_prof[i].a, g_prof[i].b);
  return true;
}
void prof_reset() {
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (auto &r : g_prof) {
    if (r.a) g_ev_pool.push_back(r.a);
    if (r.b) g_ev_pool.push_back(r.b);
  }
  g_prof.clear();
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

#define MS_LAUNCH(kern, grid, block, stream, ...)                                 \
  do {                                                                            \
    ProfScope ps_(#kern, stream);                                                 \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, S(stream), __VA_ARGS__); \
  } while (0)

hipError_t launch_set_hdr(ColHdr *h, unsigned long long n, unsigned long long runs, unsigned width, unsigned or_all,
                          unsigned or_main, unsigned sorted, void *s) {
  MS_LAUNCH(k_set_hdr, 1, 64, s, h, n, runs, width, or_all, or_main, sorted);
  return hipGetLastError();
}
hipError_t launch_finish(const FinishArgs &a, void *s) {
  MS_LAUNCH(k_finish, 1, kWG, s, a);
  return hipGetLastError();
}
hipError_t launch_narrow(const FinishArgs &a, unsigned *tmp, unsigned G, void *s) {
  MS_LAUNCH(k_narrow, G, kWG, s, a, tmp);
  MS_LAUNCH(k_narrow_copy, G, kWG, s, a, tmp);
  return hipGetLastError();
}
hipError_t launch_colstats(const ColView &in, unsigned G, unsigned *partials, void *s) {
  MS_LAUNCH(k_colstats, G, kWG, s, in, partials);
  FinishArgs f{};
  f.out = in;
  f.n_src = in.hdr;
  f.partials = partials;
  f.G = G;
  f.mode = 1;
  MS_LAUNCH(k_finish, 1, kWG, s, f);
  return hipGetLastError();
}
#define MS_BY_OUT_KIND(K, LAUNCH)                  \
  switch (K) {                                     \
    case UNCOMPR: LAUNCH(UNCOMPR); break;          \
    case STATIC_BP: LAUNCH(STATIC_BP); break;      \
    case DYN_BP: LAUNCH(DYN_BP); break;            \
    case DELTA_DYN_BP: LAUNCH(DELTA_DYN_BP); break; \
    case FOR_DYN_BP: LAUNCH(FOR_DYN_BP); break;    \
    default: return hipErrorInvalidValue;          \
  }

hipError_t launch_morph(const ColView &in, const ColView &out, unsigned auto_w, unsigned G, unsigned *partials,
                        void *s) {
#define MS_L(K) MS_LAUNCH(k_morph<K>, G, kWG, s, in, out, auto_w, partials)
  MS_BY_OUT_KIND(out.kind, MS_L)
#undef MS_L
  return hipGetLastError();
}
hipError_t launch_decode(const ColView &in, unsigned *out, unsigned G, void *s) {
  MS_LAUNCH(k_decode, G, kWG, s, in, out);
  return hipGetLastError();
}
hipError_t launch_rle(unsigned mode, const ColView &a, const ColView &b, const ColView &out, unsigned G,
                      unsigned *seg_count, unsigned *partials, void *s) {
  ChunkSrc src;
  src.mode = mode;
  src.a = a;
  src.b = b;
  if (mode == 0) {
    MS_LAUNCH(k_rle_count, G, kWG, s, src, seg_count);
    MS_LAUNCH(k_rle_emit, G, kWG, s, src, out, seg_count, partials);
  } else {
    MS_LAUNCH(k_rle_count_proj, G, kWG, s, src, seg_count);
    MS_LAUNCH(k_rle_emit_proj, G, kWG, s, src, out, seg_count, partials);
  }
  return hipGetLastError();
}
hipError_t launch_project(const ColView &pos, const ColView &data, const ColView &out, unsigned auto_w, unsigned G,
                          unsigned *partials, void *s) {
  if (data.kind == RLE) {
#define MS_L(K) MS_LAUNCH(k_project_rle<K>, G, kWG, s, pos, data, out, auto_w, partials)
    MS_BY_OUT_KIND(out.kind, MS_L)
#undef MS_L
  } else {
#define MS_L(K) MS_LAUNCH(k_project<K>, G, kWG, s, pos, data, out, auto_w, partials)
    MS_BY_OUT_KIND(out.kind, MS_L)
#undef MS_L
  }
  return hipGetLastError();
}
hipError_t launch_pred(const PredArgs &a, unsigned G, void *s) {
  if (a.mode == 0)
    MS_LAUNCH(k_pred<0>, G, kWG, s, a);
  else if (a.mode == 1)
    MS_LAUNCH(k_pred<1>, G, kWG, s, a);
  else
    MS_LAUNCH(k_pred<2>, G, kWG, s, a);
  return hipGetLastError();
}
hipError_t launch_emit(const EmitArgs &a, unsigned G, void *s) {
  MS_LAUNCH(k_emit, G, kWG, s, a);
  const unsigned k = a.out.kind;
  if (k == STATIC_BP || k == DYN_BP || k == DELTA_DYN_BP || k == FOR_DYN_BP) MS_LAUNCH(k_emit_fix, G, kWG, s, a);
  return hipGetLastError();
}
hipError_t launch_sum(const ColView &in, unsigned long long *result, unsigned G, unsigned long long *partials,
                      void *s) {
  MS_LAUNCH(k_sum, G, kWG, s, in, partials);
  MS_LAUNCH(k_sum_finish, 1, kWG, s, partials, G, result);
  return hipGetLastError();
}
hipError_t launch_group_sum(const ColView &g, const ColView &v, unsigned groups, unsigned long long *out, unsigned G,
                            unsigned long long *partials, void *s) {
  MS_LAUNCH(k_group_sum, G, kWG, s, g, v, groups, partials);
  const unsigned lds = groups <= kMaxLdsGroups ? 1u : 0u;
  MS_LAUNCH(k_group_sum_finish, (groups + 255) / 256, 256, s, partials, G, groups, lds, out);
  return hipGetLastError();
}
hipError_t launch_fill_u32(unsigned *p, unsigned long long n, unsigned v, void *s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<unsigned long long>((n + 255) / 256, 2048ull);
  MS_LAUNCH(k_fill_u32, blocks, 256, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long n, unsigned long long v, void *s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<unsigned long long>((n + 255) / 256, 2048ull);
  MS_LAUNCH(k_fill_u64, blocks, 256, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_bitmap(const ColView &pos, unsigned long long domain, unsigned *bitmap, unsigned G, void *s) {
  MS_LAUNCH(k_bitmap, G, kWG, s, pos, domain, bitmap, (unsigned *)nullptr, (unsigned *)nullptr);
  return hipGetLastError();
}
hipError_t launch_bitmap_checked(const ColView &pos, unsigned long long domain, unsigned *bitmap, unsigned *first,
                                 unsigned *last, unsigned G, void *s) {
  MS_LAUNCH(k_bitmap, G, kWG, s, pos, domain, bitmap, first, last);
  return hipGetLastError();
}
hipError_t launch_check_order(const unsigned *first, const unsigned *last, const ColView &pos, void *s) {
  MS_LAUNCH(k_check_order, 256, 256, s, first, last, pos);
  return hipGetLastError();
}
hipError_t launch_shrink_payload(const unsigned *src, const unsigned *old_off, const unsigned char *widths,
                                 const unsigned *new_off, unsigned *dst, unsigned long long nb, void *s) {
  if (nb == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<unsigned long long>((nb + kWaves - 1) / kWaves, 4096ull);
  MS_LAUNCH(k_shrink_payload, blocks, kWG, s, src, old_off, widths, new_off, dst, nb);
  return hipGetLastError();
}

hipError_t launch_footprints(const ColView &in, unsigned G, unsigned long long *part, unsigned *first, unsigned *last,
                             unsigned long long *bpart, unsigned G2, unsigned long long *out6, void *s) {
  FpArgs a{in, part, first, last};
  MS_LAUNCH(k_footprints, G, kWG, s, a);
  MS_LAUNCH(k_chunk_changes, G2, kWG, s, first, last, in, bpart);
  MS_LAUNCH(k_footprints_finish, 1, kWG, s, part, G, bpart, G2, in, out6);
  return hipGetLastError();
}
size_t stats_scratch_bytes() { return sizeof(StatChunk) * kStatChunks; }
hipError_t launch_stats(const ColView &in, void *chunks, float *feat, void *s) {
  StatChunk *c = static_cast<StatChunk *>(chunks);
  MS_LAUNCH(k_stats_chunk, kStatChunks, 64, s, in, c);
  MS_LAUNCH(k_stats_finish, 1, kWG, s, in, c, feat);
  return hipGetLastError();
}
unsigned mlp_nparam() { return kNParam; }
hipError_t launch_mlp_forward(const float *params, const float *x, unsigned n, float *y, unsigned *pick, void *s) {
  if (n == 0) return hipSuccess;
  MS_LAUNCH(k_mlp_forward, (n + 63) / 64, 64, s, params, x, n, y, pick);
  return hipGetLastError();
}
unsigned mlp_grad_workgroups(unsigned n) { return (n + kGradSamples - 1) / kGradSamples; }
hipError_t launch_mlp_grad(const float *params, const float *x, const float *t, unsigned n, float *gpart,
                           float *lpart, float *grad, float *loss, void *s) {
  const unsigned nwg = mlp_grad_workgroups(n);
  MS_LAUNCH(k_mlp_grad, nwg, kWG, s, params, x, t, n, gpart, lpart);
  MS_LAUNCH(k_mlp_grad_reduce, (kNParam + kWG - 1) / kWG, kWG, s, gpart, lpart, nwg, grad, loss);
  return hipGetLastError();
}
hipError_t launch_adam(float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps, float c1,
                       float c2, void *s) {
  MS_LAUNCH(k_adam, (kNParam + kWG - 1) / kWG, kWG, s, p, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace ms
