// ms_kernels.hip -- the operator kernels and their host-side launchers.
//
// Every operator decodes its inputs in registers and writes its output directly in
// the requested format (the paper's on-the-fly de/re-compression, section 3.2, with
// the input side at register granularity and the output side at block granularity,
// section 4.2).  Workgroup s of G owns a contiguous segment of 512-value chunks;
// its four waves stream the segment's chunks with several chunks of look-ahead.
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

#include "ms_kcommon.h"
#include "ms_launch.h"

namespace ms {

// ---------------------------------------------------------------------------------------------
// Finish: one workgroup after a column-producing kernel.  Reduces the per-workgroup
// {OR of all values, OR of the main part} and writes the header.
__device__ __forceinline__ void finish_body(const FinishArgs &a) {
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

__global__ __launch_bounds__(kWG) void k_finish(FinishArgs a) { finish_body(a); }
__global__ __launch_bounds__(kWG) void k_finish_batch(const FinishArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const FinishArgs &a, unsigned, unsigned) { finish_body(a); });
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

__device__ __forceinline__ void narrow_body(const FinishArgs &a, unsigned *tmp, const unsigned seg, const unsigned G) {
  __shared__ __attribute__((aligned(16))) unsigned lds_all[kWaves * kBlk];
  __shared__ unsigned red[kWaves];
  unsigned long long n_main;
  unsigned Wf, Wt;
  if (!narrow_plan(a, n_main, Wf, Wt, red)) return;
  const unsigned lane = lane_id(), w = wave_id();
  unsigned *lds = lds_all + w * kBlk;
  const unsigned long long C = (n_main + kBlk - 1) / kBlk;
  for (unsigned long long c = (unsigned long long)seg * kWaves + w; c < C; c += (unsigned long long)G * kWaves) {
    unsigned v[8];
    unpack8_rt(Wf, a.out.payload + c * 16ull * Wf, lane, v);
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = (idx0 + i < n_main) ? v[i] : 0u;
    pack_block(Wt, v, lane, lds, tmp + c * 16ull * Wt);
  }
}

__device__ __forceinline__ void narrow_copy_body(const FinishArgs &a, const unsigned *tmp, const unsigned seg,
                                                 const unsigned G) {
  __shared__ unsigned red[kWaves];
  unsigned long long n_main;
  unsigned Wf, Wt;
  if (!narrow_plan(a, n_main, Wf, Wt, red)) return;
  const unsigned long long words = n_main * Wt / 32;  // n_main is a multiple of 32
  for (unsigned long long q = (unsigned long long)seg * kWG + threadIdx.x; q < words; q += (unsigned long long)G * kWG)
    a.out.payload[q] = tmp[q];
}

__global__ __launch_bounds__(kWG) void k_narrow(FinishArgs a, unsigned *tmp) { narrow_body(a, tmp, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kWG) void k_narrow_copy(FinishArgs a, const unsigned *tmp) {
  narrow_copy_body(a, tmp, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kWG) void k_narrow_batch(const NarrowArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const NarrowArgs &a, unsigned seg, unsigned G) { narrow_body(a.f, a.tmp, seg, G); });
}
__global__ __launch_bounds__(kWG) void k_narrow_copy_batch(const NarrowArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const NarrowArgs &a, unsigned seg, unsigned G) { narrow_copy_body(a.f, a.tmp, seg, G); });
}

// ---------------------------------------------------------------------------------------------
// Column statistics needed by later operators: OR of all values (width bound).
__global__ __launch_bounds__(kWG) void k_colstats(ColView inv, unsigned *partials) {
  extern __shared__ __attribute__((aligned(16))) unsigned ring[];  // ring_shm() bytes
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

// Decode into a plain device array.
__global__ __launch_bounds__(kWG) void k_decode(ColView inv, unsigned *__restrict__ out) {
  extern __shared__ __attribute__((aligned(16))) unsigned ring[];  // ring_shm() bytes
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

// Both RLE phases give each wave a contiguous quarter of its workgroup's segment and
// walk it in order, so the value before a chunk (needed to see whether the chunk starts
// a new run) is the last value of the wave's previous chunk; only the wave's first
// chunk looks one value back in the column.  The count phase records each wave's run
// count (wave_count, kWaves per workgroup); the emit phase takes its offset from those,
// stages a chunk's runs in LDS and writes them with coalesced stores.  MODE 0 decodes
// column a (morph), MODE 1 gathers b at the positions in a (project).
// LDS: the run staging of RLE input (rle_ring_words(), only when column a is RLE) is
// dynamic, so that the other inputs keep the occupancy of the smaller static buffers.
constexpr unsigned kRleRingWords = kWaves * kRing * kBlk;
template <unsigned MODE, bool DRLE, bool EMIT>
__device__ __forceinline__ void rle_walk(const ChunkSrc &s, const ColView &outv, const unsigned *wave_count,
                                         unsigned *wave_out, unsigned *partials) {
  extern __shared__ __attribute__((aligned(16))) unsigned ring[];
  __shared__ __attribute__((aligned(16))) unsigned gblk[MODE == 1 ? kWaves * kBlk : 1];
  __shared__ __attribute__((aligned(16))) unsigned gstage[MODE == 1 ? kWaves * kBlk : 1];
  __shared__ __attribute__((aligned(16))) unsigned rstage[EMIT ? 2 * kWaves * kBlk : 1];
  __shared__ unsigned long long red[kWaves];
  __shared__ unsigned redu[kWaves];
  const InCol ia = load_in(s.a);
  InCol ib = ia;
  if (MODE == 1) ib = load_in(s.b);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x;
  const unsigned long long n = ia.n;
  const unsigned long long C = (n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  const unsigned long long nseg = ce - cb;
  const unsigned long long cw0 = cb + nseg * w / kWaves, cw1 = cb + nseg * (w + 1) / kWaves;
  // output offset of this wave's runs
  unsigned long long g = 0;
  if (EMIT) {
    unsigned long long before = 0, total = 0;
    const unsigned me = kWaves * blockIdx.x + w;
    for (unsigned i = threadIdx.x; i < kWaves * G; i += kWG) {
      const unsigned x = wave_count[i];
      total += x;
      before += (i < kWaves * blockIdx.x) ? x : 0u;
    }
    before = wg_add64(before, red);
    total = wg_add64(total, red);
    g = before;
    for (unsigned j = kWaves * blockIdx.x; j < me; j++) g += wave_count[j];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      outv.hdr->n = n;
      outv.hdr->runs = total;
    }
  }
  // the value before the wave's first chunk
  unsigned carry = 0;
  if (cw0 > 0 && cw0 < cw1) carry = uni(src_value(s, ia, ib, cw0 * kBlk - 1));
  unsigned or_all = 0, cnt_all = 0;
  bool bad = false;
  unsigned *rv = rstage + (EMIT ? 2 * w * kBlk : 0), *rs = rv + kBlk;
  stream_range(ia, cw0, cw1, lane, ring + w * kRing * kBlk, [&](unsigned long long c, const unsigned (&pv)[8]) {
    unsigned v[8];
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = pv[i];
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
    const unsigned valid = chunk_valid(c, lane, n);
    if (MODE == 1) {
      if constexpr (DRLE)
        gather8_rle(ib, v, valid, bad, lane, gblk + w * kBlk, gstage + w * kBlk);
      else
        gather8<false>(ib, v, valid, bad, lane, gblk + w * kBlk, gstage + w * kBlk);
    }
    unsigned prev = lane_prev(v[7]);
    if (lane == 0) prev = carry;
    unsigned flags = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const unsigned q = i ? v[i - 1] : prev;
      if ((valid >> i) & 1u) {
        or_all |= v[i];
        if (idx0 + i == 0 || v[i] != q) flags |= 1u << i;
      }
    }
    carry = lane_last(v[7]);  // full chunks only are followed by another chunk
    const unsigned cnt = __popc(flags);
    cnt_all += cnt;
    if (EMIT) {
      const unsigned off = wave_excl_scan(cnt, lane);
      const unsigned chunk_total = lane_last(off + cnt);
      if (chunk_total > 0) {
        const unsigned i0 = (unsigned)idx0;
        unsigned q = off;
#pragma unroll
        for (int i = 0; i < 8; i++) {
          if (flags & (1u << i)) {
            rv[q] = v[i];
            rs[q] = i0 + i;
            q++;
          }
        }
        wave_sync();
        if (g + chunk_total <= outv.n_cap) {
          for (unsigned t = lane; t < chunk_total; t += 64) {  // consecutive lanes, consecutive runs
            outv.rvalues[g + t] = rv[t];
            outv.rstarts[g + t] = rs[t];
          }
        } else {
          raise_err(E_INVALID);
        }
        wave_sync();
        g += chunk_total;
      }
    }
  });
  if (bad) raise_err(E_RANGE);
  if (EMIT) {
    or_all = wg_or(or_all, redu);
    if (threadIdx.x == 0) {
      partials[2 * blockIdx.x] = or_all;
      partials[2 * blockIdx.x + 1] = 0;
    }
  } else {
    const unsigned t = wave_add(cnt_all);
    if (lane == 0) wave_out[kWaves * blockIdx.x + w] = t;
  }
}

__global__ __launch_bounds__(kWG) void k_rle_count(ChunkSrc s, unsigned *wave_count) {
  rle_walk<0, false, false>(s, s.a, nullptr, wave_count, nullptr);
}
__global__ __launch_bounds__(kWG) void k_rle_emit(ChunkSrc s, ColView outv, const unsigned *wave_count,
                                                  unsigned *partials) {
  rle_walk<0, false, true>(s, outv, wave_count, nullptr, partials);
}
template <bool DRLE>
__global__ __launch_bounds__(kWG) void k_rle_count_proj(ChunkSrc s, unsigned *wave_count) {
  rle_walk<1, DRLE, false>(s, s.a, nullptr, wave_count, nullptr);
}
template <bool DRLE>
__global__ __launch_bounds__(kWG) void k_rle_emit_proj(ChunkSrc s, ColView outv, const unsigned *wave_count,
                                                       unsigned *partials) {
  rle_walk<1, DRLE, true>(s, outv, wave_count, nullptr, partials);
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
// LDS, then streams its chunks, appending outputs of owned blocks to a four-block ring
// in its LDS and packing each block as soon as it is complete, in the block's own ring
// slot (uncompressed and RLE outputs are staged in the ring).  No workgroup barrier
// inside the loop.
constexpr unsigned kEmitRing = 4 * kBlk;
constexpr unsigned kEmitUnitMax = kEmitRing - kBlk;   // outputs of one unit: fewer than a block wait in the ring
constexpr unsigned kEmitRingStride = kEmitRing + 64;  // the ring, then one spare word per lane

// VALS: the chunk's values are emitted (intersect), else its row positions (select, semi-join).
template <bool VALS>
__device__ __forceinline__ void emit_body(const EmitArgs &a, const unsigned seg, const unsigned G) {
  __shared__ __attribute__((aligned(16))) unsigned ring_all[kWaves * kEmitRingStride];
  __shared__ unsigned s_wcnt[kWaves];
  __shared__ unsigned long long red[kWaves];
  __shared__ unsigned redo[kWaves];
  const unsigned lane = lane_id(), w = wave_id();
  const unsigned long long C = (uni(a.in.hdr->n) + kBlk - 1) / kBlk;  // the phase-1 input's chunks
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
  // The bitmask is a bitmap in row order (byte b covers rows 8b .. 8b+7), so lane l's
  // eight bytes at chunk c cover rows 512c + 64l .. +63: eight chunks per wave load.
  const unsigned long long *bm64 = reinterpret_cast<const unsigned long long *>(a.bitmask);
  unsigned cnt = 0;
  {
    unsigned long long c = cw0;
    for (; c + 64 <= cw1; c += 64) {  // eight loads in flight
      unsigned long long x[8];
#pragma unroll
      for (int j = 0; j < 8; j++) x[j] = bm64[(c + 8 * j) * 8 + lane];
#pragma unroll
      for (int j = 0; j < 8; j++) cnt += __popcll(x[j]);
    }
    for (; c + 8 <= cw1; c += 8) cnt += __popcll(bm64[c * 8 + lane]);
    for (; c < cw1; c++) cnt += __popc((unsigned)a.bitmask[c * 64 + lane]);
  }
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
  unsigned *ring = ring_all + w * kEmitRingStride;
  // The value path (units of one chunk: at most 512 outputs) keeps its ring in the lower
  // half and decodes in the upper half.
  constexpr unsigned ring_mask = VALS ? kEmitRing / 2 - 1 : kEmitRing - 1;
  unsigned g_done = A32;          // owned outputs below g_done are packed
  unsigned g = (unsigned)Ow;      // next output index of this wave
  // OR of the positions written by the row-plane fast path, kept as the OR of the planes'
  // first rows and of their words (wave-uniform): the OR of base + j over the set bits j of
  // a word is base | (OR of those j), and the OR of the j distributes over words.
  unsigned or_base = 0;
  unsigned long long or_words = 0;

  // One output element outside the fast paths: output index gl, value val.
  auto store_one = [&](unsigned gl, unsigned val) {
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
      ring[(gl - A32) & ring_mask] = val;
    }
  };
  // Pack every owned block that is complete below output g (the last block of the output
  // may be partial).
  auto pack_ready = [&]() {
    if (!blocky || B32 <= A32) return;
    const unsigned have_end = min(g, B32);
    if (g_done >= have_end || (unsigned)blk_end(g_done / kBlk, Nb) > have_end) return;
    wave_sync();
    while (g_done < have_end) {
      const unsigned bend = (unsigned)blk_end(g_done / kBlk, Nb);
      if (bend > have_end) break;
      const unsigned len = bend - g_done;
      unsigned *src = ring + ((g_done - A32) & ring_mask);
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
      wave_sync();  // the block is in registers: its ring slot becomes the packing buffer
      encode_out_block(o, g_done / kBlk, x, lane, src, or_main);
      g_done = bend;
    }
    wave_sync();
  };

  // Emit one unit: lane bits m (bit i = value i, which is pos0 + i, or v[i] when the
  // chunk's values are emitted) in row order across the lanes; at most kEmitUnitMax
  // outputs.  A chunk's unit has eight bits per lane (unsigned), a group's 64 (unsigned
  // long long, walked as two 32-bit halves: cheaper bit scans and clears).
  auto emit_unit = [&](auto m, unsigned pos0, const unsigned (&v)[8], bool vals) {
    constexpr bool BYTE = sizeof(m) == 4;
    auto value = [&](unsigned i) { return vals ? select8(v, i) : pos0 + i; };
    auto lowest = [](auto x) -> unsigned {
      if constexpr (sizeof(x) == 4) return (unsigned)__ffs(x) - 1u;
      else return (unsigned)__ffsll(x) - 1u;
    };
    // stage a lane's set bits at dst[k + (set bits below)]: unrolled for eight bits,
    // else a loop over the set bits; returns the OR of the values
    auto scatter = [&](auto &dst_at, unsigned k) -> unsigned {
      unsigned orl = 0;
      if constexpr (BYTE) {
#pragma unroll
        for (unsigned i = 0; i < 8; i++) {
          if ((m >> i) & 1u) {
            const unsigned val = value(i);
            dst_at(k + __popc(m & ((1u << i) - 1u))) = val;
            orl |= val;
          }
        }
        m = 0;
      } else {
        unsigned h32 = (unsigned)m;
        while (h32) {
          const unsigned val = value((unsigned)__ffs(h32) - 1u);
          h32 &= h32 - 1u;
          dst_at(k++) = val;
          orl |= val;
        }
        h32 = (unsigned)(m >> 32);
        while (h32) {
          const unsigned val = value((unsigned)__ffs(h32) + 31u);
          h32 &= h32 - 1u;
          dst_at(k++) = val;
          orl |= val;
        }
        m = 0;
      }
      return orl;
    };
    const unsigned cntl = BYTE ? (unsigned)__popc(m) : (unsigned)__popcll(m);
    const unsigned off = wave_excl_scan(cntl, lane);
    const unsigned tot = lane_last(off + cntl);
    unsigned gl = g + off;  // this lane's first output
    const unsigned gend = gl + cntl;
    if (blocky) {
      if (cap_ok && gend <= n_main_o && gl >= A32 && gend <= B32) {
        // owned, staged block elements: append to the ring
        auto at = [&](unsigned k) -> unsigned & { return ring[k & ring_mask]; };
        or_main |= scatter(at, gl - A32);
      }
    } else if (cap_ok && tot > 0) {
      // uncompressed and RLE outputs: stage the unit's outputs, then coalesced stores
      auto at = [&](unsigned k) -> unsigned & { return ring[k]; };
      or_main |= scatter(at, off);  // n_main = N for these kinds
      wave_sync();
      if (kind == UNCOMPR) {
        for (unsigned t = lane; t < tot; t += 64) a.out.payload[g + t] = ring[t];
      } else {
        for (unsigned t = lane; t < tot; t += 64) {
          a.out.rvalues[g + t] = ring[t];
          a.out.rstarts[g + t] = g + t;
        }
      }
      wave_sync();
    }
    while (m) {  // elements outside the fast paths
      const unsigned i = lowest(m);
      m &= m - 1;
      store_one(gl++, value(i));
    }
    g += tot;
    pack_ready();
  };

  // Emit the positions of one row plane per step: a 64-row word wd of the bitmask (rows
  // base .. base + 63) is spread over the lanes, lane l taking row base + l, and each
  // selected lane finds its output slot by counting the set bits below it.  No per-lane
  // loop, so the cost per plane does not depend on how its rows are selected.  nz: the
  // lanes of m whose word has a set bit, each such lane's word being one plane; tot: the
  // step's output count.  The checks that place outputs are made once per step where the
  // whole step lies in one region (owned blocks, or an uncompressed / RLE output), else
  // per element.
  auto emit_planes = [&](unsigned long long m, unsigned long long nz, unsigned row0, unsigned tot) {
    const unsigned ge = g + tot;
    if (!cap_ok || (blocky && (g < A32 || ge > B32 || ge > n_main_o))) {
      while (nz) {  // element by element
        const unsigned i = (unsigned)__ffsll((long long)nz) - 1u;
        nz &= nz - 1;
        const unsigned lo = __builtin_amdgcn_readlane((unsigned)m, i);
        const unsigned hi = __builtin_amdgcn_readlane((unsigned)(m >> 32), i);
        const unsigned long long wd = ((unsigned long long)hi << 32) | lo;
        if ((wd >> lane) & 1ull) store_one(lanes_below(wd, g), row0 + 64u * i + lane);
        g += (unsigned)__popcll(wd);
        pack_ready();
      }
      return;
    }
    if (blocky) {
      // owned block elements: selected lanes write the ring, the others their spare word;
      // a block is packed as soon as it is complete, so at most 575 outputs wait in the ring
      unsigned k = g - A32;  // ring index of the next output, before wrapping
      unsigned next_end = (unsigned)blk_end(g_done / kBlk, Nb) - A32;
      while (nz) {
        const unsigned i = (unsigned)__ffsll((long long)nz) - 1u;
        nz &= nz - 1;
        const unsigned lo = __builtin_amdgcn_readlane((unsigned)m, i);
        const unsigned hi = __builtin_amdgcn_readlane((unsigned)(m >> 32), i);
        const unsigned long long wd = ((unsigned long long)hi << 32) | lo;
        const unsigned base = row0 + 64u * i;
        ring[lane_bit_select(wd, lanes_below(wd, k) & (kEmitRing - 1), kEmitRing + lane)] = base + lane;
        or_base |= base;
        or_words = uni(or_words | wd);
        k += (unsigned)__popcll(wd);
        if (k >= next_end) {
          g = A32 + k;
          pack_ready();
          next_end = (unsigned)blk_end(g_done / kBlk, Nb) - A32;
        }
      }
      g = ge;
      return;
    }
    // uncompressed or RLE output: the selected lanes store directly
    while (nz) {
      const unsigned i = (unsigned)__ffsll((long long)nz) - 1u;
      nz &= nz - 1;
      const unsigned lo = __builtin_amdgcn_readlane((unsigned)m, i);
      const unsigned hi = __builtin_amdgcn_readlane((unsigned)(m >> 32), i);
      const unsigned long long wd = ((unsigned long long)hi << 32) | lo;
      const unsigned base = row0 + 64u * i;
      if (lane_bit_select(wd, 1u, 0u)) {
        const unsigned gl = lanes_below(wd, g);
        if (kind == UNCOMPR) {
          a.out.payload[gl] = base + lane;
        } else {
          a.out.rvalues[gl] = base + lane;
          a.out.rstarts[gl] = gl;
        }
      }
      or_base |= base;
      or_words = uni(or_words | wd);
      g += (unsigned)__popcll(wd);
    }
  };

  const unsigned char *bm = a.bitmask + lane;
  const unsigned novals[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if constexpr (!VALS) {
    // positions, eight chunks (4096 rows, lane l's word holding rows 64l .. 64l + 63) per
    // step, loaded three steps ahead (lanes past the wave's chunks read nothing and hold 0).
    auto load_group = [&](unsigned long long cg) -> unsigned long long {
      return (cg + (lane >> 3) < cw1) ? bm64[cg * 8 + lane] : 0ull;
    };
    unsigned long long c = cw0;
    unsigned long long q0 = load_group(c), q1 = load_group(c + 8), q2 = load_group(c + 16);
    for (; c < cw1; c += 8) {
      const unsigned long long m = q0;
      q0 = q1;
      q1 = q2;
      q2 = load_group(c + 24);
      const unsigned long long nz = __ballot(m != 0ull);
      if (nz == 0ull) continue;
      const unsigned pc = (unsigned)__popcll(m);
      const unsigned row0 = (unsigned)(c * kBlk);
      const unsigned pos0 = row0 + 64u * lane;
      // Costs in cycles of a CU per step, measured on 1e8-row selections: the per-lane
      // loop about 25 per round (as many rounds as the fullest lane has set bits) plus 100;
      // a plane about 48, being one serial chain; chunk by chunk about 250 per chunk.
      // Planes pay where selected rows cluster, leaving most 64-row words empty.
      constexpr unsigned kChunkCost = 250;
      const unsigned tot = wave_add(pc), planes_cost = 48u * (unsigned)__popcll(nz);
      bool whole = false;  // the whole step as one unit of the per-lane loop
      if (tot <= kEmitUnitMax) {
        const unsigned loop_cost = 25u * wave_max(pc) + 100u;
        whole = loop_cost <= planes_cost && loop_cost <= 8u * kChunkCost;
      }
      if (!whole && planes_cost < 8u * kChunkCost) {
        emit_planes(m, nz, row0, tot);
        continue;
      }
      // else the two halves of four chunks (lanes 0..31, 32..63), each by the per-lane loop
      // where that is cheaper, else chunk by chunk with one byte per lane (byte lane & 7 of
      // lane 8k + lane / 8's word); or the whole step as one unit
      const unsigned t_lo = whole ? tot : wave_add(lane < 32 ? pc : 0u), t_hi = tot - t_lo;
      for (unsigned h = 0; h < (whole ? 1u : 2u); h++) {
        const unsigned th = h ? t_hi : t_lo;
        if (th == 0) continue;
        // (the fullest of 32 lanes holds about th / 32 + 2.5 sqrt(th / 32) set bits, at
        // least th / 24 for th <= 768: no reduction where that already costs more)
        if (whole || (th <= kEmitUnitMax && 25u * (th / 24u) + 100u <= 4u * kChunkCost &&
                      25u * wave_max((lane >> 5) == h ? pc : 0u) + 100u <= 4u * kChunkCost)) {
          emit_unit(whole || (lane >> 5) == h ? m : 0ull, pos0, novals, false);
          continue;
        }
        for (unsigned k = 4 * h; k < 4 * h + 4; k++) {
          const int src = (int)(8u * k + (lane >> 3));
          const unsigned lo = __shfl((unsigned)m, src), hi = __shfl((unsigned)(m >> 32), src);
          const unsigned sh = 8u * (lane & 7u);
          const unsigned mb = (unsigned)(((((unsigned long long)hi) << 32) | lo) >> sh) & 0xFFu;
          emit_unit((unsigned)mb, (unsigned)((c + k) * kBlk) + 8u * lane, novals, false);
        }
      }
    }
  } else {
    // values: chunk by chunk, the next chunk's loads (and bitmask byte) issued before this
    // chunk is finished
    const InCol in = load_in(a.in);  // its views only here: fewer scalar registers held above
    unsigned *dec = ring + kEmitRing / 2;
    unsigned long long c = cw0;
    if (c < cw1) {
      Raw cur = issue_chunk(in, c, lane);
      unsigned mb = bm[c * 64];
      while (true) {
        const unsigned long long cn = c + 1;
        const bool more = cn < cw1;
        Raw nxt;
        unsigned mbn = 0;
        if (more) {
          nxt = issue_chunk(in, cn, lane);
          mbn = bm[cn * 64];
        }
        unsigned v[8];
        finish_chunk(in, cur, c, lane, dec, v);
        emit_unit(mb, (unsigned)(c * kBlk) + 8u * lane, v, true);
        if (!more) break;
        cur = nxt;
        mb = mbn;
        c = cn;
      }
    }
  }
  or_main = wg_or(or_main | or_base | bit_index_or(or_words), redo);
  if (threadIdx.x == 0) {
    a.partials[2 * seg] = orv;
    a.partials[2 * seg + 1] = or_main;
  }
}

__global__ __launch_bounds__(kWG) void k_emit(EmitArgs a) { emit_body<false>(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kWG) void k_emit_vals(EmitArgs a) { emit_body<true>(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kWG) void k_emit_batch(const EmitArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const EmitArgs &a, unsigned seg, unsigned G) { emit_body<false>(a, seg, G); });
}
__global__ __launch_bounds__(kWG) void k_emit_vals_batch(const EmitArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const EmitArgs &a, unsigned seg, unsigned G) { emit_body<true>(a, seg, G); });
}

// Compaction phase 3 (block formats): a block that started before a wave's output range
// is packed from the global stage by the wave whose range holds its last element.
__device__ __forceinline__ void emit_fix_body(const EmitArgs &a, const unsigned seg) {
  __shared__ __attribute__((aligned(16))) unsigned lds_all[kWaves * kBlk];
  const unsigned lane = lane_id(), w = wave_id();
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

__global__ __launch_bounds__(kWG) void k_emit_fix(EmitArgs a) { emit_fix_body(a, blockIdx.x); }
__global__ __launch_bounds__(kWG) void k_emit_fix_batch(const EmitArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const EmitArgs &a, unsigned seg, unsigned) { emit_fix_body(a, seg); });
}

// ---------------------------------------------------------------------------------------------
// Sum and group-sum.
__device__ __forceinline__ void sum_body(const ColView &inv, unsigned long long *partials, const unsigned seg,
                                         const unsigned G) {
  extern __shared__ __attribute__((aligned(16))) unsigned ring[];  // ring_shm() bytes
  __shared__ unsigned long long red[kWaves];
  const InCol in = load_in(inv);
  const unsigned lane = lane_id(), w = wave_id();
  unsigned long long s = 0;
  if (in.kind == RLE) {
    // sum over runs: value * run length (section 2.2)
    unsigned long long rb, re;
    segment(in.runs, seg, G, rb, re);
    // eight runs per thread per round, all loads issued before the products
    constexpr unsigned kU = 8;
    for (unsigned long long r = rb + threadIdx.x; r < re; r += kU * kWG) {
      unsigned st[kU], en[kU], val[kU];
#pragma unroll
      for (unsigned k = 0; k < kU; k++) {
        const unsigned long long q = r + (unsigned long long)k * kWG;
        st[k] = en[k] = val[k] = 0u;
        if (q < re) {
          st[k] = in.rstarts[q];
          en[k] = (q + 1 < in.runs) ? in.rstarts[q + 1] : (unsigned)in.n;
          val[k] = in.rvalues[q];
        }
      }
#pragma unroll
      for (unsigned k = 0; k < kU; k++) s += (unsigned long long)val[k] * (en[k] - st[k]);
    }
  } else {
    const unsigned long long C = (in.n + kBlk - 1) / kBlk;
    unsigned long long cb, ce;
    segment(C, seg, G, cb, ce);
    stream_chunks(in, cb, ce, w, lane, ring + w * kRing * kBlk, inv.hdr, [&](unsigned long long c, const unsigned (&v)[8]) {
      const unsigned valid = chunk_valid(c, lane, in.n);
      unsigned long long t = 0;
#pragma unroll
      for (int i = 0; i < 8; i++) t += ((valid >> i) & 1u) ? v[i] : 0u;
      s += t;
    });
  }
  s = wg_add64(s, red);
  if (threadIdx.x == 0) partials[seg] = s;
}

__global__ __launch_bounds__(kWG) void k_sum(ColView inv, unsigned long long *partials) {
  sum_body(inv, partials, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kWG) void k_sum_batch(const SumArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const SumArgs &a, unsigned seg, unsigned G) { sum_body(a.in, a.partials, seg, G); });
}

__device__ __forceinline__ void sum_finish_body(const unsigned long long *partials, unsigned G,
                                                unsigned long long *result) {
  __shared__ unsigned long long red[kWaves];
  unsigned long long t = 0;
  for (unsigned i = threadIdx.x; i < G; i += kWG) t += partials[i];
  t = wg_add64(t, red);
  if (threadIdx.x == 0) *result = t;
}

__global__ __launch_bounds__(kWG) void k_sum_finish(const unsigned long long *partials, unsigned G,
                                                    unsigned long long *result) {
  sum_finish_body(partials, G, result);
}
__global__ __launch_bounds__(kWG) void k_sum_finish_batch(const SumFinishArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const SumFinishArgs &a, unsigned, unsigned) { sum_finish_body(a.partials, a.G, a.result); });
}

constexpr unsigned kMaxLdsGroups = 4096;

__device__ __forceinline__ void group_sum_body(const ColView &gv, const ColView &vv, unsigned G_groups,
                                               unsigned long long *partials, const unsigned seg, const unsigned G) {
  __shared__ unsigned long long hist[kMaxLdsGroups];
  __shared__ __attribute__((aligned(16))) unsigned lds_all[2 * kWaves * kBlk];
  const InCol ig = load_in(gv);
  const InCol iv = load_in(vv);
  const unsigned lane = lane_id(), w = wave_id();
  if (ig.n != iv.n && seg == 0 && threadIdx.x == 0) raise_err(E_LENGTH);
  const unsigned long long n = min(ig.n, iv.n);
  const bool use_lds = G_groups <= kMaxLdsGroups;
  for (unsigned i = threadIdx.x; i < kMaxLdsGroups; i += kWG) hist[i] = 0;
  __syncthreads();
  const unsigned long long C = (n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, seg, G, cb, ce);
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
      const unsigned valid = chunk_valid(c, lane, n);
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
      partials[(unsigned long long)seg * G_groups + q] = hist[q];
  }
}

__global__ __launch_bounds__(kWG) void k_group_sum(ColView gv, ColView vv, unsigned G_groups,
                                                   unsigned long long *partials) {
  group_sum_body(gv, vv, G_groups, partials, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kWG) void k_group_sum_batch(const GroupSumArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const GroupSumArgs &a, unsigned seg, unsigned G) {
    group_sum_body(a.g, a.v, a.groups, a.partials, seg, G);
  });
}

// One workgroup per group: the sum of that group's per-workgroup partials (LDS
// histograms), else a copy of the global sums.
__device__ __forceinline__ void group_sum_finish_body(const unsigned long long *partials, unsigned G,
                                                      unsigned G_groups, unsigned lds, unsigned long long *out,
                                                      const unsigned seg) {
  __shared__ unsigned long long red[kWaves];
  const unsigned q = seg;
  if (!lds) {  // the partials are the sums themselves: one group per thread
    const unsigned long long i = (unsigned long long)seg * kWG + threadIdx.x;
    if (i < G_groups) out[i] = partials[i];
    return;
  }
  unsigned long long t = 0;
  for (unsigned b = threadIdx.x; b < G; b += kWG) t += partials[(unsigned long long)b * G_groups + q];
  t = wg_add64(t, red);
  if (threadIdx.x == 0) out[q] = t;
}

__global__ __launch_bounds__(kWG) void k_group_sum_finish(const unsigned long long *partials, unsigned G,
                                                          unsigned G_groups, unsigned lds, unsigned long long *out) {
  group_sum_finish_body(partials, G, G_groups, lds, out, blockIdx.x);
}
__global__ __launch_bounds__(kWG) void k_group_sum_finish_batch(const GroupSumFinishArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const GroupSumFinishArgs &a, unsigned seg, unsigned) {
    group_sum_finish_body(a.partials, a.G, a.groups, a.lds, a.out, seg);
  });
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

// Fills of a batch: segment seg of G covers words seg, seg + G*256, ... of its array.
__global__ __launch_bounds__(kWG) void k_fill_batch(const FillArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const FillArgs &a, unsigned seg, unsigned G) {
    for (unsigned long long i = (unsigned long long)seg * kWG + threadIdx.x; i < a.n; i += (unsigned long long)G * kWG) {
      if (a.p32) a.p32[i] = (unsigned)a.v;
      else a.p64[i] = a.v;
    }
  });
}

// Bitmap from positions: bit p of the (zeroed) bitmap for every position p.  With
// chunk_first/chunk_last set it also checks that the positions strictly increase
// (inside chunks here, across chunk ends in k_bitmap_ends).
__global__ __launch_bounds__(kWG) void k_bitmap(ColView posv, unsigned long long domain, unsigned *bitmap,
                                                unsigned *chunk_first, unsigned *chunk_last, unsigned *ends) {
  __shared__ __attribute__((aligned(16))) unsigned ring[kWaves * kRing * kBlk];
  const InCol in = load_in(posv);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  bool bad_range = false, bad_order = false;
  // strictly increasing: recorded by the producer, or checked here (a failed check is an error)
  const bool recorded = uni(posv.hdr->sorted) != 0;
  const bool check = chunk_first != nullptr && !recorded;
  const bool increasing = recorded || check;
  stream_chunks(in, cb, ce, w, lane, ring + w * kRing * kBlk, posv.hdr, [&](unsigned long long c, const unsigned (&v)[8]) {
    const unsigned long long idx0 = c * kBlk + 8ull * lane;
    const unsigned valid = chunk_valid(c, lane, in.n);
    if (check) {
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
    // A sorted list's chunk covers the bitmap words [w0, w1]: no other chunk has a
    // position inside (w0, w1), so when the span is short the words are assembled in
    // LDS (the wave's ring, unused outside RLE input) and stored plainly.  The two end
    // words, which neighbouring chunks may share, go to ends[4c .. 4c+3] as (word, bits)
    // pairs that k_bitmap_ends ORs in, keeping atomics out of this kernel.
    const unsigned nv = (unsigned)min((unsigned long long)kBlk, in.n - c * kBlk);  // valid values in the chunk
    const unsigned last_lane = (nv - 1) >> 3;
    const unsigned p_first = lane_first(v[0]);
    const unsigned p_last = __builtin_amdgcn_readlane(select8(v, (nv - 1) & 7u), last_lane);
    const unsigned w0 = p_first >> 5, w1 = p_last >> 5;
    const bool staged = increasing && in.kind != RLE && p_first <= p_last && (unsigned long long)p_last < domain &&
                        w1 - w0 < (unsigned)(kRing * kBlk);
    if (staged) {
      unsigned *st = ring + w * kRing * kBlk;
      const unsigned span = w1 - w0 + 1;
      for (unsigned t = lane; t < span; t += 64) st[t] = 0u;
      wave_sync();
      // p_last < domain here, and an increasing chunk keeps every position in
      // [p_first, p_last]: one unsigned compare keeps a disordered one out of the span
      const unsigned pspan = p_last - p_first;
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const unsigned p = v[i];
        if (((valid >> i) & 1u) && p - p_first <= pspan) atomicOr(&st[(p >> 5) - w0], 1u << (p & 31));
      }
      wave_sync();
      for (unsigned t = lane; t < span; t += 64) {
        const unsigned x = st[t];
        if (t == 0) {
          ends[4 * c] = w0;
          ends[4 * c + 1] = x;
        }
        if (t == span - 1) {
          ends[4 * c + 2] = w1;
          ends[4 * c + 3] = span > 1 ? x : 0u;
        }
        if (t > 0 && t < span - 1) bitmap[w0 + t] = x;
      }
      wave_sync();
    } else {
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
      if (lane < 4) ends[4 * c + lane] = 0u;  // nothing left for k_bitmap_ends
    }
  });
  if (bad_range) raise_err(E_RANGE);
  if (bad_order) raise_err(E_NOT_SORTED);
}

// The end words of every chunk of k_bitmap (and, for a list that must increase, the
// order across chunk boundaries).
__global__ void k_bitmap_ends(const unsigned *ends, const unsigned *chunk_first, const unsigned *chunk_last,
                              unsigned *bitmap, ColView posv) {
  const unsigned long long n = posv.hdr->n;
  const unsigned long long C = (n + kBlk - 1) / kBlk;
  const bool check = chunk_first != nullptr && posv.hdr->sorted == 0;  // as k_bitmap decided
  for (unsigned long long c = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; c < C;
       c += (unsigned long long)gridDim.x * blockDim.x) {
    if (check && c > 0 && chunk_first[c] <= chunk_last[c - 1]) raise_err(E_NOT_SORTED);
    const uint4 e = reinterpret_cast<const uint4 *>(ends)[c];
    if (e.y) atomicOr(&bitmap[e.x], e.y);
    if (e.w) atomicOr(&bitmap[e.z], e.w);
  }
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

std::vector<ErrWordSetter> &err_word_setters() {
  static std::vector<ErrWordSetter> r;
  return r;
}
unsigned *g_err_dev = nullptr;
}  // namespace

int prof_begin(const char *name, void *stream) {
  if (!g_prof_on || t_prof_suspended) return -1;
  std::lock_guard<std::mutex> g(g_prof_mu);
  ProfRec r{name, ev_get(), ev_get()};
  if (r.a) (void)hipEventRecord(r.a, S(stream));
  g_prof.push_back(r);
  return (int)g_prof.size() - 1;
}
void prof_end(int rec, void *stream) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (rec >= 0 && (size_t)rec < g_prof.size() && g_prof[rec].b) (void)hipEventRecord(g_prof[rec].b, S(stream));
}

// Registration runs in static initialisers of the kernel units, before any call.
void register_err_word_setter(ErrWordSetter f) { err_word_setters().push_back(f); }

hipError_t init_err_word() {
  if (!g_err_dev) {
    hipError_t e = hipMalloc(&g_err_dev, sizeof(unsigned));
    if (e != hipSuccess) return e;
    e = hipMemset(g_err_dev, 0, sizeof(unsigned));
    if (e != hipSuccess) return e;
  }
  for (ErrWordSetter f : err_word_setters())
    if (!f(g_err_dev)) return hipErrorInvalidSymbol;
  return hipDeviceSynchronize();
}

void prof_enable(bool on) { g_prof_on = on; }
void prof_suspend(bool on) { t_prof_suspended = on; }
bool prof_suspended() { return t_prof_suspended; }
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

unsigned read_and_clear_err(void *stream) {
  unsigned e = 0;
  if (!g_err_dev || hipMemcpyAsync(&e, g_err_dev, sizeof(e), hipMemcpyDeviceToHost, S(stream)) != hipSuccess ||
      hipMemsetAsync(g_err_dev, 0, sizeof(unsigned), S(stream)) != hipSuccess ||
      hipStreamSynchronize(S(stream)) != hipSuccess)
    return E_INVALID;
  return e;
}


hipError_t launch_set_hdr(ColHdr *h, unsigned long long n, unsigned long long runs, unsigned width, unsigned or_all,
                          unsigned or_main, unsigned sorted, void *s) {
  MS_LAUNCH(k_set_hdr, 1, 64, s, h, n, runs, width, or_all, or_main, sorted);
  return hipGetLastError();
}
hipError_t launch_finish(const FinishArgs &a, void *s) {
  if (batch::recording()) return batch::record_task(BK_FINISH, &a, sizeof(a), 1, 0);
  MS_LAUNCH(k_finish, 1, kWG, s, a);
  return hipGetLastError();
}
hipError_t launch_narrow(const FinishArgs &a, unsigned *tmp, unsigned G, void *s) {
  if (batch::recording()) {
    const NarrowArgs na{a, tmp};
    hipError_t e = batch::record_task(BK_NARROW, &na, sizeof(na), G, 0);
    return e == hipSuccess ? batch::record_task(BK_NARROW_COPY, &na, sizeof(na), G, 0) : e;
  }
  MS_LAUNCH(k_narrow, G, kWG, s, a, tmp);
  MS_LAUNCH(k_narrow_copy, G, kWG, s, a, tmp);
  return hipGetLastError();
}
hipError_t launch_colstats(const ColView &in, unsigned G, unsigned *partials, void *s) {
  MS_LAUNCH_SHM("k_colstats", k_colstats, G, kWG, ring_shm(in), s, in, partials);
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
#define MS_L(K) return launch_morph_ok<K>(in, out, auto_w, G, partials, s)
  MS_BY_OUT_KIND(out.kind, MS_L)
#undef MS_L
}
hipError_t launch_decode(const ColView &in, unsigned *out, unsigned G, void *s) {
  MS_LAUNCH_SHM("k_decode", k_decode, G, kWG, ring_shm(in), s, in, out);
  return hipGetLastError();
}
hipError_t launch_rle(unsigned mode, const ColView &a, const ColView &b, const ColView &out, unsigned G,
                      unsigned *wave_count, unsigned *partials, void *s) {
  ChunkSrc src;
  src.mode = mode;
  src.a = a;
  src.b = b;
  const size_t shm = (a.kind == RLE) ? kRleRingWords * sizeof(unsigned) : 0;
  if (mode == 0) {
    MS_LAUNCH_SHM("k_rle_count", k_rle_count, G, kWG, shm, s, src, wave_count);
    MS_LAUNCH_SHM("k_rle_emit", k_rle_emit, G, kWG, shm, s, src, out, wave_count, partials);
  } else if (b.kind == RLE) {
    MS_LAUNCH_SHM("k_rle_count_proj", k_rle_count_proj<true>, G, kWG, shm, s, src, wave_count);
    MS_LAUNCH_SHM("k_rle_emit_proj", k_rle_emit_proj<true>, G, kWG, shm, s, src, out, wave_count, partials);
  } else {
    MS_LAUNCH_SHM("k_rle_count_proj", k_rle_count_proj<false>, G, kWG, shm, s, src, wave_count);
    MS_LAUNCH_SHM("k_rle_emit_proj", k_rle_emit_proj<false>, G, kWG, shm, s, src, out, wave_count, partials);
  }
  return hipGetLastError();
}
hipError_t launch_project(const ColView &pos, const ColView &data, const ColView &out, unsigned auto_w, unsigned G,
                          unsigned *partials, void *s) {
#define MS_L(K) return launch_project_ok<K>(pos, data, out, auto_w, G, partials, s)
  MS_BY_OUT_KIND(out.kind, MS_L)
#undef MS_L
}
hipError_t launch_emit(const EmitArgs &a, unsigned G, void *s) {
  const unsigned k = a.out.kind;
  const bool fix = k == STATIC_BP || k == DYN_BP || k == DELTA_DYN_BP || k == FOR_DYN_BP;
  if (batch::recording()) {
    hipError_t e = batch::record_task(a.emit_values ? BK_EMIT_VALS : BK_EMIT, &a, sizeof(a), G, 0);
    if (e == hipSuccess && fix) e = batch::record_task(BK_EMIT_FIX, &a, sizeof(a), G, 0);
    return e;
  }
  if (a.emit_values) MS_LAUNCH(k_emit_vals, G, kWG, s, a);
  else MS_LAUNCH(k_emit, G, kWG, s, a);
  if (fix) MS_LAUNCH(k_emit_fix, G, kWG, s, a);
  return hipGetLastError();
}
hipError_t launch_sum(const ColView &in, unsigned long long *result, unsigned G, unsigned long long *partials,
                      void *s) {
  if (batch::recording()) {
    const SumArgs sa{in, partials};
    const SumFinishArgs sf{partials, G, result};
    hipError_t e = batch::record_task(BK_SUM, &sa, sizeof(sa), G, ring_shm(in));
    return e == hipSuccess ? batch::record_task(BK_SUM_FINISH, &sf, sizeof(sf), 1, 0) : e;
  }
  MS_LAUNCH_SHM("k_sum", k_sum, G, kWG, ring_shm(in), s, in, partials);
  MS_LAUNCH(k_sum_finish, 1, kWG, s, partials, G, result);
  return hipGetLastError();
}
hipError_t launch_group_sum(const ColView &g, const ColView &v, unsigned groups, unsigned long long *out, unsigned G,
                            unsigned long long *partials, void *s) {
  const unsigned lds = groups <= kMaxLdsGroups ? 1u : 0u;
  if (batch::recording()) {
    const GroupSumArgs ga{g, v, groups, partials};
    const GroupSumFinishArgs gf{partials, G, groups, lds, out};
    hipError_t e = batch::record_task(BK_GROUP_SUM, &ga, sizeof(ga), G, 0);
    if (e == hipSuccess && groups > 0)
      e = batch::record_task(BK_GROUP_SUM_FINISH, &gf, sizeof(gf), lds ? groups : (groups + kWG - 1) / kWG, 0);
    return e;
  }
  MS_LAUNCH(k_group_sum, G, kWG, s, g, v, groups, partials);
  if (groups > 0) MS_LAUNCH(k_group_sum_finish, lds ? groups : (groups + kWG - 1) / kWG, kWG, s, partials, G, groups, lds, out);
  return hipGetLastError();
}
hipError_t launch_fill_u32(unsigned *p, unsigned long long n, unsigned v, void *s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<unsigned long long>((n + 255) / 256, 2048ull);
  if (batch::recording()) {
    const FillArgs f{p, nullptr, n, v};
    return batch::record_task(BK_FILL, &f, sizeof(f), blocks, 0);
  }
  MS_LAUNCH(k_fill_u32, blocks, 256, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long n, unsigned long long v, void *s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<unsigned long long>((n + 255) / 256, 2048ull);
  if (batch::recording()) {
    const FillArgs f{nullptr, p, n, v};
    return batch::record_task(BK_FILL, &f, sizeof(f), blocks, 0);
  }
  MS_LAUNCH(k_fill_u64, blocks, 256, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_batch(unsigned kind, const void *tasks, const BatchQueue &q, unsigned grid, size_t shm, void *s) {
  switch (kind) {
    case BK_PRED0:
    case BK_PRED1:
    case BK_PRED2: return launch_pred_batch(kind - BK_PRED0, static_cast<const PredArgs *>(tasks), q, grid, shm, s);
    case BK_EMIT: MS_LAUNCH(k_emit_batch, grid, kWG, s, static_cast<const EmitArgs *>(tasks), q); break;
    case BK_EMIT_VALS: MS_LAUNCH(k_emit_vals_batch, grid, kWG, s, static_cast<const EmitArgs *>(tasks), q); break;
    case BK_EMIT_FIX: MS_LAUNCH(k_emit_fix_batch, grid, kWG, s, static_cast<const EmitArgs *>(tasks), q); break;
    case BK_FINISH: MS_LAUNCH(k_finish_batch, grid, kWG, s, static_cast<const FinishArgs *>(tasks), q); break;
    case BK_SUM:
      MS_LAUNCH_SHM("k_sum_batch", k_sum_batch, grid, kWG, shm, s, static_cast<const SumArgs *>(tasks), q);
      break;
    case BK_SUM_FINISH: MS_LAUNCH(k_sum_finish_batch, grid, kWG, s, static_cast<const SumFinishArgs *>(tasks), q); break;
    case BK_GROUP_SUM: MS_LAUNCH(k_group_sum_batch, grid, kWG, s, static_cast<const GroupSumArgs *>(tasks), q); break;
    case BK_GROUP_SUM_FINISH:
      MS_LAUNCH(k_group_sum_finish_batch, grid, kWG, s, static_cast<const GroupSumFinishArgs *>(tasks), q);
      break;
    case BK_FILL: MS_LAUNCH(k_fill_batch, grid, kWG, s, static_cast<const FillArgs *>(tasks), q); break;
    case BK_NARROW: MS_LAUNCH(k_narrow_batch, grid, kWG, s, static_cast<const NarrowArgs *>(tasks), q); break;
    case BK_NARROW_COPY: MS_LAUNCH(k_narrow_copy_batch, grid, kWG, s, static_cast<const NarrowArgs *>(tasks), q); break;
    default: {
      const unsigned ok = (kind - BK_MORPH0) % 5;
      const MorphArgs *m = static_cast<const MorphArgs *>(tasks);
      const ProjectArgs *pj = static_cast<const ProjectArgs *>(tasks);
      const bool rle = kind >= BK_PROJECT_RLE0;
      if (kind >= BK_MORPH0 && kind < BK_PROJECT0) {
        switch (ok) {
          case UNCOMPR: return launch_morph_batch_ok<UNCOMPR>(m, q, grid, shm, s);
          case STATIC_BP: return launch_morph_batch_ok<STATIC_BP>(m, q, grid, shm, s);
          case DYN_BP: return launch_morph_batch_ok<DYN_BP>(m, q, grid, shm, s);
          case DELTA_DYN_BP: return launch_morph_batch_ok<DELTA_DYN_BP>(m, q, grid, shm, s);
          default: return launch_morph_batch_ok<FOR_DYN_BP>(m, q, grid, shm, s);
        }
      }
      if (kind >= BK_PROJECT0 && kind < BK_COUNT) {
        switch (ok) {
          case UNCOMPR: return launch_project_batch_ok<UNCOMPR>(pj, rle, q, grid, shm, s);
          case STATIC_BP: return launch_project_batch_ok<STATIC_BP>(pj, rle, q, grid, shm, s);
          case DYN_BP: return launch_project_batch_ok<DYN_BP>(pj, rle, q, grid, shm, s);
          case DELTA_DYN_BP: return launch_project_batch_ok<DELTA_DYN_BP>(pj, rle, q, grid, shm, s);
          default: return launch_project_batch_ok<FOR_DYN_BP>(pj, rle, q, grid, shm, s);
        }
      }
      return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_bitmap(const ColView &pos, unsigned long long domain, unsigned *bitmap, unsigned *ends,
                         unsigned *first, unsigned *last, unsigned G, void *s) {
  MS_LAUNCH(k_bitmap, G, kWG, s, pos, domain, bitmap, first, last, ends);
  MS_LAUNCH(k_bitmap_ends, 512, 256, s, ends, first, last, bitmap, pos);
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
  MS_LAUNCH_SHM("k_footprints", k_footprints, G, kWG, ring_shm(in), s, a);
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
}  // namespace ms
