// ms_kcommon.h -- device helpers shared by the operator kernels: workgroup segments and
// reductions, and the output side (static BP chunks, DynBP-family blocks, uncompressed
// stores) of operators whose output count is known up front.
#pragma once
#include <hip/hip_runtime.h>

#include "ms_device.h"
#include "ms_kernels.h"

namespace ms {

// Segment s of G over C chunks.
__device__ __forceinline__ void segment(unsigned long long C, unsigned s, unsigned G, unsigned long long &cb,
                                        unsigned long long &ce) {
  cb = C * s / G;
  ce = C * (s + 1) / G;
}

// A batched persistent launch (see BatchQueue): every workgroup takes tickets until they
// run out and runs `body(task args, segment, segments of that task)` for each.  Tasks come
// in decreasing size (longest first), so the big tasks' segments start first and the small
// ones fill in behind them.  No workgroup waits for another: a workgroup leaves once the
// tickets are gone, and every body is a complete workgroup program (its barriers are
// reached by all of the workgroup's threads).
template <class Args, class Body>
__device__ __forceinline__ void batch_run(const Args *__restrict__ tasks, const BatchQueue &q, Body &&body) {
  __shared__ unsigned s_ticket;
  const unsigned total = q.seg_prefix[q.n_tasks];
  for (;;) {
    if (threadIdx.x == 0) s_ticket = atomicAdd(q.ticket, 1u);
    __syncthreads();
    const unsigned t = __builtin_amdgcn_readfirstlane(s_ticket);
    __syncthreads();  // every thread holds t before the next ticket replaces it
    if (t >= total) break;
    unsigned lo = 0, hi = q.n_tasks;  // the task: the last i with seg_prefix[i] <= t
    while (hi - lo > 1) {
      const unsigned mid = (lo + hi) >> 1;
      if (q.seg_prefix[mid] <= t) lo = mid;
      else hi = mid;
    }
    const Args a = tasks[lo];
    body(a, t - q.seg_prefix[lo], q.seg_prefix[lo + 1] - q.seg_prefix[lo]);
    __syncthreads();  // the body's LDS is free before the next ticket's body starts
  }
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
// The same for lane `lane` of chunk c, where c and n are wave-uniform: a scalar test
// settles every full chunk.
__device__ __forceinline__ unsigned chunk_valid(unsigned long long c, unsigned lane, unsigned long long n) {
  if ((c + 1) * kBlk <= n) return 0xFFu;
  return valid_mask(c * kBlk + 8ull * lane, n);
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

}  // namespace ms
