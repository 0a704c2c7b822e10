// ms_morph.hip -- morph (and encode) into one output format; compiled once per output
// kind (MS_OK) so that the instantiations build in parallel.
#include <hip/hip_runtime.h>

#include "ms_kcommon.h"
#include "ms_launch.h"

#ifndef MS_OK
#error "MS_OK (the output kind) must be defined"
#endif

namespace ms {

// ---------------------------------------------------------------------------------------------
// Morph (and encode): out = encode_fmt(decode(in)), count known.
template <unsigned OK>
__device__ __forceinline__ void morph_body(const ColView &inv, const ColView &outv, unsigned auto_w, unsigned *partials,
                                           const unsigned seg, const unsigned G) {
  extern __shared__ __attribute__((aligned(16))) unsigned ring[];  // ring_shm() bytes
  __shared__ __attribute__((aligned(16))) unsigned lds_all[kWaves * kBlk];
  __shared__ unsigned red[kWaves];
  const InCol in = load_in(inv);
  const unsigned lane = lane_id(), w = wave_id();
  unsigned Wp = outv.width;
  if (outv.kind == STATIC_BP && auto_w) Wp = bw(inv.hdr->or_all);
  const OutCol o = make_out(outv, in.n, Wp);
  if (seg == 0 && threadIdx.x == 0) outv.hdr->sbp_width = Wp;
  const unsigned long long C = (in.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, seg, G, cb, ce);
  unsigned or_all = 0, or_main = 0;
  unsigned *lds = lds_all + w * kBlk;
  stream_chunks(in, cb, ce, w, lane, ring + w * kRing * kBlk, inv.hdr, [&](unsigned long long c, const unsigned (&v)[8]) {
    write_chunk_known<OK>(o, c, v, lane, lds, or_all, or_main);
  });
  or_all = wg_or(or_all, red);
  or_main = wg_or(or_main, red);
  if (threadIdx.x == 0) {
    partials[2 * seg] = or_all;
    partials[2 * seg + 1] = or_main;
  }
}

template <unsigned OK>
__global__ __launch_bounds__(kWG) void k_morph(ColView inv, ColView outv, unsigned auto_w, unsigned *partials) {
  morph_body<OK>(inv, outv, auto_w, partials, blockIdx.x, gridDim.x);
}
template <unsigned OK>
__global__ __launch_bounds__(kWG) void k_morph_batch(const MorphArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const MorphArgs &a, unsigned seg, unsigned G) {
    morph_body<OK>(a.in, a.out, a.auto_w, a.partials, seg, G);
  });
}

// calc (section 4.2's element-wise arithmetic): out_i = a_i op b_i modulo 2^32 (op 0 add,
// 1 sub, 2 mul).  a streams through the chunk pipeline, b is decoded chunk by chunk beside
// it.  A static BP output of automatic width is packed at 32 bits and narrowed afterwards.
template <unsigned OK>
__global__ __launch_bounds__(kWG) void k_calc(ColView av, ColView bv, unsigned op, ColView outv, unsigned *partials) {
  extern __shared__ __attribute__((aligned(16))) unsigned ring[];  // ring_shm() bytes
  __shared__ __attribute__((aligned(16))) unsigned lds_all[kWaves * kBlk];
  __shared__ unsigned red[kWaves];
  const InCol a = load_in(av);
  const InCol b = load_in(bv);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x;
  if (a.n != b.n) {
    if (threadIdx.x == 0) raise_err(E_LENGTH);
    return;
  }
  const unsigned Wp = outv.width;
  const OutCol o = make_out(outv, a.n, Wp);
  if (blockIdx.x == 0 && threadIdx.x == 0) outv.hdr->sbp_width = Wp;
  const unsigned long long C = (a.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned or_all = 0, or_main = 0;
  unsigned *lds = lds_all + w * kBlk;
  unsigned long long hint_b = 0;
  stream_chunks(a, cb, ce, w, lane, ring + w * kRing * kBlk, av.hdr, [&](unsigned long long c, const unsigned (&va)[8]) {
    unsigned vb[8], v[8];
    decode_chunk(b, c, lane, vb, hint_b);
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = op == 0 ? va[i] + vb[i] : op == 1 ? va[i] - vb[i] : va[i] * vb[i];
    write_chunk_known<OK>(o, c, v, lane, lds, or_all, or_main);
  });
  or_all = wg_or(or_all, red);
  or_main = wg_or(or_main, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = or_all;
    partials[2 * blockIdx.x + 1] = or_main;
  }
}

// Group ids of a group-by: id_i = rank of key_i among the distinct keys, from the keys'
// presence bitmap and its per-word exclusive prefix counts (keys < the bitmap's domain).
template <unsigned OK>
__global__ __launch_bounds__(kWG) void k_rank(ColView kv, unsigned long long domain, const unsigned *bitmap,
                                              const unsigned *wprefix, ColView outv, unsigned *partials) {
  extern __shared__ __attribute__((aligned(16))) unsigned ring[];  // ring_shm() bytes
  __shared__ __attribute__((aligned(16))) unsigned lds_all[kWaves * kBlk];
  __shared__ unsigned red[kWaves];
  const InCol k = load_in(kv);
  const unsigned lane = lane_id(), w = wave_id(), G = gridDim.x;
  unsigned Wp = outv.width;
  if (outv.kind == STATIC_BP && Wp > 32) Wp = 32;
  const OutCol o = make_out(outv, k.n, Wp);
  if (blockIdx.x == 0 && threadIdx.x == 0) outv.hdr->sbp_width = Wp;
  const unsigned long long C = (k.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, blockIdx.x, G, cb, ce);
  unsigned or_all = 0, or_main = 0;
  unsigned *lds = lds_all + w * kBlk;
  stream_chunks(k, cb, ce, w, lane, ring + w * kRing * kBlk, kv.hdr, [&](unsigned long long c, const unsigned (&kk)[8]) {
    const unsigned valid = chunk_valid(c, lane, k.n);
    unsigned v[8];
#pragma unroll
    for (int i = 0; i < 8; i++) {
      // a key outside the domain (raised as an error by the marking pass) reads id 0
      const unsigned x = ((valid >> i) & 1u) && (unsigned long long)kk[i] < domain ? kk[i] : 0u;
      v[i] = wprefix[x >> 5] + __popc(bitmap[x >> 5] & ((1u << (x & 31u)) - 1u));
    }
    write_chunk_known<OK>(o, c, v, lane, lds, or_all, or_main);
  });
  or_all = wg_or(or_all, red);
  or_main = wg_or(or_main, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = or_all;
    partials[2 * blockIdx.x + 1] = or_main;
  }
}

template <>
hipError_t launch_calc_ok<MS_OK>(const ColView &a, const ColView &b, unsigned op, const ColView &out, unsigned G,
                                 unsigned *partials, void *s) {
  static const char *const names[] = {"k_calc<UNCOMPR>", "k_calc<STATIC_BP>", "k_calc<DYN_BP>",
                                      "k_calc<DELTA_DYN_BP>", "k_calc<FOR_DYN_BP>"};
  MS_LAUNCH_SHM(names[MS_OK], k_calc<MS_OK>, G, kWG, ring_shm(a), s, a, b, op, out, partials);
  return hipGetLastError();
}

template <>
hipError_t launch_rank_ok<MS_OK>(const ColView &keys, unsigned long long domain, const unsigned *bitmap,
                                 const unsigned *wprefix, const ColView &out, unsigned G, unsigned *partials, void *s) {
  static const char *const names[] = {"k_rank<UNCOMPR>", "k_rank<STATIC_BP>", "k_rank<DYN_BP>",
                                      "k_rank<DELTA_DYN_BP>", "k_rank<FOR_DYN_BP>"};
  MS_LAUNCH_SHM(names[MS_OK], k_rank<MS_OK>, G, kWG, ring_shm(keys), s, keys, domain, bitmap, wprefix, out, partials);
  return hipGetLastError();
}

template <>
hipError_t launch_morph_ok<MS_OK>(const ColView &in, const ColView &out, unsigned auto_w, unsigned G,
                                  unsigned *partials, void *s) {
  static const char *const names[] = {"k_morph<UNCOMPR>", "k_morph<STATIC_BP>", "k_morph<DYN_BP>",
                                      "k_morph<DELTA_DYN_BP>", "k_morph<FOR_DYN_BP>"};
  if (batch::recording()) {
    const MorphArgs m{in, out, auto_w, partials};
    return batch::record_task(BK_MORPH0 + MS_OK, &m, sizeof(m), G, ring_shm(in));
  }
  MS_LAUNCH_SHM(names[MS_OK], k_morph<MS_OK>, G, kWG, ring_shm(in), s, in, out, auto_w, partials);
  return hipGetLastError();
}

template <>
hipError_t launch_morph_batch_ok<MS_OK>(const MorphArgs *tasks, const BatchQueue &q, unsigned grid, size_t shm,
                                        void *s) {
  static const char *const names[] = {"k_morph_batch<UNCOMPR>", "k_morph_batch<STATIC_BP>", "k_morph_batch<DYN_BP>",
                                      "k_morph_batch<DELTA_DYN_BP>", "k_morph_batch<FOR_DYN_BP>"};
  MS_LAUNCH_SHM(names[MS_OK], k_morph_batch<MS_OK>, grid, kWG, shm, s, tasks, q);
  return hipGetLastError();
}

}  // namespace ms
