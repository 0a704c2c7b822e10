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
__global__ __launch_bounds__(kWG) void k_morph(ColView inv, ColView outv, unsigned auto_w, unsigned *partials) {
  extern __shared__ __attribute__((aligned(16))) unsigned ring[];  // ring_shm() bytes
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

template <>
hipError_t launch_morph_ok<MS_OK>(const ColView &in, const ColView &out, unsigned auto_w, unsigned G,
                                  unsigned *partials, void *s) {
  static const char *const names[] = {"k_morph<UNCOMPR>", "k_morph<STATIC_BP>", "k_morph<DYN_BP>",
                                      "k_morph<DELTA_DYN_BP>", "k_morph<FOR_DYN_BP>"};
  MS_LAUNCH_SHM(names[MS_OK], k_morph<MS_OK>, G, kWG, ring_shm(in), s, in, out, auto_w, partials);
  return hipGetLastError();
}

}  // namespace ms
