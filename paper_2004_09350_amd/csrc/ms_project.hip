// ms_project.hip -- project into one output format; compiled once per output kind
// (MS_OK) so that the instantiations build in parallel.
#include <hip/hip_runtime.h>

#include "ms_kcommon.h"
#include "ms_launch.h"

#ifndef MS_OK
#error "MS_OK (the output kind) must be defined"
#endif

namespace ms {

// ---------------------------------------------------------------------------------------------
// Project: out_j = data[pos_j].
// Project: gather the data column at the positions streamed from posv and encode the
// values into the output format.  RLE data columns have their own kernel (their gather
// stages runs in LDS and needs its own registers).
template <unsigned OK, bool DRLE>
__device__ __forceinline__ void project_body(const ColView &posv, const ColView &datav, const ColView &outv,
                                             unsigned auto_w, unsigned *partials, const unsigned seg,
                                             const unsigned G) {
  extern __shared__ __attribute__((aligned(16))) unsigned ring[];  // ring_shm() bytes
  __shared__ __attribute__((aligned(16))) unsigned gblk[kWaves * kBlk];
  __shared__ __attribute__((aligned(16))) unsigned lds_all[kWaves * kBlk];
  __shared__ unsigned red[kWaves];
  const InCol ip = load_in(posv);
  const InCol id = load_in(datav);
  const unsigned lane = lane_id(), w = threadIdx.x >> 6;  // w kept in a VGPR: SGPRs run short here
  unsigned Wp = outv.width;
  if (outv.kind == STATIC_BP && auto_w) Wp = bw(datav.hdr->or_all);
  const OutCol o = make_out(outv, ip.n, Wp);
  if (seg == 0 && threadIdx.x == 0) outv.hdr->sbp_width = Wp;
  const unsigned long long C = (ip.n + kBlk - 1) / kBlk;
  unsigned long long cb, ce;
  segment(C, seg, G, cb, ce);
  unsigned or_all = 0, or_main = 0;
  unsigned *lds = lds_all + w * kBlk;
  bool bad = false;
  stream_chunks(ip, cb, ce, w, lane, ring + w * kRing * kBlk, posv.hdr, [&](unsigned long long c, const unsigned (&pv)[8]) {
    unsigned v[8];
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = pv[i];
    const unsigned valid = chunk_valid(c, lane, ip.n);
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
    partials[2 * seg] = or_all;
    partials[2 * seg + 1] = or_main;
  }
}

template <unsigned OK>
__global__ __launch_bounds__(kWG, 3) void k_project(ColView posv, ColView datav, ColView outv, unsigned auto_w,
                                                 unsigned *partials) {
  project_body<OK, false>(posv, datav, outv, auto_w, partials, blockIdx.x, gridDim.x);
}
template <unsigned OK>
__global__ __launch_bounds__(kWG) void k_project_rle(ColView posv, ColView datav, ColView outv, unsigned auto_w,
                                                     unsigned *partials) {
  project_body<OK, true>(posv, datav, outv, auto_w, partials, blockIdx.x, gridDim.x);
}
template <unsigned OK>
__global__ __launch_bounds__(kWG, 3) void k_project_batch(const ProjectArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const ProjectArgs &a, unsigned seg, unsigned G) {
    project_body<OK, false>(a.pos, a.data, a.out, a.auto_w, a.partials, seg, G);
  });
}
template <unsigned OK>
__global__ __launch_bounds__(kWG) void k_project_rle_batch(const ProjectArgs *tasks, BatchQueue q) {
  batch_run(tasks, q, [](const ProjectArgs &a, unsigned seg, unsigned G) {
    project_body<OK, true>(a.pos, a.data, a.out, a.auto_w, a.partials, seg, G);
  });
}

template <>
hipError_t launch_project_ok<MS_OK>(const ColView &pos, const ColView &data, const ColView &out, unsigned auto_w,
                                    unsigned G, unsigned *partials, void *s) {
  static const char *const names[] = {"k_project<UNCOMPR>", "k_project<STATIC_BP>", "k_project<DYN_BP>",
                                      "k_project<DELTA_DYN_BP>", "k_project<FOR_DYN_BP>"};
  static const char *const rle_names[] = {"k_project_rle<UNCOMPR>", "k_project_rle<STATIC_BP>",
                                          "k_project_rle<DYN_BP>", "k_project_rle<DELTA_DYN_BP>",
                                          "k_project_rle<FOR_DYN_BP>"};
  if (batch::recording()) {
    const ProjectArgs pa{pos, data, out, auto_w, partials};
    return batch::record_task((data.kind == RLE ? BK_PROJECT_RLE0 : BK_PROJECT0) + MS_OK, &pa, sizeof(pa), G,
                              ring_shm(pos));
  }
  if (data.kind == RLE)
    MS_LAUNCH_SHM(rle_names[MS_OK], k_project_rle<MS_OK>, G, kWG, ring_shm(pos), s, pos, data, out, auto_w, partials);
  else
    MS_LAUNCH_SHM(names[MS_OK], k_project<MS_OK>, G, kWG, ring_shm(pos), s, pos, data, out, auto_w, partials);
  return hipGetLastError();
}

template <>
hipError_t launch_project_batch_ok<MS_OK>(const ProjectArgs *tasks, bool data_rle, const BatchQueue &q, unsigned grid,
                                          size_t shm, void *s) {
  static const char *const names[] = {"k_project_batch<UNCOMPR>", "k_project_batch<STATIC_BP>",
                                      "k_project_batch<DYN_BP>", "k_project_batch<DELTA_DYN_BP>",
                                      "k_project_batch<FOR_DYN_BP>"};
  static const char *const rle_names[] = {"k_project_rle_batch<UNCOMPR>", "k_project_rle_batch<STATIC_BP>",
                                          "k_project_rle_batch<DYN_BP>", "k_project_rle_batch<DELTA_DYN_BP>",
                                          "k_project_rle_batch<FOR_DYN_BP>"};
  if (data_rle)
    MS_LAUNCH_SHM(rle_names[MS_OK], k_project_rle_batch<MS_OK>, grid, kWG, shm, s, tasks, q);
  else
    MS_LAUNCH_SHM(names[MS_OK], k_project_batch<MS_OK>, grid, kWG, shm, s, tasks, q);
  return hipGetLastError();
}

}  // namespace ms
