// ms_selector.hip -- format selection (section 5.2): the exhaustive choice (least exact
// footprint, per column, since column footprints add up) and the learned selector, a pair
// of 32-64-64-6 networks over the 32 column statistics: one predicts each format's size,
// the other each format's decode time (section 5.2's cost model estimates both the
// compression rate and the (de)compression performance).  Training targets are computed
// on the device from what the engine measures; training, inference and the argmin run in
// this unit's kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/morphgpu.h"
#include "ms_launch.h"
#include "ms_runtime.h"

namespace ms {

#include "ms_mlp.inc"

namespace {

// Label transforms (the network learns log-scaled costs; a smaller target is better).
constexpr double kSizeScale = 6.0;   // size: log2(1 + bits per value) / 6
constexpr double kCostScale = 16.0;  // decode: log2(1 + picoseconds per value) / 16

__global__ __launch_bounds__(kWG) void k_size_targets(const unsigned long long *bytes6, const unsigned long long *n,
                                                      unsigned long long count, float *T) {
  const unsigned long long i = (unsigned long long)blockIdx.x * kWG + threadIdx.x;
  if (i >= count) return;
  const double nv = n[i] > 0 ? (double)n[i] : 1.0;
#pragma unroll
  for (int k = 0; k < kOut; k++) T[i * kOut + k] = (float)(log2(1.0 + 8.0 * (double)bytes6[i * kOut + k] / nv) / kSizeScale);
}

__global__ __launch_bounds__(kWG) void k_cost_targets(const float *ns6, const unsigned long long *n,
                                                      unsigned long long count, float *T) {
  const unsigned long long i = (unsigned long long)blockIdx.x * kWG + threadIdx.x;
  if (i >= count) return;
  const double nv = n[i] > 0 ? (double)n[i] : 1.0;
#pragma unroll
  for (int k = 0; k < kOut; k++) {
    const double ns = ns6[i * kOut + k] > 0.f ? (double)ns6[i * kOut + k] : 0.0;
    T[i * kOut + k] = (float)(log2(1.0 + 1000.0 * ns / nv) / kCostScale);
  }
}

// Exhaustive choice: the format of least footprint, ties to the lower format number.
__global__ __launch_bounds__(kWG) void k_argmin6(const unsigned long long *bytes6, unsigned long long count,
                                                 unsigned *kinds) {
  const unsigned long long i = (unsigned long long)blockIdx.x * kWG + threadIdx.x;
  if (i >= count) return;
  unsigned best = 0;
  unsigned long long bb = bytes6[i * kOut];
#pragma unroll
  for (int k = 1; k < kOut; k++) {
    const unsigned long long b = bytes6[i * kOut + k];
    if (b < bb) {
      bb = b;
      best = k;
    }
  }
  kinds[i] = best;
}

unsigned blocks(unsigned long long count) { return (unsigned)((count + kWG - 1) / kWG); }

hipError_t launch_grad_map(const float *params, const float *x, const float *t, unsigned n, const BatchMap &map,
                           float *gpart, float *lpart, float *grad, float *loss, void *s) {
  const unsigned nwg = (n + kGradSamples - 1) / kGradSamples;
  MS_LAUNCH(k_mlp_grad, nwg, kWG, s, params, x, t, n, map, gpart, lpart);
  MS_LAUNCH(k_mlp_grad_reduce, (kNParam + kWG - 1) / kWG, kWG, s, gpart, lpart, nwg, grad, loss);
  return hipGetLastError();
}

}  // namespace

unsigned mlp_nparam() { return kNParam; }
hipError_t launch_mlp_forward(const float *params, const float *x, unsigned n, float *y, unsigned *pick, void *s) {
  if (n == 0) return hipSuccess;
  MS_LAUNCH(k_mlp_forward, (n + 63) / 64, 64, s, params, x, n, y, pick);
  return hipGetLastError();
}
unsigned mlp_grad_workgroups(unsigned n) { return (n + kGradSamples - 1) / kGradSamples; }
hipError_t launch_mlp_grad(const float *params, const float *x, const float *t, unsigned n, float *gpart,
                           float *lpart, float *grad, float *loss, void *s) {
  return launch_grad_map(params, x, t, n, BatchMap{0, 1, 0, n ? n : 1}, gpart, lpart, grad, loss, s);
}
hipError_t launch_adam(float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps, float c1,
                       float c2, void *s) {
  MS_LAUNCH(k_adam, (kNParam + kWG - 1) / kWG, kWG, s, p, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace ms

using namespace ms;

struct ms_selector {
  float *params[2] = {nullptr, nullptr};  // device, kNParam floats each (size, decode-cost network)
  uint32_t trained = 0;                   // bit k: network k has been trained (or loaded trained)
};

namespace {

constexpr char kMagic[8] = {'M', 'S', 'S', 'E', 'L', '0', '0', '1'};
constexpr uint64_t kParamBytes = sizeof(float) * (uint64_t)kNParam;

ms_status fail(ms_status st, const std::string &msg) {
  rt::set_error(msg.c_str());
  return st;
}
ms_status hip_fail(hipError_t e, const char *what) {
  return fail(MS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}
ms_status check_init() {
  return rt::initialized() ? MS_OK : fail(MS_ERR_NOT_INITIALIZED, "ms_init has not been called");
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the training order's generator.
uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}
// Epoch e's order of the N training rows: row of position j = (a * j + b) mod N with
// a coprime with N (a permutation), a and b drawn from the seed's SplitMix64 stream.
BatchMap epoch_map(uint64_t seed, uint64_t e, uint64_t N) {
  if (N <= 1) return BatchMap{0, 1, 0, 1};
  const uint64_t key = mix64(seed);
  const uint64_t x = mix64(key + (2 * e + 1) * 0x9E3779B97F4A7C15ull);
  const uint64_t y = mix64(key + (2 * e + 2) * 0x9E3779B97F4A7C15ull);
  uint64_t a = 1 + x % (N - 1);
  while (gcd64(a, N) != 1) a = a + 1 < N ? a + 1 : 1;
  return BatchMap{0, a, y % N, N};
}

void free_selector(ms_selector *s) {
  if (!s) return;
  for (float *p : s->params)
    if (p) rt::free(p, kParamBytes, nullptr);
  delete s;
}

ms_status new_selector(ms_selector **out) {
  ms_selector *s = new ms_selector();
  for (float *&p : s->params) {
    p = static_cast<float *>(rt::alloc(kParamBytes, nullptr));
    if (!p) {
      free_selector(s);
      return fail(MS_ERR_OOM, "parameter allocation failed");
    }
  }
  *out = s;
  return MS_OK;
}

}  // namespace

extern "C" {

ms_status ms_selector_create(const float *host_init_size, const float *host_init_cost, ms_selector **out) {
  if (!out) return fail(MS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!host_init_size || !host_init_cost) return fail(MS_ERR_INVALID_ARG, "initial parameters are NULL");
  ms_selector *s = nullptr;
  st = new_selector(&s);
  if (st != MS_OK) return st;
  hipError_t e = hipMemcpy(s->params[0], host_init_size, kParamBytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->params[1], host_init_cost, kParamBytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_selector(s);
    return hip_fail(e, "parameter upload");
  }
  *out = s;
  return MS_OK;
}

ms_status ms_selector_destroy(ms_selector *sel) {
  if (sel) (void)hipDeviceSynchronize();  // parameters may still be read by queued work
  free_selector(sel);
  return MS_OK;
}

ms_status ms_selector_params(const ms_selector *sel, uint32_t net, float *dev_dst, void *stream) {
  if (!sel || !dev_dst) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  if (net > MS_NET_COST) return fail(MS_ERR_INVALID_ARG, "net must be MS_NET_SIZE or MS_NET_COST");
  hipError_t e = hipMemcpyAsync(dev_dst, sel->params[net], kParamBytes, hipMemcpyDeviceToDevice,
                                reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? MS_OK : hip_fail(e, "parameter copy");
}

uint32_t ms_selector_trained(const ms_selector *sel) { return sel ? sel->trained : 0u; }

ms_status ms_selector_save(const ms_selector *sel, const char *path) {
  if (!sel || !path) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  std::vector<float> host(2 * (size_t)kNParam);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(host.data(), sel->params[0], kParamBytes, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(host.data() + kNParam, sel->params[1], kParamBytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "parameter download");
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(MS_ERR_INVALID_ARG, std::string("cannot open ") + path + " for writing");
  const uint32_t head[3] = {(uint32_t)kNParam, 2u, sel->trained};
  bool ok = std::fwrite(kMagic, 1, sizeof(kMagic), f) == sizeof(kMagic) &&
            std::fwrite(head, sizeof(uint32_t), 3, f) == 3 &&
            std::fwrite(host.data(), sizeof(float), host.size(), f) == host.size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? MS_OK : fail(MS_ERR_INVALID_ARG, std::string("write failed: ") + path);
}

ms_status ms_selector_load(const char *path, ms_selector **out) {
  if (!out || !path) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  ms_status st = check_init();
  if (st != MS_OK) return st;
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(MS_ERR_INVALID_ARG, std::string("cannot open ") + path);
  char magic[8];
  uint32_t head[3];
  std::vector<float> host(2 * (size_t)kNParam);
  bool ok = std::fread(magic, 1, sizeof(magic), f) == sizeof(magic) && std::memcmp(magic, kMagic, 8) == 0 &&
            std::fread(head, sizeof(uint32_t), 3, f) == 3 && head[0] == (uint32_t)kNParam && head[1] == 2u &&
            std::fread(host.data(), sizeof(float), host.size(), f) == host.size();
  char extra;
  ok = ok && std::fread(&extra, 1, 1, f) == 0;  // nothing after the parameters
  std::fclose(f);
  if (!ok) return fail(MS_ERR_INVALID_ARG, std::string("not a selector file of this library: ") + path);
  st = ms_selector_create(host.data(), host.data() + kNParam, out);
  if (st == MS_OK) (*out)->trained = head[2] & 3u;
  return st;
}

ms_status ms_selector_size_targets(const uint64_t *dev_bytes6, const uint64_t *dev_n, uint64_t count, float *dev_t6,
                                   void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (count == 0) return MS_OK;
  if (!dev_bytes6 || !dev_n || !dev_t6) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  MS_LAUNCH(k_size_targets, blocks(count), kWG, stream, reinterpret_cast<const unsigned long long *>(dev_bytes6),
            reinterpret_cast<const unsigned long long *>(dev_n), (unsigned long long)count, dev_t6);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

ms_status ms_selector_cost_targets(const float *dev_ns6, const uint64_t *dev_n, uint64_t count, float *dev_t6,
                                   void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (count == 0) return MS_OK;
  if (!dev_ns6 || !dev_n || !dev_t6) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  MS_LAUNCH(k_cost_targets, blocks(count), kWG, stream, dev_ns6, reinterpret_cast<const unsigned long long *>(dev_n),
            (unsigned long long)count, dev_t6);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

ms_status ms_selector_train(ms_selector *sel, uint32_t net, const float *dev_x, const float *dev_t, uint64_t count,
                            const ms_train_cfg *cfg, float *host_last_loss, void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!sel || !cfg || !dev_x || !dev_t) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  if (net > MS_NET_COST) return fail(MS_ERR_INVALID_ARG, "net must be MS_NET_SIZE or MS_NET_COST");
  if (count == 0 || count >= (1ull << 31)) return fail(MS_ERR_INVALID_ARG, "count must be in [1, 2^31)");
  if (cfg->epochs == 0 || cfg->batch == 0 || cfg->batch >= (1u << 26))
    return fail(MS_ERR_INVALID_ARG, "epochs >= 1 and batch in [1, 2^26) required");
  if (!(cfg->beta1 >= 0.f && cfg->beta1 < 1.f && cfg->beta2 >= 0.f && cfg->beta2 < 1.f))
    return fail(MS_ERR_INVALID_ARG, "beta out of range");
  const uint64_t batch = std::min<uint64_t>(cfg->batch, count);
  const uint64_t per_epoch = (count + batch - 1) / batch;
  const uint64_t steps = per_epoch * cfg->epochs;
  const unsigned nwg = mlp_grad_workgroups((unsigned)batch);
  // scratch: partial gradients, partial losses, gradient, Adam moments, one loss per step
  const uint64_t words = (uint64_t)nwg * kNParam + nwg + 3ull * kNParam + steps;
  float *buf = static_cast<float *>(rt::alloc(sizeof(float) * words, stream));
  if (!buf) return fail(MS_ERR_OOM, "scratch allocation failed");
  float *gpart = buf, *lpart = gpart + (uint64_t)nwg * kNParam, *grad = lpart + nwg, *m = grad + kNParam,
        *v = m + kNParam, *losses = v + kNParam;
  float *p = sel->params[net];
  hipError_t e = hipSuccess;
  // Adam starts from zero moments (all-zero bits are 0.0f)
  e = launch_fill_u32(reinterpret_cast<unsigned *>(m), 2ull * kNParam, 0u, stream);
  uint64_t step = 0;
  for (uint32_t ep = 0; ep < cfg->epochs && e == hipSuccess; ep++) {
    BatchMap map = epoch_map(cfg->seed, ep, count);
    for (uint64_t j0 = 0; j0 < count && e == hipSuccess; j0 += batch) {
      const unsigned nb = (unsigned)std::min<uint64_t>(batch, count - j0);
      map.j0 = j0;
      e = launch_grad_map(p, dev_x, dev_t, nb, map, gpart, lpart, grad, losses + step, stream);
      step++;
      const float c1 = (float)(1.0 - std::pow((double)cfg->beta1, (double)step));
      const float c2 = (float)(1.0 - std::pow((double)cfg->beta2, (double)step));
      if (e == hipSuccess) e = launch_adam(p, grad, m, v, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, c1, c2, stream);
    }
  }
  if (e == hipSuccess && host_last_loss) {
    std::vector<float> last(per_epoch);
    e = hipMemcpyAsync(last.data(), losses + (steps - per_epoch), sizeof(float) * per_epoch, hipMemcpyDeviceToHost,
                       reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    double sum = 0.0;
    for (float x : last) sum += x;
    *host_last_loss = (float)(sum / (double)per_epoch);
  }
  rt::free(buf, sizeof(float) * words, stream);
  if (e != hipSuccess) return hip_fail(e, "training launch");
  sel->trained |= 1u << net;
  return MS_OK;
}

ms_status ms_selector_pick(const ms_selector *sel, uint32_t objective, const float *dev_x, uint64_t count,
                           uint32_t *dev_kinds, float *dev_pred6, void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!sel) return fail(MS_ERR_INVALID_ARG, "selector is NULL");
  if (objective > MS_OBJ_DECODE) return fail(MS_ERR_INVALID_ARG, "objective must be MS_OBJ_FOOTPRINT or MS_OBJ_DECODE");
  if (count == 0) return MS_OK;
  if (!dev_x || (!dev_kinds && !dev_pred6)) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  if (count >= (1ull << 31)) return fail(MS_ERR_INVALID_ARG, "batch too large");
  hipError_t e = launch_mlp_forward(sel->params[objective == MS_OBJ_FOOTPRINT ? 0 : 1], dev_x, (unsigned)count,
                                    dev_pred6, dev_kinds, stream);
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

ms_status ms_select_argmin(const uint64_t *dev_bytes6, uint64_t count, uint32_t *dev_kinds, void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (count == 0) return MS_OK;
  if (!dev_bytes6 || !dev_kinds) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  MS_LAUNCH(k_argmin6, blocks(count), kWG, stream, reinterpret_cast<const unsigned long long *>(dev_bytes6),
            (unsigned long long)count, dev_kinds);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MS_OK : hip_fail(e, "kernel launch");
}

ms_status ms_select_exhaustive(const ms_column *in, uint64_t *dev_bytes6, uint32_t *dev_kind, void *stream) {
  if (!in || !dev_bytes6 || !dev_kind) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  ms_status st = ms_footprints(in, dev_bytes6, stream);
  if (st != MS_OK) return st;
  return ms_select_argmin(dev_bytes6, 1, dev_kind, stream);
}

ms_status ms_decode_cost(const ms_column *in, uint32_t reps, float *host_ns6, void *stream) {
  ms_status st = check_init();
  if (st != MS_OK) return st;
  if (!in || !host_ns6) return fail(MS_ERR_INVALID_ARG, "NULL argument");
  if (reps == 0) return fail(MS_ERR_INVALID_ARG, "reps must be at least 1");
  ms_column_info ci;
  st = ms_column_info_get(in, stream, &ci);
  if (st != MS_OK) return st;
  const uint64_t bytes = std::max<uint64_t>(4 * ci.n, 16);
  uint32_t *out = static_cast<uint32_t *>(rt::alloc(bytes, stream));
  if (!out) return fail(MS_ERR_OOM, "output allocation failed");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool was_suspended = prof_suspended();
  prof_suspend(true);  // no per-launch events inside the timed region
  for (uint32_t k = 0; k < MS_NUM_KINDS && e == hipSuccess && st == MS_OK; k++) {
    ms_column *c = nullptr;
    st = ms_morph(in, ms_format{k, k == MS_STATIC_BP ? MS_BW_AUTO : 0u}, stream, &c);
    if (st != MS_OK) break;
    st = ms_column_decode(c, out, stream);  // warm: the format's code path and the column in cache alike
    if (st == MS_OK) e = hipEventRecord(e0, s);
    for (uint32_t r = 0; r < reps && st == MS_OK && e == hipSuccess; r++) st = ms_column_decode(c, out, stream);
    if (st == MS_OK && e == hipSuccess) e = hipEventRecord(e1, s);
    if (st == MS_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (st == MS_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    host_ns6[k] = ms * 1e6f / (float)reps;
    ms_column_free(c);
  }
  prof_suspend(was_suspended);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  rt::free(out, bytes, stream);
  if (st != MS_OK) return st;
  return e == hipSuccess ? MS_OK : hip_fail(e, "decode timing");
}

}  // extern "C"
