// Replay of the benchmark's call sequence through the real column library host code
// (csrc/ms_api.hip) and plan executor (csrc/ms_plan.hip) against the host model of the
// runtime and the kernel stand-ins (test infrastructure, no GPU).  Device memory comes
// from allocator callbacks whose frees are stream ordered, as with a caching allocator.
// Sequence, per output-format policy of the star plan: a probe plan with statistics and
// footprint steps run eagerly and read back; a separate plan run eagerly twice and
// destroyed; a plan autotuned through the tune cache, launched and replayed, its results
// inspected, re-tuned to one branch and run eagerly, then destroyed; a plan with batched
// persistent launches run eagerly twice, captured and replayed; input columns morphed into
// every format and plans over them launched and destroyed.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/morphgpu.h"
#include "model.h"

#define CHECK(x)                                                                          \
  do {                                                                                    \
    ms_status st_ = (x);                                                                  \
    if (st_ != MS_OK) {                                                                   \
      std::fprintf(stderr, "%s:%d: %s -> %d (%s)\n", __FILE__, __LINE__, #x, (int)st_,    \
                   ms_last_error());                                                      \
      std::exit(1);                                                                       \
    }                                                                                     \
  } while (0)

namespace {
long g_live = 0;

void *dev_alloc(uint64_t bytes, void *stream, void *) {
  (void)stream;
  g_live++;
  return std::calloc(1, bytes ? bytes : 1);
}
void dev_free(void *p, uint64_t, void *stream, void *) {
  g_live--;
  model::submit(reinterpret_cast<hipStream_t>(stream), [p]() { std::free(p); });
}

constexpr uint64_t kDims[4] = {2000, 30000, 20000, 250};
constexpr uint64_t kFact = 300001;
// inputs in plan order: fk0..fk3, m1, m2, dimattr0..dimattr3, dimgroup3

uint32_t mix(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return (uint32_t)(x ^ (x >> 31));
}

// Input j of the star plan, encoded in `fmt`.
ms_column *input(int j, ms_format fmt, hipStream_t s) {
  uint64_t n = j < 6 ? kFact : kDims[j < 10 ? j - 6 : 3];
  std::vector<uint32_t> v(n);
  for (uint64_t i = 0; i < n; i++) {
    uint32_t r = mix(1000 * j + i);
    v[i] = j < 4 ? r % kDims[j] : j == 4 ? 1 + r % 99999 : j == 5 ? r % 11 : j < 10 ? r % 100 : (uint32_t)(i / 10);
  }
  uint32_t *dev = static_cast<uint32_t *>(std::aligned_alloc(256, ((4 * n + 255) / 256) * 256 + 256));
  std::memcpy(dev, v.data(), 4 * n);
  ms_column *c = nullptr;
  CHECK(ms_column_encode(dev, n, fmt, s, &c));
  std::free(dev);  // the encoder synchronises
  return c;
}

struct Star {
  std::vector<ms_step> steps;
  std::vector<uint32_t> names;  // column intermediates
  uint32_t out1 = 0, out2 = 0;
  std::vector<uint32_t> stats, fps;
};

ms_step step(uint32_t op, int32_t a, int32_t b, ms_format out, uint32_t cmp = 0, uint32_t c0 = 0, uint64_t param = 0) {
  ms_step s;
  std::memset(&s, 0, sizeof(s));
  s.op = op;
  s.a = a;
  s.b = b;
  s.cmp = cmp;
  s.c0 = c0;
  s.param = param;
  s.out = out;
  return s;
}

Star star_plan(const uint32_t kinds[15], bool extra) {
  Star p;
  auto add = [&](ms_step s, bool named) {
    p.steps.push_back(s);
    const uint32_t i = (uint32_t)p.steps.size() - 1;
    if (named) p.names.push_back(i);
    return (int32_t)i;
  };
  auto f = [&](int k) { return ms_format{kinds[k], kinds[k] == MS_STATIC_BP ? MS_BW_AUTO : 0u}; };
  int32_t pd[4];
  int k = 0;
  for (int d = 0; d < 4; d++) {
    const int32_t s = add(step(MS_OP_SELECT, -1 - (6 + d), -1, f(k++), MS_LT, 20), true);
    const int32_t bm = add(step(MS_OP_BITMAP, s, -1, ms_format{0, 0}, 0, 0, kDims[d]), false);
    pd[d] = add(step(MS_OP_SEMIJOIN, -1 - d, bm, f(k++), 0, 0, kDims[d]), true);
  }
  int32_t q = add(step(MS_OP_INTERSECT, pd[0], pd[1], f(k++), 0, 0, kFact), true);
  q = add(step(MS_OP_INTERSECT, q, pd[2], f(k++), 0, 0, kFact), true);
  q = add(step(MS_OP_INTERSECT, q, pd[3], f(k++), 0, 0, kFact), true);
  const int32_t m1p = add(step(MS_OP_PROJECT, -1 - 4, q, f(k++)), true);
  const int32_t m2p = add(step(MS_OP_PROJECT, -1 - 5, q, f(k++)), true);
  const int32_t kp = add(step(MS_OP_PROJECT, -1 - 3, q, f(k++)), true);
  const int32_t gp = add(step(MS_OP_PROJECT, -1 - 10, kp, f(k++)), true);
  p.out1 = (uint32_t)add(step(MS_OP_GROUP_SUM, gp, m1p, ms_format{0, 0}, 0, 0, 250), false);
  p.out2 = (uint32_t)add(step(MS_OP_GROUP_SUM, gp, m2p, ms_format{0, 0}, 0, 0, 250), false);
  if (extra) {
    const std::vector<uint32_t> names = p.names;
    for (uint32_t i : names) {
      p.stats.push_back((uint32_t)add(step(MS_OP_STATS, (int32_t)i, -1, ms_format{0, 0}), false));
      p.fps.push_back((uint32_t)add(step(MS_OP_FOOTPRINTS, (int32_t)i, -1, ms_format{0, 0}), false));
    }
  }
  return p;
}

ms_plan *make(const Star &st, const std::vector<ms_column *> &in) {
  ms_plan *p = nullptr;
  CHECK(ms_plan_create(st.steps.data(), (uint32_t)st.steps.size(), in.data(), (uint32_t)in.size(), &p));
  return p;
}

void read_results(ms_plan *p, const Star &st, hipStream_t s) {
  std::vector<unsigned char> buf(2000);
  uint64_t got = 0;
  CHECK(ms_plan_read_result(p, st.out1, buf.data(), buf.size(), s, &got));
  CHECK(ms_plan_read_result(p, st.out2, buf.data(), buf.size(), s, &got));
  for (uint32_t i : st.stats) CHECK(ms_plan_read_result(p, i, buf.data(), 128, s, &got));
  for (uint32_t i : st.fps) CHECK(ms_plan_read_result(p, i, buf.data(), 48, s, &got));
}

void inspect_columns(ms_plan *p, const Star &st, hipStream_t s) {
  for (uint32_t i : st.names) {
    const ms_column *c = nullptr;
    CHECK(ms_plan_result(p, i, &c, nullptr));
    ms_column_info ci;
    CHECK(ms_column_info_get(c, s, &ci));
  }
}

void policy(const uint32_t kinds[15], const std::vector<ms_column *> &in, hipStream_t s, const char *cache) {
  Star st = star_plan(kinds, false);
  // eager timing on its own plan
  ms_plan *pe = make(st, in);
  CHECK(ms_plan_run(pe, s));
  CHECK(ms_plan_run(pe, s));
  read_results(pe, st, s);
  CHECK(ms_plan_destroy(pe));
  // autotune, graph replays, inspection
  ms_plan *p = make(st, in);
  ms_tune best;
  float ms = 0.f;
  CHECK(ms_plan_autotune(p, s, 2, cache, &best, &ms));
  CHECK(ms_plan_launch(p, s));
  for (int r = 0; r < 3; r++) CHECK(ms_plan_launch(p, s));
  read_results(p, st, s);
  inspect_columns(p, st, s);
  CHECK(ms_plan_destroy(p));
  // batched persistent launches level by level: eager, then captured and replayed
  for (uint32_t b : {1u, 4u}) {  // the plain launches of a phase on one stream, then on four branches
    ms_plan *pb = make(st, in);
    ms_tune bt{b, best.wg_per_cu, best.chunks_per_wg, 1};
    CHECK(ms_plan_set_tune(pb, &bt));
    CHECK(ms_plan_run(pb, s));
    read_results(pb, st, s);
    CHECK(ms_plan_run(pb, s));
    CHECK(ms_plan_launch(pb, s));
    for (int r = 0; r < 2; r++) CHECK(ms_plan_launch(pb, s));
    read_results(pb, st, s);
    inspect_columns(pb, st, s);
    CHECK(ms_plan_destroy(pb));
  }
  // the profiled eager run on one branch
  ms_plan *pr = make(st, in);
  ms_tune one{1, best.wg_per_cu, best.chunks_per_wg};
  CHECK(ms_plan_set_tune(pr, &one));
  CHECK(ms_plan_run(pr, s));
  read_results(pr, st, s);
  CHECK(ms_plan_set_tune(pr, &best));
  CHECK(ms_plan_destroy(pr));
  CHECK(ms_sync(s));
}
}  // namespace

int main(int argc, char **argv) {
  const char *cache = argc > 1 ? argv[1] : nullptr;
  CHECK(ms_init(dev_alloc, dev_free, nullptr));
  hipStream_t s = nullptr;
  hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  std::vector<ms_column *> base, plain;
  for (int j = 0; j < 11; j++) {
    base.push_back(input(j, ms_format{MS_STATIC_BP, MS_BW_AUTO}, s));
    plain.push_back(input(j, ms_format{MS_UNCOMPR, 0}, s));
  }
  // the probe: statistics and footprints of every intermediate
  uint32_t dflt[15];
  for (int k = 0; k < 15; k++) dflt[k] = k < 11 ? MS_DELTA_DYN_BP : MS_STATIC_BP;
  {
    Star st = star_plan(dflt, true);
    ms_plan *p = make(st, base);
    CHECK(ms_plan_run(p, s));
    read_results(p, st, s);
    CHECK(ms_plan_destroy(p));
  }
  // policies: plain (uncompressed inputs and intermediates), then every uniform format and a mix
  uint32_t kinds[15];
  for (int k = 0; k < 15; k++) kinds[k] = MS_UNCOMPR;
  policy(kinds, plain, s, cache);
  for (uint32_t u = 0; u < MS_NUM_KINDS; u++) {
    for (int k = 0; k < 15; k++) kinds[k] = u;
    policy(kinds, base, s, cache);
  }
  for (int k = 0; k < 15; k++) kinds[k] = (uint32_t)((k * 5 + 1) % MS_NUM_KINDS);
  policy(kinds, base, s, cache);
  policy(kinds, base, s, cache);  // the tune now comes from the cache
  // greedy-style trials: every input in every other format, a fresh plan each
  for (int j = 0; j < 11; j++) {
    for (uint32_t kk = 0; kk < MS_NUM_KINDS; kk++) {
      ms_column *m = nullptr;
      CHECK(ms_morph(base[j], ms_format{kk, kk == MS_STATIC_BP ? MS_BW_AUTO : 0u}, s, &m));
      std::vector<ms_column *> in = base;
      in[j] = m;
      Star st = star_plan(dflt, false);
      ms_plan *p = make(st, in);
      ms_tune t{2, 0, 0};
      CHECK(ms_plan_set_tune(p, &t));
      CHECK(ms_plan_launch(p, s));
      CHECK(ms_plan_launch(p, s));
      read_results(p, st, s);
      CHECK(ms_plan_destroy(p));
      CHECK(ms_column_free(m));
    }
  }
  CHECK(ms_sync(s));
  for (ms_column *c : base) CHECK(ms_column_free(c));
  for (ms_column *c : plain) CHECK(ms_column_free(c));
  hipStreamSynchronize(s);
  hipStreamDestroy(s);
  model::synchronize();
  if (g_live != 0) {
    std::fprintf(stderr, "%ld device allocations not freed\n", g_live);
    return 1;
  }
  std::printf("api replay ok\n");
  return 0;
}
