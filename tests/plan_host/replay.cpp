// Replays the plan executor's call sequences on the host-only HIP model under
// AddressSanitizer / UndefinedBehaviorSanitizer (test infrastructure): the star plan
// (select -> bitmap -> semi-join per dimension, three intersects, four projections, two
// group-sums) launched as a graph on parallel branches, run eagerly, autotuned right after
// the eager run (twice: timing, then from the cache), re-formatted and relaunched; a
// 512-step batch plan run eagerly on one and on eight branches then autotuned; and the
// error paths of a capture that fails half way.  Exit status 0 and no sanitizer report
// mean no use after free, double free or leak-free misuse was seen.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/morphgpu.h"
#include "model.h"

ms_column *model_input(uint64_t n);
void model_fail_arena_alloc(int index);

namespace {
int g_failures = 0;
#define CHECK(x)                                                                                       \
  do {                                                                                                 \
    ms_status st_ = (x);                                                                               \
    if (st_ != MS_OK) {                                                                                \
      std::fprintf(stderr, "%s:%d %s -> %d (%s)\n", __FILE__, __LINE__, #x, (int)st_, ms_last_error()); \
      g_failures++;                                                                                    \
    }                                                                                                  \
  } while (0)

ms_step step(uint32_t op, int32_t a, int32_t b, uint64_t param = 0, uint32_t kind = MS_DELTA_DYN_BP) {
  ms_step s;
  std::memset(&s, 0, sizeof(s));
  s.op = op;
  s.a = a;
  s.b = b;
  s.cmp = MS_LT;
  s.c0 = 20;
  s.param = param;
  s.out.kind = kind;
  s.out.bit_width = kind == MS_STATIC_BP ? MS_BW_AUTO : 0;
  return s;
}
int32_t inp(int j) { return -1 - j; }

// The star plan over inputs fk0..3, m1, m2, dimattr0..3, dimgroup3.
std::vector<ms_step> star_steps(int *out1, int *out2) {
  const uint64_t D[4] = {200000, 3000000, 2000000, 2500};
  std::vector<ms_step> s;
  int pd[4];
  for (int d = 0; d < 4; d++) {
    s.push_back(step(MS_OP_SELECT, inp(6 + d), -1));
    const int sel = (int)s.size() - 1;
    s.push_back(step(MS_OP_BITMAP, sel, -1, D[d]));
    const int bm = (int)s.size() - 1;
    s.push_back(step(MS_OP_SEMIJOIN, inp(d), bm, D[d]));
    pd[d] = (int)s.size() - 1;
  }
  s.push_back(step(MS_OP_INTERSECT, pd[0], pd[1], 600000000));
  s.push_back(step(MS_OP_INTERSECT, (int)s.size() - 1, pd[2], 600000000));
  s.push_back(step(MS_OP_INTERSECT, (int)s.size() - 1, pd[3], 600000000));
  const int P = (int)s.size() - 1;
  s.push_back(step(MS_OP_PROJECT, inp(4), P, 0, MS_STATIC_BP));
  const int m1p = (int)s.size() - 1;
  s.push_back(step(MS_OP_PROJECT, inp(5), P, 0, MS_STATIC_BP));
  const int m2p = (int)s.size() - 1;
  s.push_back(step(MS_OP_PROJECT, inp(3), P, 0, MS_STATIC_BP));
  const int kp = (int)s.size() - 1;
  s.push_back(step(MS_OP_PROJECT, inp(10), kp, 0, MS_STATIC_BP));
  const int gp = (int)s.size() - 1;
  s.push_back(step(MS_OP_GROUP_SUM, gp, m1p, 250));
  *out1 = (int)s.size() - 1;
  s.push_back(step(MS_OP_GROUP_SUM, gp, m2p, 250));
  *out2 = (int)s.size() - 1;
  for (int k : {0, 2, 9, 12}) s.push_back(step(MS_OP_STATS, k, -1));
  s.push_back(step(MS_OP_FOOTPRINTS, P, -1));
  return s;
}

void read_all(ms_plan *p, const std::vector<ms_step> &s, hipStream_t st) {
  std::vector<unsigned char> buf(1 << 20);
  for (uint32_t i = 0; i < s.size(); i++) {
    const ms_column *c = nullptr;
    void *ptr = nullptr;
    CHECK(ms_plan_result(p, i, &c, &ptr));
    if (s[i].op == MS_OP_BITMAP || s[i].op == MS_OP_SUM || s[i].op == MS_OP_GROUP_SUM ||
        s[i].op == MS_OP_FOOTPRINTS || s[i].op == MS_OP_STATS) {
      uint64_t got = 0;
      CHECK(ms_plan_read_result(p, i, buf.data(), buf.size(), st, &got));
    } else {
      ms_column_info ci;
      CHECK(ms_column_info_get(c, st, &ci));
    }
  }
}

void star_scenario(const char *cache) {
  std::vector<ms_column *> in;
  const uint64_t n = 100000;
  for (int j = 0; j < 11; j++) in.push_back(model_input(j < 6 ? n : 1000));
  int o1 = 0, o2 = 0;
  std::vector<ms_step> s = star_steps(&o1, &o2);
  ms_plan *p = nullptr;
  CHECK(ms_plan_create(s.data(), (uint32_t)s.size(), in.data(), (uint32_t)in.size(), &p));
  hipStream_t st;
  hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  ms_tune t{2, 0};
  CHECK(ms_plan_set_tune(p, &t));
  for (int r = 0; r < 3; r++) CHECK(ms_plan_launch(p, st));
  read_all(p, s, st);
  for (int r = 0; r < 2; r++) CHECK(ms_plan_run(p, st));  // eager, after graph replays
  read_all(p, s, st);
  ms_tune best{};
  float best_ms = 0.f;
  CHECK(ms_plan_autotune(p, st, 2, cache, &best, &best_ms));  // autotune right after an eager run
  read_all(p, s, st);
  CHECK(ms_plan_launch(p, st));
  read_all(p, s, st);
  CHECK(ms_plan_run(p, st));
  ms_format f{MS_DYN_BP, 0};
  CHECK(ms_plan_set_format(p, 14, f));
  CHECK(ms_plan_launch(p, st));
  CHECK(ms_plan_launch(p, st));
  CHECK(ms_plan_autotune(p, st, 2, cache, &best, &best_ms));  // from the cache this time
  CHECK(ms_plan_autotune(p, st, 1, nullptr, &best, &best_ms));
  CHECK(ms_plan_run(p, st));
  t = ms_tune{4, 2, 16};
  CHECK(ms_plan_set_tune(p, &t));
  CHECK(ms_plan_launch(p, st));  // no sync before the next change: set_tune must wait for the replay
  t = ms_tune{8, 8};
  CHECK(ms_plan_set_tune(p, &t));
  CHECK(ms_plan_run(p, st));
  CHECK(ms_plan_launch(p, st));
  CHECK(ms_plan_destroy(p));  // right after a launch, without a sync
  hipStreamSynchronize(st);
  for (ms_column *c : in) ms_column_free(c);
  hipStreamDestroy(st);
}

void batch_scenario(const char *cache) {
  std::vector<ms_column *> in;
  std::vector<ms_step> s;
  for (int t = 0; t < 512; t++) {
    const uint64_t n = 1000 + 37 * (uint64_t)t;
    switch (t % 5) {
      case 0:
        in.push_back(model_input(n));
        s.push_back(step(MS_OP_SELECT, inp((int)in.size() - 1), -1, 0, (uint32_t)(t % 6)));
        break;
      case 1:
        in.push_back(model_input(n));
        in.push_back(model_input(n / 10));
        s.push_back(step(MS_OP_PROJECT, inp((int)in.size() - 2), inp((int)in.size() - 1), 0, (uint32_t)(t % 6)));
        break;
      case 2:
        in.push_back(model_input(n));
        in.push_back(model_input(n / 2));
        s.push_back(step(MS_OP_INTERSECT, inp((int)in.size() - 2), inp((int)in.size() - 1), n, (uint32_t)(t % 6)));
        break;
      case 3:
        in.push_back(model_input(n));
        s.push_back(step(MS_OP_SUM, inp((int)in.size() - 1), -1));
        break;
      default:
        in.push_back(model_input(n));
        s.push_back(step(MS_OP_MORPH, inp((int)in.size() - 1), -1, 0, (uint32_t)(t % 6)));
    }
  }
  ms_plan *p = nullptr;
  CHECK(ms_plan_create(s.data(), (uint32_t)s.size(), in.data(), (uint32_t)in.size(), &p));
  hipStream_t st;
  hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  CHECK(ms_plan_run(p, st));
  CHECK(ms_plan_run(p, st));
  ms_tune t{8, 8};
  CHECK(ms_plan_set_tune(p, &t));
  CHECK(ms_plan_run(p, st));
  CHECK(ms_plan_run(p, st));
  ms_tune best{};
  float best_ms = 0.f;
  CHECK(ms_plan_autotune(p, st, 2, cache, &best, &best_ms));
  CHECK(ms_plan_launch(p, st));
  if (ms_plan_arena_bytes(p) == 0) {
    std::fprintf(stderr, "arena of a launched plan reads 0\n");
    g_failures++;
  }
  read_all(p, s, st);
  CHECK(ms_plan_destroy(p));
  for (ms_column *c : in) ms_column_free(c);
  hipStreamDestroy(st);
}

// A capture that fails half way (an arena allocation refused) must leave the plan usable.
void failing_capture_scenario() {
  std::vector<ms_column *> in;
  for (int j = 0; j < 11; j++) in.push_back(model_input(5000));
  int o1 = 0, o2 = 0;
  std::vector<ms_step> s = star_steps(&o1, &o2);
  ms_plan *p = nullptr;
  CHECK(ms_plan_create(s.data(), (uint32_t)s.size(), in.data(), (uint32_t)in.size(), &p));
  hipStream_t st;
  hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  for (uint32_t b : {1u, 4u}) {
    ms_tune t{b, 0};
    CHECK(ms_plan_set_tune(p, &t));
    CHECK(ms_plan_run(p, st));
    model_fail_arena_alloc(7);
    if (ms_plan_launch(p, st) == MS_OK) {
      std::fprintf(stderr, "a refused arena allocation did not fail the capture\n");
      g_failures++;
    }
    model_fail_arena_alloc(-1);
    CHECK(ms_plan_launch(p, st));
    read_all(p, s, st);
    CHECK(ms_plan_run(p, st));
  }
  CHECK(ms_plan_destroy(p));
  for (ms_column *c : in) ms_column_free(c);
  hipStreamDestroy(st);
}
}  // namespace

int main(int argc, char **argv) {
  const char *cache = argc > 1 ? argv[1] : "plan_tune_cache.txt";
  std::remove(cache);
  star_scenario(cache);
  batch_scenario(cache);
  failing_capture_scenario();
  model::synchronize();
  if (g_failures) {
    std::fprintf(stderr, "%d failing calls\n", g_failures);
    return 1;
  }
  std::printf("replay ok\n");
  return 0;
}
