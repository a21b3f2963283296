// Host-logic checks of the uneven-batch C ABI on the stand-in runtime of
// mock_hip.cpp (no GPU).  Every kernel launch is checked against the memory
// its kernel would touch, every stream capture against unjoined branches and
// every graph launch against unknown or destroyed graphs.  Exit status: the
// number of failed checks plus the stand-in runtime's error count.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <vector>

#include "ispl.h"

int mock_errors();

static int g_fail = 0;
#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      fprintf(stderr, "CHECK failed (line %d): %s  [%s]\n", __LINE__, #cond, \
              ispl_last_error());                                          \
      ++g_fail;                                                            \
    }                                                                      \
  } while (0)

struct Mode {
  int L, N, G, P;
};

struct Setup {
  std::vector<ispl_config> cfgs;
  std::vector<ispl_batch_io> io;
  ispl_batch* b = nullptr;
  hipStream_t user = nullptr;
};

static Setup make(const std::vector<Mode>& modes, int st, int extra) {
  Setup s;
  const size_t ss = st == ISPL_SAMPLES_CI16 ? 4 : 8;
  for (size_t i = 0; i < modes.size(); ++i) {
    const Mode& m = modes[i];
    ispl_config c{};
    c.abi_version = ISPL_ABI_VERSION;
    c.code_len = m.L;
    c.fft_len = m.N;
    c.n_gates = m.G;
    c.gate_step = 25;
    c.first_gate = 3 * static_cast<int>(i);
    c.pulse_stride = c.first_gate + int64_t(m.G - 1) * c.gate_step + m.L + extra;
    c.sample_type = st;
    c.max_pulses = m.P > 0 ? m.P : 1;
    s.cfgs.push_back(c);
    const int rows = m.P > 0 ? m.P : 1;
    void *x = nullptr, *t = nullptr, *o = nullptr;
    hipMalloc(&x, size_t(rows) * c.pulse_stride * ss);
    hipMalloc(&t, size_t(rows) * m.L * 8);
    hipMalloc(&o, size_t(m.G) * m.N * 4);
    s.io.push_back(ispl_batch_io{x, static_cast<const float*>(t), 1, m.P, static_cast<float*>(o)});
  }
  CHECK(ispl_batch_create(s.cfgs.data(), static_cast<int32_t>(modes.size()), &s.b) == ISPL_OK);
  hipStreamCreateWithFlags(&s.user, 0);
  return s;
}

static void release(Setup& s) {
  ispl_batch_destroy(s.b);
  hipStreamDestroy(s.user);
  for (auto& x : s.io) {
    hipFree(const_cast<void*>(x.samples));
    hipFree(const_cast<float*>(x.tx_code));
    hipFree(x.spectra);
  }
}

static void basic_flows(Setup& s) {
  CHECK(ispl_batch_integrate(s.b, s.io.data(), 0, 1, s.user) == ISPL_OK);
  CHECK(ispl_batch_integrate(s.b, s.io.data(), 0, 1, s.user) == ISPL_OK);  // replay
  CHECK(ispl_batch_integrate(s.b, s.io.data(), 0, 0, s.user) == ISPL_OK);  // eager
  CHECK(ispl_batch_integrate(s.b, s.io.data(), 1, 1, s.user) == ISPL_OK);  // recapture
}

int main() {
  const std::vector<Mode> small = {{128, 4096, 7, 9}, {480, 8192, 5, 12}, {1000, 16384, 4, 10},
                                   {2000, 32768, 3, 11}};
  for (int st : {ISPL_SAMPLES_C64, ISPL_SAMPLES_CI16}) {
    Setup s = make(small, st, 11);
    basic_flows(s);
    release(s);
  }
  {  // hand-set plans, valid and invalid
    Setup s = make(small, ISPL_SAMPLES_C64, 11);
    const int wsets[3][4] = {{2, 4, 8, 0}, {1, 1, 2, 0}, {4, 8, 16, 0}};
    for (int k = 0; k < 3; ++k) {
      ispl_batch_plan p{};
      for (int i = 0; i < 4; ++i) {
        p.order[i] = 3 - i;
        p.waves[i] = wsets[k][i];
      }
      p.serial = k == 1;
      CHECK(ispl_batch_set_plan(s.b, &p) == ISPL_OK);
      CHECK(ispl_batch_integrate(s.b, s.io.data(), 0, 1, s.user) == ISPL_OK);
      CHECK(ispl_batch_integrate(s.b, s.io.data(), 0, 0, s.user) == ISPL_OK);
    }
    ispl_batch_plan bad{};
    for (int i = 0; i < 4; ++i) bad.order[i] = i;
    bad.order[1] = 0;
    CHECK(ispl_batch_set_plan(s.b, &bad) == ISPL_ERR_INVALID_ARG);
    release(s);
  }
  {  // a tile shape whose plan wants more chunks than the scratch holds, then an
     // error inside the capture and recovery
    Setup s = make({{128, 4096, 200, 500}, {480, 8192, 5, 12}}, ISPL_SAMPLES_C64, 11);
    ispl_batch_plan p{};
    p.order[0] = 0;
    p.order[1] = 1;
    p.waves[0] = 1;
    CHECK(ispl_batch_set_plan(s.b, &p) == ISPL_OK);
    CHECK(ispl_batch_integrate(s.b, s.io.data(), 0, 1, s.user) == ISPL_OK);
    std::vector<ispl_batch_io> bad = s.io;
    bad[1].n_pulses = 24;  // > max_pulses
    CHECK(ispl_batch_integrate(s.b, bad.data(), 0, 1, s.user) == ISPL_ERR_INVALID_ARG);
    CHECK(ispl_batch_integrate(s.b, s.io.data(), 0, 1, s.user) == ISPL_OK);
    CHECK(ispl_batch_integrate(s.b, s.io.data(), 0, 0, s.user) == ISPL_OK);
    p.serial = 1;
    CHECK(ispl_batch_set_plan(s.b, &p) == ISPL_OK);
    CHECK(ispl_batch_integrate(s.b, bad.data(), 0, 1, s.user) == ISPL_ERR_INVALID_ARG);
    CHECK(ispl_batch_integrate(s.b, s.io.data(), 0, 1, s.user) == ISPL_OK);
    release(s);
  }
  // re-captures right after launches, without a synchronisation in between,
  // more often than the object keeps replaced graphs: no graph may be
  // destroyed while the runtime still completes a launch of it
  {
    Setup s = make(small, ISPL_SAMPLES_C64, 11);
    for (int i = 0; i < 20; ++i) {
      CHECK(ispl_batch_integrate(s.b, s.io.data(), i % 2, 1, s.user) == ISPL_OK);
      CHECK(ispl_batch_integrate(s.b, s.io.data(), i % 2, 1, s.user) == ISPL_OK);
    }
    release(s);
  }
  // the autotuner's host logic on the small modes and on the full-size
  // uneven-batch workload, twice in a row on one object
  for (int full = 0; full < 2; ++full) {
    const std::vector<Mode> modes =
        full ? std::vector<Mode>{{128, 4096, 200, 500}, {480, 8192, 600, 500},
                                 {1000, 16384, 1000, 500}, {2000, 32768, 2000, 500}}
             : small;
    Setup s = make(modes, ISPL_SAMPLES_C64, full ? 0 : 11);
    ispl_batch_plan best{};
    float ms = 0.f;
    CHECK(ispl_batch_integrate(s.b, s.io.data(), 0, 1, s.user) == ISPL_OK);
    CHECK(ispl_batch_tune(s.b, s.io.data(), 3, &best, &ms) == ISPL_OK);
    CHECK(ispl_batch_integrate(s.b, s.io.data(), 0, 1, s.user) == ISPL_OK);
    const ispl_status st = ispl_batch_tune(s.b, s.io.data(), 3, &best, &ms);
    CHECK(st == ISPL_OK);
    bool seen[8] = {};
    for (int i = 0; i < 4; ++i) {
      CHECK(best.order[i] >= 0 && best.order[i] < 4 && !seen[best.order[i]]);
      if (best.order[i] >= 0 && best.order[i] < 4) seen[best.order[i]] = true;
    }
    CHECK(ms > 0.f);
    CHECK(ispl_batch_integrate(s.b, s.io.data(), 0, 1, s.user) == ISPL_OK);
    release(s);
  }
  const int me = mock_errors();
  printf("checks failed: %d, runtime errors: %d\n", g_fail, me);
  return g_fail + me;
}
