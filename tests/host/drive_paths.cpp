// Host-logic checks of the single-experiment C ABI on the stand-in runtime of
// mock_hip.cpp (no GPU): the plain path (integration, gate lists, peak pick),
// the zoom DFT, the window network, the learned zoom and the streaming
// ingest, each over several shapes, both sample types, empty pulse sets and
// rejected arguments.  Every launch is checked against the memory its kernel
// would touch; the learned zoom's window decision is replaced by a fixed
// pattern of zoomed and fallback gates so that both branches run.  Exit
// status: the number of failed checks plus the stand-in runtime's errors.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstring>
#include <vector>

#include "ispl.h"

int mock_errors();
long mock_ops();

static int g_fail = 0;
#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      fprintf(stderr, "CHECK failed (line %d): %s  [%s]\n", __LINE__, #cond, \
              ispl_last_error());                                          \
      ++g_fail;                                                            \
    }                                                                      \
  } while (0)

static std::vector<void*> g_bufs;

// Zero-filled stand-in device memory of exactly `bytes` (freed at the end).
template <typename T>
static T* dev(size_t bytes) {
  void* p = nullptr;
  (void)hipMalloc(&p, bytes);
  memset(p, 0, bytes);
  g_bufs.push_back(p);
  return static_cast<T*>(p);
}

struct Shape {
  int L, N, G, P, st, extra;
};

static ispl_config config(const Shape& s) {
  ispl_config c{};
  c.abi_version = ISPL_ABI_VERSION;
  c.code_len = s.L;
  c.fft_len = s.N;
  c.n_gates = s.G;
  c.gate_step = 25;
  c.first_gate = 7;
  c.pulse_stride = c.first_gate + int64_t(s.G - 1) * c.gate_step + s.L + s.extra;
  c.sample_type = s.st;
  c.max_pulses = s.P;
  return c;
}

struct Io {
  const void* samples;
  const float* tx;   // [P][L]
  const float* tx1;  // one shared row [L]
  float* spectra;    // [G][N]
  int32_t* peak_bin;
  float* peak_power;
  int32_t* list;     // [G]
  int32_t* count;
};

static Io buffers(const ispl_config& c) {
  Io io{};
  const size_t ss = c.sample_type == ISPL_SAMPLES_CI16 ? 4 : 8;
  // rows end exactly where the last gate's window ends in the last pulse
  const size_t P = static_cast<size_t>(c.max_pulses);
  io.samples = dev<void>(((P - 1) * c.pulse_stride + c.first_gate +
                          size_t(c.n_gates - 1) * c.gate_step + c.code_len) * ss);
  io.tx = dev<float>(P * c.code_len * 8);
  io.tx1 = dev<float>(size_t(c.code_len) * 8);
  io.spectra = dev<float>(size_t(c.n_gates) * c.fft_len * 4);
  io.peak_bin = dev<int32_t>(size_t(c.n_gates) * 4);
  io.peak_power = dev<float>(size_t(c.n_gates) * 4);
  io.list = dev<int32_t>(size_t(c.n_gates) * 4);
  io.count = dev<int32_t>(4);
  // every third gate, last first
  int n = 0;
  for (int g = c.n_gates - 1; g >= 0; g -= 3) io.list[n++] = g;
  *io.count = n;
  return io;
}

static void plain_path(const Shape& s) {
  const ispl_config c = config(s);
  ispl_ctx* ctx = nullptr;
  CHECK(ispl_create(&c, &ctx) == ISPL_OK);
  if (!ctx) return;
  const Io io = buffers(c);
  for (int P : {s.P, 1, 0, (s.P + 1) / 2}) {
    CHECK(ispl_integrate_spectra(ctx, io.samples, io.tx, 1, P, io.spectra, 0, nullptr) == ISPL_OK);
    CHECK(ispl_integrate_spectra(ctx, io.samples, io.tx1, 0, P, io.spectra, 1, nullptr) == ISPL_OK);
    CHECK(ispl_integrate_spectra_gates(ctx, io.samples, io.tx, 1, P, io.list, io.count, io.spectra,
                                       0, nullptr) == ISPL_OK);
    CHECK(ispl_integrate_spectra_gates(ctx, io.samples, io.tx1, 0, P, io.list, io.count,
                                       io.spectra, 1, nullptr) == ISPL_OK);
  }
  CHECK(ispl_find_plasma_line(ctx, io.spectra, 3, c.fft_len / 2, io.peak_bin, io.peak_power,
                              nullptr) == ISPL_OK);
  CHECK(ispl_find_plasma_line(ctx, io.spectra, c.fft_len - 5, 5, io.peak_bin, nullptr, nullptr) ==
        ISPL_OK);
  CHECK(ispl_find_plasma_line_gates(ctx, io.spectra, 0, c.fft_len, io.list, io.count, io.peak_bin,
                                    io.peak_power, nullptr) == ISPL_OK);
  // rejected without a launch
  CHECK(ispl_integrate_spectra(ctx, io.samples, io.tx, 1, s.P + 1, io.spectra, 0, nullptr) ==
        ISPL_ERR_INVALID_ARG);
  CHECK(ispl_integrate_spectra(ctx, io.samples, io.tx, 1, s.P, nullptr, 0, nullptr) ==
        ISPL_ERR_INVALID_ARG);
  CHECK(ispl_integrate_spectra(ctx, io.samples, io.tx, 2, s.P, io.spectra, 0, nullptr) ==
        ISPL_ERR_INVALID_ARG);
  CHECK(ispl_find_plasma_line(ctx, io.spectra, 4, 4, io.peak_bin, nullptr, nullptr) ==
        ISPL_ERR_INVALID_ARG);
  CHECK(ispl_integrate_spectra_gates(ctx, io.samples, io.tx, 1, s.P, nullptr, io.count,
                                     io.spectra, 0, nullptr) == ISPL_ERR_INVALID_ARG);
  // the same integrations without a context: static scratch only
  for (int P : {s.P, 1, 0}) {
    CHECK(ispl_integrate_spectra_noalloc(&c, io.samples, io.tx, 1, P, io.spectra, 0, nullptr) ==
          ISPL_OK);
    CHECK(ispl_integrate_spectra_noalloc(&c, io.samples, io.tx1, 0, P, io.spectra, 1, nullptr) ==
          ISPL_OK);
  }
  CHECK(ispl_integrate_spectra_noalloc(&c, io.samples, io.tx, 1, s.P + 1, io.spectra, 0,
                                       nullptr) == ISPL_ERR_INVALID_ARG);
  CHECK(ispl_integrate_spectra_noalloc(nullptr, io.samples, io.tx, 1, s.P, io.spectra, 0,
                                       nullptr) == ISPL_ERR_INVALID_ARG);
  int32_t chunks = 0, waves = 0, blocks = 0;
  CHECK(ispl_plan(&c, s.P, &chunks, &waves, &blocks) == ISPL_OK);
  CHECK(chunks >= 1 && waves >= 1 && blocks >= 1);
  ispl_destroy(ctx);
}

static void zoom_path(const Shape& s, int n_bins, int precision) {
  const ispl_config c = config(s);
  ispl_ctx* ctx = nullptr;
  CHECK(ispl_create(&c, &ctx) == ISPL_OK);
  if (!ctx) return;
  ispl_zoom* z = nullptr;
  CHECK(ispl_zoom_create(ctx, n_bins, precision, &z) == ISPL_OK);
  if (z) {
    const Io io = buffers(c);
    int32_t* bin_start = dev<int32_t>(size_t(c.n_gates) * 4);
    for (int g = 0; g < c.n_gates; ++g) bin_start[g] = (g * 131 - 40) % c.fft_len;
    float* win = dev<float>(size_t(c.n_gates) * n_bins * 4);
    for (int P : {s.P, 0, 1, 25, 49}) {
      if (P > s.P) continue;
      CHECK(ispl_zoom_spectra(z, io.samples, io.tx, 1, P, bin_start, win, 0, nullptr) == ISPL_OK);
      CHECK(ispl_zoom_spectra(z, io.samples, io.tx1, 0, P, bin_start, win, 1, nullptr) == ISPL_OK);
      CHECK(ispl_zoom_spectra_gates(z, io.samples, io.tx, 1, P, bin_start, io.list, io.count, win,
                                    0, nullptr) == ISPL_OK);
    }
    CHECK(ispl_zoom_find_peaks(z, win, bin_start, io.list, io.count, io.peak_bin, io.peak_power,
                               nullptr) == ISPL_OK);
    CHECK(ispl_zoom_find_peaks(z, win, bin_start, io.list, io.count, io.peak_bin, nullptr,
                               nullptr) == ISPL_OK);
    CHECK(ispl_zoom_find_peaks(z, win, bin_start, nullptr, io.count, io.peak_bin, nullptr,
                               nullptr) == ISPL_ERR_INVALID_ARG);
    CHECK(ispl_zoom_spectra(z, io.samples, io.tx, 1, s.P + 1, bin_start, win, 0, nullptr) ==
          ISPL_ERR_INVALID_ARG);
    ispl_zoom_destroy(z);
  }
  ispl_zoom* bad = nullptr;
  CHECK(ispl_zoom_create(ctx, 100, precision, &bad) == ISPL_ERR_INVALID_ARG && !bad);
  ispl_destroy(ctx);
}

static void net_path() {
  ispl_net* n = nullptr;
  const int B = 16;
  CHECK(ispl_net_create(0, B, &n) == ISPL_OK);
  if (!n) return;
  std::vector<float> params(ISPL_NET_PARAMS, 0.01f);
  CHECK(ispl_net_set_params(n, params.data()) == ISPL_OK);
  const size_t row = ISPL_NET_LEN * 4;
  float* spectra = dev<float>(3 * B * row);
  float* feats = dev<float>(3 * B * row);
  float* logits = dev<float>(3 * B * row);
  float* target = dev<float>(B * 4);
  float* grad = dev<float>(ISPL_NET_PARAMS * 4);
  float* loss = dev<float>(4);
  CHECK(ispl_net_features(n, spectra, 3 * B, feats, nullptr) == ISPL_OK);
  CHECK(ispl_net_forward(n, feats, B, logits, ISPL_NET_FP32, nullptr) == ISPL_OK);
  CHECK(ispl_net_forward(n, feats, 3 * B, logits, ISPL_NET_BF16, nullptr) == ISPL_OK);
  CHECK(ispl_net_forward(n, feats, B + 1, logits, ISPL_NET_FP32, nullptr) == ISPL_ERR_INVALID_ARG);
  CHECK(ispl_net_loss_grad(n, feats, target, B, grad, loss, nullptr) == ISPL_OK);
  CHECK(ispl_net_train_step(n, feats, target, B, 1e-3f, loss, nullptr) == ISPL_OK);
  CHECK(ispl_net_train_step(n, feats, target, B + 1, 1e-3f, loss, nullptr) == ISPL_ERR_INVALID_ARG);
  CHECK(ispl_net_forward(n, feats, 7, logits, ISPL_NET_BF16, nullptr) == ISPL_OK);  // rebuilt table
  CHECK(ispl_net_get_params(n, params.data()) == ISPL_OK);
  const int G = 3 * B;
  int32_t* bin_start = dev<int32_t>(G * 4);
  float* conf = dev<float>(G * 4);
  int32_t* flag = dev<int32_t>(G * 4);
  int32_t* zl = dev<int32_t>(G * 4);
  int32_t* fl = dev<int32_t>(G * 4);
  int32_t* counts = dev<int32_t>(8);
  for (int rep = 0; rep < 2; ++rep)
    CHECK(ispl_net_select(n, logits, G, 16384, 256, 0.9f, bin_start, conf, flag, zl, fl, counts,
                          nullptr) == ISPL_OK);
  CHECK(counts[0] + counts[1] == G);
  CHECK(ispl_net_select(n, logits, G, 16384, 32, 0.9f, bin_start, conf, flag, zl, fl, counts,
                        nullptr) == ISPL_ERR_INVALID_ARG);
  ispl_net_destroy(n);
}

static void lzoom_path(const Shape& s, int window, int precision) {
  ispl_net* n = nullptr;
  CHECK(ispl_net_create(0, 4, &n) == ISPL_OK);
  if (!n) return;
  const ispl_config c = config(s);
  ispl_lzoom* z = nullptr;
  CHECK(ispl_lzoom_create(&c, n, window, precision, 0.9f, &z) == ISPL_OK);
  if (z) {
    const Io io = buffers(c);
    for (int P : {s.P, 0, 1, (s.P + 3) / 4}) {
      CHECK(ispl_lzoom_peaks(z, io.samples, io.tx, 1, P, io.peak_bin, io.peak_power, nullptr) ==
            ISPL_OK);
      CHECK(ispl_lzoom_peaks(z, io.samples, io.tx1, 0, P, io.peak_bin, nullptr, nullptr) ==
            ISPL_OK);
    }
    CHECK(ispl_lzoom_peaks(z, io.samples, io.tx, 1, s.P + 1, io.peak_bin, nullptr, nullptr) ==
          ISPL_ERR_INVALID_ARG);
    ispl_lzoom_buffers v{};
    CHECK(ispl_lzoom_view(z, &v) == ISPL_OK);
    CHECK(v.n_gates == c.n_gates && v.window_bins == window && v.fine_len == c.fft_len);
    CHECK(v.counts[0] + v.counts[1] == c.n_gates);
    ispl_lzoom_destroy(z);
  }
  ispl_config longer = c;
  longer.code_len = ISPL_NET_LEN + 1;
  longer.pulse_stride += 1 + ISPL_NET_LEN;
  ispl_lzoom* bad = nullptr;
  CHECK(ispl_lzoom_create(&longer, n, window, precision, 0.9f, &bad) == ISPL_ERR_UNSUPPORTED);
  ispl_net_destroy(n);
}

static void stream_path(const Shape& s, int slot_pulses, int n_slots) {
  const ispl_config c = config(s);
  ispl_stream* st = nullptr;
  CHECK(ispl_stream_create(&c, slot_pulses, n_slots, &st) == ISPL_OK);
  if (!st) return;
  float* spectra = dev<float>(size_t(c.n_gates) * c.fft_len * 4);
  hipStream_t user = nullptr;
  (void)hipStreamCreateWithFlags(&user, 0);
  const size_t ss = c.sample_type == ISPL_SAMPLES_CI16 ? 4 : 8;
  for (int i = 0; i < 3 * n_slots + 1; ++i) {
    const int slot = i % n_slots;
    CHECK(ispl_stream_wait_slot(st, slot) == ISPL_OK);
    void* x = ispl_stream_slot_samples(st, slot);
    float* t = ispl_stream_slot_codes(st, slot);
    CHECK(x && t);
    if (!x || !t) break;
    const int P = i % 4 == 3 ? 0 : slot_pulses - (i % slot_pulses);
    memset(x, 1, size_t(slot_pulses) * c.pulse_stride * ss);
    memset(t, 0, size_t(slot_pulses) * c.code_len * 8);
    CHECK(ispl_stream_submit(st, slot, P, i % 2, spectra, i > 0, user) == ISPL_OK);
  }
  CHECK(ispl_stream_submit(st, n_slots, 1, 1, spectra, 1, user) == ISPL_ERR_INVALID_ARG);
  CHECK(ispl_stream_submit(st, 0, slot_pulses + 1, 1, spectra, 1, user) == ISPL_ERR_INVALID_ARG);
  CHECK(ispl_stream_slot_samples(st, -1) == nullptr);
  CHECK(ispl_stream_sync(st) == ISPL_OK);
  ispl_stream_destroy(st);
  (void)hipStreamDestroy(user);
}

int main() {
  const Shape shapes[] = {
      {256, 1024, 64, 100, ISPL_SAMPLES_C64, 25},     // zoom workload, coarse length
      {1000, 16384, 37, 30, ISPL_SAMPLES_CI16, 0},    // realistic code and transform
      {2000, 32768, 5, 7, ISPL_SAMPLES_C64, 3},       // long code: sixteen-wave sub-transforms
      {16384, 16384, 3, 4, ISPL_SAMPLES_C64, 25},     // the paper's code: sign bits, LDS prefetch
      {5000, 32768, 2, 9, ISPL_SAMPLES_CI16, 1},      // long code, partly filled last region
      {1024, 2048, 3, 1, ISPL_SAMPLES_CI16, 1},       // L = SUB, one pulse
      {1, 1024, 1, 2, ISPL_SAMPLES_C64, 0},           // one sample, one gate
      {300, 4096, 700, 80, ISPL_SAMPLES_CI16, 5},     // many gates, one-wave tiles
  };
  for (const Shape& s : shapes) plain_path(s);
  zoom_path({256, 16384, 64, 100, ISPL_SAMPLES_C64, 25}, 256, ISPL_ZOOM_FP16X3);
  zoom_path({256, 16384, 64, 100, ISPL_SAMPLES_CI16, 0}, 384, ISPL_ZOOM_BF16X3);
  zoom_path({1000, 16384, 300, 60, ISPL_SAMPLES_CI16, 0}, 128, ISPL_ZOOM_FP16X3);
  net_path();
  lzoom_path({256, 16384, 64, 100, ISPL_SAMPLES_C64, 25}, 256, ISPL_ZOOM_FP16X3);
  lzoom_path({256, 16384, 700, 300, ISPL_SAMPLES_CI16, 0}, 256, ISPL_ZOOM_FP16X3);
  lzoom_path({500, 8192, 9, 13, ISPL_SAMPLES_C64, 2}, 128, ISPL_ZOOM_BF16X3);
  stream_path({1000, 16384, 37, 30, ISPL_SAMPLES_CI16, 0}, 10, 3);
  stream_path({4000, 16384, 3, 20, ISPL_SAMPLES_C64, 25}, 4, 2);
  stream_path({256, 1024, 64, 100, ISPL_SAMPLES_C64, 25}, 7, 2);
  for (void* p : g_bufs) (void)hipFree(p);
  const int me = mock_errors();
  printf("stream operations checked: %ld\n", mock_ops());
  printf("checks failed: %d, runtime errors: %d\n", g_fail, me);
  return g_fail + me;
}
