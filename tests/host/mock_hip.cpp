// Host-only stand-in for the HIP runtime and the device launchers, so that the
// C-ABI layer's host logic (plans, scratch sizes, stream capture of the batch
// graph, error paths) runs under AddressSanitizer on a machine without a GPU.
// Test infrastructure only.  "Device" memory is host memory; every launcher
// checks the footprint its kernel would read and write against the live
// allocations; stream capture tracks fork and join like the real API (an
// unjoined branch at the end of a capture, a launch of an unknown or destroyed
// graph, a capture on a capturing stream are all counted as errors).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cassert>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "ispl_internal.h"

static std::map<uintptr_t, size_t> g_allocs;
static int g_errors = 0;

static bool check_range(const void* p, size_t bytes, const char* what) {
  if (bytes == 0) return true;
  uintptr_t a = reinterpret_cast<uintptr_t>(p);
  auto it = g_allocs.upper_bound(a);
  if (it == g_allocs.begin()) {
    fprintf(stderr, "MOCK OOB: %s %p (+%zu) not in any allocation\n", what, p, bytes);
    ++g_errors;
    return false;
  }
  --it;
  if (a < it->first || a + bytes > it->first + it->second) {
    fprintf(stderr, "MOCK OOB: %s %p +%zu outside [%p, +%zu)\n", what, p, bytes,
            reinterpret_cast<void*>(it->first), it->second);
    ++g_errors;
    return false;
  }
  return true;
}

static void mock_fail(const char* what) {
  fprintf(stderr, "MOCK: %s\n", what);
  ++g_errors;
}

int mock_errors() { return g_errors; }

static long g_ops = 0;  // stream operations executed (eagerly or by a graph replay)
long mock_ops() { return g_ops; }

struct MStream;
struct MGraph {
  std::vector<std::function<void()>> ops;
};
struct MExec {
  std::vector<std::function<void()>> ops;
  bool alive = true;
  int inflight = 0;  // launches whose completion bookkeeping has not run yet
};

// Completion of graph launches, as a runtime's own completion thread does it:
// a launch's operations run at once (stream order is kept by running every
// operation on the calling thread), its event markers are signalled at once,
// but the release of the launch's references to the executable graph happens
// later, on this thread.  Only hipDeviceSynchronize waits for those releases;
// stream and event synchronisation do not.  Destroying an executable while a
// release is pending is an error of the caller (reported at the destroy), and
// the late release then touches freed memory (reported by AddressSanitizer).
namespace completion {
std::mutex mu;
std::condition_variable cv, drained;
std::deque<std::pair<MExec*, std::chrono::steady_clock::time_point>> pending;
std::thread worker;
bool stop = false;

void run() {
  std::unique_lock<std::mutex> lock(mu);
  for (;;) {
    cv.wait(lock, [] { return stop || !pending.empty(); });
    if (pending.empty()) return;
    const auto due = pending.front().second;
    if (cv.wait_until(lock, due, [] { return stop && pending.empty(); })) return;
    if (std::chrono::steady_clock::now() < due) continue;
    MExec* e = pending.front().first;
    pending.pop_front();
    e->inflight -= 1;  // the runtime's release of its reference
    if (pending.empty()) drained.notify_all();
  }
}

void start() {
  if (!worker.joinable()) worker = std::thread(run);
}

void launched(MExec* e) {
  std::lock_guard<std::mutex> lock(mu);
  start();
  e->inflight += 1;
  pending.emplace_back(e, std::chrono::steady_clock::now() + std::chrono::milliseconds(20));
  cv.notify_all();
}

void drain() {
  std::unique_lock<std::mutex> lock(mu);
  drained.wait(lock, [] { return pending.empty(); });
}

struct Joiner {
  ~Joiner() {
    {
      std::lock_guard<std::mutex> lock(mu);
      stop = true;
    }
    cv.notify_all();
    if (worker.joinable()) worker.join();
  }
} joiner;
}  // namespace completion
struct MEvent {
  int capture = 0;  // capture id it was recorded in (0: eager)
  MStream* from = nullptr;
};
struct MStream {
  int capture = 0;     // capture id, 0 when not capturing
  bool origin = false;
  bool joined = true;  // for non-origin members: rejoined the origin
  MGraph* graph = nullptr;
};
static std::set<MStream*> g_streams;
static std::set<MEvent*> g_events;
static std::set<MGraph*> g_graphs;
static std::set<MExec*> g_execs;
static int g_next_capture = 1;
static MStream g_null_stream;

static MStream* S(hipStream_t s) {
  if (!s) return &g_null_stream;
  MStream* m = reinterpret_cast<MStream*>(s);
  if (!g_streams.count(m)) {
    fprintf(stderr, "MOCK: unknown stream %p\n", (void*)s);
    ++g_errors;
    return &g_null_stream;
  }
  return m;
}

// Records an operation on a stream: executed now, or captured into the graph.
static void run_on(hipStream_t s, std::function<void()> op) {
  MStream* m = S(s);
  auto counted = [op] {
    ++g_ops;
    op();
  };
  if (m->capture) {
    m->graph->ops.push_back(counted);
  } else {
    counted();
  }
}

extern "C" {

hipError_t hipGetDeviceCount(int* c) { *c = 1; return hipSuccess; }
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int) {
  memset(p, 0, sizeof(*p));
  strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
  p->multiProcessorCount = 256;
  return hipSuccess;
}
static int g_dev = 0;
hipError_t hipGetDevice(int* d) { *d = g_dev; return hipSuccess; }
hipError_t hipSetDevice(int d) { g_dev = d; return hipSuccess; }
hipError_t hipDeviceSynchronize() {
  completion::drain();
  return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "mock error"; }

hipError_t hipMalloc(void** p, size_t n) {
  *p = malloc(n ? n : 1);
  g_allocs[reinterpret_cast<uintptr_t>(*p)] = n;
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  auto it = g_allocs.find(reinterpret_cast<uintptr_t>(p));
  if (it == g_allocs.end()) {
    fprintf(stderr, "MOCK: hipFree of unknown %p\n", p);
    ++g_errors;
    return hipErrorInvalidValue;
  }
  g_allocs.erase(it);
  free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k) {
  if (k != hipMemcpyDeviceToHost) check_range(d, n, "memcpy dst");
  if (k != hipMemcpyHostToDevice) check_range(s, n, "memcpy src");
  memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st) {
  run_on(st, [=] { (void)hipMemcpy(d, s, n, k); });
  return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void* d, size_t dp, const void* s, size_t sp, size_t w, size_t h,
                            hipMemcpyKind k, hipStream_t st) {
  run_on(st, [=] {
    for (size_t r = 0; r < h; ++r) {
      if (k != hipMemcpyDeviceToHost) check_range((char*)d + r * dp, w, "memcpy2d dst");
      if (k != hipMemcpyHostToDevice) check_range((const char*)s + r * sp, w, "memcpy2d src");
    }
  });
  return hipSuccess;
}
hipError_t hipMemset(void* d, int v, size_t n) {
  check_range(d, n, "memset");
  memset(d, v, n);
  return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  MStream* m = new MStream;
  g_streams.insert(m);
  *s = reinterpret_cast<hipStream_t>(m);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  MStream* m = S(s);
  if (m->capture) { fprintf(stderr, "MOCK: destroying a capturing stream\n"); ++g_errors; }
  g_streams.erase(m);
  delete m;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) {
  MEvent* m = new MEvent;
  g_events.insert(m);
  *e = reinterpret_cast<hipEvent_t>(m);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  MEvent* m = reinterpret_cast<MEvent*>(e);
  if (!g_events.erase(m)) { fprintf(stderr, "MOCK: unknown event destroyed\n"); ++g_errors; }
  delete m;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  MEvent* ev = reinterpret_cast<MEvent*>(e);
  if (!g_events.count(ev)) { fprintf(stderr, "MOCK: record of unknown event\n"); ++g_errors; return hipErrorInvalidValue; }
  MStream* m = S(s);
  ev->capture = m->capture;
  ev->from = m;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  MEvent* ev = reinterpret_cast<MEvent*>(e);
  if (ev->capture) { fprintf(stderr, "MOCK: synchronize on a captured event\n"); ++g_errors; }
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 1.0f + (rand() % 100) * 0.01f;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  MStream* m = S(s);
  MEvent* ev = reinterpret_cast<MEvent*>(e);
  if (ev->capture) {
    if (m->capture == 0) {  // joins the capture as a forked branch
      m->capture = ev->capture;
      m->origin = false;
      m->joined = false;
      m->graph = ev->from->graph;
    } else if (m->capture != ev->capture) {
      fprintf(stderr, "MOCK: wait across two captures\n");
      ++g_errors;
    } else if (m->origin && ev->from != m) {
      ev->from->joined = true;  // branch rejoined
    }
  } else if (m->capture) {
    fprintf(stderr, "MOCK: capturing stream waits on an eager event\n");
    ++g_errors;
  }
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  MStream* m = S(s);
  if (m->capture) { fprintf(stderr, "MOCK: begin capture twice\n"); ++g_errors; return hipErrorIllegalState; }
  m->capture = g_next_capture++;
  m->origin = true;
  m->graph = new MGraph;
  g_graphs.insert(m->graph);
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  MStream* m = S(s);
  if (!m->capture || !m->origin) { fprintf(stderr, "MOCK: end capture on a non-origin\n"); ++g_errors; return hipErrorIllegalState; }
  bool unjoined = false;
  for (MStream* o : g_streams)
    if (o != m && o->capture == m->capture) {
      if (!o->joined) unjoined = true;
      o->capture = 0;
      o->graph = nullptr;
      o->joined = true;
    }
  m->capture = 0;
  m->origin = false;
  MGraph* gr = m->graph;
  m->graph = nullptr;
  if (unjoined) {
    fprintf(stderr, "MOCK: end capture with an unjoined branch\n");
    ++g_errors;
    g_graphs.erase(gr);
    delete gr;
    *g = nullptr;
    return hipErrorStreamCaptureUnjoined;
  }
  *g = reinterpret_cast<hipGraph_t>(gr);
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  MGraph* gr = reinterpret_cast<MGraph*>(g);
  if (!g_graphs.count(gr)) { fprintf(stderr, "MOCK: instantiate unknown graph\n"); ++g_errors; return hipErrorInvalidValue; }
  MExec* e = new MExec;
  e->ops = gr->ops;
  g_execs.insert(e);
  *x = reinterpret_cast<hipGraphExec_t>(e);
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  MGraph* gr = reinterpret_cast<MGraph*>(g);
  if (!g_graphs.erase(gr)) { fprintf(stderr, "MOCK: destroy unknown graph\n"); ++g_errors; return hipErrorInvalidValue; }
  delete gr;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  MExec* e = reinterpret_cast<MExec*>(x);
  if (!g_execs.erase(e)) { fprintf(stderr, "MOCK: destroy unknown exec\n"); ++g_errors; return hipErrorInvalidValue; }
  {
    std::lock_guard<std::mutex> lock(completion::mu);
    if (e->inflight > 0) {
      fprintf(stderr, "MOCK: executable graph destroyed while %d launch(es) of it are still "
              "being completed by the runtime\n", e->inflight);
      ++g_errors;
    }
  }
  delete e;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  MExec* e = reinterpret_cast<MExec*>(x);
  if (!g_execs.count(e)) { fprintf(stderr, "MOCK: launch unknown exec\n"); ++g_errors; return hipErrorInvalidValue; }
  if (S(s)->capture) { fprintf(stderr, "MOCK: graph launch into a capture\n"); ++g_errors; }
  for (auto& op : e->ops) op();
  completion::launched(e);
  return hipSuccess;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// launchers: footprint checks

namespace ispl {

// The gates a launch works on: all of them, or list[i] for i < min(*count, cap)
// inside [0, G) (the kernels skip other entries).
static std::vector<int> active_gates(const int32_t* list, const int32_t* count, int G, int cap) {
  std::vector<int> gs;
  if (!list) {
    for (int g = 0; g < G; ++g) gs.push_back(g);
    return gs;
  }
  if (!check_range(count, 4, "gate count")) return gs;
  const int n = std::min(std::max(*count, 0), cap);
  if (!check_range(list, size_t(n) * 4, "gate list")) return gs;
  for (int i = 0; i < n; ++i)
    if (list[i] >= 0 && list[i] < G) gs.push_back(list[i]);
  return gs;
}

// Rows [p][first + g step, + len) of pulses p < P for the gates gs.
static void check_windows(const void* samples, size_t ss, int64_t stride, int64_t first,
                          int64_t step, int64_t len, int P, const std::vector<int>& gs,
                          const char* what) {
  if (P < 1) return;
  for (int g : gs) {
    const int64_t last = int64_t(P - 1) * stride + first + g * step + len;
    check_range(samples, size_t(last) * ss, what);
  }
}

static void check_rows(const void* base, int64_t row_len, const std::vector<int>& gs,
                       const char* what) {
  for (int g : gs)
    check_range(static_cast<const float*>(base) + g * row_len, size_t(row_len) * 4, what);
}

static void check_pulse_exponents(const void* samples, int st, const float* tx, int64_t stride,
                                  int64_t lo, int64_t hi, int L, int per_pulse, int P,
                                  const int32_t* exps) {
  if (P < 1 || !exps) return;
  if (lo < 0 || hi < lo || hi > stride) mock_fail("pulse exponents: span outside the row");
  check_range(samples, size_t(int64_t(P - 1) * stride + hi) * (st == 1 ? 4 : 8), "exp samples");
  check_range(tx, size_t(per_pulse ? P : 1) * L * 8, "exp tx");
  check_range(exps, size_t(P) * 4, "exp out");
}

// Code sign bits of the zoom's pulse pass: rows x words words and one flag per row.
static void check_code_bits(const float* tx, int L, int per_pulse, int P, int words,
                            const uint32_t* bits, const int32_t* binary) {
  if (P < 1 || !bits) return;
  if (words * 32 < L) mock_fail("code bits: fewer words than codes");
  const int rows = per_pulse ? P : 1;
  check_range(tx, size_t(rows) * L * 8, "bits tx");
  check_range(bits, size_t(rows) * words * 4, "code bits");
  check_range(binary, size_t(rows) * 4, "code binary");
}


int fused_lds_bytes(int rw, int sub_len) {
  const int XWAVE = 16 * 65;
  if (sub_len == 16 * SUB) return 8 * 16 * XWAVE;
  if (rw == 1) return 8 * XWAVE;
  return 8 * (rw * XWAVE + (rw == 16 ? 2 : 1) * SUB);
}

hipError_t launch_fused(const FusedArgs& a, hipStream_t st) {
  FusedArgs c = a;
  run_on(st, [c] {
    const size_t ss = c.sample_type == 1 ? 4 : 8;
    const int R = 1 << c.log2_r;
    if (c.sub_len * R != c.n_fft) { fprintf(stderr, "MOCK: fused sub_len * R != N\n"); ++g_errors; }
    if (c.sub_len == SUB) {
      if (c.waves_per_block < 1 || c.waves_per_block > 16 || R % c.waves_per_block) {
        fprintf(stderr, "MOCK: fused rw %d with R %d\n", c.waves_per_block, R); ++g_errors;
      }
    }
    const std::vector<int> gs = active_gates(c.gate_list, c.gate_count, c.n_gates, c.n_gates);
    if (c.n_pulses > 0) {
      check_windows(c.samples, ss, c.stride, c.first_gate, c.gate_step, c.code_len, c.n_pulses,
                    gs, "fused samples");
      check_range(c.tx, size_t(c.tx_per_pulse ? c.n_pulses : 1) * c.code_len * 8, "fused tx");
    }
    if (c.chunks < 1) mock_fail("fused: no pulse chunk");
    check_range(c.twiddle, size_t(c.n_fft) * 8, "fused twiddle");
    if (c.code_bits) {  // sign bits of every code row the launch reads
      if (c.code_len <= 2 * SUB) mock_fail("fused: code bits for a code of at most 2 SUB");
      const size_t rows = c.tx_per_pulse ? size_t(c.n_pulses) : 1;
      check_range(c.code_bits, rows * CODE_BITS_WORDS * 2, "fused code bits");
      check_range(c.code_binary, rows * 4, "fused code flags");
    }
    if (c.adapt_target > 0) {  // chunk count from the list length, rows by list slot
      if (!c.gate_list) mock_fail("fused: adaptive chunking without a list");
      const int zg = c.sub_len == SUB ? R / c.waves_per_block : R;
      const int k = static_cast<int>(gs.size());
      const int C = adaptive_chunks(k, zg, c.adapt_target, c.adapt_max_chunks, c.adapt_rows);
      if (C == 1) {
        check_rows(c.out, c.n_fft, gs, "fused out");
      } else {
        if (C * k > c.adapt_rows) mock_fail("fused: adaptive partial rows overflow");
        check_range(c.adapt_partial, size_t(C) * k * c.n_fft * 4, "fused adaptive partial");
      }
      return;
    }
    for (int k = 0; k < c.chunks; ++k)
      check_rows(c.out + int64_t(k) * c.n_gates * c.n_fft, c.n_fft, gs, "fused out");
  });
  return hipSuccess;
}
// The static array of the entry point that allocates nothing: one host block
// that stays registered (the library never frees it).
hipError_t noalloc_scratch(int device, unsigned char** base) {
  static unsigned char* block = nullptr;
  if (device != 0) return hipErrorInvalidDevice;
  if (!block) {
    block = static_cast<unsigned char*>(malloc(ISPL_NOALLOC_SCRATCH_BYTES));
    g_allocs[reinterpret_cast<uintptr_t>(block)] = ISPL_NOALLOC_SCRATCH_BYTES;
  }
  *base = block;
  return hipSuccess;
}
hipError_t launch_build_twiddles(float* table, int32_t n_fft, hipStream_t st) {
  run_on(st, [=] {
    if (n_fft < 1 || size_t(n_fft) * 8 > NOALLOC_TWIDDLE_BYTES) mock_fail("twiddle table size");
    check_range(table, size_t(n_fft) * 8, "twiddle table");
  });
  return hipSuccess;
}
hipError_t launch_reduce_chunks(const float* partial, float* spectra, int64_t elems, int32_t chunks,
                                int32_t, int32_t n_fft, const int32_t* list, const int32_t* count,
                                hipStream_t st) {
  run_on(st, [=] {
    if (n_fft < 1 || elems % n_fft != 0) mock_fail("reduce: elems not whole rows");
    const int G = static_cast<int>(elems / n_fft);
    const std::vector<int> gs = active_gates(list, count, G, G);
    for (int k = 0; k < chunks; ++k) check_rows(partial + k * elems, n_fft, gs, "reduce partial");
    check_rows(spectra, n_fft, gs, "reduce spectra");
  });
  return hipSuccess;
}
hipError_t launch_pack_code_bits(const float* tx, int32_t rows, int32_t code_len, uint16_t* bits,
                                 int32_t* binary, hipStream_t st) {
  run_on(st, [=] {
    if (rows < 1 || code_len < 1 || code_len > 16 * SUB) mock_fail("pack code bits: geometry");
    check_range(tx, size_t(rows) * code_len * 8, "pack tx");
    check_range(bits, size_t(rows) * CODE_BITS_WORDS * 2, "pack bits");
    check_range(binary, size_t(rows) * 4, "pack flags");
  });
  return hipSuccess;
}
hipError_t launch_fill_zero(float* dst, int64_t elems, hipStream_t st) {
  run_on(st, [=] { check_range(dst, size_t(elems) * 4, "fill_zero"); });
  return hipSuccess;
}
hipError_t launch_fill_zero_rows(float* dst, int32_t g, int32_t n, const int32_t* list,
                                 const int32_t* count, hipStream_t st) {
  run_on(st, [=] { check_rows(dst, n, active_gates(list, count, g, g), "fill_zero_rows"); });
  return hipSuccess;
}
hipError_t launch_zoom(const ZoomArgs& a, hipStream_t st, bool prep) {
  ZoomArgs c = a;
  run_on(st, [c, prep] {
    if (c.n_pulses < 1) {
      mock_fail("zoom launch without pulses (an empty grid)");
      return;
    }
    if ((c.row_tiles != 1 && c.row_tiles != 2) || (c.col_tiles != 1 && c.col_tiles != 2) ||
        c.n_bins % (128 * c.row_tiles) != 0 || c.code_pad % 64 != 0 || c.code_pad < c.code_len ||
        c.chunks < 1 || (c.n_fft & (c.n_fft - 1)) != 0)
      mock_fail("zoom geometry");
    if (c.precision == 1) {
      if (prep)
        check_pulse_exponents(c.samples, c.sample_type, c.tx, c.stride, c.row_lo, c.row_hi,
                              c.code_len, c.tx_per_pulse, c.n_pulses, c.col_exp);
      check_range(c.col_exp, size_t(c.n_pulses) * 4, "zoom col_exp");
    }
    if (c.code_bits) {
      if (prep)
        check_code_bits(c.tx, c.code_len, c.tx_per_pulse, c.n_pulses, c.code_pad / 32,
                        c.code_bits, c.code_binary);
      const int rows = c.tx_per_pulse ? c.n_pulses : 1;
      check_range(c.code_bits, size_t(rows) * (c.code_pad / 32) * 4, "zoom code bits");
      check_range(c.code_binary, size_t(rows) * 4, "zoom code binary");
    }
    const std::vector<int> gs = active_gates(c.gate_list, c.gate_count, c.n_gates, c.n_gates);
    check_windows(c.samples, c.sample_type == 1 ? 4 : 8, c.stride, c.first_gate, c.gate_step,
                  c.code_len, c.n_pulses, gs, "zoom samples");
    check_range(c.tx, size_t(c.tx_per_pulse ? c.n_pulses : 1) * c.code_len * 8, "zoom tx");
    check_range(c.twiddle, size_t(c.n_fft) * 8, "zoom twiddle");
    const size_t table = size_t(3) * (c.n_bins / 32) * (c.code_pad / 16) * 64 * 16;
    check_range(c.a_hi, table, "zoom table hi");
    check_range(c.a_lo, table, "zoom table lo");
    for (int g : gs) check_range(c.bin_start + g, 4, "zoom bin_start");
    if (c.chunks == 1) {
      check_rows(c.out, c.n_bins, gs, "zoom out");
    } else {
      for (int k = 0; k < c.chunks; ++k)
        check_rows(c.partial + int64_t(k) * c.n_gates * c.n_bins, c.n_bins, gs, "zoom partial");
    }
  });
  return hipSuccess;
}

constexpr int64_t T_NET = NET_LEN;

hipError_t launch_net_features(const float* spectra, int rows, float* out, hipStream_t st) {
  run_on(st, [=] {
    if (rows < 1) mock_fail("features launch with an empty grid");
    check_range(spectra, size_t(rows) * T_NET * 4, "features in");
    check_range(out, size_t(rows) * T_NET * 4, "features out");
  });
  return hipSuccess;
}

static void check_f32_forward(const NetWork& w, const float* x, int B, const float* logits) {
  if (B < 1) mock_fail("FP32 forward with an empty grid");
  check_range(x, size_t(B) * T_NET * 4, "forward x");
  check_range(w.params, size_t(NET_PARAMS) * 4, "forward params");
  for (const float* a : {w.a1, w.a2, w.a3}) check_range(a, size_t(B) * 32 * T_NET * 4, "forward act");
  check_range(logits, size_t(B) * T_NET * 4, "forward logits");
}

hipError_t launch_net_forward_f32(const NetWork& w, const float* x, int batch, float* logits,
                                  hipStream_t st) {
  NetWork c = w;
  run_on(st, [=] { check_f32_forward(c, x, batch, logits); });
  return hipSuccess;
}

hipError_t launch_net_loss_grad(const NetWork& w, const float* x, const float* target_pos,
                                int batch, float* grad, float* loss_mean, hipStream_t st) {
  NetWork c = w;
  run_on(st, [=] {
    const size_t B = size_t(batch);
    check_f32_forward(c, x, batch, c.logits);
    check_range(target_pos, B * 4, "loss target");
    check_range(c.dz4, B * T_NET * 4, "loss dz4");
    check_range(c.loss, B * 4, "loss rows");
    check_range(c.dzA, B * 32 * T_NET * 4, "loss dzA");
    check_range(c.dzB, B * 32 * T_NET * 4, "loss dzB");
    check_range(c.part, B * NET_PARAMS * 4, "loss part");
    check_range(grad, size_t(NET_PARAMS) * 4, "loss grad");
    check_range(loss_mean, 4, "loss mean");
  });
  return hipSuccess;
}

size_t net_bf16_bytes() { return 65536; }

hipError_t launch_net_prep_bf16(const float* params, void* table, hipStream_t st) {
  run_on(st, [=] {
    check_range(params, size_t(NET_PARAMS) * 4, "prep params");
    check_range(table, net_bf16_bytes(), "prep table");
  });
  return hipSuccess;
}

hipError_t launch_net_forward_bf16(const void* table, const float* x, int batch, float* logits,
                                   hipStream_t st, bool from_spectra, const float* partial,
                                   int32_t chunks, float* x_out) {
  run_on(st, [=] {
    const size_t B = size_t(batch);
    if (batch < 1) mock_fail("BF16 forward with an empty grid");
    check_range(table, net_bf16_bytes(), "bf16 table");
    if (from_spectra && chunks > 1) {
      check_range(partial, size_t(chunks) * B * T_NET * 4, "bf16 partial");
      check_range(x_out, B * T_NET * 4, "bf16 x_out");
    } else {
      check_range(x, B * T_NET * 4, "bf16 x");
    }
    check_range(logits, B * T_NET * 4, "bf16 logits");
  });
  return hipSuccess;
}

hipError_t launch_adam(float* params, const float* grad, float* m, float* v, int n, float, int,
                       hipStream_t st) {
  run_on(st, [=] {
    for (const float* p : {static_cast<const float*>(params), grad, static_cast<const float*>(m),
                           static_cast<const float*>(v)})
      check_range(p, size_t(n) * 4, "adam");
  });
  return hipSuccess;
}

hipError_t launch_peak(const float* spectra, int32_t n_gates, int32_t n_fft, int32_t bin_lo,
                       int32_t bin_hi, int32_t* peak_bin, float* peak_power, const int32_t* list,
                       const int32_t* count, hipStream_t st) {
  run_on(st, [=] {
    if (n_gates < 1) mock_fail("peak launch with an empty grid");
    if (bin_lo < 0 || bin_lo >= n_fft || bin_hi < 1 || bin_hi > n_fft || bin_lo == bin_hi)
      mock_fail("peak band");
    const std::vector<int> gs = active_gates(list, count, n_gates, n_gates);
    check_rows(spectra, n_fft, gs, "peak spectra");
    check_rows(peak_bin, 1, gs, "peak bin");
    if (peak_power) check_rows(peak_power, 1, gs, "peak power");
  });
  return hipSuccess;
}

// The window decision's outputs, written the way the kernel writes them (a
// fixed pattern of zoomed gates stands in for the network's confidence).
// The decision pattern cycles over calls: one gate in five falls back, then a
// single gate, then none (the adaptive fallback chunking sees many, one and
// no fallback gates).
static int g_select_calls = 0;

static void emulate_select(const float* logits, int32_t G, int32_t fine_len, int32_t K,
                           int32_t* bin_start, float* confidence, int32_t* flag,
                           int32_t* zoom_list, int32_t* fallback_list, int32_t* counts,
                           int32_t* done) {
  const int pattern = g_select_calls++ % 3;
  if (G < 1) mock_fail("select launch with an empty grid");
  if (fine_len < T_NET || fine_len % T_NET != 0 || K < 1 || K > fine_len)
    mock_fail("select window geometry");
  bool ok = check_range(logits, size_t(G) * T_NET * 4, "select logits");
  for (const void* p : {static_cast<const void*>(bin_start), static_cast<const void*>(flag),
                        static_cast<const void*>(zoom_list), static_cast<const void*>(fallback_list)})
    ok = check_range(p, size_t(G) * 4, "select per-gate output") && ok;
  if (confidence) ok = check_range(confidence, size_t(G) * 4, "select confidence") && ok;
  ok = check_range(counts, 8, "select counts") && ok;
  ok = check_range(done, 4, "select done") && ok;
  if (!ok) return;
  if (*done != 0) mock_fail("select: completion counter not zero at the start of a call");
  int nz = 0;
  for (int g = 0; g < G; ++g) {
    const bool z = pattern == 0 ? (g * 7 + 3) % 5 != 0 : pattern == 1 ? g != G / 2 : true;
    flag[g] = z ? 1 : 0;
    bin_start[g] = static_cast<int32_t>((int64_t(g) * 997) % fine_len);
    if (confidence) confidence[g] = z ? 0.95f : 0.5f;
    if (z)
      zoom_list[nz++] = g;
    else
      fallback_list[g - nz] = g;
  }
  counts[0] = nz;
  counts[1] = G - nz;
  *done = 0;
}

hipError_t launch_select_windows(const float* logits, int32_t n_gates, int32_t fine_len,
                                 int32_t window_bins, float, int32_t* bin_start,
                                 float* confidence, int32_t* flag, int32_t* zoom_list,
                                 int32_t* fallback_list, int32_t* counts, int32_t* done,
                                 hipStream_t st) {
  run_on(st, [=] {
    emulate_select(logits, n_gates, fine_len, window_bins, bin_start, confidence, flag, zoom_list,
                   fallback_list, counts, done);
  });
  return hipSuccess;
}

hipError_t launch_select_and_exponents(const float* logits, int32_t n_gates, int32_t fine_len,
                                       int32_t window_bins, float, int32_t* bin_start,
                                       float* confidence, int32_t* flag, int32_t* zoom_list,
                                       int32_t* fallback_list, int32_t* counts, int32_t* done,
                                       const PulseExpArgs& pe, hipStream_t st) {
  PulseExpArgs e = pe;
  run_on(st, [=] {
    emulate_select(logits, n_gates, fine_len, window_bins, bin_start, confidence, flag, zoom_list,
                   fallback_list, counts, done);
    if (e.n_pulses < 0) mock_fail("negative pulse count");
    check_pulse_exponents(e.samples, e.sample_type, e.tx, e.stride, e.lo, e.hi, e.code_len,
                          e.tx_per_pulse, e.n_pulses, e.exps);
    check_code_bits(e.tx, e.code_len, e.tx_per_pulse, e.n_pulses, e.bit_words, e.bits, e.binary);
  });
  return hipSuccess;
}

hipError_t launch_split_peaks(float* window_spectra, const float* window_partial,
                              int32_t zoom_chunks, float* full_spectra, const FallbackChunks& f,
                              const int32_t* zoom_list, const int32_t* fallback_list,
                              const int32_t* bin_start, int32_t n_gates, int32_t window_bins,
                              int32_t fine_len, int32_t* peak_bin, float* peak_power,
                              hipStream_t st) {
  const FallbackChunks fb = f;
  run_on(st, [=] {
    if (n_gates < 1) mock_fail("split peaks with an empty grid");
    if (!check_range(fb.counts, 8, "split counts")) return;
    const int k = std::min(std::max(fb.counts[1], 0), n_gates);
    const int nz = std::min(std::max(fb.counts[0], 0), n_gates - k);
    const int fchunks = adaptive_chunks(k, fb.zgroups, fb.target, fb.max_chunks, fb.rows);
    if (fchunks > 1 && fchunks * k > fb.rows) mock_fail("split: fallback partial rows overflow");
    // workgroups 0..k-1 take the fallback list's slots, k..k+nz-1 the zoom list's
    if (k > 0 && !check_range(fallback_list, size_t(k) * 4, "split fallback list")) return;
    if (nz > 0 && !check_range(zoom_list, size_t(nz) * 4, "split zoom list")) return;
    for (int i = 0; i < k; ++i) {
      const int g = fallback_list[i];
      if (g < 0 || g >= n_gates) continue;
      check_range(full_spectra + int64_t(g) * fine_len, size_t(fine_len) * 4, "split full row");
      if (fchunks > 1)
        for (int c = 0; c < fchunks; ++c)
          check_range(fb.partial + (int64_t(c) * k + i) * fine_len, size_t(fine_len) * 4,
                      "split fallback partial");
      check_range(peak_bin + g, 4, "split peak bin");
      if (peak_power) check_range(peak_power + g, 4, "split peak power");
    }
    for (int i = 0; i < nz; ++i) {
      const int g = zoom_list[i];
      if (g < 0 || g >= n_gates) continue;
      const int64_t len = window_bins;
      check_range(window_spectra + g * len, size_t(len) * 4, "split window row");
      if (zoom_chunks > 1)
        for (int c = 0; c < zoom_chunks; ++c)
          check_range(window_partial + (int64_t(c) * n_gates + g) * len, size_t(len) * 4,
                      "split zoom partial");
      check_range(bin_start + g, 4, "split bin_start");
      check_range(peak_bin + g, 4, "split peak bin");
      if (peak_power) check_range(peak_power + g, 4, "split peak power");
    }
  });
  return hipSuccess;
}

hipError_t launch_window_peak(const float* spectra, int32_t n_gates, int32_t window_bins,
                              int32_t, const int32_t* bin_start, const int32_t* list,
                              const int32_t* count, int32_t* peak_bin, float* peak_power,
                              hipStream_t st) {
  run_on(st, [=] {
    if (n_gates < 1) mock_fail("window peak with an empty grid");
    const std::vector<int> gs = active_gates(list, count, n_gates, n_gates);
    check_rows(spectra, window_bins, gs, "window peak spectra");
    check_rows(bin_start, 1, gs, "window peak bin_start");
    check_rows(peak_bin, 1, gs, "window peak bin");
    if (peak_power) check_rows(peak_power, 1, gs, "window peak power");
  });
  return hipSuccess;
}

}  // namespace ispl
