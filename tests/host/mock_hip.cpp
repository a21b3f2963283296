// Host-only stand-in for the HIP runtime and the device launchers, so that the
// C-ABI layer's host logic (plans, scratch sizes, stream capture of the batch
// graph, error paths) runs under AddressSanitizer on a machine without a GPU.
// Test infrastructure only.  "Device" memory is host memory; every launcher
// checks the footprint its kernel would read and write against the live
// allocations; stream capture tracks fork and join like the real API (an
// unjoined branch at the end of a capture, a launch of an unknown or destroyed
// graph, a capture on a capturing stream are all counted as errors).
#include <hip/hip_runtime_api.h>

#include <cassert>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "ispl_internal.h"

static std::map<uintptr_t, size_t> g_allocs;
static int g_errors = 0;

static void check_range(const void* p, size_t bytes, const char* what) {
  if (bytes == 0) return;
  uintptr_t a = reinterpret_cast<uintptr_t>(p);
  auto it = g_allocs.upper_bound(a);
  if (it == g_allocs.begin()) {
    fprintf(stderr, "MOCK OOB: %s %p (+%zu) not in any allocation\n", what, p, bytes);
    ++g_errors;
    return;
  }
  --it;
  if (a < it->first || a + bytes > it->first + it->second) {
    fprintf(stderr, "MOCK OOB: %s %p +%zu outside [%p, +%zu)\n", what, p, bytes,
            reinterpret_cast<void*>(it->first), it->second);
    ++g_errors;
  }
}

int mock_errors() { return g_errors; }

struct MStream;
struct MGraph {
  std::vector<std::function<void()>> ops;
};
struct MExec {
  std::vector<std::function<void()>> ops;
  bool alive = true;
};
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
  if (m->capture) {
    m->graph->ops.push_back(op);
  } else {
    op();
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
hipError_t hipDeviceSynchronize() { return hipSuccess; }
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
  run_on(st, [=] { hipMemcpy(d, s, n, k); });
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
  delete e;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  MExec* e = reinterpret_cast<MExec*>(x);
  if (!g_execs.count(e)) { fprintf(stderr, "MOCK: launch unknown exec\n"); ++g_errors; return hipErrorInvalidValue; }
  if (S(s)->capture) { fprintf(stderr, "MOCK: graph launch into a capture\n"); ++g_errors; }
  for (auto& op : e->ops) op();
  return hipSuccess;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// launchers: footprint checks

namespace ispl {

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
    if (c.n_pulses > 0) {
      const int64_t last = int64_t(c.n_pulses - 1) * c.stride + c.first_gate +
                           int64_t(c.n_gates - 1) * c.gate_step + c.code_len;
      check_range(c.samples, size_t(last) * ss, "fused samples");
      check_range(c.tx, size_t(c.tx_per_pulse ? c.n_pulses : 1) * c.code_len * 8, "fused tx");
    }
    check_range(c.twiddle, size_t(c.n_fft) * 8, "fused twiddle");
    check_range(c.out, size_t(c.chunks) * c.n_gates * c.n_fft * 4, "fused out");
  });
  return hipSuccess;
}
hipError_t launch_reduce_chunks(const float* partial, float* spectra, int64_t elems, int32_t chunks,
                                int32_t, int32_t, const int32_t*, const int32_t*, hipStream_t st) {
  run_on(st, [=] {
    check_range(partial, size_t(chunks) * elems * 4, "reduce partial");
    check_range(spectra, size_t(elems) * 4, "reduce spectra");
  });
  return hipSuccess;
}
hipError_t launch_fill_zero(float* dst, int64_t elems, hipStream_t st) {
  run_on(st, [=] { check_range(dst, size_t(elems) * 4, "fill_zero"); });
  return hipSuccess;
}
hipError_t launch_fill_zero_rows(float* dst, int32_t g, int32_t n, const int32_t*, const int32_t*,
                                 hipStream_t st) {
  run_on(st, [=] { check_range(dst, size_t(g) * n * 4, "fill_zero_rows"); });
  return hipSuccess;
}
hipError_t launch_zoom(const ZoomArgs&, hipStream_t, bool) { return hipSuccess; }
hipError_t launch_net_features(const float*, int, float*, hipStream_t) { return hipSuccess; }
hipError_t launch_net_forward_f32(const NetWork&, const float*, int, float*, hipStream_t) { return hipSuccess; }
hipError_t launch_net_loss_grad(const NetWork&, const float*, const float*, int, float*, float*, hipStream_t) { return hipSuccess; }
size_t net_bf16_bytes() { return 65536; }
hipError_t launch_net_prep_bf16(const float*, void*, hipStream_t) { return hipSuccess; }
hipError_t launch_net_forward_bf16(const void*, const float*, int, float*, hipStream_t, bool, const float*, int32_t, float*) { return hipSuccess; }
hipError_t launch_adam(float*, const float*, float*, float*, int, float, int, hipStream_t) { return hipSuccess; }
hipError_t launch_peak(const float*, int32_t, int32_t, int32_t, int32_t, int32_t*, float*, const int32_t*, const int32_t*, hipStream_t) { return hipSuccess; }
hipError_t launch_select_windows(const float*, int32_t, int32_t, int32_t, float, int32_t*, float*, int32_t*, int32_t*, int32_t*, int32_t*, int32_t*, hipStream_t) { return hipSuccess; }
hipError_t launch_split_peaks(float*, const float*, int32_t, float*, const float*, int32_t, const int32_t*, const int32_t*, int32_t, int32_t, int32_t, int32_t*, float*, hipStream_t) { return hipSuccess; }
hipError_t launch_select_and_exponents(const float*, int32_t, int32_t, int32_t, float, int32_t*, float*, int32_t*, int32_t*, int32_t*, int32_t*, int32_t*, const PulseExpArgs&, hipStream_t) { return hipSuccess; }
hipError_t launch_window_peak(const float*, int32_t, int32_t, int32_t, const int32_t*, const int32_t*, const int32_t*, int32_t*, float*, hipStream_t) { return hipSuccess; }

}  // namespace ispl
