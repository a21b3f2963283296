// Streaming ingest: pulse rows arrive in host memory, only the samples the
// range gates read are copied to the device, and the copy of one batch
// overlaps the integration of the previous one.
//
// The paper times the whole chain including the per-row host-to-device copy
// (Section 4) against the radar's pulse cadence (one echo every 10 ms); this
// object is that chain on one GPU.  The caller (the receiver) writes pulse
// rows into pinned host slots of a ring; ispl_stream_submit copies rows
// [g0, g0 + (G-1) s + L) of each pulse of a slot, and its codes, to the
// slot's device buffer on a copy stream, then queues the integration of the
// slot on the caller's stream after the copy.  A slot is free for the next
// batch once its copy has finished (ispl_stream_wait_slot); its device
// buffer is reused once its integration has run.  Integration is the plain
// path (Eqs. 7-8, Section 3.2) on a context whose rows are the compact
// copies, so a stream of batches gives exactly the spectra of calling
// ispl_integrate_spectra batch by batch with accumulate = 1.

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstdio>
#include <new>
#include <vector>

#include "ispl.h"
#include "ispl_internal.h"

struct ispl_stream {
  ispl_config cfg;       // the caller's geometry
  ispl_ctx* dctx;        // compact rows: first_gate 0, pulse_stride = need
  int32_t slot_pulses;
  int32_t n_slots;
  int64_t need;          // samples of a row that some gate reads
  size_t elem;           // bytes per sample
  void* host_rows;       // pinned [n_slots][slot_pulses][pulse_stride] samples
  float* host_tx;        // pinned [n_slots][slot_pulses][L] complex64
  void* dev_rows;        // [n_slots][slot_pulses][need] samples
  float* dev_tx;         // [n_slots][slot_pulses][L] complex64
  hipStream_t copy;      // host-to-device copies
  std::vector<hipEvent_t> copied, integrated;
  std::vector<char> pending;  // a copy has been queued since the last wait
};

namespace {

ispl_status fail_stream(ispl_status s, const char* fmt, long long a = 0, long long b = 0) {
  char buf[256];
  snprintf(buf, sizeof buf, fmt, a, b);
  return ispl::report(s, buf);
}

void release(ispl_stream* st) {
  for (hipEvent_t e : st->copied)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : st->integrated)
    if (e) (void)hipEventDestroy(e);
  if (st->copy) (void)hipStreamDestroy(st->copy);
  if (st->dev_rows) (void)hipFree(st->dev_rows);
  if (st->dev_tx) (void)hipFree(st->dev_tx);
  if (st->host_rows) (void)hipHostFree(st->host_rows);
  if (st->host_tx) (void)hipHostFree(st->host_tx);
  if (st->dctx) ispl_destroy(st->dctx);
}

struct DeviceScope {  // restores the caller's current device
  int prev = -1;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

extern "C" {

ispl_status ispl_stream_create(const ispl_config* cfg, int32_t slot_pulses, int32_t n_slots,
                               ispl_stream** out) {
  if (!out) return fail_stream(ISPL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail_stream(ISPL_ERR_INVALID_ARG, "config is NULL");
  if (slot_pulses < 1 || slot_pulses > cfg->max_pulses)
    return fail_stream(ISPL_ERR_INVALID_ARG, "slot_pulses %lld outside [1, max_pulses %lld]",
                       slot_pulses, cfg->max_pulses);
  if (n_slots < 2 || n_slots > 64)
    return fail_stream(ISPL_ERR_INVALID_ARG, "n_slots %lld outside [2, 64]", n_slots);
  // the compact-row context validates the geometry (and the device)
  ispl_config dc = *cfg;
  const int64_t need = static_cast<int64_t>(cfg->n_gates - 1) * cfg->gate_step + cfg->code_len;
  dc.first_gate = 0;
  dc.pulse_stride = need;
  dc.max_pulses = slot_pulses;
  if (cfg->pulse_stride < static_cast<int64_t>(cfg->first_gate) + need)
    return fail_stream(ISPL_ERR_INVALID_ARG, "pulse_stride %lld < first_gate + span %lld",
                       cfg->pulse_stride, static_cast<long long>(cfg->first_gate) + need);
  ispl_stream* st = new (std::nothrow) ispl_stream{};
  if (!st) return fail_stream(ISPL_ERR_OUT_OF_MEMORY, "host allocation");
  ispl_status s = ispl_create(&dc, &st->dctx);
  if (s != ISPL_OK) {
    delete st;
    return s;  // ispl_create has set the error text
  }
  st->cfg = *cfg;
  st->slot_pulses = slot_pulses;
  st->n_slots = n_slots;
  st->need = need;
  st->elem = cfg->sample_type == ISPL_SAMPLES_CI16 ? 4 : 8;
  DeviceScope scope(cfg->device);
  const size_t rows = static_cast<size_t>(n_slots) * slot_pulses;
  const size_t tx_bytes = rows * cfg->code_len * 8;
  hipError_t e = hipHostMalloc(&st->host_rows, rows * cfg->pulse_stride * st->elem,
                               hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&st->host_tx), tx_bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(&st->dev_rows, rows * need * st->elem);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&st->dev_tx), tx_bytes);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&st->copy, hipStreamNonBlocking);
  st->copied.assign(n_slots, nullptr);
  st->integrated.assign(n_slots, nullptr);
  st->pending.assign(n_slots, 0);
  for (int i = 0; i < n_slots && e == hipSuccess; ++i) {
    e = hipEventCreateWithFlags(&st->copied[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st->integrated[i], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    const ispl_status code =
        e == hipErrorOutOfMemory ? ISPL_ERR_OUT_OF_MEMORY : ISPL_ERR_DEVICE;
    char buf[256];
    snprintf(buf, sizeof buf, "stream buffers: %s", hipGetErrorString(e));
    release(st);
    delete st;
    return ispl::report(code, buf);
  }
  *out = st;
  return ispl::report(ISPL_OK, "");
}

void ispl_stream_destroy(ispl_stream* st) {
  if (!st) return;
  {
    DeviceScope scope(st->cfg.device);
    (void)hipDeviceSynchronize();
    release(st);
  }
  delete st;
}

void* ispl_stream_slot_samples(ispl_stream* st, int32_t slot) {
  if (!st || slot < 0 || slot >= st->n_slots) return nullptr;
  return static_cast<char*>(st->host_rows) +
         static_cast<size_t>(slot) * st->slot_pulses * st->cfg.pulse_stride * st->elem;
}

float* ispl_stream_slot_codes(ispl_stream* st, int32_t slot) {
  if (!st || slot < 0 || slot >= st->n_slots) return nullptr;
  return st->host_tx + static_cast<size_t>(slot) * st->slot_pulses * st->cfg.code_len * 2;
}

ispl_status ispl_stream_wait_slot(ispl_stream* st, int32_t slot) {
  if (!st) return fail_stream(ISPL_ERR_INVALID_ARG, "stream is NULL");
  if (slot < 0 || slot >= st->n_slots)
    return fail_stream(ISPL_ERR_INVALID_ARG, "slot %lld outside [0, %lld)", slot, st->n_slots);
  if (st->pending[slot]) {
    DeviceScope scope(st->cfg.device);
    const hipError_t e = hipEventSynchronize(st->copied[slot]);
    if (e != hipSuccess) {
      char buf[256];
      snprintf(buf, sizeof buf, "wait for slot copy: %s", hipGetErrorString(e));
      return ispl::report(ISPL_ERR_DEVICE, buf);
    }
    st->pending[slot] = 0;
  }
  return ispl::report(ISPL_OK, "");
}

ispl_status ispl_stream_submit(ispl_stream* st, int32_t slot, int32_t n_pulses,
                               int32_t tx_per_pulse, float* spectra, int32_t accumulate,
                               void* stream) {
  if (!st) return fail_stream(ISPL_ERR_INVALID_ARG, "stream is NULL");
  if (slot < 0 || slot >= st->n_slots)
    return fail_stream(ISPL_ERR_INVALID_ARG, "slot %lld outside [0, %lld)", slot, st->n_slots);
  if (n_pulses < 0 || n_pulses > st->slot_pulses)
    return fail_stream(ISPL_ERR_INVALID_ARG, "n_pulses %lld outside [0, slot_pulses %lld]",
                       n_pulses, st->slot_pulses);
  if (!spectra) return fail_stream(ISPL_ERR_INVALID_ARG, "spectra is NULL");
  if ((tx_per_pulse != 0 && tx_per_pulse != 1) || (accumulate != 0 && accumulate != 1))
    return fail_stream(ISPL_ERR_INVALID_ARG, "tx_per_pulse and accumulate must be 0 or 1");
  DeviceScope scope(st->cfg.device);
  hipStream_t compute = static_cast<hipStream_t>(stream);
  const ispl_config& c = st->cfg;
  const size_t slot_row0 = static_cast<size_t>(slot) * st->slot_pulses;
  char* dst = static_cast<char*>(st->dev_rows) + slot_row0 * st->need * st->elem;
  float* dtx = st->dev_tx + slot_row0 * c.code_len * 2;
  hipError_t e = hipSuccess;
  if (n_pulses > 0) {
    // the device buffer is free once the slot's previous integration has run
    e = hipStreamWaitEvent(st->copy, st->integrated[slot], 0);
    const char* src = static_cast<const char*>(ispl_stream_slot_samples(st, slot)) +
                      static_cast<size_t>(c.first_gate) * st->elem;
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(dst, st->need * st->elem, src, c.pulse_stride * st->elem,
                           st->need * st->elem, n_pulses, hipMemcpyHostToDevice, st->copy);
    const size_t code_rows = tx_per_pulse ? static_cast<size_t>(n_pulses) : 1;
    if (e == hipSuccess)
      e = hipMemcpyAsync(dtx, ispl_stream_slot_codes(st, slot), code_rows * c.code_len * 8,
                         hipMemcpyHostToDevice, st->copy);
    if (e == hipSuccess) e = hipEventRecord(st->copied[slot], st->copy);
    if (e == hipSuccess) st->pending[slot] = 1;
    if (e == hipSuccess) e = hipStreamWaitEvent(compute, st->copied[slot], 0);
  }
  if (e != hipSuccess) {
    char buf[256];
    snprintf(buf, sizeof buf, "stream copy: %s", hipGetErrorString(e));
    return ispl::report(ISPL_ERR_DEVICE, buf);
  }
  const ispl_status s = ispl_integrate_spectra(st->dctx, dst, dtx, tx_per_pulse, n_pulses, spectra,
                                               accumulate, stream);
  if (s != ISPL_OK) return s;
  if (n_pulses > 0) {
    e = hipEventRecord(st->integrated[slot], compute);
    if (e != hipSuccess) {
      char buf[256];
      snprintf(buf, sizeof buf, "stream event: %s", hipGetErrorString(e));
      return ispl::report(ISPL_ERR_DEVICE, buf);
    }
  }
  return ispl::report(ISPL_OK, "");
}

ispl_status ispl_stream_sync(ispl_stream* st) {
  if (!st) return fail_stream(ISPL_ERR_INVALID_ARG, "stream is NULL");
  DeviceScope scope(st->cfg.device);
  hipError_t e = hipStreamSynchronize(st->copy);
  for (int i = 0; i < st->n_slots && e == hipSuccess; ++i) {
    e = hipEventSynchronize(st->integrated[i]);
    st->pending[i] = 0;
  }
  if (e != hipSuccess) {
    char buf[256];
    snprintf(buf, sizeof buf, "stream sync: %s", hipGetErrorString(e));
    return ispl::report(ISPL_ERR_DEVICE, buf);
  }
  return ispl::report(ISPL_OK, "");
}

}  // extern "C"
