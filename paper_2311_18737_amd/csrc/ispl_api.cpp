// C ABI of the plasma-line spectrum library: argument validation, launch
// planning, context-owned device state (twiddle table, chunk partials).
// Declared in include/ispl.h.

#include "ispl.h"

#include <hip/hip_runtime_api.h>

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <new>
#include <string>
#include <vector>

#include "ispl_internal.h"

struct ispl_ctx {
  ispl_config cfg;
  int32_t chunks_max;   // largest chunk count any call may plan
  float* twiddle;       // complex64 pairs, N entries
  float* partial;       // chunks_max * G * N floats (nullptr when chunks_max == 1)
  int32_t force_rw;     // tuned plan (0: automatic): waves per workgroup, L <= 1024 only
  int32_t force_chunks; // tuned plan (0: automatic): pulse chunks, <= chunks_max
  int32_t min_chunk_pulses;  // fewest pulses per chunk of an automatic plan
  // codes of L > 2 SUB as sign bits (long-code kernel), max_pulses rows
  uint16_t* code_bits;  // [max_pulses][CODE_BITS_WORDS]
  int32_t* code_binary; // [max_pulses]
};

namespace {

thread_local std::string g_last_error;

ispl_status fail(ispl_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

ispl_status fail(ispl_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

ispl_status ok() {
  g_last_error.clear();
  return ISPL_OK;
}

}  // namespace

namespace ispl {
// Error reporting for the other host-side translation units.
ispl_status report(ispl_status s, const char* msg) {
  if (s == ISPL_OK)
    g_last_error.clear();
  else
    g_last_error = msg;
  return s;
}
}  // namespace ispl

namespace {

ispl_status hip_fail(hipError_t e, const char* what) {
  return fail(ISPL_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int64_t v) {
  int r = 0;
  while ((int64_t{1} << r) < v) ++r;
  return r;
}

// Planning constants of the target: MI355X has 256 compute units with 160 KiB
// of LDS each; a wave of the fused kernel may use up to 128 VGPRs, so at most
// 16 of its waves fit on one compute unit.
constexpr int kComputeUnits = 256;
constexpr int kLdsPerCu = 160 * 1024;
constexpr int kMaxWavesPerCu = 16;
constexpr int kMaxChunks = 256;
constexpr int kMinChunkPulses = 8;
#ifndef ISPL_MAX_WAVES_PER_BLOCK  // build-time tuning knob (1, 2, 4, 8 or 16)
#define ISPL_MAX_WAVES_PER_BLOCK 16
#endif
constexpr int kMaxWavesPerBlock = ISPL_MAX_WAVES_PER_BLOCK;
static_assert(kMaxWavesPerBlock <= ispl::MAX_WAVES_PER_BLOCK, "at most 16 waves per block");
constexpr int64_t kMaxPartialBytes = int64_t{1} << 30;

struct Plan {
  int sub_len;    // M: points of one sub-transform (1024, or 16384 for L > 1024)
  int r;          // R = N / M sub-transforms (bin classes) per spectrum
  int rw;         // waves per workgroup
  int zgroups;    // workgroups per gate and chunk
  int chunks;     // pulse chunks
  int64_t blocks; // workgroups of the fused launch
};

Plan make_plan(const ispl_config& c, int32_t n_pulses, int32_t force_rw = 0,
               int32_t force_chunks = 0, int32_t min_chunk_pulses = kMinChunkPulses) {
  Plan pl{};
  pl.sub_len = c.code_len <= ispl::SUB ? ispl::SUB : 16 * ispl::SUB;
  pl.r = c.fft_len / pl.sub_len;
  if (pl.sub_len == ispl::SUB) {  // one wave per bin class
    pl.rw = pl.r < kMaxWavesPerBlock ? pl.r : kMaxWavesPerBlock;
    if (force_rw > 0 && force_rw < pl.rw) pl.rw = force_rw;  // a power of two dividing R
    pl.zgroups = pl.r / pl.rw;
  } else {                        // sixteen waves per bin class
    pl.rw = 16;
    pl.zgroups = pl.r;
  }
  int per_cu = kLdsPerCu / ispl::fused_lds_bytes(pl.rw, pl.sub_len);
  if (per_cu * pl.rw > kMaxWavesPerCu) per_cu = kMaxWavesPerCu / pl.rw;
  if (per_cu < 1) per_cu = 1;
  const int64_t slots = int64_t{kComputeUnits} * per_cu;
  const int64_t base = static_cast<int64_t>(c.n_gates) * pl.zgroups;
  // enough workgroups for two rounds over the chip, but at least kMinChunkPulses
  // pulses per chunk (a chunk's partial spectrum costs a write and a read)
  int64_t chunks = 1;
  if (base < 2 * slots) chunks = (2 * slots + base - 1) / base;
  const int64_t by_pulses = n_pulses / min_chunk_pulses;
  if (chunks > by_pulses) chunks = by_pulses;
  if (chunks > kMaxChunks) chunks = kMaxChunks;
  const int64_t gn_bytes = static_cast<int64_t>(c.n_gates) * c.fft_len * 4;
  if (chunks > 1 && chunks * gn_bytes > kMaxPartialBytes) chunks = kMaxPartialBytes / gn_bytes;
  if (force_chunks > 0) chunks = force_chunks < n_pulses ? force_chunks : n_pulses;
  if (chunks < 1) chunks = 1;
  pl.chunks = static_cast<int>(chunks);
  pl.blocks = base * pl.chunks;
  return pl;
}

ispl_status validate_config(const ispl_config* c) {
  if (!c) return fail(ISPL_ERR_INVALID_ARG, "config is NULL");
  if (c->abi_version != ISPL_ABI_VERSION)
    return fail(ISPL_ERR_INVALID_ARG, "abi_version %d, library is %d", c->abi_version,
                ISPL_ABI_VERSION);
  if (c->code_len < 1) return fail(ISPL_ERR_INVALID_ARG, "code_len %d < 1", c->code_len);
  if (!is_pow2(c->fft_len))
    return fail(ISPL_ERR_INVALID_ARG, "fft_len %d is not a power of two", c->fft_len);
  if (c->code_len > c->fft_len)
    return fail(ISPL_ERR_INVALID_ARG, "code_len %d > fft_len %d", c->code_len, c->fft_len);
  if (c->n_gates < 1) return fail(ISPL_ERR_INVALID_ARG, "n_gates %d < 1", c->n_gates);
  if (c->gate_step < 1) return fail(ISPL_ERR_INVALID_ARG, "gate_step %d < 1", c->gate_step);
  if (c->first_gate < 0) return fail(ISPL_ERR_INVALID_ARG, "first_gate %d < 0", c->first_gate);
  if (c->sample_type != ISPL_SAMPLES_C64 && c->sample_type != ISPL_SAMPLES_CI16)
    return fail(ISPL_ERR_INVALID_ARG, "unknown sample_type %d", c->sample_type);
  if (c->max_pulses < 1) return fail(ISPL_ERR_INVALID_ARG, "max_pulses %d < 1", c->max_pulses);
  if (c->device < 0) return fail(ISPL_ERR_INVALID_ARG, "device %d < 0", c->device);
  const int64_t need = static_cast<int64_t>(c->first_gate) +
                       static_cast<int64_t>(c->n_gates - 1) * c->gate_step + c->code_len;
  if (c->pulse_stride < need)
    return fail(ISPL_ERR_INVALID_ARG,
                "pulse_stride %lld < first_gate + (n_gates-1)*gate_step + code_len = %lld",
                static_cast<long long>(c->pulse_stride), static_cast<long long>(need));
  // what this library implements
  if (c->fft_len < ispl::SUB || c->fft_len > 65536)
    return fail(ISPL_ERR_UNSUPPORTED, "fft_len %d outside [1024, 65536]", c->fft_len);
  if (c->code_len > 16 * ispl::SUB)
    return fail(ISPL_ERR_UNSUPPORTED, "code_len %d > 16384", c->code_len);
  if (c->code_len > ispl::SUB && c->fft_len < 16 * ispl::SUB)
    return fail(ISPL_ERR_UNSUPPORTED, "code_len %d > 1024 needs fft_len >= 16384",
                c->code_len);
  // 64 lanes per (gate, bin class of 1024 points); keep a launch under 2^31 threads
  if (static_cast<int64_t>(c->n_gates) * (c->fft_len / ispl::SUB) * 64 >= (int64_t{1} << 31))
    return fail(ISPL_ERR_UNSUPPORTED, "n_gates %d too large for one launch", c->n_gates);
  return ISPL_OK;
}

struct DeviceGuard {  // restores the caller's current device
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// W_N^i = exp(-2 pi i / N)^i for i < N, from double-precision cos/sin of the
// first octant and exact symmetries (so 0, +-1 and the octant values are exact).
std::vector<float> twiddle_table(int n) {
  std::vector<float> t(2 * static_cast<size_t>(n));
  const int quarter = n / 4, eighth = n / 8;
  for (int i = 0; i < n; ++i) {
    const int qd = i / quarter;        // quadrant of the angle 2 pi i / N
    const int rem = i - qd * quarter;  // position inside it
    double c, s;                       // cos, sin of 2 pi rem / N
    if (rem <= eighth) {
      const double th = 2.0 * M_PI * rem / n;
      c = std::cos(th);
      s = std::sin(th);
    } else {
      const double th = 2.0 * M_PI * (quarter - rem) / n;
      c = std::sin(th);
      s = std::cos(th);
    }
    double ci, si;  // cos, sin of 2 pi i / N
    switch (qd) {
      case 0: ci = c; si = s; break;
      case 1: ci = -s; si = c; break;
      case 2: ci = -c; si = -s; break;
      default: ci = s; si = -c; break;
    }
    t[2 * i] = static_cast<float>(ci);
    t[2 * i + 1] = static_cast<float>(-si);
  }
  return t;
}

bool misaligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) != 0; }

// Round to a 16-bit float: BF16 (round to nearest even on the FP32 bits) or
// FP16 (the compiler's conversion).  Returns the bits and the value.
uint16_t round16(double v, int precision, double* value) {
  const float f = static_cast<float>(v);
  if (precision == ISPL_ZOOM_BF16X3) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    const uint16_t h = static_cast<uint16_t>(u >> 16);
    const uint32_t back = static_cast<uint32_t>(h) << 16;
    float bf;
    std::memcpy(&bf, &back, 4);
    *value = bf;
    return h;
  }
  const _Float16 h = static_cast<_Float16>(f);
  uint16_t bits;
  std::memcpy(&bits, &h, 2);
  *value = static_cast<double>(static_cast<float>(h));
  return bits;
}

// The three real matrices of the zoom GEMM in its three-multiplication
// complex form, split into high and low 16-bit parts, in MFMA A-operand
// order: for product pr, bin tile bt (32 bins), k-step ks (16 samples) and
// lane l, 8 values A_pr[32 bt + l % 32][16 ks + 8 (l / 32) + i].  With
// theta = 2 pi ((j n) mod N) / N the DFT matrix is W = cos theta - i sin theta,
// and A_0 = Re W + Im W = cos - sin, A_1 = Re W = cos, A_2 = Im W = -sin;
// samples n >= L give zero columns.
void zoom_table(int n_fft, int n_bins, int code_len, int code_pad, int precision,
                std::vector<uint16_t>& hi, std::vector<uint16_t>& lo) {
  const int n_bt = n_bins / 32, n_ks = code_pad / 16;
  hi.assign(static_cast<size_t>(3) * n_bt * n_ks * 64 * 8, 0);
  lo.assign(hi.size(), 0);
  size_t idx = 0;
  for (int pr = 0; pr < 3; ++pr)
    for (int bt = 0; bt < n_bt; ++bt)
      for (int ks = 0; ks < n_ks; ++ks)
        for (int l = 0; l < 64; ++l)
          for (int i = 0; i < 8; ++i, ++idx) {
            const int j = 32 * bt + l % 32, n = 16 * ks + 8 * (l / 32) + i;
            double v = 0.0;
            if (n < code_len) {
              const int64_t m = (static_cast<int64_t>(j) * n) % n_fft;
              const double th = 2.0 * M_PI * static_cast<double>(m) / n_fft;
              const double c = std::cos(th), sn = std::sin(th);
              v = pr == 0 ? c - sn : (pr == 1 ? c : -sn);
            }
            double hv, lv;
            hi[idx] = round16(v, precision, &hv);
            lo[idx] = round16(v - hv, precision, &lv);
          }
}

}  // namespace

struct ispl_zoom {
  ispl_ctx* ctx;
  int32_t n_bins;
  int32_t precision;
  int32_t code_pad;
  int32_t chunks_max;
  void* a_hi;
  void* a_lo;
  float* partial;    // [chunks_max][G][K] when chunks_max > 1
  int32_t* col_exp;  // [max_pulses] (FP16 only)
  uint32_t* code_bits;    // [max_pulses][code_pad / 32] sign bits of +-1 codes
  int32_t* code_binary;   // [max_pulses]
};

namespace {

struct ZoomPlan {
  int rt, ct, chunks;
};

// Bins per workgroup: 256 when K allows it (each staged sample feeds twice the
// matrix work), else 128.  Pulse chunks until there are two workgroups per
// compute unit (two rounds over the chip: one 12-wave workgroup fits a CU), but
// at least 24 pulses per chunk; one or two 32-pulse column tiles per block
// (four would not fit the matrix waves' registers).
ZoomPlan zoom_plan(int32_t n_gates, int32_t n_bins, int32_t n_pulses) {
  ZoomPlan z{};
  z.rt = n_bins % 256 == 0 ? 2 : 1;
  const int64_t base = static_cast<int64_t>(n_gates) * (n_bins / (128 * z.rt));
  int64_t chunks = base < 2 * kComputeUnits ? (2 * kComputeUnits + base - 1) / base : 1;
  const int64_t by_pulses = n_pulses / 24 > 1 ? n_pulses / 24 : 1;
  if (chunks > by_pulses) chunks = by_pulses;
  z.chunks = static_cast<int>(chunks);
  const int64_t per = (n_pulses + chunks - 1) / chunks;
  z.ct = per <= 32 ? 1 : 2;  // more column tiles per block would spill
  return z;
}

}  // namespace

static void zoom_free(ispl_zoom* z) {
  void* bufs[] = {z->a_hi, z->a_lo, z->partial, z->col_exp, z->code_bits, z->code_binary};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
}

extern "C" {

int32_t ispl_abi_version(void) { return ISPL_ABI_VERSION; }

const char* ispl_status_string(ispl_status s) {
  switch (s) {
    case ISPL_OK: return "ok";
    case ISPL_ERR_INVALID_ARG: return "invalid argument";
    case ISPL_ERR_UNSUPPORTED: return "unsupported";
    case ISPL_ERR_OUT_OF_MEMORY: return "out of memory";
    case ISPL_ERR_DEVICE: return "device error";
  }
  return "unknown status";
}

const char* ispl_last_error(void) { return g_last_error.c_str(); }

ispl_status ispl_plan(const ispl_config* cfg, int32_t n_pulses, int32_t* chunks,
                      int32_t* waves_per_block, int32_t* blocks) {
  const ispl_status st = validate_config(cfg);
  if (st != ISPL_OK) return st;
  if (n_pulses < 0 || n_pulses > cfg->max_pulses)
    return fail(ISPL_ERR_INVALID_ARG, "n_pulses %d outside [0, max_pulses %d]", n_pulses,
                cfg->max_pulses);
  const Plan pl = make_plan(*cfg, n_pulses > 0 ? n_pulses : 1);
  if (chunks) *chunks = n_pulses > 0 ? pl.chunks : 0;
  if (waves_per_block) *waves_per_block = pl.rw;
  if (blocks) *blocks = n_pulses > 0 ? static_cast<int32_t>(pl.blocks) : 0;
  return ok();
}

// The device exists and is a gfx950.
static ispl_status check_device(int32_t device) {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0)
    return fail(ISPL_ERR_DEVICE, "no HIP device (%s)", hipGetErrorString(e));
  if (device >= count) return fail(ISPL_ERR_DEVICE, "device %d of %d", device, count);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(ISPL_ERR_DEVICE, "device %d is %s; this library is built for gfx950", device,
                prop.gcnArchName);
  return ISPL_OK;
}

// A context whose automatic plans keep at least min_chunk_pulses pulses per
// chunk (ispl_create: kMinChunkPulses).
static ispl_status create_ctx(const ispl_config* cfg, int32_t min_chunk_pulses, ispl_ctx** out) {
  if (!out) return fail(ISPL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ispl_status st = validate_config(cfg);
  if (st != ISPL_OK) return st;

  st = check_device(cfg->device);
  if (st != ISPL_OK) return st;

  DeviceGuard guard(cfg->device);
  hipError_t e;
  ispl_ctx* ctx = new (std::nothrow) ispl_ctx{};
  if (!ctx) return fail(ISPL_ERR_OUT_OF_MEMORY, "host allocation");
  ctx->cfg = *cfg;
  ctx->min_chunk_pulses = min_chunk_pulses;
  const Plan worst = make_plan(*cfg, cfg->max_pulses, 0, 0, min_chunk_pulses);

  const std::vector<float> tw = twiddle_table(cfg->fft_len);
  e = hipMalloc(reinterpret_cast<void**>(&ctx->twiddle), tw.size() * sizeof(float));
  if (e != hipSuccess) {
    delete ctx;
    return fail(ISPL_ERR_OUT_OF_MEMORY, "twiddle table: %s", hipGetErrorString(e));
  }
  e = hipMemcpy(ctx->twiddle, tw.data(), tw.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(ctx->twiddle);
    delete ctx;
    return hip_fail(e, "twiddle upload");
  }
  // A plan's chunk count is its unclamped count capped at n_pulses, so the
  // plan for max_pulses has the largest one and bounds the partial buffer.
  const int32_t cmax = worst.chunks;
  ctx->chunks_max = cmax;
  if (cmax > 1) {
    const size_t bytes = static_cast<size_t>(cmax) * cfg->n_gates * cfg->fft_len * sizeof(float);
    e = hipMalloc(reinterpret_cast<void**>(&ctx->partial), bytes);
    if (e != hipSuccess) {
      (void)hipFree(ctx->twiddle);
      delete ctx;
      return fail(ISPL_ERR_OUT_OF_MEMORY, "chunk partials (%zu bytes): %s", bytes,
                  hipGetErrorString(e));
    }
  }
  if (cfg->code_len > 2 * ispl::SUB) {  // the long-code kernel reads binary codes as sign bits
    const size_t rows = static_cast<size_t>(cfg->max_pulses);
    e = hipMalloc(reinterpret_cast<void**>(&ctx->code_bits),
                  rows * ispl::CODE_BITS_WORDS * sizeof(uint16_t));
    if (e == hipSuccess)
      e = hipMalloc(reinterpret_cast<void**>(&ctx->code_binary), rows * sizeof(int32_t));
    if (e != hipSuccess) {
      if (ctx->code_bits) (void)hipFree(ctx->code_bits);
      if (ctx->partial) (void)hipFree(ctx->partial);
      (void)hipFree(ctx->twiddle);
      delete ctx;
      return fail(ISPL_ERR_OUT_OF_MEMORY, "code sign bits: %s", hipGetErrorString(e));
    }
  }
  *out = ctx;
  return ok();
}

ispl_status ispl_create(const ispl_config* cfg, ispl_ctx** out) {
  return create_ctx(cfg, kMinChunkPulses, out);
}

void ispl_destroy(ispl_ctx* ctx) {
  if (!ctx) return;
  {
    DeviceGuard guard(ctx->cfg.device);
    (void)hipDeviceSynchronize();
    if (ctx->partial) (void)hipFree(ctx->partial);
    if (ctx->twiddle) (void)hipFree(ctx->twiddle);
    if (ctx->code_bits) (void)hipFree(ctx->code_bits);
    if (ctx->code_binary) (void)hipFree(ctx->code_binary);
  }
  delete ctx;
}

// Arguments of one integration against the geometry c (nothing is launched).
static ispl_status check_integrate_args(const ispl_config& c, const void* samples,
                                        const float* tx_code, int32_t tx_per_pulse,
                                        int32_t n_pulses, const float* spectra,
                                        int32_t accumulate) {
  if (n_pulses < 0 || n_pulses > c.max_pulses)
    return fail(ISPL_ERR_INVALID_ARG, "n_pulses %d outside [0, max_pulses %d]", n_pulses,
                c.max_pulses);
  if (!spectra) return fail(ISPL_ERR_INVALID_ARG, "spectra is NULL");
  if (misaligned(spectra, 4)) return fail(ISPL_ERR_INVALID_ARG, "spectra not 4-byte aligned");
  if (n_pulses > 0) {
    if (!samples) return fail(ISPL_ERR_INVALID_ARG, "samples is NULL");
    if (!tx_code) return fail(ISPL_ERR_INVALID_ARG, "tx_code is NULL");
    const size_t sa = c.sample_type == ISPL_SAMPLES_CI16 ? 4 : 8;
    if (misaligned(samples, sa))
      return fail(ISPL_ERR_INVALID_ARG, "samples not %zu-byte aligned", sa);
    if (misaligned(tx_code, 8)) return fail(ISPL_ERR_INVALID_ARG, "tx_code not 8-byte aligned");
  }
  if ((tx_per_pulse != 0 && tx_per_pulse != 1) || (accumulate != 0 && accumulate != 1))
    return fail(ISPL_ERR_INVALID_ARG, "tx_per_pulse and accumulate must be 0 or 1");
  return ISPL_OK;
}

// Adaptive chunking of a gate-list launch (see ispl::FusedArgs): partial rows
// by list slot in `partial` ([rows][N]); the chunk count follows from the
// device-side list length, so the partials are always left for the caller to
// sum (ispl::launch_split_peaks does).
struct AdaptiveFallback {
  float* partial;
  int32_t target, max_chunks, rows;
};

// The adaptive parameters for a context's fallback launches over n_pulses: at
// most one round of the chip, at most 64 chunks (the reduction reads each
// chunk's row) of at least kMinChunkPulses pulses.
static AdaptiveFallback adaptive_plan(const ispl_config& c, int32_t n_pulses, float* partial) {
  const Plan pl = make_plan(c, n_pulses > 0 ? n_pulses : 1);
  int per_cu = kLdsPerCu / ispl::fused_lds_bytes(pl.rw, pl.sub_len);
  if (per_cu * pl.rw > kMaxWavesPerCu) per_cu = kMaxWavesPerCu / pl.rw;
  if (per_cu < 1) per_cu = 1;
  AdaptiveFallback f{};
  f.partial = partial;
  f.target = kComputeUnits * per_cu;
  f.rows = f.target / pl.zgroups;
  f.max_chunks = std::max(1, std::min(64, n_pulses / kMinChunkPulses));
  return f;
}

static int32_t adaptive_zgroups(const ispl_config& c) { return make_plan(c, 1).zgroups; }

// With deferred_chunks non-NULL a pulse-chunked plan leaves its partial
// spectra in the context's scratch ([C][G][N]) instead of reducing them into
// `spectra`; *deferred_chunks reports C (1: `spectra` holds the result).
// With `adapt` (gate lists only) the chunking is adaptive and its partials
// are always left in adapt->partial (*deferred_chunks = 0).
static ispl_status integrate_impl(ispl_ctx* ctx, const void* samples, const float* tx_code,
                                  int32_t tx_per_pulse, int32_t n_pulses,
                                  const int32_t* gate_list, const int32_t* gate_count,
                                  float* spectra, int32_t accumulate, void* stream,
                                  int32_t* deferred_chunks = nullptr,
                                  const AdaptiveFallback* adapt = nullptr) {
  if (deferred_chunks) *deferred_chunks = 1;
  if (adapt && (!gate_list || !deferred_chunks || accumulate))
    return fail(ISPL_ERR_INVALID_ARG, "internal: adaptive chunking needs a list and no accumulate");
  if (!ctx) return fail(ISPL_ERR_INVALID_ARG, "context is NULL");
  const ispl_config& c = ctx->cfg;
  const ispl_status st =
      check_integrate_args(c, samples, tx_code, tx_per_pulse, n_pulses, spectra, accumulate);
  if (st != ISPL_OK) return st;

  DeviceGuard guard(c.device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t elems = static_cast<int64_t>(c.n_gates) * c.fft_len;
  hipError_t e;
  if (n_pulses == 0) {
    if (!accumulate) {
      e = gate_list ? ispl::launch_fill_zero_rows(spectra, c.n_gates, c.fft_len, gate_list,
                                                  gate_count, s)
                    : ispl::launch_fill_zero(spectra, elems, s);
      if (e != hipSuccess) return hip_fail(e, "fill_zero launch");
    }
    return ok();
  }
  Plan pl = make_plan(c, n_pulses, ctx->force_rw, ctx->force_chunks, ctx->min_chunk_pulses);
  // a tuned tile shape can ask for more chunks than the scratch was sized for;
  // fewer chunks only change how the pulses are split
  if (pl.chunks > ctx->chunks_max) pl.chunks = ctx->chunks_max;

  ispl::FusedArgs a{};
  a.samples = samples;
  a.tx = tx_code;
  a.twiddle = ctx->twiddle;
  a.out = pl.chunks == 1 ? spectra : ctx->partial;
  a.stride = c.pulse_stride;
  a.n_fft = c.fft_len;
  a.sub_len = pl.sub_len;
  a.log2_r = ilog2(pl.r);
  a.code_len = c.code_len;
  a.n_gates = c.n_gates;
  a.gate_step = c.gate_step;
  a.first_gate = c.first_gate;
  a.n_pulses = n_pulses;
  a.chunks = pl.chunks;
  a.tx_per_pulse = tx_per_pulse;
  a.accumulate = accumulate;
  a.sample_type = c.sample_type;
  a.waves_per_block = pl.rw;
  a.gate_list = gate_list;
  a.gate_count = gate_count;
  if (adapt) {
    a.out = spectra;
    a.chunks = 1;
    a.adapt_partial = adapt->partial;
    a.adapt_target = adapt->target;
    a.adapt_max_chunks = adapt->max_chunks;
    a.adapt_rows = adapt->rows;
  }
  if (ctx->code_bits) {  // binary code rows go to the long-code kernel as sign bits
    const int32_t rows = tx_per_pulse ? n_pulses : 1;
    e = ispl::launch_pack_code_bits(tx_code, rows, c.code_len, ctx->code_bits, ctx->code_binary,
                                    s);
    if (e != hipSuccess) return hip_fail(e, "code bits launch");
    a.code_bits = ctx->code_bits;
    a.code_binary = ctx->code_binary;
  }
  e = ispl::launch_fused(a, s);
  if (e != hipSuccess) return hip_fail(e, "fused launch");
  if (adapt) {
    *deferred_chunks = 0;
    return ok();
  }
  if (pl.chunks > 1) {
    if (deferred_chunks && !accumulate) {
      *deferred_chunks = pl.chunks;
      return ok();
    }
    e = ispl::launch_reduce_chunks(ctx->partial, spectra, elems, pl.chunks, accumulate,
                                   c.fft_len, gate_list, gate_count, s);
    if (e != hipSuccess) return hip_fail(e, "chunk reduce launch");
  }
  return ok();
}

static ispl_status check_gate_list(const int32_t* gate_list, const int32_t* gate_count) {
  if (!gate_list || !gate_count) return fail(ISPL_ERR_INVALID_ARG, "gate_list or gate_count is NULL");
  if (misaligned(gate_list, 4) || misaligned(gate_count, 4))
    return fail(ISPL_ERR_INVALID_ARG, "gate_list or gate_count not 4-byte aligned");
  return ISPL_OK;
}

ispl_status ispl_integrate_spectra(ispl_ctx* ctx, const void* samples, const float* tx_code,
                                   int32_t tx_per_pulse, int32_t n_pulses, float* spectra,
                                   int32_t accumulate, void* stream) {
  return integrate_impl(ctx, samples, tx_code, tx_per_pulse, n_pulses, nullptr, nullptr, spectra,
                        accumulate, stream);
}

ispl_status ispl_integrate_spectra_gates(ispl_ctx* ctx, const void* samples,
                                         const float* tx_code, int32_t tx_per_pulse,
                                         int32_t n_pulses, const int32_t* gate_list,
                                         const int32_t* gate_count, float* spectra,
                                         int32_t accumulate, void* stream) {
  const ispl_status st = check_gate_list(gate_list, gate_count);
  if (st != ISPL_OK) return st;
  return integrate_impl(ctx, samples, tx_code, tx_per_pulse, n_pulses, gate_list, gate_count,
                        spectra, accumulate, stream);
}

ispl_status ispl_integrate_spectra_noalloc(const ispl_config* cfg, const void* samples,
                                           const float* tx_code, int32_t tx_per_pulse,
                                           int32_t n_pulses, float* spectra, int32_t accumulate,
                                           void* stream) {
  ispl_status st = validate_config(cfg);
  if (st != ISPL_OK) return st;
  st = check_integrate_args(*cfg, samples, tx_code, tx_per_pulse, n_pulses, spectra, accumulate);
  if (st != ISPL_OK) return st;
  // the plan of a context created from cfg; its partials stay below 64 MiB
  // (chunks x workgroups per chunk < 4 x the chip's workgroup slots), which
  // the static array holds
  const Plan pl = make_plan(*cfg, n_pulses > 0 ? n_pulses : 1);
  const int64_t row_bytes = static_cast<int64_t>(cfg->n_gates) * cfg->fft_len * 4;
  if (pl.chunks > 1 &&
      pl.chunks * row_bytes > static_cast<int64_t>(ispl::NOALLOC_PARTIAL_BYTES))
    return fail(ISPL_ERR_UNSUPPORTED,
                "plan needs %lld bytes of chunk partials; the static scratch holds %zu",
                static_cast<long long>(pl.chunks * row_bytes), ispl::NOALLOC_PARTIAL_BYTES);
  if (static_cast<size_t>(cfg->fft_len) * 8 > ispl::NOALLOC_TWIDDLE_BYTES)
    return fail(ISPL_ERR_UNSUPPORTED, "fft_len %d: twiddle table exceeds the static scratch",
                cfg->fft_len);
  // the gfx950 check once per device (device properties are not cheap)
  static std::atomic<int> checked[64];
  if (cfg->device >= 64) return fail(ISPL_ERR_UNSUPPORTED, "device %d >= 64", cfg->device);
  if (checked[cfg->device].load(std::memory_order_acquire) == 0) {
    st = check_device(cfg->device);
    if (st != ISPL_OK) return st;
    checked[cfg->device].store(1, std::memory_order_release);
  }
  DeviceGuard guard(cfg->device);
  unsigned char* base = nullptr;
  hipError_t e = ispl::noalloc_scratch(cfg->device, &base);
  if (e != hipSuccess) return hip_fail(e, "static scratch lookup");
  // a context on the stack whose tables are the static array's regions
  ispl_ctx tmp{};
  tmp.cfg = *cfg;
  tmp.chunks_max = pl.chunks;
  tmp.twiddle = reinterpret_cast<float*>(base);
  tmp.partial = pl.chunks > 1 ? reinterpret_cast<float*>(base + ispl::NOALLOC_TWIDDLE_BYTES)
                              : nullptr;
  tmp.min_chunk_pulses = kMinChunkPulses;
  if (n_pulses > 0) {
    e = ispl::launch_build_twiddles(tmp.twiddle, cfg->fft_len, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "twiddle launch");
  }
  return integrate_impl(&tmp, samples, tx_code, tx_per_pulse, n_pulses, nullptr, nullptr, spectra,
                        accumulate, stream);
}

ispl_status ispl_zoom_create(ispl_ctx* ctx, int32_t n_bins, int32_t precision,
                             ispl_zoom** out) {
  if (!out) return fail(ISPL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(ISPL_ERR_INVALID_ARG, "context is NULL");
  const ispl_config& c = ctx->cfg;
  if (precision != ISPL_ZOOM_BF16X3 && precision != ISPL_ZOOM_FP16X3)
    return fail(ISPL_ERR_INVALID_ARG, "unknown zoom precision %d", precision);
  if (n_bins < 128 || n_bins % 128 != 0 || n_bins > c.fft_len)
    return fail(ISPL_ERR_INVALID_ARG, "n_bins %d: need a multiple of 128 in [128, fft_len %d]",
                n_bins, c.fft_len);
  const int32_t code_pad = (c.code_len + 63) / 64 * 64;
  const int64_t bytes = int64_t{6} * n_bins * code_pad;  // one of the two split tables
  if (bytes > (int64_t{512} << 20))
    return fail(ISPL_ERR_UNSUPPORTED, "zoom table of %lld bytes exceeds 512 MiB",
                static_cast<long long>(bytes));
  std::vector<uint16_t> hi, lo;
  zoom_table(c.fft_len, n_bins, c.code_len, code_pad, precision, hi, lo);
  DeviceGuard guard(c.device);
  ispl_zoom* z = new (std::nothrow) ispl_zoom{};
  if (!z) return fail(ISPL_ERR_OUT_OF_MEMORY, "host allocation");
  z->ctx = ctx;
  z->n_bins = n_bins;
  z->precision = precision;
  z->code_pad = code_pad;
  z->chunks_max = zoom_plan(c.n_gates, n_bins, c.max_pulses).chunks;
  const size_t half = hi.size() * sizeof(uint16_t);
  hipError_t e = hipMalloc(&z->a_hi, half);
  if (e == hipSuccess) e = hipMalloc(&z->a_lo, half);
  if (e == hipSuccess && z->chunks_max > 1)
    e = hipMalloc(&z->partial, sizeof(float) * static_cast<size_t>(z->chunks_max) * c.n_gates *
                                   static_cast<size_t>(n_bins));
  if (e == hipSuccess && precision == ISPL_ZOOM_FP16X3)
    e = hipMalloc(&z->col_exp, sizeof(int32_t) * static_cast<size_t>(c.max_pulses));
  if (e == hipSuccess)
    e = hipMalloc(&z->code_bits, sizeof(uint32_t) * static_cast<size_t>(c.max_pulses) *
                                     static_cast<size_t>(code_pad / 32));
  if (e == hipSuccess)
    e = hipMalloc(&z->code_binary, sizeof(int32_t) * static_cast<size_t>(c.max_pulses));
  if (e != hipSuccess) {
    zoom_free(z);
    delete z;
    return fail(ISPL_ERR_OUT_OF_MEMORY, "zoom table: %s", hipGetErrorString(e));
  }
  e = hipMemcpy(z->a_hi, hi.data(), half, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(z->a_lo, lo.data(), half, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    zoom_free(z);
    delete z;
    return hip_fail(e, "zoom table upload");
  }
  *out = z;
  return ok();
}

void ispl_zoom_destroy(ispl_zoom* z) {
  if (!z) return;
  {
    DeviceGuard guard(z->ctx->cfg.device);
    (void)hipDeviceSynchronize();
    zoom_free(z);
  }
  delete z;
}

// deferred_chunks: as for integrate_impl (partial windows [C][G][K] stay in
// the zoom's scratch).  exponents_ready: the per-pulse pass has already
// written the FP16 column exponents and the code sign bits into the zoom's
// col_exp and code_bits (see launch_select_and_exponents).
static ispl_status zoom_impl(ispl_zoom* z, const void* samples, const float* tx_code,
                             int32_t tx_per_pulse, int32_t n_pulses, const int32_t* bin_start,
                             const int32_t* gate_list, const int32_t* gate_count, float* spectra,
                             int32_t accumulate, void* stream, int32_t* deferred_chunks = nullptr,
                             bool exponents_ready = false) {
  if (deferred_chunks) *deferred_chunks = 1;
  if (!z) return fail(ISPL_ERR_INVALID_ARG, "zoom is NULL");
  const ispl_config& c = z->ctx->cfg;
  if (n_pulses < 0 || n_pulses > c.max_pulses)
    return fail(ISPL_ERR_INVALID_ARG, "n_pulses %d outside [0, max_pulses %d]", n_pulses,
                c.max_pulses);
  if (!spectra || !bin_start) return fail(ISPL_ERR_INVALID_ARG, "spectra or bin_start is NULL");
  if (misaligned(spectra, 4) || misaligned(bin_start, 4))
    return fail(ISPL_ERR_INVALID_ARG, "spectra or bin_start not 4-byte aligned");
  if (n_pulses > 0) {
    if (!samples || !tx_code) return fail(ISPL_ERR_INVALID_ARG, "samples or tx_code is NULL");
    const size_t sa = c.sample_type == ISPL_SAMPLES_CI16 ? 4 : 8;
    if (misaligned(samples, sa) || misaligned(tx_code, 8))
      return fail(ISPL_ERR_INVALID_ARG, "samples or tx_code misaligned");
  }
  if ((tx_per_pulse != 0 && tx_per_pulse != 1) || (accumulate != 0 && accumulate != 1))
    return fail(ISPL_ERR_INVALID_ARG, "tx_per_pulse and accumulate must be 0 or 1");
  DeviceGuard guard(c.device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n_pulses == 0) {
    if (!accumulate) {
      const hipError_t e =
          gate_list ? ispl::launch_fill_zero_rows(spectra, c.n_gates, z->n_bins, gate_list,
                                                  gate_count, s)
                    : ispl::launch_fill_zero(spectra, static_cast<int64_t>(c.n_gates) * z->n_bins, s);
      if (e != hipSuccess) return hip_fail(e, "fill_zero launch");
    }
    return ok();
  }
  ispl::ZoomArgs a{};
  a.samples = samples;
  a.tx = tx_code;
  a.twiddle = z->ctx->twiddle;
  a.a_hi = z->a_hi;
  a.a_lo = z->a_lo;
  a.bin_start = bin_start;
  a.out = spectra;
  a.stride = c.pulse_stride;
  a.n_fft = c.fft_len;
  a.code_len = c.code_len;
  a.code_pad = z->code_pad;
  a.n_gates = c.n_gates;
  a.gate_step = c.gate_step;
  a.first_gate = c.first_gate;
  a.n_pulses = n_pulses;
  a.n_bins = z->n_bins;
  a.tx_per_pulse = tx_per_pulse;
  a.accumulate = accumulate;
  a.sample_type = c.sample_type;
  a.precision = z->precision;
  a.gate_list = gate_list;
  a.gate_count = gate_count;
  const ZoomPlan zp = zoom_plan(c.n_gates, z->n_bins, n_pulses);
  if (zp.chunks > z->chunks_max)
    return fail(ISPL_ERR_INVALID_ARG, "internal: zoom plan needs %d chunks > %d", zp.chunks,
                z->chunks_max);
  a.chunks = zp.chunks;
  a.row_tiles = zp.rt;
  a.col_tiles = zp.ct;
  a.partial = z->partial;
  a.col_exp = z->col_exp;
  a.code_bits = z->code_bits;
  a.code_binary = z->code_binary;
  a.row_lo = c.first_gate;
  a.row_hi = static_cast<int64_t>(c.first_gate) + static_cast<int64_t>(c.n_gates - 1) * c.gate_step +
             c.code_len;
  hipError_t e = ispl::launch_zoom(a, s, !exponents_ready);
  if (e != hipSuccess) return hip_fail(e, "zoom launch");
  if (zp.chunks > 1 && deferred_chunks && !accumulate) {
    *deferred_chunks = zp.chunks;
    return ok();
  }
  if (zp.chunks > 1) {
    e = ispl::launch_reduce_chunks(z->partial, spectra, static_cast<int64_t>(c.n_gates) * z->n_bins,
                                   zp.chunks, accumulate, z->n_bins, gate_list, gate_count, s);
    if (e != hipSuccess) return hip_fail(e, "zoom chunk reduce launch");
  }
  return ok();
}

ispl_status ispl_zoom_spectra(ispl_zoom* z, const void* samples, const float* tx_code,
                              int32_t tx_per_pulse, int32_t n_pulses, const int32_t* bin_start,
                              float* spectra, int32_t accumulate, void* stream) {
  return zoom_impl(z, samples, tx_code, tx_per_pulse, n_pulses, bin_start, nullptr, nullptr,
                   spectra, accumulate, stream);
}

ispl_status ispl_zoom_spectra_gates(ispl_zoom* z, const void* samples, const float* tx_code,
                                    int32_t tx_per_pulse, int32_t n_pulses,
                                    const int32_t* bin_start, const int32_t* gate_list,
                                    const int32_t* gate_count, float* spectra, int32_t accumulate,
                                    void* stream) {
  const ispl_status st = check_gate_list(gate_list, gate_count);
  if (st != ISPL_OK) return st;
  return zoom_impl(z, samples, tx_code, tx_per_pulse, n_pulses, bin_start, gate_list, gate_count,
                   spectra, accumulate, stream);
}

ispl_status ispl_zoom_find_peaks(ispl_zoom* z, const float* spectra, const int32_t* bin_start,
                                 const int32_t* gate_list, const int32_t* gate_count,
                                 int32_t* peak_bin, float* peak_power, void* stream) {
  if (!z) return fail(ISPL_ERR_INVALID_ARG, "zoom is NULL");
  const ispl_status st = check_gate_list(gate_list, gate_count);
  if (st != ISPL_OK) return st;
  if (!spectra || !bin_start || !peak_bin)
    return fail(ISPL_ERR_INVALID_ARG, "spectra, bin_start or peak_bin is NULL");
  if (misaligned(spectra, 4) || misaligned(bin_start, 4) || misaligned(peak_bin, 4) ||
      misaligned(peak_power, 4))
    return fail(ISPL_ERR_INVALID_ARG, "pointer not 4-byte aligned");
  const ispl_config& c = z->ctx->cfg;
  DeviceGuard guard(c.device);
  const hipError_t e =
      ispl::launch_window_peak(spectra, c.n_gates, z->n_bins, c.fft_len, bin_start, gate_list,
                               gate_count, peak_bin, peak_power, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "window peak launch");
  return ok();
}

}  // extern "C"

struct ispl_net {
  int32_t device;
  int32_t max_batch;
  int32_t step;
  ispl::NetWork w;
  float* grad;
  float* adam_m;
  float* adam_v;
  float* bf16_weights;  // matrix-core copies, rebuilt when the parameters change
  int32_t* select_done; // completion counter of the window decision (zero between calls)
  bool bf16_stale;
};

namespace {

void net_free(ispl_net* n) {
  void* bufs[] = {n->w.params, n->w.a1, n->w.a2, n->w.a3, n->w.logits, n->w.dz4, n->w.dzA,
                  n->w.dzB, n->w.part, n->w.loss, n->grad, n->adam_m, n->adam_v,
                  n->bf16_weights, n->select_done};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
}

}  // namespace

extern "C" {

ispl_status ispl_net_create(int32_t device, int32_t max_batch, ispl_net** out) {
  if (!out) return fail(ISPL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > 65536)
    return fail(ISPL_ERR_INVALID_ARG, "max_batch %d outside [1, 65536]", max_batch);
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0)
    return fail(ISPL_ERR_DEVICE, "no HIP device (%s)", hipGetErrorString(e));
  if (device < 0 || device >= count) return fail(ISPL_ERR_DEVICE, "device %d of %d", device, count);
  DeviceGuard guard(device);
  ispl_net* n = new (std::nothrow) ispl_net{};
  if (!n) return fail(ISPL_ERR_OUT_OF_MEMORY, "host allocation");
  n->device = device;
  n->max_batch = max_batch;
  const size_t B = static_cast<size_t>(max_batch), T = ispl::NET_LEN, P = ispl::NET_PARAMS;
  struct { float** p; size_t n; } plan[] = {
      {&n->w.params, P}, {&n->w.a1, B * 32 * T}, {&n->w.a2, B * 32 * T}, {&n->w.a3, B * 32 * T},
      {&n->w.logits, B * T}, {&n->w.dz4, B * T}, {&n->w.dzA, B * 32 * T}, {&n->w.dzB, B * 32 * T},
      {&n->w.part, B * P}, {&n->w.loss, B}, {&n->grad, P}, {&n->adam_m, P}, {&n->adam_v, P},
      {&n->bf16_weights, (ispl::net_bf16_bytes() + sizeof(float) - 1) / sizeof(float)},
      {reinterpret_cast<float**>(&n->select_done), 1}};
  for (auto& a : plan) {
    e = hipMalloc(reinterpret_cast<void**>(a.p), a.n * sizeof(float));
    if (e != hipSuccess) {
      net_free(n);
      delete n;
      return fail(ISPL_ERR_OUT_OF_MEMORY, "network workspace: %s", hipGetErrorString(e));
    }
  }
  for (float* z : {n->w.params, n->adam_m, n->adam_v}) (void)hipMemset(z, 0, P * sizeof(float));
  (void)hipMemset(n->select_done, 0, sizeof(int32_t));
  e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    net_free(n);
    delete n;
    return hip_fail(e, "network init");
  }
  n->bf16_stale = true;
  *out = n;
  return ok();
}

void ispl_net_destroy(ispl_net* n) {
  if (!n) return;
  {
    DeviceGuard guard(n->device);
    (void)hipDeviceSynchronize();
    net_free(n);
  }
  delete n;
}

ispl_status ispl_net_set_params(ispl_net* n, const float* host_params) {
  if (!n || !host_params) return fail(ISPL_ERR_INVALID_ARG, "net or params is NULL");
  DeviceGuard guard(n->device);
  const size_t bytes = ispl::NET_PARAMS * sizeof(float);
  hipError_t e = hipMemcpy(n->w.params, host_params, bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(n->adam_m, 0, bytes);
  if (e == hipSuccess) e = hipMemset(n->adam_v, 0, bytes);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "set_params");
  n->step = 0;
  n->bf16_stale = true;
  return ok();
}

ispl_status ispl_net_get_params(ispl_net* n, float* host_params) {
  if (!n || !host_params) return fail(ISPL_ERR_INVALID_ARG, "net or params is NULL");
  DeviceGuard guard(n->device);
  const hipError_t e = hipMemcpy(host_params, n->w.params, ispl::NET_PARAMS * sizeof(float),
                                 hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "get_params");
  return ok();
}

ispl_status ispl_net_features(ispl_net* n, const float* spectra, int32_t rows, float* features,
                              void* stream) {
  if (!n) return fail(ISPL_ERR_INVALID_ARG, "NULL net");
  if (rows < 0) return fail(ISPL_ERR_INVALID_ARG, "rows %d < 0", rows);
  if (rows == 0) return ok();  // empty tensors may carry NULL pointers
  if (!spectra || !features) return fail(ISPL_ERR_INVALID_ARG, "NULL argument");
  if (misaligned(spectra, 16) || misaligned(features, 16))
    return fail(ISPL_ERR_INVALID_ARG, "spectra and features must be 16-byte aligned");
  DeviceGuard guard(n->device);
  const hipError_t e = ispl::launch_net_features(spectra, rows, features,
                                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "features launch");
  return ok();
}

ispl_status ispl_net_forward(ispl_net* n, const float* features, int32_t batch, float* logits,
                             int32_t precision, void* stream) {
  if (!n) return fail(ISPL_ERR_INVALID_ARG, "NULL net");
  if (precision != ISPL_NET_FP32 && precision != ISPL_NET_BF16)
    return fail(ISPL_ERR_INVALID_ARG, "unknown precision %d", precision);
  // the FP32 forward stages activations in the workspace; BF16 keeps them in LDS
  const int32_t limit = precision == ISPL_NET_FP32 ? n->max_batch : INT32_MAX;
  if (batch < 0 || batch > limit)
    return fail(ISPL_ERR_INVALID_ARG, "batch %d outside [0, %d]", batch, limit);
  if (batch == 0) return ok();  // empty tensors may carry NULL pointers
  if (!features || !logits) return fail(ISPL_ERR_INVALID_ARG, "NULL argument");
  if (misaligned(features, 16) || misaligned(logits, 16))
    return fail(ISPL_ERR_INVALID_ARG, "features and logits must be 16-byte aligned");
  DeviceGuard guard(n->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (precision == ISPL_NET_BF16) {
    if (n->bf16_stale) {
      e = ispl::launch_net_prep_bf16(n->w.params, n->bf16_weights, s);
      if (e != hipSuccess) return hip_fail(e, "bf16 weight prep launch");
      n->bf16_stale = false;
    }
    e = ispl::launch_net_forward_bf16(n->bf16_weights, features, batch, logits, s);
  } else {
    e = ispl::launch_net_forward_f32(n->w, features, batch, logits, s);
  }
  if (e != hipSuccess) return hip_fail(e, "forward launch");
  return ok();
}

ispl_status ispl_net_loss_grad(ispl_net* n, const float* features, const float* target_pos,
                               int32_t batch, float* grad, float* loss, void* stream) {
  if (!n || !features || !target_pos || !grad || !loss)
    return fail(ISPL_ERR_INVALID_ARG, "NULL argument");
  if (batch < 1 || batch > n->max_batch)
    return fail(ISPL_ERR_INVALID_ARG, "batch %d outside [1, max_batch %d]", batch, n->max_batch);
  if (misaligned(features, 16)) return fail(ISPL_ERR_INVALID_ARG, "features not 16-byte aligned");
  DeviceGuard guard(n->device);
  const hipError_t e = ispl::launch_net_loss_grad(n->w, features, target_pos, batch, grad, loss,
                                                  static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "loss_grad launch");
  return ok();
}

ispl_status ispl_net_train_step(ispl_net* n, const float* features, const float* target_pos,
                                int32_t batch, float lr, float* loss, void* stream) {
  const ispl_status st = ispl_net_loss_grad(n, features, target_pos, batch, n ? n->grad : nullptr,
                                            loss, stream);
  if (st != ISPL_OK) return st;
  if (!(lr > 0.f)) return fail(ISPL_ERR_INVALID_ARG, "learning rate must be > 0");
  DeviceGuard guard(n->device);
  n->step += 1;
  n->bf16_stale = true;
  const hipError_t e = ispl::launch_adam(n->w.params, n->grad, n->adam_m, n->adam_v,
                                         ispl::NET_PARAMS, lr, n->step,
                                         static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "adam launch");
  return ok();
}

static ispl_status peak_impl(ispl_ctx* ctx, const float* spectra, int32_t bin_lo,
                             int32_t bin_hi, const int32_t* gate_list, const int32_t* gate_count,
                             int32_t* peak_bin, float* peak_power, void* stream) {
  if (!ctx) return fail(ISPL_ERR_INVALID_ARG, "context is NULL");
  const ispl_config& c = ctx->cfg;
  if (!spectra || !peak_bin) return fail(ISPL_ERR_INVALID_ARG, "spectra or peak_bin is NULL");
  if (misaligned(spectra, 4) || misaligned(peak_bin, 4) || misaligned(peak_power, 4))
    return fail(ISPL_ERR_INVALID_ARG, "pointer not 4-byte aligned");
  if (bin_lo < 0 || bin_lo >= c.fft_len || bin_hi < 1 || bin_hi > c.fft_len || bin_lo == bin_hi)
    return fail(ISPL_ERR_INVALID_ARG, "band [%d, %d) invalid for fft_len %d", bin_lo, bin_hi,
                c.fft_len);
  DeviceGuard guard(c.device);
  const hipError_t e =
      ispl::launch_peak(spectra, c.n_gates, c.fft_len, bin_lo, bin_hi, peak_bin, peak_power,
                        gate_list, gate_count, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "peak launch");
  return ok();
}

ispl_status ispl_find_plasma_line(ispl_ctx* ctx, const float* spectra, int32_t bin_lo,
                                  int32_t bin_hi, int32_t* peak_bin, float* peak_power,
                                  void* stream) {
  return peak_impl(ctx, spectra, bin_lo, bin_hi, nullptr, nullptr, peak_bin, peak_power, stream);
}

ispl_status ispl_find_plasma_line_gates(ispl_ctx* ctx, const float* spectra, int32_t bin_lo,
                                        int32_t bin_hi, const int32_t* gate_list,
                                        const int32_t* gate_count, int32_t* peak_bin,
                                        float* peak_power, void* stream) {
  const ispl_status st = check_gate_list(gate_list, gate_count);
  if (st != ISPL_OK) return st;
  return peak_impl(ctx, spectra, bin_lo, bin_hi, gate_list, gate_count, peak_bin, peak_power,
                   stream);
}

static ispl_status check_window(int32_t fine_len, int32_t window_bins, float threshold) {
  if (fine_len < ispl::NET_LEN || fine_len % ispl::NET_LEN != 0 || !is_pow2(fine_len))
    return fail(ISPL_ERR_INVALID_ARG, "fine_len %d: need a power of two >= %d", fine_len,
                ispl::NET_LEN);
  const int32_t S = fine_len / ispl::NET_LEN;
  if (window_bins < 1 || window_bins > fine_len || window_bins / 2 <= S)
    return fail(ISPL_ERR_INVALID_ARG, "window_bins %d: need 2 * %d < window_bins <= %d",
                window_bins, S, fine_len);
  if (!(threshold > 0.f && threshold <= 1.f))
    return fail(ISPL_ERR_INVALID_ARG, "threshold must lie in (0, 1]");
  return ISPL_OK;
}

static void bf16_table_ready(ispl_net* n, hipStream_t s, hipError_t* e) {
  *e = hipSuccess;
  if (n->bf16_stale) {
    *e = ispl::launch_net_prep_bf16(n->w.params, n->bf16_weights, s);
    if (*e == hipSuccess) n->bf16_stale = false;
  }
}

ispl_status ispl_net_select(ispl_net* n, const float* logits, int32_t n_gates, int32_t fine_len,
                            int32_t window_bins, float threshold, int32_t* bin_start,
                            float* confidence, int32_t* flag, int32_t* zoom_list,
                            int32_t* fallback_list, int32_t* counts, void* stream) {
  if (!n) return fail(ISPL_ERR_INVALID_ARG, "NULL net");
  ispl_status st = check_window(fine_len, window_bins, threshold);
  if (st != ISPL_OK) return st;
  if (n_gates < 1) return fail(ISPL_ERR_INVALID_ARG, "n_gates %d < 1", n_gates);
  if (!logits || !bin_start || !flag || !zoom_list || !fallback_list || !counts)
    return fail(ISPL_ERR_INVALID_ARG, "NULL argument");
  if (misaligned(logits, 16)) return fail(ISPL_ERR_INVALID_ARG, "logits must be 16-byte aligned");
  if (misaligned(bin_start, 4) || misaligned(confidence, 4) || misaligned(flag, 4) ||
      misaligned(zoom_list, 4) || misaligned(fallback_list, 4) || misaligned(counts, 4))
    return fail(ISPL_ERR_INVALID_ARG, "pointer not 4-byte aligned");
  DeviceGuard guard(n->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const hipError_t e =
      ispl::launch_select_windows(logits, n_gates, fine_len, window_bins, threshold, bin_start,
                                  confidence, flag, zoom_list, fallback_list, counts,
                                  n->select_done, s);
  if (e != hipSuccess) return hip_fail(e, "select launch");
  return ok();
}

}  // extern "C"

struct ispl_lzoom {
  ispl_ctx* coarse;
  ispl_ctx* fine;
  ispl_zoom* zoom;
  ispl_net* net;
  int32_t n_gates;
  int32_t window_bins;
  float threshold;
  float* coarse_spectra;  // [G][1024]
  float* logits;          // [G][1024]
  float* confidence;      // [G]
  float* window_spectra;  // [G][K]
  float* full_spectra;    // [G][N]
  int32_t* bin_start;     // [G]
  int32_t* flag;          // [G]
  int32_t* zoom_list;     // [G]
  int32_t* fallback_list; // [G]
  int32_t* counts;        // [2]: zoomed, fallback
  int32_t* done;          // completion counter of the decision (zero between calls)
  float* fb_partial;      // [fb_rows][N]: chunk partials of the fallback launch
  int32_t fb_rows;
};

namespace {

void lzoom_free(ispl_lzoom* z) {
  void* bufs[] = {z->coarse_spectra, z->logits, z->confidence, z->window_spectra,
                  z->full_spectra, z->bin_start, z->flag, z->zoom_list, z->fallback_list,
                  z->counts, z->done, z->fb_partial};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (z->zoom) ispl_zoom_destroy(z->zoom);
  if (z->fine) ispl_destroy(z->fine);
  if (z->coarse) ispl_destroy(z->coarse);
}

}  // namespace

extern "C" {

ispl_status ispl_lzoom_create(const ispl_config* cfg, ispl_net* net, int32_t window_bins,
                              int32_t zoom_precision, float threshold, ispl_lzoom** out) {
  if (!out) return fail(ISPL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!net) return fail(ISPL_ERR_INVALID_ARG, "NULL net");
  ispl_status st = validate_config(cfg);
  if (st != ISPL_OK) return st;
  if (cfg->device != net->device)
    return fail(ISPL_ERR_INVALID_ARG, "net is on device %d, config on %d", net->device,
                cfg->device);
  if (cfg->code_len > ispl::NET_LEN)
    return fail(ISPL_ERR_UNSUPPORTED, "code_len %d > %d: the coarse spectrum would truncate it",
                cfg->code_len, ispl::NET_LEN);
  st = check_window(cfg->fft_len, window_bins, threshold);
  if (st != ISPL_OK) return st;
  ispl_lzoom* z = new (std::nothrow) ispl_lzoom{};
  if (!z) return fail(ISPL_ERR_OUT_OF_MEMORY, "host allocation");
  z->net = net;
  z->n_gates = cfg->n_gates;
  z->window_bins = window_bins;
  z->threshold = threshold;
  ispl_config cc = *cfg;
  cc.fft_len = ispl::NET_LEN;
  // the coarse transforms are short: chunks of 4 pulses give enough waves to
  // fill the chip on small workloads, and the network sums the partials
  st = create_ctx(&cc, 4, &z->coarse);
  // the fine context runs only the fallback, whose chunking is adaptive and
  // whose partials live in the object's own buffer: no scratch of its own
  if (st == ISPL_OK) st = create_ctx(cfg, INT32_MAX, &z->fine);
  if (st == ISPL_OK) st = ispl_zoom_create(z->fine, window_bins, zoom_precision, &z->zoom);
  if (st != ISPL_OK) {
    const std::string why = g_last_error;
    lzoom_free(z);
    delete z;
    return fail(st, "%s", why.c_str());
  }
  DeviceGuard guard(cfg->device);
  const int64_t G = cfg->n_gates;
  z->fb_rows = adaptive_plan(*cfg, cfg->max_pulses, nullptr).rows;
  struct {
    void** p;
    int64_t bytes;
  } want[] = {{reinterpret_cast<void**>(&z->coarse_spectra), 4 * G * ispl::NET_LEN},
              {reinterpret_cast<void**>(&z->logits), 4 * G * ispl::NET_LEN},
              {reinterpret_cast<void**>(&z->confidence), 4 * G},
              {reinterpret_cast<void**>(&z->window_spectra), 4 * G * window_bins},
              {reinterpret_cast<void**>(&z->full_spectra), 4 * G * cfg->fft_len},
              {reinterpret_cast<void**>(&z->bin_start), 4 * G},
              {reinterpret_cast<void**>(&z->flag), 4 * G},
              {reinterpret_cast<void**>(&z->zoom_list), 4 * G},
              {reinterpret_cast<void**>(&z->fallback_list), 4 * G},
              {reinterpret_cast<void**>(&z->counts), 8},
              {reinterpret_cast<void**>(&z->done), 4},
              {reinterpret_cast<void**>(&z->fb_partial), int64_t{4} * z->fb_rows * cfg->fft_len}};
  for (auto& w : want) {
    const hipError_t e = hipMalloc(w.p, static_cast<size_t>(w.bytes));
    if (e != hipSuccess) {
      lzoom_free(z);
      delete z;
      return fail(ISPL_ERR_OUT_OF_MEMORY, "learned-zoom buffers: %s", hipGetErrorString(e));
    }
  }
  hipError_t e = hipMemset(z->done, 0, sizeof(int32_t));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    lzoom_free(z);
    delete z;
    return hip_fail(e, "learned-zoom init");
  }
  *out = z;
  return ok();
}

void ispl_lzoom_destroy(ispl_lzoom* z) {
  if (!z) return;
  {
    DeviceGuard guard(z->fine ? z->fine->cfg.device : 0);
    (void)hipDeviceSynchronize();
    lzoom_free(z);
  }
  delete z;
}

ispl_status ispl_lzoom_peaks(ispl_lzoom* z, const void* samples, const float* tx_code,
                             int32_t tx_per_pulse, int32_t n_pulses, int32_t* peak_bin,
                             float* peak_power, void* stream) {
  if (!z) return fail(ISPL_ERR_INVALID_ARG, "learned zoom is NULL");
  if (!peak_bin) return fail(ISPL_ERR_INVALID_ARG, "peak_bin is NULL");
  if (misaligned(peak_bin, 4) || misaligned(peak_power, 4))
    return fail(ISPL_ERR_INVALID_ARG, "peak_bin or peak_power not 4-byte aligned");
  const ispl_config& c = z->fine->cfg;
  const int32_t G = z->n_gates;
  DeviceGuard guard(c.device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // coarse spectra of every gate (the plain path at N = 1024); pulse-chunk
  // partials are summed by the network kernel, which writes coarse_spectra
  int32_t coarse_chunks = 1, zoom_chunks = 1, fine_chunks = 1;
  ispl_status st = integrate_impl(z->coarse, samples, tx_code, tx_per_pulse, n_pulses, nullptr,
                                  nullptr, z->coarse_spectra, 0, stream, &coarse_chunks);
  if (st != ISPL_OK) return st;
  // network on the coarse spectra (features formed in the kernel), BF16 logits;
  // then windows, the two gate lists and the zoom's FP16 pulse exponents in
  // one launch
  hipError_t e;
  bf16_table_ready(z->net, s, &e);
  if (e == hipSuccess)
    e = ispl::launch_net_forward_bf16(z->net->bf16_weights, z->coarse_spectra, G, z->logits, s,
                                      true, z->coarse->partial, coarse_chunks, z->coarse_spectra);
  if (e == hipSuccess) {
    ispl::PulseExpArgs pe{};
    pe.samples = samples;
    pe.tx = tx_code;
    pe.exps = z->zoom->precision == ISPL_ZOOM_FP16X3 ? z->zoom->col_exp : nullptr;
    pe.bits = z->zoom->code_bits;
    pe.binary = z->zoom->code_binary;
    pe.bit_words = z->zoom->code_pad / 32;
    pe.stride = c.pulse_stride;
    pe.lo = c.first_gate;
    pe.hi = static_cast<int64_t>(c.first_gate) + static_cast<int64_t>(c.n_gates - 1) * c.gate_step +
            c.code_len;
    pe.sample_type = c.sample_type;
    pe.code_len = c.code_len;
    pe.tx_per_pulse = tx_per_pulse;
    pe.n_pulses = n_pulses > 0 ? n_pulses : 0;
    e = ispl::launch_select_and_exponents(z->logits, G, c.fft_len, z->window_bins, z->threshold,
                                          z->bin_start, z->confidence, z->flag, z->zoom_list,
                                          z->fallback_list, z->counts, z->done, pe,
                                          s);
  }
  if (e != hipSuccess) return hip_fail(e, "learned-zoom network launch");
  // zoomed gates: K bins around the proposed centre; the others: full spectra;
  // chunk partials of both are summed by the peak launch
  st = zoom_impl(z->zoom, samples, tx_code, tx_per_pulse, n_pulses, z->bin_start, z->zoom_list,
                 z->counts, z->window_spectra, 0, stream, &zoom_chunks, true);
  if (st != ISPL_OK) return st;
  // the fallback's pulse chunks follow from the device-side number of
  // fallback gates: few gates take many chunks and still fill the chip
  const AdaptiveFallback fb = adaptive_plan(c, n_pulses, z->fb_partial);
  if (fb.rows > z->fb_rows)
    return fail(ISPL_ERR_INVALID_ARG, "internal: fallback plan needs %d rows > %d", fb.rows,
                z->fb_rows);
  st = integrate_impl(z->fine, samples, tx_code, tx_per_pulse, n_pulses, z->fallback_list,
                      z->counts + 1, z->full_spectra, 0, stream, &fine_chunks, &fb);
  if (st != ISPL_OK) return st;
  ispl::FallbackChunks fc{};
  fc.counts = z->counts;
  fc.partial = z->fb_partial;
  fc.zgroups = adaptive_zgroups(c);
  fc.target = fb.target;
  fc.max_chunks = fb.max_chunks;
  fc.rows = fb.rows;
  e = ispl::launch_split_peaks(z->window_spectra, z->zoom->partial, zoom_chunks, z->full_spectra,
                               fc, z->zoom_list, z->fallback_list, z->bin_start, G,
                               z->window_bins, c.fft_len, peak_bin, peak_power, s);
  if (e != hipSuccess) return hip_fail(e, "learned-zoom peak launch");
  return ok();
}

ispl_status ispl_lzoom_view(const ispl_lzoom* z, ispl_lzoom_buffers* out) {
  if (!z || !out) return fail(ISPL_ERR_INVALID_ARG, "NULL argument");
  out->n_gates = z->n_gates;
  out->window_bins = z->window_bins;
  out->fine_len = z->fine->cfg.fft_len;
  out->coarse_spectra = z->coarse_spectra;
  out->logits = z->logits;
  out->bin_start = z->bin_start;
  out->confidence = z->confidence;
  out->zoom_list = z->zoom_list;
  out->fallback_list = z->fallback_list;
  out->counts = z->counts;
  out->window_spectra = z->window_spectra;
  out->full_spectra = z->full_spectra;
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Uneven batch: several experiments launched together from one HIP graph.

struct ispl_batch {
  int32_t n_modes;
  int32_t device;
  ispl_ctx* ctx[ispl::MAX_BATCH_MODES];
  hipStream_t branch[ispl::MAX_BATCH_MODES];  // capture streams of the parallel branches
  hipStream_t cap;
  hipEvent_t fork, join[ispl::MAX_BATCH_MODES];
  ispl_batch_plan plan;
  ispl_batch_io cached[ispl::MAX_BATCH_MODES];
  int32_t cached_acc;
  hipGraphExec_t exec;
  bool graph_valid;
  // Executable graphs replaced by a new capture.  A launch of one may still be
  // in the runtime's hands (its completion bookkeeping can outlive the events
  // that follow it), so they are destroyed only after a device-wide
  // synchronisation: when kMaxRetired have gathered, or with the object.
  hipGraphExec_t retired[8];
  int32_t n_retired;
};

namespace {

constexpr int kMaxRetired = 8;

// The caller has synchronised the device (or no graph was ever launched).
void batch_free(ispl_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  for (int i = 0; i < b->n_retired; ++i) (void)hipGraphExecDestroy(b->retired[i]);
  b->n_retired = 0;
  for (int i = 0; i < b->n_modes; ++i) {
    if (b->branch[i]) (void)hipStreamDestroy(b->branch[i]);
    if (b->join[i]) (void)hipEventDestroy(b->join[i]);
    if (b->ctx[i]) ispl_destroy(b->ctx[i]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->cap) (void)hipStreamDestroy(b->cap);
}

void apply_plan(ispl_batch* b) {
  for (int m = 0; m < b->n_modes; ++m) {
    b->ctx[m]->force_rw = b->plan.waves[m];
    b->ctx[m]->force_chunks = b->plan.chunks[m];
  }
}

ispl_status batch_run(ispl_batch* b, const ispl_batch_io* io, int32_t accumulate,
                      hipStream_t s) {
  for (int k = 0; k < b->n_modes; ++k) {
    const int m = b->plan.order[k];
    const ispl_status st = integrate_impl(b->ctx[m], io[m].samples, io[m].tx_code,
                                          io[m].tx_per_pulse, io[m].n_pulses, nullptr, nullptr,
                                          io[m].spectra, accumulate, s);
    if (st != ISPL_OK) {
      const std::string why = g_last_error;
      return fail(st, "mode %d: %s", m, why.c_str());
    }
  }
  return ISPL_OK;
}

// Captures every mode's launches: on parallel branches (fork / join events)
// or one after another in plan order, then instantiates the graph.
ispl_status batch_capture(ispl_batch* b, const ispl_batch_io* io, int32_t accumulate) {
  // until a new graph is instantiated there is none to replay, also after a
  // failed capture; the old executable is retired, never destroyed while a
  // launch of it may be in flight
  b->graph_valid = false;
  if (b->exec) {
    if (b->n_retired == kMaxRetired) {
      const hipError_t se = hipDeviceSynchronize();
      if (se != hipSuccess) return hip_fail(se, "batch: synchronise before freeing old graphs");
      for (int i = 0; i < b->n_retired; ++i) (void)hipGraphExecDestroy(b->retired[i]);
      b->n_retired = 0;
    }
    b->retired[b->n_retired++] = b->exec;
    b->exec = nullptr;
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "batch capture");
  ispl_status st = ISPL_OK;
  if (b->plan.serial) {
    st = batch_run(b, io, accumulate, b->cap);
  } else {
    e = hipEventRecord(b->fork, b->cap);
    for (int k = 0; k < b->n_modes && e == hipSuccess && st == ISPL_OK; ++k) {
      const int m = b->plan.order[k];
      e = hipStreamWaitEvent(b->branch[m], b->fork, 0);
      if (e != hipSuccess) break;
      st = integrate_impl(b->ctx[m], io[m].samples, io[m].tx_code, io[m].tx_per_pulse,
                          io[m].n_pulses, nullptr, nullptr, io[m].spectra, accumulate,
                          b->branch[m]);
      // rejoin the branch even after an error, so the capture ends cleanly
      e = hipEventRecord(b->join[m], b->branch[m]);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->join[m], 0);
    }
  }
  const hipError_t ee = hipStreamEndCapture(b->cap, &g);
  if (e == hipSuccess) e = ee;
  if (st == ISPL_OK && e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (st != ISPL_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "batch graph");
  for (int m = 0; m < b->n_modes; ++m) b->cached[m] = io[m];
  b->cached_acc = accumulate;
  b->graph_valid = true;
  return ISPL_OK;
}

// The modes' launches queued eagerly in the plan's shape: on the object's
// parallel branches (fork and join events on `s`, as the graph's branches) or
// one after another on `s`.
ispl_status batch_launch_eager(ispl_batch* b, const ispl_batch_io* io, int32_t accumulate,
                               hipStream_t s) {
  if (b->plan.serial) return batch_run(b, io, accumulate, s);
  hipError_t e = hipEventRecord(b->fork, s);
  ispl_status st = ISPL_OK;
  for (int k = 0; k < b->n_modes && e == hipSuccess && st == ISPL_OK; ++k) {
    const int m = b->plan.order[k];
    e = hipStreamWaitEvent(b->branch[m], b->fork, 0);
    if (e != hipSuccess) break;
    st = integrate_impl(b->ctx[m], io[m].samples, io[m].tx_code, io[m].tx_per_pulse,
                        io[m].n_pulses, nullptr, nullptr, io[m].spectra, accumulate,
                        b->branch[m]);
    const hipError_t je = hipEventRecord(b->join[m], b->branch[m]);
    e = je == hipSuccess ? hipStreamWaitEvent(s, b->join[m], 0) : je;
  }
  if (st != ISPL_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "batch branches");
  return ISPL_OK;
}

bool same_io(const ispl_batch_io& x, const ispl_batch_io& y) {
  return x.samples == y.samples && x.tx_code == y.tx_code && x.tx_per_pulse == y.tx_per_pulse &&
         x.n_pulses == y.n_pulses && x.spectra == y.spectra;
}

}  // namespace

extern "C" {

ispl_status ispl_batch_create(const ispl_config* cfgs, int32_t n_modes, ispl_batch** out) {
  if (!out) return fail(ISPL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!cfgs) return fail(ISPL_ERR_INVALID_ARG, "configs are NULL");
  if (n_modes < 1 || n_modes > ispl::MAX_BATCH_MODES)
    return fail(ISPL_ERR_INVALID_ARG, "n_modes %d outside [1, %d]", n_modes,
                ispl::MAX_BATCH_MODES);
  for (int m = 0; m < n_modes; ++m) {
    const ispl_status st = validate_config(&cfgs[m]);
    if (st != ISPL_OK) return st;
    if (cfgs[m].device != cfgs[0].device)
      return fail(ISPL_ERR_INVALID_ARG, "mode %d: all modes need one device", m);
  }
  ispl_batch* b = new (std::nothrow) ispl_batch{};
  if (!b) return fail(ISPL_ERR_OUT_OF_MEMORY, "host allocation");
  b->n_modes = n_modes;
  b->device = cfgs[0].device;
  for (int m = 0; m < n_modes; ++m) {
    const ispl_status st = ispl_create(&cfgs[m], &b->ctx[m]);
    if (st != ISPL_OK) {
      const std::string why = g_last_error;
      batch_free(b);
      delete b;
      return fail(st, "mode %d: %s", m, why.c_str());
    }
    b->plan.order[m] = m;
  }
  DeviceGuard guard(b->device);
  hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int m = 0; m < n_modes && e == hipSuccess; ++m) {
    e = hipStreamCreateWithFlags(&b->branch[m], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[m], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    batch_free(b);
    delete b;
    return hip_fail(e, "batch setup");
  }
  *out = b;
  return ok();
}

void ispl_batch_destroy(ispl_batch* b) {
  if (!b) return;
  {
    DeviceGuard guard(b->device);
    (void)hipDeviceSynchronize();
    batch_free(b);
  }
  delete b;
}

ispl_status ispl_batch_integrate(ispl_batch* b, const ispl_batch_io* io, int32_t accumulate,
                                 int32_t use_graph, void* stream) {
  if (!b || !io) return fail(ISPL_ERR_INVALID_ARG, "batch or io is NULL");
  if ((accumulate != 0 && accumulate != 1) || (use_graph != 0 && use_graph != 1))
    return fail(ISPL_ERR_INVALID_ARG, "accumulate and use_graph must be 0 or 1");
  DeviceGuard guard(b->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!use_graph) {
    const ispl_status st = batch_run(b, io, accumulate, s);
    return st == ISPL_OK ? ok() : st;
  }
  bool same = b->graph_valid && b->cached_acc == accumulate;
  for (int m = 0; m < b->n_modes && same; ++m) same = same_io(io[m], b->cached[m]);
  if (!same) {
    const ispl_status st = batch_capture(b, io, accumulate);
    if (st != ISPL_OK) return st;
  }
  const hipError_t e = hipGraphLaunch(b->exec, s);
  if (e != hipSuccess) return hip_fail(e, "batch graph launch");
  return ok();
}

ispl_status ispl_batch_get_plan(const ispl_batch* b, ispl_batch_plan* plan) {
  if (!b || !plan) return fail(ISPL_ERR_INVALID_ARG, "NULL argument");
  *plan = b->plan;
  return ok();
}

ispl_status ispl_batch_set_plan(ispl_batch* b, const ispl_batch_plan* plan) {
  if (!b || !plan) return fail(ISPL_ERR_INVALID_ARG, "NULL argument");
  bool seen[ispl::MAX_BATCH_MODES] = {};
  for (int k = 0; k < b->n_modes; ++k) {
    const int m = plan->order[k];
    if (m < 0 || m >= b->n_modes || seen[m])
      return fail(ISPL_ERR_INVALID_ARG, "order is not a permutation of the %d modes", b->n_modes);
    seen[m] = true;
  }
  for (int m = 0; m < b->n_modes; ++m) {
    const ispl_config& c = b->ctx[m]->cfg;
    const int w = plan->waves[m];
    const int r = c.fft_len / ispl::SUB;
    if (w != 0 && (c.code_len > ispl::SUB || !is_pow2(w) || w > 16 || w > r))
      return fail(ISPL_ERR_INVALID_ARG, "mode %d: waves %d not a power of two <= min(16, N/1024) "
                  "(or the mode has L > 1024)", m, w);
    if (plan->chunks[m] < 0 || plan->chunks[m] > b->ctx[m]->chunks_max)
      return fail(ISPL_ERR_INVALID_ARG, "mode %d: chunks %d outside [0, %d]", m, plan->chunks[m],
                  b->ctx[m]->chunks_max);
  }
  if (plan->serial != 0 && plan->serial != 1)
    return fail(ISPL_ERR_INVALID_ARG, "serial must be 0 or 1");
  b->plan = *plan;
  apply_plan(b);
  b->graph_valid = false;
  return ok();
}

ispl_status ispl_batch_tune(ispl_batch* b, const ispl_batch_io* io, int32_t trials,
                            ispl_batch_plan* best, float* best_ms) {
  if (!b || !io) return fail(ISPL_ERR_INVALID_ARG, "batch or io is NULL");
  if (trials < 1 || trials > 100)
    return fail(ISPL_ERR_INVALID_ARG, "trials %d outside [1, 100]", trials);
  DeviceGuard guard(b->device);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(e, "tune events");
  hipStream_t s = b->cap;
  // median time of the batch under a plan, its launches queued eagerly in the
  // plan's shape on the object's own streams (no graph per candidate: the
  // graph of the chosen plan is captured once, by the next ispl_batch_integrate)
  auto measure = [&](const ispl_batch_plan& p, float* ms) -> ispl_status {
    b->plan = p;
    apply_plan(b);
    std::vector<float> t;
    for (int r = 0; r <= trials; ++r) {
      hipError_t ee = hipEventRecord(e0, s);
      if (ee == hipSuccess) {
        const ispl_status st = batch_launch_eager(b, io, 0, s);
        if (st != ISPL_OK) return st;
      }
      if (ee == hipSuccess) ee = hipEventRecord(e1, s);
      if (ee == hipSuccess) ee = hipEventSynchronize(e1);
      float x = 0.f;
      if (ee == hipSuccess) ee = hipEventElapsedTime(&x, e0, e1);
      if (ee != hipSuccess) return hip_fail(ee, "tune run");
      if (r > 0) t.push_back(x);  // the first run warms up
    }
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return ISPL_OK;
  };
  const ispl_batch_plan saved = b->plan;
  ispl_batch_plan cur = saved;
  float cur_ms = 0.f;
  ispl_status st = measure(cur, &cur_ms);
  // coordinate descent, heaviest mode (most spectra x transform length) first:
  // waves per workgroup (the tile shape: bin classes per workgroup) and pulse
  // chunks of each mode, then branch topology and launch order
  std::vector<int> by_work(b->n_modes);
  for (int m = 0; m < b->n_modes; ++m) by_work[m] = m;
  auto work = [&](int m) {
    const ispl_config& c = b->ctx[m]->cfg;
    return static_cast<double>(c.n_gates) * c.fft_len * (io[m].n_pulses > 0 ? io[m].n_pulses : 1);
  };
  std::sort(by_work.begin(), by_work.end(), [&](int x, int y) { return work(x) > work(y); });
  for (int m : by_work) {
    if (st != ISPL_OK) break;
    const ispl_config& c = b->ctx[m]->cfg;
    const Plan auto_pl = make_plan(c, io[m].n_pulses > 0 ? io[m].n_pulses : 1);
    std::vector<std::pair<int, int>> cands;  // (waves, chunks)
    if (c.code_len <= ispl::SUB)
      for (int w = auto_pl.rw; w >= 1 && w >= auto_pl.rw / 4; w /= 2) cands.push_back({w, 0});
    cands.push_back({0, 1});
    if (auto_pl.chunks > 2) cands.push_back({0, auto_pl.chunks / 2});
    if (2 * auto_pl.chunks <= b->ctx[m]->chunks_max) cands.push_back({0, 2 * auto_pl.chunks});
    for (const auto& wc : cands) {
      ispl_batch_plan p = cur;
      p.waves[m] = wc.first == auto_pl.rw ? 0 : wc.first;
      p.chunks[m] = wc.second;
      if (p.waves[m] == cur.waves[m] && p.chunks[m] == cur.chunks[m]) continue;
      float ms = 0.f;
      st = measure(p, &ms);
      if (st != ISPL_OK) break;
      if (ms < cur_ms) {
        cur = p;
        cur_ms = ms;
      }
    }
  }
  if (st == ISPL_OK) {
    ispl_batch_plan p = cur;
    p.serial = 1 - cur.serial;
    float ms = 0.f;
    st = measure(p, &ms);
    if (st == ISPL_OK && ms < cur_ms) {
      cur = p;
      cur_ms = ms;
    }
  }
  if (st == ISPL_OK && cur.serial) {  // heaviest first, and the given order
    ispl_batch_plan p = cur;
    for (int k = 0; k < b->n_modes; ++k) p.order[k] = by_work[k];
    float ms = 0.f;
    st = measure(p, &ms);
    if (st == ISPL_OK && ms < cur_ms) {
      cur = p;
      cur_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->plan = st == ISPL_OK ? cur : saved;
  apply_plan(b);
  b->graph_valid = false;
  if (st != ISPL_OK) return st;
  if (best) *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return ok();
}

}  // extern "C"
