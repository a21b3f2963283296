/*
 * ispl.h - C ABI of the incoherent-scatter plasma-line spectrum library
 * (MI355X / gfx950).
 *
 * The library computes, for a batch of transmitted pulses and a set of radar
 * range gates, the incoherently integrated power spectrum
 *
 *   S[g][k] = sum_{p < P} | sum_{n < L} conj(c_p[n]) * x_p[g0 + g*s + n]
 *                                      * exp(-2 pi i k n / N) |^2
 *
 * i.e. the conjugated transmit code is multiplied into one range gate of the
 * echo, the product is Fourier transformed, squared in modulus and added over
 * pulses (Hilliard, Vierinen & Erickson, "GPGPU Acceleration of Incoherent
 * Scatter Radar Plasma Line Analysis", Section 2.2, Eqs. 7-8 and the
 * processing recipe after them; Section 3.2 for the decode, transform and
 * accumulate steps).  It then finds the plasma line of every gate as the peak
 * of S over a frequency band.
 *
 * Conventions for every call:
 *   - All array pointers are DEVICE pointers (hipMalloc or torch tensors) and
 *     stay owned by the caller; they must stay valid until the work queued on
 *     `stream` has completed.  Pointers must be aligned to their element size
 *     (4 bytes for ci16 samples and float/int32 outputs, 8 bytes for complex64).
 *   - Work is queued asynchronously on `stream` (a hipStream_t; NULL = the
 *     null stream).  The caller synchronises.
 *   - Every argument is validated before anything is queued.  On any error
 *     nothing is launched and no output is written; the call returns a
 *     non-zero ispl_status and ispl_last_error() describes the problem.
 *   - Nothing throws or aborts across this ABI.
 *   - A context is not thread-safe: one thread at a time per context.  A
 *     context and the objects built on it (zoom, learned zoom) own scratch
 *     (pulse-chunk partials, FP16 exponents, code sign bits) that every call
 *     reuses, so calls on one context or object must not overlap on
 *     different streams either.
 *   - Results are bit-identical from run to run for the same context,
 *     arguments and device (no atomics, fixed reduction order).
 */
#ifndef ISPL_H
#define ISPL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ISPL_ABI_VERSION 1

typedef struct ispl_ctx ispl_ctx; /* opaque, owned by the library */

typedef enum {
  ISPL_OK = 0,
  ISPL_ERR_INVALID_ARG = 1,  /* bad pointer, size or layout */
  ISPL_ERR_UNSUPPORTED = 2,  /* valid, but outside what this library implements */
  ISPL_ERR_OUT_OF_MEMORY = 3,
  ISPL_ERR_DEVICE = 4        /* no usable gfx950 device, or a HIP runtime error */
} ispl_status;

typedef enum {
  ISPL_SAMPLES_C64 = 0,  /* complex64: float re, float im per sample */
  ISPL_SAMPLES_CI16 = 1  /* complex int16: int16 re, int16 im per sample (raw ADC) */
} ispl_sample_type;

/*
 * Fixed geometry of one experiment (Section 4 describes the paper's: 16384-
 * sample codes, 250,000-sample echo rows, 4096 gates with a step of 25 starting
 * at the first sample, FFT length 16384).
 */
typedef struct {
  int32_t abi_version;  /* must be ISPL_ABI_VERSION */
  int32_t code_len;     /* L >= 1: transmit code length in samples */
  int32_t fft_len;      /* N: power of two, L <= N.  This library: 1024 <= N <= 65536
                           with L <= 1024, or 16384 <= N <= 65536 with
                           L <= 16384 (other valid shapes: ISPL_ERR_UNSUPPORTED) */
  int32_t n_gates;      /* G >= 1 range gates */
  int32_t gate_step;    /* s >= 1 samples between consecutive gate starts */
  int32_t first_gate;   /* g0 >= 0: echo sample where gate 0 starts */
  int64_t pulse_stride; /* samples from one echo row to the next;
                           must be >= g0 + (G - 1) * s + L */
  int32_t sample_type;  /* ispl_sample_type */
  int32_t max_pulses;   /* >= 1: largest n_pulses a call may pass (sizes scratch) */
  int32_t device;       /* HIP device ordinal */
} ispl_config;

/* Validates `cfg`, selects `cfg->device`, builds the twiddle table and the
 * scratch buffers the plan needs, and returns a new context in *out.
 * Config errors are reported before the device is touched.  Returns
 * ISPL_ERR_DEVICE when the device is missing or is not gfx950. */
ispl_status ispl_create(const ispl_config* cfg, ispl_ctx** out);

/*
 * Integrated spectra of n_pulses pulses (Eqs. 7-8; Section 3.2):
 *   samples   device [n_pulses][pulse_stride] samples of `sample_type`,
 *             interleaved (re, im).  Gate g of pulse p reads samples
 *             p*pulse_stride + g0 + g*s + n, n < L.
 *   tx_code   device complex64 (re, im float pairs): [n_pulses][L] when
 *             tx_per_pulse != 0 (one code per pulse), else [L] shared by all.
 *   spectra   device float [n_gates][fft_len], natural FFT order (bin k is
 *             frequency k*fs/N for k < N/2, (k-N)*fs/N above), unnormalised
 *             forward transform exp(-2 pi i k n / N), |X|^2 summed (not
 *             averaged) over the pulses.
 *   accumulate  0: spectra = sum;  1: spectra += sum (resumable integration).
 *   n_pulses  0 <= n_pulses <= max_pulses.  With 0 pulses the sum is empty:
 *             spectra is zeroed (accumulate = 0) or left as is (accumulate = 1).
 * Arithmetic: decode, transform, power and accumulation in FP32.
 */
ispl_status ispl_integrate_spectra(ispl_ctx* ctx, const void* samples,
                                   const float* tx_code, int32_t tx_per_pulse,
                                   int32_t n_pulses, float* spectra,
                                   int32_t accumulate, void* stream);

/*
 * Plasma-line pick per gate (the line frequency is the quantity the spectra
 * are computed for, Section 2.1): peak_bin[g] = the lowest bin k in the band
 * attaining max_k spectra[g][k]; peak_power[g] = that maximum.
 *   spectra   device float [n_gates][fft_len] (e.g. from ispl_integrate_spectra)
 *   band      bins [bin_lo, bin_hi) in natural order, 0 <= bin_lo < N,
 *             0 < bin_hi <= N, bin_lo != bin_hi; bin_lo > bin_hi wraps through
 *             N, i.e. [bin_lo, N) then [0, bin_hi).  The full band is
 *             bin_lo = 0, bin_hi = N.
 *   peak_bin  device int32 [n_gates]
 *   peak_power device float [n_gates], or NULL when not wanted.
 * Values are compared as FP32; spectra holding NaN give an unspecified bin.
 */
ispl_status ispl_find_plasma_line(ispl_ctx* ctx, const float* spectra,
                                  int32_t bin_lo, int32_t bin_hi,
                                  int32_t* peak_bin, float* peak_power,
                                  void* stream);

/*
 * Gate-list variants: the same computation restricted to the gates
 * gate_list[i], i < *gate_count, where gate_list is a device int32 array of
 * n_gates entries and gate_count a device int32 read by the kernels (so a
 * list built on the device needs no host round trip).  Rows of other gates
 * of spectra / peak_bin / peak_power are left untouched; entries outside
 * [0, n_gates) are skipped; the listed gates must be distinct.  Both
 * pointers are required (ISPL_ERR_INVALID_ARG when NULL).  Used for the
 * full-resolution fallback of the learned zoom.
 */
ispl_status ispl_integrate_spectra_gates(ispl_ctx* ctx, const void* samples,
                                         const float* tx_code, int32_t tx_per_pulse,
                                         int32_t n_pulses, const int32_t* gate_list,
                                         const int32_t* gate_count, float* spectra,
                                         int32_t accumulate, void* stream);
ispl_status ispl_find_plasma_line_gates(ispl_ctx* ctx, const float* spectra, int32_t bin_lo,
                                        int32_t bin_hi, const int32_t* gate_list,
                                        const int32_t* gate_count, int32_t* peak_bin,
                                        float* peak_power, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as ispl_integrate_spectra on a context created from *cfg, with
 * no context and no allocation at all.
 *   cfg       as for ispl_create (validated on every call; max_pulses bounds
 *             n_pulses as it does for a context).
 *   samples, tx_code, tx_per_pulse, n_pulses, spectra, accumulate, stream:
 *             as for ispl_integrate_spectra (caller-owned device buffers).
 * The twiddle table and the pulse-chunk partial spectra live in a static
 * device array of ISPL_NOALLOC_SCRATCH_BYTES bytes (512 KiB of twiddles, 64
 * MiB of partials) that the library holds on every GPU it runs on until the
 * process ends; the table is rebuilt on `stream` by every call (one small
 * launch).  The launch plan is ispl_create's automatic plan, whose partials
 * never exceed 64 MiB (fewer than four workgroup slots of the chip per chunk
 * row); a plan that needed more would be rejected with ISPL_ERR_UNSUPPORTED
 * before anything is queued.  Results equal those of ispl_integrate_spectra
 * (the same plan, the same kernels).  Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents: calls that overlap on one GPU
 * (on different streams, or from different threads) race and give wrong
 * results.  The first call on a device looks up its copy of the array
 * (hipGetSymbolAddress); it never calls hipMalloc or hipFree.
 */
#define ISPL_NOALLOC_SCRATCH_BYTES ((64 << 20) + (512 << 10))

ispl_status ispl_integrate_spectra_noalloc(const ispl_config* cfg, const void* samples,
                                           const float* tx_code, int32_t tx_per_pulse,
                                           int32_t n_pulses, float* spectra, int32_t accumulate,
                                           void* stream);

/*
 * Zoom DFT on the matrix cores: K bins of the N-point spectrum of every gate,
 * starting at a per-gate bin, without the full transform.  Each gate's
 * decoded rows are shifted so that its window starts at bin 0 and multiplied
 * by one K x L DFT matrix shared by all gates and pulses (the complex product
 * as three real products), on BF16 or FP16 MFMA with both operands split into
 * high and low halves (three split products each, FP32 accumulation);
 * decode, shift and the pulse sum stay FP32.  The result is the same
 * quantity as ispl_integrate_spectra at those bins (Section 2.2, Eqs. 7-8),
 * at the precision of the chosen split.
 */
typedef enum {
  ISPL_ZOOM_BF16X3 = 0,  /* BF16 hi/lo split: ~16 significant bits per product */
  ISPL_ZOOM_FP16X3 = 1   /* FP16 hi/lo split with per-pulse power-of-two scaling: ~22 bits */
} ispl_zoom_precision;

typedef struct ispl_zoom ispl_zoom; /* opaque; must not outlive its context */

/* Builds the split DFT-matrix table for windows of n_bins bins (a multiple of
 * 128, at most fft_len) of ctx's geometry: two halves of 6 * n_bins *
 * round_up(code_len, 64) bytes each; ISPL_ERR_UNSUPPORTED above 512 MiB per
 * half.  Also holds the per-call scratch: FP16 exponents and the sign bits of
 * +-1 codes for max_pulses pulses. */
ispl_status ispl_zoom_create(ispl_ctx* ctx, int32_t n_bins, int32_t precision,
                             ispl_zoom** out);

/*
 * spectra[g][j] (+)= sum_p | sum_{n<L} conj(c_p[n]) x_p[g0+g*s+n]
 *                             * exp(-2 pi i (bin_start[g] + j) n / N) |^2,  j < n_bins.
 *   samples, tx_code, tx_per_pulse, n_pulses, accumulate: as ispl_integrate_spectra.
 *   bin_start  device int32 [n_gates]; any integer, taken modulo N.
 *   spectra    device float [n_gates][n_bins].
 */
ispl_status ispl_zoom_spectra(ispl_zoom* zoom, const void* samples, const float* tx_code,
                              int32_t tx_per_pulse, int32_t n_pulses,
                              const int32_t* bin_start, float* spectra, int32_t accumulate,
                              void* stream);

/* ispl_zoom_spectra for the listed gates only (gate lists as for
 * ispl_integrate_spectra_gates). */
ispl_status ispl_zoom_spectra_gates(ispl_zoom* zoom, const void* samples, const float* tx_code,
                                    int32_t tx_per_pulse, int32_t n_pulses,
                                    const int32_t* bin_start, const int32_t* gate_list,
                                    const int32_t* gate_count, float* spectra,
                                    int32_t accumulate, void* stream);

/* Peak of each listed gate's window (Section 3.2's peak search on the zoomed
 * bins): peak_bin[g] = (bin_start[g] + j) mod N for the lowest j attaining
 * max_j spectra[g][j]; peak_power[g] = that maximum (NULL: not wanted).
 * spectra device float [n_gates][n_bins]; other gates untouched. */
ispl_status ispl_zoom_find_peaks(ispl_zoom* zoom, const float* spectra, const int32_t* bin_start,
                                 const int32_t* gate_list, const int32_t* gate_count,
                                 int32_t* peak_bin, float* peak_power, void* stream);

void ispl_zoom_destroy(ispl_zoom* zoom);

/*
 * Window-proposal network of the learned zoom.  It reads one integrated
 * coarse spectrum per gate (ISPL_NET_LEN = 1024 bins) as the feature
 * x[t] = log(max(S[t] / mean S, 1e-30)) and returns one logit per coarse bin:
 * four circular 7-tap 1-D convolutions, 1 -> 32 -> 32 -> 32 -> 1 channels,
 * ReLU after the first three.  Training minimises the softmax cross entropy
 * against a two-hot target at the line's coarse position u (1 - frac(u) on
 * floor(u), frac(u) on floor(u) + 1, modulo 1024) with Adam (beta 0.9,
 * 0.999, eps 1e-8) on FP32 master weights; training kernels run in FP32.
 * Parameters (ISPL_NET_PARAMS floats): W1[32][1][7] b1[32] W2[32][32][7]
 * b2[32] W3[32][32][7] b3[32] W4[1][32][7] b4[1].  Not thread-safe; runs
 * on the device it was created on.
 */
#define ISPL_NET_LEN 1024
#define ISPL_NET_PARAMS 14881

typedef struct ispl_net ispl_net;

typedef enum {
  ISPL_NET_FP32 = 0,  /* vector-ALU forward, FP32 weights and activations */
  ISPL_NET_BF16 = 1   /* matrix-core forward, BF16 weights and activations, FP32 accumulation */
} ispl_net_precision;

/* Allocates parameters (zero), Adam state and the workspace of batches of up
 * to max_batch gates on `device`. */
ispl_status ispl_net_create(int32_t device, int32_t max_batch, ispl_net** out);
void ispl_net_destroy(ispl_net* net);
/* Host float arrays of ISPL_NET_PARAMS values; set_params also resets Adam. */
ispl_status ispl_net_set_params(ispl_net* net, const float* host_params);
ispl_status ispl_net_get_params(ispl_net* net, float* host_params);
/* features[r][t] from spectra[r][t], device [rows][ISPL_NET_LEN] each. */
ispl_status ispl_net_features(ispl_net* net, const float* spectra, int32_t rows,
                              float* features, void* stream);
/* logits[b][t] of features[b][t], device [batch][ISPL_NET_LEN] (16-byte aligned);
 * precision ISPL_NET_FP32 needs batch <= max_batch (its activations use the
 * workspace), ISPL_NET_BF16 takes any batch >= 0. */
ispl_status ispl_net_forward(ispl_net* net, const float* features, int32_t batch,
                             float* logits, int32_t precision, void* stream);
/* Mean loss (device float [1]) and its gradient (device float [ISPL_NET_PARAMS])
 * over a batch; target_pos device float [batch] in coarse-bin units. */
ispl_status ispl_net_loss_grad(ispl_net* net, const float* features, const float* target_pos,
                               int32_t batch, float* grad, float* loss, void* stream);
/* loss_grad, then one Adam step of learning rate lr. */
ispl_status ispl_net_train_step(ispl_net* net, const float* features, const float* target_pos,
                                int32_t batch, float lr, float* loss, void* stream);

/*
 * Window decision of the learned zoom, from logits [n_gates][ISPL_NET_LEN]
 * (device, 16-byte aligned).  With T = 1024 coarse bins, S = fine_len / T:
 *   p = softmax(logits), m = lowest index of the largest logit,
 *   u = m + sum_d d p[m+d] / sum_d p[m+d], d = -2..2 (indices mod T),
 *   c = S u, bin_start[g] = (floor(c + 1/2) - window_bins / 2) mod fine_len,
 *   confidence[g] = sum of p[t] over the t whose fine position S t lies
 *                   within window_bins / 2 - S of c (circular distance),
 *   flag[g] = confidence >= threshold.
 * zoom_list / fallback_list (device int32 [n_gates]) receive the flagged and
 * the other gates in increasing order, counts[0] / counts[1] (device int32
 * [2]) their numbers.  confidence may be NULL.  fine_len: a power of two
 * >= 1024; 2 S < window_bins <= fine_len; 0 < threshold <= 1.  This rule is
 * the project's (the paper computes every gate at full resolution); all
 * arithmetic is FP32.  Decision and compaction run in one launch whose last
 * workgroup compacts, using a completion counter owned by `net`: calls on one
 * net must not overlap on different streams.
 */
ispl_status ispl_net_select(ispl_net* net, const float* logits, int32_t n_gates,
                            int32_t fine_len, int32_t window_bins, float threshold,
                            int32_t* bin_start, float* confidence, int32_t* flag,
                            int32_t* zoom_list, int32_t* fallback_list, int32_t* counts,
                            void* stream);

/*
 * Learned zoom: peak frequency of every gate without the full-resolution
 * spectrum of every gate.  One call runs, on `stream`, what these calls
 * compute one after another (in six launches):
 *   1. ispl_integrate_spectra at N_c = 1024 (the coarse spectra; its pulses
 *      are split into chunks of at least 4, so the coarse sums may differ
 *      from a context's own in rounding);
 *   2. the network's features and BF16 logits;
 *   3. ispl_net_select with (cfg->fft_len, window_bins, threshold);
 *   4. ispl_zoom_spectra_gates over the zoomed gates (window_bins bins from
 *      bin_start, zoom_precision) and ispl_integrate_spectra_gates at
 *      cfg->fft_len over the fallback gates -- the latter with its pulses
 *      split into as many chunks as the number k of fallback gates leaves
 *      room for (k x chunks workgroups fill the chip once; at most 64 chunks
 *      of at least 8 pulses), chosen on the device from k, so that a few
 *      fallback gates cost a small part of a full integration;
 *   5. ispl_zoom_find_peaks and ispl_find_plasma_line_gates (full band).
 * Given the coarse spectra of step 1, steps 2, 3 and the zoomed gates' part
 * of steps 4-5 equal those calls bit for bit; the fallback rows equal
 * ispl_integrate_spectra_gates' up to the order of the pulse sum.
 * peak_bin[g] / peak_power[g] (device int32 / float [n_gates]; peak_power
 * may be NULL) then hold every gate's line bin at N = cfg->fft_len.
 * ispl_lzoom_create: cfg as for ispl_create with code_len <= 1024 and
 * fft_len >= 1024; window_bins a multiple of 128 with 2 fft_len / 1024 <
 * window_bins <= fft_len; zoom_precision an ispl_zoom_precision; threshold
 * in (0, 1].  `net` stays owned by the caller, must outlive the object and
 * be on cfg->device; its current parameters are used at every call.  The
 * object owns two contexts, a zoom table, [n_gates] x (2 * 1024 +
 * window_bins + fft_len) floats of buffers and up to 16 MiB of fallback
 * chunk partials.  Not thread-safe, and calls on
 * one object must not overlap on different streams (it owns the scratch and
 * the decision's completion counter).  Capturable in a HIP graph (it neither
 * allocates nor synchronises).
 */
typedef struct ispl_lzoom ispl_lzoom;

ispl_status ispl_lzoom_create(const ispl_config* cfg, ispl_net* net, int32_t window_bins,
                              int32_t zoom_precision, float threshold, ispl_lzoom** out);
void ispl_lzoom_destroy(ispl_lzoom* lzoom);
ispl_status ispl_lzoom_peaks(ispl_lzoom* lzoom, const void* samples, const float* tx_code,
                             int32_t tx_per_pulse, int32_t n_pulses, int32_t* peak_bin,
                             float* peak_power, void* stream);

/* Device pointers to the intermediate results of the last ispl_lzoom_peaks
 * (owned by the object, valid until it is destroyed; read after the stream
 * has completed): for diagnostics, tests and accounting of the split. */
typedef struct {
  int32_t n_gates, window_bins, fine_len;
  const float* coarse_spectra;   /* [n_gates][1024] */
  const float* logits;           /* [n_gates][1024] */
  const int32_t* bin_start;      /* [n_gates] */
  const float* confidence;       /* [n_gates] */
  const int32_t* zoom_list;      /* [n_gates], first counts[0] entries valid */
  const int32_t* fallback_list;  /* [n_gates], first counts[1] entries valid */
  const int32_t* counts;         /* [2] */
  const float* window_spectra;   /* [n_gates][window_bins], zoomed gates' rows */
  const float* full_spectra;     /* [n_gates][fine_len], fallback gates' rows */
} ispl_lzoom_buffers;

ispl_status ispl_lzoom_view(const ispl_lzoom* lzoom, ispl_lzoom_buffers* out);

/* Frees the context and its device memory (synchronises its device first).
 * NULL is a no-op. */
void ispl_destroy(ispl_ctx* ctx);

/*
 * Uneven batch: several experiments ("modes": different code lengths, FFT
 * lengths and gate counts on one device) integrated by ONE launch of a HIP
 * graph whose branches run the modes side by side (or one after another),
 * so light and heavy modes share the chip without host launches between them.
 * Each mode computes exactly what ispl_integrate_spectra computes for it; the
 * plan of each mode (waves per workgroup, pulse chunks) and the graph's shape
 * come from the automatic plan, a hand-set plan or the project's autotuner.
 *   ispl_batch_create   1 <= n_modes <= 8 configs (as for ispl_create).
 *   ispl_batch_io       per mode: samples, tx_code, tx_per_pulse, n_pulses,
 *                       spectra, with the meanings of ispl_integrate_spectra.
 *   ispl_batch_integrate  io[n_modes]; accumulate 0/1 for every mode;
 *                       use_graph = 1 launches the object's graph (captured
 *                       on first use and again when io, accumulate or the plan
 *                       change); use_graph = 0 queues the modes' launches on
 *                       `stream` one after another (a caller may capture that).
 *                       A replaced graph is kept until the device has been
 *                       synchronised (a launch of it may still be running):
 *                       every eighth re-capture synchronises the device once
 *                       and frees the replaced graphs.
 *   ispl_batch_tune     the autotuner: coordinate descent over each mode's
 *                       waves per workgroup (bin classes a workgroup computes:
 *                       the tile shape) and pulse chunks, heaviest mode first,
 *                       then parallel vs serial branches and the order; each
 *                       candidate is the median time over `trials` runs of
 *                       its launches, queued in the plan's branch shape on the
 *                       object's own streams (the graph of the chosen plan is
 *                       captured by the next ispl_batch_integrate).  Keeps and
 *                       returns the fastest plan and its time (either pointer
 *                       may be NULL).  It writes the spectra of io and blocks
 *                       until its runs are done.
 *   ispl_batch_get_plan / set_plan  the plan in use (waves 0 and chunks 0 mean
 *                       the automatic choice; waves only for modes with
 *                       L <= 1024: a power of two <= min(16, N/1024)).
 * Waves per workgroup change no result between shapes that share a twiddle
 * factorization (eight-wave workgroups use a geometric form of the inner
 * passes' twiddles, every other shape the direct form) and only the rounding
 * across the two; pulse chunks change the summation order (results within
 * rounding).  The object owns one context per
 * mode and its streams; calls on one object must not overlap.
 */
typedef struct ispl_batch ispl_batch;

typedef struct {
  const void* samples;
  const float* tx_code;
  int32_t tx_per_pulse;
  int32_t n_pulses;
  float* spectra;
} ispl_batch_io;

typedef struct {
  int32_t order[8];   /* launch order of the modes (their order on serial branches) */
  int32_t waves[8];   /* per mode: waves per workgroup, 0 = automatic */
  int32_t chunks[8];  /* per mode: pulse chunks, 0 = automatic */
  int32_t serial;     /* 0: one parallel branch per mode; 1: one branch in `order` */
} ispl_batch_plan;

ispl_status ispl_batch_create(const ispl_config* cfgs, int32_t n_modes, ispl_batch** out);
void ispl_batch_destroy(ispl_batch* batch);
ispl_status ispl_batch_integrate(ispl_batch* batch, const ispl_batch_io* io,
                                 int32_t accumulate, int32_t use_graph, void* stream);
ispl_status ispl_batch_tune(ispl_batch* batch, const ispl_batch_io* io, int32_t trials,
                            ispl_batch_plan* best, float* best_ms);
ispl_status ispl_batch_get_plan(const ispl_batch* batch, ispl_batch_plan* plan);
ispl_status ispl_batch_set_plan(ispl_batch* batch, const ispl_batch_plan* plan);

/*
 * Streaming ingest (the paper's timing scope, Section 4: host rows copied to
 * the device and integrated, against one echo every 10 ms).  A ring of
 * n_slots pinned host slots, each holding up to slot_pulses pulse rows
 * ([slot_pulses][pulse_stride] samples of cfg's sample_type) and their codes
 * ([slot_pulses][code_len] complex64, or one row when shared).  For each
 * submitted slot only the samples the gates read (rows [first_gate,
 * first_gate + (n_gates-1)*gate_step + code_len)) and the codes go to the
 * device, on the object's own copy stream; the integration is queued on
 * `stream` after that copy and equals ispl_integrate_spectra of the same
 * pulses (so a run of submits with accumulate = 1 after the first equals
 * calling ispl_integrate_spectra batch by batch).  The copy of one slot
 * overlaps the integration of the previous one.
 *   ispl_stream_create   cfg as for ispl_create; 1 <= slot_pulses <= max_pulses;
 *                        2 <= n_slots <= 64.  Allocates the pinned slots, the
 *                        device buffers and a context of its own.
 *   ispl_stream_slot_samples / _codes  pinned host pointers of slot i (NULL for
 *                        a bad slot); owned by the object.
 *   ispl_stream_wait_slot  blocks until the slot's last copy has finished:
 *                        call it before writing into a slot that was submitted.
 *   ispl_stream_submit   0 <= n_pulses <= slot_pulses; spectra device
 *                        [n_gates][fft_len] as for ispl_integrate_spectra.
 *   ispl_stream_sync     blocks until every queued copy and integration of
 *                        the object has finished.
 * Not thread-safe; one producer thread.
 */
typedef struct ispl_stream ispl_stream;

ispl_status ispl_stream_create(const ispl_config* cfg, int32_t slot_pulses, int32_t n_slots,
                               ispl_stream** out);
void ispl_stream_destroy(ispl_stream* st);
void* ispl_stream_slot_samples(ispl_stream* st, int32_t slot);
float* ispl_stream_slot_codes(ispl_stream* st, int32_t slot);
ispl_status ispl_stream_wait_slot(ispl_stream* st, int32_t slot);
ispl_status ispl_stream_submit(ispl_stream* st, int32_t slot, int32_t n_pulses,
                               int32_t tx_per_pulse, float* spectra, int32_t accumulate,
                               void* stream);
ispl_status ispl_stream_sync(ispl_stream* st);

/* Launch plan the library would use for n_pulses pulses with this config;
 * host-only (no device call), for tests and tooling.  Fills, when non-NULL:
 * chunks = number of pulse chunks integrated side by side (1 = no partial
 * buffers), waves_per_block, blocks = workgroups of the fused launch. */
ispl_status ispl_plan(const ispl_config* cfg, int32_t n_pulses, int32_t* chunks,
                      int32_t* waves_per_block, int32_t* blocks);

/* Static string for a status code. */
const char* ispl_status_string(ispl_status s);

/* Detail of the last error on the calling thread ("" if none). */
const char* ispl_last_error(void);

/* ABI version the library was built with (ISPL_ABI_VERSION). */
int32_t ispl_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ISPL_H */
