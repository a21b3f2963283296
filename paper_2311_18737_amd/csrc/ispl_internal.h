// Internal interface between the C-ABI layer (ispl_api.cpp) and the device
// code (ispl_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "ispl.h"

namespace ispl {

// Sets the calling thread's ispl_last_error() text (cleared for ISPL_OK) and
// returns s.
ispl_status report(ispl_status s, const char* msg);

// Points one wave transforms.  A decoded row of L samples is zero-padded to
// N = R * M and split into R interleaved sub-spectra of M points each, with
// M = SUB (L <= 1024, one wave per sub-transform) or M = 16 SUB
// (1024 < L <= 16384, sixteen waves per sub-transform).
constexpr int SUB = 1024;
constexpr int MAX_WAVES_PER_BLOCK = 16;

#if defined(__HIP__)
#define ISPL_HOST_DEVICE __host__ __device__
#else
#define ISPL_HOST_DEVICE
#endif

// Pulse chunks of a gate-list launch whose list length k is only known on the
// device: as many chunks as keep k x zgroups x chunks workgroups within one
// round of the chip (`target` workgroup slots), at most max_chunks and at most
// rows / k (partial rows available), at least one.  The host sizes the grid
// and the partial buffer with the same rule, the kernels and the partial
// reduction derive the chunk count from the device-side k.
ISPL_HOST_DEVICE inline int adaptive_chunks(int k, int zgroups, int target, int max_chunks,
                                            int rows) {
  if (k <= 0) return 1;
  int c = target / (k * zgroups);
  if (c > max_chunks) c = max_chunks;
  if (c > rows / k) c = rows / k;
  return c > 1 ? c : 1;
}

// Geometry and plan of one fused launch.
struct FusedArgs {
  const void* samples;     // [P][stride] ci16 or c64
  const float* tx;         // complex64 pairs, [P][L] or [L]
  const float* twiddle;    // complex64 pairs, W_N^i for i < N
  float* out;              // S [G][N] when chunks == 1, else partials [C][G][N]
  int64_t stride;          // samples per echo row
  int32_t n_fft;           // N
  int32_t sub_len;         // M: SUB or 16 * SUB
  int32_t log2_r;          // log2(N / M)
  int32_t code_len;        // L
  int32_t n_gates;         // G
  int32_t gate_step;       // s
  int32_t first_gate;      // g0
  int32_t n_pulses;        // P
  int32_t chunks;          // C
  int32_t tx_per_pulse;    // 0 / 1
  int32_t accumulate;      // only read when chunks == 1
  int32_t sample_type;     // 0 c64, 1 ci16
  int32_t waves_per_block; // RW in {1, 2, 4, 8, 16} (16 when M = 16 SUB)
  const int32_t* gate_list;  // optional: work on gate_list[i], i < *gate_count, only
  const int32_t* gate_count; // device int32, read by the kernels
  // Adaptive chunking (gate lists only; adapt_target 0 = off): the chunk count
  // is adaptive_chunks(*gate_count, R / RW, adapt_target, adapt_max_chunks,
  // adapt_rows) and `chunks` is not read.  With one chunk `out` receives the
  // rows as usual; with more, chunk c of list slot i goes to row c * k + i of
  // adapt_partial ([adapt_rows][N]).
  float* adapt_partial;
  int32_t adapt_target;
  int32_t adapt_max_chunks;
  int32_t adapt_rows;
  // Optional (long codes, L > 2 SUB): codes as sign bits, written by
  // launch_pack_code_bits for the same tx; NULL = always read tx.
  const uint16_t* code_bits;     // [rows][SUB]: bit j of word lg is code[lg + SUB j] == -1
  const int32_t* code_binary;    // [rows]: 1 when every code of the row is +-1 + 0i
};

// Words of one code row in the sign-bit form (one per first-pass thread).
constexpr int CODE_BITS_WORDS = SUB;

// Sign bits of binary (+-1 + 0i) codes, for the long-code kernel: for each of
// `rows` code rows of length L <= 16 SUB, word lg of bits[row] has bit j set
// when code[row][lg + SUB j] == -1 (positions past L read as +1), and
// binary[row] = 1 when every code of the row is exactly +-1 with a zero
// imaginary part (0 otherwise: the row is then read as complex codes).
hipError_t launch_pack_code_bits(const float* tx, int32_t rows, int32_t code_len,
                                 uint16_t* bits, int32_t* binary, hipStream_t stream);

constexpr int MAX_BATCH_MODES = 8;

// Static LDS bytes of one fused workgroup with `rw` waves and sub-transform M.
int fused_lds_bytes(int rw, int sub_len);

hipError_t launch_fused(const FusedArgs& a, hipStream_t stream);

// S[g][k] = (accumulate ? S[g][k] : 0) + sum_{c < C} partial[c][g][k], c ascending.
// spectra (+)= sum over chunks of partial; with a list, only the rows of the
// listed gates (list[i], i < *count) are touched.
hipError_t launch_reduce_chunks(const float* partial, float* spectra, int64_t elems,
                                int32_t chunks, int32_t accumulate, int32_t n_fft,
                                const int32_t* list, const int32_t* count, hipStream_t stream);

// Static scratch of ispl_integrate_spectra_noalloc: twiddle table first, the
// chunk partials after it.
constexpr size_t NOALLOC_TWIDDLE_BYTES = size_t{512} << 10;  // N <= 65536 complex64
constexpr size_t NOALLOC_PARTIAL_BYTES = ISPL_NOALLOC_SCRATCH_BYTES - NOALLOC_TWIDDLE_BYTES;
// This GPU's copy of the array (`device` must be current); looked up once per
// device.
hipError_t noalloc_scratch(int device, unsigned char** base);
// W_N^i, i < n_fft, into `table` (complex64 pairs), as the context builds it.
hipError_t launch_build_twiddles(float* table, int32_t n_fft, hipStream_t stream);

hipError_t launch_fill_zero(float* dst, int64_t elems, hipStream_t stream);
hipError_t launch_fill_zero_rows(float* dst, int32_t n_gates, int32_t n_fft, const int32_t* list,
                                 const int32_t* count, hipStream_t stream);

// Zoom DFT of a K-bin window per gate on the matrix cores.
struct ZoomArgs {
  const void* samples;      // [P][stride] ci16 or c64
  const float* tx;          // complex64 pairs, [P][L] or [L]
  const float* twiddle;     // complex64 pairs, W_N^i for i < N
  const void* a_hi;         // DFT-matrix table, high halves, MFMA A-operand order
  const void* a_lo;         // low halves
  const int32_t* bin_start; // [G] first bin of each gate's window (taken mod N)
  float* out;               // [G][K]
  float* partial;           // [chunks][G][K] when chunks > 1
  int32_t* col_exp;         // [P] per-pulse FP16 exponents (written by the launch)
  int64_t stride;
  int64_t row_lo, row_hi;   // samples of a pulse row that some gate reads
  int32_t n_fft;            // N
  int32_t code_len;         // L
  int32_t code_pad;         // L rounded up to 64
  int32_t n_gates;
  int32_t gate_step;
  int32_t first_gate;
  int32_t n_pulses;
  int32_t n_bins;           // K, a multiple of 128 RT
  int32_t tx_per_pulse;
  int32_t accumulate;       // read when chunks == 1
  int32_t sample_type;
  int32_t precision;        // 0: BF16 x3, 1: FP16 x3
  int32_t chunks;           // pulse chunks (workgroups per gate and bin tile)
  int32_t row_tiles;        // RT: 1 or 2 (128 or 256 bins per workgroup)
  int32_t col_tiles;        // CT: 1 or 2 (32 or 64 pulses per block)
  const int32_t* gate_list; // optional: only gates gate_list[i], i < *gate_count
  const int32_t* gate_count;
  // Optional sign bits of +-1 codes (NULL: always read tx as complex codes),
  // written by the launch's pulse pass (launch_zoom with prep) or by
  // launch_select_and_exponents: [rows][code_pad / 32] words, bit b of word w
  // set when code[32 w + b] == -1, and per row 1 when the whole row is +-1.
  uint32_t* code_bits;
  int32_t* code_binary;
};

// With prep = false the FP16 column exponents (FP16) and the code sign bits
// (a.code_bits) must already be written (launch_select_and_exponents does).
hipError_t launch_zoom(const ZoomArgs& a, hipStream_t stream, bool prep = true);

// Window-proposal network (learned zoom).
constexpr int NET_LEN = 1024;      // coarse bins per gate
constexpr int NET_PARAMS = 14881;  // 4 circular 7-tap conv layers, 1-32-32-32-1 channels

struct NetWork {  // device buffers of a training batch (FP32)
  float* params;  // [NET_PARAMS]
  float* a1;      // [B][32][T] activations after layers 1..3
  float* a2;
  float* a3;
  float* logits;  // [B][T]
  float* dz4;     // [B][T]
  float* dzA;     // [B][32][T] gradient ping-pong
  float* dzB;
  float* part;    // [B][NET_PARAMS] per-gate weight gradients
  float* loss;    // [B]
};

hipError_t launch_net_features(const float* spectra, int rows, float* out, hipStream_t s);
hipError_t launch_net_forward_f32(const NetWork& w, const float* x, int batch, float* logits,
                                  hipStream_t s);
hipError_t launch_net_loss_grad(const NetWork& w, const float* x, const float* target_pos,
                                int batch, float* grad, float* loss_mean, hipStream_t s);
size_t net_bf16_bytes();  // matrix-core weight table of the BF16 forward
hipError_t launch_net_prep_bf16(const float* params, void* table, hipStream_t s);
// logits of features x (or, with from_spectra, of coarse spectra x whose
// features the kernel forms itself; with chunks > 1 those spectra are first
// summed from [chunks][batch][1024] partials and written to x_out)
hipError_t launch_net_forward_bf16(const void* table, const float* x, int batch, float* logits,
                                   hipStream_t s, bool from_spectra = false,
                                   const float* partial = nullptr, int32_t chunks = 1,
                                   float* x_out = nullptr);
hipError_t launch_adam(float* params, const float* grad, float* m, float* v, int n, float lr,
                       int step, hipStream_t s);

hipError_t launch_peak(const float* spectra, int32_t n_gates, int32_t n_fft, int32_t bin_lo,
                       int32_t bin_hi, int32_t* peak_bin, float* peak_power,
                       const int32_t* list, const int32_t* count, hipStream_t stream);

// Learned-zoom decision kernels.
hipError_t launch_select_windows(const float* logits, int32_t n_gates, int32_t fine_len,
                                 int32_t window_bins, float threshold, int32_t* bin_start,
                                 float* confidence, int32_t* flag, int32_t* zoom_list,
                                 int32_t* fallback_list, int32_t* counts, int32_t* done,
                                 hipStream_t s);
// Peak per gate over its window (zoomed) or its full row (fallback); with
// zoom_chunks or fine_chunks > 1 the rows are first summed from the chunk
// partials ([C][G][len], ascending c) and written to window_spectra /
// full_spectra.
// Adaptive chunking of the fallback launch (see FusedArgs): the fallback
// list length counts[1], the slot of each fallback gate in that list, and the
// rule's parameters.
struct FallbackChunks {
  const int32_t* counts;  // [2]: zoomed, fallback
  const float* partial;   // [rows][N]
  int32_t zgroups, target, max_chunks, rows;
};
hipError_t launch_split_peaks(float* window_spectra, const float* window_partial,
                              int32_t zoom_chunks, float* full_spectra, const FallbackChunks& fb,
                              const int32_t* zoom_list, const int32_t* fallback_list,
                              const int32_t* bin_start, int32_t n_gates, int32_t window_bins,
                              int32_t fine_len, int32_t* peak_bin, float* peak_power,
                              hipStream_t s);
// Per-pulse FP16 exponents of the zoom DFT (pulses 0 .. n_pulses - 1).
struct PulseExpArgs {
  const void* samples;
  const float* tx;
  int32_t* exps;           // NULL: no exponents (BF16 zoom)
  uint32_t* bits;          // NULL: no code sign bits
  int32_t* binary;
  int64_t stride, lo, hi;  // rows and the span [lo, hi) some gate reads
  int32_t sample_type, code_len, tx_per_pulse, n_pulses, bit_words;
};
// select_windows and, in the same launch, the zoom's per-pulse pass: FP16
// exponents and code sign bits (n_pulses = 0: none).
hipError_t launch_select_and_exponents(const float* logits, int32_t n_gates, int32_t fine_len,
                                       int32_t window_bins, float threshold, int32_t* bin_start,
                                       float* confidence, int32_t* flag, int32_t* zoom_list,
                                       int32_t* fallback_list, int32_t* counts, int32_t* done,
                                       const PulseExpArgs& pe, hipStream_t s);
hipError_t launch_window_peak(const float* spectra, int32_t n_gates, int32_t window_bins,
                              int32_t fine_len, const int32_t* bin_start, const int32_t* list,
                              const int32_t* count, int32_t* peak_bin, float* peak_power,
                              hipStream_t s);

}  // namespace ispl
