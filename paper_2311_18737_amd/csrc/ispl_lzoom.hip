// Learned zoom: the decision and bookkeeping kernels between the network and
// the two spectrum paths.
//
// For every gate the network's logits over the T = 1024 coarse bins give a
// window of K fine bins (N = S T point spectrum) and a confidence:
//   p = softmax(logits), m = lowest index of the largest logit,
//   u = m + sum_d d p[m+d] / sum_d p[m+d] over d = -2..2 (indices mod T),
//   c = S u (fine bins), start = (floor(c + 1/2) - K/2) mod N,
//   confidence = sum of p[t] over the coarse bins whose fine position S t
//                lies within K/2 - S of c (circular distance mod N).
// Gates with confidence >= threshold take the zoom DFT over their window; the
// others fall back to the full-resolution spectrum.  Two ordered gate lists
// (zoomed, fallback) and their counts stay on the device, so the following
// launches need no host round trip.  Decision and compaction share one launch
// (the last workgroup to finish compacts).  The peak search of Section 3.2 then runs
// over each gate's window or full row.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ispl_device.h"
#include "ispl_internal.h"

namespace ispl {
namespace {

constexpr int T = NET_LEN;
constexpr int NT = 256;
static_assert(T == 4 * NT, "four coarse bins per thread");

__device__ __forceinline__ bool better(float v, int k, float bv, int bk) {
  return v > bv || (v == bv && k < bk);
}

// (value, index) maximum over the workgroup, lowest index on ties; every
// thread returns the result.
__device__ void block_argmax(float& v, int& k, float* sv, int* sk) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float ov = __shfl_xor(v, off);
    const int ok = __shfl_xor(k, off);
    if (better(ov, ok, v, k)) {
      v = ov;
      k = ok;
    }
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sv[threadIdx.x >> 6] = v;
    sk[threadIdx.x >> 6] = k;
  }
  __syncthreads();
  v = sv[0];
  k = sk[0];
  for (int i = 1; i < NT / 64; ++i)
    if (better(sv[i], sk[i], v, k)) {
      v = sv[i];
      k = sk[i];
    }
}

__device__ float block_sum(float x, float* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Ordered compaction of the flags into the zoomed and fallback gate lists by
// one workgroup of NT threads sweeping the gates in order.
__device__ void compact_gates(const int32_t* flag, int32_t n_gates, int32_t* zoom_list,
                              int32_t* fallback_list, int32_t* counts, int* wtot) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int done_zoom = 0;  // zoomed gates before this sweep step (uniform)
  for (int b0 = 0; b0 < n_gates; b0 += NT) {
    const int g = b0 + tid;
    const bool live = g < n_gates;
    const bool z = live && flag[g] != 0;
    const uint64_t mask = __ballot(z);
    const int below = __popcll(mask & ((uint64_t{1} << lane) - 1));
    __syncthreads();
    if (lane == 0) wtot[wave] = __popcll(mask);
    __syncthreads();
    int before = 0, all = 0;
    for (int w = 0; w < NT / 64; ++w) {
      before += w < wave ? wtot[w] : 0;
      all += wtot[w];
    }
    const int zi = done_zoom + before + below;  // zoomed gates before g
    if (z)
      zoom_list[zi] = g;
    else if (live)
      fallback_list[g - zi] = g;
    done_zoom += all;
  }
  if (tid == 0) {
    counts[0] = done_zoom;
    counts[1] = n_gates - done_zoom;
  }
}

// One workgroup per gate decides its window; the workgroup that finishes
// last (a device-scope counter over the n_gates deciding workgroups, reset by
// that workgroup for the next call) compacts the lists, so decision and lists
// take one launch.
__device__ __forceinline__ void select_window_block(
    int g, const float* __restrict__ logits, int32_t n_gates, int32_t fine_len,
    int32_t window_bins, float threshold, int32_t* __restrict__ bin_start,
    float* __restrict__ confidence, int32_t* __restrict__ flag, int32_t* __restrict__ zoom_list,
    int32_t* __restrict__ fallback_list, int32_t* __restrict__ counts,
    int32_t* __restrict__ done) {
  __shared__ int is_last;
  __shared__ int wtot[NT / 64];
  __shared__ float sv[NT / 64];
  __shared__ int sk[NT / 64];
  __shared__ float red[NT / 64];
  const int j = threadIdx.x;
  const float* row = logits + static_cast<int64_t>(g) * T;
  const float4 l4 = reinterpret_cast<const float4*>(row)[j];
  const float l[4] = {l4.x, l4.y, l4.z, l4.w};

  float mx = -INFINITY;
  int m = INT_MAX;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (better(l[i], 4 * j + i, mx, m)) {
      mx = l[i];
      m = 4 * j + i;
    }
  block_argmax(mx, m, sv, sk);
  if (m == INT_MAX) m = 0;  // all NaN: nothing is confident (below)

  float e[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) e[i] = expf(l[i] - mx);
  const float total = block_sum((e[0] + e[1]) + (e[2] + e[3]), red);

  // centre from the five neighbours of m (the 1 / total factor cancels)
  float wsum = 0.f, dsum = 0.f;
#pragma unroll
  for (int d = -2; d <= 2; ++d) {
    const float w = expf(row[(m + d) & (T - 1)] - mx);
    wsum += w;
    dsum += static_cast<float>(d) * w;
  }
  const int S = fine_len / T;
  const float c = static_cast<float>(S) * (static_cast<float>(m) + dsum / wsum);
  const float half_n = 0.5f * static_cast<float>(fine_len);
  const float margin = 0.5f * static_cast<float>(window_bins) - static_cast<float>(S);
  float part = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float x = static_cast<float>(S * (4 * j + i)) - c + half_n;  // offset + N/2, then mod N
    x -= static_cast<float>(fine_len) * floorf(x / static_cast<float>(fine_len));
    if (fabsf(x - half_n) <= margin) part += e[i];
  }
  const float conf = block_sum(part, red) / total;
  if (j == 0) {
    const float cc = isfinite(c) ? c : 0.f;  // NaN logits: start at bin 0, not confident
    int64_t st = static_cast<int64_t>(floorf(cc + 0.5f)) - window_bins / 2;
    st %= fine_len;
    if (st < 0) st += fine_len;
    bin_start[g] = static_cast<int32_t>(st);
    const bool ok = conf >= threshold;  // false for NaN
    if (confidence) confidence[g] = conf;
    flag[g] = ok ? 1 : 0;
    __threadfence();  // release this gate's outputs before counting it
    is_last = atomicAdd(done, 1) == n_gates - 1;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();  // acquire every other workgroup's flag
  compact_gates(flag, n_gates, zoom_list, fallback_list, counts, wtot);
  if (j == 0) *done = 0;
}

__global__ void __launch_bounds__(NT)
select_windows(const float* __restrict__ logits, int32_t n_gates, int32_t fine_len,
               int32_t window_bins, float threshold, int32_t* __restrict__ bin_start,
               float* __restrict__ confidence, int32_t* __restrict__ flag,
               int32_t* __restrict__ zoom_list, int32_t* __restrict__ fallback_list,
               int32_t* __restrict__ counts, int32_t* __restrict__ done) {
  select_window_block(static_cast<int>(blockIdx.x), logits, n_gates, fine_len, window_bins,
                      threshold, bin_start, confidence, flag, zoom_list, fallback_list, counts,
                      done);
}

// The window decision (workgroups g < n_gates) and, in the same launch, the
// zoom DFT's per-pulse FP16 exponents (workgroup n_gates + p for pulse p).
__global__ void __launch_bounds__(NT)
select_and_exponents(const float* __restrict__ logits, int32_t n_gates, int32_t fine_len,
                     int32_t window_bins, float threshold, int32_t* __restrict__ bin_start,
                     float* __restrict__ confidence, int32_t* __restrict__ flag,
                     int32_t* __restrict__ zoom_list, int32_t* __restrict__ fallback_list,
                     int32_t* __restrict__ counts, int32_t* __restrict__ done, PulseExpArgs pe) {
  static_assert(NT == 256, "the exponent role runs 256 threads");
  const int b = static_cast<int>(blockIdx.x);
  if (b < n_gates) {
    select_window_block(b, logits, n_gates, fine_len, window_bins, threshold, bin_start,
                        confidence, flag, zoom_list, fallback_list, counts, done);
  } else {
    if (pe.exps)
      pulse_exponent_block(pe.samples, pe.sample_type, pe.tx, pe.stride, pe.lo, pe.hi,
                           pe.code_len, pe.tx_per_pulse, b - n_gates, pe.exps);
    if (pe.bits)
      code_bits_block(pe.tx, pe.code_len, pe.tx_per_pulse, pe.bit_words, b - n_gates, pe.bits,
                      pe.binary);
  }
}

// Peak of each listed gate's window: (value, -local index) maximum of row g
// of the [n_gates][K] window spectra, reported as the bin (start + j) mod N.
__global__ void __launch_bounds__(NT)
window_peak(const float* __restrict__ spectra, int32_t n_gates, int32_t window_bins,
            int32_t fine_len, const int32_t* __restrict__ bin_start,
            const int32_t* __restrict__ list, const int32_t* __restrict__ count,
            int32_t* __restrict__ peak_bin, float* __restrict__ peak_power) {
  __shared__ float sv[NT / 64];
  __shared__ int sk[NT / 64];
  if (static_cast<int>(blockIdx.x) >= *count) return;
  const int g = list[blockIdx.x];
  if (g < 0 || g >= n_gates) return;
  const float* row = spectra + static_cast<int64_t>(g) * window_bins;
  float bv = -INFINITY;
  int bk = INT_MAX;
  for (int i = threadIdx.x; i < window_bins; i += NT) {
    const float v = row[i];
    if (better(v, i, bv, bk)) {
      bv = v;
      bk = i;
    }
  }
  block_argmax(bv, bk, sv, sk);
  if (threadIdx.x == 0) {
    if (bk == INT_MAX) {  // only NaN
      bk = 0;
      bv = row[0];
    }
    int64_t st = bin_start[g] % fine_len;
    if (st < 0) st += fine_len;
    peak_bin[g] = static_cast<int32_t>((st + bk) % fine_len);
    if (peak_power) peak_power[g] = bv;
  }
}

// Peak of every gate of the learned zoom: over its window when it was zoomed,
// over the whole full-resolution row otherwise (ties to the lowest bin, NaN
// never wins).  Workgroup b < k takes slot b of the fallback list (k = its
// device-side count), the others the zoom list in order.  When the zoom or
// the fallback launch split its pulses into chunks, the gate's row is first
// summed from the chunk partials in ascending chunk order and written out:
// [C][G][K] partials of the zoom, and for the fallback the [C][k][N] partials
// by list slot of its adaptive chunking (C from k by the rule the fallback
// launch used).  A few fallback gates with many chunks are the heavy items:
// each thread keeps eight bins' loads of four chunks in flight.
__global__ void __launch_bounds__(NT)
split_peaks(float* __restrict__ window_spectra, const float* __restrict__ window_partial,
            int32_t zoom_chunks, float* __restrict__ full_spectra, FallbackChunks fb,
            const int32_t* __restrict__ zoom_list, const int32_t* __restrict__ fallback_list,
            const int32_t* __restrict__ bin_start, int32_t n_gates, int32_t window_bins,
            int32_t fine_len, int32_t* __restrict__ peak_bin, float* __restrict__ peak_power) {
  __shared__ float sv[NT / 64];
  __shared__ int sk[NT / 64];
  const int k = min(max(fb.counts[1], 0), n_gates);
  const int b = blockIdx.x;
  const bool zoomed = b >= k;
  const int slot = zoomed ? b - k : b;
  if (zoomed && slot >= min(max(fb.counts[0], 0), n_gates - k)) return;
  const int g = zoomed ? zoom_list[slot] : fallback_list[slot];
  if (g < 0 || g >= n_gates) return;
  const int len = zoomed ? window_bins : fine_len;
  float* row = zoomed ? window_spectra + static_cast<int64_t>(g) * window_bins
                      : full_spectra + static_cast<int64_t>(g) * fine_len;
  int chunks;
  const float* part;
  int64_t cstride;
  if (zoomed) {
    chunks = zoom_chunks;
    part = window_partial + static_cast<int64_t>(g) * len;
    cstride = static_cast<int64_t>(n_gates) * len;
  } else {
    chunks = adaptive_chunks(k, fb.zgroups, fb.target, fb.max_chunks, fb.rows);
    part = fb.partial + static_cast<int64_t>(slot) * len;
    cstride = static_cast<int64_t>(k) * len;
  }
  constexpr int U = 8;  // bins per thread and step
  float bv = -INFINITY;
  int bk = INT_MAX;
  for (int i0 = threadIdx.x; i0 < len; i0 += U * NT) {
    float v[U];
    if (chunks > 1) {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = 0.f;
      int c = 0;
      for (; c + 4 <= chunks; c += 4) {  // 4 U loads in flight, then the sums in chunk order
        float t[4][U];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int i = min(i0 + u * NT, len - 1);
            t[cc][u] = part[(c + cc) * cstride + i];
          }
#pragma unroll
        for (int cc = 0; cc < 4; ++cc)
#pragma unroll
          for (int u = 0; u < U; ++u) v[u] += t[cc][u];
      }
      for (; c < chunks; ++c)
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] += part[c * cstride + min(i0 + u * NT, len - 1)];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (i0 + u * NT < len) row[i0 + u * NT] = v[u];
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = i0 + u * NT < len ? row[i0 + u * NT] : -INFINITY;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * NT;
      if (i < len && better(v[u], i, bv, bk)) {
        bv = v[u];
        bk = i;
      }
    }
  }
  block_argmax(bv, bk, sv, sk);
  if (threadIdx.x == 0) {
    if (bk == INT_MAX) {  // only NaN; thread 0 itself formed bin 0
      bk = 0;
      bv = row[0];
    }
    int64_t pb = bk;
    if (zoomed) {
      int64_t st = bin_start[g] % fine_len;
      if (st < 0) st += fine_len;
      pb = (st + bk) % fine_len;
    }
    peak_bin[g] = static_cast<int32_t>(pb);
    if (peak_power) peak_power[g] = bv;
  }
}

}  // namespace

hipError_t launch_select_windows(const float* logits, int32_t n_gates, int32_t fine_len,
                                 int32_t window_bins, float threshold, int32_t* bin_start,
                                 float* confidence, int32_t* flag, int32_t* zoom_list,
                                 int32_t* fallback_list, int32_t* counts, int32_t* done,
                                 hipStream_t s) {
  hipLaunchKernelGGL(select_windows, dim3(static_cast<unsigned>(n_gates)), dim3(NT), 0, s, logits,
                     n_gates, fine_len, window_bins, threshold, bin_start, confidence, flag,
                     zoom_list, fallback_list, counts, done);
  return hipGetLastError();
}

hipError_t launch_split_peaks(float* window_spectra, const float* window_partial,
                              int32_t zoom_chunks, float* full_spectra, const FallbackChunks& fb,
                              const int32_t* zoom_list, const int32_t* fallback_list,
                              const int32_t* bin_start, int32_t n_gates, int32_t window_bins,
                              int32_t fine_len, int32_t* peak_bin, float* peak_power,
                              hipStream_t s) {
  hipLaunchKernelGGL(split_peaks, dim3(static_cast<unsigned>(n_gates)), dim3(NT), 0, s,
                     window_spectra, window_partial, zoom_chunks, full_spectra, fb, zoom_list,
                     fallback_list, bin_start, n_gates, window_bins, fine_len, peak_bin,
                     peak_power);
  return hipGetLastError();
}

hipError_t launch_select_and_exponents(const float* logits, int32_t n_gates, int32_t fine_len,
                                       int32_t window_bins, float threshold, int32_t* bin_start,
                                       float* confidence, int32_t* flag, int32_t* zoom_list,
                                       int32_t* fallback_list, int32_t* counts, int32_t* done,
                                       const PulseExpArgs& pe, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>(n_gates) + static_cast<unsigned>(pe.n_pulses);
  hipLaunchKernelGGL(select_and_exponents, dim3(blocks), dim3(NT), 0, s, logits, n_gates,
                     fine_len, window_bins, threshold, bin_start, confidence, flag, zoom_list,
                     fallback_list, counts, done, pe);
  return hipGetLastError();
}

hipError_t launch_window_peak(const float* spectra, int32_t n_gates, int32_t window_bins,
                              int32_t fine_len, const int32_t* bin_start, const int32_t* list,
                              const int32_t* count, int32_t* peak_bin, float* peak_power,
                              hipStream_t s) {
  hipLaunchKernelGGL(window_peak, dim3(static_cast<unsigned>(n_gates)), dim3(NT), 0, s, spectra,
                     n_gates, window_bins, fine_len, bin_start, list, count, peak_bin, peak_power);
  return hipGetLastError();
}

}  // namespace ispl
