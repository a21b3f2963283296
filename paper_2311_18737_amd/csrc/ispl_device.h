// Device helpers shared by several kernel files (HIP only; never included by
// host-only translation units).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ispl {

// Sample i of a row: complex64, or an int16 (re, im) pair (exact in float).
__device__ __forceinline__ float2 load_any_sample(const void* base, int32_t sample_type,
                                                  int64_t i) {
  if (sample_type == 1) {
    const uint32_t r = reinterpret_cast<const uint32_t*>(base)[i];
    return make_float2(static_cast<float>(static_cast<int16_t>(r & 0xffffu)),
                       static_cast<float>(static_cast<int32_t>(r) >> 16));
  }
  return reinterpret_cast<const float2*>(base)[i];
}

// FP16 column exponent of pulse p, computed by one workgroup of 256 threads:
// the e with max|x| max|c| 2^e < 2^14 over the samples [lo, hi) of the pulse
// row that some gate reads and over the pulse's code, so that no split FP16
// value of the zoom DFT overflows and the low halves stay normal down to about
// 2^-17 of that maximum.  Clamped to [-60, 60]; 0 for an all-zero pulse.
__device__ __forceinline__ void pulse_exponent_block(const void* __restrict__ samples,
                                                     int32_t sample_type,
                                                     const float* __restrict__ tx,
                                                     int64_t stride, int64_t lo, int64_t hi,
                                                     int32_t code_len, int32_t tx_per_pulse,
                                                     int p, int32_t* __restrict__ exps) {
  __shared__ float red[2][4];
  float mx = 0.f, mc = 0.f;
  const int64_t base = static_cast<int64_t>(p) * stride;
  // eight loads in flight per thread (indices clamped into the span, the
  // clamped ones counted as zero); the maximum does not depend on the order
  constexpr int U = 8;
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += 256 * U) {
    float2 x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + 256 * u;
      x[u] = load_any_sample(samples, sample_type, base + (i < hi ? i : hi - 1));
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + 256 * u < hi) mx = fmaxf(mx, x[u].x * x[u].x + x[u].y * x[u].y);
  }
  const float2* txp = reinterpret_cast<const float2*>(tx) +
                      (tx_per_pulse ? static_cast<int64_t>(p) * code_len : 0);
  for (int n0 = threadIdx.x; n0 < code_len; n0 += 256 * U) {
    float2 c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int n = n0 + 256 * u;
      c[u] = txp[n < code_len ? n : code_len - 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (n0 + 256 * u < code_len) mc = fmaxf(mc, c[u].x * c[u].x + c[u].y * c[u].y);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmaxf(mx, __shfl_xor(mx, off));
    mc = fmaxf(mc, __shfl_xor(mc, off));
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = mx;
    red[1][threadIdx.x >> 6] = mc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = fmaxf(fmaxf(red[0][0], red[0][1]), fmaxf(red[0][2], red[0][3]));
    mc = fmaxf(fmaxf(red[1][0], red[1][1]), fmaxf(red[1][2], red[1][3]));
    int e = 0;
    const float m = sqrtf(mx) * sqrtf(mc);
    if (m > 0.f && isfinite(m)) {
      int ex;
      frexpf(m, &ex);  // m < 2^ex
      e = 14 - ex;
    }
    exps[p] = max(-60, min(60, e));
  }
}

// Sign bits of pulse p's code for the zoom DFT, by one workgroup of 256
// threads: bit b of word w of bits[p] is set when code[32 w + b] == -1 + 0i
// (positions past L read as +1), and binary[p] = 1 when every code of the row
// is exactly +-1 + 0i (0: the zoom then reads the row as complex codes).
// words * 32 must be a multiple of 64 (one ballot of a wave gives two words).
// With a code shared by all pulses only row 0 exists (p == 0 writes it).
__device__ __forceinline__ void code_bits_block(const float* __restrict__ tx, int32_t code_len,
                                                int32_t tx_per_pulse, int32_t words, int p,
                                                uint32_t* __restrict__ bits,
                                                int32_t* __restrict__ binary) {
  if (!tx_per_pulse && p != 0) return;  // uniform over the workgroup
  const float2* txp = reinterpret_cast<const float2*>(tx) +
                      (tx_per_pulse ? static_cast<int64_t>(p) * code_len : 0);
  const int lane = threadIdx.x & 63;
  bool ok = true;
  for (int n0 = 64 * (threadIdx.x >> 6); n0 < 32 * words; n0 += 256) {  // wave-uniform
    const int n = n0 + lane;
    bool neg = false;
    if (n < code_len) {
      const float2 c = txp[n];
      ok = ok && c.y == 0.f && (c.x == 1.f || c.x == -1.f);
      neg = c.x < 0.f;
    }
    const uint64_t m = __ballot(neg);
    if (lane == 0) {
      uint32_t* w = bits + static_cast<int64_t>(p) * words + n0 / 32;
      w[0] = static_cast<uint32_t>(m);
      w[1] = static_cast<uint32_t>(m >> 32);
    }
  }
  ok = __syncthreads_and(ok);
  if (threadIdx.x == 0) binary[p] = ok ? 1 : 0;
}

}  // namespace ispl
