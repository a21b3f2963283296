// Zoom DFT on the matrix cores (gfx950 MFMA): a window of K bins of the
// N-point spectrum of every gate, S[g][j] = sum_p |Z_{p,g}[j]|^2 with
//
//   Z_{p,g}[j] = sum_{n < L} y'_{p,g}[n] W_N^{j n},
//   y'_{p,g}[n] = conj(c_p[n]) x_p[g0 + g s + n] W_N^{k0_g n},
//
// i.e. the decoded row of Section 3.2 shifted so that bin k0_g (the window
// start of gate g) sits at 0, then a direct DFT onto K bins.  The DFT matrix
// W_N^{j n} is the same for every gate and pulse, so the work is one real
// GEMM per gate: rows 2j, 2j+1 hold Re/Im of bin j, columns are pulses and
// the reduction runs over (Re, Im) of the L samples.
//
// Precision: both operands are split into a high and a low 16-bit part
// (BF16 or FP16) and D = A_hi B_hi + A_hi B_lo + A_lo B_hi accumulates in
// FP32; the dropped A_lo B_lo term and the split residuals are about 2^-16
// (BF16) or 2^-22 (FP16) of each product.  FP16 columns are scaled by a power
// of two so their largest sample sits near 2^14 (no overflow, low parts stay
// normal) and the scale is removed exactly before the pulse sum.  Decode,
// shift and pulse integration run in FP32.
//
// Tiling: a workgroup of 8 waves owns one gate and 128 bins (16 per wave, a
// 32-row MFMA tile each) and sweeps the pulses in blocks of 128 columns (four
// 32x32 tiles per wave).  The decoded, shifted and split samples of a block
// are built once per 64-sample chunk in LDS in the MFMA B-operand layout; the
// A operand (DFT matrix, split) streams from a table laid out in the
// A-operand order, 16 bytes per lane per step.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ispl_internal.h"

namespace ispl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int ZW = 8;              // waves per workgroup
constexpr int ZT = 64 * ZW;        // threads
constexpr int ZCOLS = 128;         // pulses per block (four 32-column tiles)
constexpr int ZCHUNK = 64;         // samples per B chunk (8 MFMA k-steps of 16 rows)
constexpr int ZKS = 2 * ZCHUNK / 16;

struct alignas(16) Frag {  // 8 x 16-bit MFMA operand of one lane
  uint32_t w[4];
};

__device__ __forceinline__ uint32_t bf16_bits(float x) {  // round to nearest even
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ uint32_t f16_bits(float x) {
  _Float16 h = static_cast<_Float16>(x);
  return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, h));
}
__device__ __forceinline__ float f16_value(uint32_t h) {
  return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(h)));
}

template <int PREC>
__device__ __forceinline__ void split2(float x, uint32_t& hi, uint32_t& lo) {
  if (PREC == 0) {
    hi = bf16_bits(x);
    lo = bf16_bits(x - bf16_value(hi));
  } else {
    hi = f16_bits(x);
    lo = f16_bits(x - f16_value(hi));
  }
}

template <int PREC>
__device__ __forceinline__ f32x16 mfma(const Frag& a, const Frag& b, f32x16 c) {
  if constexpr (PREC == 0)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

template <int ST>
__device__ __forceinline__ float2 load_sample(const void* base, int64_t i) {
  if constexpr (ST == 0) {
    return reinterpret_cast<const float2*>(base)[i];
  } else {
    const uint32_t r = reinterpret_cast<const uint32_t*>(base)[i];
    return make_float2(static_cast<float>(static_cast<int16_t>(r & 0xffffu)),
                       static_cast<float>(static_cast<int32_t>(r) >> 16));
  }
}

template <int PREC, int ST>
__global__ void __launch_bounds__(ZT) zoom_spectra(ZoomArgs a) {
  __shared__ Frag bh[4][ZKS][64];  // B operand, high parts: [column tile][k-step][lane]
  __shared__ Frag bl[4][ZKS][64];  // low parts
  __shared__ int col_exp[ZCOLS];
  __shared__ float col_max[4][ZCOLS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int btiles = a.n_bins / 128;
  int g = blockIdx.x / btiles;
  const int bt = blockIdx.x % btiles;
  if (a.gate_list) {  // uniform over the workgroup, before any barrier
    if (g >= *a.gate_count) return;
    g = a.gate_list[g];
    if (g < 0 || g >= a.n_gates) return;
  }
  const int L = a.code_len, N = a.n_fft, P = a.n_pulses;
  const int nchunks = a.code_pad / ZCHUNK;
  const int k0 = ((a.bin_start[g] % N) + N) % N;
  const float2* __restrict__ tw = reinterpret_cast<const float2*>(a.twiddle);
  const float2* __restrict__ txb = reinterpret_cast<const float2*>(a.tx);
  const int64_t gate_off = static_cast<int64_t>(a.first_gate) + static_cast<int64_t>(g) * a.gate_step;

  // A operand of this wave: row tile rt of the table, k-steps along the code
  const int rt = bt * ZW + wave;
  const Frag* __restrict__ ah_t = reinterpret_cast<const Frag*>(a.a_hi) +
                                  static_cast<int64_t>(rt) * (a.code_pad / 8) * 64;
  const Frag* __restrict__ al_t = reinterpret_cast<const Frag*>(a.a_lo) +
                                  static_cast<int64_t>(rt) * (a.code_pad / 8) * 64;

  // per-lane sums of the 8 bins this lane reduces (bins 2 (4 q + s) + h ... see below)
  float total[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) total[i] = 0.f;

  // B-building role: column (pulse) pc of the block, sample groups q, q + 4, ...
  const int pc = tid % ZCOLS, q0 = tid / ZCOLS;  // q0 in 0..3

  for (int pb = 0; pb < P; pb += ZCOLS) {
    const int p = pb + pc;
    const bool live = p < P;
    const int64_t rowp = static_cast<int64_t>(live ? p : 0) * a.stride + gate_off;
    const float2* txp = txb + (a.tx_per_pulse ? static_cast<int64_t>(live ? p : 0) * L : 0);

    // column scale: 2^e with max |y'| 2^e near 2^14 (FP16), 1 (BF16)
    if (PREC == 1) {
      float m = 0.f;
      if (live)
        for (int n = q0; n < L; n += 4) {
          const float2 x = load_sample<ST>(a.samples, rowp + n);
          const float2 c = txp[n];
          m = fmaxf(m, (x.x * x.x + x.y * x.y) * (c.x * c.x + c.y * c.y));
        }
      col_max[q0][pc] = m;
      __syncthreads();
      if (q0 == 0) {
        const float mm = fmaxf(fmaxf(col_max[0][pc], col_max[1][pc]),
                               fmaxf(col_max[2][pc], col_max[3][pc]));
        int e = 0;
        if (mm > 0.f) {
          int ex;
          frexpf(sqrtf(mm), &ex);  // sqrt(mm) < 2^ex
          e = 14 - ex;
        }
        col_exp[pc] = e;
      }
      __syncthreads();
    }
    const float scale = PREC == 1 ? ldexpf(1.f, col_exp[pc]) : 1.f;

    f32x16 acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[ct][r] = 0.f;

    for (int ch = 0; ch < nchunks; ++ch) {
      // build the B chunk: group q covers samples 4 q .. 4 q + 3 of the chunk,
      // i.e. reduction rows 8 q .. 8 q + 7 = k-step q / 2, lane half q % 2
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int qg = q0 + 4 * i;
        Frag fh, fl;
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const int n = ch * ZCHUNK + 4 * qg + s2;
          float2 y = make_float2(0.f, 0.f);
          if (live && n < L) {
            const float2 x = load_sample<ST>(a.samples, rowp + n);
            const float2 c = txp[n];
            const float2 d = make_float2(fmaf(c.x, x.x, c.y * x.y), fmaf(c.x, x.y, -(c.y * x.x)));
            // N is a power of two, so k0 n mod N survives the 32-bit wrap
            const float2 w = tw[(static_cast<uint32_t>(k0) * static_cast<uint32_t>(n)) &
                                static_cast<uint32_t>(N - 1)];
            y = make_float2(fmaf(d.x, w.x, -(d.y * w.y)) * scale, fmaf(d.x, w.y, d.y * w.x) * scale);
          }
          uint32_t rh, rl, ih, il;
          split2<PREC>(y.x, rh, rl);
          split2<PREC>(y.y, ih, il);
          fh.w[s2] = rh | (ih << 16);
          fl.w[s2] = rl | (il << 16);
        }
        const int ks = qg >> 1, ln = (pc & 31) + 32 * (qg & 1), ct = pc >> 5;
        bh[ct][ks][ln] = fh;
        bl[ct][ks][ln] = fl;
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < ZKS; ++ks) {
        const int64_t ai = static_cast<int64_t>(ch * ZKS + ks) * 64 + lane;
        const Frag fah = ah_t[ai], fal = al_t[ai];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          const Frag fbh = bh[ct][ks][lane], fbl = bl[ct][ks][lane];
          acc[ct] = mfma<PREC>(fah, fbh, acc[ct]);
          acc[ct] = mfma<PREC>(fah, fbl, acc[ct]);
          acc[ct] = mfma<PREC>(fal, fbh, acc[ct]);
        }
      }
      __syncthreads();
    }

    // |Z|^2 per (bin, pulse).  D row (r % 4) + 8 (r / 4) + 4 h (h = lane / 32)
    // is Re (even) or Im (odd) of wave bin row / 2, so registers r, r + 1 with
    // r % 4 in {0, 2} are one bin: local bin 2 (r / 4)... b = {0,1} + 4 (r / 4) + 2 h.
    float pw[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) pw[i] = 0.f;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int pcol = pb + 32 * ct + (lane & 31);
      const float un = PREC == 1 && pcol < P ? ldexpf(1.f, -2 * col_exp[32 * ct + (lane & 31)]) : 1.f;
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const float re = acc[ct][4 * qa + 2 * s], im = acc[ct][4 * qa + 2 * s + 1];
          pw[2 * qa + s] += fmaf(re, re, im * im) * un;
        }
    }
    // sum over the 32 pulse columns of each half wave, fixed order
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float v = pw[i];
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) v += __shfl_xor(v, off);
      total[i] += v;
    }
    __syncthreads();  // column scales are rewritten by the next block
  }

  // lane 0 holds bins b = s + 4 qa (h = 0), lane 32 bins s + 4 qa + 2 (h = 1)
  if ((lane & 31) == 0) {
    const int h = lane >> 5;
    float* out = a.out + static_cast<int64_t>(g) * a.n_bins + bt * 128 + 16 * wave;
#pragma unroll
    for (int qa = 0; qa < 4; ++qa)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        float* dst = out + s + 4 * qa + 2 * h;
        *dst = a.accumulate ? *dst + total[2 * qa + s] : total[2 * qa + s];
      }
  }
}

template <int PREC>
hipError_t launch_zoom_t(const ZoomArgs& a, hipStream_t stream) {
  const unsigned blocks = static_cast<unsigned>(a.n_gates) * (a.n_bins / 128);
  if (a.sample_type == 1)
    hipLaunchKernelGGL((zoom_spectra<PREC, 1>), dim3(blocks), dim3(ZT), 0, stream, a);
  else
    hipLaunchKernelGGL((zoom_spectra<PREC, 0>), dim3(blocks), dim3(ZT), 0, stream, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_zoom(const ZoomArgs& a, hipStream_t stream) {
  return a.precision == 1 ? launch_zoom_t<1>(a, stream) : launch_zoom_t<0>(a, stream);
}

}  // namespace ispl
