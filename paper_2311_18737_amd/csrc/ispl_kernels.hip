// Device code of the plasma-line spectrum library (gfx950, wave64).
//
// One fused kernel runs the whole per-pulse chain of Section 3.2 -- decode by
// the conjugated transmit code (3.2.1), Fourier transform (3.2.2), squared
// modulus and accumulation over pulses (3.2.3) -- without ever writing the
// decoded rows or their transforms to memory.
//
// Transform layout.  The decoded row y has L <= 1024 non-zero samples and is
// zero-padded to N = R * 1024.  Splitting the output bin as k = k1 + R * kk,
//
//   X[k1 + R kk] = sum_{n < 1024} (y[n] W_N^{k1 n}) W_1024^{kk n},
//
// so each bin class k1 is one pre-twiddled 1024-point DFT (the radix-R first
// pass of the full transform is empty apart from its twiddles).  One wave owns
// one k1 and computes its 1024-point DFT as 16 x 16 x 4:
//   pass 1  lane l holds y[l + 64 j], j < 16: 16-point DFT over j, twiddle;
//   pass 2  via an LDS transpose, lane (ka, r) holds u_ka[r + 4 m]: 16-point
//           DFT over m, twiddle W_64^{r kc};
//   pass 3  via a second transpose, 4-point DFTs over r give bin
//           kk = ka + 16 kc + 256 kd.
// Every lane keeps the running |X|^2 of its 16 bins in registers across the
// whole pulse loop, so the only spectrum traffic is one store per bin at the
// end.  The waves of a workgroup share one gate and one pulse at a time: the
// row is decoded once into LDS and read by every wave.

#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>
#include <stdint.h>

#include "ispl_internal.h"

namespace ispl {
namespace {

constexpr int XPITCH = 68;          // float2 per 64-entry row of the exchange buffer
constexpr int XWAVE = 16 * XPITCH;  // float2 of one wave's exchange buffer

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ float2 conj_mul(float2 c, float2 x) {  // conj(c) * x
  return make_float2(fmaf(c.x, x.x, c.y * x.y), fmaf(c.x, x.y, -(c.y * x.x)));
}

// 4-point forward DFT in place, natural order in and out.
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float t0x = a0.x + a2.x, t0y = a0.y + a2.y;
  const float t1x = a0.x - a2.x, t1y = a0.y - a2.y;
  const float t2x = a1.x + a3.x, t2y = a1.y + a3.y;
  const float t3x = a1.x - a3.x, t3y = a1.y - a3.y;
  a0 = make_float2(t0x + t2x, t0y + t2y);
  a2 = make_float2(t0x - t2x, t0y - t2y);
  a1 = make_float2(t1x + t3y, t1y - t3x);  // t1 - i t3
  a3 = make_float2(t1x - t3y, t1y + t3x);  // t1 + i t3
}

constexpr float kC8 = 0.923879532511286756f;  // cos(pi / 8)
constexpr float kS8 = 0.382683432365089772f;  // sin(pi / 8)
constexpr float kR2 = 0.707106781186547524f;  // cos(pi / 4)

// Multiplication by W_16^m = exp(-2 pi i m / 16).
__device__ __forceinline__ float2 w16_1(float2 a) { return cmul(a, make_float2(kC8, -kS8)); }
__device__ __forceinline__ float2 w16_2(float2 a) {
  return make_float2(kR2 * (a.x + a.y), kR2 * (a.y - a.x));
}
__device__ __forceinline__ float2 w16_3(float2 a) { return cmul(a, make_float2(kS8, -kC8)); }
__device__ __forceinline__ float2 w16_4(float2 a) { return make_float2(a.y, -a.x); }
__device__ __forceinline__ float2 w16_6(float2 a) {
  return make_float2(kR2 * (a.y - a.x), -kR2 * (a.x + a.y));
}
__device__ __forceinline__ float2 w16_9(float2 a) { return cmul(a, make_float2(-kC8, kS8)); }

// 16-point forward DFT in registers, natural order in and out:
// j = j1 + 4 j2, k = k1 + 4 k2; DFT4 over j2, twiddle W_16^{j1 k1}, DFT4 over j1.
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
  dft4(v[0], v[4], v[8], v[12]);
  dft4(v[1], v[5], v[9], v[13]);
  dft4(v[2], v[6], v[10], v[14]);
  dft4(v[3], v[7], v[11], v[15]);
  v[5] = w16_1(v[5]);
  v[9] = w16_2(v[9]);
  v[13] = w16_3(v[13]);
  v[6] = w16_2(v[6]);
  v[10] = w16_4(v[10]);
  v[14] = w16_6(v[14]);
  v[7] = w16_3(v[7]);
  v[11] = w16_6(v[11]);
  v[15] = w16_9(v[15]);
  dft4(v[0], v[1], v[2], v[3]);
  dft4(v[4], v[5], v[6], v[7]);
  dft4(v[8], v[9], v[10], v[11]);
  dft4(v[12], v[13], v[14], v[15]);
  float2 t[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) t[k] = v[4 * (k & 3) + (k >> 2)];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = t[k];
}

// Orders this wave's LDS accesses around a cross-lane exchange.  LDS requests
// of one wave are served in issue order, so only the compiler needs fencing.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int ST>
struct SampleIO;

template <>
struct SampleIO<0> {  // complex64
  using raw_t = float2;
  __device__ static raw_t load(const void* base, int64_t i) {
    return reinterpret_cast<const float2*>(base)[i];
  }
  __device__ static raw_t zero() { return make_float2(0.f, 0.f); }
  __device__ static float2 cvt(raw_t r) { return r; }
};

template <>
struct SampleIO<1> {  // int16 (re, im) pairs; int16 -> float is exact
  using raw_t = uint32_t;
  __device__ static raw_t load(const void* base, int64_t i) {
    return reinterpret_cast<const uint32_t*>(base)[i];
  }
  __device__ static raw_t zero() { return 0u; }
  __device__ static float2 cvt(raw_t r) {
    return make_float2(static_cast<float>(static_cast<int16_t>(r & 0xffffu)),
                       static_cast<float>(static_cast<int32_t>(r) >> 16));
  }
};

template <int RW, int ST>
__global__ void __launch_bounds__(64 * RW) fused_spectra(FusedArgs a) {
  constexpr int NT = 64 * RW;
  constexpr int E = SUB / NT;          // decoded samples staged per thread
  constexpr bool DBUF = (RW == 16);    // double-buffer the decoded row when LDS allows
  using IO = SampleIO<ST>;
  using raw_t = typename IO::raw_t;

  __shared__ float2 xs[RW * XWAVE];
  __shared__ float2 ys[DBUF ? 2 : 1][SUB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int R = 1 << a.log2_r;
  const int zgroups = R / RW;
  int bid = blockIdx.x;
  const int c = bid % a.chunks;
  bid /= a.chunks;
  const int zg = bid % zgroups;
  const int g = bid / zgroups;
  const int k1 = zg * RW + wave;
  const int N = a.n_fft;
  const int nmask = N - 1;
  const int L = a.code_len;
  const float2* __restrict__ tw = reinterpret_cast<const float2*>(a.twiddle);

  const int p0 = static_cast<int>((static_cast<int64_t>(c) * a.n_pulses) / a.chunks);
  const int p1 = static_cast<int>((static_cast<int64_t>(c + 1) * a.n_pulses) / a.chunks);

  // Twiddles, fixed over the pulse loop.
  float2 pre[16];  // W_N^{64 k1 j}: same for every lane
  float2 tw1[16];  // W_N^{l (k1 + R ka)} = W_N^{k1 l} W_1024^{l ka}
  float2 tw2[16];  // W_64^{r kc}
  const int r2 = lane & 3;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    pre[j] = tw[(64 * k1 * j) & nmask];
    tw1[j] = tw[(lane * (k1 + R * j)) & nmask];
    tw2[j] = tw[((N >> 6) * r2 * j) & nmask];
  }

  float acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;

  const int64_t gate_off = static_cast<int64_t>(a.first_gate) + static_cast<int64_t>(g) * a.gate_step;
  const float2* __restrict__ txb = reinterpret_cast<const float2*>(a.tx);

  raw_t raw[E];
  float2 cod[E];
  auto load = [&](int p) {
    const int64_t row = static_cast<int64_t>(p) * a.stride + gate_off;
    const float2* txp = txb + (a.tx_per_pulse ? static_cast<int64_t>(p) * L : 0);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int n = tid + i * NT;
      if (n < L) {
        raw[i] = IO::load(a.samples, row + n);
        cod[i] = txp[n];
      } else {
        raw[i] = IO::zero();
        cod[i] = make_float2(0.f, 0.f);
      }
    }
  };

  float2* xw = xs + wave * XWAVE;
  const int ka2 = lane >> 2;  // pass-2 lane role (ka, r)
  const int ka3 = lane & 15;  // pass-3 lane role (ka, q)
  const int q3 = lane >> 4;

  if (p0 < p1) load(p0);
  for (int p = p0; p < p1; ++p) {
    const int buf = DBUF ? ((p - p0) & 1) : 0;
    if (!DBUF) __syncthreads();  // every wave has read the previous row
#pragma unroll
    for (int i = 0; i < E; ++i) ys[buf][tid + i * NT] = conj_mul(cod[i], IO::cvt(raw[i]));
    if (p + 1 < p1) load(p + 1);
    __syncthreads();

    // pass 1: 16-point DFTs over the stride-64 samples of each lane
    float2 v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = ys[buf][lane + 64 * j];
    if (k1 != 0) {
#pragma unroll
      for (int j = 1; j < 16; ++j) v[j] = cmul(v[j], pre[j]);
    }
    dft16(v);
#pragma unroll
    for (int ka = 0; ka < 16; ++ka) xw[ka * XPITCH + lane] = cmul(v[ka], tw1[ka]);
    wave_lds_sync();

    // pass 2: lane (ka2, r2) transforms u_ka[r2 + 4 m] over m; it rewrites
    // exactly the entries it read, so no other lane's input is overwritten
#pragma unroll
    for (int m = 0; m < 16; ++m) v[m] = xw[ka2 * XPITCH + r2 + 4 * m];
    dft16(v);
    xw[ka2 * XPITCH + r2] = v[0];
#pragma unroll
    for (int kc = 1; kc < 16; ++kc) xw[ka2 * XPITCH + 4 * kc + r2] = cmul(v[kc], tw2[kc]);
    wave_lds_sync();

    // pass 3: 4-point DFTs over r, then |X|^2 into the running sums
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int base = ka3 * XPITCH + 4 * (4 * q3 + t);
      float2 c0 = xw[base + 0], c1 = xw[base + 1], c2 = xw[base + 2], c3 = xw[base + 3];
      dft4(c0, c1, c2, c3);
      acc[4 * t + 0] = fmaf(c0.y, c0.y, fmaf(c0.x, c0.x, acc[4 * t + 0]));
      acc[4 * t + 1] = fmaf(c1.y, c1.y, fmaf(c1.x, c1.x, acc[4 * t + 1]));
      acc[4 * t + 2] = fmaf(c2.y, c2.y, fmaf(c2.x, c2.x, acc[4 * t + 2]));
      acc[4 * t + 3] = fmaf(c3.y, c3.y, fmaf(c3.x, c3.x, acc[4 * t + 3]));
    }
  }

  // bin of acc[4 t + kd] within this k1 class: kk = ka + 16 (4 q + t) + 256 kd
  float* out = a.out + (a.chunks == 1 ? static_cast<int64_t>(g) * N
                                      : (static_cast<int64_t>(c) * a.n_gates + g) * N);
  const bool add = (a.chunks == 1) && a.accumulate;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int kd = 0; kd < 4; ++kd) {
      const int kk = ka3 + 16 * (4 * q3 + t) + 256 * kd;
      float* dst = out + k1 + R * kk;
      *dst = add ? (*dst + acc[4 * t + kd]) : acc[4 * t + kd];
    }
  }
}

__global__ void __launch_bounds__(256)
reduce_chunks(const float* __restrict__ partial, float* __restrict__ spectra, int64_t elems,
              int32_t chunks, int32_t accumulate) {
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < elems;
       i += step) {
    float s = accumulate ? spectra[i] : 0.f;
    for (int c = 0; c < chunks; ++c) s += partial[static_cast<int64_t>(c) * elems + i];
    spectra[i] = s;
  }
}

__global__ void __launch_bounds__(256) fill_zero(float* __restrict__ dst, int64_t elems) {
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < elems;
       i += step)
    dst[i] = 0.f;
}

__device__ __forceinline__ bool peak_better(float v, int k, float bv, int bk) {
  return v > bv || (v == bv && k < bk);
}

// One workgroup per gate: (value, -bin) maximum over the band.
__global__ void __launch_bounds__(256)
peak_pick(const float* __restrict__ spectra, int32_t n_fft, int32_t lo, int32_t hi,
          int32_t* __restrict__ peak_bin, float* __restrict__ peak_power) {
  const int g = blockIdx.x;
  const float* row = spectra + static_cast<int64_t>(g) * n_fft;
  const int len = lo < hi ? hi - lo : (n_fft - lo) + hi;
  float bv = -INFINITY;
  int bk = INT_MAX;
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    int k = lo + i;
    if (k >= n_fft) k -= n_fft;
    const float v = row[k];
    if (peak_better(v, k, bv, bk)) {
      bv = v;
      bk = k;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float ov = __shfl_xor(bv, off);
    const int ok = __shfl_xor(bk, off);
    if (peak_better(ov, ok, bv, bk)) {
      bv = ov;
      bk = ok;
    }
  }
  __shared__ float sv[4];
  __shared__ int sk[4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sv[w] = bv;
    sk[w] = bk;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 4; ++i)
      if (peak_better(sv[i], sk[i], bv, bk)) {
        bv = sv[i];
        bk = sk[i];
      }
    if (bk == INT_MAX) {  // only NaN in the band
      bk = lo;
      bv = row[lo];
    }
    peak_bin[g] = bk;
    if (peak_power) peak_power[g] = bv;
  }
}

template <int RW, int ST>
hipError_t launch_fused_t(const FusedArgs& a, hipStream_t stream) {
  const int zgroups = (1 << a.log2_r) / RW;
  const int64_t blocks = static_cast<int64_t>(a.n_gates) * zgroups * a.chunks;
  hipLaunchKernelGGL((fused_spectra<RW, ST>), dim3(static_cast<unsigned>(blocks)),
                     dim3(64 * RW), 0, stream, a);
  return hipGetLastError();
}

template <int ST>
hipError_t launch_fused_st(const FusedArgs& a, hipStream_t stream) {
  switch (a.waves_per_block) {
    case 1: return launch_fused_t<1, ST>(a, stream);
    case 2: return launch_fused_t<2, ST>(a, stream);
    case 4: return launch_fused_t<4, ST>(a, stream);
    case 8: return launch_fused_t<8, ST>(a, stream);
    case 16: return launch_fused_t<16, ST>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

unsigned grid_for(int64_t elems) {
  int64_t b = (elems + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

}  // namespace

int fused_lds_bytes(int rw) {
  return static_cast<int>(sizeof(float2)) * (rw * XWAVE + (rw == 16 ? 2 : 1) * SUB);
}

hipError_t launch_fused(const FusedArgs& a, hipStream_t stream) {
  return a.sample_type == 1 ? launch_fused_st<1>(a, stream) : launch_fused_st<0>(a, stream);
}

hipError_t launch_reduce_chunks(const float* partial, float* spectra, int64_t elems,
                                int32_t chunks, int32_t accumulate, hipStream_t stream) {
  hipLaunchKernelGGL(reduce_chunks, dim3(grid_for(elems)), dim3(256), 0, stream, partial,
                     spectra, elems, chunks, accumulate);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float* dst, int64_t elems, hipStream_t stream) {
  hipLaunchKernelGGL(fill_zero, dim3(grid_for(elems)), dim3(256), 0, stream, dst, elems);
  return hipGetLastError();
}

hipError_t launch_peak(const float* spectra, int32_t n_gates, int32_t n_fft, int32_t bin_lo,
                       int32_t bin_hi, int32_t* peak_bin, float* peak_power,
                       hipStream_t stream) {
  hipLaunchKernelGGL(peak_pick, dim3(static_cast<unsigned>(n_gates)), dim3(256), 0, stream,
                     spectra, n_fft, bin_lo, bin_hi, peak_bin, peak_power);
  return hipGetLastError();
}

}  // namespace ispl
