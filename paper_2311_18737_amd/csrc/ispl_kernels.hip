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
//   pass 1  lane l holds y[l + 64 j], j < 16: pre-twiddle W_N^{64 k1 j},
//           16-point DFT over j;
//   pass 2  via an LDS transpose, lane ka + 16 r holds u_ka[r + 4 m]:
//           twiddle W_N^{(r + 4 m)(k1 + R ka)}, 16-point DFT over m;
//   pass 3  the four 16-lane rows swap values in registers
//           (v_permlane16/32_swap), then twiddle W_64^{r kc} and 4-point DFTs
//           over r give bin kk = ka + 16 kc + 256 kd.
// Every twiddle product is folded into the first butterfly layer that
// follows it (a + w b and 2 a - (a + w b) as fused multiply-adds).
// Every lane keeps the running |X|^2 of its 16 bins in registers across the
// whole pulse loop, so the only spectrum traffic is one store per bin at the
// end.  The waves of a workgroup share one gate and one pulse at a time: the
// row is decoded once into LDS and read by every wave.

#include <hip/hip_runtime.h>
#include <limits.h>

#include <algorithm>
#include <math.h>
#include <stdint.h>
#include <type_traits>
#include <utility>

#include "ispl_internal.h"

namespace ispl {
namespace {

// Per-wave exchange buffer: 16 rows of 64 complex at a pitch of 65, so that
// the pass-2 reads (16 rows, one column, per 16 lanes) hit 16 different bank
// pairs and the pass-1 writes (one row, 64 columns) are contiguous.
constexpr int XPITCH = 65;
constexpr int XWAVE = 16 * XPITCH;  // float2 of one wave's exchange buffer

// A value the compiler must keep in a VGPR: VALU instructions whose operands
// are all VGPRs (or inline constants) can dual-issue on gfx950, those reading
// an SGPR cannot.
__device__ __forceinline__ float in_vgpr(float x) {
  float r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ float2 conj_mul(float2 c, float2 x) {  // conj(c) * x
  return make_float2(fmaf(c.x, x.x, c.y * x.y), fmaf(c.x, x.y, -(c.y * x.x)));
}

// a + w b, two fused multiply-adds per component.
__device__ __forceinline__ float2 cmuladd(float2 a, float2 w, float2 b) {
  return make_float2(fmaf(w.x, b.x, fmaf(-w.y, b.y, a.x)), fmaf(w.x, b.y, fmaf(w.y, b.x, a.y)));
}

// 2 a - s: with s = a + w b this is a - w b at one FMA per component.
__device__ __forceinline__ float2 twice_minus(float2 a, float2 s) {
  return make_float2(fmaf(2.f, a.x, -s.x), fmaf(2.f, a.y, -s.y));
}

// Second layer of a 4-point forward DFT from s02 = x0 + x2, d02 = x0 - x2,
// s13 = x1 + x3, d13 = x1 - x3; outputs in natural order.
__device__ __forceinline__ void dft4_tail(float2 s02, float2 d02, float2 s13, float2 d13,
                                          float2& y0, float2& y1, float2& y2, float2& y3) {
  y0 = make_float2(s02.x + s13.x, s02.y + s13.y);
  y2 = make_float2(s02.x - s13.x, s02.y - s13.y);
  y1 = make_float2(d02.x + d13.y, d02.y - d13.x);  // d02 - i d13
  y3 = make_float2(d02.x - d13.y, d02.y + d13.x);  // d02 + i d13
}

// 4-point forward DFT in place, natural order in and out.
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 s02 = make_float2(a0.x + a2.x, a0.y + a2.y);
  const float2 d02 = make_float2(a0.x - a2.x, a0.y - a2.y);
  const float2 s13 = make_float2(a1.x + a3.x, a1.y + a3.y);
  const float2 d13 = make_float2(a1.x - a3.x, a1.y - a3.y);
  dft4_tail(s02, d02, s13, d13, a0, a1, a2, a3);
}

// DFT4 of (a0, w1 a1, w2 a2, w3 a3): the twiddle products fold into the first
// butterfly layer as multiply-adds (a + w b, then 2 a - (a + w b)).
__device__ __forceinline__ void dft4_w123(float2& a0, float2& a1, float2& a2, float2& a3,
                                          float2 w1, float2 w2, float2 w3) {
  const float2 s02 = cmuladd(a0, w2, a2);
  const float2 d02 = twice_minus(a0, s02);
  const float2 p1 = cmul(a1, w1);
  const float2 s13 = cmuladd(p1, w3, a3);
  const float2 d13 = twice_minus(p1, s13);
  dft4_tail(s02, d02, s13, d13, a0, a1, a2, a3);
}

// DFT4 of (w0 a0, w1 a1, w2 a2, w3 a3).
__device__ __forceinline__ void dft4_w0123(float2& a0, float2& a1, float2& a2, float2& a3,
                                           float2 w0, float2 w1, float2 w2, float2 w3) {
  a0 = cmul(a0, w0);
  dft4_w123(a0, a1, a2, a3, w1, w2, w3);
}

constexpr float kC8 = 0.923879532511286756f;  // cos(pi / 8)
constexpr float kS8 = 0.382683432365089772f;  // sin(pi / 8)
constexpr float kR2 = 0.707106781186547524f;  // cos(pi / 4)

// Constants of the 16-point DFT, held in VGPRs for the whole kernel.
struct Dft16Consts {
  float c8, s8, r2;
};

__device__ __forceinline__ Dft16Consts dft16_consts() {
  return Dft16Consts{in_vgpr(kC8), in_vgpr(kS8), in_vgpr(kR2)};
}

// Second stage of a 16-point DFT (j = j1 + 4 j2, k = k1 + 4 k2): after the
// DFT4s over j2, v[j1 + 4 k1] holds a[j1][k1]; twiddle W_16^{j1 k1} and DFT4
// over j1, then leave X[k] in v[k].  W_16^m = exp(-2 pi i m / 16).
__device__ __forceinline__ void dft16_stage_b(float2 (&v)[16], const Dft16Consts& k) {
  const float2 w1 = make_float2(k.c8, -k.s8), w2 = make_float2(k.r2, -k.r2);
  const float2 w3 = make_float2(k.s8, -k.c8), w9 = make_float2(-k.c8, k.s8);
  const float2 w6 = make_float2(-k.r2, -k.r2);
  dft4(v[0], v[1], v[2], v[3]);                       // k1 = 0: W^0, W^0, W^0, W^0
  dft4_w123(v[4], v[5], v[6], v[7], w1, w2, w3);      // k1 = 1: W^0, W^1, W^2, W^3
  {                                                   // k1 = 2: W^0, W^2, W^4, W^6
    const float2 a0 = v[8], a2 = v[10];
    const float2 s02 = make_float2(a0.x + a2.y, a0.y - a2.x);  // a0 + (-i) a2
    const float2 d02 = make_float2(a0.x - a2.y, a0.y + a2.x);
    const float2 p1 = make_float2(k.r2 * (v[9].x + v[9].y), k.r2 * (v[9].y - v[9].x));
    const float2 s13 = cmuladd(p1, w6, v[11]);
    const float2 d13 = twice_minus(p1, s13);
    dft4_tail(s02, d02, s13, d13, v[8], v[9], v[10], v[11]);
  }
  dft4_w123(v[12], v[13], v[14], v[15], w3, w6, w9);  // k1 = 3: W^0, W^3, W^6, W^9
  // position 4 k1 + k2 holds X[k1 + 4 k2]
  float2 t[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) t[i] = v[4 * (i & 3) + (i >> 2)];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = t[i];
}

// 16-point forward DFT of (w[j] v[j]) with w[0] = 1.
__device__ __forceinline__ void dft16_pre1(float2 (&v)[16], const float2 (&w)[16],
                                           const Dft16Consts& k) {
  dft4_w123(v[0], v[4], v[8], v[12], w[4], w[8], w[12]);
#pragma unroll
  for (int j1 = 1; j1 < 4; ++j1)
    dft4_w0123(v[j1], v[j1 + 4], v[j1 + 8], v[j1 + 12], w[j1], w[j1 + 4], w[j1 + 8], w[j1 + 12]);
  dft16_stage_b(v, k);
}

// 16-point forward DFT of v.
__device__ __forceinline__ void dft16(float2 (&v)[16], const Dft16Consts& k) {
#pragma unroll
  for (int j1 = 0; j1 < 4; ++j1) dft4(v[j1], v[j1 + 4], v[j1 + 8], v[j1 + 12]);
  dft16_stage_b(v, k);
}

// 16-point DFT of v when v[4..15] are zero: the first radix-4 stage then
// only replicates v[j1] (the 4-point DFT of (a, 0, 0, 0) is (a, a, a, a)).
__device__ __forceinline__ void dft16_first4(float2 (&v)[16], const Dft16Consts& k) {
#pragma unroll
  for (int j1 = 0; j1 < 4; ++j1) v[j1 + 4] = v[j1 + 8] = v[j1 + 12] = v[j1];
  dft16_stage_b(v, k);
}

// 16-point forward DFT of (w[j] v[j]).
__device__ __forceinline__ void dft16_pre(float2 (&v)[16], const float2 (&w)[16],
                                          const Dft16Consts& k) {
#pragma unroll
  for (int j1 = 0; j1 < 4; ++j1)
    dft4_w0123(v[j1], v[j1 + 4], v[j1 + 8], v[j1 + 12], w[j1], w[j1 + 4], w[j1 + 8], w[j1 + 12]);
  dft16_stage_b(v, k);
}

// Orders this wave's LDS accesses around a cross-lane exchange.  LDS requests
// of one wave are served in issue order, so only the compiler needs fencing.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 4 x 4 transpose between the four 16-lane rows of a wave and four registers
// (v_permlane16_swap / v_permlane32_swap): on entry register g of row r holds
// M[r][g], on exit register r of row g does.
__device__ __forceinline__ void row_transpose4(float (&m)[4]) {
  const auto s01 = __builtin_amdgcn_permlane16_swap(__float_as_uint(m[0]), __float_as_uint(m[1]),
                                                    false, false);
  const auto s23 = __builtin_amdgcn_permlane16_swap(__float_as_uint(m[2]), __float_as_uint(m[3]),
                                                    false, false);
  const auto s02 = __builtin_amdgcn_permlane32_swap(s01[0], s23[0], false, false);
  const auto s13 = __builtin_amdgcn_permlane32_swap(s01[1], s23[1], false, false);
  m[0] = __uint_as_float(s02[0]);
  m[1] = __uint_as_float(s13[0]);
  m[2] = __uint_as_float(s02[1]);
  m[3] = __uint_as_float(s13[1]);
}

template <int ST>
struct SampleIO;

// The same global-memory pointer, read from the first active lane: for
// values that are uniform over the workgroup, so that they stay in scalar
// registers and loads through them take a scalar base and a 32-bit lane offset.
// Element types are read as builtin types (complex64 as a 2-vector), since
// the class types cannot be loaded through an address-space pointer.
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <typename T>
struct Builtin {
  using type = T;
};
template <>
struct Builtin<float2> {
  using type = f32x2;
};
template <typename T>
using gptr = const __attribute__((address_space(1))) typename Builtin<T>::type*;
template <typename T>
__device__ __forceinline__ gptr<T> uniform_ptr(const T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return reinterpret_cast<gptr<T>>((static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ __forceinline__ uint32_t from_builtin(uint32_t v) { return v; }
__device__ __forceinline__ float2 from_builtin(f32x2 v) { return make_float2(v.x, v.y); }

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

// DFT4 of (a0, T a1, T^2 a2, T^3 a3), twiddles in geometric progression: with
// t02 = a0 + T^2 a2 and t13 = a1 + T^2 a3 the outputs are t02 +- T t13 and
// (a0 - T^2 a2) -+ i T (a1 - T^2 a3), so only T and T^2 are needed and every
// product folds into a multiply-add (24 operations, as for three free twiddles).
__device__ __forceinline__ void dft4_geo(float2& a0, float2& a1, float2& a2, float2& a3, float2 t,
                                         float2 t2) {
  const float2 t02 = cmuladd(a0, t2, a2);
  const float2 d02 = twice_minus(a0, t02);
  const float2 t13 = cmuladd(a1, t2, a3);
  const float2 u13 = twice_minus(a1, t13);
  a0 = cmuladd(t02, t, t13);
  a2 = twice_minus(t02, a0);
  a1 = cmuladd(d02, make_float2(t.y, -t.x), u13);  // -i T
  a3 = twice_minus(d02, a1);
}

// Twiddles of a 16-point DFT whose inputs carry the factors P^j (j < 16):
// with j = j1 + 4 j2 the first stage is a DFT4 over j2 with ratio G = P^4, the
// second a DFT4 over j1 with ratio H_k1 = P W_16^{k1}; each as (ratio, ratio^2).
struct GeoTwiddles {
  float2 g, g2;
  float2 h[4], h2[4];
};

// sum_j v[j] P^j W_16^{j k} into v[k], for the progression of `w`.
__device__ __forceinline__ void dft16_geo(float2 (&v)[16], const GeoTwiddles& w) {
#pragma unroll
  for (int j1 = 0; j1 < 4; ++j1) dft4_geo(v[j1], v[j1 + 4], v[j1 + 8], v[j1 + 12], w.g, w.g2);
  // v[j1 + 4 k1] holds the first-stage output k1 of group j1
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
    dft4_geo(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3], w.h[k1], w.h2[k1]);
  // position 4 k1 + k2 holds X[k1 + 4 k2]
  float2 t[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) t[i] = v[4 * (i & 3) + (i >> 2)];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = t[i];
}

// GeoTwiddles of the progression P = W_N^e (all from the table, so every
// factor is correctly rounded): G = W_N^{4 e}, H_k1 = W_N^{e + k1 N / 16}.
__device__ __forceinline__ void load_geo(GeoTwiddles& w, const float2* __restrict__ tw, int n_fft,
                                         int e) {
  const int nmask = n_fft - 1, n16 = n_fft >> 4;
  w.g = tw[(4 * e) & nmask];
  w.g2 = tw[(8 * e) & nmask];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    w.h[k1] = tw[(e + k1 * n16) & nmask];
    w.h2[k1] = tw[(2 * e + 2 * k1 * n16) & nmask];
  }
}

// Twiddles of one wave's 1024-point transform of bin class kappa: the wave
// produces bins kappa + S kb (S = N / 1024, kb < 1024) of the N-point
// spectrum, so its input carries the factor W_N^{kappa n} on top of the
// 1024-point DFT kernel W_N^{S kb n}.  Fixed over the pulse loop.
struct WaveTwiddles {
  float2 pre[16];    // pass 1: W_N^{64 kappa j}, the same for every lane
  float2 tw2[16];    // pass 2: W_N^{l (kappa + S ka)} for the pass-1 lane l = row + 4 m
  float2 tw3[4][3];  // pass 3: W_64^{r kc}, r = 1..3, kc = 4 row + t
};

__device__ __forceinline__ void load_wave_twiddles(WaveTwiddles& w, const float2* __restrict__ tw,
                                                   int n_fft, int kappa, int lane) {
  const int nmask = n_fft - 1, S = n_fft >> 10;
  const int ka = lane & 15, row = lane >> 4;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    w.pre[j] = tw[(64 * kappa * j) & nmask];
    w.tw2[j] = tw[((row + 4 * j) * (kappa + S * ka)) & nmask];
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 1; r < 4; ++r) w.tw3[t][r - 1] = tw[((n_fft >> 6) * r * (4 * row + t)) & nmask];
}

// The same transform with passes 2 and 3 in geometric form (36 instead of 56
// registers of per-lane twiddles; the long-code kernels need the room).  With
// q = kappa + S ka, lane (ka, r) weighs u_ka[r + 4 m] in pass 2 by
// W_N^{(r + 4 m) q} = W_N^{r q} (W_N^{4 q})^m: a progression of ratio W_N^{4 q},
// whose common factor W_N^{r q} moves into pass 3, where the 4-point DFT over r
// then weighs term r by (W_N^{q} W_64^{kc})^r = T_kc^r, T_kc = W_N^{q + 16 S kc},
// kc = 4 row + t.
struct WaveTwiddlesGeo {
  float2 pre[16];            // pass 1, as above
  GeoTwiddles p2;            // pass 2: progression W_N^{4 q}
  float2 t3[4], t3sq[4];     // pass 3: T_kc and T_kc^2
};

__device__ __forceinline__ void load_wave_twiddles(WaveTwiddlesGeo& w,
                                                   const float2* __restrict__ tw, int n_fft,
                                                   int kappa, int lane) {
  const int nmask = n_fft - 1, S = n_fft >> 10;
  const int ka = lane & 15, row = lane >> 4;
  const int q = kappa + S * ka;
#pragma unroll
  for (int j = 0; j < 16; ++j) w.pre[j] = tw[(64 * kappa * j) & nmask];
  load_geo(w.p2, tw, n_fft, 4 * q);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = q + 16 * S * (4 * row + t);
    w.t3[t] = tw[e & nmask];
    w.t3sq[t] = tw[(2 * e) & nmask];
  }
}

template <typename TW>
constexpr bool kGeo = false;
template <>
constexpr bool kGeo<WaveTwiddlesGeo> = true;

// One wave's 1024-point transform and power accumulation.  On entry lane l
// holds f[l + 64 j] in v[j]; xw is the wave's exchange buffer.  On exit
// acc[4 t + kd] += |F[kb]|^2 for kb = ka + 16 (4 row + t) + 256 kd, with
// ka = lane & 15, row = lane >> 4 (F including the bin-class factors).
// K0: the wave's bin class is 0 (N = 1024), so the pass-1 factors are all 1.
// F4 (with K0): only v[0..3] carry samples (L <= 256); v[4..15] are not read.
struct NoHook {
  __device__ void operator()() const {}
};

// `after_exchange` runs right after this wave has issued the reads of its
// pass-2 inputs: from then until the next call the exchange buffer is free.
template <bool K0 = false, bool F4 = false, typename TW = WaveTwiddles, typename Hook = NoHook>
__device__ __forceinline__ void wave_fft_accumulate(float2 (&v)[16], float2* xw, const TW& w,
                                                    const Dft16Consts& dk, float (&acc)[16],
                                                    int lane, Hook after_exchange = Hook{}) {
  const int ka = lane & 15, row = lane >> 4;
  // pass 1: pre-twiddle and 16-point DFT over the stride-64 samples of a lane
  static_assert(!F4 || K0, "four non-zero inputs only in bin class 0");
  if constexpr (F4)
    dft16_first4(v, dk);
  else if constexpr (K0)
    dft16(v, dk);
  else
    dft16_pre1(v, w.pre, dk);
#pragma unroll
  for (int k = 0; k < 16; ++k) xw[k * XPITCH + lane] = v[k];
  wave_lds_sync();

  // pass 2: lane (ka, r) twiddles u_ka[r + 4 m] and transforms over m, giving
  // the partial bins v_{ka,r}[kc]
  const int p2base = ka * XPITCH + row;
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = xw[p2base + 4 * m];
  after_exchange();
  if constexpr (kGeo<TW>)
    dft16_geo(v, w.p2);
  else
    dft16_pre(v, w.tw2, dk);

  // pass 3: the 4-point DFT over r runs across the four 16-lane rows.  For
  // each t a row transpose hands row g the four values v_{ka,r}[4 g + t],
  // r = 0..3; then twiddle W_64^{r kc}, DFT over r, |X|^2 into the sums.
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float re[4] = {v[t].x, v[4 + t].x, v[8 + t].x, v[12 + t].x};
    float im[4] = {v[t].y, v[4 + t].y, v[8 + t].y, v[12 + t].y};
    row_transpose4(re);
    row_transpose4(im);
    float2 c0 = make_float2(re[0], im[0]), c1 = make_float2(re[1], im[1]);
    float2 c2 = make_float2(re[2], im[2]), c3 = make_float2(re[3], im[3]);
    if constexpr (kGeo<TW>)
      dft4_geo(c0, c1, c2, c3, w.t3[t], w.t3sq[t]);
    else
      dft4_w123(c0, c1, c2, c3, w.tw3[t][0], w.tw3[t][1], w.tw3[t][2]);
    acc[4 * t + 0] = fmaf(c0.y, c0.y, fmaf(c0.x, c0.x, acc[4 * t + 0]));
    acc[4 * t + 1] = fmaf(c1.y, c1.y, fmaf(c1.x, c1.x, acc[4 * t + 1]));
    acc[4 * t + 2] = fmaf(c2.y, c2.y, fmaf(c2.x, c2.x, acc[4 * t + 2]));
    acc[4 * t + 3] = fmaf(c3.y, c3.y, fmaf(c3.x, c3.x, acc[4 * t + 3]));
  }
  (void)row;
}

// Workgroups are dealt to the 8 XCDs round-robin; renumber them so that each
// XCD runs a contiguous range of (gate, bin group, chunk) work items and
// neighbouring gates, whose windows overlap, share that XCD's L2.
__device__ __forceinline__ int xcd_block_id() {
  const int nblk = gridDim.x;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int per = nblk >> 3, extra = nblk & 7;
  return xcd < extra ? xcd * (per + 1) + slot : extra * (per + 1) + (xcd - extra) * per + slot;
}

// Gate of work slot `slot`: the slot itself, or the slot-th entry of a gate
// list.  Returns -1 for slots past the list's device-side count and for
// entries outside [0, n_gates), whose workgroups then do nothing.
__device__ __forceinline__ int slot_gate(const FusedArgs& a, int slot) {
  if (!a.gate_list) return slot;
  if (slot >= *a.gate_count) return -1;
  const int g = a.gate_list[slot];
  return (g >= 0 && g < a.n_gates) ? g : -1;
}

// Listed launches keep the hardware order, which deals the active (leading)
// slots round-robin over all XCDs; full launches use the XCD-contiguous order.
__device__ __forceinline__ int work_id(const FusedArgs& a) {
  return a.gate_list ? static_cast<int>(blockIdx.x) : xcd_block_id();
}

// The work item of this workgroup: gate g (-1: nothing to do), bin group zg,
// pulse chunk c of `chunks`; `slot` is the gate's position in the list and
// `rows` the rows of one chunk's partials.  Work items are numbered
// (slot, zg, c) with c fastest.  With adaptive chunking the chunk count comes
// from the device-side list length (the same rule the host sized the grid
// with), and workgroups past the work of that length return at once.
struct WorkItem {
  int g, zg, c, chunks, slot, rows;
};

__device__ __forceinline__ WorkItem work_item(const FusedArgs& a, int zgroups) {
  WorkItem w;
  int bid = work_id(a);
  if (a.adapt_target > 0) {
    const int k = min(max(*a.gate_count, 0), a.n_gates);
    w.chunks = adaptive_chunks(k, zgroups, a.adapt_target, a.adapt_max_chunks, a.adapt_rows);
    w.rows = k;
    if (bid >= k * zgroups * w.chunks) {
      w.g = -1;
      return w;
    }
  } else {
    w.chunks = a.chunks;
    w.rows = a.n_gates;
  }
  w.c = bid % w.chunks;
  bid /= w.chunks;
  w.zg = bid % zgroups;
  w.slot = bid / zgroups;
  w.g = slot_gate(a, w.slot);
  return w;
}

// Output row of a work item: the gate's row of `out` with one chunk, else
// the chunk's partial row (chunk-major [C][G][N] in `out`, or [C][k][N] by
// list slot in adapt_partial).
__device__ __forceinline__ float* out_row(const FusedArgs& a, const WorkItem& w) {
  if (w.chunks == 1) return a.out + static_cast<int64_t>(w.g) * a.n_fft;
  if (a.adapt_target > 0)
    return a.adapt_partial + (static_cast<int64_t>(w.c) * w.rows + w.slot) * a.n_fft;
  return a.out + (static_cast<int64_t>(w.c) * a.n_gates + w.g) * a.n_fft;
}

// Code lengths L <= 1024: one wave per bin class k1 (sub-transform length 1024).
// RW waves share a gate and a pulse: the decoded row is staged once in LDS.
// PF (one-wave workgroups only): fetch the next pulse during this pulse's
// transform, for launches too small to hide memory latency with other waves
// (the extra registers cost a wave per SIMD on large launches).  K0 (one-wave
// workgroups at N = 1024 only): the single bin class is 0, so pass 1 has no
// pre-twiddles.  F4 (with K0, L <= 256): each lane's samples 4..15 are zero,
// so they are neither fetched nor decoded and pass 1 starts from four inputs.
template <int RW, int ST, bool PF = false, bool K0 = false, bool F4 = false>
__global__ void __launch_bounds__(64 * RW) fused_spectra(FusedArgs a) {
  static_assert(!K0 || RW == 1, "bin class 0 alone: one-wave workgroups at N = 1024");
  static_assert(!F4 || K0, "four non-zero inputs only in bin class 0");
  constexpr int NT = 64 * RW;
  constexpr int E = SUB / NT;          // decoded samples staged per thread
  constexpr int EL = F4 ? 4 : E;       // of which can be non-zero
  constexpr bool DBUF = (RW == 16);    // double-buffer the decoded row when LDS allows
  using IO = SampleIO<ST>;
  using raw_t = typename IO::raw_t;

  __shared__ float2 xs[RW * XWAVE];
  __shared__ float2 ys[RW == 1 ? 1 : (DBUF ? 2 : 1)][RW == 1 ? 1 : SUB];  // unused for RW = 1

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int R = 1 << a.log2_r;
  const int zgroups = R / RW;
  const WorkItem w = work_item(a, zgroups);
  const int g = w.g, zg = w.zg, c = w.c;
  if (g < 0) return;  // uniform over the workgroup, before any barrier
  const int k1 = zg * RW + wave;
  const int L = a.code_len;
  const float2* __restrict__ tw = reinterpret_cast<const float2*>(a.twiddle);

  const int p0 = static_cast<int>((static_cast<int64_t>(c) * a.n_pulses) / w.chunks);
  const int p1 = static_cast<int>((static_cast<int64_t>(c + 1) * a.n_pulses) / w.chunks);

  // the geometric form where its lower register count lets eight-wave
  // workgroups keep four waves per SIMD (measured: N = 8192 16 % faster; at
  // 16, 4 and 1 waves the original form is as fast or faster)
  std::conditional_t<RW == 8, WaveTwiddlesGeo, WaveTwiddles> wt;
  load_wave_twiddles(wt, tw, a.n_fft, k1, lane);
  const Dft16Consts dk = dft16_consts();

  float acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;

  const int64_t gate_off = static_cast<int64_t>(a.first_gate) + static_cast<int64_t>(g) * a.gate_step;
  const float2* __restrict__ txb = reinterpret_cast<const float2*>(a.tx);

  raw_t raw[E];
  float2 cod[E];
  auto load = [&](int p) {
    // per-pulse row bases as workgroup-uniform values: the loads then take a
    // scalar base plus a 32-bit lane offset, and no per-lane 64-bit pointer
    // is kept live across the pulse loop
    const gptr<raw_t> srow = uniform_ptr(reinterpret_cast<const raw_t*>(a.samples) +
                                         (static_cast<int64_t>(p) * a.stride + gate_off));
    const gptr<float2> txp =
        uniform_ptr(txb + (a.tx_per_pulse ? static_cast<int64_t>(p) * L : 0));
#pragma unroll
    for (int i = 0; i < EL; ++i) {
      const int n = tid + i * NT;
      if (n < L) {
        raw[i] = from_builtin(srow[static_cast<uint32_t>(n)]);
        cod[i] = from_builtin(txp[static_cast<uint32_t>(n)]);
      } else {
        raw[i] = IO::zero();
        cod[i] = make_float2(0.f, 0.f);
      }
    }
  };

  float2* xw = xs + wave * XWAVE;
  if constexpr (RW == 1) {
    // One wave owns the gate: thread tid loads samples tid + 64 i, which are
    // exactly its pass-1 inputs, so the row needs no LDS stage and no barrier.
    if constexpr (PF) {
      // the next pulse's samples and codes are in flight during this pulse's
      // transform, so a wave alone on its SIMD does not wait once per pulse
      if (p0 < p1) load(p0);
      for (int p = p0; p < p1; ++p) {
        float2 v[16];
#pragma unroll
        for (int j = 0; j < EL; ++j) v[j] = conj_mul(cod[j], IO::cvt(raw[j]));
        if (p + 1 < p1) load(p + 1);
        wave_fft_accumulate<K0, F4>(v, xw, wt, dk, acc, lane);
      }
    } else {
      // the other waves on the SIMD hide the load latency
      for (int p = p0; p < p1; ++p) {
        load(p);
        float2 v[16];
#pragma unroll
        for (int j = 0; j < EL; ++j) v[j] = conj_mul(cod[j], IO::cvt(raw[j]));
        wave_fft_accumulate<K0, F4>(v, xw, wt, dk, acc, lane);
      }
    }
  } else {
  if (p0 < p1) load(p0);
  for (int p = p0; p < p1; ++p) {
    const int buf = DBUF ? ((p - p0) & 1) : 0;
    if (!DBUF) __syncthreads();  // every wave has read the previous row
#pragma unroll
    for (int i = 0; i < E; ++i) ys[buf][tid + i * NT] = conj_mul(cod[i], IO::cvt(raw[i]));
    if (p + 1 < p1) load(p + 1);
    __syncthreads();
    float2 v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = ys[buf][lane + 64 * j];
    wave_fft_accumulate(v, xw, wt, dk, acc, lane);
  }
  }

  // Stage the sums through LDS in bin order (bin k1 + R kb, k1 = zg RW + wave),
  // then store runs of RW consecutive bins (the whole row when one workgroup
  // owns the gate).
  __syncthreads();
  float* st = reinterpret_cast<float*>(xs);
  const int ka = lane & 15, row = lane >> 4;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int kd = 0; kd < 4; ++kd)
      st[(ka + 16 * (4 * row + t) + 256 * kd) * RW + wave] = acc[4 * t + kd];
  __syncthreads();
  float* out = out_row(a, w);
  const bool add = (w.chunks == 1) && a.accumulate;
  for (int e = tid; e < RW * SUB; e += NT) {
    float* dst = out + zg * RW + e % RW + R * (e / RW);
    *dst = add ? (*dst + st[e]) : st[e];
  }
}

// Code lengths 1024 < L <= 16384: the 16 waves of a workgroup share one
// 16384-point sub-transform (bin class k1 of N = R * 16384).  With
// n = lg + 1024 j and kk = ka + 16 kb, thread lg = tid first does the 16-point
// DFT over j (pre-twiddled by W_N^{1024 k1 j}); an all-to-all exchange through
// LDS then hands wave ka the values U_ka[lg], whose 1024-point transform, with
// the bin-class factor W_N^{lg (k1 + R ka)}, is bins k1 + R (ka + 16 kb).
// Codes of at most 2048 samples (fused_spectra_long) carry samples in j = 0, 1
// only: the first pass is X[k] = y0 + t W_16^k with t = y1 W_N^{1024 k1} (half
// of the outputs as y0 + t W_16^k, the other half as y0 - t W_16^k), and the
// two samples and codes of the next pulse are fetched during this pulse's
// work.  Longer codes take fused_spectra_long_dma.  K0: N = 16384, so the only
// bin class is k1 = 0 and the first pass has no pre-twiddles.
__device__ __forceinline__ void two_point_pass(float2 (&v)[16], float2 y0, float2 t,
                                               const Dft16Consts& k) {
  // u_m = t W_16^m for m < 8, W_16^m = exp(-2 pi i m / 16)
  float2 u[8];
  u[0] = t;
  u[1] = cmul(t, make_float2(k.c8, -k.s8));
  u[2] = make_float2(k.r2 * (t.x + t.y), k.r2 * (t.y - t.x));
  u[3] = cmul(t, make_float2(k.s8, -k.c8));
  u[4] = make_float2(t.y, -t.x);
  u[5] = cmul(t, make_float2(-k.s8, -k.c8));
  u[6] = make_float2(k.r2 * (t.y - t.x), -k.r2 * (t.x + t.y));
  u[7] = cmul(t, make_float2(-k.c8, -k.s8));
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    v[m] = make_float2(y0.x + u[m].x, y0.y + u[m].y);
    v[m + 8] = make_float2(y0.x - u[m].x, y0.y - u[m].y);
  }
}

// Writes the accumulated bins of a 16-wave sub-transform workgroup: acc[4 t + kd]
// is bin k1 + R kk with kk = wave + 16 kb, kb = ka + 16 (4 row + t) + 256 kd.
// Staged through LDS in bin order (the caller has passed a barrier after its
// last use of xs), then stored as runs of R-strided bins.
__device__ __forceinline__ void store_long_bins(const FusedArgs& a, const WorkItem& w,
                                                float2* xs, const float (&acc)[16], int tid,
                                                int k1, int R) {
  const int lane = tid & 63, wave = tid >> 6;
  float* st = reinterpret_cast<float*>(xs);
  const int ka = lane & 15, row = lane >> 4;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int kd = 0; kd < 4; ++kd)
      st[wave + 16 * (ka + 16 * (4 * row + t) + 256 * kd)] = acc[4 * t + kd];
  __syncthreads();
  float* out = out_row(a, w);
  const bool add = (w.chunks == 1) && a.accumulate;
  for (int e = tid; e < 16 * SUB; e += 1024) {
    float* dst = out + k1 + R * e;
    *dst = add ? (*dst + st[e]) : st[e];
  }
}

// Whether every code row of pulses [p0, p1) is binary (sign bits usable).
__device__ __forceinline__ bool range_binary(const FusedArgs& a, int p0, int p1) {
  if (!a.code_bits) return false;
  if (!a.tx_per_pulse) return a.code_binary[0] != 0;
  int all = 1;
  for (int p = p0; p < p1; ++p) all &= a.code_binary[p];
  return all != 0;
}

// TWO: L <= 2048 (see above).  Otherwise every pulse's 16 samples and codes
// per thread are loaded at the start of its first pass; this variant runs the
// pulse ranges whose codes are not all binary (fused_spectra_long_dma runs the
// others, from the same grid).
template <int ST, bool TWO, bool K0>
__global__ void __launch_bounds__(1024) fused_spectra_long(FusedArgs a) {
  using IO = SampleIO<ST>;
  __shared__ float2 xs[16 * XWAVE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int R = 1 << a.log2_r;  // N / 16384
  const WorkItem w = work_item(a, R);
  const int g = w.g, k1 = w.zg, c = w.c;
  if (g < 0) return;  // uniform over the workgroup, before any barrier
  const int N = a.n_fft;
  const int L = a.code_len;
  const float2* __restrict__ tw = reinterpret_cast<const float2*>(a.twiddle);

  const int p0 = static_cast<int>((static_cast<int64_t>(c) * a.n_pulses) / w.chunks);
  const int p1 = static_cast<int>((static_cast<int64_t>(c + 1) * a.n_pulses) / w.chunks);
  if (!TWO && range_binary(a, p0, p1)) return;  // the DMA variant's work item

  float2 xpre[16];  // W_N^{1024 k1 j}: same for every thread (unused with K0)
#pragma unroll
  for (int j = 0; j < 16; ++j) xpre[j] = K0 ? make_float2(1.f, 0.f) : tw[(1024 * k1 * j) & (N - 1)];
  WaveTwiddlesGeo wt;  // the form that leaves these kernels room
  load_wave_twiddles(wt, tw, N, k1 + R * wave, lane);
  const Dft16Consts dk = dft16_consts();

  float acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;

  const int64_t gate_off = static_cast<int64_t>(a.first_gate) + static_cast<int64_t>(g) * a.gate_step;
  const float2* __restrict__ txb = reinterpret_cast<const float2*>(a.tx);
  float2* xw = xs + wave * XWAVE;

  // TWO: samples and codes of slices j = 0, 1 of the next pulse
  using raw_t = typename IO::raw_t;
  raw_t nr[2] = {IO::zero(), IO::zero()};
  float2 nc[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
  auto fetch2 = [&](int p) {
    const gptr<raw_t> srow = uniform_ptr(reinterpret_cast<const raw_t*>(a.samples) +
                                         (static_cast<int64_t>(p) * a.stride + gate_off));
    const gptr<float2> txp =
        uniform_ptr(txb + (a.tx_per_pulse ? static_cast<int64_t>(p) * L : 0));
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = tid + 1024 * j;
      if (n < L) {
        nr[j] = from_builtin(srow[static_cast<uint32_t>(n)]);
        nc[j] = from_builtin(txp[static_cast<uint32_t>(n)]);
      } else {
        nr[j] = IO::zero();
        nc[j] = make_float2(0.f, 0.f);
      }
    }
  };
  if (TWO && p0 < p1) fetch2(p0);

  for (int p = p0; p < p1; ++p) {
    float2 v[16];
    if constexpr (TWO) {
      const float2 y0 = conj_mul(nc[0], IO::cvt(nr[0]));
      const float2 y1 = conj_mul(nc[1], IO::cvt(nr[1]));
      if (p + 1 < p1) fetch2(p + 1);
      two_point_pass(v, y0, K0 ? y1 : cmul(y1, xpre[1]), dk);
    } else {
      const gptr<raw_t> srow = uniform_ptr(reinterpret_cast<const raw_t*>(a.samples) +
                                           (static_cast<int64_t>(p) * a.stride + gate_off));
      const gptr<float2> txp =
          uniform_ptr(txb + (a.tx_per_pulse ? static_cast<int64_t>(p) * L : 0));
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t n = static_cast<uint32_t>(tid + 1024 * j);
        v[j] = n < static_cast<uint32_t>(L)
                   ? conj_mul(from_builtin(txp[n]), IO::cvt(from_builtin(srow[n])))
                   : make_float2(0.f, 0.f);
      }
      if constexpr (K0)
        dft16(v, dk);
      else
        dft16_pre1(v, xpre, dk);
    }
    __syncthreads();  // every wave has finished its exchanges of the previous pulse
#pragma unroll
    for (int k = 0; k < 16; ++k) xs[k * XWAVE + tid] = v[k];  // region k: U_k[lg]
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = xw[lane + 64 * j];    // U_wave[lane + 64 j]
    wave_lds_sync();  // read before this wave reuses its region for its own exchange
    wave_fft_accumulate(v, xw, wt, dk, acc, lane);
  }
  __syncthreads();
  store_long_bins(a, w, xs, acc, tid, k1, R);
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void global_void_t;

// One wave copies 4096 bytes from global memory straight into LDS: 16
// instructions of one dword per lane, at byte 256 i + 4 lane of both the
// source (g plus the lane's offset `lo` = 4 lane) and the LDS block l.
template <int... I>
__device__ __forceinline__ void wave_dma_4k(const char* g, uint32_t lo, char* l,
                                            std::integer_sequence<int, I...>) {
  (__builtin_amdgcn_global_load_lds((global_void_t*)(g + lo), (lds_void_t*)l, 4, 256 * I, 0), ...);
}

// One wave copies `bytes` (a multiple of 4, > 0) from src (uniform over the
// wave) into LDS at dst.  The data is in LDS once the wave's vector-memory
// counter has drained.
__device__ __forceinline__ void wave_copy_to_lds(const char* src, char* dst, int bytes, int lane) {
  const uint32_t lo = 4u * static_cast<uint32_t>(lane);
  int done = 0;
  for (; done + 4096 <= bytes; done += 4096) {
    // the block's base as a wave-uniform (scalar) address
    const uint64_t b = reinterpret_cast<uint64_t>(src + done);
    const uint32_t blo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b));
    const uint32_t bhi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b >> 32));
    const char* g = reinterpret_cast<const char*>((static_cast<uint64_t>(bhi) << 32) | blo);
    wave_dma_4k(g, lo, dst + done, std::make_integer_sequence<int, 16>{});
  }
  for (; done < bytes; done += 256)  // tail: only the lanes inside the range copy
    if (static_cast<uint32_t>(done) + lo < static_cast<uint32_t>(bytes))
      __builtin_amdgcn_global_load_lds((global_void_t*)(src + done + lo), (lds_void_t*)(dst + done),
                                       4, 0, 0);
}

__device__ __forceinline__ void wait_lds_ops() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void wait_vmem_ops() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Code lengths 2048 < L <= 16384 with binary codes.  Sixteen waves share one
// 16384-point sub-transform, so a workgroup fills the LDS of a compute unit
// and no other workgroup hides its memory waits: loaded at the start of each
// pulse, the pulse's samples and codes stall all sixteen waves together.  But
// each wave's exchange region is free from the moment its pass-2 inputs are
// read back until the next pulse's all-to-all exchange: wave w then copies
// samples [1024 w, 1024 w + 1024) of the next pulse's gate window straight
// into its region (LDS DMA), and after a barrier the first pass reads sample
// lg + 1024 j from region j.  The codes (+-1, as most radar codes are) come as
// one word of sign bits per thread and pulse, fetched with the samples.  Runs
// the pulse ranges whose code rows are all binary (fused_spectra_long runs the
// others, from the same grid).
template <int ST, bool K0>
__global__ void __launch_bounds__(1024) fused_spectra_long_dma(FusedArgs a) {
  using IO = SampleIO<ST>;
  using raw_t = typename IO::raw_t;
  constexpr int SB = static_cast<int>(sizeof(raw_t));
  __shared__ float2 xs[16 * XWAVE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int R = 1 << a.log2_r;  // N / 16384
  const WorkItem w = work_item(a, R);
  const int g = w.g, k1 = w.zg, c = w.c;
  if (g < 0) return;  // uniform over the workgroup, before any barrier
  const int N = a.n_fft;
  const int L = a.code_len;
  const float2* __restrict__ tw = reinterpret_cast<const float2*>(a.twiddle);

  const int p0 = static_cast<int>((static_cast<int64_t>(c) * a.n_pulses) / w.chunks);
  const int p1 = static_cast<int>((static_cast<int64_t>(c + 1) * a.n_pulses) / w.chunks);
  if (!range_binary(a, p0, p1)) return;  // fused_spectra_long's work item

  float2 xpre[16];  // W_N^{1024 k1 j}: same for every thread (unused with K0)
#pragma unroll
  for (int j = 0; j < 16; ++j) xpre[j] = K0 ? make_float2(1.f, 0.f) : tw[(1024 * k1 * j) & (N - 1)];
  WaveTwiddlesGeo wt;  // the form that leaves these kernels room
  load_wave_twiddles(wt, tw, N, k1 + R * wave, lane);
  const Dft16Consts dk = dft16_consts();

  float acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;

  const int64_t gate_off = static_cast<int64_t>(a.first_gate) + static_cast<int64_t>(g) * a.gate_step;
  float2* xw = xs + wave * XWAVE;

  // this wave's share of a pulse's gate window: samples [1024 wave, + cnt);
  // the rest of the region (all of it past the code) reads as zero samples
  const int cnt = max(0, min(SUB, L - SUB * wave));
  auto prefetch = [&](int p) {
    if (cnt > 0)
      wave_copy_to_lds(static_cast<const char*>(a.samples) +
                           (static_cast<int64_t>(p) * a.stride + gate_off + SUB * wave) * SB,
                       reinterpret_cast<char*>(xw), cnt * SB, lane);
    if (cnt < SUB) {
      raw_t* rw = reinterpret_cast<raw_t*>(xw);
      for (int e = cnt + lane; e < SUB; e += 64) rw[e] = IO::zero();
    }
  };
  // sign bits of pulse p's codes
  auto fetch_bits = [&](int p) {
    return static_cast<uint32_t>(
        a.code_bits[static_cast<int64_t>(a.tx_per_pulse ? p : 0) * CODE_BITS_WORDS + tid]);
  };
  uint32_t cbits = 0, nbits = 0;
  if (p0 < p1) {
    prefetch(p0);
    cbits = fetch_bits(p0);
  }
  wait_vmem_ops();
  __syncthreads();

  for (int p = p0; p < p1; ++p) {
    float2 v[16];
    // conj(c) x with c = +-1: the sign bit of both parts flips where c = -1
    // (past the code the bits are clear and the samples zero)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const float2 x = IO::cvt(reinterpret_cast<const raw_t*>(xs + j * XWAVE)[tid]);
      const uint32_t sgn = (cbits << (31 - j)) & 0x80000000u;
      v[j] = make_float2(__uint_as_float(__float_as_uint(x.x) ^ sgn),
                         __uint_as_float(__float_as_uint(x.y) ^ sgn));
    }
    if constexpr (K0)
      dft16(v, dk);
    else
      dft16_pre1(v, xpre, dk);
    __syncthreads();  // every thread has read the sample regions
#pragma unroll
    for (int k = 0; k < 16; ++k) xs[k * XWAVE + tid] = v[k];  // region k: U_k[lg]
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = xw[lane + 64 * j];    // U_wave[lane + 64 j]
    wave_lds_sync();  // read before this wave reuses its region for its own exchange
    const bool more = p + 1 < p1;
    wave_fft_accumulate(v, xw, wt, dk, acc, lane, [&] {
      if (more) {
        wait_lds_ops();  // the region's last reads are served before the copy lands
        prefetch(p + 1);
        nbits = fetch_bits(p + 1);
      }
    });
    cbits = nbits;
    wait_vmem_ops();  // this wave's copy has landed
    __syncthreads();  // every region holds the next pulse's samples
  }
  store_long_bins(a, w, xs, acc, tid, k1, R);
}

// Sign bits of binary codes: one workgroup of SUB threads per code row;
// thread lg packs code[lg + SUB j], j < 16, and the workgroup decides whether
// the whole row is +-1 + 0i.
__global__ void __launch_bounds__(1024)
pack_code_bits(const float2* __restrict__ tx, int32_t code_len, uint16_t* __restrict__ bits,
               int32_t* __restrict__ binary) {
  const int row = blockIdx.x, lg = threadIdx.x;
  const float2* c = tx + static_cast<int64_t>(row) * code_len;
  uint32_t word = 0;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int n = lg + SUB * j;
    if (n < code_len) {
      const float2 v = c[n];
      ok = ok && (v.x == 1.f || v.x == -1.f) && v.y == 0.f;
      word |= (v.x < 0.f ? 1u : 0u) << j;
    }
  }
  bits[static_cast<int64_t>(row) * CODE_BITS_WORDS + lg] = static_cast<uint16_t>(word);
  const int all = __syncthreads_and(ok ? 1 : 0);
  if (lg == 0) binary[row] = all ? 1 : 0;
}

// S = sum over chunks of the partial spectra (fixed order), for every gate or
// for the listed gates only (rows of the other gates are left untouched).
__global__ void __launch_bounds__(256)
reduce_chunks(const float* __restrict__ partial, float* __restrict__ spectra, int64_t elems,
              int32_t chunks, int32_t accumulate, int32_t n_fft, const int32_t* __restrict__ list,
              const int32_t* __restrict__ count) {
  const int64_t n_gates = elems / n_fft;
  int64_t active = elems;
  if (list) active = static_cast<int64_t>(min(max(*count, 0), static_cast<int32_t>(n_gates))) * n_fft;
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < active;
       i += step) {
    int64_t j = i;
    if (list) {
      const int g = list[i / n_fft];
      if (g < 0 || g >= n_gates) continue;
      j = static_cast<int64_t>(g) * n_fft + i % n_fft;
    }
    float s = accumulate ? spectra[j] : 0.f;
    for (int c = 0; c < chunks; ++c) s += partial[static_cast<int64_t>(c) * elems + j];
    spectra[j] = s;
  }
}

__global__ void __launch_bounds__(256) fill_zero(float* __restrict__ dst, int64_t elems) {
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < elems;
       i += step)
    dst[i] = 0.f;
}

// Zero the rows of the listed gates of a [n_gates][n_fft] array.
__global__ void __launch_bounds__(256)
fill_zero_rows(float* __restrict__ dst, int32_t n_gates, int32_t n_fft,
               const int32_t* __restrict__ list, const int32_t* __restrict__ count) {
  const int64_t active = static_cast<int64_t>(min(max(*count, 0), n_gates)) * n_fft;
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < active;
       i += step) {
    const int g = list[i / n_fft];
    if (g >= 0 && g < n_gates) dst[static_cast<int64_t>(g) * n_fft + i % n_fft] = 0.f;
  }
}

__device__ __forceinline__ bool peak_better(float v, int k, float bv, int bk) {
  return v > bv || (v == bv && k < bk);
}

// One workgroup per gate (per listed gate): (value, -bin) maximum over the band.
__global__ void __launch_bounds__(256)
peak_pick(const float* __restrict__ spectra, int32_t n_gates, int32_t n_fft, int32_t lo,
          int32_t hi, int32_t* __restrict__ peak_bin, float* __restrict__ peak_power,
          const int32_t* __restrict__ list, const int32_t* __restrict__ count) {
  int g = blockIdx.x;
  if (list) {
    if (g >= *count) return;
    g = list[g];
    if (g < 0 || g >= n_gates) return;
  }
  const float* row = spectra + static_cast<int64_t>(g) * n_fft;
  const int len = lo < hi ? hi - lo : (n_fft - lo) + hi;
  float bv = -INFINITY;
  int bk = INT_MAX;
  // PEAK_UNROLL loads in flight per thread before any comparison; the
  // (value, -bin) order is total, so the visiting order does not matter.
  constexpr int PEAK_UNROLL = 16;
  for (int i0 = threadIdx.x; i0 < len; i0 += PEAK_UNROLL * blockDim.x) {
    float v[PEAK_UNROLL];
    int k[PEAK_UNROLL];
#pragma unroll
    for (int u = 0; u < PEAK_UNROLL; ++u) {
      const int i = i0 + u * static_cast<int>(blockDim.x);
      k[u] = lo + i;
      if (k[u] >= n_fft) k[u] -= n_fft;
      v[u] = i < len ? row[k[u]] : -INFINITY;
      if (i >= len) k[u] = INT_MAX;  // never better than anything
    }
#pragma unroll
    for (int u = 0; u < PEAK_UNROLL; ++u)
      if (peak_better(v[u], k[u], bv, bk)) {
        bv = v[u];
        bk = k[u];
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

// Workgroups of a fused launch: every (gate, bin group, chunk) work item, or
// with adaptive chunking the most work items any list length can ask for.
int64_t fused_blocks(const FusedArgs& a, int zgroups) {
  if (a.adapt_target <= 0) return static_cast<int64_t>(a.n_gates) * zgroups * a.chunks;
  auto items = [&](int k) {
    return static_cast<int64_t>(k) * zgroups *
           adaptive_chunks(k, zgroups, a.adapt_target, a.adapt_max_chunks, a.adapt_rows);
  };
  int64_t most = items(a.n_gates);
  const int kmax = std::min(a.n_gates, a.adapt_target / zgroups + 1);
  for (int k = 1; k <= kmax; ++k) most = std::max(most, items(k));
  return most;
}

template <int RW, int ST>
hipError_t launch_fused_t(const FusedArgs& a, hipStream_t stream) {
  const int zgroups = (1 << a.log2_r) / RW;
  const int64_t blocks = fused_blocks(a, zgroups);
  // one-wave workgroups prefetch when the launch has at most two waves per SIMD
  constexpr int64_t kPrefetchMaxWaves = 2 * 4 * 256;
  if constexpr (RW == 1) {
    const bool pf = blocks <= kPrefetchMaxWaves, k0 = a.log2_r == 0;
    const bool f4 = k0 && a.code_len <= 4 * 64;  // lane samples 4..15 all past L
    const dim3 grid(static_cast<unsigned>(blocks)), block(64);
    if (pf && f4)
      hipLaunchKernelGGL((fused_spectra<1, ST, true, true, true>), grid, block, 0, stream, a);
    else if (f4)
      hipLaunchKernelGGL((fused_spectra<1, ST, false, true, true>), grid, block, 0, stream, a);
    else if (pf && k0)
      hipLaunchKernelGGL((fused_spectra<1, ST, true, true>), grid, block, 0, stream, a);
    else if (pf)
      hipLaunchKernelGGL((fused_spectra<1, ST, true, false>), grid, block, 0, stream, a);
    else if (k0)
      hipLaunchKernelGGL((fused_spectra<1, ST, false, true>), grid, block, 0, stream, a);
    else
      hipLaunchKernelGGL((fused_spectra<1, ST, false, false>), grid, block, 0, stream, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((fused_spectra<RW, ST, false>), dim3(static_cast<unsigned>(blocks)),
                     dim3(64 * RW), 0, stream, a);
  return hipGetLastError();
}

template <int ST>
hipError_t launch_fused_long_t(const FusedArgs& a, hipStream_t stream) {
  const int64_t blocks = fused_blocks(a, 1 << a.log2_r);
  const dim3 grid(static_cast<unsigned>(blocks)), block(1024);
  const bool two = a.code_len <= 2 * SUB, k0 = a.log2_r == 0;
  if (two) {
    if (k0)
      hipLaunchKernelGGL((fused_spectra_long<ST, true, true>), grid, block, 0, stream, a);
    else
      hipLaunchKernelGGL((fused_spectra_long<ST, true, false>), grid, block, 0, stream, a);
    return hipGetLastError();
  }
  // work items whose codes are all binary run in the DMA variant, the others
  // in the plain one; each workgroup of either grid decides for itself
  if (a.code_bits) {
    if (k0)
      hipLaunchKernelGGL((fused_spectra_long_dma<ST, true>), grid, block, 0, stream, a);
    else
      hipLaunchKernelGGL((fused_spectra_long_dma<ST, false>), grid, block, 0, stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (k0)
    hipLaunchKernelGGL((fused_spectra_long<ST, false, true>), grid, block, 0, stream, a);
  else
    hipLaunchKernelGGL((fused_spectra_long<ST, false, false>), grid, block, 0, stream, a);
  return hipGetLastError();
}

template <int ST>
hipError_t launch_fused_st(const FusedArgs& a, hipStream_t stream) {
  if (a.sub_len == 16 * SUB) return launch_fused_long_t<ST>(a, stream);
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

int fused_lds_bytes(int rw, int sub_len) {
  if (sub_len == 16 * SUB) return static_cast<int>(sizeof(float2)) * 16 * XWAVE;
  if (rw == 1) return static_cast<int>(sizeof(float2)) * XWAVE;  // no staged row
  return static_cast<int>(sizeof(float2)) * (rw * XWAVE + (rw == 16 ? 2 : 1) * SUB);
}

hipError_t launch_fused(const FusedArgs& a, hipStream_t stream) {
  return a.sample_type == 1 ? launch_fused_st<1>(a, stream) : launch_fused_st<0>(a, stream);
}

hipError_t launch_reduce_chunks(const float* partial, float* spectra, int64_t elems,
                                int32_t chunks, int32_t accumulate, int32_t n_fft,
                                const int32_t* list, const int32_t* count, hipStream_t stream) {
  hipLaunchKernelGGL(reduce_chunks, dim3(grid_for(elems)), dim3(256), 0, stream, partial,
                     spectra, elems, chunks, accumulate, n_fft, list, count);
  return hipGetLastError();
}

hipError_t launch_pack_code_bits(const float* tx, int32_t rows, int32_t code_len,
                                 uint16_t* bits, int32_t* binary, hipStream_t stream) {
  hipLaunchKernelGGL(pack_code_bits, dim3(static_cast<unsigned>(rows)), dim3(SUB), 0, stream,
                     reinterpret_cast<const float2*>(tx), code_len, bits, binary);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float* dst, int64_t elems, hipStream_t stream) {
  hipLaunchKernelGGL(fill_zero, dim3(grid_for(elems)), dim3(256), 0, stream, dst, elems);
  return hipGetLastError();
}

hipError_t launch_fill_zero_rows(float* dst, int32_t n_gates, int32_t n_fft, const int32_t* list,
                                 const int32_t* count, hipStream_t stream) {
  hipLaunchKernelGGL(fill_zero_rows, dim3(grid_for(static_cast<int64_t>(n_gates) * n_fft)),
                     dim3(256), 0, stream, dst, n_gates, n_fft, list, count);
  return hipGetLastError();
}

hipError_t launch_peak(const float* spectra, int32_t n_gates, int32_t n_fft, int32_t bin_lo,
                       int32_t bin_hi, int32_t* peak_bin, float* peak_power,
                       const int32_t* list, const int32_t* count, hipStream_t stream) {
  hipLaunchKernelGGL(peak_pick, dim3(static_cast<unsigned>(n_gates)), dim3(256), 0, stream,
                     spectra, n_gates, n_fft, bin_lo, bin_hi, peak_bin, peak_power, list, count);
  return hipGetLastError();
}

}  // namespace ispl
