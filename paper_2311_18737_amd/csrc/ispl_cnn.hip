// Window-proposal network of the learned zoom: training kernels (FP32 on
// the vector ALUs).
//
// The network maps one gate's coarse spectrum feature
// x[t] = log(max(S[t] / mean S, 1e-30)), t < T = 1024, to one logit per coarse bin through four circular 7-tap 1-D
// convolutions, 1 -> 32 -> 32 -> 32 -> 1 channels with ReLU after the first
// three.  Training minimises the softmax cross entropy against a two-hot
// target at the line's coarse position u (1 - frac(u) on floor(u), frac(u)
// on floor(u) + 1, modulo T).  One workgroup handles one gate; per-gate
// weight gradients are summed over the batch in a fixed order (no atomics),
// so a training step is bit-reproducible.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ispl_internal.h"

namespace ispl {
namespace {

constexpr int T = NET_LEN;      // 1024 positions
constexpr int TAPS = 7;
constexpr int PAD = 3;
constexpr int NT = 256;         // threads: four consecutive positions each
static_assert(T == 4 * NT, "one thread per four positions");

__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }

// The 10 values v[(4 j - 3 + i) mod T], i < 10, of row `row` (length T, in LDS).
__device__ __forceinline__ void window10(const float* row, int j, float (&w)[10]) {
  const float4 l = ld4(row + ((4 * j - 4) & (T - 1)));
  const float4 m = ld4(row + 4 * j);
  const float4 r = ld4(row + ((4 * j + 4) & (T - 1)));
  w[0] = l.y; w[1] = l.z; w[2] = l.w;
  w[3] = m.x; w[4] = m.y; w[5] = m.z; w[6] = m.w;
  w[7] = r.x; w[8] = r.y; w[9] = r.z;
}

// z[co][t] = b[co] + sum_{ci,k} W[co][ci][k] a[ci][(t + k - 3) mod T]; out = relu(z) or z.
template <int CIN, int COUT, bool RELU>
__global__ void __launch_bounds__(NT) conv_fwd(const float* __restrict__ in,
                                               const float* __restrict__ params, int w_off,
                                               float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) float a_s[CIN][T];
  const int b = blockIdx.x, j = threadIdx.x;
  const float* src = in + static_cast<int64_t>(b) * CIN * T;
  for (int i = j; i < CIN * T / 4; i += NT)
    reinterpret_cast<float4*>(&a_s[0][0])[i] = reinterpret_cast<const float4*>(src)[i];
  __syncthreads();
  const float* W = params + w_off;
  const float* bias = W + COUT * CIN * TAPS;
  float* dst = out + static_cast<int64_t>(b) * COUT * T;
  for (int co = 0; co < COUT; ++co) {
    float acc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[m] = bias[co];
    for (int ci = 0; ci < CIN; ++ci) {
      float w[10];
      window10(a_s[ci], j, w);
      const float* wk = W + (co * CIN + ci) * TAPS;
#pragma unroll
      for (int k = 0; k < TAPS; ++k)
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[m] = fmaf(wk[k], w[m + k], acc[m]);
    }
    float4 o;
    o.x = RELU ? fmaxf(acc[0], 0.f) : acc[0];
    o.y = RELU ? fmaxf(acc[1], 0.f) : acc[1];
    o.z = RELU ? fmaxf(acc[2], 0.f) : acc[2];
    o.w = RELU ? fmaxf(acc[3], 0.f) : acc[3];
    *reinterpret_cast<float4*>(dst + co * T + 4 * j) = o;
  }
}

// Data gradient: da[ci][t] = sum_{co,k} W[co][ci][k] dz[co][(t - k + 3) mod T],
// returned as the pre-activation gradient dz_in = da * (a_in > 0).
template <int CIN, int COUT>
__global__ void __launch_bounds__(NT) conv_bwd_data(const float* __restrict__ dz,
                                                    const float* __restrict__ params, int w_off,
                                                    const float* __restrict__ a_in,
                                                    float* __restrict__ dz_in) {
  __shared__ __attribute__((aligned(16))) float d_s[COUT][T];
  const int b = blockIdx.x, j = threadIdx.x;
  const float* src = dz + static_cast<int64_t>(b) * COUT * T;
  for (int i = j; i < COUT * T / 4; i += NT)
    reinterpret_cast<float4*>(&d_s[0][0])[i] = reinterpret_cast<const float4*>(src)[i];
  __syncthreads();
  const float* W = params + w_off;
  const float* mask = a_in + static_cast<int64_t>(b) * CIN * T;
  float* dst = dz_in + static_cast<int64_t>(b) * CIN * T;
  for (int ci = 0; ci < CIN; ++ci) {
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int co = 0; co < COUT; ++co) {
      float w[10];  // w[i] = dz[co][4 j - 3 + i]
      window10(d_s[co], j, w);
      const float* wk = W + (co * CIN + ci) * TAPS;
      // t = 4 j + m needs dz[t - k + 3] = w[m - k + 6]
#pragma unroll
      for (int k = 0; k < TAPS; ++k)
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[m] = fmaf(wk[k], w[m - k + 6], acc[m]);
    }
    const float4 a = ld4(mask + ci * T + 4 * j);
    float4 o;
    o.x = a.x > 0.f ? acc[0] : 0.f;
    o.y = a.y > 0.f ? acc[1] : 0.f;
    o.z = a.z > 0.f ? acc[2] : 0.f;
    o.w = a.w > 0.f ? acc[3] : 0.f;
    *reinterpret_cast<float4*>(dst + ci * T + 4 * j) = o;
  }
}

// Weight gradient of one gate: dW[co][ci][k] = sum_t dz[co][t] a[ci][(t + k - 3) mod T],
// db[co] = sum_t dz[co][t], written to that gate's row of the partial buffer
// (layer segment at w_off, flat parameter order).  Positions are swept in
// chunks of 256 staged in LDS; each thread owns fixed (co, ci) pairs.
constexpr int WCH = 256;
constexpr int APITCH = WCH + 7;  // 263: odd pitch spreads the 32 rows over the banks

template <int CIN, int COUT>
__global__ void __launch_bounds__(NT) conv_bwd_weight(const float* __restrict__ dz,
                                                      const float* __restrict__ a_in,
                                                      int w_off, int n_params,
                                                      float* __restrict__ part) {
  constexpr int PAIRS = CIN * COUT;
  constexpr int PER = (PAIRS + NT - 1) / NT;
  __shared__ float d_s[COUT][WCH];
  __shared__ float a_s[CIN][APITCH];
  const int b = blockIdx.x, tid = threadIdx.x;
  const float* dzb = dz + static_cast<int64_t>(b) * COUT * T;
  const float* ab = a_in + static_cast<int64_t>(b) * CIN * T;
  float acc[PER][TAPS];
  float bacc = 0.f;
#pragma unroll
  for (int q = 0; q < PER; ++q)
#pragma unroll
    for (int k = 0; k < TAPS; ++k) acc[q][k] = 0.f;

  for (int t0 = 0; t0 < T; t0 += WCH) {
    __syncthreads();
    for (int i = tid; i < COUT * WCH; i += NT) d_s[i / WCH][i % WCH] = dzb[(i / WCH) * T + t0 + i % WCH];
    for (int i = tid; i < CIN * (WCH + 6); i += NT) {
      const int ci = i / (WCH + 6), tt = i % (WCH + 6);
      a_s[ci][tt] = ab[ci * T + ((t0 + tt - PAD) & (T - 1))];  // a[ci][t0 + tt - 3]
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int pr = tid + NT * q;
      if (pr < PAIRS) {
        const int co = pr / CIN, ci = pr % CIN;
        for (int tt = 0; tt < WCH; ++tt) {
          const float d = d_s[co][tt];
#pragma unroll
          for (int k = 0; k < TAPS; ++k) acc[q][k] = fmaf(d, a_s[ci][tt + k], acc[q][k]);
        }
      }
    }
    if (tid < COUT)
      for (int tt = 0; tt < WCH; ++tt) bacc += d_s[tid][tt];
  }
  float* out = part + static_cast<int64_t>(b) * n_params + w_off;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int pr = tid + NT * q;
    if (pr < PAIRS)
#pragma unroll
      for (int k = 0; k < TAPS; ++k) out[pr * TAPS + k] = acc[q][k];
  }
  if (tid < COUT) out[PAIRS * TAPS + tid] = bacc;
}

// Fixed-order block reduction helpers (256 threads).
__device__ float block_sum(float v, float* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}
__device__ float block_max(float v, float* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// Softmax cross entropy against the two-hot target at coarse position u[b];
// dlogits = softmax - target, loss[b].
__global__ void __launch_bounds__(NT) softmax_ce(const float* __restrict__ logits,
                                                 const float* __restrict__ target_pos,
                                                 float* __restrict__ dlogits,
                                                 float* __restrict__ loss) {
  __shared__ float red[4];
  const int b = blockIdx.x, j = threadIdx.x;
  const float4 z = ld4(logits + static_cast<int64_t>(b) * T + 4 * j);
  const float mx = block_max(fmaxf(fmaxf(z.x, z.y), fmaxf(z.z, z.w)), red);
  const float e0 = expf(z.x - mx), e1 = expf(z.y - mx), e2 = expf(z.z - mx), e3 = expf(z.w - mx);
  const float sum = block_sum((e0 + e1) + (e2 + e3), red);
  const float u = target_pos[b];
  const float fl = floorf(u);
  const float f = u - fl;
  const int lo = static_cast<int>(fl) & (T - 1), hi = (lo + 1) & (T - 1);
  const float inv = 1.f / sum;
  float e[4] = {e0, e1, e2, e3};
  float4 d;
  float* dp = &d.x;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int t = 4 * j + m;
    const float tgt = (t == lo ? 1.f - f : 0.f) + (t == hi ? f : 0.f);
    dp[m] = e[m] * inv - tgt;
  }
  *reinterpret_cast<float4*>(dlogits + static_cast<int64_t>(b) * T + 4 * j) = d;
  if (j == 0) {
    const float lse = mx + logf(sum);  // -log p[t] = lse - z[t]
    const float zlo = logits[static_cast<int64_t>(b) * T + lo];
    const float zhi = logits[static_cast<int64_t>(b) * T + hi];
    loss[b] = (1.f - f) * (lse - zlo) + f * (lse - zhi);
  }
}

// grad[i] = (1 / B) sum_b part[b][i] in increasing b; loss_mean likewise.
__global__ void __launch_bounds__(256) mean_rows(const float* __restrict__ part, int rows,
                                                 int cols, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += part[static_cast<int64_t>(r) * cols + i];
  out[i] = s / static_cast<float>(rows);
}

__global__ void __launch_bounds__(256) adam_update(float* __restrict__ params,
                                                   const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int n, float lr, float beta1, float beta2,
                                                   float eps, float corr1, float corr2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mi = beta1 * m[i] + (1.f - beta1) * g;
  const float vi = beta2 * v[i] + (1.f - beta2) * g * g;
  m[i] = mi;
  v[i] = vi;
  params[i] -= lr * (mi / corr1) / (sqrtf(vi / corr2) + eps);
}

// x[t] = log(max(S[t] / mean S, 1e-30)) per row.
__global__ void __launch_bounds__(NT) log_features(const float* __restrict__ spectra,
                                                   float* __restrict__ out) {
  __shared__ float red[4];
  const int b = blockIdx.x, j = threadIdx.x;
  const float4 s = ld4(spectra + static_cast<int64_t>(b) * T + 4 * j);
  const float mean = block_sum((s.x + s.y) + (s.z + s.w), red) / static_cast<float>(T);
  const float inv = 1.f / mean;
  float4 o;
  o.x = logf(fmaxf(s.x * inv, 1e-30f));
  o.y = logf(fmaxf(s.y * inv, 1e-30f));
  o.z = logf(fmaxf(s.z * inv, 1e-30f));
  o.w = logf(fmaxf(s.w * inv, 1e-30f));
  *reinterpret_cast<float4*>(out + static_cast<int64_t>(b) * T + 4 * j) = o;
}

}  // namespace

// Parameter layout (floats): W1[32][1][7] b1[32] W2[32][32][7] b2[32]
// W3[32][32][7] b3[32] W4[1][32][7] b4[1].
constexpr int L1_OFF = 0, L2_OFF = 256, L3_OFF = 7456, L4_OFF = 14656;
static_assert(L4_OFF + 225 == NET_PARAMS, "parameter layout");

hipError_t launch_net_features(const float* spectra, int rows, float* out, hipStream_t s) {
  hipLaunchKernelGGL(log_features, dim3(rows), dim3(NT), 0, s, spectra, out);
  return hipGetLastError();
}

hipError_t launch_net_forward_f32(const NetWork& w, const float* x, int batch, float* logits,
                                  hipStream_t s) {
  hipLaunchKernelGGL((conv_fwd<1, 32, true>), dim3(batch), dim3(NT), 0, s, x, w.params, L1_OFF, w.a1);
  hipLaunchKernelGGL((conv_fwd<32, 32, true>), dim3(batch), dim3(NT), 0, s, w.a1, w.params, L2_OFF, w.a2);
  hipLaunchKernelGGL((conv_fwd<32, 32, true>), dim3(batch), dim3(NT), 0, s, w.a2, w.params, L3_OFF, w.a3);
  hipLaunchKernelGGL((conv_fwd<32, 1, false>), dim3(batch), dim3(NT), 0, s, w.a3, w.params, L4_OFF, logits);
  return hipGetLastError();
}

hipError_t launch_net_loss_grad(const NetWork& w, const float* x, const float* target_pos,
                                int batch, float* grad, float* loss_mean, hipStream_t s) {
  hipError_t e = launch_net_forward_f32(w, x, batch, w.logits, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(softmax_ce, dim3(batch), dim3(NT), 0, s, w.logits, target_pos, w.dz4, w.loss);
  // layer 4 (32 -> 1), then 3, 2, 1
  hipLaunchKernelGGL((conv_bwd_weight<32, 1>), dim3(batch), dim3(NT), 0, s, w.dz4, w.a3, L4_OFF, NET_PARAMS, w.part);
  hipLaunchKernelGGL((conv_bwd_data<32, 1>), dim3(batch), dim3(NT), 0, s, w.dz4, w.params, L4_OFF, w.a3, w.dzA);
  hipLaunchKernelGGL((conv_bwd_weight<32, 32>), dim3(batch), dim3(NT), 0, s, w.dzA, w.a2, L3_OFF, NET_PARAMS, w.part);
  hipLaunchKernelGGL((conv_bwd_data<32, 32>), dim3(batch), dim3(NT), 0, s, w.dzA, w.params, L3_OFF, w.a2, w.dzB);
  hipLaunchKernelGGL((conv_bwd_weight<32, 32>), dim3(batch), dim3(NT), 0, s, w.dzB, w.a1, L2_OFF, NET_PARAMS, w.part);
  hipLaunchKernelGGL((conv_bwd_data<32, 32>), dim3(batch), dim3(NT), 0, s, w.dzB, w.params, L2_OFF, w.a1, w.dzA);
  hipLaunchKernelGGL((conv_bwd_weight<1, 32>), dim3(batch), dim3(NT), 0, s, w.dzA, x, L1_OFF, NET_PARAMS, w.part);
  hipLaunchKernelGGL(mean_rows, dim3((NET_PARAMS + 255) / 256), dim3(256), 0, s, w.part, batch, NET_PARAMS, grad);
  hipLaunchKernelGGL(mean_rows, dim3(1), dim3(256), 0, s, w.loss, batch, 1, loss_mean);
  return hipGetLastError();
}

hipError_t launch_adam(float* params, const float* grad, float* m, float* v, int n, float lr,
                       int step, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, static_cast<float>(step));
  const float c2 = 1.f - powf(b2, static_cast<float>(step));
  hipLaunchKernelGGL(adam_update, dim3((n + 255) / 256), dim3(256), 0, s, params, grad, m, v, n,
                     lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

}  // namespace ispl

// ---------------------------------------------------------------------------
// Inference on the matrix cores: BF16 weights and activations, FP32
// accumulation.  One workgroup (4 waves) per gate keeps the whole gate in
// LDS: the input row, and two [T][32] BF16 activation buffers used in turn.
// Layers 1-3 are GEMMs D[co][t] = sum_k A[co][k] B[k][t] on
// v_mfma_f32_32x32x16_bf16: layer 1 with k = tap (7 of 16 used), layers 2 and
// 3 with k = 32 tap + ci (14 k-steps); each wave holds its A fragments in
// registers for the whole layer and sweeps eight 32-position tiles.  Layer 4
// (one output channel) runs on the vector ALUs.  Activation rows are 64 bytes
// (32 channels); the four 16-byte channel groups of row t are stored at group
// position g ^ ((t >> 1) & 3), which puts the eight 16-byte accesses of
// consecutive rows that one LDS cycle serves on distinct banks.

namespace ispl {
namespace {

typedef __bf16 nbf16x8 __attribute__((ext_vector_type(8)));
typedef float nf32x16 __attribute__((ext_vector_type(16)));

struct alignas(16) Frag8 {
  uint32_t w[4];
};

__device__ __forceinline__ uint32_t to_bf16(float x) {  // round to nearest even
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float from_bf16(uint32_t h) { return __uint_as_float(h << 16); }

// 2-byte index of channel ci of row t in a swizzled [T][32] activation buffer
__device__ __forceinline__ int act_idx(int t, int ci) {
  return t * 32 + 8 * ((ci >> 3) ^ ((t >> 1) & 3)) + (ci & 7);
}

// Weight tables of the matrix-core layers.  w1[ln]: layer 1's A fragment,
// W1[co = ln % 32][k = 8 (ln / 32) + i] for k < 7, zero above.  w2, w3 [ks][ln]:
// the 8 BF16 values W[co = ln % 32][ci][kk] with k = 16 ks + 8 (ln / 32) + i,
// kk = k / 32, ci = k % 32.  w4: BF16-rounded W4[ci][kk] as floats.  Biases FP32.
struct NetBf16 {
  Frag8 w1[64];
  Frag8 w2[14][64];
  Frag8 w3[14][64];
  float w4[32 * 7];
  float b1[32], b2[32], b3[32], b4;
};

__global__ void __launch_bounds__(256) prep_bf16(const float* __restrict__ p, NetBf16* out) {
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * 14 * 64; e += 256) {
    const int layer = e / (14 * 64), ks = (e / 64) % 14, ln = e % 64;
    const float* W = p + (layer == 0 ? 256 : 7456);
    Frag8 f;
    for (int i = 0; i < 8; i += 2) {
      uint32_t half[2];
      for (int u = 0; u < 2; ++u) {
        const int k = 16 * ks + 8 * (ln / 32) + i + u, kk = k / 32, ci = k % 32, co = ln % 32;
        half[u] = to_bf16(W[(co * 32 + ci) * 7 + kk]);
      }
      f.w[i / 2] = half[0] | (half[1] << 16);
    }
    (layer == 0 ? out->w2 : out->w3)[ks][ln] = f;
  }
  if (tid < 64) {
    Frag8 f;
    for (int i = 0; i < 8; i += 2) {
      uint32_t half[2];
      for (int u = 0; u < 2; ++u) {
        const int k = 8 * (tid / 32) + i + u, co = tid % 32;
        half[u] = k < 7 ? to_bf16(p[co * 7 + k]) : 0u;
      }
      f.w[i / 2] = half[0] | (half[1] << 16);
    }
    out->w1[tid] = f;
  }
  for (int e = tid; e < 224; e += 256) out->w4[e] = from_bf16(to_bf16(p[14656 + e]));
  if (tid < 32) {
    out->b1[tid] = p[224 + tid];
    out->b2[tid] = p[7424 + tid];
    out->b3[tid] = p[14624 + tid];
  }
  if (tid == 0) out->b4 = p[14880];
}

// The 16 biases of this lane's accumulator rows: bv[r] = bias[co(r)] with
// co(r) = (r % 4) + 8 (r / 4) + 4 h (h = lane / 32), loaded once per layer.
__device__ __forceinline__ void load_bias(const float* bias, int h, float (&bv)[16]) {
#pragma unroll
  for (int r = 0; r < 16; ++r) bv[r] = bias[(r & 3) + 8 * (r >> 2) + 4 * h];
}

// bias + ReLU of one 32 x 32 accumulator tile (D[co][t], t = this lane's
// column), rounded to BF16 and stored as four 8-byte groups.
__device__ __forceinline__ void store_tile(const nf32x16& acc, const float (&bv)[16], int h, int t,
                                           uint16_t* dst) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int co = 8 * q + 4 * h;
    const uint32_t v01 = to_bf16(fmaxf(acc[4 * q + 0] + bv[4 * q + 0], 0.f)) |
                         (to_bf16(fmaxf(acc[4 * q + 1] + bv[4 * q + 1], 0.f)) << 16);
    const uint32_t v23 = to_bf16(fmaxf(acc[4 * q + 2] + bv[4 * q + 2], 0.f)) |
                         (to_bf16(fmaxf(acc[4 * q + 3] + bv[4 * q + 3], 0.f)) << 16);
    *reinterpret_cast<uint2*>(dst + act_idx(t, co)) = make_uint2(v01, v23);
  }
}

// Forward workgroup: FW_WAVES waves, each owning FW_SPAN consecutive positions
// of the matrix-core layers.  The input stage (features) runs on the first
// FW_IN_THREADS threads, two positions each, whatever FW_WAVES is, so its
// reduction order (and hence every result) does not depend on the tiling.
constexpr int FW_WAVES = 16;
constexpr int FW_THREADS = 64 * FW_WAVES;
constexpr int FW_SPAN = T / FW_WAVES;   // 64 positions per wave
constexpr int FW_PAIRS = FW_SPAN / 64;  // pairs of 32-position tiles per wave
constexpr int FW_PER_THREAD = T / FW_THREADS;
constexpr int FW_IN_THREADS = T / 2;
constexpr int FW_IN_WAVES = FW_IN_THREADS / 64;
static_assert(FW_SPAN % 64 == 0 && T % FW_THREADS == 0, "forward tiling");

// One 32-channel layer: each wave sweeps its positions as pairs of
// 32-position tiles; the two tiles' accumulation chains are interleaved and
// the B fragments of the next k-step are read from LDS one step ahead, so
// neither the matrix-core latency nor the LDS latency stalls a lone wave.
__device__ __forceinline__ void mfma_layer(const uint16_t* __restrict__ src, uint16_t* __restrict__ dst,
                                           const Frag8 (*__restrict__ wt)[64], const float* bias,
                                           int wave, int lane) {
  const int h = lane >> 5, c = lane & 31;
  Frag8 afr[14];
#pragma unroll
  for (int ks = 0; ks < 14; ++ks) afr[ks] = wt[ks][lane];
  float bv[16];
  load_bias(bias, h, bv);
  auto bfrag = [&](int t, int ks) {
    const int kk = ks >> 1, ci0 = 16 * (ks & 1) + 8 * h;
    const int row = (t + kk - PAD) & (T - 1);
    return *reinterpret_cast<const Frag8*>(src + act_idx(row, ci0));
  };
  for (int pair = 0; pair < FW_PAIRS; ++pair) {
    const int t0 = FW_SPAN * wave + 64 * pair + c, t1 = t0 + 32;  // this lane's two columns
    nf32x16 acc0, acc1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      acc0[r] = 0.f;
      acc1[r] = 0.f;
    }
    Frag8 b0 = bfrag(t0, 0), b1 = bfrag(t1, 0);
#pragma unroll
    for (int ks = 0; ks < 14; ++ks) {
      Frag8 n0 = b0, n1 = b1;
      if (ks + 1 < 14) {
        n0 = bfrag(t0, ks + 1);
        n1 = bfrag(t1, ks + 1);
      }
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(nbf16x8, afr[ks]),
                                                     __builtin_bit_cast(nbf16x8, b0), acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(nbf16x8, afr[ks]),
                                                     __builtin_bit_cast(nbf16x8, b1), acc1, 0, 0, 0);
      b0 = n0;
      b1 = n1;
    }
    store_tile(acc0, bv, h, t0, dst);
    store_tile(acc1, bv, h, t1, dst);
  }
}

// FROM_SPECTRA: the input rows are coarse spectra and the features
// log(max(S / mean S, 1e-30)) are formed here (as log_features does).  With
// chunks > 1 the spectra are still split over pulse chunks ([chunks][batch][T]
// partials): each row is summed in ascending chunk order, as the separate
// chunk reduction does, and written to x_out before use.
template <bool FROM_SPECTRA>
__global__ void __launch_bounds__(FW_THREADS) net_forward_bf16(const float* __restrict__ x,
                                                               const NetBf16* __restrict__ nw,
                                                               float* __restrict__ logits,
                                                               const float* __restrict__ partial,
                                                               int32_t chunks,
                                                               float* __restrict__ x_out) {
  __shared__ __attribute__((aligned(16))) float xs[T];
  __shared__ __attribute__((aligned(16))) uint16_t act0[T * 32];
  __shared__ __attribute__((aligned(16))) uint16_t act1[T * 32];
  __shared__ float red[FW_IN_WAVES];
  __shared__ float w4s[32 * TAPS];  // layer-4 weights, read by every lane
  const int g = blockIdx.x, j = threadIdx.x, lane = j & 63;
  const int wave = __builtin_amdgcn_readfirstlane(j >> 6);
  const int h = lane >> 5, c = lane & 31;
  if (j < 32 * TAPS) w4s[j] = nw->w4[j];
  // input stage: thread j < FW_IN_THREADS holds positions 2 j, 2 j + 1
  const bool in = j < FW_IN_THREADS;  // whole waves
  float2 v = make_float2(0.f, 0.f);
  if (!in) {
  } else if (FROM_SPECTRA && chunks > 1) {
    const int64_t cs = static_cast<int64_t>(gridDim.x) * T;
    const float2* pr = reinterpret_cast<const float2*>(partial + static_cast<int64_t>(g) * T) + j;
    v = make_float2(0.f, 0.f);
    // eight loads in flight, then the sums in ascending chunk order
    for (int c0 = 0; c0 < chunks; c0 += 8) {
      float2 q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        q[u] = c0 + u < chunks ? pr[(c0 + u) * (cs / 2)] : make_float2(0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c0 + u < chunks) {
          v.x += q[u].x;
          v.y += q[u].y;
        }
    }
    reinterpret_cast<float2*>(x_out + static_cast<int64_t>(g) * T)[j] = v;
  } else {
    v = reinterpret_cast<const float2*>(x + static_cast<int64_t>(g) * T)[j];
  }
  if (FROM_SPECTRA) {
    if (in) {
      float sum = v.x + v.y;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
      if (lane == 0) red[wave] = sum;
    }
    __syncthreads();
    float tot = 0.f;
#pragma unroll
    for (int w = 0; w < FW_IN_WAVES; ++w) tot += red[w];  // fixed order
    const float inv = 1.f / (tot / static_cast<float>(T));
    v = make_float2(logf(fmaxf(v.x * inv, 1e-30f)), logf(fmaxf(v.y * inv, 1e-30f)));
  }
  if (in) reinterpret_cast<float2*>(xs)[j] = v;
  __syncthreads();
  // layer 1: one k-step, B[k][t] = bf16(x[t + k - 3]) for k < 7 (lanes h = 1 hold k >= 8: zero)
  {
    const Frag8 a1 = nw->w1[lane];
    float bv[16];
    load_bias(nw->b1, h, bv);
    for (int tile = 0; tile < FW_SPAN / 32; ++tile) {
      const int t = FW_SPAN * wave + 32 * tile + c;
      Frag8 bfr;
#pragma unroll
      for (int i = 0; i < 8; i += 2) {
        uint32_t lo = 0, hi = 0;
        if (h == 0) {
          lo = to_bf16(xs[(t + i - PAD) & (T - 1)]);
          if (i + 1 < TAPS) hi = to_bf16(xs[(t + i + 1 - PAD) & (T - 1)]);
        }
        bfr.w[i / 2] = lo | (hi << 16);
      }
      nf32x16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.f;
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(nbf16x8, a1),
                                                    __builtin_bit_cast(nbf16x8, bfr), acc, 0, 0, 0);
      store_tile(acc, bv, h, t, act0);
    }
  }
  __syncthreads();
  mfma_layer(act0, act1, nw->w2, nw->b2, wave, lane);
  __syncthreads();
  mfma_layer(act1, act0, nw->w3, nw->b3, wave, lane);
  __syncthreads();
  // layer 4: thread j computes positions t = j + FW_THREADS m (consecutive lanes
  // read consecutive rows: conflict-free 16-byte LDS reads)
  float* out = logits + static_cast<int64_t>(g) * T;
  float acc[FW_PER_THREAD];
#pragma unroll
  for (int m = 0; m < FW_PER_THREAD; ++m) acc[m] = nw->b4;
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int kk = 0; kk < TAPS; ++kk) {
      float w[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) w[i] = w4s[(8 * q + i) * TAPS + kk];
#pragma unroll
      for (int m = 0; m < FW_PER_THREAD; ++m) {
        const int row = (j + FW_THREADS * m + kk - PAD) & (T - 1);
        const uint4 u4 = *reinterpret_cast<const uint4*>(act0 + act_idx(row, 8 * q));
        const uint32_t u[4] = {u4.x, u4.y, u4.z, u4.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          acc[m] = fmaf(w[2 * i], __uint_as_float(u[i] << 16), acc[m]);
          acc[m] = fmaf(w[2 * i + 1], __uint_as_float(u[i] & 0xffff0000u), acc[m]);
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < FW_PER_THREAD; ++m) out[j + FW_THREADS * m] = acc[m];
}

// Forward split over S workgroups per gate, for batches too small to fill the
// chip with one workgroup per gate.  Part q owns the W = T / S output
// positions [a, a + W), a = q W, and computes layers 1..3 on the 32-aligned
// range [a - 32, a + W + 32) (W / 32 + 2 tiles, two per wave), enough for the
// 3-position halo that each later 7-tap layer consumes; the edge tiles read
// zero margin rows and are not used.  Every output takes the same operations
// in the same order as in net_forward_bf16 (the input stage reproduces its
// reduction tree over the whole row), so the logits are bit-identical.
template <int S>
struct SplitGeo {
  static constexpr int W = T / S;            // output positions per part
  static constexpr int NL = W + 64;          // computed positions per layer
  static constexpr int WAVES = NL / 64;      // matrix-layer waves: two 32-position tiles each
  // at least one wave per input-stage wave, so the row sum takes one pass
  static constexpr int THREADS = 64 * (WAVES > FW_IN_WAVES ? WAVES : FW_IN_WAVES);
  static constexpr int ROWS = NL + 2 * PAD;  // local rows: PAD zero margins each side
  static_assert(W % 64 == 0 && THREADS >= W, "split tiling");
};

// One 32-channel layer over the local rows (row u + PAD holds position
// a - 32 + u); same per-output arithmetic as mfma_layer.
template <int S>
__device__ __forceinline__ void mfma_layer_split(const uint16_t* __restrict__ src,
                                                 uint16_t* __restrict__ dst,
                                                 const Frag8 (*__restrict__ wt)[64],
                                                 const float* bias, int wave, int lane) {
  const int h = lane >> 5, c = lane & 31;
  Frag8 afr[14];
#pragma unroll
  for (int ks = 0; ks < 14; ++ks) afr[ks] = wt[ks][lane];
  float bv[16];
  load_bias(bias, h, bv);
  // all weight loads in flight before the first multiply (left to itself the
  // scheduler spreads them between the multiplies, one latency each)
  __builtin_amdgcn_sched_barrier(0);
  auto bfrag = [&](int u, int ks) {
    const int kk = ks >> 1, ci0 = 16 * (ks & 1) + 8 * h;
    return *reinterpret_cast<const Frag8*>(src + act_idx(u + kk, ci0));  // row (u + PAD) + kk - PAD
  };
  const int u0 = 64 * wave + c, u1 = u0 + 32;
  nf32x16 acc0, acc1;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    acc0[r] = 0.f;
    acc1[r] = 0.f;
  }
  Frag8 b0 = bfrag(u0, 0), b1 = bfrag(u1, 0);
#pragma unroll
  for (int ks = 0; ks < 14; ++ks) {
    Frag8 n0 = b0, n1 = b1;
    if (ks + 1 < 14) {
      n0 = bfrag(u0, ks + 1);
      n1 = bfrag(u1, ks + 1);
    }
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(nbf16x8, afr[ks]),
                                                   __builtin_bit_cast(nbf16x8, b0), acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(nbf16x8, afr[ks]),
                                                   __builtin_bit_cast(nbf16x8, b1), acc1, 0, 0, 0);
    b0 = n0;
    b1 = n1;
  }
  store_tile(acc0, bv, h, u0 + PAD, dst);
  store_tile(acc1, bv, h, u1 + PAD, dst);
}

template <bool FROM_SPECTRA, int S>
__global__ void __launch_bounds__(SplitGeo<S>::THREADS)
net_forward_split(const float* __restrict__ x, const NetBf16* __restrict__ nw,
                  float* __restrict__ logits, const float* __restrict__ partial, int32_t chunks,
                  float* __restrict__ x_out, int32_t batch) {
  using Geo = SplitGeo<S>;
  constexpr int W = Geo::W, NL = Geo::NL, ROWS = Geo::ROWS;
  __shared__ __attribute__((aligned(16))) float row_s[T];  // the gate's whole input row
  __shared__ __attribute__((aligned(16))) float xs[ROWS];  // local features
  __shared__ __attribute__((aligned(16))) uint16_t act0[ROWS * 32];
  __shared__ __attribute__((aligned(16))) uint16_t act1[ROWS * 32];
  __shared__ float red[FW_IN_WAVES];
  __shared__ float w4s[32 * TAPS];
  const int b = blockIdx.x, q = b / batch, g = b - q * batch;
  const int a = q * W;
  const int j = threadIdx.x, lane = j & 63;
  const int wave = __builtin_amdgcn_readfirstlane(j >> 6);
  const int h = lane >> 5, c = lane & 31;
  if (j < 32 * TAPS) w4s[j] = nw->w4[j];
  // zero margin rows of both activation buffers
  for (int e = j; e < 2 * PAD * 32; e += Geo::THREADS) {
    const int r = e / 32 < PAD ? e / 32 : NL + e / 32;  // rows 0..PAD-1 and NL+PAD..NL+2PAD-1
    act0[r * 32 + e % 32] = 0;
    act1[r * 32 + e % 32] = 0;
  }
  // input stage over the whole row: thread j < FW_IN_THREADS holds positions
  // 2 j, 2 j + 1 and wave w its share of the total, exactly as the
  // one-workgroup forward does, so the row total is the same float
  if (wave < FW_IN_WAVES) {
    const int jj = j;
    const int vw = wave;
    float2 v;
    if (FROM_SPECTRA && chunks > 1) {
      const int64_t cs = static_cast<int64_t>(batch) * T;
      const float2* pr =
          reinterpret_cast<const float2*>(partial + static_cast<int64_t>(g) * T) + jj;
      v = make_float2(0.f, 0.f);
      // sixteen loads in flight, then the sums in ascending chunk order
      for (int c0 = 0; c0 < chunks; c0 += 16) {
        float2 qv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          qv[u] = c0 + u < chunks ? pr[(c0 + u) * (cs / 2)] : make_float2(0.f, 0.f);
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (c0 + u < chunks) {
            v.x += qv[u].x;
            v.y += qv[u].y;
          }
      }
    } else {
      v = reinterpret_cast<const float2*>(x + static_cast<int64_t>(g) * T)[jj];
    }
    reinterpret_cast<float2*>(row_s)[jj] = v;
    if (FROM_SPECTRA) {
      float sum = v.x + v.y;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
      if (lane == 0) red[vw] = sum;
    }
  }
  __syncthreads();
  float inv = 1.f;
  if (FROM_SPECTRA) {
    float tot = 0.f;
#pragma unroll
    for (int w = 0; w < FW_IN_WAVES; ++w) tot += red[w];  // fixed order
    inv = 1.f / (tot / static_cast<float>(T));
    if (chunks > 1 && j < W) x_out[static_cast<int64_t>(g) * T + a + j] = row_s[a + j];
  }
  // features of the local rows: row u + PAD holds position a - 32 + u (mod T)
  for (int u = j - PAD; u < NL + PAD; u += Geo::THREADS) {
    const float sv = row_s[(a - 32 + u) & (T - 1)];
    xs[u + PAD] = FROM_SPECTRA ? logf(fmaxf(sv * inv, 1e-30f)) : sv;
  }
  __syncthreads();
  // layer 1: one k-step, B[k][u] = bf16(x[u + k - 3]) for k < 7
  const bool mat = wave < Geo::WAVES;  // whole waves
  if (mat) {
    const Frag8 a1 = nw->w1[lane];
    float bv[16];
    load_bias(nw->b1, h, bv);
#pragma unroll
    for (int tile = 0; tile < 2; ++tile) {
      const int u = 64 * wave + 32 * tile + c;
      Frag8 bfr;
#pragma unroll
      for (int i = 0; i < 8; i += 2) {
        uint32_t lo = 0, hi = 0;
        if (h == 0) {
          lo = to_bf16(xs[u + i]);  // local row u + PAD + i - PAD
          if (i + 1 < TAPS) hi = to_bf16(xs[u + i + 1]);
        }
        bfr.w[i / 2] = lo | (hi << 16);
      }
      nf32x16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.f;
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(nbf16x8, a1),
                                                    __builtin_bit_cast(nbf16x8, bfr), acc, 0, 0, 0);
      store_tile(acc, bv, h, u + PAD, act0);
    }
  }
  __syncthreads();
  if (mat) mfma_layer_split<S>(act0, act1, nw->w2, nw->b2, wave, lane);
  __syncthreads();
  if (mat) mfma_layer_split<S>(act1, act0, nw->w3, nw->b3, wave, lane);
  __syncthreads();
  // layer 4 on the part's W positions: thread j < W takes position a + j
  // (local u = 32 + j), in the one-workgroup forward's order
  if (j < W) {
    const int u = 32 + j;
    float acc = nw->b4;
#pragma unroll 1
    for (int qq = 0; qq < 4; ++qq) {
#pragma unroll
      for (int kk = 0; kk < TAPS; ++kk) {
        float w[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] = w4s[(8 * qq + i) * TAPS + kk];
        const uint4 u4 = *reinterpret_cast<const uint4*>(act0 + act_idx(u + kk, 8 * qq));
        const uint32_t uu[4] = {u4.x, u4.y, u4.z, u4.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          acc = fmaf(w[2 * i], __uint_as_float(uu[i] << 16), acc);
          acc = fmaf(w[2 * i + 1], __uint_as_float(uu[i] & 0xffff0000u), acc);
        }
      }
    }
    logits[static_cast<int64_t>(g) * T + a + j] = acc;
  }
}

}  // namespace

size_t net_bf16_bytes() { return sizeof(NetBf16); }

constexpr int kSplitFourMax = 128;  // batches up to this many gates: four parts per gate
constexpr int kSplitTwoMax = 256;   // up to this many: two parts

hipError_t launch_net_prep_bf16(const float* params, void* table, hipStream_t s) {
  hipLaunchKernelGGL(prep_bf16, dim3(1), dim3(256), 0, s, params, static_cast<NetBf16*>(table));
  return hipGetLastError();
}

template <int S>
hipError_t launch_split(const void* table, const float* x, int batch, float* logits, hipStream_t s,
                        bool from_spectra, const float* partial, int32_t chunks, float* x_out) {
  const dim3 grid(static_cast<unsigned>(batch) * S), block(SplitGeo<S>::THREADS);
  const NetBf16* nw = static_cast<const NetBf16*>(table);
  if (from_spectra)
    hipLaunchKernelGGL((net_forward_split<true, S>), grid, block, 0, s, x, nw, logits, partial,
                       chunks, x_out, batch);
  else
    hipLaunchKernelGGL((net_forward_split<false, S>), grid, block, 0, s, x, nw, logits, nullptr, 1,
                       nullptr, batch);
  return hipGetLastError();
}

hipError_t launch_net_forward_bf16(const void* table, const float* x, int batch, float* logits,
                                   hipStream_t s, bool from_spectra, const float* partial,
                                   int32_t chunks, float* x_out) {
  // fewer gates than compute units: several workgroups per gate
  if (batch <= kSplitFourMax)
    return launch_split<4>(table, x, batch, logits, s, from_spectra, partial, chunks, x_out);
  if (batch <= kSplitTwoMax)
    return launch_split<2>(table, x, batch, logits, s, from_spectra, partial, chunks, x_out);
  if (from_spectra)
    hipLaunchKernelGGL(net_forward_bf16<true>, dim3(batch), dim3(FW_THREADS), 0, s, x,
                       static_cast<const NetBf16*>(table), logits, partial, chunks, x_out);
  else
    hipLaunchKernelGGL(net_forward_bf16<false>, dim3(batch), dim3(FW_THREADS), 0, s, x,
                       static_cast<const NetBf16*>(table), logits, nullptr, 1, nullptr);
  return hipGetLastError();
}

}  // namespace ispl
