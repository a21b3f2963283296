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
// (BF16) or 2^-22 (FP16) of each product.  FP16 columns (pulses) are scaled by a
// power of two that puts the largest decoded sample of the pulse below 2^14
// (no overflow; low parts stay normal) and the scale is removed exactly
// before the pulse sum.  Decode,
// shift and pulse integration run in FP32.
//
// Tiling: a workgroup owns one gate, 128 or 256 bins and a chunk of the
// pulses, which it sweeps in blocks of 32 or 64 columns (one or two 32x32
// tiles).  Eight matrix waves hold one or two 32-row MFMA tiles each; four
// building waves decode, shift and split the samples of the next 64-sample
// chunk into LDS, in the MFMA B-operand layout, while the matrix waves
// multiply the current one (double buffer).  The A operand (DFT matrix,
// split) streams from a table laid out in the A-operand order, 16 bytes per
// lane per k-step, two k-steps ahead.  Pulse chunks of one gate write
// partial windows that a fixed-order pass sums.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ispl_device.h"
#include "ispl_internal.h"

namespace ispl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int ZW = 8;              // matrix waves per workgroup
constexpr int ZP = 4;              // building waves per workgroup
constexpr int ZTA = 64 * (ZW + ZP);  // threads
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

// Raw form of one sample as fetched: complex64, or the int16 pair in one dword
// (converted when the chunk is stored, so a fetched chunk holds fewer registers).
template <int ST>
struct RawSample {
  using type = float2;
};
template <>
struct RawSample<1> {
  using type = uint32_t;
};

template <int ST>
__device__ __forceinline__ typename RawSample<ST>::type load_raw(const void* base, int64_t i) {
  return reinterpret_cast<const typename RawSample<ST>::type*>(base)[i];
}
// Four consecutive elements from element i of a row, as one access.
struct alignas(4) Dword4 {
  uint32_t v[4];
};
struct alignas(8) Complex4 {
  float2 v[4];
};
__device__ __forceinline__ void load4(const void* base, int64_t i, uint32_t (&out)[4]) {
  const Dword4 q = *reinterpret_cast<const Dword4*>(static_cast<const uint32_t*>(base) + i);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = q.v[k];
}
__device__ __forceinline__ void load4(const void* base, int64_t i, float2 (&out)[4]) {
  const Complex4 q = *reinterpret_cast<const Complex4*>(static_cast<const float2*>(base) + i);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = q.v[k];
}
__device__ __forceinline__ float2 to_complex(float2 x) { return x; }
__device__ __forceinline__ float2 to_complex(uint32_t r) {
  return make_float2(static_cast<float>(static_cast<int16_t>(r & 0xffffu)),
                     static_cast<float>(static_cast<int32_t>(r) >> 16));
}

// One fetched 64-sample chunk of the B operand.  A building thread owns items
// (column pc, group qg of 4 consecutive samples) with qg = thread % 16 fixed
// and pc = thread / 16 + 16 i, so the 16 lanes of one column read one
// contiguous run of the pulse row (and of its code).  fetch_chunk loads the
// samples, codes and shift twiddles (the same for every column), with indices
// clamped into the row and pulses past the workgroup's range replaced by its
// first one, so every load is valid and unconditional; the FP16 column scales
// are read once per pulse block, so that no wait for them sits between a
// chunk's loads; put_chunk zeroes samples past L and pulses past the range,
// decodes, shifts, scales and splits them into high and low halves and stores
// them in the MFMA B layout (k-step qg / 2, lane half qg % 2).
template <int ST, int NI>
struct ChunkRegs {
  typename RawSample<ST>::type x[NI][4];
  float2 c[NI][4];
  float2 w[4];
};

// Per pulse block: the rows each item reads and its FP16 column scale.
template <int NI>
struct BlockItems {
  int64_t rowp[NI];         // sample index of the gate window in the item's pulse row
  const float2* txp[NI];    // code row of the item's pulse
  float scale[NI];
};

// Column pc's B fragment of k-step ks sits at slot lane ^ swz(ks, lane) of the
// k-step's 64 slots: a bijection that keeps the matrix reads conflict-free and
// spreads the 16 lanes of one column's store over 16 bank groups.
__device__ __forceinline__ int b_slot(int ks, int ln) { return ln ^ ((2 * ks + (ln >> 5)) & 15); }

// Item context of pulse block pb: pulses pb + pc0 + 16 i past p1 read the
// first pulse of the range instead (valid loads, zeroed when stored).
template <int PREC, int NI>
__device__ __forceinline__ void block_items(const ZoomArgs& a, BlockItems<NI>& it, int pb,
                                            int pc0, int p0, int p1, int64_t gate_off) {
  const float2* __restrict__ txb = reinterpret_cast<const float2*>(a.tx);
  int e[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int p = pb + pc0 + 16 * i;
    const int pr = p < p1 ? p : p0;
    it.rowp[i] = static_cast<int64_t>(pr) * a.stride + gate_off;
    it.txp[i] = txb + (a.tx_per_pulse ? static_cast<int64_t>(pr) * a.code_len : 0);
    e[i] = PREC == 1 ? a.col_exp[pr] : 0;
  }
  __builtin_amdgcn_sched_barrier(0);  // the exponent loads overlap
#pragma unroll
  for (int i = 0; i < NI; ++i)
    it.scale[i] = PREC == 1 && pb + pc0 + 16 * i < p1 ? ldexpf(1.f, e[i]) : 1.f;
}

// Fetches chunk ch for the items of a pulse block.
template <int ST, int NI, bool VEC>
__device__ __forceinline__ void fetch_chunk(const ZoomArgs& a, ChunkRegs<ST, NI>& r,
                                            const BlockItems<NI>& it, int ch, int qg,
                                            uint32_t k0) {
  const float2* __restrict__ tw = reinterpret_cast<const float2*>(a.twiddle);
  const uint32_t nmask = static_cast<uint32_t>(a.n_fft - 1);
  const int L = a.code_len;
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2) {
    const int n = ch * ZCHUNK + 4 * qg + s2;
    const int ne = n < L ? n : L - 1;  // always inside the row
    // N is a power of two, so k0 n mod N survives the 32-bit wrap
    r.w[s2] = tw[(k0 * static_cast<uint32_t>(ne)) & nmask];
  }
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    if constexpr (VEC) {
      // L % 4 == 0, so a group lies wholly inside [0, L) or wholly past it;
      // groups past it fetch the row's last four samples (zeroed when stored)
      const int nq = ch * ZCHUNK + 4 * qg;
      const int n0 = nq < L ? nq : L - 4;
      load4(a.samples, it.rowp[i] + n0, r.x[i]);
      load4(it.txp[i], n0, r.c[i]);
    } else {
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int n = ch * ZCHUNK + 4 * qg + s2;
        const int ne = n < L ? n : L - 1;
        r.x[i][s2] = load_raw<ST>(a.samples, it.rowp[i] + ne);
        r.c[i][s2] = it.txp[i][ne];
      }
    }
  }
}

// Stores a fetched chunk (see fetch_chunk) into one LDS B buffer.
template <int PREC, int ST, int NI>
__device__ __forceinline__ void put_chunk(const ChunkRegs<ST, NI>& r, const BlockItems<NI>& it,
                                          Frag (*bh)[ZKS][64], Frag (*bl)[ZKS][64], int pb,
                                          int ch, int pc0, int qg, int p1, int L) {
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int pc = pc0 + 16 * i;
    const bool live = pb + pc < p1;
    Frag fh, fl;
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      // samples past L and pulses past the range contribute zero (their
      // split words are cleared; they were fetched from valid addresses)
      const bool keep = live && ch * ZCHUNK + 4 * qg + s2 < L;
      const float2 x = to_complex(r.x[i][s2]);
      const float2 c = r.c[i][s2];
      const float2 w = r.w[s2];
      const float2 d = make_float2(fmaf(c.x, x.x, c.y * x.y), fmaf(c.x, x.y, -(c.y * x.x)));
      const float2 y = make_float2(fmaf(d.x, w.x, -(d.y * w.y)) * it.scale[i],
                                   fmaf(d.x, w.y, d.y * w.x) * it.scale[i]);
      uint32_t rh, rl, ih, il;
      split2<PREC>(y.x, rh, rl);
      split2<PREC>(y.y, ih, il);
      fh.w[s2] = keep ? rh | (ih << 16) : 0u;
      fl.w[s2] = keep ? rl | (il << 16) : 0u;
    }
    const int ks = qg >> 1, ln = (pc & 31) + 32 * (qg & 1), ct = pc >> 5;
    bh[ct][ks][b_slot(ks, ln)] = fh;
    bl[ct][ks][b_slot(ks, ln)] = fl;
  }
}

// Workgroups are dealt to the 8 XCDs round-robin; renumber the first nblk of
// them so that each XCD runs a contiguous range of work items (neighbouring
// gates, whose sample windows overlap, then share that XCD's L2).
__device__ __forceinline__ int zoom_xcd_id(int b, int nblk) {
  const int xcd = b & 7, slot = b >> 3;
  const int per = nblk >> 3, extra = nblk & 7;
  return xcd < extra ? xcd * (per + 1) + slot : extra * (per + 1) + (xcd - extra) * per + slot;
}

// RT: 32-row MFMA tiles per wave (16 bins each); CT: 32-pulse column tiles per
// pulse block.  A workgroup owns one gate, 128 RT bins and one chunk of the
// pulses.  Its waves have two roles: ZW matrix waves multiply, ZP building
// waves fetch, decode and split the samples of the next 64-sample chunk into
// the other half of a double-buffered LDS B operand at the same time (one
// barrier per chunk; both roles pass the same number of barriers).  The
// matrix waves stream their A fragments through a two-deep register ring.
template <int PREC, int ST, int RT, int CT>
__global__ void __launch_bounds__(ZTA) zoom_spectra(ZoomArgs a) {
  constexpr int NCOL = 32 * CT;
  constexpr int NI = NCOL / 16;        // items per building thread
  __shared__ Frag bh[2][CT][ZKS][64];  // B operand, high parts: [buffer][tile][k-step][lane]
  __shared__ Frag bl[2][CT][ZKS][64];  // low parts

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int btiles = a.n_bins / (128 * RT);
  const int per_gate = btiles * a.chunks;
  // With a gate list only the first count * per_gate workgroups have work;
  // those are renumbered among themselves (uniform, before any barrier).
  int nblk = static_cast<int>(gridDim.x);
  if (a.gate_list) {
    const int cnt = min(max(*a.gate_count, 0), nblk / per_gate);
    nblk = cnt * per_gate;
    if (static_cast<int>(blockIdx.x) >= nblk) return;
  }
  int bid = zoom_xcd_id(static_cast<int>(blockIdx.x), nblk);
  const int chunk = bid % a.chunks;
  bid /= a.chunks;
  const int bt = bid % btiles;
  int g = bid / btiles;
  if (a.gate_list) {
    g = a.gate_list[g];
    if (g < 0 || g >= a.n_gates) return;
  }
  const int L = a.code_len, N = a.n_fft;
  const int p0 = static_cast<int>((static_cast<int64_t>(chunk) * a.n_pulses) / a.chunks);
  const int p1 = static_cast<int>((static_cast<int64_t>(chunk + 1) * a.n_pulses) / a.chunks);
  const int nchunks = a.code_pad / ZCHUNK;
  const int n_ks = nchunks * ZKS;

  if (wave >= ZW) {
    // ---- building waves ----
    // Chunks in the matrix waves' order, each fetched and stored between two
    // barriers.  Per pulse block both roles pass one barrier after each
    // stored chunk and one more at the block's end.
    const uint32_t k0 = static_cast<uint32_t>(((a.bin_start[g] % N) + N) % N);
    const int64_t gate_off =
        static_cast<int64_t>(a.first_gate) + static_cast<int64_t>(g) * a.gate_step;
    const int bt_id = tid - 64 * ZW;
    const int qg = bt_id & 15, pc0 = bt_id >> 4;
    static_assert(64 * ZP / 16 * NI == NCOL, "items cover the block's columns");
    // With L a multiple of 4 each group of 4 samples is fetched as one
    // contiguous 16- or 32-byte run (whole cache lines per instruction).
    auto build = [&](auto vec) {
      constexpr bool VEC = decltype(vec)::value;
      ChunkRegs<ST, NI> r;
      BlockItems<NI> it;
      for (int pb = p0; pb < p1; pb += NCOL) {
        block_items<PREC, NI>(a, it, pb, pc0, p0, p1, gate_off);
        for (int ch = 0; ch < nchunks; ++ch) {
          fetch_chunk<ST, NI, VEC>(a, r, it, ch, qg, k0);
          // every load of the chunk is issued before the first use of any
          __builtin_amdgcn_sched_barrier(0);
          put_chunk<PREC, ST, NI>(r, it, bh[ch & 1], bl[ch & 1], pb, ch, pc0, qg, p1, L);
          __syncthreads();
        }
        __syncthreads();  // the block's last chunk is consumed
      }
    };
    if (L % 4 == 0)
      build(std::true_type{});
    else
      build(std::false_type{});
    return;
  }

  // ---- matrix waves ----
  // A operand of this wave: row tiles (bt ZW + wave) RT + r, k-steps along the code
  const Frag* __restrict__ ah_t[RT];
  const Frag* __restrict__ al_t[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int64_t rt = static_cast<int64_t>((bt * ZW + wave) * RT + r);
    ah_t[r] = reinterpret_cast<const Frag*>(a.a_hi) + rt * n_ks * 64 + lane;
    al_t[r] = reinterpret_cast<const Frag*>(a.a_lo) + rt * n_ks * 64 + lane;
  }

  float total[RT][8];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int i = 0; i < 8; ++i) total[r][i] = 0.f;

  // A fragments are fetched AD k-steps ahead into a ring (slot ks % AD, which
  // AD | ZKS makes static).  The refill after the last k-step of a pulse
  // block wraps to the first ones, which the next block uses.
  // Four k-steps ahead where the registers allow it (one column tile): on
  // small launches every workgroup reaches the same k-steps at once, so the
  // table misses are not warmed in L2 by anyone ahead.
  constexpr int AD = CT == 1 ? 4 : 2;
  static_assert(ZKS % AD == 0, "static ring slots");
  Frag ah[AD][RT], al[AD][RT];
#pragma unroll
  for (int d = 0; d < AD; ++d)
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const int kk = d < n_ks ? d : n_ks - 1;
      ah[d][r] = ah_t[r][static_cast<int64_t>(kk) * 64];
      al[d][r] = al_t[r][static_cast<int64_t>(kk) * 64];
    }

  for (int pb = p0; pb < p1; pb += NCOL) {
    f32x16 acc[RT][CT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[r][ct][i] = 0.f;
    __syncthreads();  // chunk 0 is built
    for (int ch = 0; ch < nchunks; ++ch) {
      const int b = ch & 1;
#pragma unroll
      for (int ks = 0; ks < ZKS; ++ks) {
        const int slot = ks % AD;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          const Frag fbh = bh[b][ct][ks][b_slot(ks, lane)], fbl = bl[b][ct][ks][b_slot(ks, lane)];
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            acc[r][ct] = mfma<PREC>(ah[slot][r], fbh, acc[r][ct]);
            acc[r][ct] = mfma<PREC>(ah[slot][r], fbl, acc[r][ct]);
            acc[r][ct] = mfma<PREC>(al[slot][r], fbh, acc[r][ct]);
          }
        }
        // refill the slot with k-step kk + AD, wrapping into the next block
        int kn = ch * ZKS + ks + AD;
        if (kn >= n_ks) kn -= n_ks;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          ah[slot][r] = ah_t[r][static_cast<int64_t>(kn) * 64];
          al[slot][r] = al_t[r][static_cast<int64_t>(kn) * 64];
        }
      }
      __syncthreads();  // chunk ch is consumed, chunk ch + 1 is built
    }
    // |Z|^2 per (bin, pulse).  D row (i % 4) + 8 (i / 4) + 4 h (h = lane / 32) is Re
    // (even) or Im (odd) of tile bin row / 2: registers 4 qa + 2 s and 4 qa + 2 s + 1
    // are bin s + 4 qa + 2 h of the tile.
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      float pw[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) pw[i] = 0.f;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int pcol = pb + 32 * ct + (lane & 31);
        const float un = (PREC == 1 && pcol < p1) ? ldexpf(1.f, -2 * a.col_exp[pcol]) : 1.f;
#pragma unroll
        for (int qa = 0; qa < 4; ++qa)
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const float re = acc[r][ct][4 * qa + 2 * s], im = acc[r][ct][4 * qa + 2 * s + 1];
            pw[2 * qa + s] += fmaf(re, re, im * im) * un;
          }
      }
      // sum over the 32 pulse columns of each half wave, fixed order
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        float v = pw[i];
#pragma unroll
        for (int off = 1; off < 32; off <<= 1) v += __shfl_xor(v, off);
        total[r][i] += v;
      }
    }
  }

  // lane 0 holds tile bins s + 4 qa (h = 0), lane 32 bins s + 4 qa + 2 (h = 1)
  if ((lane & 31) == 0) {
    const int h = lane >> 5;
    float* row = a.chunks == 1
                     ? a.out + static_cast<int64_t>(g) * a.n_bins
                     : a.partial + (static_cast<int64_t>(chunk) * a.n_gates + g) * a.n_bins;
    const bool add = a.chunks == 1 && a.accumulate;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      float* out = row + bt * 128 * RT + 16 * (wave * RT + r);
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          float* dst = out + s + 4 * qa + 2 * h;
          *dst = add ? *dst + total[r][2 * qa + s] : total[r][2 * qa + s];
        }
    }
  }
}

// Per-pulse FP16 exponents, one workgroup per pulse.
__global__ void __launch_bounds__(256)
pulse_exponents(const void* __restrict__ samples, int32_t sample_type, const float* __restrict__ tx,
                int64_t stride, int64_t lo, int64_t hi, int32_t code_len, int32_t tx_per_pulse,
                int32_t* __restrict__ exps) {
  pulse_exponent_block(samples, sample_type, tx, stride, lo, hi, code_len, tx_per_pulse,
                       static_cast<int>(blockIdx.x), exps);
}

template <int PREC, int ST, int RT>
hipError_t launch_zoom_rt(const ZoomArgs& a, int ct, hipStream_t stream) {
  const unsigned blocks =
      static_cast<unsigned>(a.n_gates) * (a.n_bins / (128 * RT)) * static_cast<unsigned>(a.chunks);
  if (ct == 1)
    hipLaunchKernelGGL((zoom_spectra<PREC, ST, RT, 1>), dim3(blocks), dim3(ZTA), 0, stream, a);
  else if (ct == 2)
    hipLaunchKernelGGL((zoom_spectra<PREC, ST, RT, 2>), dim3(blocks), dim3(ZTA), 0, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int PREC, int ST>
hipError_t launch_zoom_st(const ZoomArgs& a, hipStream_t stream) {
  return a.row_tiles == 2 ? launch_zoom_rt<PREC, ST, 2>(a, a.col_tiles, stream)
                          : launch_zoom_rt<PREC, ST, 1>(a, a.col_tiles, stream);
}

template <int PREC>
hipError_t launch_zoom_t(const ZoomArgs& a, hipStream_t stream) {
  return a.sample_type == 1 ? launch_zoom_st<PREC, 1>(a, stream) : launch_zoom_st<PREC, 0>(a, stream);
}

}  // namespace

hipError_t launch_zoom(const ZoomArgs& a, hipStream_t stream, bool exponents) {
  if (a.precision == 1) {
    if (exponents) {
      hipLaunchKernelGGL(pulse_exponents, dim3(static_cast<unsigned>(a.n_pulses)), dim3(256), 0,
                         stream, a.samples, a.sample_type, a.tx, a.stride, a.row_lo, a.row_hi,
                         a.code_len, a.tx_per_pulse, a.col_exp);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return launch_zoom_t<1>(a, stream);
  }
  return launch_zoom_t<0>(a, stream);
}

}  // namespace ispl
