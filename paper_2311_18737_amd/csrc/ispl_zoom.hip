// Zoom DFT on the matrix cores (gfx950 MFMA): a window of K bins of the
// N-point spectrum of every gate, S[g][j] = sum_p |Z_{p,g}[j]|^2 with
//
//   Z_{p,g}[j] = sum_{n < L} y'_{p,g}[n] W_N^{j n},
//   y'_{p,g}[n] = conj(c_p[n]) x_p[g0 + g s + n] W_N^{k0_g n},
//
// i.e. the decoded row of Section 3.2 shifted so that bin k0_g (the window
// start of gate g) sits at 0, then a direct DFT onto K bins.  The DFT matrix
// W = W_N^{j n} = Wr + i Wi is the same for every gate and pulse; the complex
// product Z = W y takes three real GEMMs per gate (rows: bins, columns:
// pulses, reduction: the L samples), k1 = (Wr + Wi) yr, k2 = Wr (yi - yr),
// k3 = Wi (yr + yi), with Re Z = k1 - k3 and Im Z = k1 + k2.
//
// Precision: both operands are split into a high and a low 16-bit part
// (BF16 or FP16) and D = A_hi B_hi + A_hi B_lo + A_lo B_hi accumulates in
// FP32; the dropped A_lo B_lo term and the split residuals are about 2^-16
// (BF16) or 2^-22 (FP16) of each product.  FP16 columns (pulses) are scaled by a
// power of two that puts the largest decoded sample of the pulse below 2^14
// (no overflow, yr + yi stays below 2^15; low parts stay normal) and the
// scale is removed exactly before the pulse sum.  Decode, shift and pulse
// integration run in FP32.
//
// Tiling: a workgroup owns one gate, 128 or 256 bins and a chunk of the
// pulses, which it sweeps in blocks of 32 or 64 columns (one or two 32x32
// tiles).  Eight matrix waves hold k1, k2, k3 of one 32-bin tile each; four
// building waves decode, shift and split the samples of the next 64-sample
// chunk into LDS, in the MFMA B-operand layout, while the matrix waves
// multiply the current one (double buffer).  The A operands (the three split
// matrices) stream from a table laid out in the A-operand order, 16 bytes per
// lane per k-step and product, one k-step ahead.  +-1 codes are read as sign
// bits, the gate's shift twiddles from LDS.  Pulse chunks of one gate write
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
constexpr int ZCHUNK = 64;         // samples per B chunk (built in two halves)
constexpr int ZKS = ZCHUNK / 16;   // MFMA k-steps of 16 samples per chunk and product
constexpr int ZTWMAX = 4096;       // longest code whose shift twiddles are staged in LDS

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

// A-table fragments read through a workgroup-uniform global base and a
// 32-bit byte offset per lane (scalar base + vector offset addressing).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
using gbytes = const __attribute__((address_space(1))) char*;
using gfrag = const __attribute__((address_space(1))) u32x4*;
__device__ __forceinline__ gbytes uniform_bytes(const void* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return reinterpret_cast<gbytes>((static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ __forceinline__ Frag load_frag(gbytes base, uint32_t byte_off) {
  const u32x4 v = *reinterpret_cast<gfrag>(base + byte_off);
  Frag f;
  f.w[0] = v.x;
  f.w[1] = v.y;
  f.w[2] = v.z;
  f.w[3] = v.w;
  return f;
}

// One fetched half (32 samples) of a 64-sample chunk of the B operand.  A
// building thread owns one item per half: column pc = thread / 4 of the pulse
// block and group q = thread % 4 of 8 consecutive samples (group 4 hf + q of
// the chunk in half hf), so the 4 lanes of one column read one contiguous run
// of the pulse row (and of its code).  Loads are valid and unconditional:
// indices are clamped into the row and pulses past the workgroup's range read
// its first one (both zeroed when stored).  The put step decodes, shifts and
// scales the samples, forms the three B operands of the product (below),
// splits each into high and low halves and stores them in the MFMA B layout
// (k-step of the group / 2, lane half group % 2); in a half past L or a block
// past the last pulse the samples outside the range are zeroed first.  Two
// forms: complex codes (samples, codes and shift twiddles fetched together),
// and +-1 codes read as sign bits, whose next half's samples are in flight
// while the current one is stored.
template <int ST>
struct ChunkRegs {
  typename RawSample<ST>::type x[8];
  float2 c[8];
  float2 w[8];
};
template <int ST>
struct BitRegs {
  typename RawSample<ST>::type x[8];
  uint32_t bits;  // bit s: code of sample s of the group is -1
};

// Per pulse block: the rows the item reads and its FP16 column scale.
struct Item {
  int64_t rowp;         // sample index of the gate window in the item's pulse row
  const float2* txp;    // code row of the item's pulse (complex codes)
  const uint32_t* bitp; // code-bit row of the item's pulse (sign bits)
  float scale;
};

// Column pc's B fragment of k-step ks sits at slot lane ^ swz(ks, lane) of the
// k-step's 64 slots: a bijection that keeps the matrix reads conflict-free and
// spreads the 16 lanes of each quarter wave's store over 16 bank groups.
__device__ __forceinline__ int b_slot(int ks, int ln) { return ln ^ ((8 * ks + 4 * (ln >> 5)) & 15); }

// Item context of pulse block pb: pulse pb + pc past p1 reads the first pulse
// of the range instead (valid loads, zeroed when stored).
template <int PREC>
__device__ __forceinline__ void item_of(const ZoomArgs& a, Item& it, int pb, int pc, int p0,
                                        int p1, int64_t gate_off, int words) {
  const int p = pb + pc;
  const int pr = p < p1 ? p : p0;
  it.rowp = static_cast<int64_t>(pr) * a.stride + gate_off;
  const int64_t row = a.tx_per_pulse ? pr : 0;
  it.txp = reinterpret_cast<const float2*>(a.tx) + row * a.code_len;
  it.bitp = a.code_bits ? a.code_bits + row * words : nullptr;
  const int e = PREC == 1 ? a.col_exp[pr] : 0;
  it.scale = PREC == 1 && p < p1 ? ldexpf(1.f, e) : 1.f;
}

// The shift twiddle W_N^{k0 n} of sample n: from the gate's table in LDS
// (tws != NULL, samples [0, code_pad)) or from the global twiddle table.
__device__ __forceinline__ float2 shift_twiddle(const float2* tws, const float2* __restrict__ tw,
                                                uint32_t k0, uint32_t nmask, int n, int L) {
  if (tws) return tws[n];
  const int ne = n < L ? n : L - 1;  // always inside the row
  // N is a power of two, so k0 n mod N survives the 32-bit wrap
  return tw[(k0 * static_cast<uint32_t>(ne)) & nmask];
}

// The item's 8 samples from sample nb on (VEC: L % 4 == 0, so each half group
// lies wholly inside [0, L) or wholly past it and is one 16- or 32-byte
// access).
template <int ST, bool VEC>
__device__ __forceinline__ void fetch_samples(const ZoomArgs& a, typename RawSample<ST>::type (&x)[8],
                                              const Item& it, int nb) {
  const int L = a.code_len;
  if constexpr (VEC) {
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int nq = nb + 4 * hh;
      const int n0 = nq < L ? nq : L - 4;
      typename RawSample<ST>::type xs[4];
      load4(a.samples, it.rowp + n0, xs);
#pragma unroll
      for (int k = 0; k < 4; ++k) x[4 * hh + k] = xs[k];
    }
  } else {
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      const int n = nb + s2;
      x[s2] = load_raw<ST>(a.samples, it.rowp + (n < L ? n : L - 1));
    }
  }
}

template <int ST, bool VEC>
__device__ __forceinline__ void fetch_chunk(const ZoomArgs& a, ChunkRegs<ST>& r, const Item& it,
                                            int nb, uint32_t k0, const float2* tws) {
  const float2* __restrict__ tw = reinterpret_cast<const float2*>(a.twiddle);
  const uint32_t nmask = static_cast<uint32_t>(a.n_fft - 1);
  const int L = a.code_len;
#pragma unroll
  for (int s2 = 0; s2 < 8; ++s2) r.w[s2] = shift_twiddle(tws, tw, k0, nmask, nb + s2, L);
  fetch_samples<ST, VEC>(a, r.x, it, nb);
  if constexpr (VEC) {
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int nq = nb + 4 * hh;
      float2 cs[4];
      load4(it.txp, nq < L ? nq : L - 4, cs);
#pragma unroll
      for (int k = 0; k < 4; ++k) r.c[4 * hh + k] = cs[k];
    }
  } else {
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      const int n = nb + s2;
      r.c[s2] = it.txp[n < L ? n : L - 1];
    }
  }
}

template <int ST, bool VEC>
__device__ __forceinline__ void fetch_bits(const ZoomArgs& a, BitRegs<ST>& r, const Item& it,
                                           int nb) {
  fetch_samples<ST, VEC>(a, r.x, it, nb);
  r.bits = it.bitp[nb >> 5] >> (nb & 31);  // bit s of the group in bit s
}

// FP16 split of v = b sc (sc a power of two, possibly negative) into the low
// (H = 0) or high (H = 1) half of the words hi and lo: hi = f16(v) and
// lo = f16(v - hi), each one fused multiply-add with an FP16 result that
// leaves the other half of its word alone -- the same bits as rounding v and
// then v - hi separately (both are exact in FP32 before the final rounding).
template <int H>
__device__ __forceinline__ void split_f16_scaled(float b, float sc, uint32_t& hi, uint32_t& lo) {
  if constexpr (H == 0) {
    asm("v_fma_mixlo_f16 %0, %1, %2, 0" : "+v"(hi) : "v"(b), "v"(sc));
    asm("v_fma_mixlo_f16 %0, %1, %2, -%3 op_sel_hi:[0,0,1]" : "+v"(lo) : "v"(b), "v"(sc), "v"(hi));
  } else {
    asm("v_fma_mixhi_f16 %0, %1, %2, 0" : "+v"(hi) : "v"(b), "v"(sc));
    asm("v_fma_mixhi_f16 %0, %1, %2, -%3 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
        : "+v"(lo)
        : "v"(b), "v"(sc), "v"(hi));
  }
}

// Splits the three B operands of y sc, y = yr + i yi (yr, yi - yr, yr + yi;
// sc the column scale, its sign the code's for sign-bit codes), of the
// group's sample s2 into the fragments.
template <int PREC>
__device__ __forceinline__ void split_b(float yr, float yi, float sc, int s2, Frag (&fh)[3],
                                        Frag (&fl)[3]) {
  const float b[3] = {yr, yi - yr, yr + yi};
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    if constexpr (PREC == 1) {
      if (s2 % 2 == 0)
        split_f16_scaled<0>(b[pr], sc, fh[pr].w[s2 / 2], fl[pr].w[s2 / 2]);
      else
        split_f16_scaled<1>(b[pr], sc, fh[pr].w[s2 / 2], fl[pr].w[s2 / 2]);
    } else {
      uint32_t hi, lo;
      split2<PREC>(b[pr] * sc, hi, lo);
      if (s2 % 2 == 0) {
        fh[pr].w[s2 / 2] = hi;
        fl[pr].w[s2 / 2] = lo;
      } else {
        fh[pr].w[s2 / 2] |= hi << 16;
        fl[pr].w[s2 / 2] |= lo << 16;
      }
    }
  }
}

__device__ __forceinline__ void store_b(const Frag (&fh)[3], const Frag (&fl)[3],
                                        Frag (*bh)[2][ZKS][64], Frag (*bl)[2][ZKS][64], int pc,
                                        int qq) {
  const int ks = qq >> 1, ln = (pc & 31) + 32 * (qq & 1), ct = pc >> 5;
  const int sl = b_slot(ks, ln);
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    bh[pr][ct][ks][sl] = fh[pr];
    bl[pr][ct][ks][sl] = fl[pr];
  }
}

// Stores a fetched chunk of complex codes into one LDS B buffer.
template <int PREC, int ST, bool MASK>
__device__ __forceinline__ void put_chunk(const ChunkRegs<ST>& r, const Item& it,
                                          Frag (*bh)[2][ZKS][64], Frag (*bl)[2][ZKS][64], int pb,
                                          int nb, int qq, int pc, int p1, int L) {
  const bool live = pb + pc < p1;
  Frag fh[3], fl[3];
#pragma unroll
  for (int s2 = 0; s2 < 8; ++s2) {
    const float2 x = to_complex(r.x[s2]);
    const float2 c = r.c[s2];
    const float2 w = r.w[s2];
    const float2 d = make_float2(fmaf(c.x, x.x, c.y * x.y), fmaf(c.x, x.y, -(c.y * x.x)));
    float yr = fmaf(d.x, w.x, -(d.y * w.y));
    float yi = fmaf(d.x, w.y, d.y * w.x);
    if constexpr (MASK) {
      // samples past L and pulses past the range contribute zero (they were
      // fetched from valid addresses)
      const bool keep = live && nb + s2 < L;
      yr = keep ? yr : 0.f;
      yi = keep ? yi : 0.f;
    }
    split_b<PREC>(yr, yi, it.scale, s2, fh, fl);
  }
  store_b(fh, fl, bh, bl, pc, qq);
}

// The same for sign-bit codes: conj(c) x = x with both signs flipped when
// c = -1 (exactly the complex product for c = +-1 + 0i, up to the sign of a
// zero), applied as the sign of the column scale; twiddles from LDS.
template <int PREC, int ST, bool MASK>
__device__ __forceinline__ void put_bits(const BitRegs<ST>& r, const Item& it, const float2* tws,
                                         Frag (*bh)[2][ZKS][64], Frag (*bl)[2][ZKS][64], int pb,
                                         int nb, int qq, int pc, int p1, int L) {
  const bool live = pb + pc < p1;
  Frag fh[3], fl[3];
#pragma unroll
  for (int s2 = 0; s2 < 8; ++s2) {
    const float2 x = to_complex(r.x[s2]);
    const float2 w = tws[nb + s2];
    // conj(c) x w sc = x w (+-sc): the code's sign rides on the scale
    const uint32_t sg = (r.bits << (31 - s2)) & 0x80000000u;
    const float sc = __uint_as_float(__float_as_uint(it.scale) ^ sg);
    float yr = fmaf(x.x, w.x, -(x.y * w.y));
    float yi = fmaf(x.x, w.y, x.y * w.x);
    if constexpr (MASK) {
      const bool keep = live && nb + s2 < L;
      yr = keep ? yr : 0.f;
      yi = keep ? yi : 0.f;
    }
    split_b<PREC>(yr, yi, sc, s2, fh, fl);
  }
  store_b(fh, fl, bh, bl, pc, qq);
}

// True (wave-uniform) when the code rows of pulses [p0, p1) are all +-1.
__device__ __forceinline__ bool rows_binary(const ZoomArgs& a, int p0, int p1, int lane) {
  if (!a.tx_per_pulse) return a.code_binary[0] != 0;
  bool ok = true;
  for (int p = p0 + lane; p < p1; p += 64) ok = ok && a.code_binary[p] != 0;
  return __all(ok);
}

// Workgroups are dealt to the 8 XCDs round-robin; renumber the first nblk of
// them so that each XCD runs a contiguous range of work items (neighbouring
// gates, whose sample windows overlap, then share that XCD's L2).
__device__ __forceinline__ int zoom_xcd_id(int b, int nblk) {
  const int xcd = b & 7, slot = b >> 3;
  const int per = nblk >> 3, extra = nblk & 7;
  return xcd < extra ? xcd * (per + 1) + slot : extra * (per + 1) + (xcd - extra) * per + slot;
}

// RT: the workgroup owns 128 RT bins (4 RT tiles of 32 bins); CT: 32-pulse
// column tiles per pulse block.  A workgroup owns one gate, its bins and one
// chunk of the pulses.  Its waves have two roles: ZW matrix waves multiply,
// ZP building waves fetch, decode and split the samples of the next
// 64-sample chunk into the other half of a double-buffered LDS B operand at
// the same time (one barrier per chunk; both roles pass the same number of
// barriers).  With 4 RT bin tiles over ZW matrix waves, CG = ZW / (4 RT)
// waves share a bin tile and split the column tiles between them (their
// sums are added in LDS at the end).
//
// The complex product Z = W y with W = Wr + i Wi takes three real GEMMs
// (Gauss): k1 = (Wr + Wi) yr, k2 = Wr (yi - yr), k3 = Wi (yr + yi), then
// Re Z = k1 - k3, Im Z = k1 + k2 -- three quarters of the matrix work of the
// real 2K x 2L form.  Each matrix wave keeps k1, k2, k3 of its 32 bins x its
// columns in registers; its A fragments (the table of the three matrices in
// A-operand order) are refilled in place, each product's right after its
// multiplies, one k-step ahead.
template <int PREC, int ST, int RT, int CT>
__global__ void __launch_bounds__(ZTA) zoom_spectra(ZoomArgs a) {
  constexpr int NCOL = 32 * CT;
  constexpr int BG = 4 * RT;                   // bin tiles per workgroup
  constexpr int CG = ZW / BG;                  // matrix waves per bin tile
  constexpr int CTW = (CT + CG - 1) / CG;      // column tiles per matrix wave
  __shared__ Frag bh[2][3][2][ZKS][64];        // B operand, high parts: [buffer][product][tile][k-step][lane]
  __shared__ Frag bl[2][3][2][ZKS][64];        // low parts
  __shared__ float red[CG > 1 ? BG : 1][64];   // second column group's sums
  __shared__ float2 tw_gate[ZTWMAX];           // W_N^{k0 n}, n < code_pad (code_pad <= ZTWMAX)

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

  const bool tw_lds = a.code_pad <= ZTWMAX;
  if (wave >= ZW) {
    // ---- building waves ----
    // Chunks in the matrix waves' order, each fetched and stored between two
    // barriers.  Per pulse block both roles pass one barrier after each
    // stored chunk and one more at the block's end.
    const uint32_t k0 = static_cast<uint32_t>(((a.bin_start[g] % N) + N) % N);
    const int64_t gate_off =
        static_cast<int64_t>(a.first_gate) + static_cast<int64_t>(g) * a.gate_step;
    // the arbiter prefers these waves' instructions: left at the matrix
    // waves' priority, their decode and split work was issued so rarely
    // between the multiplies that the matrix waves waited for it at every
    // chunk barrier
    __builtin_amdgcn_s_setprio(2);
    const int bt_id = tid - 64 * ZW;
    const int q = bt_id & 3, pc = bt_id >> 2;  // one item per thread and half chunk
    static_assert(64 * ZP / 4 == 64, "items cover two column tiles");
    if (tw_lds) {  // the gate's shift twiddles, once
      const float2* __restrict__ tw = reinterpret_cast<const float2*>(a.twiddle);
      const uint32_t nmask = static_cast<uint32_t>(N - 1);
      for (int n = bt_id; n < a.code_pad; n += 64 * ZP)
        tw_gate[n] = tw[(k0 * static_cast<uint32_t>(n < L ? n : L - 1)) & nmask];
    }
    __syncthreads();  // both roles: the twiddles are staged
    const float2* tws = tw_lds ? tw_gate : nullptr;
    // columns past the block width (one column tile): the wave only passes
    // the barriers
    const bool item = pc < NCOL;
    const int words = a.code_pad / 32;
    // a chunk is built in two halves of 32 samples: group q of half hf is
    // group 4 hf + q of the chunk
    auto build = [&](auto vec) {
      constexpr bool VEC = decltype(vec)::value;
      ChunkRegs<ST> r;
      Item it;
      for (int pb = p0; pb < p1; pb += NCOL) {
        if (item) item_of<PREC>(a, it, pb, pc, p0, p1, gate_off, words);
        const bool full_block = pb + NCOL <= p1;
        for (int ch = 0; ch < nchunks; ++ch) {
          if (item) {
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
              const int nb = ch * ZCHUNK + 32 * hf + 8 * q;
              fetch_chunk<ST, VEC>(a, r, it, nb, k0, tws);
              // every load of the half is issued before the first use of any
              __builtin_amdgcn_sched_barrier(0);
              if (full_block && ch * ZCHUNK + 32 * hf + 32 <= L)
                put_chunk<PREC, ST, false>(r, it, bh[ch & 1], bl[ch & 1], pb, nb, 4 * hf + q, pc,
                                           p1, L);
              else
                put_chunk<PREC, ST, true>(r, it, bh[ch & 1], bl[ch & 1], pb, nb, 4 * hf + q, pc,
                                          p1, L);
            }
          }
          __syncthreads();
        }
        __syncthreads();  // the block's last chunk is consumed
      }
    };
    // +-1 codes as sign bits, the next half's samples in flight while the
    // current one is stored (across chunks and pulse blocks too)
    auto build_bits = [&](auto vec) {
      constexpr bool VEC = decltype(vec)::value;
      BitRegs<ST> ra, rb;  // first halves in ra, second halves in rb
      Item it, itn;
      if (item) {
        item_of<PREC>(a, it, p0, pc, p0, p1, gate_off, words);
        fetch_bits<ST, VEC>(a, ra, it, 8 * q);
      }
      for (int pb = p0; pb < p1; pb += NCOL) {
        const bool has_next = pb + NCOL < p1;
        if (item && has_next) item_of<PREC>(a, itn, pb + NCOL, pc, p0, p1, gate_off, words);
        const bool full_block = pb + NCOL <= p1;
        for (int ch = 0; ch < nchunks; ++ch) {
          if (item) {
            auto half = [&](BitRegs<ST>& cur, BitRegs<ST>& nxt, int hf) {
              const int nb = ch * ZCHUNK + 32 * hf + 8 * q;
              if (hf == 0)
                fetch_bits<ST, VEC>(a, nxt, it, nb + 32);
              else if (ch + 1 < nchunks)
                fetch_bits<ST, VEC>(a, nxt, it, nb + 32);
              else if (has_next)
                fetch_bits<ST, VEC>(a, nxt, itn, 8 * q);
              __builtin_amdgcn_sched_barrier(0);
              if (full_block && ch * ZCHUNK + 32 * hf + 32 <= L)
                put_bits<PREC, ST, false>(cur, it, tw_gate, bh[ch & 1], bl[ch & 1], pb, nb,
                                          4 * hf + q, pc, p1, L);
              else
                put_bits<PREC, ST, true>(cur, it, tw_gate, bh[ch & 1], bl[ch & 1], pb, nb,
                                         4 * hf + q, pc, p1, L);
            };
            half(ra, rb, 0);
            half(rb, ra, 1);
          }
          __syncthreads();
        }
        __syncthreads();  // the block's last chunk is consumed
        it = itn;
      }
    };
    const bool bits = tw_lds && a.code_bits && rows_binary(a, p0, p1, lane);
    if (bits) {
      if (L % 4 == 0)
        build_bits(std::true_type{});
      else
        build_bits(std::false_type{});
    } else if (L % 4 == 0) {
      build(std::true_type{});
    } else {
      build(std::false_type{});
    }
    if constexpr (CG > 1) __syncthreads();  // the matrix waves' final sum
    return;
  }

  // ---- matrix waves ----
  __syncthreads();  // the building waves have staged the twiddles
  const int btl = wave % BG, cg = wave / BG;
  const int ct0 = cg * CTW;                    // first column tile of this wave
  const bool cols = ct0 < CT;                  // false: a wave with no column tile (CT < CG)
  // A operand of this wave: product pr, bin tile bt * BG + btl, k-steps along
  // the code; one workgroup-uniform base per product and table
  const int n_bt = a.n_bins / 32;
  gbytes ahb[3], alb[3];
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    const int64_t t0 = (static_cast<int64_t>(pr) * n_bt + bt * BG + btl) * n_ks * 64;
    ahb[pr] = uniform_bytes(reinterpret_cast<const Frag*>(a.a_hi) + t0);
    alb[pr] = uniform_bytes(reinterpret_cast<const Frag*>(a.a_lo) + t0);
  }
  auto a_off = [&](int kk) { return static_cast<uint32_t>(kk * 64 + lane) * 16u; };

  // power summed over the pulses so far: lane l holds D register (l / 2) % 16
  // of tile half l / 32 (see the reduction below)
  float total = 0.f;

  Frag ah[3], al[3];
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    ah[pr] = load_frag(ahb[pr], a_off(0));
    al[pr] = load_frag(alb[pr], a_off(0));
  }

  for (int pb = p0; pb < p1; pb += NCOL) {
    f32x16 acc[3][CTW];
#pragma unroll
    for (int pr = 0; pr < 3; ++pr)
#pragma unroll
      for (int c = 0; c < CTW; ++c)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[pr][c][i] = 0.f;
    __syncthreads();  // chunk 0 is built
    for (int ch = 0; ch < nchunks; ++ch) {
      const int b = ch & 1;
      if (cols) {
#pragma unroll
        for (int ks = 0; ks < ZKS; ++ks) {
          // the next k-step's fragments, wrapping into the next pulse block
          int kn = ch * ZKS + ks + 1;
          if (kn >= n_ks) kn -= n_ks;
#pragma unroll
          for (int pr = 0; pr < 3; ++pr) {
            Frag fbh[CTW], fbl[CTW];
#pragma unroll
            for (int c = 0; c < CTW; ++c) {
              fbh[c] = bh[b][pr][ct0 + c][ks][b_slot(ks, lane)];
              fbl[c] = bl[b][pr][ct0 + c][ks][b_slot(ks, lane)];
            }
#pragma unroll
            for (int c = 0; c < CTW; ++c) acc[pr][c] = mfma<PREC>(ah[pr], fbh[c], acc[pr][c]);
#pragma unroll
            for (int c = 0; c < CTW; ++c) acc[pr][c] = mfma<PREC>(ah[pr], fbl[c], acc[pr][c]);
#pragma unroll
            for (int c = 0; c < CTW; ++c) acc[pr][c] = mfma<PREC>(al[pr], fbh[c], acc[pr][c]);
            // refill in place right after the product's multiplies; the
            // barrier keeps the loads here (the compiler would sink them to
            // the end of the k-step, just before their next use)
            ah[pr] = load_frag(ahb[pr], a_off(kn));
            al[pr] = load_frag(alb[pr], a_off(kn));
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      __syncthreads();  // chunk ch is consumed, chunk ch + 1 is built
    }
    if (!cols) continue;
    // |Z|^2 per (bin, pulse): D register i of lane l is bin row
    // (i % 4) + 8 (i / 4) + 4 (l / 32) of the tile, column l % 32
    float pw[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) pw[i] = 0.f;
#pragma unroll
    for (int c = 0; c < CTW; ++c) {
      const int pcol = pb + 32 * (ct0 + c) + (lane & 31);
      const float un = (PREC == 1 && pcol < p1) ? ldexpf(1.f, -2 * a.col_exp[pcol]) : 1.f;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float re = acc[0][c][i] - acc[2][c][i], im = acc[0][c][i] + acc[1][c][i];
        pw[i] += fmaf(re, re, im * im) * un;
      }
    }
    // sum over the 32 pulse columns of each half wave in a fixed order,
    // scattered: xor 16, 8, 4 and 2 each halve the registers a lane keeps,
    // xor 1 adds the rest, and lane l ends with register (l / 2) % 16
    float w8[8], w4[4], w2[2];
    const bool b4 = lane & 16, b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      w8[k] = (b4 ? pw[k + 8] : pw[k]) + __shfl_xor(b4 ? pw[k] : pw[k + 8], 16);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      w4[k] = (b3 ? w8[k + 4] : w8[k]) + __shfl_xor(b3 ? w8[k] : w8[k + 4], 8);
#pragma unroll
    for (int k = 0; k < 2; ++k)
      w2[k] = (b2 ? w4[k + 2] : w4[k]) + __shfl_xor(b2 ? w4[k] : w4[k + 2], 4);
    float w1 = (b1 ? w2[1] : w2[0]) + __shfl_xor(b1 ? w2[0] : w2[1], 2);
    w1 += __shfl_xor(w1, 1);
    total += w1;
  }

  if constexpr (CG > 1) {
    // waves of the second column group hand their sums to the first (fixed order)
    if (cg == 1) red[btl][lane] = total;
    __syncthreads();
    if (cg != 0) return;
    total += red[btl][lane];
  }
  if ((lane & 1) == 0) {
    const int i = (lane >> 1) & 15, h = lane >> 5;
    float* row = a.chunks == 1
                     ? a.out + static_cast<int64_t>(g) * a.n_bins
                     : a.partial + (static_cast<int64_t>(chunk) * a.n_gates + g) * a.n_bins;
    const bool add = a.chunks == 1 && a.accumulate;
    float* dst = row + 32 * (bt * BG + btl) + (i & 3) + 8 * (i >> 2) + 4 * h;
    *dst = add ? *dst + total : total;
  }
}

// Per-pulse pass, one workgroup per pulse: FP16 exponents (exps != NULL)
// and code sign bits (bits != NULL).
__global__ void __launch_bounds__(256)
pulse_prep(const void* __restrict__ samples, int32_t sample_type, const float* __restrict__ tx,
           int64_t stride, int64_t lo, int64_t hi, int32_t code_len, int32_t tx_per_pulse,
           int32_t* __restrict__ exps, int32_t words, uint32_t* __restrict__ bits,
           int32_t* __restrict__ binary) {
  const int p = static_cast<int>(blockIdx.x);
  if (exps)
    pulse_exponent_block(samples, sample_type, tx, stride, lo, hi, code_len, tx_per_pulse, p,
                         exps);
  if (bits) code_bits_block(tx, code_len, tx_per_pulse, words, p, bits, binary);
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

hipError_t launch_zoom(const ZoomArgs& a, hipStream_t stream, bool prep) {
  int32_t* exps = a.precision == 1 ? a.col_exp : nullptr;
  if (prep && (exps || a.code_bits)) {
    hipLaunchKernelGGL(pulse_prep, dim3(static_cast<unsigned>(a.n_pulses)), dim3(256), 0, stream,
                       a.samples, a.sample_type, a.tx, a.stride, a.row_lo, a.row_hi, a.code_len,
                       a.tx_per_pulse, exps, a.code_pad / 32, a.code_bits, a.code_binary);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return a.precision == 1 ? launch_zoom_t<1>(a, stream) : launch_zoom_t<0>(a, stream);
}

}  // namespace ispl
