// Device memory of ispl_integrate_spectra_noalloc, the entry point that
// allocates nothing: its twiddle table and its pulse-chunk partial spectra live
// in one file-scope device array instead of context-owned allocations.  The
// array is part of the library's code object, so every GPU the library runs on
// holds its own copy until the process ends.
//
// Layout of the array (ISPL_NOALLOC_SCRATCH_BYTES):
//   [0, 512 KiB)        twiddle table W_N^i, i < N <= 65536, complex64
//   [512 KiB, end)      chunk partials [C][G][N] float32 (64 MiB)

#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>

#include "ispl_internal.h"

static __device__ __align__(256) unsigned char scratch[ISPL_NOALLOC_SCRATCH_BYTES];

namespace ispl {
namespace {

// W_N^i = exp(-2 pi i / N)^i for i < N, computed as the context's table is:
// double-precision cos/sin of an angle in the first octant of its quadrant,
// the other octant and the quadrant by exact symmetries, then rounded to float.
__global__ void __launch_bounds__(256) build_twiddles(float* __restrict__ table, int32_t n) {
  const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  const int32_t quarter = n / 4, eighth = n / 8;
  const int32_t qd = i / quarter;
  const int32_t rem = i - qd * quarter;
  double c, s;  // cos, sin of 2 pi rem / N
  if (rem <= eighth) {
    const double th = 2.0 * M_PI * rem / n;
    c = cos(th);
    s = sin(th);
  } else {
    const double th = 2.0 * M_PI * (quarter - rem) / n;
    c = sin(th);
    s = cos(th);
  }
  double ci, si;  // cos, sin of 2 pi i / N
  switch (qd) {
    case 0: ci = c; si = s; break;
    case 1: ci = -s; si = c; break;
    case 2: ci = -c; si = -s; break;
    default: ci = s; si = -c; break;
  }
  table[2 * i] = static_cast<float>(ci);
  table[2 * i + 1] = static_cast<float>(-si);
}

constexpr int kMaxDevices = 64;

}  // namespace

hipError_t noalloc_scratch(int device, unsigned char** base) {
  static std::mutex mu;
  static unsigned char* ptrs[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[device]) {
    // The caller has made `device` current.  The array's name is a host-side
    // stand-in; the device address of this GPU's copy comes from the runtime.
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptrs[device] = static_cast<unsigned char*>(p);
  }
  *base = ptrs[device];
  return hipSuccess;
}

hipError_t launch_build_twiddles(float* table, int32_t n_fft, hipStream_t stream) {
  hipLaunchKernelGGL(build_twiddles, dim3(static_cast<unsigned>((n_fft + 255) / 256)), dim3(256), 0,
                     stream, table, n_fft);
  return hipGetLastError();
}

}  // namespace ispl
