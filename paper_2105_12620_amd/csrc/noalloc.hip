// Library-resident scratch of the allocation-free entry point
// (bn_delta_energy_noalloc): one fixed device array per GPU, located once per
// device with hipGetSymbolAddress, plus the kernel that lays recounted hits
// out as host rows.  Nothing here allocates device memory.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "bnlat_dev.h"

namespace bnlat {
namespace {

// The scratch array.  In host code this name is only a stand-in for the
// symbol: kernels and copies must use the address hipGetSymbolAddress returns
// for the current device, never the name itself.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// Tiled counts [tp/8][rows][8] -> rows [rows][t] (one thread per entry).
__global__ __launch_bounds__(256) void k_untile_counts(const uint16_t* __restrict__ tiled, uint32_t rows,
                                                       uint32_t t, uint16_t* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (uint64_t)rows * t) return;
  const uint32_t r = (uint32_t)(i / t), c = (uint32_t)(i - (uint64_t)r * t);
  out[i] = tiled[((size_t)(c >> 3) * rows + r) * 8 + (c & 7)];
}

}  // namespace

hipError_t noalloc_scratch(int device, void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (!ptr || device < 0 || device >= kMaxDevices) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    addr[device] = a;
  }
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t launch_untile_counts(const uint16_t* tiled, uint32_t rows, uint32_t t, uint16_t* out, hipStream_t s) {
  const uint64_t n = (uint64_t)rows * t;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_untile_counts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tiled, rows, t, out);
  return hipGetLastError();
}

}  // namespace bnlat
