// Attainable peaks of the device, measured with plain loops, so that a
// kernel's roofline fraction can be stated against what this GPU delivers
// as well as against the vendor figures:
//   - HBM: a device-to-device copy of a large buffer (16-byte loads/stores);
//   - vector ALU: independent chains of v_dot2_i32_i16 (the counting
//     kernel's instruction), one lane-operation each;
//   - matrix cores: independent v_mfma_f32_32x32x16_bf16 accumulations.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bnlat_dev.h"
#include "device_common.h"

namespace bnlat {
namespace {

__global__ __launch_bounds__(256) void k_peak_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                   size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// CH independent dot2 chains per lane; the saturating form keeps the compiler
// from folding a chain into one multiply.
constexpr int CH = 8;
__global__ __launch_bounds__(256) void k_peak_dot2(int* __restrict__ out, uint32_t iters) {
  const uint32_t x = 0x00030001u * (threadIdx.x + 1);
  int acc[CH];
  uint32_t y[CH];
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    acc[k] = k;
    y[k] = 0x00010002u * (uint32_t)(k + 1) ^ threadIdx.x;
  }
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < CH; ++k) acc[k] = dot2(x, y[k], acc[k]);
  }
  int s = 0;
#pragma unroll
  for (int k = 0; k < CH; ++k) s ^= acc[k];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// four independent 32x32 accumulators per wave
__global__ __launch_bounds__(256) void k_peak_mfma(float* __restrict__ out, uint32_t iters) {
  bf16x8 a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(float)((threadIdx.x + i) & 7);
    b[i] = (__bf16)(float)((i * 3 + threadIdx.x) & 7);
  }
  f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (uint32_t it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b, a, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, a, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b, b, c3, 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += (c0[i] + c1[i]) + (c2[i] + c3[i]);
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

hipError_t peak_launch(int kind, void* buf, void* buf2, uint64_t size, uint32_t iters, uint32_t blocks,
                       hipStream_t s) {
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(k_peak_copy, dim3(blocks), dim3(256), 0, s, (const uint4*)buf, (uint4*)buf2,
                         (size_t)(size / 16));
      break;
    case 1: hipLaunchKernelGGL(k_peak_dot2, dim3(blocks), dim3(256), 0, s, (int*)buf, iters); break;
    case 2: hipLaunchKernelGGL(k_peak_mfma, dim3(blocks), dim3(256), 0, s, (float*)buf, iters); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace bnlat
