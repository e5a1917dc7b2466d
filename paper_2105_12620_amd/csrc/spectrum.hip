// Radially averaged power spectrum of the error tile (the |FFT(e)|^2 insets
// of Fig. 1b), as a diagnostic beside the blur criterion of Sec. 3.3.  A
// direct separable DFT over the W x H torus, 64 integrand rows at a time:
// first along x (one thread per (row, frequency u, integrand)), then along y
// with |.|^2 summed over the chunk's integrands per frequency (u, v).  FP32
// twiddles and sums within a row or column, FP64 across integrands.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bnlat_dev.h"

namespace bnlat {
namespace {

constexpr uint32_t SPEC_CHUNK = 64;

__global__ __launch_bounds__(256) void k_dft_x(const float* __restrict__ field, uint32_t pitch, uint32_t valid,
                                               uint32_t t0, uint32_t w, uint32_t h,
                                               const float2* __restrict__ tw, float2* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)h * w * SPEC_CHUNK) return;
  const uint32_t j = (uint32_t)(i % SPEC_CHUNK);
  const uint32_t u = (uint32_t)((i / SPEC_CHUNK) % w), y = (uint32_t)(i / ((size_t)SPEC_CHUNK * w));
  const uint32_t t = t0 + j;
  float re = 0.0f, im = 0.0f;
  if (t < valid) {
    const float* row = field + (size_t)y * w * pitch + t;
    uint32_t k = 0;
    for (uint32_t x = 0; x < w; ++x) {
      const float e = row[(size_t)x * pitch];
      const float2 c = tw[k];
      re = fmaf(e, c.x, re);
      im = fmaf(e, c.y, im);
      k += u;
      if (k >= w) k -= w;
    }
  }
  out[i] = make_float2(re, im);
}

// One wave per frequency (u, v), lanes over the chunk's integrands.
__global__ __launch_bounds__(256) void k_dft_y_power(const float2* __restrict__ rows, uint32_t w, uint32_t h,
                                                     const float2* __restrict__ tw, double* __restrict__ power) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (wave >= w * h) return;
  const uint32_t v = wave / w, u = wave - v * w;
  float re = 0.0f, im = 0.0f;
  uint32_t k = 0;
  for (uint32_t y = 0; y < h; ++y) {
    const float2 a = rows[((size_t)y * w + u) * SPEC_CHUNK + lane];
    const float2 c = tw[k];
    re = fmaf(a.x, c.x, fmaf(-a.y, c.y, re));
    im = fmaf(a.x, c.y, fmaf(a.y, c.x, im));
    k += v;
    if (k >= h) k -= h;
  }
  double pw = (double)re * re + (double)im * im;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) pw += __shfl_xor(pw, off);
  if (lane == 0) power[wave] += pw;
}

}  // namespace

size_t spectrum_scratch_floats2(const DevView& v) { return (size_t)v.w * v.h * SPEC_CHUNK; }

hipError_t launch_spectrum_chunk(const DevView& v, const float* field, uint32_t pitch, uint32_t valid, uint32_t t0,
                                 const float2* twx, const float2* twy, float2* rows, double* power, hipStream_t s) {
  const size_t n = (size_t)v.w * v.h * SPEC_CHUNK;
  hipLaunchKernelGGL(k_dft_x, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, field, pitch, valid, t0, v.w, v.h,
                     twx, rows);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t waves = v.w * v.h;
  hipLaunchKernelGGL(k_dft_y_power, dim3((waves + 3) / 4), dim3(256), 0, s, (const float2*)rows, v.w, v.h, twy,
                     power);
  return hipGetLastError();
}

uint32_t spectrum_chunk() { return SPEC_CHUNK; }

}  // namespace bnlat
