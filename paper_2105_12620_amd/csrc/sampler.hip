// gfx950 sampler query: sample k of screen pixel p for every dimension pair of
// a padded screen-space sampler (Sec. 3.1: dimensions are consumed in pairs,
// each pair with its own tile; Sec. 3.2: s^k_p = mod(Phi(k) d + u_p, 1) with
// the rank-1 lattice in van der Corput order).  Values are exact: Q0.16
// coordinates converted to float.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sampler_dev.h"

namespace bnlat {
namespace {

// One thread per (query, pair).
__global__ __launch_bounds__(256) void k_sample(const SamplerPair* __restrict__ pairs, uint32_t npairs,
                                                const uint32_t* __restrict__ x, const uint32_t* __restrict__ y,
                                                const uint32_t* __restrict__ k, uint32_t m, float* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (uint64_t)m * npairs) return;
  const uint32_t j = (uint32_t)(i / npairs), d = (uint32_t)(i - (uint64_t)j * npairs);
  const SamplerPair pr = pairs[d];
  const uint32_t px = x[j] % pr.w, py = y[j] % pr.h;
  const uint32_t kk = k[j] & (pr.n - 1);
  const uint32_t li = pr.log2n ? (__brev(kk) >> (32 - pr.log2n)) : 0u;
  const uint32_t l = pr.lat[li], u = pr.U[py * pr.w + px];
  const uint32_t sx = (l + u) & 0xFFFFu, sy = ((l >> 16) + (u >> 16)) & 0xFFFFu;
  const float inv = 1.0f / 65536.0f;
  out[(size_t)j * 2 * npairs + 2 * d] = (float)sx * inv;
  out[(size_t)j * 2 * npairs + 2 * d + 1] = (float)sy * inv;
}

}  // namespace

hipError_t launch_sample(const SamplerPair* pairs, uint32_t npairs, const uint32_t* x, const uint32_t* y,
                         const uint32_t* k, uint32_t m, float* out, hipStream_t s) {
  const uint64_t items = (uint64_t)m * npairs;
  if (!items) return hipSuccess;
  hipLaunchKernelGGL(k_sample, dim3((uint32_t)((items + 255) / 256)), dim3(256), 0, s, pairs, npairs, x, y, k, m,
                     out);
  return hipGetLastError();
}

}  // namespace bnlat
