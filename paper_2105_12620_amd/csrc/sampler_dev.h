// Internal interface of the sampler query kernel (the padded screen-space
// sampler a renderer reads, Sec. 3.1 and Sec. 3.2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bnlat {

// One dimension pair: its lattice, offset tile and sizes.
struct SamplerPair {
  const uint32_t* lat;   // [n] lattice points, x | y << 16, index order
  const uint32_t* U;     // [h][w] offsets, x | y << 16
  uint32_t w, h, n, log2n;
};

// out[j][2d + a] = component a of sample k[j] (van der Corput order, modulo n)
// of screen pixel (x[j] mod w, y[j] mod h) in pair d, as float in [0, 1).
// All pointers are device pointers.
hipError_t launch_sample(const SamplerPair* pairs, uint32_t npairs, const uint32_t* x, const uint32_t* y,
                         const uint32_t* k, uint32_t m, float* out, hipStream_t s);

}  // namespace bnlat
