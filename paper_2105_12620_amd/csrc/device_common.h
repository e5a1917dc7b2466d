// Device helpers shared by the gfx950 kernel sources: Philox, Q0.16
// arithmetic, tiled count indexing, the int16 dot product, colour-class
// pixel order, proposals and the window offset tables.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bnlat_dev.h"

// v_writelane_b32: write a wave-uniform value into one lane of a register.
extern "C" __device__ int bnlat_writelane_i32(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

namespace bnlat {
namespace {

typedef short v2i16 __attribute__((ext_vector_type(2)));
// Native 4 x u32 vector: kept in registers where HIP's uint4 struct is not.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));


// Philox4x32-10 (Salmon et al., SC 2011): two 32x32->64 products per round,
// key advanced by the Weyl constants between rounds.  Returns words 0 and 1.
__device__ inline uint2 philox_w01(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                   uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return make_uint2(c0, c1);
}

// Q0.16 pair from the top halves of words 0 and 1.
__device__ inline uint32_t q16_pair(uint2 w) { return (w.x >> 16) | (w.y & 0xFFFF0000u); }

// Componentwise (a + b) mod 2^16 of two packed Q0.16 pairs: the toroidal
// shift mod(s + u, 1) of Sec. 3.2.
__device__ inline uint32_t wrap_add(uint32_t a, uint32_t b) {
  return ((a + b) & 0xFFFFu) | (((a >> 16) + (b >> 16)) << 16);
}

// S - 2^15 per component, as two int16.
__device__ inline uint32_t centre(uint32_t s) { return s ^ 0x80008000u; }

// Element (row, t) of a tiled count buffer with `rows` rows.
__device__ inline size_t tix(uint32_t row, uint32_t t, uint32_t rows) {
  return ((size_t)(t >> 3) * rows + row) * 8 + (t & 7);
}

// Signed int16x2 dot product plus accumulator (v_dot2_i32_i16).  The clamp
// bit keeps the three-operand encoding; it never engages because every
// product sum here stays below 2^31 in magnitude.
__device__ inline int dot2(uint32_t a, uint32_t b, int c) {
  return __builtin_amdgcn_sdot2(__builtin_bit_cast(v2i16, a), __builtin_bit_cast(v2i16, b), c, true);
}

__device__ inline uint32_t wave_id() {
  return __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

// Workgroup barrier of the kernels that fill LDS with global_load_lds: waits
// until at most N of this wave's vector-memory loads are in flight (they
// complete in order, so every earlier one has landed) and its LDS accesses
// are done, then meets the other waves (a __syncthreads would also wait for
// the loads still meant to be in flight).  The empty asm statements keep the
// compiler from moving memory accesses across.  s_waitcnt immediate in the
// gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt (bits 6:4) left open,
// lgkmcnt (bits 11:8) zero.
template <int N>
__device__ inline void barrier_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt");
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Workgroups go to the eight XCDs in turn (workgroup b to XCD b mod 8), each
// with its own L2.  This renumbers them so that every XCD's workgroups form one
// contiguous range of logical indices: neighbouring work then shares an L2.
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t g) {
  const uint32_t x = b & 7, i = b >> 3, q = g >> 3, r = g & 7;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

__device__ inline uint32_t class_pixel(const DevView& v, uint32_t kappa, uint32_t j) {
  const uint32_t ky = kappa / v.k, kx = kappa - ky * v.k;
  const uint32_t a = j / v.cw, b = j - a * v.cw;
  return (ky + v.k * a) * v.w + (kx + v.k * b);
}

__device__ inline uint32_t proposal(const DevView& v, uint32_t p, uint32_t sweep) {
  return q16_pair(philox_w01(p, sweep, v.problem, S_PROP, v.seed_lo, v.seed_hi));
}

// ------------------------------------------------- BF16 error field values

// Round to the nearest BF16 (ties to even); bits of two values packed.
__device__ inline uint32_t bf16x2_bits(float lo, float hi) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)lo) | ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)hi) << 16);
}

// Field value of 8 Heaviside counts (one 16-byte count tile) in either mode.
__device__ inline uint4 heaviside_field_tile(const DevView& v, const uint4 c8, uint32_t t) {
  const uint32_t w[4] = {c8.x, c8.y, c8.z, c8.w};
  uint32_t o[4];
  const float inv_n = 1.0f / (float)v.n;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float c0 = (float)(w[k] & 0xFFFFu), c1 = (float)(w[k] >> 16);
    if (v.mfma == 1) {
      o[k] = bf16x2_bits(c0, c1);
    } else {
      o[k] = bf16x2_bits(__fsub_rn(__fmul_rn(c0, inv_n), v.area[t + 2 * k]),
                         __fsub_rn(__fmul_rn(c1, inv_n), v.area[t + 2 * k + 1]));
    }
  }
  return make_uint4(o[0], o[1], o[2], o[3]);
}

// Field value of Gaussian row t (FP32 estimate g): g - I rounded to FP32,
// then to BF16 by the caller; padded rows are 0.
__device__ inline float gaussian_error(const DevView& v, float g, uint32_t t) {
  return t < v.tg ? (float)((double)g - v.gint[t]) : 0.0f;
}

// --------------------------------------------------------- window tables

// Offsets of the (2R+1)^2 - 1 window grouped by squared distance d in
// increasing d (row-major inside a group), with their group index.
template <int R>
struct Window {
  static constexpr int M = (2 * R + 1) * (2 * R + 1) - 1;
  static constexpr int DMAX = 2 * R * R;
  int ox[M], oy[M], cls[M];
  int ncls;
  int d[DMAX + 1], csize[DMAX + 1];
  int cmap[(2 * R + 1) * (2 * R + 1)];   // group of offset (x, y) at (y + R)(2R + 1) + x + R; -1 at (0, 0)
  constexpr Window() : ox(), oy(), cls(), ncls(0), d(), csize(), cmap() {
    int idx = 0;
    for (int dd = 1; dd <= DMAX; ++dd) {
      int found = 0;
      for (int y = -R; y <= R; ++y)
        for (int x = -R; x <= R; ++x)
          if (x * x + y * y == dd) {
            ox[idx] = x;
            oy[idx] = y;
            cls[idx] = ncls;
            cmap[(y + R) * (2 * R + 1) + x + R] = ncls;
            ++idx;
            ++found;
          }
      if (found) {
        d[ncls] = dd;
        csize[ncls] = found;
        ++ncls;
      }
    }
    cmap[R * (2 * R + 1) + R] = -1;
  }
};

template <int R>
struct WinConst {
  static constexpr Window<R> w{};
  static constexpr int NCLS = w.ncls;
};

// Member of a batch that owns launch block blk (prefix sums of blocks per member).
__device__ inline uint32_t batch_member(const uint32_t* __restrict__ pre, uint32_t nmem, uint32_t blk) {
  uint32_t i = 0;
  while (i + 1 < nmem && pre[i + 1] <= blk) ++i;
  return __builtin_amdgcn_readfirstlane(i);
}

}  // namespace
}  // namespace bnlat
