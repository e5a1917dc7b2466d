// gfx950 hit-counting kernels: the estimator of the test-integrand map
// (Sec. 2) for every pixel (bn_compute_errors), for the proposals of one
// colour class, of a pixel list, or of a whole sweep (the overlapped
// schedule), plus their batched form.
//
// Counts land in the tiled layout uint16 [Tp/8][rows][8]; the Heaviside
// predicate n.(S - 2^15) > D' is an exact int16 dot product against an int32
// threshold on Q0.16 sample coordinates.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "bnlat_dev.h"
#include "device_common.h"

namespace bnlat {
namespace {

// Resolve the pixel, offset and output buffer (row index, row count) of work
// item j of a count launch.
template <int MODE>
__device__ inline void count_target(const DevView& v, uint32_t kappa, uint32_t j, uint32_t m,
                                    uint32_t& p, uint32_t& u, uint16_t*& buf, uint32_t& row,
                                    uint32_t& rows) {
  if (MODE == MODE_ALL) {
    p = j;
    u = v.U[p];
    buf = v.cnt;
    row = p;
    rows = v.w * v.h;
  } else if (MODE == MODE_CLASS) {
    p = class_pixel(v, kappa, j);
    u = proposal(v, p, (uint32_t)v.ctr[0]);
    buf = v.c_new;
    row = j;
    rows = v.pc;
  } else if (MODE == MODE_SWEEP) {
    const uint32_t cls = j / v.pc, jj = j - cls * v.pc;
    p = class_pixel(v, cls, jj);
    u = proposal(v, p, (uint32_t)v.ctr[0] + kappa);
    buf = v.c_new + (size_t)cls * v.pc * v.tp;
    row = jj;
    rows = v.pc;
  } else {
    p = v.pix_list[j];
    u = v.u_new[j];
    buf = v.c_new;
    row = j;
    rows = m;
  }
}

// ----------------------------------------------------------- hit counting
//
// Estimator of the test-integrand map (Sec. 2): c[p][t] = number of the N
// scrambled samples on the hit side of Heaviside t.
//
// k_count_points (N >= 128): the 64 lanes of a wave hold 64*PPL samples of one
// pixel (PPL per lane); the wave walks integrands with wave-uniform
// parameters in scalar registers.  Per (sample, integrand): one v_dot2 and
// one v_cmp; the 64 predicate bits of a compare are counted with a scalar
// popcount.  Counts for 64 consecutive integrands are gathered one per lane
// and stored as one coalesced 128-byte row segment.  N > 64*PPL is handled
// in groups of 64*PPL samples.
template <int PPL, int MODE>
__device__ __forceinline__ void count_points_body(const DevView& v, const int2* __restrict__ ihp,
                                                  uint32_t kappa, uint32_t m, uint32_t tch,
                                                  uint32_t blk) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(blk * 4 + (threadIdx.x >> 6));
  const uint32_t nch = (v.tp + tch - 1) / tch;
  const uint32_t j = wave / nch, ch = wave - j * nch;
  if (j >= m) return;
  uint32_t p, u, row, rows;
  uint16_t* buf;
  count_target<MODE>(v, kappa, j, m, p, u, buf, row, rows);
  if ((MODE == MODE_CLASS || MODE == MODE_SWEEP) && ch == 0 && lane == 0) v.u_new[j] = u;

  const uint32_t groups = v.n / (64u * PPL);
  uint32_t sp[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) sp[k] = centre(wrap_add(v.lat[lane + 64 * k], u));
  const float inv_n = 1.0f / (float)v.n;
  const uint32_t t0 = ch * tch, t1 = min(t0 + tch, v.tp);
  for (uint32_t tb = t0; tb < t1; tb += 64) {
    int total = 0;
    if (tb < v.t) {
      for (uint32_t g = 0; g < groups; ++g) {
        if (groups > 1) {
#pragma unroll
          for (int k = 0; k < PPL; ++k)
            sp[k] = centre(wrap_add(v.lat[g * 64 * PPL + lane + 64 * k], u));
        }
        // one integrand per step: PPL dot products and compares on the
        // vector ALU, popcounts and adds on the scalar ALU, and the count
        // written into lane tt
        int myc = 0;
        const int4* ip = (const int4*)(ihp + tb);
#pragma unroll 1
        for (int blk = 0; blk < 8; ++blk) {
          // eight integrands' parameters in one scalar load
          const int4 q0 = ip[4 * blk], q1 = ip[4 * blk + 1], q2 = ip[4 * blk + 2], q3 = ip[4 * blk + 3];
          const int nn[8] = {q0.x, q0.z, q1.x, q1.z, q2.x, q2.z, q3.x, q3.z};
          const int dd[8] = {q0.y, q0.w, q1.y, q1.w, q2.y, q2.w, q3.y, q3.w};
#pragma unroll
          for (int k8 = 0; k8 < 8; ++k8) {
            int c = 0;
#pragma unroll
            for (int k = 0; k < PPL; ++k)
              c += __popcll(__ballot(dot2((uint32_t)nn[k8], sp[k], 0) > dd[k8]));
            myc = bnlat_writelane_i32(c, 8 * blk + k8, myc);
          }
        }
        total += myc;
      }
    }
    buf[tix(row, tb + lane, rows)] = (uint16_t)total;
    if (MODE == MODE_ALL)
      v.err[(size_t)p * v.tp + tb + lane] = (float)total * inv_n - v.area[tb + lane];
  }
}

// The launch may have fewer workgroups than the vblocks its work needs (the
// sweep-wide recount of the overlapped schedule is capped so that it leaves
// room on every CU for the colour phases running beside it): workgroups then
// stride over the virtual blocks.
//
// Eight waves per SIMD: the compiler then keeps the compare masks in VCC and
// a few scalar registers (72 instead of 100, which allowed seven waves); the
// sweep-wide recount measured 11 % faster so.
template <int PPL, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_count_points(
    DevView v, const int2* __restrict__ ihp, uint32_t kappa, uint32_t m, uint32_t tch, uint32_t vblocks) {
  for (uint32_t b = blockIdx.x; b < vblocks; b += gridDim.x) count_points_body<PPL, MODE>(v, ihp, kappa, m, tch, b);
}

template <int PPL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_count_points_batch(
    const DevView* __restrict__ views, const uint32_t* __restrict__ pre, uint32_t nmem, uint32_t kappa) {
  const uint32_t i = batch_member(pre, nmem, blockIdx.x);
  const DevView v = views[i];
  count_points_body<PPL, MODE_CLASS>(v, v.ihp, kappa, v.pc, v.tch, blockIdx.x - pre[i]);
}

// k_count_pixels (N <= 64): lanes hold 64 consecutive work items (pixels or
// proposals), each with its N samples in registers; a wave walks 64
// integrands with wave-uniform parameters from scalar loads and, per 8
// integrands, stores each lane's 8 counts as one 16-byte tile piece.  Per
// two (sample, integrand) pairs: two v_dot2 (threshold folded in), two shifts
// and one three-way add.
template <int NS, int MODE>
__device__ __forceinline__ void count_pixels_body(const DevView& v, uint32_t kappa, uint32_t m, uint32_t blk) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(blk * 4 + (threadIdx.x >> 6));
  const uint32_t nch = v.tp >> 6;
  const uint32_t jg = wave / nch, ch = wave - jg * nch;
  const uint32_t j = jg * 64 + lane;
  if (jg * 64 >= m || j >= m) return;
  uint32_t p, u, row, rows;
  uint16_t* buf;
  count_target<MODE>(v, kappa, j, m, p, u, buf, row, rows);
  if ((MODE == MODE_CLASS || MODE == MODE_SWEEP) && ch == 0) v.u_new[j] = u;
  uint32_t sp[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) sp[k] = centre(wrap_add(v.lat[k], u));
  const float inv_n = 1.0f / (float)NS;
  const int4* ip = (const int4*)(v.ihp + ch * 64);
#pragma unroll 1
  for (int tt = 0; tt < 8; ++tt) {
    const int4 q0 = ip[4 * tt], q1 = ip[4 * tt + 1], q2 = ip[4 * tt + 2], q3 = ip[4 * tt + 3];
    const int nn[8] = {q0.x, q0.z, q1.x, q1.z, q2.x, q2.z, q3.x, q3.z};
    const int dd[8] = {q0.y, q0.w, q1.y, q1.w, q2.y, q2.w, q3.y, q3.w};
    // n.s > D' exactly when r = n.s - D' - 1 >= 0 (|n.s|, |D'| <= 2^30, so r
    // never overflows): misses are the sign bits, summed three at a time
    uint32_t c[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int thr = -dd[i] - 1;
      uint32_t miss = 0;
#pragma unroll
      for (int k = 0; k < NS; k += 2) {
        const uint32_t r0 = (uint32_t)dot2((uint32_t)nn[i], sp[k], thr) >> 31;
        const uint32_t r1 = k + 1 < NS ? (uint32_t)dot2((uint32_t)nn[i], sp[k + 1], thr) >> 31 : 0u;
        miss = miss + r0 + r1;
      }
      c[i] = NS - miss;
    }
    const uint32_t t = ch * 64 + 8 * tt;
    *(uint4*)(buf + tix(row, t, rows)) =
        make_uint4(c[0] | (c[1] << 16), c[2] | (c[3] << 16), c[4] | (c[5] << 16), c[6] | (c[7] << 16));
    if (MODE == MODE_ALL) {
      float* e = v.err + (size_t)p * v.tp + t;
#pragma unroll
      for (int i = 0; i < 8; ++i) e[i] = (float)c[i] * inv_n - v.area[t + i];
    }
  }
}

template <int NS, int MODE>
__global__ __launch_bounds__(256) void k_count_pixels(DevView v, uint32_t kappa, uint32_t m) {
  count_pixels_body<NS, MODE>(v, kappa, m, blockIdx.x);
}

template <int NS>
__global__ __launch_bounds__(256) void k_count_pixels_batch(const DevView* __restrict__ views,
                                                            const uint32_t* __restrict__ pre, uint32_t nmem,
                                                            uint32_t kappa) {
  const uint32_t i = batch_member(pre, nmem, blockIdx.x);
  const DevView v = views[i];
  count_pixels_body<NS, MODE_CLASS>(v, kappa, v.pc, blockIdx.x - pre[i]);
}

// waves of a k_count_pixels launch over m work items
inline uint64_t count_pixel_waves(const DevView& v, uint32_t m) { return (uint64_t)((m + 63) / 64) * (v.tp >> 6); }

template <int MODE>
hipError_t count_dispatch(const DevView& v, uint32_t kappa, uint32_t m, hipStream_t s) {
  if (m == 0) return hipSuccess;
  if (v.n <= 64) {
    const dim3 g((unsigned)((count_pixel_waves(v, m) + 3) / 4)), b(256);
    switch (v.n) {
      case 1: hipLaunchKernelGGL((k_count_pixels<1, MODE>), g, b, 0, s, v, kappa, m); break;
      case 2: hipLaunchKernelGGL((k_count_pixels<2, MODE>), g, b, 0, s, v, kappa, m); break;
      case 4: hipLaunchKernelGGL((k_count_pixels<4, MODE>), g, b, 0, s, v, kappa, m); break;
      case 8: hipLaunchKernelGGL((k_count_pixels<8, MODE>), g, b, 0, s, v, kappa, m); break;
      case 16: hipLaunchKernelGGL((k_count_pixels<16, MODE>), g, b, 0, s, v, kappa, m); break;
      case 32: hipLaunchKernelGGL((k_count_pixels<32, MODE>), g, b, 0, s, v, kappa, m); break;
      case 64: hipLaunchKernelGGL((k_count_pixels<64, MODE>), g, b, 0, s, v, kappa, m); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  // integrands per wave: v.tch (whole rows at T <= 1024 by default: the
  // proposal and samples are set up once per wave), halved while the launch
  // would hold fewer than 8192 waves
  uint32_t tch = v.tch;
  while (tch > 64 && (uint64_t)m * ((v.tp + tch - 1) / tch) < 8192) tch >>= 1;
  const uint64_t waves = (uint64_t)m * ((v.tp + tch - 1) / tch);
  const uint32_t vb = (uint32_t)((waves + 3) / 4);
  const uint32_t nb = (MODE == MODE_SWEEP && v.count_cap) ? std::min(vb, v.count_cap) : vb;
  const dim3 grid(nb), block(256);
  switch (v.n) {
    case 128: hipLaunchKernelGGL((k_count_points<2, MODE>), grid, block, 0, s, v, v.ihp, kappa, m, tch, vb); break;
    // N >= 256: four samples per lane, N / 256 sample groups (more samples
    // per lane would keep more compare masks live than the scalar registers
    // hold, and the spills cost more than the group reloads)
    default: hipLaunchKernelGGL((k_count_points<4, MODE>), grid, block, 0, s, v, v.ihp, kappa, m, tch, vb); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_count(const DevView& v, int mode, uint32_t kappa, uint32_t m, hipStream_t s) {
  switch (mode) {
    case MODE_ALL: return count_dispatch<MODE_ALL>(v, kappa, m, s);
    case MODE_CLASS: return count_dispatch<MODE_CLASS>(v, kappa, m, s);
    case MODE_SWEEP: return count_dispatch<MODE_SWEEP>(v, kappa, m, s);
    default: return count_dispatch<MODE_LIST>(v, kappa, m, s);
  }
}

// Launch kind of a batch member's recount: N itself up to 64 (one kernel per
// N), 64 + samples per lane above.
int count_kind(const DevView& v) {
  if (v.n <= 64) return (int)v.n;
  return v.n == 128 ? 66 : 68;
}

uint32_t count_blocks(const DevView& v) {
  if (v.n <= 64) return (uint32_t)((count_pixel_waves(v, v.pc) + 3) / 4);
  const uint64_t waves = (uint64_t)v.pc * ((v.tp + v.tch - 1) / v.tch);
  return (uint32_t)((waves + 3) / 4);
}

hipError_t launch_count_batch(int kind, const DevView* views, const uint32_t* pre, uint32_t nmem,
                              uint32_t blocks, uint32_t kappa, hipStream_t s) {
  const dim3 grid(blocks), block(256);
  switch (kind) {
    case 1: hipLaunchKernelGGL(k_count_pixels_batch<1>, grid, block, 0, s, views, pre, nmem, kappa); break;
    case 2: hipLaunchKernelGGL(k_count_pixels_batch<2>, grid, block, 0, s, views, pre, nmem, kappa); break;
    case 4: hipLaunchKernelGGL(k_count_pixels_batch<4>, grid, block, 0, s, views, pre, nmem, kappa); break;
    case 8: hipLaunchKernelGGL(k_count_pixels_batch<8>, grid, block, 0, s, views, pre, nmem, kappa); break;
    case 16: hipLaunchKernelGGL(k_count_pixels_batch<16>, grid, block, 0, s, views, pre, nmem, kappa); break;
    case 32: hipLaunchKernelGGL(k_count_pixels_batch<32>, grid, block, 0, s, views, pre, nmem, kappa); break;
    case 64: hipLaunchKernelGGL(k_count_pixels_batch<64>, grid, block, 0, s, views, pre, nmem, kappa); break;
    case 66: hipLaunchKernelGGL(k_count_points_batch<2>, grid, block, 0, s, views, pre, nmem, kappa); break;
    case 68: hipLaunchKernelGGL(k_count_points_batch<4>, grid, block, 0, s, views, pre, nmem, kappa); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace bnlat
