// gfx950 kernels of the swap mutation (Sec. 3.4, with the pixel permutation
// of Sec. 2): the tile is optimised by exchanging the offsets of couples of
// pixels.  A couple's hit-count vectors move with its offsets, so a pass is a
// pure neighbourhood evaluation with no recount.
//
// The couple (a, b) changes the windowed energy of Eq. (1) by the two single
// moves c_a -> c_b and c_b -> c_a evaluated on the unmodified state plus a
// pair correction.  With dc = c_b - c_a, in exact integers per distance class d:
//   X_d = -2 sum_{o in d} sum_t dc_t (c_{a+o,t} - c_{b+o,t})  +  2 m_d sum_t dc_t^2,
// where m_d counts the offsets o of class d with a + o = b on the torus (the
// terms |d| (c_b^2 - c_a^2) of the two single moves cancel).  Then
//   dE = (2 / N^2) sum_d w(d) X_d,
// summed in FP64 in increasing d exactly as for the redraw mutation.
//
// During a swap sweep the counts live in a pixel-major copy cpm [P][tp], so a
// wave reads a neighbour's 256 integrands as one 512-byte run.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "bnlat_dev.h"
#include "device_common.h"
#include "swap_dev.h"

namespace bnlat {
namespace {

// XOR mask of pass kappa of the sweep in the device counter.
__device__ inline uint32_t swap_mask(const DevView& v, uint32_t kappa) {
  const uint32_t sweep = (uint32_t)v.ctr[0];
  return philox_w01(kappa, sweep, v.problem, S_SWAP, v.seed_lo, v.seed_hi).x & (v.w * v.h - 1);
}

// One thread per 16-byte integrand tile of a pixel.
__global__ __launch_bounds__(256) void k_to_pixel_major(DevView v, SwapView sv) {
  const uint32_t P = v.w * v.h, tiles = v.tp >> 3;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)P * tiles) return;
  const uint32_t tt = (uint32_t)(i / P), p = (uint32_t)(i - (size_t)tt * P);
  *(uint4*)(sv.cpm + (size_t)p * v.tp + 8 * tt) = *(const uint4*)(v.cnt + i * 8);
}

__global__ __launch_bounds__(256) void k_from_pixel_major(DevView v, SwapView sv) {
  const uint32_t P = v.w * v.h, tiles = v.tp >> 3;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)P * tiles) return;
  const uint32_t tt = (uint32_t)(i / P), p = (uint32_t)(i - (size_t)tt * P);
  *(uint4*)(v.cnt + i * 8) = *(const uint4*)(sv.cpm + (size_t)p * v.tp + 8 * tt);
}

__global__ void k_swap_reset(SwapView sv) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *sv.nsel = 0;
}

// Every pixel p of the tile tests whether its scrambled list position
// pinv[p ^ mask] falls in the pass; members are appended (wave by wave, in
// roughly raster order) to order[] as list slots j = L - kappa M.
__global__ __launch_bounds__(256) void k_swap_select(DevView v, SwapView sv, uint32_t kappa) {
  const uint32_t P = v.w * v.h;
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t mask = swap_mask(v, kappa);
  bool in = false;
  uint32_t j = 0;
  if (p < P) {
    const uint32_t L = sv.pinv[p ^ mask];
    in = L / sv.m == kappa;
    j = L - kappa * sv.m;
  }
  const unsigned long long bal = __ballot(in);
  const uint32_t rank = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
  uint32_t base = 0;
  if (lane == 0 && bal) base = atomicAdd(sv.nsel, (uint32_t)__popcll(bal));
  base = __shfl(base, 0);
  if (in && base + rank < sv.m) sv.order[base + rank] = j;
}

// One wave per couple member (list slot j) and integrand slice: lanes hold 4
// integrands each of dc = c_partner - c_own and take the int16 dot products
// with the 4 counts of every window neighbour of the member (one 512-byte run
// per neighbour and 256 integrands).  Per-lane partial sums of one chunk stay
// below 2^31 (at most 12 offsets per class x 4 integrands x N^2, N <= 4096)
// and are widened to 64 bits after each chunk; slices meet in exact int64
// atomics.
//
// Launch order: hardware workgroup i runs on XCD i mod 8, so XCD x is given
// the contiguous run of member blocks [x nbx, (x + 1) nbx) and walks it once
// per integrand slice; its L2 then holds the window rows of one band of the
// tile for one slice.
template <int R>
__global__ __launch_bounds__(256) void k_swap_eval(DevView v, SwapView sv, uint32_t kappa, uint32_t nbx,
                                                   uint32_t nz, uint32_t tslice) {
  constexpr Window<R> W = WinConst<R>::w;
  constexpr int NCLS = WinConst<R>::NCLS;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
  const uint32_t z = q / nbx, mb = xcd * nbx + (q - z * nbx);
  const uint32_t slot = mb * 4 + (threadIdx.x >> 6);
  if (z >= nz || slot >= sv.m) return;
  const uint32_t j = __builtin_amdgcn_readfirstlane(sv.order[slot]);
  if (j >= sv.m) return;
  const uint32_t mask = swap_mask(v, kappa);
  const uint32_t L = kappa * sv.m + j;
  const uint32_t a = sv.perm[L] ^ mask, b = sv.perm[L ^ 1u] ^ mask;
  const uint32_t y = a / v.w, x = a - y * v.w;
  uint32_t rowq[2 * R + 1], colq[2 * R + 1];
#pragma unroll
  for (int i = 0; i < 2 * R + 1; ++i) {
    rowq[i] = ((y + v.h + i - R) % v.h) * v.w;
    colq[i] = (x + v.w + i - R) % v.w;
  }
  long long zd[NCLS];
#pragma unroll
  for (int c = 0; c < NCLS; ++c) zd[c] = 0;
  long long dd = 0;
  const uint32_t t_begin = z * tslice, t_end = min(t_begin + tslice, v.tp);
  for (uint32_t t0 = t_begin; t0 < t_end; t0 += 256) {
    const uint32_t t = t0 + 4 * lane;
    if (t >= t_end) continue;
    const uint2 ca = *(const uint2*)(sv.cpm + (size_t)a * v.tp + t);
    const uint2 cb = *(const uint2*)(sv.cpm + (size_t)b * v.tp + t);
    const uint32_t aw[2] = {ca.x, ca.y}, bw[2] = {cb.x, cb.y};
    uint32_t dl[2];
    int sq = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int d0 = (int)(bw[k] & 0xFFFFu) - (int)(aw[k] & 0xFFFFu);
      const int d1 = (int)(bw[k] >> 16) - (int)(aw[k] >> 16);
      dl[k] = ((uint32_t)d0 & 0xFFFFu) | ((uint32_t)d1 << 16);
      sq = dot2(dl[k], dl[k], sq);
    }
    dd += sq;
    int part[NCLS];
#pragma unroll
    for (int c = 0; c < NCLS; ++c) part[c] = 0;
#pragma unroll
    for (int mm = 0; mm < W.M; ++mm) {
      const uint32_t qq = rowq[W.oy[mm] + R] + colq[W.ox[mm] + R];
      const uint2 cq = *(const uint2*)(sv.cpm + (size_t)qq * v.tp + t);
      int acc = part[W.cls[mm]];
      acc = dot2(dl[0], cq.x, acc);
      acc = dot2(dl[1], cq.y, acc);
      part[W.cls[mm]] = acc;
    }
#pragma unroll
    for (int c = 0; c < NCLS; ++c) zd[c] += part[c];
  }
#pragma unroll
  for (int c = 0; c < NCLS; ++c) {
    long long s = zd[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0 && s) atomicAdd((unsigned long long*)&sv.xs[(size_t)c * sv.m + j], (unsigned long long)(-2 * s));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dd += __shfl_xor(dd, off);
  if (lane == 0 && !(j & 1u) && dd) atomicAdd((unsigned long long*)&sv.d2[j >> 1], (unsigned long long)dd);
}

// One thread per couple: add the two members' class sums and the pair
// correction, take the FP64 weighted sum in increasing d and decide; the sums
// are cleared for the next pass.
__global__ __launch_bounds__(256) void k_swap_finish(DevView v, SwapView sv, uint32_t kappa) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t half = sv.m >> 1;
  if (i >= half) return;
  const uint32_t mask = swap_mask(v, kappa);
  const uint32_t L = kappa * sv.m + 2 * i;
  const uint32_t a = sv.perm[L] ^ mask, b = sv.perm[L + 1] ^ mask;
  const uint32_t ay = a / v.w, ax = a - ay * v.w, by = b / v.w, bx = b - by * v.w;
  // offsets o with a + o = b: at most two per axis because r < min(W, H)
  int l0 = -1, l1 = -1, l2 = -1, l3 = -1;
  const int r = (int)v.radius;
  for (int oy = -r; oy <= r; ++oy) {
    if ((ay + v.h + oy) % v.h != by) continue;
    for (int ox = -r; ox <= r; ++ox) {
      if ((ox == 0 && oy == 0) || (ax + v.w + ox) % v.w != bx) continue;
      const int cl = sv.dcls[ox * ox + oy * oy];
      if (l0 < 0) l0 = cl;
      else if (l1 < 0) l1 = cl;
      else if (l2 < 0) l2 = cl;
      else l3 = cl;
    }
  }
  const long long d2 = sv.d2[i];
  sv.d2[i] = 0;
  double acc = 0.0;
  for (uint32_t c = 0; c < v.ncls; ++c) {
    const int ci = (int)c;
    long long* xp = sv.xs + (size_t)c * sv.m + 2 * i;
    long long x = xp[0] + xp[1];
    xp[0] = 0;
    xp[1] = 0;
    x += 2 * d2 * (long long)((l0 == ci) + (l1 == ci) + (l2 == ci) + (l3 == ci));
    acc = __dadd_rn(acc, __dmul_rn(v.wd[c], (double)x));
  }
  const double total = __dmul_rn(acc, 2.0 / ((double)v.n * (double)v.n));
  v.delta[i] = total;
  v.accept[i] = (v.objective > 0) ? (total < 0.0) : (total > 0.0);
  v.u_new[2 * i] = a;
  v.u_new[2 * i + 1] = b;
}

// One wave per accepted couple: exchange offsets and count rows.
__global__ __launch_bounds__(256) void k_swap_commit(DevView v, SwapView sv) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t i = wave_id();
  if (i >= (sv.m >> 1) || !v.accept[i]) return;
  const uint32_t a = v.u_new[2 * i], b = v.u_new[2 * i + 1];
  if (lane == 0) {
    const uint32_t ua = v.U[a], ub = v.U[b];
    v.U[a] = ub;
    v.U[b] = ua;
    atomicAdd(&v.ctr[1], 1ull);
  }
  for (uint32_t t = 8 * lane; t < v.tp; t += 512) {
    uint4* ra = (uint4*)(sv.cpm + (size_t)a * v.tp + t);
    uint4* rb = (uint4*)(sv.cpm + (size_t)b * v.tp + t);
    const uint4 qa = *ra, qb = *rb;
    *ra = qb;
    *rb = qa;
  }
}

}  // namespace

hipError_t launch_to_pixel_major(const DevView& v, const SwapView& sv, hipStream_t s) {
  const size_t items = (size_t)v.w * v.h * (v.tp >> 3);
  hipLaunchKernelGGL(k_to_pixel_major, dim3((uint32_t)((items + 255) / 256)), dim3(256), 0, s, v, sv);
  return hipGetLastError();
}

hipError_t launch_from_pixel_major(const DevView& v, const SwapView& sv, hipStream_t s) {
  const size_t items = (size_t)v.w * v.h * (v.tp >> 3);
  hipLaunchKernelGGL(k_from_pixel_major, dim3((uint32_t)((items + 255) / 256)), dim3(256), 0, s, v, sv);
  return hipGetLastError();
}

hipError_t launch_swap_select(const DevView& v, const SwapView& sv, uint32_t kappa, hipStream_t s) {
  hipLaunchKernelGGL(k_swap_reset, dim3(1), dim3(64), 0, s, sv);
  const uint32_t P = v.w * v.h;
  hipLaunchKernelGGL(k_swap_select, dim3((P + 255) / 256), dim3(256), 0, s, v, sv, kappa);
  return hipGetLastError();
}

hipError_t launch_swap_evaluate(const DevView& v, const SwapView& sv, uint32_t kappa, hipStream_t s) {
  // integrand slices of 256 (at most 4), member blocks of 4 waves split over 8 XCDs
  const uint32_t nz = std::min<uint32_t>(4, (v.tp + 255) / 256);
  const uint32_t tslice = ((v.tp + nz - 1) / nz + 255) / 256 * 256;
  const uint32_t nblk = (sv.m + 3) / 4, nbx = (nblk + 7) / 8;
  const dim3 grid(8 * nbx * nz), block(256);
  switch (v.radius) {
    case 1: hipLaunchKernelGGL(k_swap_eval<1>, grid, block, 0, s, v, sv, kappa, nbx, nz, tslice); break;
    case 2: hipLaunchKernelGGL(k_swap_eval<2>, grid, block, 0, s, v, sv, kappa, nbx, nz, tslice); break;
    case 3: hipLaunchKernelGGL(k_swap_eval<3>, grid, block, 0, s, v, sv, kappa, nbx, nz, tslice); break;
    case 4: hipLaunchKernelGGL(k_swap_eval<4>, grid, block, 0, s, v, sv, kappa, nbx, nz, tslice); break;
    case 5: hipLaunchKernelGGL(k_swap_eval<5>, grid, block, 0, s, v, sv, kappa, nbx, nz, tslice); break;
    case 6: hipLaunchKernelGGL(k_swap_eval<6>, grid, block, 0, s, v, sv, kappa, nbx, nz, tslice); break;
    default: return hipErrorInvalidValue;
  }
  const uint32_t half = sv.m >> 1;
  hipLaunchKernelGGL(k_swap_finish, dim3((half + 255) / 256), dim3(256), 0, s, v, sv, kappa);
  return hipGetLastError();
}

hipError_t launch_swap_commit(const DevView& v, const SwapView& sv, hipStream_t s) {
  const uint32_t half = sv.m >> 1;
  hipLaunchKernelGGL(k_swap_commit, dim3((half + 3) / 4), dim3(256), 0, s, v, sv);
  return hipGetLastError();
}

}  // namespace bnlat
