// gfx950 kernels of the screen-space lattice-offset optimiser.
//
// Data layout in HBM (P = W*H pixels, Tp = T rounded up to 128):
//   U    uint32 [P]        offset of pixel p = y*W + x, Q0.16 x | y << 16
//   cnt  uint16 [Tp/8][P][8] hit counts in 16-byte integrand tiles: the 8
//                          counts of integrands 8i..8i+7 of a pixel are
//                          contiguous and neighbouring pixels' tiles are
//                          adjacent, so a row of pixels for 8 integrands is
//                          one contiguous run
//   err  float  [P][Tp]    error vectors c/N - A_t (refreshed from the counts
//                          when read)
//   lat  uint32 [N]        rank-1 lattice points (Sec. 3.2), x | y << 16
//   ihp  int2   [Tp]       Heaviside (n packed as two int16, D' = n.(C - 2^15))
//   gest float  [P][TGp]   Gaussian estimates (TGp = Gaussian count rounded
//                          up to 64; padded rows evaluate exp(0) = 1)
// Side buffers of one colour phase (M class pixels): u_new [M],
// c_new [Tp/8][M][8] (same tiling), delta [M], accept [M].
//
// All arithmetic that decides anything is exact: sample coordinates are
// Q0.16, the Heaviside predicate n.(S - 2^15) > D' is an int16 dot product
// against an int32 threshold, and the energy change is assembled from
// integer class sums before one FP64 weighted sum in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bnlat_dev.h"
#include "device_common.h"

namespace bnlat {
namespace {

// ------------------------------------------------------------ energy change
//
// Energy change of one pixel's move (Eq. (1) over the window, both pair
// orderings):  dE = (2/N^2) sum_d w(d) X_d,
//   X_d = |class d| * Z0 - 2 Z_d,  Z0 = sum_t dc_t (c'_t + c_t),
//   Z_d = sum_{o in class d} sum_t dc_t c_{p+o,t},  dc = c' - c,
// all in exact integers.  One wave per moved pixel; a lane handles two
// adjacent integrands and each (neighbour, integrand pair) costs one v_dot2 of
// packed int16 pairs.  Used for explicit pixel lists; colour phases use the
// LDS-staged kernel below.
template <int R, int MODE>
__global__ __launch_bounds__(256) void k_delta(DevView v, uint32_t kappa, uint32_t m) {
  constexpr Window<R> W = WinConst<R>::w;
  constexpr int NCLS = WinConst<R>::NCLS;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t j = wave_id();
  if (j >= m) return;
  const uint32_t p = (MODE == MODE_CLASS) ? class_pixel(v, kappa, j) : v.pix_list[j];
  const uint32_t y = p / v.w, x = p - y * v.w;
  uint32_t rowq[2 * R + 1], colq[2 * R + 1];
#pragma unroll
  for (int i = 0; i < 2 * R + 1; ++i) {
    rowq[i] = ((y + v.h + i - R) % v.h) * v.w;
    colq[i] = (x + v.w + i - R) % v.w;
  }
  const uint32_t P = v.w * v.h;
  long long z0 = 0;
  long long zd[NCLS];
#pragma unroll
  for (int c = 0; c < NCLS; ++c) zd[c] = 0;

  for (uint32_t base = 0; base < v.tp; base += 128) {
    const uint32_t t = base + 2 * lane;
    const uint32_t cn = *(const uint32_t*)(v.c_new + tix(j, t, m));
    const uint32_t co = *(const uint32_t*)(v.cnt + tix(p, t, P));
    const int n0 = (int)(cn & 0xFFFFu), n1 = (int)(cn >> 16);
    const int o0 = (int)(co & 0xFFFFu), o1 = (int)(co >> 16);
    const int dc0 = n0 - o0, dc1 = n1 - o1;
    const uint32_t dcp = ((uint32_t)dc0 & 0xFFFFu) | ((uint32_t)dc1 << 16);
    z0 += (long long)(dc0 * (n0 + o0) + dc1 * (n1 + o1));
    int part = 0;
#pragma unroll
    for (int mm = 0; mm < W.M; ++mm) {
      const uint32_t q = rowq[W.oy[mm] + R] + colq[W.ox[mm] + R];
      const uint32_t cq = *(const uint32_t*)(v.cnt + tix(q, t, P));
      part = dot2(dcp, cq, part);
      if (mm == W.M - 1 || W.cls[mm + 1] != W.cls[mm]) {
        zd[W.cls[mm]] += part;
        part = 0;
      }
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < NCLS; ++c) {
    long long xv = (long long)W.csize[c] * z0 - 2 * zd[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) xv += __shfl_xor(xv, off);
    acc = __dadd_rn(acc, __dmul_rn(v.wd[c], (double)xv));
  }
  if (lane == 0) {
    double total = __dmul_rn(acc, 2.0 / ((double)v.n * (double)v.n));
    if (v.tgp) total = __dadd_rn(total, v.gdelta[j]);
    v.delta[j] = total;
    v.accept[j] = (v.objective > 0) ? (total < 0.0) : (total > 0.0);
  }
}

// LDS-staged energy change for one colour phase.  A workgroup owns a block of
// 32 x (BY V) class pixels; thread (tx, ty) owns the V class pixels of column
// tx in class rows ty V .. ty V + V - 1.  Their windows overlap, so each count
// word the thread reads from LDS serves all of them.  The workgroup also owns
// a slice of the integrands: for 8 integrands at a time it stages the counts of
// its block plus the window halo (region of RH x RW pixels, 16 bytes each) and
// the class pixels' recounted rows in LDS.  Region columns are grouped by
// residue mod K, so the 32 lanes of a class row read 32 consecutive 16-byte
// words for every window offset, each with one ds_read_b128 at a compile-time
// offset from the thread's base.  Where the staging words fit in registers,
// the next stage's global loads are issued before the current stage is
// evaluated.  Class sums stay in int32 over a
// slice: its length is bounded so that |sum_t dc_t c_q,t| < 2^31 for every
// class; they are added into xsum[class][pixel] with 64-bit integer atomics
// (exact, so the order of the slices does not matter); k_delta_finish takes
// the decision and clears xsum.
template <int R, int K, int BY, int V>
struct StageGeom {
  static constexpr int BX = 32;
  static constexpr int CR = BY * V;                                // class rows per block
  static constexpr int RH = K * (CR - 1) + 2 * R + 1;
  static constexpr int RW = ((K * (BX - 1) + 2 * R + 1 + K - 1) / K) * K;
  static constexpr int RWK = RW / K;
  static constexpr int RA = RH * RW;                               // region pixels
  static constexpr int NB = BX * CR;                               // class pixels per block
  static constexpr int NT = BX * BY;                               // threads per block
  static constexpr int DR = K * (V - 1) + 2 * R + 1;               // region rows one thread reads
  static constexpr int LDS_BYTES = 16 * (RA + NB);
  // word of region column K tx + R + ox relative to that of column K tx
  static constexpr int dcol(int ox) { return ((R + ox) % K) * RWK + (R + ox) / K; }
};

// Block shape of the staged kernel for K colour classes per axis and radius R:
// class rows per thread (V) and thread rows (BY), within 64 KiB of LDS.
// Shape 0 is the single-problem default; the batched form's tuner also tries
// shape 1 (twice the waves per workgroup for K = 4, half for K = 1, 2).
template <int R, int K, int SH = 0>
struct StageShape {
  static constexpr int V = (K == 4) ? 1 : 2;
  static constexpr int BY = (K == 4) ? (SH ? 4 : 2) : (SH ? 4 : 8);
};

// Largest slice (a multiple of 8 integrands) whose class sums fit int32: every
// product dc_t c_q,t is at most N^2 in size and a class has at most 12 offsets
// for radii up to 6.
inline uint32_t stage_max_slice(uint32_t n) {
  const uint64_t per = (uint64_t)12 * n * n;
  uint64_t t = 0x7FFFFFFFull / per;
  t &= ~(uint64_t)7;
  return t < 8 ? 8 : (t > 0x40000000u ? 0x40000000u : (uint32_t)t);
}

// Count changes of a 16-byte count word (8 integrands) as four int16 pairs, and
// sum_t dc_t (c'_t + c_t) over the word.
__device__ __forceinline__ int stage_dc(const u32x4 cn, const u32x4 co, uint32_t d[4]) {
  int z = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int n0 = (int)(cn[k] & 0xFFFFu), n1 = (int)(cn[k] >> 16);
    const int o0 = (int)(co[k] & 0xFFFFu), o1 = (int)(co[k] >> 16);
    d[k] = ((uint32_t)(n0 - o0) & 0xFFFFu) | ((uint32_t)(n1 - o1) << 16);
    z += (n0 - o0) * (n0 + o0) + (n1 - o1) * (n1 + o1);
  }
  return z;
}

template <int R, int K, int BY, int V>
__device__ __forceinline__ void delta_stage_body(const DevView& v, uint32_t kappa, uint32_t trlen,
                                                 long long* __restrict__ xpart, uint32_t bkx,
                                                 uint32_t bky, uint32_t bkz) {
  using G = StageGeom<R, K, BY, V>;
  constexpr Window<R> W = WinConst<R>::w;
  constexpr int NCLS = WinConst<R>::NCLS;
  constexpr int ITER = (G::RA + G::NT - 1) / G::NT;
  constexpr bool PREFETCH = ITER <= 16;
  constexpr int WS = 2 * R + 1;
  extern __shared__ u32x4 lds4[];
  u32x4* reg = lds4;                 // [RA] region counts
  u32x4* cnb = lds4 + G::RA;         // [NB] recounted rows of the class pixels
  const uint32_t tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const uint32_t a0 = bky * G::CR, b0 = bkx * G::BX;
  const uint32_t b = b0 + tx;
  const uint32_t ky = kappa / K, kx = kappa - ky * K;
  // top-left region pixel, made non-negative modulo the tile
  const uint32_t ys = (ky + K * a0 + v.h * (R / v.h + 1) - R) % v.h;
  const uint32_t xs = (kx + K * b0 + v.w * (R / v.w + 1) - R) % v.w;
  const uint32_t P = v.w * v.h;

  // staging byte offsets: the region is the same for every stage.  Lanes past
  // the region load pixel 0 and do not store it.
  uint32_t poff[ITER], wi[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const uint32_t i = threadIdx.x + it * G::NT;
    poff[it] = 0;
    wi[it] = 0xFFFFFFFFu;
    if (i < (uint32_t)G::RA) {
      const uint32_t rr = i / G::RW, cc = i - rr * G::RW;
      uint32_t gy = ys + rr, gx = xs + cc;
      while (gy >= v.h) gy -= v.h;
      while (gx >= v.w) gx -= v.w;
      poff[it] = (gy * v.w + gx) * 16;
      wi[it] = rr * G::RW + (cc % K) * G::RWK + cc / K;
    }
  }
  uint32_t coff[V];
  bool act[V];
#pragma unroll
  for (int vv = 0; vv < V; ++vv) {
    const uint32_t a = a0 + ty * V + vv;
    act[vv] = (a < v.ch) && (b < v.cw);
    coff[vv] = act[vv] ? (a * v.cw + b) * 16 : 0;
  }
  const uint32_t top = K * ty * V * G::RW + tx;

  int z0[V];
  int part[V][NCLS];
#pragma unroll
  for (int vv = 0; vv < V; ++vv) {
    z0[vv] = 0;
#pragma unroll
    for (int c = 0; c < NCLS; ++c) part[vv][c] = 0;
  }

  const uint32_t t_begin = bkz * trlen, t_end = min(t_begin + trlen, v.tp);
  u32x4 q[ITER], qc[V];
  auto issue = [&](uint32_t t0) {
    const char* cs = (const char*)(v.cnt + (size_t)(t0 >> 3) * P * 8);
    const char* ns = (const char*)(v.c_new + (size_t)(t0 >> 3) * v.pc * 8);
#pragma unroll
    for (int it = 0; it < ITER; ++it) q[it] = *(const u32x4*)(cs + poff[it]);
#pragma unroll
    for (int vv = 0; vv < V; ++vv) qc[vv] = *(const u32x4*)(ns + coff[vv]);
  };
  if (PREFETCH && t_begin < t_end) issue(t_begin);
  for (uint32_t t0 = t_begin; t0 < t_end; t0 += 8) {
    __syncthreads();
    if (!PREFETCH) issue(t0);
#pragma unroll
    for (int it = 0; it < ITER; ++it)
      if (wi[it] != 0xFFFFFFFFu) reg[wi[it]] = q[it];
#pragma unroll
    for (int vv = 0; vv < V; ++vv) cnb[(ty * V + vv) * G::BX + tx] = qc[vv];
    __syncthreads();
    if (PREFETCH && t0 + 8 < t_end) issue(t0 + 8);
    uint32_t d[V][4];
#pragma unroll
    for (int vv = 0; vv < V; ++vv)
      z0[vv] += stage_dc(cnb[(ty * V + vv) * G::BX + tx], reg[top + (R + K * vv) * G::RW + G::dcol(0)], d[vv]);
#pragma unroll
    for (int dr = 0; dr < G::DR; ++dr) {
      // a row's words are loaded together, so their LDS latencies overlap
      u32x4 row[WS];
#pragma unroll
      for (int ox = -R; ox <= R; ++ox) row[ox + R] = reg[top + dr * G::RW + G::dcol(ox)];
#pragma unroll
      for (int ox = -R; ox <= R; ++ox) {
        const u32x4 cq = row[ox + R];
#pragma unroll
        for (int vv = 0; vv < V; ++vv) {
          const int oy = dr - R - K * vv;
          if (oy < -R || oy > R || (ox == 0 && oy == 0)) continue;
          const int c = W.cmap[(oy + R) * WS + ox + R];
          int x = part[vv][c];
          x = dot2(d[vv][0], cq[0], x);
          x = dot2(d[vv][1], cq[1], x);
          x = dot2(d[vv][2], cq[2], x);
          part[vv][c] = dot2(d[vv][3], cq[3], x);
        }
      }
    }
  }
#pragma unroll
  for (int vv = 0; vv < V; ++vv) {
    if (act[vv]) {
      const uint32_t j = (a0 + ty * V + vv) * v.cw + b;
#pragma unroll
      for (int c = 0; c < NCLS; ++c)
        atomicAdd((unsigned long long*)&xpart[(size_t)c * v.pc + j],
                  (unsigned long long)((long long)W.csize[c] * z0[vv] - 2 * (long long)part[vv][c]));
    }
  }
}

// One-dimensional grid of gx x gy blocks x slices, renumbered per XCD: the
// blocks one L2 serves at a time are whole rows of blocks of one slice, whose
// window halos are then read from HBM once.
template <int R, int K, int BY, int V>
__global__ __launch_bounds__(32 * BY) void k_delta_stage(DevView v, uint32_t kappa, uint32_t trlen,
                                                         long long* __restrict__ xpart, uint32_t gx,
                                                         uint32_t gy) {
  // the colour phases' waves issue ahead of the sweep-wide recount running
  // beside them (k_delta_finish, k_commit and the BF16 form's k_delta_bf
  // and k_delta_refine likewise), which fills the remaining issue slots
  __builtin_amdgcn_s_setprio(2);
  const uint32_t wk = xcd_block(blockIdx.x, gridDim.x), bxy = wk % (gx * gy);
  delta_stage_body<R, K, BY, V>(v, kappa, trlen, xpart, bxy % gx, bxy / gx, wk / (gx * gy));
}

// Batched form: member i owns blocks pre[i] .. pre[i+1]-1, laid out as its own
// (x, y, slice) grid; its slice length is in trl[i].
template <int R, int K, int BY, int V>
__global__ __launch_bounds__(32 * BY) void k_delta_stage_batch(const DevView* __restrict__ views,
                                                               const uint32_t* __restrict__ pre,
                                                               const uint32_t* __restrict__ geo,
                                                               uint32_t nmem, uint32_t kappa) {
  // like the single problem's phase kernels: issue ahead of the recount
  __builtin_amdgcn_s_setprio(2);
  const uint32_t i = batch_member(pre, nmem, blockIdx.x);
  const DevView v = views[i];
  const uint32_t lb = blockIdx.x - pre[i];
  const uint32_t gx = geo[3 * i], gy = geo[3 * i + 1], trlen = geo[3 * i + 2];
  delta_stage_body<R, K, BY, V>(v, kappa, trlen, v.xpart, lb % gx, (lb / gx) % gy, lb / (gx * gy));
}

// Decide from the summed class sums (one thread per pixel) and clear them.
__device__ __forceinline__ void delta_finish_body(const DevView& v, long long* __restrict__ xsum,
                                                  uint32_t blk) {
  const uint32_t j = blk * blockDim.x + threadIdx.x;
  if (j >= v.pc) return;
  double acc = 0.0;
  for (uint32_t c = 0; c < v.ncls; ++c) {
    const long long x = xsum[(size_t)c * v.pc + j];
    xsum[(size_t)c * v.pc + j] = 0;
    acc = __dadd_rn(acc, __dmul_rn(v.wd[c], (double)x));
  }
  double total = __dmul_rn(acc, v.xscale);
  // the approximate BF16 form's class sums already hold the Gaussian rows
  if (v.tgp && v.mfma != 2) total = __dadd_rn(total, v.gdelta[j]);
  v.delta[j] = total;
  if (v.delta_bf) v.delta_bf[j] = total;
  v.accept[j] = (v.objective > 0) ? (total < 0.0) : (total > 0.0);
}

__global__ __launch_bounds__(256) void k_delta_finish(DevView v, long long* __restrict__ xsum) {
  __builtin_amdgcn_s_setprio(2);
  delta_finish_body(v, xsum, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_delta_finish_batch(const DevView* __restrict__ views,
                                                            const uint32_t* __restrict__ pre,
                                                            uint32_t nmem) {
  __builtin_amdgcn_s_setprio(2);
  const uint32_t i = batch_member(pre, nmem, blockIdx.x);
  const DevView v = views[i];
  delta_finish_body(v, v.xpart, blockIdx.x - pre[i]);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ commit
// Accepted moves of the phase become the state (Sec. 3.4): offset and hit
// counts of the pixel (error vectors are refreshed from the counts on
// demand).  A thread copies CT consecutive 8-integrand tiles of one class
// pixel; pixels are fastest across the threads, so every tile's proposal rows
// are read coalesced.
constexpr uint32_t CT = 8;
__device__ __forceinline__ void commit_body(const DevView& v, uint32_t kappa, uint32_t blk) {
  const uint32_t ngrp = ((v.tp >> 3) + CT - 1) / CT;
  const uint64_t i = (uint64_t)blk * 256 + threadIdx.x;
  const bool in = i < (uint64_t)v.pc * ngrp;
  const uint32_t g = in ? (uint32_t)(i / v.pc) : 0, j = in ? (uint32_t)(i - (uint64_t)g * v.pc) : 0;
  const bool acc = in && v.accept[j];
  // one counter update per wave for the accepted pixels it holds in group 0
  const unsigned long long first = __ballot(acc && g == 0);
  if ((threadIdx.x & 63) == 0 && first) atomicAdd(&v.ctr[1], (unsigned long long)__popcll(first));
  if (!acc) return;
  const uint32_t p = class_pixel(v, kappa, j);
  if (g == 0) v.U[p] = v.u_new[j];
  const uint32_t t0 = g * CT, t1 = min(t0 + CT, v.tp >> 3);
  const size_t P = (size_t)v.w * v.h;
  for (uint32_t tt = t0; tt < t1; ++tt) {
    const uint4 c8 = *(const uint4*)(v.c_new + ((size_t)tt * v.pc + j) * 8);
    *(uint4*)(v.cnt + (tt * P + p) * 8) = c8;
    if (v.bf) *(uint4*)(v.bf + (tt * P + p) * 8) = heaviside_field_tile(v, c8, tt * 8);
  }
}

// FP32 error vectors e = c/N - A_t of every pixel from the exact counts
// (refreshed on demand; thread per (integrand tile, pixel), pixels fastest).
__global__ __launch_bounds__(256) void k_errors(DevView v) {
  const uint32_t P = v.w * v.h;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)P * (v.tp >> 3)) return;
  const uint32_t tt = (uint32_t)(i / P), p = (uint32_t)(i - (size_t)tt * P);
  const uint4 c8 = *(const uint4*)(v.cnt + i * 8);
  const uint32_t t = tt * 8;
  const float inv_n = 1.0f / (float)v.n;
  const float4 a = *(const float4*)(v.area + t), b = *(const float4*)(v.area + t + 4);
  float4 lo, hi;
  lo.x = (float)(c8.x & 0xFFFFu) * inv_n - a.x;
  lo.y = (float)(c8.x >> 16) * inv_n - a.y;
  lo.z = (float)(c8.y & 0xFFFFu) * inv_n - a.z;
  lo.w = (float)(c8.y >> 16) * inv_n - a.w;
  hi.x = (float)(c8.z & 0xFFFFu) * inv_n - b.x;
  hi.y = (float)(c8.z >> 16) * inv_n - b.y;
  hi.z = (float)(c8.w & 0xFFFFu) * inv_n - b.z;
  hi.w = (float)(c8.w >> 16) * inv_n - b.w;
  float* e = v.err + (size_t)p * v.tp + t;
  *(float4*)e = lo;
  *(float4*)(e + 4) = hi;
}

__global__ __launch_bounds__(256) void k_commit(DevView v, uint32_t kappa) {
  __builtin_amdgcn_s_setprio(2);
  commit_body(v, kappa, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_commit_batch(const DevView* __restrict__ views,
                                                      const uint32_t* __restrict__ pre, uint32_t nmem,
                                                      uint32_t kappa) {
  __builtin_amdgcn_s_setprio(2);
  const uint32_t i = batch_member(pre, nmem, blockIdx.x);
  const DevView v = views[i];
  commit_body(v, kappa, blockIdx.x - pre[i]);
}

__global__ void k_advance(unsigned long long* ctr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) atomicAdd(&ctr[0], 1ull);
}

// The overlapped schedule's recount index (counter word 3) one past the sweep
// counter, and its advance by a pair of sweeps.
__global__ void k_recount_index(unsigned long long* ctr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctr[3] = ctr[0] + 1ull;
}

__global__ void k_recount_advance_pair(unsigned long long* ctr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctr[3] += 2ull;
}

__global__ void k_advance_batch(const DevView* __restrict__ views, uint32_t nmem) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nmem) atomicAdd(&views[i].ctr[0], 1ull);
}

__global__ __launch_bounds__(256) void k_init_offsets(DevView v) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= v.w * v.h) return;
  v.U[p] = q16_pair(philox_w01(p, 0, v.problem, S_INIT, v.seed_lo, v.seed_hi));
}

// The N samples of one pixel in van der Corput order: s^k = L(bitrev_m(k)).
__global__ void k_points(DevView v, uint32_t pixel, uint32_t* out) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= v.n) return;
  const uint32_t i = v.log2n ? (__brev(k) >> (32 - v.log2n)) : 0u;
  out[k] = wrap_add(v.lat[i], v.U[pixel]);
}

// ------------------------------------------------------------------ energy
// Y_d = sum_{o in class d} sum_p sum_t (c_p - c_{p+o})^2 over the half window
// (the other half gives the same total).  Lanes run over 64 consecutive
// pixels of a row, so every 16-byte tile load of a wave (8 integrands of 64
// neighbouring pixels) is one contiguous 1 KiB run; per tile a lane's int32
// partial sums (at most 12 offsets x 8 integrands x N^2 < 2^31) are widened
// to 64 bits; atomics on integers only.
template <int R>
__global__ __launch_bounds__(256) void k_energy(DevView v, unsigned long long* ysum) {
  constexpr Window<R> W = WinConst<R>::w;
  constexpr int NCLS = WinConst<R>::NCLS;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t P = v.w * v.h;
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  long long yd[NCLS];
#pragma unroll
  for (int c = 0; c < NCLS; ++c) yd[c] = 0;
  if (p < P) {
    const uint32_t y = p / v.w, x = p - y * v.w;
    uint32_t q[W.M];
#pragma unroll
    for (int mm = 0; mm < W.M; ++mm)
      q[mm] = ((y + v.h + W.oy[mm]) % v.h) * v.w + (x + v.w + W.ox[mm]) % v.w;
    for (uint32_t tt = 0; tt < (v.tp >> 3); ++tt) {
      const uint4 cp = *(const uint4*)(v.cnt + ((size_t)tt * P + p) * 8);
      const uint32_t pw[4] = {cp.x, cp.y, cp.z, cp.w};
      int part[NCLS];
#pragma unroll
      for (int c = 0; c < NCLS; ++c) part[c] = 0;
#pragma unroll
      for (int mm = 0; mm < W.M; ++mm) {
        if (!(W.oy[mm] > 0 || (W.oy[mm] == 0 && W.ox[mm] > 0))) continue;
        const uint4 cq = *(const uint4*)(v.cnt + ((size_t)tt * P + q[mm]) * 8);
        const uint32_t qw[4] = {cq.x, cq.y, cq.z, cq.w};
        int a = part[W.cls[mm]];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int d0 = (int)(pw[k] & 0xFFFFu) - (int)(qw[k] & 0xFFFFu);
          const int d1 = (int)(pw[k] >> 16) - (int)(qw[k] >> 16);
          const uint32_t dp = ((uint32_t)d0 & 0xFFFFu) | ((uint32_t)d1 << 16);
          a = dot2(dp, dp, a);
        }
        part[W.cls[mm]] = a;
      }
#pragma unroll
      for (int c = 0; c < NCLS; ++c) yd[c] += part[c];
    }
  }
#pragma unroll
  for (int c = 0; c < NCLS; ++c) {
    long long s = yd[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0 && s) atomicAdd(&ysum[c], (unsigned long long)s);
  }
}

// ------------------------------------------------------------ blur criterion
// Separable periodised Gaussian blur of an error tile (Sec. 3.3): taps
// (d_i, k_i) with d_i in [0, W); b(x) = sum_i k_i e((x - d_i) mod W).  The
// field is float [P][pitch] with `valid` meaningful columns.
__global__ __launch_bounds__(256) void k_blur_x(DevView v, const float* __restrict__ field, uint32_t pitch,
                                                const float* __restrict__ kx, const int32_t* __restrict__ dx,
                                                uint32_t nk, float* __restrict__ out) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = wave_id();
  const uint32_t nch = pitch >> 6;
  const uint32_t p = wave / nch, ch = wave - p * nch;
  if (p >= v.w * v.h) return;
  const uint32_t y = p / v.w, x = p - y * v.w;
  const uint32_t t = ch * 64 + lane;
  const float* rowbase = field + (size_t)y * v.w * pitch + t;
  float acc = 0.0f;
  for (uint32_t i = 0; i < nk; ++i) {
    uint32_t xs = x + v.w - (uint32_t)dx[i];
    if (xs >= v.w) xs -= v.w;
    acc = fmaf(kx[i], rowbase[(size_t)xs * pitch], acc);
  }
  out[(size_t)p * pitch + t] = acc;
}

__global__ __launch_bounds__(256) void k_blur_y_sq(DevView v, uint32_t pitch, uint32_t valid,
                                                   const float* __restrict__ ky,
                                                   const int32_t* __restrict__ dy, uint32_t nk,
                                                   const float* __restrict__ in,
                                                   double* __restrict__ partial) {
  __shared__ double red[4];
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = wave_id();
  const uint32_t nch = pitch >> 6;
  // waves walk down one column (and 64-integrand chunk) at a time, so the
  // waves in flight share the column's taps in L2
  const uint32_t y = wave % v.h, rest = wave / v.h;
  const uint32_t x = rest / nch, ch = rest - x * nch;
  double sq = 0.0;
  if (x < v.w) {
    const uint32_t t = ch * 64 + lane;
    float acc = 0.0f;
    for (uint32_t i = 0; i < nk; ++i) {
      uint32_t ys = y + v.h - (uint32_t)dy[i];
      if (ys >= v.h) ys -= v.h;
      acc = fmaf(ky[i], in[((size_t)ys * v.w + x) * pitch + t], acc);
    }
    if (t < valid) sq = (double)acc * (double)acc;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
  if (lane == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ----------------------------------------------------- Gaussian integrands
// Low-frequency test integrands (Sec. 3.5): f_t(x) = exp(-|x - mu_t|^2 / (2 s_t^2)).
// Estimates g = (1/N) sum_k f_t(s_p^k) per pixel.  A wave owns one pixel and
// 16 Gaussians; its lanes hold the samples (8 per lane at a time, as FP64
// x, y and |x|^2, all exact: Q0.16 coordinates) and the Gaussians' exponent
// coefficients come from scalar registers, so a term costs three FP64 FMAs
// (a |x|^2 + bx x + by y + c, the base-2 exponent -log2(e) |x - mu|^2 / (2 s^2),
// accurate to FP64 rounding of terms below 600), one conversion to FP32,
// v_exp_f32 (results below 2^-126 flush to zero, far below the estimate's
// resolution) and one FP32 add.  Each lane sums its 8 terms of a Gaussian in
// FP32 and the groups in FP64; the lanes' sums are added in FP64 through LDS.
// The estimate is stored in FP32.
template <bool CHECK>
__device__ __forceinline__ void gauss_chunk(const DevView& v, uint32_t u, uint32_t c0, uint32_t lane,
                                            const double* __restrict__ gc, double acc[16]) {
  constexpr int SC = 8;
  double sx[SC], sy[SC], s2[SC];
  bool ok[SC];
#pragma unroll
  for (int k = 0; k < SC; ++k) {
    const uint32_t i = c0 + 64 * k + lane;
    ok[k] = !CHECK || i < v.n;
    const uint32_t sv = wrap_add(v.lat[ok[k] ? i : 0], u);
    sx[k] = (double)(sv & 0xFFFFu) * 0x1p-16;
    sy[k] = (double)(sv >> 16) * 0x1p-16;
    s2[k] = __fma_rn(sx[k], sx[k], sy[k] * sy[k]);
  }
  // two halves of 8 Gaussians: their 32 coefficients fit the scalar registers
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double* gh = gc + 32 * h;
    double cf[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) cf[i] = gh[i];
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const double a = cf[4 * g], bx = cf[4 * g + 1], by = cf[4 * g + 2], c = cf[4 * g + 3];
      float part = 0.0f;
#pragma unroll
      for (int k = 0; k < SC; ++k) {
        const double e = __fma_rn(a, s2[k], __fma_rn(bx, sx[k], __fma_rn(by, sy[k], c)));
        const float f = __builtin_amdgcn_exp2f((float)e);
        part = __fadd_rn(part, CHECK && !ok[k] ? 0.0f : f);
      }
      acc[8 * h + g] = __dadd_rn(acc[8 * h + g], (double)part);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_gauss_est(DevView v, uint32_t kappa, uint32_t m) {
  constexpr uint32_t GB = 16, CH = 512;         // Gaussians per wave, samples per chunk
  __shared__ double red[4][GB / 2][65];
  const uint32_t lane = threadIdx.x & 63, wl = threadIdx.x >> 6;
  const uint32_t wave = wave_id();
  const uint32_t ngb = v.tgp / GB;
  const uint32_t j = wave / ngb, gb = wave - j * ngb;
  if (j >= m) return;
  uint32_t u;
  float* out;
  if (MODE == MODE_ALL) {
    u = v.U[j];
    out = v.gest + (size_t)j * v.tgp;
  } else {
    u = v.u_new[j];
    out = v.g_new + (size_t)j * v.tgp;
  }
  const double* gc = v.gcoef + (size_t)gb * GB * 4;
  double acc[GB];
#pragma unroll
  for (uint32_t g = 0; g < GB; ++g) acc[g] = 0.0;
  uint32_t c0 = 0;
  for (; c0 + CH <= v.n; c0 += CH) gauss_chunk<false>(v, u, c0, lane, gc, acc);
  if (c0 < v.n) gauss_chunk<true>(v, u, c0, lane, gc, acc);
  // lane sums -> per-Gaussian totals, eight Gaussians at a time: lane l adds
  // 8 of Gaussian l % 8's lane sums, then the eight groups are added across
  // lanes
#pragma unroll
  for (uint32_t h = 0; h < 2; ++h) {
#pragma unroll
    for (uint32_t g = 0; g < GB / 2; ++g) red[wl][g][lane] = acc[8 * h + g];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint32_t g = lane & 7, q = lane >> 3;
    double t = 0.0;
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) t = __dadd_rn(t, red[wl][g][8 * q + k]);
    t = __dadd_rn(t, __shfl_xor(t, 8));
    t = __dadd_rn(t, __shfl_xor(t, 16));
    t = __dadd_rn(t, __shfl_xor(t, 32));
    if (lane < GB / 2) out[gb * GB + 8 * h + g] = (float)(t / (double)v.n);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Gaussian rows' part of a move's energy change (plain form of Eq. (1) over
// the window, FP64 arithmetic on the FP32 estimates); one wave per moved
// pixel, lanes over integrands, workgroups renumbered per XCD so that moved
// pixels whose windows overlap read the shared rows through one L2.  Written
// to gdelta[j]; the decision adds it to the exact Heaviside part.
template <int R, int MODE>
__global__ __launch_bounds__(256) void k_delta_gauss(DevView v, uint32_t kappa, uint32_t m) {
  constexpr Window<R> W = WinConst<R>::w;
  constexpr int NCLS = WinConst<R>::NCLS;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t j = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6));
  if (j >= m) return;
  const uint32_t p = (MODE == MODE_CLASS) ? class_pixel(v, kappa, j) : v.pix_list[j];
  const uint32_t y = p / v.w, x = p - y * v.w;
  double cs[NCLS];
#pragma unroll
  for (int c = 0; c < NCLS; ++c) cs[c] = 0.0;
  for (uint32_t base = 0; base < v.tgp; base += 64) {
    const uint32_t t = base + lane;
    const double gn = v.g_new[(size_t)j * v.tgp + t], go = v.gest[(size_t)p * v.tgp + t];
    const double d = gn - go, sm = gn + go;
#pragma unroll
    for (int mm = 0; mm < W.M; ++mm) {
      const uint32_t q = ((y + v.h + W.oy[mm]) % v.h) * v.w + (x + v.w + W.ox[mm]) % v.w;
      cs[W.cls[mm]] += d * (sm - 2.0 * (double)v.gest[(size_t)q * v.tgp + t]);
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < NCLS; ++c) {
    double xv = cs[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) xv += __shfl_xor(xv, off);
    acc += v.wd[c] * xv;
  }
  if (lane == 0) v.gdelta[j] = 2.0 * acc;
}

// Colour-phase form of the same sum: a workgroup owns 4 x 2 class pixels (one
// wave each) and, for 64 Gaussians at a time, stages the estimate rows of
// their window region ((K + 2r + 1) x (3K + 2r + 1) pixels) in LDS, so that
// each row is read from memory once per workgroup rather than once per moved
// pixel.  Same arithmetic and summation order as k_delta_gauss.
template <int R, int K>
struct GaussStage {
  static constexpr int BCX = 4, BCY = 2, NW = BCX * BCY;
  static constexpr int RH = K * (BCY - 1) + 2 * R + 1;
  static constexpr int RW = K * (BCX - 1) + 2 * R + 1;
  static constexpr int RA = RH * RW;
  static constexpr int LDS_BYTES = RA * 64 * 4;
};

template <int R, int K>
__global__ __launch_bounds__(512) void k_delta_gauss_stage(DevView v, uint32_t kappa) {
  using G = GaussStage<R, K>;
  constexpr Window<R> W = WinConst<R>::w;
  constexpr int NCLS = WinConst<R>::NCLS;
  constexpr int NT = 64 * G::NW;
  constexpr int ITER = (G::RA * 16 + NT - 1) / NT;
  extern __shared__ float gl[];                  // [RA][64] estimates of the region
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t a0 = blockIdx.y * G::BCY, b0 = blockIdx.x * G::BCX;
  const uint32_t cy = w / G::BCX, cx = w - cy * G::BCX;
  const uint32_t a = a0 + cy, b = b0 + cx;
  const bool act = (a < v.ch) && (b < v.cw);
  const uint32_t j = act ? a * v.cw + b : 0;
  const uint32_t ky = kappa / K, kx = kappa - ky * K;
  const uint32_t ys = (ky + K * a0 + v.h * (R / v.h + 1) - R) % v.h;
  const uint32_t xs = (kx + K * b0 + v.w * (R / v.w + 1) - R) % v.w;
  // staging: float4 it of a thread is quad (idx & 15) of region pixel idx >> 4
  // (threads past the region reload its last pixel and do not store it)
  uint32_t goff[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const uint32_t idx = threadIdx.x + it * NT;
    const uint32_t r = min(idx >> 4, (uint32_t)G::RA - 1);
    const uint32_t rr = r / G::RW, cc = r - rr * G::RW;
    uint32_t gy = ys + rr, gx = xs + cc;
    while (gy >= v.h) gy -= v.h;
    while (gx >= v.w) gx -= v.w;
    goff[it] = gy * v.w + gx;
  }
  const int own = (K * cy + R) * G::RW + K * cx + R;
  double cs[NCLS];
#pragma unroll
  for (int c = 0; c < NCLS; ++c) cs[c] = 0.0;
  for (uint32_t base = 0; base < v.tgp; base += 64) {
    f32x4 q[ITER];
#pragma unroll
    for (int it = 0; it < ITER; ++it)
      q[it] = *(const f32x4*)(v.gest + (size_t)goff[it] * v.tgp + base + 4 * ((threadIdx.x + it * NT) & 15));
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const uint32_t idx = threadIdx.x + it * NT;
      if (idx < (uint32_t)G::RA * 16) *(f32x4*)&gl[idx * 4] = q[it];
    }
    __syncthreads();
    if (act) {
      const double gn = v.g_new[(size_t)j * v.tgp + base + lane], go = gl[own * 64 + lane];
      const double d = gn - go, sm = gn + go;
#pragma unroll
      for (int mm = 0; mm < W.M; ++mm) {
        const int q = own + W.oy[mm] * G::RW + W.ox[mm];
        cs[W.cls[mm]] += d * (sm - 2.0 * (double)gl[q * 64 + lane]);
      }
    }
  }
  if (!act) return;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < NCLS; ++c) {
    double xv = cs[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) xv += __shfl_xor(xv, off);
    acc += v.wd[c] * xv;
  }
  if (lane == 0) v.gdelta[j] = 2.0 * acc;
}

// Gaussian rows' part of the energy: per distance class, sum over the half
// window of |g_p - g_q|^2 (FP64 atomics; doubled by the host).
template <int R>
__global__ __launch_bounds__(256) void k_energy_gauss(DevView v, double* gsum) {
  constexpr Window<R> W = WinConst<R>::w;
  constexpr int NCLS = WinConst<R>::NCLS;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t p = wave_id();
  if (p >= v.w * v.h) return;
  const uint32_t y = p / v.w, x = p - y * v.w;
  double cs[NCLS];
#pragma unroll
  for (int c = 0; c < NCLS; ++c) cs[c] = 0.0;
  for (uint32_t base = 0; base < v.tgp; base += 64) {
    const uint32_t t = base + lane;
    const double gp = v.gest[(size_t)p * v.tgp + t];
#pragma unroll
    for (int mm = 0; mm < W.M; ++mm) {
      if (W.oy[mm] > 0 || (W.oy[mm] == 0 && W.ox[mm] > 0)) {
        const uint32_t q = ((y + v.h + W.oy[mm]) % v.h) * v.w + (x + v.w + W.ox[mm]) % v.w;
        const double d = gp - (double)v.gest[(size_t)q * v.tgp + t];
        cs[W.cls[mm]] += d * d;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NCLS; ++c) {
    double xv = cs[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) xv += __shfl_xor(xv, off);
    if (lane == 0 && xv != 0.0) atomicAdd(&gsum[c], xv);
  }
}

// Commit of accepted moves' Gaussian estimate rows.
__global__ __launch_bounds__(256) void k_commit_gauss(DevView v, uint32_t kappa) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t j = wave_id();
  if (j >= v.pc || !v.accept[j]) return;
  const uint32_t p = class_pixel(v, kappa, j);
  const uint32_t P = v.w * v.h;
  for (uint32_t t = lane; t < v.tgp; t += 64) {
    const float g = v.g_new[(size_t)j * v.tgp + t];
    v.gest[(size_t)p * v.tgp + t] = g;
    if (v.bf)
      v.bf[tix(p, v.tp + t, P)] = __builtin_bit_cast(uint16_t, (__bf16)gaussian_error(v, g, t));
  }
}

// Gaussian error rows g - I (refreshed on demand).
__global__ __launch_bounds__(256) void k_gauss_errors(DevView v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)v.w * v.h * v.tgp) return;
  const uint32_t t = (uint32_t)(i % v.tgp);
  v.gerr[i] = (float)((double)v.gest[i] - v.gint[t]);
}


template <int MODE>
hipError_t delta_dispatch(const DevView& v, uint32_t kappa, uint32_t m, hipStream_t s) {
  if (m == 0) return hipSuccess;
  const dim3 grid((m + 3) / 4), block(256);
  switch (v.radius) {
    case 1: hipLaunchKernelGGL((k_delta<1, MODE>), grid, block, 0, s, v, kappa, m); break;
    case 2: hipLaunchKernelGGL((k_delta<2, MODE>), grid, block, 0, s, v, kappa, m); break;
    case 3: hipLaunchKernelGGL((k_delta<3, MODE>), grid, block, 0, s, v, kappa, m); break;
    case 4: hipLaunchKernelGGL((k_delta<4, MODE>), grid, block, 0, s, v, kappa, m); break;
    case 5: hipLaunchKernelGGL((k_delta<5, MODE>), grid, block, 0, s, v, kappa, m); break;
    case 6: hipLaunchKernelGGL((k_delta<6, MODE>), grid, block, 0, s, v, kappa, m); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Integrand slices of a staged launch: about slice_target workgroups in total
// (512 by default), each slice a whole number of stages of `gran` integrands
// (8 for the integer stencil, 16 for the matrix-core form), at least `min_len`
// integrands long where the rows have that many and at most `cap` long.
inline uint32_t stage_slices(const DevView& v, uint32_t blocks, uint32_t* trlen, uint32_t gran = 8,
                             uint32_t cap = 0xFFFFFFFFu, uint32_t min_len = 0) {
  const uint32_t chunks = v.tp / gran;
  const uint32_t target = v.slice_target ? v.slice_target : 512;
  uint32_t want = (target + blocks - 1) / blocks;
  if (want > chunks) want = chunks;
  uint32_t per = (chunks + want - 1) / want;
  const uint32_t min_per = min(chunks, min_len / gran);
  if (per < min_per) per = min_per;
  const uint32_t cap_stages = cap / gran ? cap / gran : 1;
  if (per > cap_stages) per = cap_stages;
  *trlen = per * gran;
  return (chunks + per - 1) / per;
}

template <int R, int K>
hipError_t stage_launch(const DevView& v, uint32_t kappa, long long* xpart, hipStream_t s, bool finish = true) {
  using S = StageShape<R, K>;
  using G = StageGeom<R, K, S::BY, S::V>;
  static_assert(G::LDS_BYTES <= 65536, "staged block exceeds 64 KiB of LDS");
  uint32_t trlen = 0;
  const uint32_t blocks = ((v.cw + G::BX - 1) / G::BX) * ((v.ch + G::CR - 1) / G::CR);
  // slices of at least 64 integrands: each adds its class sums with atomics
  // and restages the window halo
  const uint32_t ns = stage_slices(v, blocks, &trlen, 8, stage_max_slice(v.n), 64);
  const uint32_t gx = (v.cw + G::BX - 1) / G::BX, gy = (v.ch + G::CR - 1) / G::CR;
  hipLaunchKernelGGL((k_delta_stage<R, K, S::BY, S::V>), dim3(gx * gy * ns), dim3(G::NT), (size_t)G::LDS_BYTES, s,
                     v, kappa, trlen, xpart, gx, gy);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !finish) return e;
  return launch_finish(v, s);
}

template <int R>
hipError_t stage_by_k(const DevView& v, uint32_t kappa, long long* xpart, hipStream_t s, bool finish = true) {
  switch (v.k) {
    case 1: return stage_launch<R, 1>(v, kappa, xpart, s, finish);
    case 2: return stage_launch<R, 2>(v, kappa, xpart, s, finish);
    case 4: return stage_launch<R, 4>(v, kappa, xpart, s, finish);
    default: return delta_dispatch<MODE_CLASS>(v, kappa, v.pc, s);
  }
}

}  // namespace

hipError_t launch_init_offsets(const DevView& v, hipStream_t s) {
  const uint32_t P = v.w * v.h;
  hipLaunchKernelGGL(k_init_offsets, dim3((P + 255) / 256), dim3(256), 0, s, v);
  return hipGetLastError();
}


hipError_t launch_delta(const DevView& v, int mode, uint32_t kappa, uint32_t m, hipStream_t s) {
  // BF16 precision form: matrix-core Gram pass, decision, exact re-evaluation
  if (mode == MODE_CLASS && v.mfma) return launch_delta_bf16(v, kappa, s);
  if (mode == MODE_CLASS && v.xpart) {
    switch (v.radius) {
      case 1: return stage_by_k<1>(v, kappa, v.xpart, s);
      case 2: return stage_by_k<2>(v, kappa, v.xpart, s);
      case 3: return stage_by_k<3>(v, kappa, v.xpart, s);
      case 4: return stage_by_k<4>(v, kappa, v.xpart, s);
      case 5: return stage_by_k<5>(v, kappa, v.xpart, s);
      case 6: return stage_by_k<6>(v, kappa, v.xpart, s);
      default: return hipErrorInvalidValue;
    }
  }
  return mode == MODE_CLASS ? delta_dispatch<MODE_CLASS>(v, kappa, m, s)
                            : delta_dispatch<MODE_LIST>(v, kappa, m, s);
}

uint32_t xpart_words(const DevView& v) { return v.ncls * v.pc; }

hipError_t launch_finish(const DevView& v, hipStream_t s) {
  hipLaunchKernelGGL(k_delta_finish, dim3((v.pc + 255) / 256), dim3(256), 0, s, v, v.xpart);
  return hipGetLastError();
}

uint32_t commit_blocks(const DevView& v) {
  return (uint32_t)(((uint64_t)v.pc * (((v.tp >> 3) + CT - 1) / CT) + 255) / 256);
}

hipError_t launch_commit(const DevView& v, uint32_t kappa, hipStream_t s) {
  hipLaunchKernelGGL(k_commit, dim3(commit_blocks(v)), dim3(256), 0, s, v, kappa);
  return hipGetLastError();
}

hipError_t launch_errors(const DevView& v, hipStream_t s) {
  const size_t n = (size_t)v.w * v.h * (v.tp >> 3);
  hipLaunchKernelGGL(k_errors, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v);
  return hipGetLastError();
}

hipError_t launch_advance(const DevView& v, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, v.ctr);
  return hipGetLastError();
}

hipError_t launch_recount_index(const DevView& v, hipStream_t s) {
  hipLaunchKernelGGL(k_recount_index, dim3(1), dim3(64), 0, s, v.ctr);
  return hipGetLastError();
}

hipError_t launch_recount_advance_pair(const DevView& v, hipStream_t s) {
  hipLaunchKernelGGL(k_recount_advance_pair, dim3(1), dim3(64), 0, s, v.ctr);
  return hipGetLastError();
}

hipError_t launch_points(const DevView& v, uint32_t pixel, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_points, dim3((v.n + 255) / 256), dim3(256), 0, s, v, pixel, out);
  return hipGetLastError();
}

hipError_t launch_energy(const DevView& v, unsigned long long* y, hipStream_t s) {
  const uint32_t P = v.w * v.h;
  const dim3 grid((P + 255) / 256), block(256);
  switch (v.radius) {
    case 1: hipLaunchKernelGGL(k_energy<1>, grid, block, 0, s, v, y); break;
    case 2: hipLaunchKernelGGL(k_energy<2>, grid, block, 0, s, v, y); break;
    case 3: hipLaunchKernelGGL(k_energy<3>, grid, block, 0, s, v, y); break;
    case 4: hipLaunchKernelGGL(k_energy<4>, grid, block, 0, s, v, y); break;
    case 5: hipLaunchKernelGGL(k_energy<5>, grid, block, 0, s, v, y); break;
    case 6: hipLaunchKernelGGL(k_energy<6>, grid, block, 0, s, v, y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

uint32_t blur_partials(const DevView& v, uint32_t pitch) {
  const uint64_t waves = (uint64_t)v.w * v.h * (pitch >> 6);
  return (uint32_t)((waves + 3) / 4);
}

hipError_t launch_blur(const DevView& v, const float* field, uint32_t pitch, uint32_t valid, const float* kx,
                       uint32_t nkx, const int32_t* dx, const float* ky, uint32_t nky, const int32_t* dy,
                       float* tmp, double* partial, uint32_t* npartial, hipStream_t s) {
  const uint32_t blocks = blur_partials(v, pitch);
  hipLaunchKernelGGL(k_blur_x, dim3(blocks), dim3(256), 0, s, v, field, pitch, kx, dx, nkx, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_blur_y_sq, dim3(blocks), dim3(256), 0, s, v, pitch, valid, ky, dy, nky,
                     (const float*)tmp, partial);
  *npartial = blocks;
  return hipGetLastError();
}

hipError_t launch_gauss_est(const DevView& v, int mode, uint32_t m, hipStream_t s) {
  if (!v.tgp || m == 0) return hipSuccess;
  const uint64_t waves = (uint64_t)m * (v.tgp >> 4);
  const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
  if (mode == MODE_ALL) hipLaunchKernelGGL(k_gauss_est<MODE_ALL>, grid, block, 0, s, v, 0u, m);
  else hipLaunchKernelGGL(k_gauss_est<MODE_CLASS>, grid, block, 0, s, v, 0u, m);
  return hipGetLastError();
}

namespace {
template <int MODE>
hipError_t gauss_delta_dispatch(const DevView& v, uint32_t kappa, uint32_t m, hipStream_t s) {
  const dim3 grid((m + 3) / 4), block(256);
  switch (v.radius) {
    case 1: hipLaunchKernelGGL((k_delta_gauss<1, MODE>), grid, block, 0, s, v, kappa, m); break;
    case 2: hipLaunchKernelGGL((k_delta_gauss<2, MODE>), grid, block, 0, s, v, kappa, m); break;
    case 3: hipLaunchKernelGGL((k_delta_gauss<3, MODE>), grid, block, 0, s, v, kappa, m); break;
    case 4: hipLaunchKernelGGL((k_delta_gauss<4, MODE>), grid, block, 0, s, v, kappa, m); break;
    case 5: hipLaunchKernelGGL((k_delta_gauss<5, MODE>), grid, block, 0, s, v, kappa, m); break;
    case 6: hipLaunchKernelGGL((k_delta_gauss<6, MODE>), grid, block, 0, s, v, kappa, m); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int R, int K>
hipError_t gauss_stage_launch(const DevView& v, uint32_t kappa, hipStream_t s) {
  using G = GaussStage<R, K>;
  if constexpr (G::LDS_BYTES > 65536) {
    return gauss_delta_dispatch<MODE_CLASS>(v, kappa, v.pc, s);
  } else {
    const dim3 grid((v.cw + G::BCX - 1) / G::BCX, (v.ch + G::BCY - 1) / G::BCY);
    hipLaunchKernelGGL((k_delta_gauss_stage<R, K>), grid, dim3(64 * G::NW), (size_t)G::LDS_BYTES, s, v, kappa);
    return hipGetLastError();
  }
}

template <int R>
hipError_t gauss_stage_by_k(const DevView& v, uint32_t kappa, hipStream_t s) {
  switch (v.k) {
    case 1: return gauss_stage_launch<R, 1>(v, kappa, s);
    case 2: return gauss_stage_launch<R, 2>(v, kappa, s);
    case 4: return gauss_stage_launch<R, 4>(v, kappa, s);
    default: return gauss_delta_dispatch<MODE_CLASS>(v, kappa, v.pc, s);
  }
}
}  // namespace

hipError_t launch_gauss_delta(const DevView& v, int mode, uint32_t kappa, uint32_t m, hipStream_t s) {
  if (!v.tgp || m == 0) return hipSuccess;
  // the approximate BF16 form evaluates the Gaussian rows in its Gram pass
  // and re-evaluates accepted moves exactly
  if (mode == MODE_CLASS && v.mfma == 2) return hipSuccess;
  if (mode == MODE_CLASS) {
    switch (v.radius) {
      case 1: return gauss_stage_by_k<1>(v, kappa, s);
      case 2: return gauss_stage_by_k<2>(v, kappa, s);
      case 3: return gauss_stage_by_k<3>(v, kappa, s);
      case 4: return gauss_stage_by_k<4>(v, kappa, s);
      case 5: return gauss_stage_by_k<5>(v, kappa, s);
      case 6: return gauss_stage_by_k<6>(v, kappa, s);
      default: return hipErrorInvalidValue;
    }
  }
  return mode == MODE_CLASS ? gauss_delta_dispatch<MODE_CLASS>(v, kappa, m, s)
                            : gauss_delta_dispatch<MODE_LIST>(v, kappa, m, s);
}

hipError_t launch_stage_exact(const DevView& v, uint32_t kappa, hipStream_t s) {
  switch (v.radius) {
    case 1: return stage_by_k<1>(v, kappa, v.xpart, s, false);
    case 2: return stage_by_k<2>(v, kappa, v.xpart, s, false);
    case 3: return stage_by_k<3>(v, kappa, v.xpart, s, false);
    case 4: return stage_by_k<4>(v, kappa, v.xpart, s, false);
    case 5: return stage_by_k<5>(v, kappa, v.xpart, s, false);
    case 6: return stage_by_k<6>(v, kappa, v.xpart, s, false);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gauss_delta_exact(const DevView& v, uint32_t kappa, hipStream_t s) {
  if (!v.tgp) return hipSuccess;
  switch (v.radius) {
    case 1: return gauss_stage_by_k<1>(v, kappa, s);
    case 2: return gauss_stage_by_k<2>(v, kappa, s);
    case 3: return gauss_stage_by_k<3>(v, kappa, s);
    case 4: return gauss_stage_by_k<4>(v, kappa, s);
    case 5: return gauss_stage_by_k<5>(v, kappa, s);
    case 6: return gauss_stage_by_k<6>(v, kappa, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gauss_commit(const DevView& v, uint32_t kappa, hipStream_t s) {
  if (!v.tgp) return hipSuccess;
  hipLaunchKernelGGL(k_commit_gauss, dim3((v.pc + 3) / 4), dim3(256), 0, s, v, kappa);
  return hipGetLastError();
}

hipError_t launch_gauss_errors(const DevView& v, hipStream_t s) {
  if (!v.tgp) return hipSuccess;
  const size_t n = (size_t)v.w * v.h * v.tgp;
  hipLaunchKernelGGL(k_gauss_errors, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v);
  return hipGetLastError();
}

hipError_t launch_gauss_energy(const DevView& v, double* gsum, hipStream_t s) {
  if (!v.tgp) return hipSuccess;
  const uint32_t P = v.w * v.h;
  const dim3 grid((P + 3) / 4), block(256);
  switch (v.radius) {
    case 1: hipLaunchKernelGGL(k_energy_gauss<1>, grid, block, 0, s, v, gsum); break;
    case 2: hipLaunchKernelGGL(k_energy_gauss<2>, grid, block, 0, s, v, gsum); break;
    case 3: hipLaunchKernelGGL(k_energy_gauss<3>, grid, block, 0, s, v, gsum); break;
    case 4: hipLaunchKernelGGL(k_energy_gauss<4>, grid, block, 0, s, v, gsum); break;
    case 5: hipLaunchKernelGGL(k_energy_gauss<5>, grid, block, 0, s, v, gsum); break;
    case 6: hipLaunchKernelGGL(k_energy_gauss<6>, grid, block, 0, s, v, gsum); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}


// ------------------------------------------------------------------ batches

uint32_t stage_rows(uint32_t k, uint32_t shape) {
  if (k == 4) return shape ? StageShape<1, 4, 1>::BY * StageShape<1, 4, 1>::V : StageShape<1, 4>::BY * StageShape<1, 4>::V;
  return shape ? StageShape<1, 2, 1>::BY * StageShape<1, 2, 1>::V : StageShape<1, 2>::BY * StageShape<1, 2>::V;
}

void stage_geometry(const DevView& v, uint32_t shape, uint32_t* gx, uint32_t* gy, uint32_t* gz, uint32_t* trlen) {
  const uint32_t cr = stage_rows(v.k, shape);
  *gx = (v.cw + 31) / 32;
  *gy = (v.ch + cr - 1) / cr;
  *gz = stage_slices(v, *gx * *gy, trlen, 8, stage_max_slice(v.n), 64);
}


namespace {
template <int R, int K, int SH>
hipError_t stage_batch_rk(const DevView* views, const uint32_t* pre, const uint32_t* geo, uint32_t nmem,
                          uint32_t blocks, uint32_t kappa, hipStream_t s) {
  using S = StageShape<R, K, SH>;
  using G = StageGeom<R, K, S::BY, S::V>;
  static_assert(G::LDS_BYTES <= 65536, "staged block exceeds 64 KiB of LDS");
  static_assert(G::CR == StageShape<1, K == 4 ? 4 : 2, SH>::BY * StageShape<1, K == 4 ? 4 : 2, SH>::V,
                "batched geometry assumes one block shape per (K, shape)");
  hipLaunchKernelGGL((k_delta_stage_batch<R, K, S::BY, S::V>), dim3(blocks), dim3(G::NT), (size_t)G::LDS_BYTES, s,
                     views, pre, geo, nmem, kappa);
  return hipGetLastError();
}

template <int R>
hipError_t stage_batch_r(uint32_t k, uint32_t shape, const DevView* views, const uint32_t* pre, const uint32_t* geo,
                         uint32_t nmem, uint32_t blocks, uint32_t kappa, hipStream_t s) {
  switch (k * 2 + (shape ? 1 : 0)) {
    case 2: return stage_batch_rk<R, 1, 0>(views, pre, geo, nmem, blocks, kappa, s);
    case 3: return stage_batch_rk<R, 1, 1>(views, pre, geo, nmem, blocks, kappa, s);
    case 4: return stage_batch_rk<R, 2, 0>(views, pre, geo, nmem, blocks, kappa, s);
    case 5: return stage_batch_rk<R, 2, 1>(views, pre, geo, nmem, blocks, kappa, s);
    case 8: return stage_batch_rk<R, 4, 0>(views, pre, geo, nmem, blocks, kappa, s);
    case 9: return stage_batch_rk<R, 4, 1>(views, pre, geo, nmem, blocks, kappa, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t launch_stage_batch(uint32_t radius, uint32_t k, uint32_t shape, const DevView* views, const uint32_t* pre,
                              const uint32_t* geo, uint32_t nmem, uint32_t blocks, uint32_t kappa,
                              hipStream_t s) {
  switch (radius) {
    case 1: return stage_batch_r<1>(k, shape, views, pre, geo, nmem, blocks, kappa, s);
    case 2: return stage_batch_r<2>(k, shape, views, pre, geo, nmem, blocks, kappa, s);
    case 3: return stage_batch_r<3>(k, shape, views, pre, geo, nmem, blocks, kappa, s);
    case 4: return stage_batch_r<4>(k, shape, views, pre, geo, nmem, blocks, kappa, s);
    case 5: return stage_batch_r<5>(k, shape, views, pre, geo, nmem, blocks, kappa, s);
    case 6: return stage_batch_r<6>(k, shape, views, pre, geo, nmem, blocks, kappa, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_finish_batch(const DevView* views, const uint32_t* pre, uint32_t nmem, uint32_t blocks,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_delta_finish_batch, dim3(blocks), dim3(256), 0, s, views, pre, nmem);
  return hipGetLastError();
}

hipError_t launch_commit_batch(const DevView* views, const uint32_t* pre, uint32_t nmem, uint32_t blocks,
                               uint32_t kappa, hipStream_t s) {
  hipLaunchKernelGGL(k_commit_batch, dim3(blocks), dim3(256), 0, s, views, pre, nmem, kappa);
  return hipGetLastError();
}

hipError_t launch_advance_batch(const DevView* views, uint32_t nmem, hipStream_t s) {
  hipLaunchKernelGGL(k_advance_batch, dim3((nmem + 63) / 64), dim3(64), 0, s, views, nmem);
  return hipGetLastError();
}
}  // namespace bnlat
