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

// LDS-staged member evaluation.  A workgroup owns a 32 x 6 block of tile
// pixels; its pass members (pixels whose scrambled list position falls in the
// pass) are listed in LDS.  For 64 integrands at a time the counts of the
// block plus its window halo are staged in LDS (region RH x RW), and every
// member is served by a group of 16 lanes, lane k holding integrands
// 4k .. 4k+3 of dc = c_partner - c_own (partner counts read from HBM, own
// counts from LDS).  Per window offset a group reads the neighbour's 32 words
// with one ds_read_b64 per lane and takes two v_dot2 per lane.
//
// Staging goes straight from HBM to LDS (global_load_lds_dwordx4: lane l of a
// load writes 16 bytes at the wave's LDS base + 16 l).  LDS holds eight planes
// (one per 8-integrand tile) of RA_PAD pixels x 4 words; the plane stride is 4
// words past a multiple of 32, so the 32 words a group reads for one
// neighbour fall in 32 distinct banks.
//
// Integrand slices of the tile run in separate workgroups (grid z) and meet
// in exact int64 atomics; per-lane int32 partial sums stay below 2^31 because
// the host bounds a slice to S stages with S * 48 N^2 < 2^31 (at most 12
// offsets per distance class, 4 integrands per lane per stage).

template <int R>
struct SwapGeom {
  static constexpr int BW = 32, BH = 6;          // tile pixels per workgroup
  static constexpr int RW = BW + 2 * R, RH = BH + 2 * R;
  static constexpr int RA = RW * RH;             // region pixels
  static constexpr int RA_PAD = (RA + 63) / 64 * 64;
  static constexpr int PLANE = RA_PAD * 4 + 4;   // words per 8-integrand plane
  static constexpr int NPLANE = 8;               // 8-integrand tiles per stage (64 integrands)
  static constexpr int BUF = NPLANE * PLANE;     // words of the stage buffer
  static constexpr int GL = 16;                  // lanes per member group
  static constexpr int NT = 512;                 // threads
  static constexpr int NWAVE = NT / 64;
  static constexpr int LOADS = NPLANE * RA_PAD / 64;   // 64-lane 16-byte loads per stage
  static constexpr int GROUPS = NT / GL;         // 32 member groups
  static constexpr int SLOTS = 2;                // members per group and round
  static constexpr int CAP = GROUPS * SLOTS;     // members per round
  static constexpr int NPIX = BW * BH;
  static constexpr int NWV = (NPIX + 63) / 64;   // waves that test membership
  static constexpr int LDS_WORDS = BUF + 3 * NPIX + NWV;
};

template <int R>
__global__ __launch_bounds__(512, (R <= 4) ? 4 : 2) void k_swap_stage(DevView v, SwapView sv, uint32_t kappa,
                                                                    uint32_t slen) {
  using G = SwapGeom<R>;
  constexpr Window<R> W = WinConst<R>::w;
  constexpr int NCLS = WinConst<R>::NCLS;
  extern __shared__ uint32_t lds[];
  uint32_t* mpos = lds + G::BUF;                   // [NPIX] region pixel of each member
  uint32_t* mj = mpos + G::NPIX;                   // [NPIX] list slot
  uint32_t* mb = mj + G::NPIX;                     // [NPIX] partner pixel
  uint32_t* wcnt = mb + G::NPIX;                   // [NWV] members per wave
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint32_t P = v.w * v.h;
  const uint32_t mask = swap_mask(v, kappa);
  const uint32_t x0 = blockIdx.x * G::BW, y0 = blockIdx.y * G::BH;

  // members of the block, in raster order
  bool in = false;
  uint32_t j = 0, b = 0, pos = 0;
  if (tid < (uint32_t)G::NPIX) {
    const uint32_t ly = tid / G::BW, lx = tid % G::BW;
    if (y0 + ly < v.h && x0 + lx < v.w) {
      const uint32_t L = sv.pinv[((y0 + ly) * v.w + x0 + lx) ^ mask];
      in = L / sv.m == kappa;
      j = L - kappa * sv.m;
      b = sv.perm[L ^ 1u] ^ mask;
      pos = (ly + R) * G::RW + lx + R;
    }
  }
  const unsigned long long bal = __ballot(in);
  if (lane == 0 && wv < (uint32_t)G::NWV) wcnt[wv] = (uint32_t)__popcll(bal);
  __syncthreads();
  uint32_t before = 0, nm = 0;
#pragma unroll
  for (int q = 0; q < G::NWV; ++q) {
    if ((uint32_t)q < wv) before += wcnt[q];
    nm += wcnt[q];
  }
  if (in) {
    const uint32_t idx = before + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
    mpos[idx] = pos;
    mj[idx] = j;
    mb[idx] = b;
  }

  // region pixel -> tile pixel (W and H are powers of two for swap problems)
  const uint32_t ys = (y0 + v.h * (R / v.h + 1) - R) % v.h;
  const uint32_t xs = (x0 + v.w * (R / v.w + 1) - R) % v.w;
  const uint32_t wm = v.w - 1, hm = v.h - 1;
  // the stage at t0: load n covers plane n / (RA_PAD / 64), region pixels
  // 64 (n mod RA_PAD/64) + lane (padding lanes reload pixel 0)
  auto issue_stage = [&](uint32_t t0) {
    for (uint32_t n = wv; n < (uint32_t)G::LOADS; n += G::NWAVE) {
      const uint32_t plane = n / (G::RA_PAD / 64), pix0 = (n % (G::RA_PAD / 64)) * 64;
      const uint32_t pix = pix0 + lane;
      uint32_t gq = 0;
      if (pix < (uint32_t)G::RA) {
        const uint32_t rr = pix / G::RW, cc = pix - rr * G::RW;
        gq = ((ys + rr) & hm) * v.w + ((xs + cc) & wm);
      }
      const uint16_t* src = v.cnt + tix(gq, t0 + 8 * plane, P);
      uint32_t* dst = lds + plane * G::PLANE + 4 * pix0;
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                       (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
  };

  const uint32_t grp = tid / G::GL, k = tid % G::GL;
  const uint32_t lane_word = (k >> 1) * G::PLANE + 2 * (k & 1);
  const uint32_t t_begin = blockIdx.z * slen, t_end = min(t_begin + slen, v.tp);
  __syncthreads();
  for (uint32_t base = 0; base < nm; base += G::CAP) {
    int acc[G::SLOTS][NCLS];
    int dd[G::SLOTS];
    uint32_t spos[G::SLOTS], sb[G::SLOTS];
    bool ok[G::SLOTS];
#pragma unroll
    for (int s = 0; s < G::SLOTS; ++s) {
      const uint32_t mi = base + grp * G::SLOTS + s;
      ok[s] = mi < nm;
      spos[s] = ok[s] ? mpos[mi] : 0;
      sb[s] = ok[s] ? mb[mi] : 0;
      dd[s] = 0;
#pragma unroll
      for (int c = 0; c < NCLS; ++c) acc[s][c] = 0;
    }
    for (uint32_t t0 = t_begin; t0 < t_end; t0 += 64) {
      // partner counts: integrands t0 + 4k .. +3 (one 8-byte piece of a tile)
      uint2 pw[G::SLOTS];
#pragma unroll
      for (int s = 0; s < G::SLOTS; ++s) pw[s] = *(const uint2*)(v.cnt + tix(sb[s], t0 + 4 * k, P));
      __syncthreads();
      issue_stage(t0);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      const uint32_t* reg = lds + lane_word;
#pragma unroll
      for (int s = 0; s < G::SLOTS; ++s) {
        if (ok[s]) {
          const uint32_t* rp = reg + 4 * spos[s];
          const uint2 own = *(const uint2*)rp;
          const uint32_t pws[2] = {pw[s].x, pw[s].y}, ows[2] = {own.x, own.y};
          uint32_t dl[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int d0 = (int)(pws[h] & 0xFFFFu) - (int)(ows[h] & 0xFFFFu);
            const int d1 = (int)(pws[h] >> 16) - (int)(ows[h] >> 16);
            dl[h] = ((uint32_t)d0 & 0xFFFFu) | ((uint32_t)d1 << 16);
            dd[s] = dot2(dl[h], dl[h], dd[s]);
          }
#pragma unroll
          for (int mm = 0; mm < W.M; ++mm) {
            const int disp = 4 * (W.oy[mm] * G::RW + W.ox[mm]);
            const uint2 c = *(const uint2*)(rp + disp);
            int a = acc[s][W.cls[mm]];
            a = dot2(dl[0], c.x, a);
            a = dot2(dl[1], c.y, a);
            acc[s][W.cls[mm]] = a;
          }
        }
      }
    }
    // all reads of the buffers are done before a next round stages again
    __syncthreads();
    // members' class sums: reduce over the group's 16 lanes, add to HBM
#pragma unroll
    for (int s = 0; s < G::SLOTS; ++s) {
      if (!ok[s]) break;   // slots fill in order
      const uint32_t js = mj[base + grp * G::SLOTS + s];
#pragma unroll
      for (int c = 0; c < NCLS; ++c) {
        long long x = acc[s][c];
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (k == 0 && x) atomicAdd((unsigned long long*)&sv.xs[(size_t)c * sv.m + js], (unsigned long long)(-2 * x));
      }
      long long d = dd[s];
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) d += __shfl_xor(d, off);
      if (k == 0 && !(js & 1u) && d) atomicAdd((unsigned long long*)&sv.d2[js >> 1], (unsigned long long)d);
    }
  }
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

// One wave per accepted couple: exchange offsets and count tiles.
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
  const uint32_t P = v.w * v.h;
  for (uint32_t tt = lane; tt < (v.tp >> 3); tt += 64) {
    uint4* ra = (uint4*)(v.cnt + ((size_t)tt * P + a) * 8);
    uint4* rb = (uint4*)(v.cnt + ((size_t)tt * P + b) * 8);
    const uint4 qa = *ra, qb = *rb;
    *ra = qb;
    *rb = qa;
  }
}

}  // namespace

// The staged kernels use more than 64 KiB of LDS per workgroup (gfx950 has
// 160 KiB per CU); the launch limit is raised once per process.
hipError_t prepare_swap_kernels() {
  static hipError_t status = [] {
    hipError_t e = hipSuccess;
#define BN_SWAP_ATTR(RR)                                                                               \
  if (e == hipSuccess)                                                                                 \
    e = hipFuncSetAttribute((const void*)k_swap_stage<RR>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                            (int)(SwapGeom<RR>::LDS_WORDS * 4));
    BN_SWAP_ATTR(1)
    BN_SWAP_ATTR(2)
    BN_SWAP_ATTR(3)
    BN_SWAP_ATTR(4)
    BN_SWAP_ATTR(5)
    BN_SWAP_ATTR(6)
#undef BN_SWAP_ATTR
    return e;
  }();
  return status;
}

// Integrand slices: enough workgroups to fill the device, and few enough
// stages per slice that every per-lane int32 partial sum stays below 2^31.
hipError_t launch_swap_evaluate(const DevView& v, const SwapView& sv, uint32_t kappa, hipStream_t s) {
  const uint32_t gx = (v.w + 31) / 32, gy = (v.h + 5) / 6, chunks = v.tp / 64;
  const double n2 = (double)v.n * v.n;
  const uint32_t smax = (uint32_t)std::max(1.0, std::floor(2147483647.0 / (48.0 * n2)));
  uint32_t nz = std::max<uint32_t>(1, std::min<uint32_t>(chunks, (1024 + gx * gy - 1) / (gx * gy)));
  uint32_t per = (chunks + nz - 1) / nz;
  if (per > smax) per = smax;
  nz = (chunks + per - 1) / per;
  const uint32_t slen = per * 64;
  const dim3 grid(gx, gy, nz), block(512);
  switch (v.radius) {
#define BN_SWAP_STAGE(RR)                                                                           \
  case RR:                                                                                          \
    hipLaunchKernelGGL(k_swap_stage<RR>, grid, block, (size_t)SwapGeom<RR>::LDS_WORDS * 4, s, v, sv, \
                       kappa, slen);                                                                \
    break;
    BN_SWAP_STAGE(1)
    BN_SWAP_STAGE(2)
    BN_SWAP_STAGE(3)
    BN_SWAP_STAGE(4)
    BN_SWAP_STAGE(5)
    BN_SWAP_STAGE(6)
#undef BN_SWAP_STAGE
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
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
