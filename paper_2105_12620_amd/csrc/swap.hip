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

// LDS-staged member evaluation.  A workgroup owns a BW x BH block of tile
// pixels; its pass members (pixels whose scrambled list position falls in the
// pass) are listed in LDS.  For 16 integrands at a time (two 8-integrand count
// planes, one stage) the counts of the block plus its window halo (region
// RH x RW, row pitch RWP = RW + 1) and the two partner words of every member
// are staged in LDS, and every member is served by a group of 16 lanes: lane
// (i, p) forms dc = c_partner - c_own of plane p and, per step, reads one
// 16-byte word of plane p at window offset i of the step.  A row step covers
// eight consecutive offsets of a window row, a column step eight consecutive
// rows of one of the columns the row steps leave over.  gfx950's LDS serves a
// ds_read_b128 in passes of 16 lanes over 64 four-byte banks: with the plane
// stride 8 words of 16 bytes past a multiple of 16 and RWP odd, the 16 words
// a group reads fall in 16 distinct bank quads wherever the member lies, so
// every pass is conflict-free.
//
// Staging is a ring of three stage buffers filled straight from HBM by
// global_load_lds_dwordx4 (lane l of a load writes 16 bytes at the wave's LDS
// base + 16 l): the loads of stage s + 2 are issued while stage s is
// evaluated.  Every wave issues the same number D of loads per stage (slots
// past the stage's loads repeat one of them), so waiting for stage s is
// s_waitcnt vmcnt(D) while stage s + 1 is in flight (loads return in order),
// followed by a barrier without a memory fence (a fence would wait for every
// load in flight).  A stage buffer is refilled only after the barrier that
// follows the last reads of it.
//
// A lane accumulates its product of each step separately (int32 per step);
// when the member's integrand slice is done, the steps' sums are gathered
// into distance classes (the lane's offset of a step fixes the class),
// reduced over the group and added to HBM with exact int64 atomics, member
// by member in a contiguous row of classes.  The workgroups are renumbered
// per XCD (xcd_block), so that the blocks one L2 serves at a time are whole
// rows of blocks of one integrand slice and their halos are read from HBM
// once.
//
// Integrand slices of the tile run in separate workgroups; per-lane int32
// step sums stay below 2^31 because the host bounds a slice to S stages with
// S * 8 N^2 < 2^31 (eight products of at most N^2 per lane and stage).

template <int R>
struct SwapGeom {
  static constexpr int BW = 32, BH = (R <= 4) ? 8 : 4;   // tile pixels per workgroup
  static constexpr int WS = 2 * R + 1;                   // window side
  static constexpr int RW = BW + 2 * R, RH = BH + 2 * R;
  static constexpr int RWP = RW + 1;                     // odd row pitch (16-byte words)
  static constexpr int RA = RH * RWP;                    // words of one plane's region
  static constexpr int RA_PAD = (RA + 63) / 64 * 64;     // whole 64-lane loads
  static constexpr int PLANE = RA_PAD + 8;               // plane stride: 8 past a multiple of 16
  static constexpr int NT = 512;                         // threads
  static constexpr int NWAVE = NT / 64;
  static constexpr int GL = 16;                          // lanes per member group
  static constexpr int GROUPS = NT / GL;
  static constexpr int SLOTS = (R <= 4) ? 3 : 2;         // members per group and round
  static constexpr int CAP = GROUPS * SLOTS;             // members per round
  static constexpr int PART = 2 * CAP;                   // partner words per stage
  static constexpr int SBUF = 2 * PLANE + PART;          // words of one stage buffer
  static constexpr int NBUF = 3;                         // ring depth
  static constexpr int PD = NBUF - 1;                    // stages loaded ahead
  static constexpr int NRL = 2 * RA_PAD / 64;            // region loads per stage
  static constexpr int NLD = NRL + PART / 64;            // loads per stage
  static constexpr int D = (NLD + NWAVE - 1) / NWAVE;    // loads per wave and stage
  static constexpr int RC = WS < 8 ? WS : 8;             // offsets of a row step
  static constexpr int LC = WS - RC;                     // columns left to column steps
  static constexpr int CH = (WS + 7) / 8;                // column steps per such column
  static constexpr int LASTROWS = WS - 8 * (CH - 1);     // rows of a column's last step
  static constexpr int STEPS = WS + LC * CH;
  static constexpr int NPIX = BW * BH;
  static constexpr int NWV = NPIX / 64;                  // waves that test membership
  static constexpr int LDS_BYTES = NBUF * SBUF * 16 + (3 * NPIX + NWV + 8 * STEPS) * 4;
  static_assert(NPIX % 64 == 0 && RWP % 2 == 1 && PLANE % 16 == 8 && PART % 64 == 0, "swap block geometry");
  static_assert(D * NWAVE < 2 * NLD, "repeated load slots");
  static_assert(PD >= 1 && PD <= 3 && (PD - 1) * D < 64, "ring depth and vmcnt");
};

// Window offset of lane slot i at step st (row steps first, then column
// steps), and whether the slot holds one.
template <int R>
__device__ inline bool swap_step_offset(int st, int i, int& ox, int& oy) {
  using G = SwapGeom<R>;
  if (st < G::WS) {
    oy = st - R;
    ox = -R + i;
    return i < G::RC;
  }
  const int t = st - G::WS, col = t / G::CH, part = t % G::CH;
  ox = -R + G::RC + col;
  oy = -R + 8 * part + i;
  return oy <= R;
}

template <int R>
__global__ __launch_bounds__(SwapGeom<R>::NT, (R <= 4) ? 4 : 2) void k_swap_stage(DevView v, SwapView sv, uint32_t kappa,
                                                                    uint32_t slen, uint32_t gx, uint32_t gy) {
  using G = SwapGeom<R>;
  constexpr int NCLS = WinConst<R>::NCLS;
  extern __shared__ u32x4 lds4[];
  uint32_t* mpos = (uint32_t*)(lds4 + G::NBUF * G::SBUF);   // [NPIX] region word of each member
  uint32_t* mj = mpos + G::NPIX;                   // [NPIX] list slot
  uint32_t* mb = mj + G::NPIX;                     // [NPIX] partner pixel
  uint32_t* wcnt = mb + G::NPIX;                   // [NWV] members per wave
  int* ctab = (int*)(wcnt + G::NWV);               // [STEPS][8] class of each step's slot (-1: none)
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t P = v.w * v.h;
  const uint32_t mask = swap_mask(v, kappa);
  const uint32_t wk = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxy = wk % (gx * gy), bz = wk / (gx * gy);
  const uint32_t x0 = (bxy % gx) * G::BW, y0 = (bxy / gx) * G::BH;

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
      pos = (ly + R) * G::RWP + lx + R;
    }
  }
  const unsigned long long bal = __ballot(in);
  if (lane == 0 && wv < (uint32_t)G::NWV) wcnt[wv] = (uint32_t)__popcll(bal);
  if (tid < 8u * G::STEPS) {
    int ox, oy;
    ctab[tid] = swap_step_offset<R>((int)tid / 8, (int)tid % 8, ox, oy) ? sv.dcls[ox * ox + oy * oy] : -1;
  }
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

  // load slot k of this wave issues load d = wv + NWAVE k of a stage (slots
  // past the stage's loads repeat load d - NLD).  Region load d < NRL covers
  // plane d / (RA_PAD / 64), region words 64 (d mod RA_PAD/64) + lane (the
  // padding column and words past the region load pixel 0); partner load d
  // covers partner words 64 (d - NRL) + lane = 2 m + plane of round member m,
  // read from the pixel-major copy (lsrc holds the partner pixel and plane).
  // W and H are powers of two.
  const uint32_t ys = (y0 + v.h * (R / v.h + 1) - R) % v.h;
  const uint32_t xs = (x0 + v.w * (R / v.w + 1) - R) % v.w;
  const uint32_t wm = v.w - 1, hm = v.h - 1;
  uint32_t ldst[G::D], lsrc[G::D];
#pragma unroll
  for (int k = 0; k < G::D; ++k) {
    uint32_t d = wv + G::NWAVE * k;
    if (d >= (uint32_t)G::NLD) d -= G::NLD;
    if (d < (uint32_t)G::NRL) {
      const uint32_t pl = d / (G::RA_PAD / 64), u0 = (d % (G::RA_PAD / 64)) * 64, u = u0 + lane;
      const uint32_t rr = u / G::RWP, cc = u - rr * G::RWP;
      const uint32_t gq = (u < (uint32_t)G::RA && cc < (uint32_t)G::RW) ? ((ys + rr) & hm) * v.w + ((xs + cc) & wm) : 0;
      ldst[k] = pl * G::PLANE + u0;
      lsrc[k] = pl * P + gq;
    } else {
      ldst[k] = 2 * G::PLANE + 64 * (d - G::NRL);
      lsrc[k] = 0;
    }
  }
  const uint32_t tp8 = v.tp >> 3;
  auto issue = [&](uint32_t t0, uint32_t buf) {
    const u32x4* cs = (const u32x4*)(v.cnt + (size_t)(t0 >> 3) * P * 8);
    const u32x4* rs = (const u32x4*)sv.row + (t0 >> 3);
#pragma unroll
    for (int k = 0; k < G::D; ++k) {
      const u32x4* src = ldst[k] < 2u * G::PLANE ? cs + lsrc[k] : rs + (size_t)(lsrc[k] >> 1) * tp8 + (lsrc[k] & 1);
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                       (__attribute__((address_space(3))) void*)(lds4 + buf * G::SBUF + ldst[k]),
                                       16, 0, 0);
    }
  };

  const uint32_t grp = tid / G::GL, li = tid & 7, lp = (tid >> 3) & 1;
  // word of the lane's slot relative to the member's own word of plane lp:
  // row steps, column steps, a column's last step (lanes past the window
  // repeat its last offset)
  const uint32_t lr = min(li, (uint32_t)G::RC - 1), lc = li * G::RWP,
                 lcl = min(li, (uint32_t)G::LASTROWS - 1) * G::RWP;
  // the same shifted so that every step reads at a non-negative constant
  // offset, and the partner word of the group's first slot
  const uint32_t rof = lr - (R * G::RWP + R), cof = lc - (R * G::RWP + R - G::RC),
                 clof = lcl - (R * G::RWP + R - G::RC), pe0 = 2 * G::PLANE + 2 * grp + lp;
  const uint32_t t_begin = bz * slen, t_end = min(t_begin + slen, v.tp);
  const uint32_t nst = t_end > t_begin ? (t_end - t_begin) / 16 : 0;
  __syncthreads();
  for (uint32_t base = 0; base < nm; base += G::CAP) {
    // this round's partner pixels
#pragma unroll
    for (int k = 0; k < G::D; ++k) {
      if (ldst[k] >= 2u * G::PLANE) {
        // partner word 2 base + e of the round (its member and plane), with
        // the wave-uniform part summed first: kept per load across rounds,
        // the lane parts spilled at radius 4
        const uint32_t e2 = __builtin_amdgcn_readfirstlane(2 * base + ldst[k] - 2 * G::PLANE) + lane,
                       m = e2 >> 1;
        lsrc[k] = (m < nm ? mb[m] : 0) * 2 + (e2 & 1);
      }
    }
    int acc[G::SLOTS][G::STEPS];
    int dd[G::SLOTS];
    // per slot: the member's own word of plane lp; the lane's reads are at
    // fixed offsets from it (one register per slot rather than one per step
    // kind: fewer spills at radius 4)
    uint32_t sp[G::SLOTS];
    bool ok[G::SLOTS];
#pragma unroll
    for (int s = 0; s < G::SLOTS; ++s) {
      const uint32_t mi = grp + G::GROUPS * s;
      ok[s] = base + mi < nm;
      sp[s] = lp * G::PLANE + (ok[s] ? mpos[base + mi] : (uint32_t)(R * G::RWP + R));
      dd[s] = 0;
#pragma unroll
      for (int st = 0; st < G::STEPS; ++st) acc[s][st] = 0;
    }
    // the previous round's reads of the ring are done
    barrier_vm<0>();
#pragma unroll
    for (int k = 0; k < G::PD; ++k)
      if ((uint32_t)k < nst) issue(t_begin + 16 * k, k);
    for (uint32_t si = 0; si < nst; ++si) {
      // stage si has landed once at most the loads of the stages issued
      // after it (up to PD - 1 of them) are in flight
      const uint32_t ahead = min((uint32_t)G::PD - 1, nst - 1 - si);
      if (G::PD >= 3 && ahead == 2) barrier_vm<2 * G::D>();
      else if (G::PD >= 2 && ahead == 1) barrier_vm<G::D>();
      else barrier_vm<0>();
      if (si + G::PD < nst) issue(t_begin + 16 * (si + G::PD), (si + G::PD) % G::NBUF);
      const u32x4* bf = lds4 + (si % G::NBUF) * G::SBUF;
#pragma unroll
      for (int s = 0; s < G::SLOTS; ++s) {
        if (ok[s]) {
          const u32x4 own = bf[sp[s]], pc = bf[pe0 + 2 * G::GROUPS * s];
          uint32_t dl[4];
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            // per int16 half: partner minus own count (|dc| <= N, no wrap); the
            // words go through scalars (a bit cast straight from the vector
            // element read only the first word)
            const uint32_t pw_h = pc[h], ow_h = own[h];
            dl[h] = __builtin_bit_cast(uint32_t, (v2i16)(__builtin_bit_cast(v2i16, pw_h) -
                                                         __builtin_bit_cast(v2i16, ow_h)));
            dd[s] = dot2(dl[h], dl[h], dd[s]);
          }
          const u32x4* rp = bf + (sp[s] + rof);
          const u32x4* cp = bf + (sp[s] + cof);
          const u32x4* clp = bf + (sp[s] + clof);
#pragma unroll
          for (int st = 0; st < G::STEPS; ++st) {
            u32x4 c;
            if (st < G::WS) {
              c = rp[st * G::RWP];
            } else {
              const int t = st - G::WS, col = t / G::CH, part = t % G::CH;
              c = (part < G::CH - 1 ? cp : clp)[col + 8 * part * G::RWP];
            }
            int a = acc[s][st];
            a = dot2(dl[0], c[0], a);
            a = dot2(dl[1], c[1], a);
            a = dot2(dl[2], c[2], a);
            acc[s][st] = dot2(dl[3], c[3], a);
          }
        }
      }
    }
    // gather each member's step sums into classes, reduce over the group's
    // 16 lanes and add them to HBM
#pragma unroll
    for (int s = 0; s < G::SLOTS; ++s) {
      if (!ok[s]) continue;
      long long cl[NCLS];
#pragma unroll
      for (int c = 0; c < NCLS; ++c) cl[c] = 0;
#pragma unroll
      for (int st = 0; st < G::STEPS; ++st) {
        const int c = ctab[st * 8 + li];
#pragma unroll
        for (int cc = 0; cc < NCLS; ++cc) cl[cc] += (c == cc) ? (long long)acc[s][st] : 0ll;
      }
#pragma unroll
      for (int c = 0; c < NCLS; ++c) {
#pragma unroll
        for (int off = 1; off < G::GL; off <<= 1) cl[c] += __shfl_xor(cl[c], off);
      }
      // dc^2 of plane lp is the same in the group's eight slots
      long long d = li == 0 ? (long long)dd[s] : 0ll;
#pragma unroll
      for (int off = 1; off < G::GL; off <<= 1) d += __shfl_xor(d, off);
      const uint32_t js = mj[base + grp + G::GROUPS * s];
      const uint32_t l16 = tid & 15;
#pragma unroll
      for (int c0 = 0; c0 < NCLS; c0 += G::GL) {
        const uint32_t c = c0 + l16;
        long long x = 0;
#pragma unroll
        for (int cc = c0; cc < c0 + G::GL && cc < NCLS; ++cc) x = (c == (uint32_t)cc) ? cl[cc] : x;
        if (c < (uint32_t)NCLS && x)
          atomicAdd((unsigned long long*)&sv.xs[(size_t)js * NCLS + c], (unsigned long long)(-2 * x));
      }
      if (l16 == 0 && !(js & 1u) && d) atomicAdd((unsigned long long*)&sv.d2[js >> 1], (unsigned long long)d);
    }
  }
}

// Decision of couple i: add the two members' class sums and the pair
// correction, take the FP64 weighted sum in increasing d and decide; the sums
// are cleared for the next pass (all of a couple's sums are loaded before any
// is cleared, so the loads are in flight together).  Writes delta, accept and
// the couple's pixels (u_new); returns the decision and the pixels.
template <int R>
__device__ __forceinline__ bool swap_decide(const DevView& v, const SwapView& sv, uint32_t kappa, uint32_t i,
                                            uint32_t& a, uint32_t& b) {
  constexpr int NCLS = WinConst<R>::NCLS;
  const uint32_t mask = swap_mask(v, kappa);
  const uint32_t L = kappa * sv.m + 2 * i;
  a = sv.perm[L] ^ mask;
  b = sv.perm[L + 1] ^ mask;
  long long* xp = sv.xs + (size_t)2 * i * NCLS;
  long long x[NCLS];
#pragma unroll
  for (int c = 0; c < NCLS; ++c) x[c] = xp[c] + xp[NCLS + c];
  const long long d2 = sv.d2[i];
  // the rows of the two members: 2 NCLS int64, 16-byte aligned
#pragma unroll
  for (int c = 0; c < NCLS; ++c) ((uint4*)xp)[c] = make_uint4(0u, 0u, 0u, 0u);
  sv.d2[i] = 0;
  // offsets o with a + o = b on the torus: o = d or d - W per axis with
  // d = (b - a) mod W (two per axis at most because r < min(W, H)); W and H
  // are powers of two
  const uint32_t lw = __builtin_ctz(v.w), wm = v.w - 1, hm = v.h - 1;
  const int dx = (int)(((b & wm) - (a & wm)) & wm), dy = (int)(((b >> lw) - (a >> lw)) & hm);
  const int cx[2] = {dx, dx - (int)v.w}, cy[2] = {dy, dy - (int)v.h};
#pragma unroll
  for (int ky = 0; ky < 2; ++ky) {
#pragma unroll
    for (int kx = 0; kx < 2; ++kx) {
      const int ox = cx[kx], oy = cy[ky];
      if (ox < -R || ox > R || oy < -R || oy > R || (ox == 0 && oy == 0)) continue;
      const int cl = sv.dcls[ox * ox + oy * oy];
#pragma unroll
      for (int c = 0; c < NCLS; ++c) x[c] += (c == cl) ? 2 * d2 : 0ll;
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < NCLS; ++c) acc = __dadd_rn(acc, __dmul_rn(v.wd[c], (double)x[c]));
  const double total = __dmul_rn(acc, 2.0 / ((double)v.n * (double)v.n));
  const bool ok = (v.objective > 0) ? (total < 0.0) : (total > 0.0);
  v.delta[i] = total;
  v.accept[i] = ok;
  v.u_new[2 * i] = a;
  v.u_new[2 * i + 1] = b;
  return ok;
}

// Exchange of an accepted couple's offsets and count tiles by one wave: the
// counts are read from the pixel-major copy (whole lines), written to both
// layouts.
__device__ __forceinline__ void swap_exchange(const DevView& v, const SwapView& sv, uint32_t a, uint32_t b,
                                              uint32_t lane) {
  if (lane == 0) {
    const uint32_t ua = v.U[a], ub = v.U[b];
    v.U[a] = ub;
    v.U[b] = ua;
    atomicAdd(&v.ctr[1], 1ull);
  }
  const uint32_t P = v.w * v.h;
  uint4* wa = (uint4*)(sv.row + (size_t)a * v.tp);
  uint4* wb = (uint4*)(sv.row + (size_t)b * v.tp);
  for (uint32_t tt = lane; tt < (v.tp >> 3); tt += 64) {
    const uint4 qa = wa[tt], qb = wb[tt];
    wa[tt] = qb;
    wb[tt] = qa;
    *(uint4*)(v.cnt + ((size_t)tt * P + a) * 8) = qb;
    *(uint4*)(v.cnt + ((size_t)tt * P + b) * 8) = qa;
  }
}

// One thread per couple: the decision alone (the phase-stepping calls).
template <int R>
__global__ __launch_bounds__(128) void k_swap_finish(DevView v, SwapView sv, uint32_t kappa) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (sv.m >> 1)) return;
  uint32_t a, b;
  (void)swap_decide<R>(v, sv, kappa, i, a, b);
}

// One wave per couple: decision and, if accepted, the exchange (the sweeps:
// one launch less per pass, and no round trip of the decision through HBM).
// Lane 0 decides; the wave then exchanges the couple.
template <int R>
__global__ __launch_bounds__(256) void k_swap_decide_exchange(DevView v, SwapView sv, uint32_t kappa) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t i = wave_id();
  if (i >= (sv.m >> 1)) return;
  uint32_t a = 0, b = 0, ok = 0;
  if (lane == 0) ok = swap_decide<R>(v, sv, kappa, i, a, b) ? 1u : 0u;
  ok = __builtin_amdgcn_readfirstlane(ok);
  if (!ok) return;
  a = __builtin_amdgcn_readfirstlane(a);
  b = __builtin_amdgcn_readfirstlane(b);
  swap_exchange(v, sv, a, b, lane);
}

// One wave per accepted couple: exchange offsets and count tiles.
__global__ __launch_bounds__(256) void k_swap_commit(DevView v, SwapView sv) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t i = wave_id();
  if (i >= (sv.m >> 1) || !v.accept[i]) return;
  swap_exchange(v, sv, v.u_new[2 * i], v.u_new[2 * i + 1], lane);
}

// Pixel-major copy of the tiled counts: thread per (pixel, 8-integrand tile),
// pixels fastest, so that the tiled reads are coalesced.
__global__ __launch_bounds__(256) void k_swap_rows(DevView v, SwapView sv) {
  const uint32_t P = v.w * v.h;
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (uint64_t)P * (v.tp >> 3)) return;
  const uint32_t tt = (uint32_t)(i / P), p = (uint32_t)(i - (uint64_t)tt * P);
  *((uint4*)(sv.row + (size_t)p * v.tp) + tt) = *(const uint4*)(v.cnt + ((size_t)tt * P + p) * 8);
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
                            (int)SwapGeom<RR>::LDS_BYTES);
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

// Integrand slices: enough workgroups for about 1024 threads on each of the
// 256 CUs, and few enough stages per slice that every per-lane int32 step sum
// stays below 2^31.
template <int R>
hipError_t swap_stage_launch(const DevView& v, const SwapView& sv, uint32_t kappa, hipStream_t s, bool decide) {
  using G = SwapGeom<R>;
  const uint32_t gx = (v.w + G::BW - 1) / G::BW, gy = (v.h + G::BH - 1) / G::BH, chunks = v.tp / 16;
  const double n2 = (double)v.n * v.n;
  const uint32_t smax = (uint32_t)std::max(1.0, std::floor(2147483647.0 / (8.0 * n2)));
  // about 1024 threads per CU of 256 CUs
  const uint32_t target = 262144 / G::NT;
  uint32_t nz = std::max<uint32_t>(1, std::min<uint32_t>(chunks, (target + gx * gy - 1) / (gx * gy)));
  uint32_t per = (chunks + nz - 1) / nz;
  if (per > smax) per = smax;
  nz = (chunks + per - 1) / per;
  hipLaunchKernelGGL(k_swap_stage<R>, dim3(gx * gy * nz), dim3(G::NT), (size_t)G::LDS_BYTES, s, v, sv, kappa,
                     per * 16, gx, gy);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !decide) return e;
  const uint32_t half = sv.m >> 1;
  hipLaunchKernelGGL(k_swap_finish<R>, dim3((half + 127) / 128), dim3(128), 0, s, v, sv, kappa);
  return hipGetLastError();
}

hipError_t launch_swap_evaluate(const DevView& v, const SwapView& sv, uint32_t kappa, hipStream_t s, bool decide) {
  switch (v.radius) {
    case 1: return swap_stage_launch<1>(v, sv, kappa, s, decide);
    case 2: return swap_stage_launch<2>(v, sv, kappa, s, decide);
    case 3: return swap_stage_launch<3>(v, sv, kappa, s, decide);
    case 4: return swap_stage_launch<4>(v, sv, kappa, s, decide);
    case 5: return swap_stage_launch<5>(v, sv, kappa, s, decide);
    case 6: return swap_stage_launch<6>(v, sv, kappa, s, decide);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_swap_decide_exchange(const DevView& v, const SwapView& sv, uint32_t kappa, hipStream_t s) {
  const dim3 g(((sv.m >> 1) + 3) / 4), b(256);
  switch (v.radius) {
    case 1: hipLaunchKernelGGL(k_swap_decide_exchange<1>, g, b, 0, s, v, sv, kappa); break;
    case 2: hipLaunchKernelGGL(k_swap_decide_exchange<2>, g, b, 0, s, v, sv, kappa); break;
    case 3: hipLaunchKernelGGL(k_swap_decide_exchange<3>, g, b, 0, s, v, sv, kappa); break;
    case 4: hipLaunchKernelGGL(k_swap_decide_exchange<4>, g, b, 0, s, v, sv, kappa); break;
    case 5: hipLaunchKernelGGL(k_swap_decide_exchange<5>, g, b, 0, s, v, sv, kappa); break;
    case 6: hipLaunchKernelGGL(k_swap_decide_exchange<6>, g, b, 0, s, v, sv, kappa); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_swap_rows(const DevView& v, const SwapView& sv, hipStream_t s) {
  const uint64_t n = (uint64_t)v.w * v.h * (v.tp >> 3);
  hipLaunchKernelGGL(k_swap_rows, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, v, sv);
  return hipGetLastError();
}

hipError_t launch_swap_commit(const DevView& v, const SwapView& sv, hipStream_t s) {
  const uint32_t half = sv.m >> 1;
  hipLaunchKernelGGL(k_swap_commit, dim3((half + 3) / 4), dim3(256), 0, s, v, sv);
  return hipGetLastError();
}

}  // namespace bnlat
