// BF16 precision form of the colour phases' energy change, on the matrix
// cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation).
//
// The energy change of a move (Eq. (1) over the window, both orderings of a
// pair) splits as
//     dE = 2 [ W sum_t d_t (e'_t + e_t)  -  2 sum_o w_o sum_t d_t e_{p+o,t} ],
// d = e' - e, W = sum_o w_o.  The neighbour products sum_t d_t e_q,t (a Gram
// block of the moved pixels against their window region) run on the matrix
// cores with BF16 operands read from a BF16 copy of the error field kept in
// HBM (tiled like the counts, [Tb/8][P][8], Tb = Tp + TGp: Heaviside rows then
// Gaussian rows).  Two modes:
//   exact (N <= 256, Heaviside rows only): the BF16 field holds the hit
//     counts themselves and the change operand is c' - c, both exact in
//     BF16; a slice whose partial sums stay below 2^24 is exact in FP32
//     (certified when N sum_t |c' - c| < 2^24), and the result is the exact
//     integer class sum.  Uncertified accepted moves are re-checked.
//   approximate (N > 256 or Gaussian rows): the field holds e = c/N - A (or
//     g - I) formed in FP32 and rounded to BF16, the change operand is
//     d = e' - e rounded to BF16, the self term is kept in full precision.
//     Every move this value accepts is re-evaluated exactly (integer
//     Heaviside part, FP64 Gaussian part) and committed only if confirmed;
//     a reversed decision counts as a veto.
// Class sums of a slice are added across slices with 64-bit integer atomics:
// exact integers, or in the approximate mode FP32 sums converted to fixed
// point with 40 fraction bits (so the total, and the decision, do not depend
// on the order of the slices).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bnlat_dev.h"
#include "device_common.h"

namespace bnlat {
namespace {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// LDS words written by global_load_lds are read as clang vector types: reads
// through HIP's struct vector types make the compiler wait for every load
// into LDS in flight (the waits here are explicit)
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// The whole BF16 field from the current counts and Gaussian estimates; one
// thread per (8-integrand tile, pixel), pixels fastest.
__global__ __launch_bounds__(256) void k_bf_field(DevView v) {
  const uint32_t P = v.w * v.h;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)P * (v.tb >> 3)) return;
  const uint32_t t8 = (uint32_t)(i / P), p = (uint32_t)(i - (size_t)t8 * P);
  uint4 out;
  if (t8 < (v.tp >> 3)) {
    out = heaviside_field_tile(v, *(const uint4*)(v.cnt + ((size_t)t8 * P + p) * 8), t8 * 8);
  } else {
    const uint32_t t = (t8 - (v.tp >> 3)) * 8;
    const float* g = v.gest + (size_t)p * v.tgp + t;
    uint32_t o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      o[k] = bf16x2_bits(gaussian_error(v, g[2 * k], t + 2 * k), gaussian_error(v, g[2 * k + 1], t + 2 * k + 1));
    out = make_uint4(o[0], o[1], o[2], o[3]);
  }
  *(uint4*)(v.bf + i * 8) = out;
}

// ----------------------------------------------------------- the Gram kernel
//
// A workgroup owns BYC class rows x 16 class pixels; wave w owns class row w,
// the 16 rows of its MFMA tiles.  Per 16-integrand slice the field words of
// the window region (RROWS x RUSED pixels, two 16-byte words of 8 integrands
// each) go from HBM straight into a ring of LDS slots (global_load_lds, no
// registers), PD = NBUF - 1 slices ahead of the one multiplied, and the
// class pixels' count words likewise one slice ahead; every lane forms its
// own change operand (class pixel lane % 16, integrands 4 (lane / 16) .. +3
// of the slice).  Gaussian rows (approximate mode) go one slice at a time,
// their estimates through registers.  For every neighbour row oy of the pass and
// column tile ct, v_mfma_f32_16x16x16_bf16 accumulates
//     C[b][col] += sum_t d[b][t] * f[row][col][t]
// and pixel b's window entries are the columns K b + R + ox (the columns past
// RUSED read the next row's words or the slot's tail: their outputs are never
// read back).  Window rows are split into passes when their accumulators
// would exceed 40 tiles (160 registers); the self term is added by pass 0
// only.
template <int R, int K, int BYC, int OY0, int NOY>
struct BfGeom {
  static constexpr int BXC = 16;
  static constexpr int RROWS = K * (BYC - 1) + NOY;
  static constexpr int RUSED = K * (BXC - 1) + 2 * R + 1;
  static constexpr int NT = (RUSED + 15) / 16;               // column tiles
  static constexpr int RCOLS = 16 * NT;
  static constexpr int NTH = 64 * BYC;                       // threads
  static constexpr int PLANE = RROWS * RUSED;                // region pixels
  // a plane per tile half, padded to 256 bytes: the four 16-lane groups of a
  // read then agree modulo 256 bytes
  static constexpr int PLANE_PAD = (PLANE + 15) / 16 * 16;
  // region loads per thread and slice: every wave issues the same number
  // (words past the planes load pixel 0 into the slot's tail), and the reads
  // of the column tiles past RUSED stay inside the slot
  static constexpr int ITERD = (2 * PLANE_PAD + RCOLS - RUSED + NTH - 1) / NTH;
  static constexpr int SLOT = ITERD * NTH;                   // 16-byte words
  // change-operand words: two slots of 128 16-byte words per wave
  static constexpr int ARING_BYTES = 2 * BYC * 128 * 16;
  // three region slots where two workgroups still fit on a CU, else two
  static constexpr int NBUF = 3 * SLOT * 16 + ARING_BYTES <= 81920 ? 3 : 2;
  static constexpr int PD = NBUF - 1;
  static constexpr int STAGE_BYTES = NBUF * SLOT * 16 + ARING_BYTES;
  static constexpr int EXTRACT_BYTES = BYC * 16 * RCOLS * 4;
  static constexpr int LDS_BYTES = STAGE_BYTES > EXTRACT_BYTES ? STAGE_BYTES : EXTRACT_BYTES;
};

template <int R, int K, int BYC, int OY0, int NOY>
__global__ __launch_bounds__(64 * BYC) void k_delta_bf(DevView v, uint32_t kappa, uint32_t trlen,
                                                      long long* __restrict__ xsum, uint32_t* __restrict__ unsure) {
  // raised issue priority beside the sweep-wide recount (as the FP32 phase kernels)
  __builtin_amdgcn_s_setprio(2);
  using G = BfGeom<R, K, BYC, OY0, NOY>;
  constexpr Window<R> W = WinConst<R>::w;
  constexpr int NCLS = WinConst<R>::NCLS;
  extern __shared__ uint4 lds16[];
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t a0 = blockIdx.y * BYC, b0 = blockIdx.x * G::BXC;
  const uint32_t ky = kappa / K, kx = kappa - ky * K;
  const uint32_t ys = (ky + K * a0 + v.h * (R / v.h + 1) - R + OY0) % v.h;
  const uint32_t xs = (kx + K * b0 + v.w * (R / v.w + 1) - R) % v.w;
  const uint32_t P = v.w * v.h;
  const bool approx = v.mfma == 2;

  // region loads: load it of wave w moves slot words it NTH + 64 w + lane;
  // word i is (tile half i / PLANE_PAD, region pixel i mod PLANE_PAD), its
  // source the byte offset below from the slice's first field word
  uint32_t src[G::ITERD];
#pragma unroll
  for (int it = 0; it < G::ITERD; ++it) {
    const uint32_t i = it * G::NTH + threadIdx.x;
    const uint32_t half = i / G::PLANE_PAD, pix = i - half * G::PLANE_PAD;
    src[it] = 0;
    if (half < 2 && pix < (uint32_t)G::PLANE) {
      const uint32_t rr = pix / G::RUSED, cc = pix - rr * G::RUSED;
      uint32_t gy = ys + rr, gx = xs + cc;
      while (gy >= v.h) gy -= v.h;
      while (gx >= v.w) gx -= v.w;
      src[it] = (half * P + gy * v.w + gx) * 16;
    }
  }

  // the lane's class pixel and quarter (four integrands) of the slice
  const uint32_t quarter = lane >> 4, m = lane & 15;
  const uint32_t own_a = a0 + w, own_b = b0 + m;
  const bool own_ok = own_a < v.ch && own_b < v.cw;
  const uint32_t own_p = own_ok ? (ky + K * own_a) * v.w + (kx + K * own_b) : 0;
  const uint32_t own_j = own_ok ? own_a * v.cw + own_b : 0;
  long long z0 = 0;          // exact mode: sum_t dc (c' + c)
  double s0 = 0.0;           // approximate mode: sum_t d (e' + e)
  uint32_t absdc = 0;        // exact mode: sum_t |dc|

  f32x4 acc[NOY][G::NT];
#pragma unroll
  for (int oy = 0; oy < NOY; ++oy)
#pragma unroll
    for (int ct = 0; ct < G::NT; ++ct) acc[oy][ct] = f32x4{0.f, 0.f, 0.f, 0.f};

  const uint32_t t_begin = blockIdx.z * trlen, t_end = min(t_begin + trlen, v.tb);
  // Heaviside rows [t_begin, h_end) first, then Gaussian rows [g_begin,
  // t_end): a slice lies wholly in one kind (both counts are multiples of 16)
  const uint32_t h_end = min(t_end, v.tp), g_begin = max(t_begin, v.tp);
  const uint32_t nsh = h_end > t_begin ? (h_end - t_begin) / 16 : 0;
  const uint32_t nsg = t_end > g_begin ? (t_end - g_begin) / 16 : 0;
  uint4* aring = lds16 + G::NBUF * G::SLOT;   // [2][BYC][128] change-operand words

  // region loads of the slice at t0 into ring slot buf
  auto issue = [&](uint32_t t0, uint32_t buf) {
    const char* fs = (const char*)(v.bf + (size_t)(t0 >> 3) * P * 8);
#pragma unroll
    for (int it = 0; it < G::ITERD; ++it)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(fs + src[it]),
                                       (__attribute__((address_space(3))) void*)(lds16 + buf * G::SLOT +
                                                                                 it * G::NTH + 64 * w),
                                       16, 0, 0);
  };
  // change-operand words of the wave's 16 class pixels for the Heaviside
  // slice at t0 into its slot: words 0..63 the new (lanes 0..31) and current
  // (32..63) count words of pixel lane % 16, tile half (lane / 16) % 2;
  // approximate mode: words 64..67 the slice's 16 exact integrals (four
  // lanes' worth, repeated by the others)
  // (the lane's pixel is its own class pixel; lanes without one read row 0)
  const uint32_t ah = (lane >> 4) & 1;
  auto issue_a = [&](uint32_t t0, uint32_t buf) {
    uint4* dst = aring + (buf * BYC + w) * 128;
    const uint16_t* s = lane < 32 ? v.c_new + tix(own_j, t0 + 8 * ah, v.pc) : v.cnt + tix(own_p, t0 + 8 * ah, P);
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)s,
                                     (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    if (approx)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(v.area + t0 + 4 * (lane & 3)),
                                       (__attribute__((address_space(3))) void*)(dst + 64), 16, 0, 0);
  };
  // the lane's change operand (BF16) of a Heaviside slice and its part of
  // the self term, from the wave's change-operand words
  auto operand_h = [&](const uint4* aw) -> bf16x4 {
    float f[4] = {0.f, 0.f, 0.f, 0.f};
    if (own_ok) {
      const u32x2 cn = ((const u32x2*)aw)[2 * ((quarter >> 1) * 16 + m) + (quarter & 1)];
      const u32x2 co = ((const u32x2*)aw)[2 * (32 + (quarter >> 1) * 16 + m) + (quarter & 1)];
      const uint32_t nw[2] = {cn.x, cn.y}, ow[2] = {co.x, co.y};
      const float inv_n = 1.0f / (float)v.n;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int n = (int)((nw[i >> 1] >> (16 * (i & 1))) & 0xFFFFu);
        const int c = (int)((ow[i >> 1] >> (16 * (i & 1))) & 0xFFFFu);
        const int d = n - c;
        if (!approx) {
          z0 += (long long)(d * (n + c));
          absdc += (uint32_t)abs(d);
          f[i] = (float)d;
        } else {
          const double ar = (double)((const float*)(aw + 64))[4 * quarter + i];
          f[i] = __fmul_rn((float)d, inv_n);
          s0 = __dadd_rn(s0, __dmul_rn((double)f[i], (double)(n + c) / (double)v.n - 2.0 * ar));
        }
      }
    }
    return __builtin_bit_cast(bf16x4, make_uint2(bf16x2_bits(f[0], f[1]), bf16x2_bits(f[2], f[3])));
  };
  auto mfma_slice = [&](uint32_t buf, const bf16x4 af) {
    const u32x2* fb = (const u32x2*)(lds16 + buf * G::SLOT);
#pragma unroll
    for (int oy = 0; oy < NOY; ++oy) {
      const uint32_t rr = K * w + oy;
#pragma unroll
      for (int ct = 0; ct < G::NT; ++ct) {
        const u32x2 b2 = fb[2 * ((quarter >> 1) * G::PLANE_PAD + rr * G::RUSED + ct * 16 + m) + (quarter & 1)];
        acc[oy][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, __builtin_bit_cast(bf16x4, b2), acc[oy][ct],
                                                                0, 0, 0);
      }
    }
  };

  // Heaviside slices: region words PD slices ahead, change-operand words one
  // slice ahead, all through LDS, so that no register waits on a load.  Each
  // step issues one slice of region loads (past the range a repeat of the
  // first slice, into the slot that is never read again), after that step's
  // change-operand loads: the loads issued after slice si's are then always
  // the region loads of the PD - 1 slices that follow it.
  if (nsh > 0) {
    issue_a(t_begin, 0);
#pragma unroll
    for (int k = 0; k < G::PD; ++k) issue((uint32_t)k < nsh ? t_begin + 16 * k : t_begin, k);
  }
  for (uint32_t si = 0; si < nsh; ++si) {
    const uint32_t t0 = t_begin + 16 * si;
    barrier_vm<(G::PD - 1) * G::ITERD>();
    const bf16x4 af = operand_h(aring + ((si & 1) * BYC + w) * 128);
    // the slots refilled here were last read by every wave before the barrier
    issue_a(si + 1 < nsh ? t0 + 16 : t_begin, (si + 1) & 1);
    issue(si + G::PD < nsh ? t0 + 16 * G::PD : t_begin, (si + G::PD) % G::NBUF);
    mfma_slice(si % G::NBUF, af);
  }
  __syncthreads();

  // Gaussian slices (approximate mode only): one slice at a time through
  // ring slot 0, the change operands from the estimates in registers
  for (uint32_t si = 0; si < nsg; ++si) {
    const uint32_t t0 = g_begin + 16 * si;
    issue(t0, 0);
    const uint32_t tg = t0 + 4 * quarter - v.tp;
    float4 gn4 = make_float4(0.f, 0.f, 0.f, 0.f), go4 = gn4;
    double gi[4] = {0.0, 0.0, 0.0, 0.0};
    if (own_ok) {
      gn4 = *(const float4*)(v.g_new + (size_t)own_j * v.tgp + tg);
      go4 = *(const float4*)(v.gest + (size_t)own_p * v.tgp + tg);
#pragma unroll
      for (int i = 0; i < 4; ++i) gi[i] = v.gint[tg + i];
    }
    const float gn[4] = {gn4.x, gn4.y, gn4.z, gn4.w}, go[4] = {go4.x, go4.y, go4.z, go4.w};
    float f[4] = {0.f, 0.f, 0.f, 0.f};
    if (own_ok) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (tg + i < v.tg) {
          f[i] = __fsub_rn(gn[i], go[i]);
          s0 = __dadd_rn(s0, __dmul_rn((double)f[i], (double)gn[i] + (double)go[i] - 2.0 * gi[i]));
        }
      }
    }
    const bf16x4 af = __builtin_bit_cast(bf16x4, make_uint2(bf16x2_bits(f[0], f[1]), bf16x2_bits(f[2], f[3])));
    barrier_vm<0>();
    mfma_slice(0, af);
    __syncthreads();
  }

  // self terms and certificates: the four quarters of a class pixel meet in
  // lane m
  z0 += __shfl_xor(z0, 16);
  z0 += __shfl_xor(z0, 32);
  absdc += __shfl_xor(absdc, 16);
  absdc += __shfl_xor(absdc, 32);
  s0 = __dadd_rn(s0, __shfl_xor(s0, 16));
  s0 = __dadd_rn(s0, __shfl_xor(s0, 32));

  // window entries: per neighbour row, the wave's tiles go through LDS and
  // lanes 0..15 (one per class pixel) collect their 2R+1 columns
  float* gsh = (float*)lds16 + w * (16 * G::RCOLS);   // [16][RCOLS] per wave
  const uint32_t b = lane;
  double zd[NCLS];   // exact mode: sums of exact integers below 2^24 each
#pragma unroll
  for (int c = 0; c < NCLS; ++c) zd[c] = 0.0;
#pragma unroll
  for (int oy = 0; oy < NOY; ++oy) {
#pragma unroll
    for (int ct = 0; ct < G::NT; ++ct)
#pragma unroll
      for (int i = 0; i < 4; ++i) gsh[(4 * (lane >> 4) + i) * G::RCOLS + ct * 16 + (lane & 15)] = acc[oy][ct][i];
    // only this wave touches its gsh: order its lanes' stores before the
    // cross-lane reads (wavefront-scope release/acquire around a wave barrier)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < 16) {
      const int wy = OY0 + oy - R;
#pragma unroll
      for (int ox = -R; ox <= R; ++ox) {
        if (ox == 0 && wy == 0) continue;
        const int cidx = W.cmap[(wy + R) * (2 * R + 1) + ox + R];
        zd[cidx] += (double)gsh[b * G::RCOLS + K * b + R + ox];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const uint32_t a = a0 + w, bb = b0 + b;
  if (lane < 16 && a < v.ch && bb < v.cw) {
    const uint32_t j = a * v.cw + bb;
    const double self = OY0 == 0 ? (approx ? s0 : (double)z0) : 0.0;
    if (!approx && (unsigned long long)absdc * v.n >= (1ull << 24)) atomicOr(&unsure[j], 1u);
#pragma unroll
    for (int c = 0; c < NCLS; ++c) {
      long long x;
      if (approx) {
        x = (long long)rint(0x1p40 * __dsub_rn(__dmul_rn((double)W.csize[c], self), 2.0 * zd[c]));
      } else {
        x = (long long)W.csize[c] * (long long)self - 2 * (long long)zd[c];
      }
      atomicAdd((unsigned long long*)&xsum[(size_t)c * v.pc + j], (unsigned long long)x);
    }
  }
}

// Exact mode: re-check of the accepted moves whose slices could not certify
// exactness, with the integer class sums (a move the exact value rejects is a
// veto).  A wave screens 64 consecutive class pixels, clearing their flags,
// and re-checks its flagged accepted ones one after another: flagged pixels
// are rare, and one wave per pixel spent most of the kernel's time launching
// and retiring waves with nothing to do.
template <int R>
__global__ __launch_bounds__(256) void k_delta_refine(DevView v, uint32_t kappa, uint32_t* __restrict__ unsure) {
  __builtin_amdgcn_s_setprio(2);
  constexpr Window<R> W = WinConst<R>::w;
  constexpr int NCLS = WinConst<R>::NCLS;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t j0 = wave_id() * 64;
  bool flag = false;
  if (j0 + lane < v.pc) {
    flag = v.accept[j0 + lane] != 0 && unsure[j0 + lane] != 0;
    unsure[j0 + lane] = 0;
  }
  for (uint64_t todo = __ballot(flag); todo != 0; todo &= todo - 1) {
    const uint32_t j = j0 + (uint32_t)__builtin_ctzll(todo);
    const uint32_t p = class_pixel(v, kappa, j);
    const uint32_t y = p / v.w, x = p - y * v.w, P = v.w * v.h;
    long long z0 = 0, zd[NCLS];
#pragma unroll
    for (int c = 0; c < NCLS; ++c) zd[c] = 0;
    for (uint32_t base = 0; base < v.tp; base += 128) {
      const uint32_t t = base + 2 * lane;
      const uint32_t cn = *(const uint32_t*)(v.c_new + tix(j, t, v.pc));
      const uint32_t co = *(const uint32_t*)(v.cnt + tix(p, t, P));
      const int n0 = (int)(cn & 0xFFFFu), n1 = (int)(cn >> 16);
      const int o0 = (int)(co & 0xFFFFu), o1 = (int)(co >> 16);
      const int dc0 = n0 - o0, dc1 = n1 - o1;
      const uint32_t dcp = ((uint32_t)dc0 & 0xFFFFu) | ((uint32_t)dc1 << 16);
      z0 += (long long)(dc0 * (n0 + o0) + dc1 * (n1 + o1));
#pragma unroll
      for (int mm = 0; mm < W.M; ++mm) {
        const uint32_t q = ((y + v.h + W.oy[mm]) % v.h) * v.w + (x + v.w + W.ox[mm]) % v.w;
        zd[W.cls[mm]] += dot2(dcp, *(const uint32_t*)(v.cnt + tix(q, t, P)), 0);
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
    double total = __dmul_rn(acc, 2.0 / ((double)v.n * (double)v.n));
    if (v.tgp) {
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
      double ga = 0.0;
#pragma unroll
      for (int c = 0; c < NCLS; ++c) {
        double xv = cs[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) xv += __shfl_xor(xv, off);
        ga += v.wd[c] * xv;
      }
      total = __dadd_rn(total, 2.0 * ga);
    }
    if (lane == 0) {
      const bool ok = (v.objective > 0) ? (total < 0.0) : (total > 0.0);
      v.delta[j] = total;
      if (!ok) {
        v.accept[j] = 0;
        atomicAdd(&v.ctr[2], 1ull);
      }
    }
  }
}

// Approximate mode: every move the BF16 value accepted is re-evaluated with
// the FP32 form's arithmetic (its staged stencils have just summed the exact
// integer class sums into xsum and the Gaussian rows' part into gdelta, for
// every class pixel of the phase: staging the window costs the same for one
// pixel of a block as for all of them).  The exact value is combined in the
// FP32 form's order; a move it rejects is a veto.  Clears xsum.
__global__ __launch_bounds__(256) void k_refine_combine(DevView v, long long* __restrict__ xsum) {
  __builtin_amdgcn_s_setprio(2);
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= v.pc) return;
  double acc = 0.0;
  for (uint32_t c = 0; c < v.ncls; ++c) {
    const long long x = xsum[(size_t)c * v.pc + j];
    xsum[(size_t)c * v.pc + j] = 0;
    acc = __dadd_rn(acc, __dmul_rn(v.wd[c], (double)x));
  }
  if (!v.accept[j]) return;
  double total = __dmul_rn(acc, 2.0 / ((double)v.n * (double)v.n));
  if (v.tgp) total = __dadd_rn(total, v.gdelta[j]);
  v.delta[j] = total;
  if (!((v.objective > 0) ? (total < 0.0) : (total > 0.0))) {
    v.accept[j] = 0;
    atomicAdd(&v.ctr[2], 1ull);
  }
}

// BF16 energy of Eq. (1): the half window's sums of |f_p - f_q|^2 over the
// field, per distance class (FP32 per 8-integrand tile, FP64 across tiles,
// FP64 atomics); the host doubles them and scales them by 1/N^2 in the exact
// mode (the field then holds counts).
template <int R>
__global__ __launch_bounds__(256) void k_energy_bf(DevView v, double* __restrict__ ysum) {
  constexpr Window<R> W = WinConst<R>::w;
  constexpr int NCLS = WinConst<R>::NCLS;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t P = v.w * v.h;
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  double yd[NCLS];
#pragma unroll
  for (int c = 0; c < NCLS; ++c) yd[c] = 0.0;
  if (p < P) {
    const uint32_t y = p / v.w, x = p - y * v.w;
    for (uint32_t tt = 0; tt < (v.tb >> 3); ++tt) {
      const uint4 fp = *(const uint4*)(v.bf + ((size_t)tt * P + p) * 8);
      const uint32_t pw[4] = {fp.x, fp.y, fp.z, fp.w};
      float part[NCLS];
#pragma unroll
      for (int c = 0; c < NCLS; ++c) part[c] = 0.0f;
#pragma unroll
      for (int mm = 0; mm < W.M; ++mm) {
        if (!(W.oy[mm] > 0 || (W.oy[mm] == 0 && W.ox[mm] > 0))) continue;
        const uint32_t q = ((y + v.h + W.oy[mm]) % v.h) * v.w + (x + v.w + W.ox[mm]) % v.w;
        const uint4 fq = *(const uint4*)(v.bf + ((size_t)tt * P + q) * 8);
        const uint32_t qw[4] = {fq.x, fq.y, fq.z, fq.w};
        float a = part[W.cls[mm]];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float d0 = __uint_as_float(pw[k] << 16) - __uint_as_float(qw[k] << 16);
          const float d1 = __uint_as_float(pw[k] & 0xFFFF0000u) - __uint_as_float(qw[k] & 0xFFFF0000u);
          a = __fadd_rn(a, __fmul_rn(d0, d0));
          a = __fadd_rn(a, __fmul_rn(d1, d1));
        }
        part[W.cls[mm]] = a;
      }
#pragma unroll
      for (int c = 0; c < NCLS; ++c) yd[c] += (double)part[c];
    }
  }
#pragma unroll
  for (int c = 0; c < NCLS; ++c) {
    double s = yd[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0 && s != 0.0) atomicAdd(&ysum[c], s);
  }
}

// Integrand slices of a launch: about slice_target workgroups, each slice a
// whole number of 16-integrand stages.
inline uint32_t bf_slices(const DevView& v, uint32_t blocks, uint32_t* trlen) {
  const uint32_t chunks = v.tb / 16;
  const uint32_t target = v.slice_target ? v.slice_target : 512;
  uint32_t want = (target + blocks - 1) / blocks;
  if (want > chunks) want = chunks;
  if (want < 1) want = 1;
  const uint32_t per = (chunks + want - 1) / want;
  *trlen = per * 16;
  return (chunks + per - 1) / per;
}

constexpr int BF_BYC = 4;   // class rows (waves) per workgroup
constexpr int BF_MAX_TILES = 40;

template <int R, int K, int OY0, int NOY>
hipError_t bf_pass(const DevView& v, uint32_t kappa, hipStream_t s) {
  using G = BfGeom<R, K, BF_BYC, OY0, NOY>;
  static_assert(G::LDS_BYTES <= 163840, "BF16 block exceeds the 160 KiB of LDS of a CU");
  const uint32_t bx = (v.cw + G::BXC - 1) / G::BXC, by = (v.ch + BF_BYC - 1) / BF_BYC;
  uint32_t trlen = 0;
  const uint32_t ns = bf_slices(v, bx * by, &trlen);
  hipLaunchKernelGGL((k_delta_bf<R, K, BF_BYC, OY0, NOY>), dim3(bx, by, ns), dim3(64 * BF_BYC),
                     (size_t)G::LDS_BYTES, s, v, kappa, trlen, v.xpart, v.unsure);
  return hipGetLastError();
}

// Window rows [OY0, 2R] in passes of at most BF_MAX_TILES accumulator tiles.
template <int R, int K, int OY0>
hipError_t bf_passes(const DevView& v, uint32_t kappa, hipStream_t s) {
  if constexpr (OY0 > 2 * R) {
    return hipSuccess;
  } else {
    constexpr int NT = BfGeom<R, K, BF_BYC, 0, 1>::NT;
    constexpr int LEFT = 2 * R + 1 - OY0;
    constexpr int FIT = BF_MAX_TILES / NT;
    constexpr int NOY = LEFT < FIT ? LEFT : FIT;
    hipError_t e = bf_pass<R, K, OY0, NOY>(v, kappa, s);
    if (e != hipSuccess) return e;
    return bf_passes<R, K, OY0 + NOY>(v, kappa, s);
  }
}

// Launch limit of the passes' kernels raised to their LDS use where it is
// above 64 KiB (gfx950 has 160 KiB per CU).
template <int R, int K, int OY0>
hipError_t bf_prepare_passes() {
  if constexpr (OY0 > 2 * R) {
    return hipSuccess;
  } else {
    constexpr int NT = BfGeom<R, K, BF_BYC, 0, 1>::NT;
    constexpr int LEFT = 2 * R + 1 - OY0;
    constexpr int FIT = BF_MAX_TILES / NT;
    constexpr int NOY = LEFT < FIT ? LEFT : FIT;
    using G = BfGeom<R, K, BF_BYC, OY0, NOY>;
    if constexpr (G::LDS_BYTES > 65536) {
      const hipError_t e = hipFuncSetAttribute((const void*)k_delta_bf<R, K, BF_BYC, OY0, NOY>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)G::LDS_BYTES);
      if (e != hipSuccess) return e;
    }
    return bf_prepare_passes<R, K, OY0 + NOY>();
  }
}

template <int R>
hipError_t bf_prepare(uint32_t k) {
  switch (k) {
    case 1: return bf_prepare_passes<R, 1, 0>();
    case 2: return bf_prepare_passes<R, 2, 0>();
    case 4: return bf_prepare_passes<R, 4, 0>();
    default: return hipErrorInvalidValue;
  }
}

template <int R>
hipError_t bf_launch(const DevView& v, uint32_t kappa, hipStream_t s) {
  hipError_t e;
  switch (v.k) {
    case 1: e = bf_passes<R, 1, 0>(v, kappa, s); break;
    case 2: e = bf_passes<R, 2, 0>(v, kappa, s); break;
    case 4: e = bf_passes<R, 4, 0>(v, kappa, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  e = launch_finish(v, s);
  if (e != hipSuccess) return e;
  if (v.mfma == 1) {
    hipLaunchKernelGGL((k_delta_refine<R>), dim3((v.pc + 255) / 256), dim3(256), 0, s, v, kappa, v.unsure);
    return hipGetLastError();
  }
  if ((e = launch_stage_exact(v, kappa, s)) != hipSuccess) return e;
  if ((e = launch_gauss_delta_exact(v, kappa, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_refine_combine, dim3((v.pc + 255) / 256), dim3(256), 0, s, v, v.xpart);
  return hipGetLastError();
}

}  // namespace

bool bf16_supported_k(uint32_t k) { return k == 1 || k == 2 || k == 4; }

hipError_t launch_bf_field(const DevView& v, hipStream_t s) {
  if (!v.bf) return hipSuccess;
  const size_t n = (size_t)v.w * v.h * (v.tb >> 3);
  hipLaunchKernelGGL(k_bf_field, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v);
  return hipGetLastError();
}

hipError_t prepare_bf_kernels(uint32_t radius, uint32_t k) {
  switch (radius) {
    case 1: return bf_prepare<1>(k);
    case 2: return bf_prepare<2>(k);
    case 3: return bf_prepare<3>(k);
    case 4: return bf_prepare<4>(k);
    case 5: return bf_prepare<5>(k);
    case 6: return bf_prepare<6>(k);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_delta_bf16(const DevView& v, uint32_t kappa, hipStream_t s) {
  switch (v.radius) {
    case 1: return bf_launch<1>(v, kappa, s);
    case 2: return bf_launch<2>(v, kappa, s);
    case 3: return bf_launch<3>(v, kappa, s);
    case 4: return bf_launch<4>(v, kappa, s);
    case 5: return bf_launch<5>(v, kappa, s);
    case 6: return bf_launch<6>(v, kappa, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_energy_bf16(const DevView& v, double* ysum, hipStream_t s) {
  const uint32_t P = v.w * v.h;
  const dim3 grid((P + 255) / 256), block(256);
  switch (v.radius) {
    case 1: hipLaunchKernelGGL(k_energy_bf<1>, grid, block, 0, s, v, ysum); break;
    case 2: hipLaunchKernelGGL(k_energy_bf<2>, grid, block, 0, s, v, ysum); break;
    case 3: hipLaunchKernelGGL(k_energy_bf<3>, grid, block, 0, s, v, ysum); break;
    case 4: hipLaunchKernelGGL(k_energy_bf<4>, grid, block, 0, s, v, ysum); break;
    case 5: hipLaunchKernelGGL(k_energy_bf<5>, grid, block, 0, s, v, ysum); break;
    case 6: hipLaunchKernelGGL(k_energy_bf<6>, grid, block, 0, s, v, ysum); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace bnlat
