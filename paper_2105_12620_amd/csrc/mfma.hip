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
// the 16 rows of its MFMA tiles.  Per 16-integrand slice the field values of
// the window region (RROWS x RUSED pixels) are copied into LDS as they are
// (already BF16), in four quarter planes of 4 integrands (8 bytes per pixel);
// the class pixels' change operands go beside them.  For every neighbour row
// oy of the pass and column tile ct, v_mfma_f32_16x16x16_bf16 accumulates
//     C[b][col] += sum_t d[b][t] * f[row][col][t]
// and pixel b's window entries are the columns K b + R + ox.  Window rows are
// split into passes when their accumulators would exceed 40 tiles (160
// registers); the self term is added by pass 0 only.
template <int R, int K, int BYC, int OY0, int NOY>
struct BfGeom {
  static constexpr int BXC = 16;
  static constexpr int RROWS = K * (BYC - 1) + NOY;
  static constexpr int RUSED = K * (BXC - 1) + 2 * R + 1;
  static constexpr int NT = (RUSED + 15) / 16;
  static constexpr int RCOLS = 16 * NT;
  static constexpr int NB = BYC * BXC;
  static constexpr int REG8 = 4 * RROWS * RCOLS;   // region, 8-byte words
  static constexpr int DC8 = 4 * NB;               // change operands, 8-byte words
  static constexpr int STAGE_BYTES = 8 * (REG8 + DC8);
  static constexpr int EXTRACT_BYTES = 16 * NB + BYC * 16 * RCOLS * 4;
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
  constexpr int NT = 64 * BYC;
  constexpr int NITEM = 2 * G::RROWS * G::RUSED;
  constexpr int ITER = (NITEM + NT - 1) / NT;
  extern __shared__ uint2 lds8[];
  uint2* reg = lds8;                 // [4][RROWS][RCOLS]
  uint2* dcs = lds8 + G::REG8;       // [4][NB]
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t a0 = blockIdx.y * BYC, b0 = blockIdx.x * G::BXC;
  const uint32_t ky = kappa / K, kx = kappa - ky * K;
  const uint32_t ys = (ky + K * a0 + v.h * (R / v.h + 1) - R + OY0) % v.h;
  const uint32_t xs = (kx + K * b0 + v.w * (R / v.w + 1) - R) % v.w;
  const uint32_t P = v.w * v.h;
  const bool approx = v.mfma == 2;

  // columns past the used ones are never read back; keep them finite
  for (uint32_t i = threadIdx.x; i < (uint32_t)(4 * G::RROWS * (G::RCOLS - G::RUSED)); i += blockDim.x) {
    const uint32_t q = i / (G::RCOLS - G::RUSED), c = G::RUSED + i % (G::RCOLS - G::RUSED);
    reg[q * G::RCOLS + c] = make_uint2(0, 0);
  }

  // change-operand roles: thread i < 2 NB owns (class pixel i >> 1, tile i & 1 of the slice)
  const uint32_t own_cp = threadIdx.x >> 1, own_half = threadIdx.x & 1;
  const uint32_t own_a = a0 + own_cp / G::BXC, own_b = b0 + own_cp % G::BXC;
  const bool own_ok = threadIdx.x < 2u * G::NB && own_a < v.ch && own_b < v.cw;
  const uint32_t own_p = own_ok ? (ky + K * own_a) * v.w + (kx + K * own_b) : 0;
  const uint32_t own_j = own_ok ? own_a * v.cw + own_b : 0;
  long long z0 = 0;          // exact mode: sum_t dc (c' + c)
  double s0 = 0.0;           // approximate mode: sum_t d (e' + e)
  uint32_t absdc = 0;        // exact mode: sum_t |dc|

  // staging plan: item i = (tile half, region pixel), fixed for the whole range
  uint32_t item_pix[ITER], item_lds[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const uint32_t i = threadIdx.x + it * NT;
    item_pix[it] = 0xFFFFFFFFu;
    item_lds[it] = 0;
    if (i < (uint32_t)NITEM) {
      const uint32_t half = i / (G::RROWS * G::RUSED), pix = i - half * (G::RROWS * G::RUSED);
      const uint32_t rr = pix / G::RUSED, cc = pix - rr * G::RUSED;
      uint32_t gy = ys + rr, gx = xs + cc;
      while (gy >= v.h) gy -= v.h;
      while (gx >= v.w) gx -= v.w;
      item_pix[it] = (gy * v.w + gx) | (half << 31);
      item_lds[it] = ((2 * half) * G::RROWS + rr) * G::RCOLS + cc;
    }
  }

  f32x4 acc[NOY][G::NT];
#pragma unroll
  for (int oy = 0; oy < NOY; ++oy)
#pragma unroll
    for (int ct = 0; ct < G::NT; ++ct) acc[oy][ct] = f32x4{0.f, 0.f, 0.f, 0.f};

  const uint32_t t_begin = blockIdx.z * trlen, t_end = min(t_begin + trlen, v.tb);
  uint4 q[ITER];
  auto load_region = [&](uint32_t t0) {
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      if (item_pix[it] != 0xFFFFFFFFu) {
        const uint32_t half = item_pix[it] >> 31, pix = item_pix[it] & 0x7FFFFFFFu;
        q[it] = *(const uint4*)(v.bf + tix(pix, t0 + 8 * half, P));
      }
    }
  };
  if (t_begin < t_end) load_region(t_begin);
  for (uint32_t t0 = t_begin; t0 < t_end; t0 += 16) {
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      if (item_pix[it] != 0xFFFFFFFFu) {
        reg[item_lds[it]] = make_uint2(q[it].x, q[it].y);
        reg[item_lds[it] + G::RROWS * G::RCOLS] = make_uint2(q[it].z, q[it].w);
      }
    }
    // change operands of the moved pixels (and their self terms)
    if (threadIdx.x < 2u * G::NB) {
      uint32_t o[4] = {0u, 0u, 0u, 0u};
      if (own_ok) {
        const uint32_t t = t0 + 8 * own_half;
        if (t < v.tp) {
          const uint4 cn4 = *(const uint4*)(v.c_new + tix(own_j, t, v.pc));
          const uint4 co4 = *(const uint4*)(v.cnt + tix(own_p, t, P));
          const uint32_t nw[4] = {cn4.x, cn4.y, cn4.z, cn4.w}, ow[4] = {co4.x, co4.y, co4.z, co4.w};
          const float inv_n = 1.0f / (float)v.n;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int n0 = (int)(nw[k] & 0xFFFFu), n1 = (int)(nw[k] >> 16);
            const int c0 = (int)(ow[k] & 0xFFFFu), c1 = (int)(ow[k] >> 16);
            const int d0 = n0 - c0, d1 = n1 - c1;
            if (!approx) {
              z0 += (long long)(d0 * (n0 + c0) + d1 * (n1 + c1));
              absdc += (uint32_t)(abs(d0) + abs(d1));
              o[k] = bf16x2_bits((float)d0, (float)d1);
            } else {
              const float f0 = __fmul_rn((float)d0, inv_n), f1 = __fmul_rn((float)d1, inv_n);
              const double a0d = v.area[t + 2 * k], a1d = v.area[t + 2 * k + 1];
              s0 = __dadd_rn(s0, __dmul_rn((double)f0, (double)(n0 + c0) / (double)v.n - 2.0 * a0d));
              s0 = __dadd_rn(s0, __dmul_rn((double)f1, (double)(n1 + c1) / (double)v.n - 2.0 * a1d));
              o[k] = bf16x2_bits(f0, f1);
            }
          }
        } else {
          const uint32_t tg = t - v.tp;
          const float* gn = v.g_new + (size_t)own_j * v.tgp + tg;
          const float* go = v.gest + (size_t)own_p * v.tgp + tg;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            float f[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
              const uint32_t i = 2 * k + e;
              f[e] = 0.0f;
              if (tg + i < v.tg) {
                f[e] = __fsub_rn(gn[i], go[i]);
                s0 = __dadd_rn(s0, __dmul_rn((double)f[e], (double)gn[i] + (double)go[i] - 2.0 * v.gint[tg + i]));
              }
            }
            o[k] = bf16x2_bits(f[0], f[1]);
          }
        }
      }
      dcs[(2 * own_half) * G::NB + own_cp] = make_uint2(o[0], o[1]);
      dcs[(2 * own_half + 1) * G::NB + own_cp] = make_uint2(o[2], o[3]);
    }
    __syncthreads();
    if (t0 + 16 < t_end) load_region(t0 + 16);
    // lane l: MFMA row (class pixel) l % 16, integrands 4 (l / 16) .. +3 of the slice
    const uint32_t quarter = lane >> 4, m = lane & 15;
    const bf16x4 af = __builtin_bit_cast(bf16x4, dcs[quarter * G::NB + w * G::BXC + m]);
#pragma unroll
    for (int oy = 0; oy < NOY; ++oy) {
      const uint32_t rr = K * w + oy;
#pragma unroll
      for (int ct = 0; ct < G::NT; ++ct) {
        const uint2 b2 = reg[(quarter * G::RROWS + rr) * G::RCOLS + ct * 16 + m];
        acc[oy][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, __builtin_bit_cast(bf16x4, b2), acc[oy][ct],
                                                                0, 0, 0);
      }
    }
    __syncthreads();
  }
  __syncthreads();

  // self terms and certificates: the two tile halves of a pixel meet in LDS
  double* zsh = (double*)lds8;                         // [NB] (exact mode: integer, exact in FP64)
  uint32_t* ash = (uint32_t*)(zsh + G::NB);            // [NB]
  if (threadIdx.x < 2u * G::NB && own_half == 0) {
    zsh[own_cp] = approx ? s0 : (double)z0;
    ash[own_cp] = absdc;
  }
  __syncthreads();
  if (threadIdx.x < 2u * G::NB && own_half == 1) {
    zsh[own_cp] = __dadd_rn(zsh[own_cp], approx ? s0 : (double)z0);
    ash[own_cp] += absdc;
  }
  __syncthreads();

  // window entries: per neighbour row, the wave's tiles go through LDS and
  // lanes 0..15 (one per class pixel) collect their 2R+1 columns
  float* gsh = (float*)(lds8 + 2 * G::NB) + w * (16 * G::RCOLS);   // [16][RCOLS] per wave
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
    const uint32_t cp = w * G::BXC + b;
    const uint32_t j = a * v.cw + bb;
    const double self = OY0 == 0 ? zsh[cp] : 0.0;
    if (!approx && (unsigned long long)ash[cp] * v.n >= (1ull << 24)) atomicOr(&unsure[j], 1u);
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
// exactness, with the integer class sums (one wave per flagged pixel; a move
// the exact value rejects is a veto).
template <int R>
__global__ __launch_bounds__(256) void k_delta_refine(DevView v, uint32_t kappa, uint32_t* __restrict__ unsure) {
  __builtin_amdgcn_s_setprio(2);
  constexpr Window<R> W = WinConst<R>::w;
  constexpr int NCLS = WinConst<R>::NCLS;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t j = wave_id();
  if (j >= v.pc) return;
  const bool todo = v.accept[j] != 0 && unsure[j] != 0;
  if (lane == 0) unsure[j] = 0;
  if (!todo) return;
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
  static_assert(G::LDS_BYTES <= 65536, "BF16 block exceeds 64 KiB of LDS");
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
    hipLaunchKernelGGL((k_delta_refine<R>), dim3((v.pc + 3) / 4), dim3(256), 0, s, v, kappa, v.unsure);
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
