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
// k_count: every lane holds NS samples of one work item (a pixel, or a
// proposal), and L = N / NS consecutive lanes share the item (NS = N up to 64,
// else 64).  A wave walks a chunk of integrands with wave-uniform parameters
// from scalar loads, two integrands at a time.  Per (sample, integrand) the
// only vector work is one v_dot2 with the threshold folded in (n.s > D'
// exactly when r = n.s - D' - 1 >= 0; |n.s|, |D'| <= 2^30, so r never
// overflows); per sample one v_perm_b32 turns the sign bits of the two
// integrands' residues into 0x00/0xFF bytes in the two 16-bit halves of a
// word, and per two such words one v_add3_u32 sums them.  A lane's halves then
// hold 255 x its misses of integrands i and i + 1 (at most 255 * 64, so no
// carry crosses the halves); they become miss counts, the L lanes of an item
// add them with DPP / lane shuffles, and N - misses is the item's pair of
// counts, already packed as the tile layout stores them.

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Sign bytes of a sample's residues for two integrands: byte 0 is 0xFF when
// lo < 0 and byte 2 is 0xFF when hi < 0 (v_perm_b32 selectors 9 and 11 repeat
// bit 31 of the second and of the first operand; selector 12 is a zero byte).
__device__ inline uint32_t sign_bytes(int lo, int hi) {
  return __builtin_amdgcn_perm((uint32_t)hi, (uint32_t)lo, 0x0C0B0C09u);
}

// Per 16-bit half, x = 255 m with 0 <= m <= 255 becomes m:
// floor(255 (m + 1) / 256) = m, so m = (x + 255) >> 8.
__device__ inline uint32_t halves_div255(uint32_t x) {
  const u16x2 h = __builtin_bit_cast(u16x2, x);
  return __builtin_bit_cast(uint32_t, (u16x2)((h + (u16x2){255, 255}) >> (u16x2){8, 8}));
}

// Sum of x over each aligned group of L consecutive lanes, in every lane of
// the group.
template <int L>
__device__ inline uint32_t lane_group_sum(uint32_t x) {
  if (L >= 2) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, true);  // quad_perm 1,0,3,2
  if (L >= 4) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, true);  // quad_perm 2,3,0,1
#pragma unroll
  for (int o = 4; o < L; o <<= 1) x += (uint32_t)__shfl_xor((int)x, o);
  return x;
}

template <int NS, int L, int MODE>
__device__ __forceinline__ void count_lanes_body(const DevView& v, const int2* __restrict__ ihp, uint32_t kappa,
                                                 uint32_t m, uint32_t tch, uint32_t blk) {
  constexpr uint32_t IPW = 64 / L;  // work items per wave
  constexpr uint32_t N = NS * L;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(blk * 4 + (threadIdx.x >> 6));
  const uint32_t nch = (v.tp + tch - 1) / tch;
  const uint32_t jg = wave / nch, ch = wave - jg * nch;
  if (jg * IPW >= m) return;
  const uint32_t slot = lane % L, j0 = jg * IPW + lane / L;
  // lanes past the last item repeat it (the group sums need whole lane
  // groups) and store nothing
  const bool live = j0 < m;
  const uint32_t j = live ? j0 : m - 1;
  uint32_t p, u, row, rows;
  uint16_t* buf;
  count_target<MODE>(v, kappa, j, m, p, u, buf, row, rows);
  if ((MODE == MODE_CLASS || MODE == MODE_SWEEP) && ch == 0 && slot == 0 && live) v.u_new[j] = u;
  uint32_t sp[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) sp[k] = centre(wrap_add(v.lat[slot * NS + k], u));
  const float inv_n = 1.0f / (float)N;
  const uint32_t t0 = ch * tch, t1 = min(t0 + tch, v.tp);
  const int4* ip = (const int4*)(ihp + t0);
#pragma unroll 1
  for (uint32_t t = t0; t < t1; t += 8, ip += 4) {
    // eight integrands' parameters in one scalar load
    const int4 q0 = ip[0], q1 = ip[1], q2 = ip[2], q3 = ip[3];
    const int nn[8] = {q0.x, q0.z, q1.x, q1.z, q2.x, q2.z, q3.x, q3.z};
    const int dd[8] = {q0.y, q0.w, q1.y, q1.w, q2.y, q2.w, q3.y, q3.w};
    uint32_t c[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t n0 = (uint32_t)nn[2 * i], n1 = (uint32_t)nn[2 * i + 1];
      const int thr0 = -dd[2 * i] - 1, thr1 = -dd[2 * i + 1] - 1;
      uint32_t a = 0;
      // four samples' residues first, then their sign words: a v_perm then
      // reads a v_dot2 result several instructions after it
      constexpr int G = NS < 4 ? NS : 4;
#pragma unroll
      for (int k = 0; k < NS; k += G) {
        int r0[4], r1[4];
        uint32_t w[4];
#pragma unroll
        for (int e = 0; e < G; ++e) r0[e] = dot2(n0, sp[k + e], thr0), r1[e] = dot2(n1, sp[k + e], thr1);
#pragma unroll
        for (int e = 0; e < G; ++e) w[e] = sign_bytes(r0[e], r1[e]);
        if (G == 4) a = a + w[0] + w[1], a = a + w[2] + w[3];
        else if (G == 2) a = a + w[0] + w[1];
        else a += w[0];
      }
      // misses per half: at most 64 per lane, N per item (no carry)
      c[i] = (N | (N << 16)) - lane_group_sum<L>(halves_div255(a));
    }
    // computed in every lane (an empty asm consumes them): otherwise, with
    // one lane per item, the counting would move under the store's branch
    asm volatile("" : : "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    if (slot == 0 && live) {
      *(uint4*)(buf + tix(row, t, rows)) = make_uint4(c[0], c[1], c[2], c[3]);
      if (MODE == MODE_ALL) {
        float* e = v.err + (size_t)p * v.tp + t;
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = (float)((c[i >> 1] >> (16 * (i & 1))) & 0xFFFFu) * inv_n - v.area[t + i];
      }
    }
  }
}

// The launch may have fewer workgroups than the vblocks its work needs (the
// sweep-wide recount of the overlapped schedule is capped so that it leaves
// room on every CU for the colour phases running beside it): workgroups then
// stride over the virtual blocks.
//
// Occupancy target four waves per SIMD: aiming higher, the compiler fed each
// v_perm from the v_dot2 just before it and padded the pair with s_nop (about
// 250 per eight integrands at N = 64).
template <int NS, int L, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_count(
    DevView v, const int2* __restrict__ ihp, uint32_t kappa, uint32_t m, uint32_t tch, uint32_t vblocks) {
  for (uint32_t b = blockIdx.x; b < vblocks; b += gridDim.x) count_lanes_body<NS, L, MODE>(v, ihp, kappa, m, tch, b);
}

// Batched form: member i owns blocks pre[i] .. pre[i+1]-1.  MODE_CLASS counts
// the proposals of colour class kappa; MODE_SWEEP those of every pixel of the
// sweep kappa steps ahead of the member's sweep counter (the overlapped
// schedule's sweep-wide recount).
template <int NS, int L, int MODE>
__global__ __launch_bounds__(256) void k_count_batch(const DevView* __restrict__ views,
                                                     const uint32_t* __restrict__ pre, uint32_t nmem,
                                                     uint32_t kappa) {
  const uint32_t i = batch_member(pre, nmem, blockIdx.x);
  const DevView v = views[i];
  const uint32_t m = MODE == MODE_SWEEP ? v.w * v.h : v.pc;
  count_lanes_body<NS, L, MODE>(v, v.ihp, kappa, m, L == 1 ? 64u : v.tch, blockIdx.x - pre[i]);
}

// Lanes per work item (N / 64 above N = 64) and the integrand chunk of a wave:
// 64 integrands up to N = 64, else v.tch (whole rows at T <= 1024 by
// default), halved while a launch over m items would hold under 8192 waves.
inline uint32_t count_lanes(uint32_t n) { return n <= 64 ? 1u : n / 64; }

inline uint32_t count_chunk(const DevView& v, uint32_t m, uint32_t tch) {
  if (v.n <= 64) return 64;
  const uint64_t groups = (m + 64 / count_lanes(v.n) - 1) / (64 / count_lanes(v.n));
  while (tch > 64 && groups * ((v.tp + tch - 1) / tch) < 8192) tch >>= 1;
  return tch;
}

inline uint64_t count_waves(const DevView& v, uint32_t m, uint32_t tch) {
  const uint32_t ipw = 64 / count_lanes(v.n);
  return (uint64_t)((m + ipw - 1) / ipw) * ((v.tp + tch - 1) / tch);
}

template <int MODE>
hipError_t count_dispatch(const DevView& v, uint32_t kappa, uint32_t m, hipStream_t s) {
  if (m == 0) return hipSuccess;
  const uint32_t tch = count_chunk(v, m, v.tch);
  const uint32_t vb = (uint32_t)((count_waves(v, m, tch) + 3) / 4);
  // a capped launch gets the fewest rounds the cap allows and as few
  // workgroups as those rounds need, so that every workgroup strides over the
  // same number of blocks
  uint32_t nb = vb;
  if (MODE == MODE_SWEEP && v.count_cap && vb > v.count_cap) {
    const uint32_t rounds = (vb + v.count_cap - 1) / v.count_cap;
    nb = (vb + rounds - 1) / rounds;
  }
  const dim3 g(nb), b(256);
#define BN_COUNT(NS, L) hipLaunchKernelGGL((k_count<NS, L, MODE>), g, b, 0, s, v, v.ihp, kappa, m, tch, vb); break
  switch (v.n) {
    case 1: BN_COUNT(1, 1);
    case 2: BN_COUNT(2, 1);
    case 4: BN_COUNT(4, 1);
    case 8: BN_COUNT(8, 1);
    case 16: BN_COUNT(16, 1);
    case 32: BN_COUNT(32, 1);
    case 64: BN_COUNT(64, 1);
    case 128: BN_COUNT(64, 2);
    case 256: BN_COUNT(64, 4);
    case 512: BN_COUNT(64, 8);
    case 1024: BN_COUNT(64, 16);
    case 2048: BN_COUNT(64, 32);
    case 4096: BN_COUNT(64, 64);
    default: return hipErrorInvalidValue;
  }
#undef BN_COUNT
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

// Launch kind of a batch member's recount: N itself up to 64, else 64 + the
// lanes per work item (one kernel per N either way).
int count_kind(const DevView& v) { return v.n <= 64 ? (int)v.n : 64 + (int)count_lanes(v.n); }

uint32_t count_blocks(const DevView& v, bool sweep) {
  return (uint32_t)((count_waves(v, sweep ? v.w * v.h : v.pc, v.n <= 64 ? 64u : v.tch) + 3) / 4);
}

template <int MODE>
hipError_t count_batch_dispatch(int kind, const DevView* views, const uint32_t* pre, uint32_t nmem,
                                uint32_t blocks, uint32_t kappa, hipStream_t s) {
  const dim3 g(blocks), b(256);
#define BN_COUNT(NS, L) \
  hipLaunchKernelGGL((k_count_batch<NS, L, MODE>), g, b, 0, s, views, pre, nmem, kappa); break
  switch (kind) {
    case 1: BN_COUNT(1, 1);
    case 2: BN_COUNT(2, 1);
    case 4: BN_COUNT(4, 1);
    case 8: BN_COUNT(8, 1);
    case 16: BN_COUNT(16, 1);
    case 32: BN_COUNT(32, 1);
    case 64: BN_COUNT(64, 1);
    case 66: BN_COUNT(64, 2);
    case 68: BN_COUNT(64, 4);
    case 72: BN_COUNT(64, 8);
    case 80: BN_COUNT(64, 16);
    case 96: BN_COUNT(64, 32);
    case 128: BN_COUNT(64, 64);
    default: return hipErrorInvalidValue;
  }
#undef BN_COUNT
  return hipGetLastError();
}

hipError_t launch_count_batch(int kind, const DevView* views, const uint32_t* pre, uint32_t nmem,
                              uint32_t blocks, uint32_t kappa, bool sweep, hipStream_t s) {
  return sweep ? count_batch_dispatch<MODE_SWEEP>(kind, views, pre, nmem, blocks, kappa, s)
               : count_batch_dispatch<MODE_CLASS>(kind, views, pre, nmem, blocks, kappa, s);
}

}  // namespace bnlat
