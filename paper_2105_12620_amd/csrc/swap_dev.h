// Internal interface of the swap-mutation kernels (Sec. 3.4: couples of
// pixels exchange their scrambling offsets, so no recount is needed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bnlat_dev.h"

namespace bnlat {

// Philox stream tags of the swap mutation (fourth counter word).
constexpr uint32_t S_PERM = 0xE;   // sort keys of the pixel permutation
constexpr uint32_t S_SWAP = 0xF;   // XOR masks of the passes

// Tables and scratch of the swap passes.  The pixel count P is a power of two;
// a pass takes M = P / K^2 list positions [kappa M, (kappa + 1) M) of the
// XOR-scrambled permutation and couples positions 2i and 2i + 1.
struct SwapView {
  const uint32_t* perm;   // [P] pixel at list position L
  const uint32_t* pinv;   // [P] list position of pixel p
  long long* xs;          // [ncls][M] integer class sums of each couple member's move (zero between passes)
  long long* d2;          // [M/2] sum_t (c_a,t - c_b,t)^2 of each couple (zero between passes)
  const int32_t* dcls;    // [2 r^2 + 1] class index of a squared distance (-1: none)
  uint16_t* row;          // [P][Tp] pixel-major copy of the hit counts: a couple's partner counts
                          // are read whole lines at a time (kept in step by the exchanges)
  uint32_t m;             // list positions per pass
};

// Pass kappa of the sweep in the device counter: evaluate every couple
// (delta/accept [M/2], couple pixels into u_new[2i], u_new[2i+1]), then
// exchange the accepted couples' offsets and count tiles.
// Once per process, before the first swap launch (not under stream capture).
hipError_t prepare_swap_kernels();
// class sums of the pass's couples (and, with decide, their decisions)
hipError_t launch_swap_evaluate(const DevView& v, const SwapView& sv, uint32_t kappa, hipStream_t s,
                                bool decide = true);
// decisions of the pass's couples and the exchange of the accepted ones
hipError_t launch_swap_decide_exchange(const DevView& v, const SwapView& sv, uint32_t kappa, hipStream_t s);
hipError_t launch_swap_commit(const DevView& v, const SwapView& sv, hipStream_t s);
// Rebuild the pixel-major copy from the tiled counts (after every recount).
hipError_t launch_swap_rows(const DevView& v, const SwapView& sv, hipStream_t s);

}  // namespace bnlat
