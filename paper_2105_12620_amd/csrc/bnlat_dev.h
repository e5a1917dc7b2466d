// Internal interface between the C-ABI host code and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bnlat {

// Philox stream tags (fourth counter word).
constexpr uint32_t S_INIT = 0xA;
constexpr uint32_t S_INTEG = 0xB;
constexpr uint32_t S_PROP = 0xC;

// Integrand rows are padded to a multiple of this many entries; padded rows
// have normal (0, 0) and threshold 0, so their hit count is always 0 and they
// contribute nothing to energies.
constexpr uint32_t T_ALIGN = 128;
constexpr uint32_t MAX_RADIUS = 8;
constexpr uint32_t MAX_N = 4096;
// Size of the per-GPU scratch array of the allocation-free entry point.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;

// MODE_SWEEP: proposals of every pixel of a sweep, rows grouped by colour
// class ([class][class pixel]); the kernel argument kappa is then the sweep
// look-ahead added to the device sweep counter.
enum CountMode : int { MODE_ALL = 0, MODE_CLASS = 1, MODE_LIST = 2, MODE_SWEEP = 3 };

// Everything a kernel needs to know about one problem, passed by value.
struct DevView {
  uint32_t n, log2n, w, h, t, tp, k, cw, ch, pc;
  uint32_t problem, seed_lo, seed_hi;
  int32_t objective;
  uint32_t radius, ncls;
  const uint32_t* lat;       // [n] lattice points, x | y << 16, index order i
  const int2* ihp;           // [tp] (nx | ny << 16, D' = n . (C - 2^15))
  const float* area;         // [tp] FP32 exact integrals (0 for padding)
  const double* wd;          // [ncls] class weights exp(-d / sigma^2)
  uint32_t* U;               // [P] offsets, x | y << 16
  uint16_t* cnt;             // [tp/8][P][8] hit counts (16-byte integrand tiles)
  float* err;                // [P][tp] error vectors
  uint32_t* u_new;           // [M] proposals of the current phase / list
  uint16_t* c_new;           // [tp/8][M][8] recounted hits of the proposals
  double* delta;             // [M] energy change
  uint8_t* accept;           // [M] decision
  const uint32_t* pix_list;  // [M] pixels (list mode)
  unsigned long long* ctr;   // [0] sweep index, [1] accepted total, [2] BF16 vetoes,
                             // [3] the overlapped schedule's recount index
  long long* xpart;          // [ncls][pc] integer class sums of the staged evaluation (kept zero between phases)
  uint32_t* unsure;          // [pc] matrix-core results not certified exact (kept zero between phases)
  uint32_t mfma;             // colour phases' evaluation: 0 FP32 form (exact integer stencil), 1 BF16 matrix
                             // cores on exact counts (N <= 256, Heaviside rows only), 2 BF16 matrix cores on
                             // rounded error vectors with exact re-evaluation of accepted moves
  uint32_t tb;               // rows of the BF16 field: tp + tgp
  uint16_t* bf;              // [tb/8][P][8] BF16 field (mode 1: counts; mode 2: errors), else null
  double* delta_bf;          // [M] energy change the BF16 pass computed (before re-evaluation), else null
  double xscale;             // energy change = xscale * sum_d w_d X_d of the class sums X_d
  uint32_t tch;              // integrands per wave in the counting kernels (launch shape)
  uint32_t slice_target;     // workgroups the staged energy-change launch aims for
  uint32_t count_cap;        // workgroup cap of the sweep-wide recount launch (0: none)
  // Gaussian integrands (tgp = 0 when there are none)
  uint32_t tg, tgp;          // count, padded to 64
  const double* gcoef;       // [tgp][4] exponent coefficients a, bx, by, c (base 2; 0 for padding)
  const double* gint;        // [tgp] exact integrals
  float* gest;               // [P][tgp] estimates
  float* gerr;               // [P][tgp] errors g - I (refreshed on demand)
  float* g_new;              // [M][tgp] estimates of the proposals
  double* gdelta;            // [M] Gaussian part of the energy change
};

hipError_t launch_init_offsets(const DevView& v, hipStream_t s);
hipError_t launch_count(const DevView& v, int mode, uint32_t kappa, uint32_t m, hipStream_t s);
hipError_t launch_delta(const DevView& v, int mode, uint32_t kappa, uint32_t m, hipStream_t s);
uint32_t xpart_words(const DevView& v);
hipError_t launch_commit(const DevView& v, uint32_t kappa, hipStream_t s);
uint32_t commit_blocks(const DevView& v);
hipError_t launch_errors(const DevView& v, hipStream_t s);
hipError_t launch_advance(const DevView& v, hipStream_t s);
hipError_t launch_recount_index(const DevView& v, hipStream_t s);
hipError_t launch_recount_advance_pair(const DevView& v, hipStream_t s);
hipError_t launch_points(const DevView& v, uint32_t pixel, uint32_t* out, hipStream_t s);
hipError_t launch_energy(const DevView& v, unsigned long long* y, hipStream_t s);
hipError_t launch_blur(const DevView& v, const float* field, uint32_t pitch, uint32_t valid, const float* kx,
                       uint32_t nkx, const int32_t* dx, const float* ky, uint32_t nky, const int32_t* dy,
                       float* tmp, double* partial, uint32_t* npartial, hipStream_t s);
uint32_t blur_partials(const DevView& v, uint32_t pitch);
hipError_t launch_gauss_est(const DevView& v, int mode, uint32_t m, hipStream_t s);
hipError_t launch_gauss_delta(const DevView& v, int mode, uint32_t kappa, uint32_t m, hipStream_t s);
hipError_t launch_gauss_commit(const DevView& v, uint32_t kappa, hipStream_t s);
hipError_t launch_gauss_errors(const DevView& v, hipStream_t s);
hipError_t launch_gauss_energy(const DevView& v, double* gsum, hipStream_t s);

// batched launches: member i of a group owns blocks pre[i] .. pre[i+1]-1
int count_kind(const DevView& v);
uint32_t count_blocks(const DevView& v, bool sweep);
// staged-kernel block shape 0 (default) or 1 (the tuner's alternative)
uint32_t stage_rows(uint32_t k, uint32_t shape);
void stage_geometry(const DevView& v, uint32_t shape, uint32_t* gx, uint32_t* gy, uint32_t* gz, uint32_t* trlen);
hipError_t launch_count_batch(int kind, const DevView* views, const uint32_t* pre, uint32_t nmem,
                              uint32_t blocks, uint32_t kappa, bool sweep, hipStream_t s);
hipError_t launch_stage_batch(uint32_t radius, uint32_t k, uint32_t shape, const DevView* views, const uint32_t* pre,
                              const uint32_t* geo, uint32_t nmem, uint32_t blocks, uint32_t kappa,
                              hipStream_t s);
hipError_t launch_finish_batch(const DevView* views, const uint32_t* pre, uint32_t nmem, uint32_t blocks,
                               hipStream_t s);
hipError_t launch_commit_batch(const DevView* views, const uint32_t* pre, uint32_t nmem, uint32_t blocks,
                               uint32_t kappa, hipStream_t s);
hipError_t launch_advance_batch(const DevView* views, uint32_t nmem, hipStream_t s);

// BF16 precision form (mfma.hip): the field from counts / estimates, the
// colour phase's evaluation (Gram pass + decision + exact re-evaluation), the
// field's energy
bool bf16_supported_k(uint32_t k);
hipError_t launch_bf_field(const DevView& v, hipStream_t s);
// raises the LDS launch limit of the BF16 kernels of this radius and K (once per process)
hipError_t prepare_bf_kernels(uint32_t radius, uint32_t k);
hipError_t launch_delta_bf16(const DevView& v, uint32_t kappa, hipStream_t s);
hipError_t launch_energy_bf16(const DevView& v, double* ysum, hipStream_t s);
// decision from the summed class sums of a colour phase (clears them)
hipError_t launch_finish(const DevView& v, hipStream_t s);
// the FP32 form's staged evaluation of a colour phase without its decision:
// exact Heaviside class sums into xpart, Gaussian rows' part into gdelta
hipError_t launch_stage_exact(const DevView& v, uint32_t kappa, hipStream_t s);
hipError_t launch_gauss_delta_exact(const DevView& v, uint32_t kappa, hipStream_t s);

// error spectrum (spectrum.hip): DFT of SPEC_CHUNK integrand rows along x
// into rows [H][W][chunk] (complex), then along y with |.|^2 summed over the
// chunk into power [H][W] (added to)
uint32_t spectrum_chunk();
size_t spectrum_scratch_floats2(const DevView& v);
hipError_t launch_spectrum_chunk(const DevView& v, const float* field, uint32_t pitch, uint32_t valid, uint32_t t0,
                                 const float2* twx, const float2* twy, float2* rows, double* power, hipStream_t s);

// device peak loops: kind 0 copy (buf -> buf2, size bytes), 1 dot2 chains,
// 2 BF16 MFMA accumulations (iters iterations each); blocks workgroups of 256
hipError_t peak_launch(int kind, void* buf, void* buf2, uint64_t size, uint32_t iters, uint32_t blocks,
                       hipStream_t s);

// allocation-free entry point: device address of the scratch array on
// `device` (located once per device), and tiled counts -> host row layout
hipError_t noalloc_scratch(int device, void** ptr);
hipError_t launch_untile_counts(const uint16_t* tiled, uint32_t rows, uint32_t t, uint16_t* out, hipStream_t s);

}  // namespace bnlat
