/*
 * bnlat.h -- C ABI of the MI355X (gfx950) screen-space lattice-offset optimiser.
 *
 * The method (Belcour & Heitz, "Lessons Learned and Improvements when
 * Building Screen-Space Samplers with Blue-Noise Error Distribution",
 * SIGGRAPH 2021 Talks):
 *   - Sec. 2: a screen-space sampler is a main sequence plus a tile of
 *     per-pixel scrambling parameters u_p; the tile is optimised so that the
 *     pixels' Monte Carlo errors on random test integrands minimise the
 *     Gaussian-windowed energy of Eq. (1);
 *   - Sec. 3.2: main sequence = 2D rank-1 lattice s^k = mod(Phi(k) g / N, 1),
 *     scrambled per pixel by the toroidal shift mod(s^k + u_p, 1) (Fig. 1a);
 *   - Sec. 3.3: a sampler is assessed by the RMSE of its error tile after
 *     Gaussian blurs of several sizes (Fig. 1c);
 *   - Sec. 3.4: the optimiser mutates disjoint pixel sets in parallel.
 *
 * Conventions shared by every entry point
 *   - Return value: bn_status; BN_OK (0) on success, a negative code on
 *     failure.  On failure bn_last_error() holds a message (thread local) and
 *     the problem keeps its previous state unless stated otherwise.
 *   - Fixed point: offsets and sample coordinates are Q0.16 (uint16 v means
 *     v / 65536); the modulo-one wrap is uint16 wrap-around.  N = 2^m must
 *     divide 65536.
 *   - Memory: the library allocates and owns every device buffer of a
 *     problem (created in bn_create_problem, freed in bn_destroy_problem),
 *     except those a caller hands to bn_create_problem_ext.
 *     Every pointer argument named host_* or out is caller-owned host
 *     memory of the size stated; the library never keeps it.
 *   - Streams: all device work of a problem is ordered on its HIP stream
 *     (given at creation, or created by the library).  Entry points that
 *     return data to host memory synchronise that stream first.
 *   - Thread safety: a problem (or batch) may be used by one host thread at a
 *     time; distinct problems may be used concurrently.
 *   - The library has no CPU fallback: without a usable gfx950 device every
 *     entry point that needs one returns BN_EHIP.
 */
#ifndef BNLAT_H
#define BNLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bn_problem_s* bn_problem;
typedef struct bn_batch_s* bn_batch;

typedef enum {
  BN_OK = 0,
  BN_EINVAL = -1,       /* invalid argument or configuration                  */
  BN_ENOMEM = -2,       /* device or host allocation failed                   */
  BN_EHIP = -3,         /* HIP runtime error (no device, launch failure, ...) */
  BN_ESTATE = -4,       /* call out of order (e.g. sweep before errors)       */
  BN_EUNSUPPORTED = -5, /* valid request this build does not implement        */
  BN_ENUMERIC = -6      /* non-finite or out-of-range numeric result          */
} bn_status;

/* Arithmetic of the colour phases' energy change (Eq. (1) over the window).
 * BN_FP32: exact integer class sums of the hit counts on the vector ALUs
 *          (Gaussian rows: FP64 arithmetic on FP32 estimates).
 * BN_BF16: the neighbour (Gram) products sum_t d_t e_{p+o,t}, d = e' - e, on
 *          the matrix cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation)
 *          from a BF16 copy of the error field kept in device memory; the
 *          self term W sum_t d_t (e'_t + e_t) stays in full precision.
 *          - N <= 256 with Heaviside rows only: the operands are the hit
 *            counts and their changes, exact in BF16, and a slice whose
 *            partial sums stay below 2^24 is exact; decisions equal BN_FP32's
 *            (uncertified accepted moves are re-checked exactly).
 *          - otherwise: the operands are e = c/N - A (g - I for Gaussians)
 *            formed in FP32 and rounded to BF16, and d rounded to BF16: an
 *            approximate energy change.  Every move it accepts is
 *            re-evaluated with the BN_FP32 arithmetic and committed only if
 *            that accepts it too (else counted in bf16_vetoes); moves it
 *            rejects stay rejected.
 *          colour_k must be 1, 2 or 4; redraw moves only.                   */
typedef enum { BN_FP32 = 0, BN_BF16 = 1 } bn_precision;

/* Mutation.
 * BN_REDRAW: the pixel's offset is redrawn from the Philox stream and its hit
 *   counts recomputed (Sec. 3.4 run with random offset proposals); a sweep is
 *   K*K colour phases.
 * BN_SWAP: the paper's own move (the tile is optimised by permuting its
 *   pixels, Sec. 2; couples are swapped in parallel, Sec. 3.4).  A fixed
 *   permutation pi of the P pixels sorts them by the 64-bit keys
 *   (w0 << 32) | w1 of Philox((p, 0, problem_id, 0xE)); pass kappa of sweep s
 *   XORs the listed pixel indices with word 0 of Philox((kappa, s,
 *   problem_id, 0xF)) mod P, takes list positions [kappa M, (kappa+1) M)
 *   with M = P / (K*K), and couples positions 2i and 2i+1.  Every couple is
 *   evaluated on the pass-start state (exact integer energy change including
 *   the pair term when the two pixels are within each other's window) and
 *   accepted couples exchange offsets and hit counts; nothing is recounted.
 *   A sweep is K*K passes.  Requires W*H a power of two, W*H >= 2 K*K, FP32
 *   precision and Heaviside integrands only (else BN_EUNSUPPORTED). */
typedef enum { BN_REDRAW = 0, BN_SWAP = 1 } bn_move;

/* Problem description (Eq. (1) window, Sec. 3.2 lattice, Sec. 3.4 classes). */
typedef struct {
  uint32_t n;            /* samples per pixel N = 2^m, 1 <= N <= 32768 (N > 4096: BN_EUNSUPPORTED) */
  uint32_t g[2];         /* lattice generator; each component odd (coprime to N) */
  uint32_t width;        /* toroidal tile width W  (multiple of colour_k)        */
  uint32_t height;       /* toroidal tile height H (multiple of colour_k)        */
  uint32_t t_heaviside;  /* number T of Heaviside test integrands, >= 1          */
  uint32_t t_gauss;      /* number of Gaussian integrands (Sec. 3.5), >= 0      */
  double sigma;          /* energy weight w_o = exp(-|o|^2 / sigma^2), > 0       */
  uint32_t radius;       /* window offsets o in [-r, r]^2 \ {0}; 1 <= r < min(W,H), r <= 8 (r > 6: BN_EUNSUPPORTED) */
  uint32_t colour_k;     /* colour modulus K: K*K classes (y mod K) K + (x mod K) */
  int32_t objective;     /* +1: accept dE < 0 (descend Eq. (1)); -1: accept dE > 0 */
  uint64_t seed;         /* Philox key (low, high 32 bits)                       */
  uint32_t problem_id;   /* third Philox counter word; batch member index        */
  bn_precision precision;
  bn_move move;
} bn_config;

/* One Heaviside test integrand (Sec. 2): f(x) = 1 iff n . (x - c/65536) > 0
 * (edge excluded); n is an int16 normal of length about 2^14, c a Q0.16
 * point on the edge.  8 bytes, no padding. */
typedef struct {
  int16_t nx, ny;
  uint16_t cx, cy;
} bn_heaviside;

/* One isotropic Gaussian test integrand (Sec. 3.5 low-frequency family):
 * f(x) = exp(-|x - (mx, my)|^2 / (2 s^2)), s > 0, no wrap. */
typedef struct {
  double mx, my, s;
} bn_gaussian;

typedef struct {
  uint64_t proposals;    /* moves evaluated (redraw: pixels; swap: couples)    */
  uint64_t accepts;      /* moves committed                                    */
  uint64_t bf16_vetoes;  /* BF16 accepts rejected by the exact re-check        */
  uint64_t sweep_index;  /* sweep index after the call                         */
} bn_sweep_stats;

/* ---------------------------------------------------------------- lifecycle */

/* Create a problem.  cfg is validated before any device work (rules above).
 * heavisides: host array [cfg->t_heaviside], or NULL to draw them from the
 *   Philox stream (counter (t, 0, problem_id, 0xB): angle 2 pi w0 2^-32,
 *   normal = round-half-even(2^14 (cos, sin)), edge point (w1>>16, w2>>16)).
 * gaussians: host array [cfg->t_gauss], or NULL to draw them (counter
 *   (t, 1, problem_id, 0xB): centre (w0, w1) 2^-32, s = 0.05 + 0.25 w2 2^-32).
 * stream: hipStream_t to order all work on, or NULL to let the library create
 *   (and later destroy) a non-blocking stream.
 * Exact integrals are computed on the host in FP64: the area of the unit
 * square on a Heaviside's hit side, and the erf product for a Gaussian.
 * Gaussian rows enter the energy in the plain form (FP32 estimates, FP64
 * arithmetic); Heaviside rows stay exact.  *out receives the handle. */
bn_status bn_create_problem(const bn_config* cfg, const bn_heaviside* heavisides,
                            const bn_gaussian* gaussians, void* stream, bn_problem* out);
/* Device buffers the caller owns (for example PyTorch tensors), so that a
 * problem's state lives in memory the caller allocates and can read in
 * place.  Every pointer is nullable (the library then allocates that buffer
 * itself).  Layouts, with P = W H and Tp = T rounded up to 128:
 *   offsets  uint32 [P]           pixel p = y W + x, Q0.16 x | y << 16;
 *   counts   uint16 [Tp/8][P][8]  hit counts in 16-byte tiles of 8 integrands
 *                                 (integrand t of pixel p at ((t/8) P + p) 8 + t%8;
 *                                 rows past T hold 0);
 *   errors   float  [P][Tp]       error vectors c/N - A (brought up to date from
 *                                 the counts by the calls that read them).
 * Each must be device memory of at least that size, 256-byte aligned (else
 * BN_EINVAL), alive and unmoved until bn_destroy_problem; the library never
 * frees them and the caller must not write them while the problem's stream
 * has work pending.  Otherwise identical to bn_create_problem (the
 * ownership convention of the C ABI's boundary). */
typedef struct {
  void* offsets;
  void* counts;
  void* errors;
} bn_device_buffers;
bn_status bn_create_problem_ext(const bn_config* cfg, const bn_heaviside* heavisides,
                                const bn_gaussian* gaussians, void* stream, const bn_device_buffers* bufs,
                                bn_problem* out);
bn_status bn_destroy_problem(bn_problem p);

/* Set the offset tile U = {u_p} (Sec. 2).  host_u: uint16 [H][W][2] (x then y), or
 * NULL for Philox offsets (counter (p, 0, problem_id, 0xA), p = y W + x,
 * u = (w0 >> 16, w1 >> 16)).  Invalidates hit counts and errors. */
bn_status bn_init_offsets(bn_problem p, const uint16_t* host_u);

/* Hit counts c[p][t] = #{k : f_t(s_p^k) = 1} and error vectors
 * e[p][t] = c/N - A_t (FP32) of every pixel (Sec. 2, estimator of the test
 * integrand map).  Requires offsets. */
bn_status bn_compute_errors(bn_problem p);

/* Run k sweeps of the parallel optimiser (Sec. 3.4).  One sweep visits the
 * K*K colour classes in increasing order; for every pixel of a class it
 * draws a proposal (counter (p, sweep, problem_id, 0xC)), recounts its hits,
 * evaluates the energy change of Eq. (1) against the state at the start of
 * the phase and commits the accepted moves; then the sweep index advances.
 * A proposal and its recount depend only on (pixel, sweep), never on the
 * state, so the recount of sweep s+1 runs on an auxiliary stream while sweep
 * s is evaluated and committed (two sweeps per replay of a captured graph);
 * the result equals the plain sequential schedule bit for bit.
 * stats (nullable) receives totals over the k sweeps (synchronises).
 * Returns BN_ESTATE before bn_compute_errors. */
bn_status bn_sweep(bn_problem p, uint32_t k, bn_sweep_stats* stats);

/* Energy of Eq. (1) over the window, both orderings of each pair:
 * E = sum_p sum_o w_o |e_p - e_{p+o}|^2, evaluated exactly in integers per
 * distance class and combined in FP64.  Synchronises. */
bn_status bn_energy(bn_problem p, double* out);

/* BF16 precision form only: Eq. (1) over the window evaluated from the BF16
 * field (FP32 squares per 8 integrands, FP64 sums): the counts' exact energy
 * when N <= 256 with Heaviside rows only, else the energy of the BF16-rounded
 * error vectors, to be compared with bn_energy's FP64 value (the error of
 * the form).  BN_ESTATE for BN_FP32 problems.  Synchronises. */
bn_status bn_energy_bf16(bn_problem p, double* out);

/* Blur criterion of Sec. 3.3 / Fig. 1c: for each sigmas[i] > 0,
 * out[i] = sqrt(mean_{p,t} ((k_sigma * e_t)(p))^2) over all T + T_G rows, with k_sigma the
 * normalised Gaussian of standard deviation sigma periodised on the torus,
 * applied separably.  n <= 64.  Synchronises. */
bn_status bn_quality_metric(bn_problem p, const double* sigmas, uint32_t n, double* out);
/* The same criterion over one family of integrand rows (Sec. 3.5 evaluates
 * low-frequency integrands on tiles optimised for Heavisides):
 * BN_ROWS_ALL as above, BN_ROWS_HEAVISIDE the T Heaviside rows only,
 * BN_ROWS_GAUSSIAN the T_G Gaussian rows only (BN_EINVAL when T_G = 0). */
typedef enum { BN_ROWS_ALL = 0, BN_ROWS_HEAVISIDE = 1, BN_ROWS_GAUSSIAN = 2 } bn_rows;
bn_status bn_quality_metric_family(bn_problem p, bn_rows rows, const double* sigmas, uint32_t n, double* out);

/* Error spectrum beside the blur criterion (the |FFT(e)|^2 insets of
 * Fig. 1b): for every integrand row of the family (BN_ROWS_* as above) the
 * power |DFT2(e_t)(u, v)|^2 / (W H) over the W x H torus, averaged over the
 * rows and over the frequencies of each radial bin.  Frequency (u, v) has
 * the radius of (u/W, v/H) folded to [-1/2, 1/2) in cycles per pixel; its bin
 * is that radius times min(W, H), rounded to the nearest integer; bins from
 * nbins on are dropped.  out double [nbins] (0 for an empty bin), counts
 * uint32 [nbins] frequencies per bin (nullable).  White noise of variance s^2
 * gives s^2 in every bin.  Direct DFT on the device (FP32 within a row or
 * column, FP64 across rows); allocates scratch for the call.  Synchronises. */
bn_status bn_error_spectrum(bn_problem p, bn_rows rows, uint32_t nbins, double* out, uint32_t* counts);

/* Copy the offset tile to host_u: uint16 [H][W][2].  Synchronises. */
bn_status bn_get_offsets(bn_problem p, uint16_t* host_u);

/* ------------------------------------------------------- inspection / parity */

/* host: uint16 [H*W][T] hit counts.  Requires bn_compute_errors. */
bn_status bn_get_counts(bn_problem p, uint16_t* host);
/* host: float [H*W][T + T_G] error vectors (Heaviside rows, then Gaussian
 * rows).  Requires bn_compute_errors. */
bn_status bn_get_errors(bn_problem p, float* host);
/* Integrand tables as used and their FP64 exact integrals; every pointer is
 * nullable: heavisides [T], areas [T], gaussians [T_G], gauss_integrals [T_G]. */
bn_status bn_get_integrands(bn_problem p, bn_heaviside* heavisides, double* areas,
                            bn_gaussian* gaussians, double* gauss_integrals);
/* The N scrambled samples of one pixel in van der Corput order k = 0..N-1,
 * computed on the device: host uint16 [N][2].  Synchronises. */
bn_status bn_get_points(bn_problem p, uint32_t pixel, uint16_t* host);
/* Energy change of moving pixels[j] (raster index y W + x, distinct) to
 * offset proposals[j] (uint16 [m][2]) against the current state, each
 * evaluated alone; no state change.  out_de: double [m]; out_counts
 * (nullable): uint16 [m][T] recounted hits.  m <= H*W.  Synchronises. */
bn_status bn_delta_energy(bn_problem p, const uint32_t* pixels, const uint16_t* proposals,
                          uint32_t m, double* out_de, uint16_t* out_counts);
/* Allocation-free variant of bn_delta_energy, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * bn_delta_energy; its list buffers (pixels, proposals, recounted hits,
 * energy changes, decisions, Gaussian estimates and, when out_counts is
 * given, the hits in row layout) live in a fixed 32 MiB scratch array that
 * the library holds on each GPU until the process ends, instead of buffers
 * the problem allocates.  It calls no hipMalloc/hipFree.  A call whose lists
 * do not fit returns BN_EINVAL before any device work: each pixel takes about
 * 2 Tp + 4 TGp + 25 bytes (Tp = T rounded up to 128, TGp = T_G rounded up to
 * 64) plus 2 T with out_counts, e.g. about 8000 pixels at T = 1024.  Every
 * call on a GPU shares that GPU's array and leaves its contents behind
 * (nothing in it has to start at zero); calls that overlap in time on one GPU
 * (from several host threads or streams) race and must be serialised by the
 * caller.  Synchronises the problem's stream. */
bn_status bn_delta_energy_noalloc(bn_problem p, const uint32_t* pixels, const uint16_t* proposals,
                                  uint32_t m, double* out_de, uint16_t* out_counts);
bn_status bn_get_sweep_index(bn_problem p, uint64_t* out);
bn_status bn_set_sweep_index(bn_problem p, uint64_t sweep);

/* Kernel timing of bn_sweep.  While profiling is on, bn_sweep runs the same
 * overlapped schedule eagerly (no graph replay) and records HIP events on
 * each launch's own stream: around the sweep-wide recount (the counting
 * kernel, on the library's auxiliary stream), around each colour phase's
 * evaluation and around its commit (problem stream).  bn_set_profiling
 * synchronises and clears the record; bn_get_profile synchronises and sums
 * the event intervals. */
typedef struct {
  uint64_t recount_launches;  /* sweep-wide counting launches recorded          */
  double recount_ms;          /* their total duration                           */
  uint64_t phases;            /* colour phases recorded                         */
  double evaluate_ms;         /* total duration of the phases' evaluations      */
  double commit_ms;           /* total duration of the phases' commits          */
} bn_profile_stats;
bn_status bn_set_profiling(bn_problem p, int enable);
/* Launch shape of the sweep-wide recount in bn_sweep's overlapped schedule:
 * at most `blocks` workgroups of 256 threads, each striding over the work, so
 * that the recount leaves room on every CU for the colour phases running
 * beside it (rounded down to the workgroup count that gives every workgroup
 * the same number of blocks); 0 removes the cap.  Default: four workgroups per
 * CU.  Results do not depend on it.
 * Synchronises. */
bn_status bn_set_recount_blocks(bn_problem p, uint32_t blocks);
bn_status bn_get_profile(bn_problem p, bn_profile_stats* out);

/* The three steps of one colour phase kappa < K*K at the current sweep
 * index, as bn_sweep runs them: propose + recount, evaluate, commit.
 * bn_phase_advance moves the sweep index on by one (device and host).
 * bn_get_phase copies the last phase's per-pixel results (class order is
 * raster order of the class pixels); every pointer is nullable:
 * u_new uint16 [M][2], c_new uint16 [M][T], delta double [M], accept uint8 [M],
 * with M = H*W / (K*K). */
bn_status bn_phase_propose(bn_problem p, uint32_t kappa);
bn_status bn_phase_evaluate(bn_problem p, uint32_t kappa);
bn_status bn_phase_commit(bn_problem p, uint32_t kappa);
bn_status bn_phase_advance(bn_problem p);
bn_status bn_get_phase(bn_problem p, uint16_t* u_new, uint16_t* c_new, double* delta,
                       uint8_t* accept);

/* BF16 form: the last phase's energy changes as the matrix-core pass
 * computed them, before the exact re-evaluation of accepted moves
 * (bn_get_phase's delta holds the re-evaluated value for those):
 * delta_bf16 double [M].  BN_ESTATE for BN_FP32 problems.  Synchronises. */
bn_status bn_get_phase_bf16(bn_problem p, double* delta_bf16);

/* Swap problems (BN_SWAP): the phase steps above run swap pass kappa
 * (propose lists the pass's couples, evaluate decides them, commit exchanges
 * the accepted ones), and bn_get_swap_pass copies the last evaluated pass in
 * couple order: pixels a, b uint32 [M/2] (y*W + x), delta double [M/2],
 * accept uint8 [M/2]; every pointer is nullable.  bn_get_phase returns
 * BN_ESTATE for swap problems and bn_get_swap_pass for redraw problems. */
bn_status bn_get_swap_pass(bn_problem p, uint32_t* a, uint32_t* b, double* delta, uint8_t* accept);

/* -------------------------------------------------------------- measurement */

/* Attainable device peaks, the denominators of measured roofline fractions
 * (measurement infrastructure, not part of the method).  Each kind times a
 * plain loop on the current device and returns the best of `reps` launches
 * (1..1000) in *out:
 *   BN_PEAK_HBM_COPY   device-to-device copy of `bytes` (a multiple of 16,
 *                      >= 1 MiB; the library allocates and frees two buffers
 *                      of that size), by the library's copy kernel and by the
 *                      runtime's hipMemcpyAsync in alternate repetitions (the
 *                      better rate is returned): bytes read + written per
 *                      second;
 *   BN_PEAK_VALU_DOT2  independent chains of v_dot2_i32_i16 in eight
 *                      workgroups of 256 threads per CU: lane-operations per
 *                      second (`bytes` ignored);
 *   BN_PEAK_MFMA_BF16  independent v_mfma_f32_32x32x16_bf16 accumulations,
 *                      same launch: dense BF16 flops per second. */
typedef enum { BN_PEAK_HBM_COPY = 0, BN_PEAK_VALU_DOT2 = 1, BN_PEAK_MFMA_BF16 = 2 } bn_peak;
bn_status bn_measure_peak(bn_peak kind, uint64_t bytes, uint32_t reps, double* out);

/* ------------------------------------------------------------ sampler query */

/* The padded screen-space sampler a renderer reads (Sec. 3.1: dimensions are
 * consumed in pairs, each pair (2d, 2d+1) with its own tile; a 1-D effect
 * takes one dimension of a pair and discards the other.  Sec. 3.2: sample k
 * of pixel p is mod(Phi(k) g / N + u_p, 1), Phi the base-2 radical inverse).
 * pairs[d] is the problem that holds pair d's lattice and offset tile (for
 * example the members of a batch).  For query j: screen pixel (x[j], y[j]),
 * any values, wrapped modulo each tile; sample index k[j] in van der Corput
 * order, taken modulo that pair's N.  out[j * 2 npairs + 2d + a] = component a
 * of pair d's sample, a float in [0, 1) (exact: the Q0.16 value / 65536).
 * Every pair must have offsets (bn_init_offsets); the pairs' pending work is
 * waited for.  bn_sample takes host arrays x, y, k uint32 [m] and host out
 * float [m][2 npairs]; bn_sample_device takes device arrays and a stream
 * (NULL: pairs[0]'s stream) and synchronises it.  Both allocate a small
 * device table per call. */
bn_status bn_sample(const bn_problem* pairs, uint32_t npairs, const uint32_t* x, const uint32_t* y,
                    const uint32_t* k, uint32_t m, float* out);
bn_status bn_sample_device(const bn_problem* pairs, uint32_t npairs, const uint32_t* x, const uint32_t* y,
                           const uint32_t* k, uint32_t m, float* out, void* stream);

/* ----------------------------------------------------------------- batching */

/* Independent problems (e.g. the dimension pairs of a padded sampler,
 * Sec. 3.1) swept together in one captured HIP graph of two sweeps.  Members
 * in the FP32 form with Heaviside rows only and redraw moves share grouped
 * launches: one sweep-wide recount launch per samples-per-pixel class (on an
 * auxiliary stream, for the next sweep) beside, per colour class, one launch
 * per window radius for the energy change and one decision and one commit
 * launch over all of them.  Members in the BF16 form, with Gaussian rows or
 * with swap moves have their own overlapped sweeps recorded into the same
 * graph as independent branches.  Each member's trajectory equals the one
 * bn_sweep gives it alone.  Requirements: members distinct, created on one
 * stream, bn_compute_errors done, profiling off, one common colour_k in
 * {1, 2, 4}.  tune_cache (nullable) names a text file of launch choices
 * keyed by the members' shapes; when the key is absent (or its choice is not
 * one of the candidates) the tuner times the candidates on the device (a
 * recount and evaluations without commit, no state change) and appends its
 * choice.  Members stay owned by the caller and must outlive the batch;
 * sweeping a member on its own between batched sweeps is allowed. */
bn_status bn_create_batch(const bn_problem* members, uint32_t m, const char* tune_cache,
                          bn_batch* out);
bn_status bn_batch_sweep(bn_batch b, uint32_t k);
/* Launch choices the tuner picked (integrands per counting wave, workgroup
 * target of the staged energy-change launch, its block shape: 0 the
 * single-problem shape, 1 the alternative with half the waves per workgroup
 * for K = 1, 2 and twice for K = 4); every pointer nullable; no device work. */
bn_status bn_batch_tuning(bn_batch b, uint32_t* tch, uint32_t* slice_target, uint32_t* stage_shape);
bn_status bn_destroy_batch(bn_batch b);

/* ------------------------------------------------ host-only (no device work) */

bn_status bn_validate_config(const bn_config* cfg);
/* Distinct squared distances d of the window offsets in increasing order and
 * their weights exp(-d / sigma^2) (FP64): class_d uint32 [*n_classes],
 * class_w double [*n_classes]; pass NULL arrays to query the count. */
bn_status bn_window_classes(const bn_config* cfg, uint32_t* n_classes, uint32_t* class_d,
                            double* class_w);
/* Pixel permutation pi of the swap mutation (see BN_SWAP): out uint32 [W*H]
 * receives pi[L] for L = 0 .. W*H-1.  Requires W*H a power of two. */
bn_status bn_swap_permutation(const bn_config* cfg, uint32_t* out);
/* Exact area (FP64) of the unit square on the hit side of one Heaviside. */
bn_status bn_heaviside_area(const bn_heaviside* h, double* out);
/* The Philox-drawn Heavisides bn_create_problem uses when given NULL. */
bn_status bn_draw_heavisides(uint64_t seed, uint32_t problem_id, uint32_t t, bn_heaviside* out);
/* The Philox-drawn Gaussians bn_create_problem uses when given NULL. */
bn_status bn_draw_gaussians(uint64_t seed, uint32_t problem_id, uint32_t t, bn_gaussian* out);
/* Exact integral (FP64) of one Gaussian over the unit square (erf product). */
bn_status bn_gaussian_integral(const bn_gaussian* g, double* out);

const char* bn_status_string(bn_status s);
const char* bn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BNLAT_H */
