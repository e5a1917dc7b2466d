// C-ABI of the lattice-offset optimiser: validation, host tables, device
// buffers, stream-ordered launches and graph-captured sweeps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <iterator>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bnlat.h"
#include "bnlat_dev.h"
#include "swap_dev.h"
#include "sampler_dev.h"

using namespace bnlat;

namespace {

thread_local std::string g_last_error;

// Diagnostics, read from the environment at each use:
//   BNLAT_LOG=1          failures and problem creation / destruction are
//                        reported on stderr, one line each;
//   BNLAT_FAULT=alloc:K  the K-th device allocation of every problem being
//                        created (counted from 1) fails as if the device were
//                        out of memory: the error paths can be exercised.
bool log_on() {
  const char* e = std::getenv("BNLAT_LOG");
  return e && *e && std::strcmp(e, "0") != 0;
}

void log_msg(const char* fmt, ...) {
  if (!log_on()) return;
  char buf[640];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[bnlat] %s\n", buf);
}

long fault_alloc_index() {
  const char* e = std::getenv("BNLAT_FAULT");
  if (!e || std::strncmp(e, "alloc:", 6) != 0) return 0;
  return std::strtol(e + 6, nullptr, 10);
}

bn_status fail(bn_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  log_msg("error %d: %s", (int)s, buf);
  return s;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(BN_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

uint32_t round_up(uint32_t v, uint32_t a) { return (v + a - 1) / a * a; }

bool is_pow2(uint32_t v) { return v && !(v & (v - 1)); }

std::vector<uint32_t> swap_permutation(const bn_config& c);

// ------------------------------------------------------------------ Philox
// Host Philox4x32-10 (Salmon et al., SC 2011) for drawing integrands.
void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint32_t)p1;
    c[2] = n2;
    c[3] = (uint32_t)p0;
  }
}

// ------------------------------------------------------ Heaviside integrals
// Area of {x in [0,1]^2 : a x + b y >= k}: walk the square's boundary, keep
// the corners on the hit side and the points where the edge crosses the
// line, then take the polygon's shoelace area.
double half_plane_area(double a, double b, double k) {
  static const double cx[4] = {0.0, 1.0, 1.0, 0.0};
  static const double cy[4] = {0.0, 0.0, 1.0, 1.0};
  double px[8], py[8];
  int m = 0;
  for (int i = 0; i < 4; ++i) {
    const int j = (i + 1) & 3;
    const double fi = a * cx[i] + b * cy[i] - k;
    const double fj = a * cx[j] + b * cy[j] - k;
    if (fi >= 0.0) {
      px[m] = cx[i];
      py[m] = cy[i];
      ++m;
    }
    if ((fi >= 0.0) != (fj >= 0.0)) {
      const double s = fi / (fi - fj);
      px[m] = cx[i] + s * (cx[j] - cx[i]);
      py[m] = cy[i] + s * (cy[j] - cy[i]);
      ++m;
    }
  }
  if (m < 3) return 0.0;
  double twice = 0.0;
  for (int i = 0; i < m; ++i) {
    const int j = (i + 1) % m;
    twice += px[i] * py[j] - px[j] * py[i];
  }
  return std::fabs(twice) * 0.5;
}

bn_status heaviside_area_checked(const bn_heaviside& h, double* out) {
  if (h.nx == 0 && h.ny == 0) return fail(BN_EINVAL, "Heaviside normal is (0, 0)");
  if (h.nx < -16384 || h.nx > 16384 || h.ny < -16384 || h.ny > 16384)
    return fail(BN_EINVAL, "Heaviside normal components must lie in [-16384, 16384]");
  const double k = ((double)h.nx * h.cx + (double)h.ny * h.cy) / 65536.0;
  *out = half_plane_area((double)h.nx, (double)h.ny, k);
  return BN_OK;
}

// Integral of exp(-|x - mu|^2 / (2 s^2)) over [0,1]^2 (separable, erf).
double gaussian_integral(double mx, double my, double sd) {
  const double c = sd * std::sqrt(M_PI / 2.0), r = sd * std::sqrt(2.0);
  return c * (std::erf((1.0 - mx) / r) + std::erf(mx / r)) * c * (std::erf((1.0 - my) / r) + std::erf(my / r));
}

bn_status gaussian_checked(const bn_gaussian& g, double* out) {
  if (!(g.s > 0.0) || !std::isfinite(g.s) || !std::isfinite(g.mx) || !std::isfinite(g.my))
    return fail(BN_EINVAL, "Gaussian needs finite centre and s > 0");
  *out = gaussian_integral(g.mx, g.my, g.s);
  return BN_OK;
}

// ---------------------------------------------------------------- windows
void window_classes(uint32_t r, double sigma, std::vector<uint32_t>& d, std::vector<double>& w) {
  d.clear();
  w.clear();
  for (uint32_t dd = 1; dd <= 2 * r * r; ++dd) {
    bool found = false;
    for (int y = -(int)r; y <= (int)r && !found; ++y)
      for (int x = -(int)r; x <= (int)r && !found; ++x)
        if ((uint32_t)(x * x + y * y) == dd) found = true;
    if (found) {
      d.push_back(dd);
      w.push_back(std::exp(-(double)dd / (sigma * sigma)));
    }
  }
}

// Periodised, normalised Gaussian of standard deviation s on a ring of n
// pixels; returns the taps above a negligible relative level.
void blur_taps(uint32_t n, double s, std::vector<float>& k, std::vector<int32_t>& d) {
  std::vector<double> kd(n, 0.0);
  const int reps = (int)std::ceil(6.0 * s / n) + 1;
  double total = 0.0, kmax = 0.0;
  for (uint32_t i = 0; i < n; ++i) {
    for (int m = -reps; m <= reps; ++m) {
      const double z = (double)i + (double)m * n;
      kd[i] += std::exp(-(z * z) / (2.0 * s * s));
    }
    total += kd[i];
  }
  for (uint32_t i = 0; i < n; ++i) kmax = std::max(kmax, kd[i]);
  k.clear();
  d.clear();
  for (uint32_t i = 0; i < n; ++i)
    if (kd[i] > 1e-12 * kmax) {
      k.push_back((float)(kd[i] / total));
      d.push_back((int32_t)i);
    }
}

}  // namespace

// --------------------------------------------------------------- the handle
struct bn_problem_s {
  bn_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;   // the GPU the problem's buffers live on
  DevView v{};
  std::vector<bn_heaviside> heav;
  std::vector<double> area64;
  std::vector<bn_gaussian> gauss;
  std::vector<double> gint64;
  double* gsum = nullptr;
  float* list_g = nullptr;
  double* list_gdelta = nullptr;
  std::vector<uint32_t> cls_d;
  std::vector<double> cls_w;
  std::vector<void*> allocs;
  uint32_t list_cap = 0;
  uint16_t* list_cnt = nullptr;
  uint32_t* list_u = nullptr;
  uint32_t* list_pix = nullptr;
  double* list_delta = nullptr;
  uint8_t* list_accept = nullptr;
  unsigned long long* ysum = nullptr;
  uint64_t sweep = 0;
  bool have_offsets = false;
  bool have_counts = false;
  bool errors_valid = false;   // FP32 error vectors match the counts
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool graph_failed = false;
  // Overlapped sweeps: proposals of a whole sweep, rows grouped by colour
  // class, in two buffer sets; set 0 always holds the proposals of the
  // current sweep index `prefetched` when that equals `sweep`.
  struct SweepSet {
    uint16_t* cn = nullptr;
    uint32_t* un = nullptr;
    float* gn = nullptr;
  } sets[2];
  bool sets_ready = false;
  uint64_t prefetched = ~0ull;
  hipStream_t aux = nullptr;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  hipGraph_t pair_graph = nullptr;
  hipGraphExec_t pair_exec = nullptr;
  bool pair_failed = false;
  // profiling: eager overlapped sweeps with events around the launches
  bool profiling = false;
  std::vector<hipEvent_t> prof_recount, prof_eval, prof_commit;   // start/stop pairs
  // Swap mutation: permutation tables, pixel-major counts and pass scratch;
  // one captured sweep of K^2 passes.
  SwapView sv{};
  hipGraph_t swap_graph = nullptr;
  hipGraphExec_t swap_exec = nullptr;
  bool swap_failed = false;

  template <class T>
  bn_status alloc(T** ptr, size_t count) {
    void* p = nullptr;
    const long k = fault_alloc_index();
    if (k > 0 && (long)allocs.size() + 1 == k)
      return fail(BN_ENOMEM, "hipMalloc of %zu bytes failed: injected by BNLAT_FAULT", count * sizeof(T));
    hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(BN_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
    }
    allocs.push_back(p);
    *ptr = (T*)p;
    return BN_OK;
  }
  // A caller-owned buffer when given (never freed here), else a new allocation.
  template <class T>
  bn_status adopt(T** ptr, void* given, size_t count) {
    if (!given) return alloc(ptr, count);
    *ptr = (T*)given;
    return BN_OK;
  }
  ~bn_problem_s() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (pair_exec) (void)hipGraphExecDestroy(pair_exec);
    if (pair_graph) (void)hipGraphDestroy(pair_graph);
    if (swap_exec) (void)hipGraphExecDestroy(swap_exec);
    if (swap_graph) (void)hipGraphDestroy(swap_graph);
    if (stream) (void)hipStreamSynchronize(stream);
    if (aux) (void)hipStreamSynchronize(aux);
    for (void* p : allocs) (void)hipFree(p);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto* vec : {&prof_recount, &prof_eval, &prof_commit})
      for (hipEvent_t e : *vec) (void)hipEventDestroy(e);
    if (aux) (void)hipStreamDestroy(aux);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

// A group of batch members served by one launch of one kernel variant.
struct BatchGroup {
  int kind = 0;               // counting-kernel variant (count_kind: N up to 64, else 64 + lanes per item)
  uint32_t radius = 0, k = 0; // staged energy-change variant
  std::vector<uint32_t> idx;  // member indices
  // member view tables on the device: counting groups, one per proposal set
  // (whole sweep); phase groups, one per (set, colour class): set * K^2 + kappa
  std::vector<DevView*> views;
  uint32_t* d_pre = nullptr;  // block prefix sums, idx.size() + 1 entries
  uint32_t* d_geo = nullptr;  // per member (gx, gy, slice length) for the staged kernel
  uint32_t blocks = 0;
};

struct bn_batch_s {
  std::vector<bn_problem> members;
  hipStream_t stream = nullptr;
  uint32_t colour_k = 0;
  std::vector<BatchGroup> count_groups, stage_groups;
  BatchGroup finish_all, commit_all;
  // members outside the grouped FP32 redraw launches (BF16, Gaussian rows or
  // swap moves): their own overlapped sweeps are recorded into the same graph
  std::vector<uint32_t> solo;
  std::vector<void*> allocs;
  // overlapped schedule of the grouped members: the sweep-wide recount of
  // sweep s+1 on `aux` beside the colour phases of sweep s; two sweeps per
  // replay of the captured graph
  hipStream_t aux = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  uint32_t tch = 256, slice_target = 512, shape = 0;
  ~bn_batch_s() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (stream) (void)hipStreamSynchronize(stream);
    if (aux) (void)hipStreamSynchronize(aux);
    for (void* q : allocs) (void)hipFree(q);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (aux) (void)hipStreamDestroy(aux);
  }
};

namespace {

bn_status validate(const bn_config* c) {
  if (!c) return fail(BN_EINVAL, "config is NULL");
  if (!is_pow2(c->n) || c->n > 32768) return fail(BN_EINVAL, "N=%u must be a power of two in [1, 32768]", c->n);
  if (c->n > 1 && (!(c->g[0] & 1) || !(c->g[1] & 1)))
    return fail(BN_EINVAL, "generator components must be odd (coprime to N)");
  if (c->colour_k < 1 || c->width % c->colour_k || c->height % c->colour_k)
    return fail(BN_EINVAL, "colour_k=%u must divide width and height", c->colour_k);
  if (c->width < 2 || c->height < 2) return fail(BN_EINVAL, "tile must be at least 2x2");
  if (c->radius < 1 || c->radius >= std::min(c->width, c->height))
    return fail(BN_EINVAL, "radius must satisfy 1 <= r < min(W, H)");
  if (c->radius > MAX_RADIUS) return fail(BN_EINVAL, "radius must be <= %u", MAX_RADIUS);
  if (c->t_heaviside + c->t_gauss < 1) return fail(BN_EINVAL, "at least one integrand is required");
  if (!(c->sigma > 0.0) || !std::isfinite(c->sigma)) return fail(BN_EINVAL, "sigma must be finite and > 0");
  if (c->objective != 1 && c->objective != -1) return fail(BN_EINVAL, "objective must be +1 or -1");
  if (c->precision != BN_FP32 && c->precision != BN_BF16) return fail(BN_EINVAL, "unknown precision");
  if (c->move != BN_REDRAW && c->move != BN_SWAP) return fail(BN_EINVAL, "unknown move");
  if ((uint64_t)c->width * c->height > (1u << 26)) return fail(BN_EINVAL, "tile larger than 2^26 pixels");
  if (c->t_heaviside > (1u << 16)) return fail(BN_EINVAL, "more than 65536 integrands");
  return BN_OK;
}

bn_status supported(const bn_config* c) {
  if (c->n > MAX_N) return fail(BN_EUNSUPPORTED, "N > %u is not supported by this build", MAX_N);
  if (c->radius > 6) return fail(BN_EUNSUPPORTED, "radius > 6 is not supported by this build");
  if (c->t_heaviside == 0) return fail(BN_EUNSUPPORTED, "at least one Heaviside integrand is required");
  if (c->t_gauss > (1u << 16)) return fail(BN_EINVAL, "more than 65536 Gaussian integrands");
  if (c->precision == BN_BF16 && !bf16_supported_k(c->colour_k))
    return fail(BN_EUNSUPPORTED, "the BF16 matrix-core form needs colour_k in {1, 2, 4}");
  if (c->move == BN_SWAP) {
    const uint64_t P = (uint64_t)c->width * c->height;
    if (!is_pow2((uint32_t)P) || P < 2ull * c->colour_k * c->colour_k)
      return fail(BN_EUNSUPPORTED, "swap moves need W*H a power of two and at least 2 K^2");
    if (c->precision != BN_FP32) return fail(BN_EUNSUPPORTED, "swap moves run in the FP32 (exact integer) form only");
    if (c->t_gauss) return fail(BN_EUNSUPPORTED, "swap moves support Heaviside integrands only");
  }
  return BN_OK;
}

bn_status check_device() {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count < 1) {
    (void)hipGetLastError();
    return fail(BN_EHIP, "no HIP device available");
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(BN_EHIP, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
  return BN_OK;
}

bn_status sync(bn_problem p) {
  HIPCHK(hipStreamSynchronize(p->stream));
  return BN_OK;
}

// Copy a tiled count buffer ([tp/8][rows][8] uint16 on the device) to host
// rows [rows][t].  Synchronises.
bn_status untile_counts(bn_problem p, const uint16_t* dev, uint32_t rows, uint16_t* host) {
  const uint32_t t = p->v.t, tp = p->v.tp;
  std::vector<uint16_t> tmp((size_t)rows * tp);
  HIPCHK(hipMemcpyAsync(tmp.data(), dev, tmp.size() * 2, hipMemcpyDeviceToHost, p->stream));
  bn_status s = sync(p);
  if (s != BN_OK) return s;
  for (uint32_t r = 0; r < rows; ++r)
    for (uint32_t i = 0; i < t; ++i) host[(size_t)r * t + i] = tmp[((size_t)(i >> 3) * rows + r) * 8 + (i & 7)];
  return BN_OK;
}

bn_status ensure_list(bn_problem p, uint32_t m) {
  if (m <= p->list_cap) return BN_OK;
  bn_status s;
  if ((s = p->alloc(&p->list_cnt, (size_t)m * p->v.tp)) != BN_OK) return s;
  if ((s = p->alloc(&p->list_u, m)) != BN_OK) return s;
  if ((s = p->alloc(&p->list_pix, m)) != BN_OK) return s;
  if ((s = p->alloc(&p->list_delta, m)) != BN_OK) return s;
  if ((s = p->alloc(&p->list_accept, m)) != BN_OK) return s;
  if ((s = p->alloc(&p->list_g, (size_t)m * std::max<uint32_t>(p->v.tgp, 1))) != BN_OK) return s;
  if ((s = p->alloc(&p->list_gdelta, m)) != BN_OK) return s;
  p->list_cap = m;
  return BN_OK;
}

// Regions of one pixel list carved from a fixed scratch area (256-byte
// aligned); with a null base it only measures.
struct Carve {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* r = (T*)(base + off);
    off += std::max<size_t>(count, 1) * sizeof(T);
    return r;
  }
};

// The list buffers of a delta-energy call over m pixels (and, when untiled
// counts are returned, their row layout) in scratch area c.
DevView list_view_in(bn_problem p, Carve& c, uint32_t m, bool counts, uint16_t** rows) {
  DevView lv = p->v;
  lv.pix_list = c.take<uint32_t>(m);
  lv.u_new = c.take<uint32_t>(m);
  lv.c_new = c.take<uint16_t>((size_t)m * p->v.tp);
  lv.delta = c.take<double>(m);
  lv.accept = c.take<uint8_t>(m);
  lv.g_new = c.take<float>((size_t)m * std::max<uint32_t>(p->v.tgp, 1));
  lv.gdelta = c.take<double>(m);
  *rows = counts ? c.take<uint16_t>((size_t)m * p->v.t) : nullptr;
  return lv;
}

// Bring the FP32 error vectors up to date with the counts.
bn_status refresh_errors(bn_problem p) {
  if (p->errors_valid) return BN_OK;
  HIPCHK(launch_errors(p->v, p->stream));
  HIPCHK(launch_gauss_errors(p->v, p->stream));
  p->errors_valid = true;
  return BN_OK;
}

bn_status record_sweep(bn_problem p) {
  for (uint32_t kappa = 0; kappa < p->cfg.colour_k * p->cfg.colour_k; ++kappa) {
    HIPCHK(launch_count(p->v, MODE_CLASS, kappa, p->v.pc, p->stream));
    HIPCHK(launch_gauss_est(p->v, MODE_CLASS, p->v.pc, p->stream));
    HIPCHK(launch_gauss_delta(p->v, MODE_CLASS, kappa, p->v.pc, p->stream));
    HIPCHK(launch_delta(p->v, MODE_CLASS, kappa, p->v.pc, p->stream));
    HIPCHK(launch_commit(p->v, kappa, p->stream));
    HIPCHK(launch_gauss_commit(p->v, kappa, p->stream));
  }
  HIPCHK(launch_advance(p->v, p->stream));
  return BN_OK;
}

// The view of colour phase kappa reading proposals from sweep buffer set b.
DevView phase_view(bn_problem p, int b, uint32_t kappa) {
  DevView v = p->v;
  v.c_new = p->sets[b].cn + (size_t)kappa * v.pc * v.tp;
  v.u_new = p->sets[b].un + (size_t)kappa * v.pc;
  if (v.tgp) v.g_new = p->sets[b].gn + (size_t)kappa * v.pc * v.tgp;
  return v;
}

DevView sweep_view(bn_problem p, int b) {
  DevView v = p->v;
  v.c_new = p->sets[b].cn;
  v.u_new = p->sets[b].un;
  if (v.tgp) v.g_new = p->sets[b].gn;
  return v;
}

// The recount of the single-problem overlapped schedule reads its own sweep
// index, counter word 3, kept one past the sweep counter by the schedule:
// it then waits on the main stream only for the phases that last read its
// proposal set, not for the advance of the sweep counter.
DevView recount_view(bn_problem p, int b) {
  DevView v = sweep_view(p, b);
  v.ctr = p->v.ctr + 3;
  return v;
}

bn_status ensure_sweep_sets(bn_problem p) {
  if (p->sets_ready) return BN_OK;
  const size_t P = (size_t)p->v.w * p->v.h;
  bn_status s;
  for (int b = 0; b < 2; ++b) {
    if ((s = p->alloc(&p->sets[b].cn, P * p->v.tp)) != BN_OK) return s;
    if ((s = p->alloc(&p->sets[b].un, P)) != BN_OK) return s;
    if (p->v.tgp && (s = p->alloc(&p->sets[b].gn, P * p->v.tgp)) != BN_OK) return s;
  }
  HIPCHK(hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking));
  for (hipEvent_t& e : p->ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  p->sets_ready = true;
  return BN_OK;
}

// Proposals (offsets, recounts, Gaussian estimates) of every pixel for the
// sweep `ahead` steps after the device sweep counter, into buffer set b.
// Event pair recorded around a launch when profiling (eager mode only).
struct ProfMark {
  bn_problem p;
  std::vector<hipEvent_t>* vec;
  hipStream_t st;
  hipEvent_t stop = nullptr;
  bn_status s = BN_OK;
  ProfMark(bn_problem p_, std::vector<hipEvent_t>* v_, hipStream_t st_) : p(p_), vec(v_), st(st_) {
    if (!p->profiling) return;
    // timing-only events: no system-scope fence (cache write-back) when they
    // are recorded, so they disturb the work around them less
    hipEvent_t a, b;
    if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess || hipEventRecord(a, st) != hipSuccess) {
      s = fail(BN_EHIP, "profiling events");
      return;
    }
    vec->push_back(a);
    vec->push_back(b);
    stop = b;
  }
  bn_status end() {
    if (stop && hipEventRecord(stop, st) != hipSuccess) return fail(BN_EHIP, "profiling event record");
    return s;
  }
};

bn_status record_proposals(bn_problem p, int b, uint32_t ahead, hipStream_t st, bool own_index = false) {
  const DevView v = own_index ? recount_view(p, b) : sweep_view(p, b);
  const uint32_t P = v.w * v.h;
  ProfMark m(p, &p->prof_recount, st);
  HIPCHK(launch_count(v, MODE_SWEEP, ahead, P, st));
  bn_status s = m.end();
  if (s != BN_OK) return s;
  HIPCHK(launch_gauss_est(v, MODE_SWEEP, P, st));
  return BN_OK;
}

bn_status record_phases(bn_problem p, int b) {
  for (uint32_t kappa = 0; kappa < p->cfg.colour_k * p->cfg.colour_k; ++kappa) {
    const DevView v = phase_view(p, b, kappa);
    ProfMark me(p, &p->prof_eval, p->stream);
    HIPCHK(launch_gauss_delta(v, MODE_CLASS, kappa, v.pc, p->stream));
    HIPCHK(launch_delta(v, MODE_CLASS, kappa, v.pc, p->stream));
    bn_status s = me.end();
    if (s != BN_OK) return s;
    ProfMark mc(p, &p->prof_commit, p->stream);
    HIPCHK(launch_commit(v, kappa, p->stream));
    HIPCHK(launch_gauss_commit(v, kappa, p->stream));
    if ((s = mc.end()) != BN_OK) return s;
  }
  return BN_OK;
}

// Two sweeps with the recount of the next sweep overlapping the evaluation of
// the current one: [recount(s+1) -> set 1 || phases(s) from set 0], join,
// advance, [recount(s+2) -> set 0 || phases(s+1) from set 1], join, advance.
// The sweep counter only moves after a join, so every recount reads a stable
// index.  Set 0 holds the current sweep's proposals before and after.  (The
// batch's ungrouped members; a single problem chains its recounts, below.)
bn_status record_pair(bn_problem p) {
  bn_status s;
  for (int half = 0; half < 2; ++half) {
    const int cur = half, nxt = 1 - half;
    HIPCHK(hipEventRecord(p->ev[2 * half], p->stream));
    HIPCHK(hipStreamWaitEvent(p->aux, p->ev[2 * half], 0));
    if ((s = record_proposals(p, nxt, 1, p->aux)) != BN_OK) return s;
    HIPCHK(hipEventRecord(p->ev[2 * half + 1], p->aux));
    if ((s = record_phases(p, cur)) != BN_OK) return s;
    HIPCHK(hipStreamWaitEvent(p->stream, p->ev[2 * half + 1], 0));
    HIPCHK(launch_advance(p->v, p->stream));
  }
  return BN_OK;
}

// The single problem's two sweeps, chained: the same halves, but the
// recounts read the recount index, the second half's one past it (the index
// advances by two on the auxiliary stream after the pair's second recount),
// and each waits only for the phases that last read its set: those of the
// first half for the second recount; for the first, those of the previous
// pair's second half, or, at the start of a captured pair or of a call
// (`fork`), everything before on the main stream.  The phases of a sweep are
// done long before the recount beside them, so a recount does not wait for
// the join and advance after the previous one; the main stream still joins
// each recount before its advance.
bn_status record_pair_chained(bn_problem p, bool fork) {
  bn_status s;
  for (int half = 0; half < 2; ++half) {
    const int cur = half, nxt = 1 - half;
    if (half == 1) {
      HIPCHK(hipStreamWaitEvent(p->aux, p->ev[2], 0));
    } else if (fork) {
      HIPCHK(hipEventRecord(p->ev[0], p->stream));
      HIPCHK(hipStreamWaitEvent(p->aux, p->ev[0], 0));
    } else {
      HIPCHK(hipStreamWaitEvent(p->aux, p->ev[4], 0));
    }
    if ((s = record_proposals(p, nxt, (uint32_t)half, p->aux, true)) != BN_OK) return s;
    if (half == 1) HIPCHK(launch_recount_advance_pair(p->v, p->aux));
    HIPCHK(hipEventRecord(p->ev[2 * half + 1], p->aux));
    if ((s = record_phases(p, cur)) != BN_OK) return s;
    HIPCHK(hipEventRecord(p->ev[half == 0 ? 2 : 4], p->stream));
    HIPCHK(hipStreamWaitEvent(p->stream, p->ev[2 * half + 1], 0));
    HIPCHK(launch_advance(p->v, p->stream));
  }
  return BN_OK;
}

bn_status build_pair_graph(bn_problem p) {
  if (p->pair_exec || p->pair_failed) return BN_OK;
  HIPCHK(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
  bn_status s = record_pair_chained(p, true);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(p->stream, &g);
  if (s != BN_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p->pair_failed = true;
    return BN_OK;
  }
  e = hipGraphInstantiate(&p->pair_exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g);
    p->pair_exec = nullptr;
    p->pair_failed = true;
    return BN_OK;
  }
  p->pair_graph = g;
  return BN_OK;
}

// k sweeps through the overlapped path.
bn_status overlapped_sweeps(bn_problem p, uint32_t k) {
  bn_status s;
  if ((s = ensure_sweep_sets(p)) != BN_OK) return s;
  if (p->prefetched != p->sweep) {
    if ((s = record_proposals(p, 0, 0, p->stream)) != BN_OK) return s;
    p->prefetched = p->sweep;
  }
  if (k >= 2 && !p->profiling && (s = build_pair_graph(p)) != BN_OK) return s;
  // the recount index one past the sweep counter, which other calls may have
  // moved
  if (k >= 2) HIPCHK(launch_recount_index(p->v, p->stream));
  uint32_t done = 0;
  while (k - done >= 2) {
    if (p->pair_exec && !p->profiling) {
      HIPCHK(hipGraphLaunch(p->pair_exec, p->stream));
    } else if ((s = record_pair_chained(p, done == 0)) != BN_OK) {
      return s;
    }
    done += 2;
  }
  if (done < k) {
    // one more sweep, then the next sweep's proposals into set 0
    if ((s = record_phases(p, 0)) != BN_OK) return s;
    HIPCHK(launch_advance(p->v, p->stream));
    if ((s = record_proposals(p, 0, 0, p->stream)) != BN_OK) return s;
    done += 1;
  }
  p->prefetched = p->sweep + k;
  return BN_OK;
}

// ------------------------------------------------------------ swap mutation
// Pixel permutation of the swap passes: pixels sorted by the 64-bit keys
// (w0 << 32) | w1 of Philox((p, 0, problem, S_PERM)), ties by pixel index.
std::vector<uint32_t> swap_permutation(const bn_config& c) {
  const uint32_t P = c.width * c.height;
  std::vector<uint64_t> key(P);
  for (uint32_t q = 0; q < P; ++q) {
    uint32_t w[4] = {q, 0u, c.problem_id, S_PERM};
    philox10(w, (uint32_t)c.seed, (uint32_t)(c.seed >> 32));
    key[q] = ((uint64_t)w[0] << 32) | w[1];
  }
  std::vector<uint32_t> perm(P);
  for (uint32_t q = 0; q < P; ++q) perm[q] = q;
  std::stable_sort(perm.begin(), perm.end(), [&](uint32_t a, uint32_t b) { return key[a] < key[b]; });
  return perm;
}

bn_status setup_swap(bn_problem p) {
  const uint32_t P = p->v.w * p->v.h, M = P / (p->v.k * p->v.k);
  HIPCHK(prepare_swap_kernels());
  const std::vector<uint32_t> perm = swap_permutation(p->cfg);
  std::vector<uint32_t> pinv(P);
  for (uint32_t L = 0; L < P; ++L) pinv[perm[L]] = L;
  const uint32_t r = p->v.radius, dmax = 2 * r * r;
  std::vector<int32_t> dcls(dmax + 1, -1);
  for (size_t c = 0; c < p->cls_d.size(); ++c) dcls[p->cls_d[c]] = (int32_t)c;
  SwapView& sv = p->sv;
  uint32_t *perm_d, *pinv_d;
  int32_t* dcls_d;
  bn_status s;
  if ((s = p->alloc(&perm_d, P)) != BN_OK || (s = p->alloc(&pinv_d, P)) != BN_OK ||
      (s = p->alloc(&dcls_d, dmax + 1)) != BN_OK || (s = p->alloc(&sv.xs, (size_t)p->v.ncls * M)) != BN_OK ||
      (s = p->alloc(&sv.d2, M / 2)) != BN_OK || (s = p->alloc(&sv.row, (size_t)P * p->v.tp)) != BN_OK)
    return s;
  sv.perm = perm_d;
  sv.pinv = pinv_d;
  sv.dcls = dcls_d;
  sv.m = M;
  HIPCHK(hipMemcpyAsync(perm_d, perm.data(), (size_t)P * 4, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemcpyAsync(pinv_d, pinv.data(), (size_t)P * 4, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemcpyAsync(dcls_d, dcls.data(), dcls.size() * 4, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemsetAsync(sv.xs, 0, (size_t)p->v.ncls * M * 8, p->stream));
  HIPCHK(hipMemsetAsync(sv.d2, 0, (size_t)(M / 2) * 8, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return BN_OK;
}

// One swap pass: evaluate and decide every couple, then exchange.
bn_status swap_evaluate(bn_problem p, uint32_t kappa) {
  HIPCHK(launch_swap_evaluate(p->v, p->sv, kappa, p->stream));
  return BN_OK;
}

bn_status swap_commit(bn_problem p) {
  HIPCHK(launch_swap_commit(p->v, p->sv, p->stream));
  return BN_OK;
}

// A sweep's passes: the class sums of the couples (timed as the evaluation),
// then their decisions and exchanges in one launch (timed as the commit).
bn_status record_swap_sweep(bn_problem p) {
  bn_status s;
  for (uint32_t kappa = 0; kappa < p->v.k * p->v.k; ++kappa) {
    ProfMark me(p, &p->prof_eval, p->stream);
    HIPCHK(launch_swap_evaluate(p->v, p->sv, kappa, p->stream, false));
    if ((s = me.end()) != BN_OK) return s;
    ProfMark mc(p, &p->prof_commit, p->stream);
    HIPCHK(launch_swap_decide_exchange(p->v, p->sv, kappa, p->stream));
    if ((s = mc.end()) != BN_OK) return s;
  }
  HIPCHK(launch_advance(p->v, p->stream));
  return BN_OK;
}

bn_status build_swap_graph(bn_problem p) {
  if (p->swap_exec || p->swap_failed) return BN_OK;
  HIPCHK(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
  bn_status s = record_swap_sweep(p);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(p->stream, &g);
  if (s != BN_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p->swap_failed = true;
    return BN_OK;
  }
  e = hipGraphInstantiate(&p->swap_exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g);
    p->swap_exec = nullptr;
    p->swap_failed = true;
    return BN_OK;
  }
  p->swap_graph = g;
  return BN_OK;
}

// k swap sweeps of K^2 passes (graph-replayed unless profiling).
bn_status swap_sweeps(bn_problem p, uint32_t k) {
  if (!k) return BN_OK;
  bn_status s;
  if (!p->profiling && (s = build_swap_graph(p)) != BN_OK) return s;
  for (uint32_t i = 0; i < k; ++i) {
    if (p->swap_exec && !p->profiling) {
      HIPCHK(hipGraphLaunch(p->swap_exec, p->stream));
    } else if ((s = record_swap_sweep(p)) != BN_OK) {
      return s;
    }
  }
  return BN_OK;
}

bn_status build_graph(bn_problem p) {
  if (p->graph_exec || p->graph_failed) return BN_OK;
  if (p->stream == nullptr) {
    p->graph_failed = true;
    return BN_OK;
  }
  HIPCHK(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
  bn_status s = record_sweep(p);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(p->stream, &g);
  if (s != BN_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p->graph_failed = true;
    return BN_OK;
  }
  e = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g);
    p->graph_exec = nullptr;
    p->graph_failed = true;
    return BN_OK;
  }
  p->graph = g;
  return BN_OK;
}


// Candidates of the launch-shape tuner: integrands per counting wave and the
// workgroup target of the staged energy-change launch.
const uint32_t kTuneTch[] = {64, 128, 256, 512};
const uint32_t kTuneSlices[] = {128, 256, 512, 1024, 2048};
const uint32_t kTuneShapes[] = {0, 1};

bool tune_choice_valid(uint32_t tch, uint32_t slices, uint32_t shape) {
  return std::find(std::begin(kTuneTch), std::end(kTuneTch), tch) != std::end(kTuneTch) &&
         std::find(std::begin(kTuneSlices), std::end(kTuneSlices), slices) != std::end(kTuneSlices) &&
         std::find(std::begin(kTuneShapes), std::end(kTuneShapes), shape) != std::end(kTuneShapes);
}

// (Re)build the per-group device tables from the members' current launch
// choices and proposal sets.  Invalidates any captured graph.
bn_status batch_upload(bn_batch b) {
  if (b->graph_exec) {
    (void)hipGraphExecDestroy(b->graph_exec);
    b->graph_exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  if (!tune_choice_valid(b->tch, b->slice_target, b->shape))
    return fail(BN_EINVAL, "launch choice tch=%u slices=%u shape=%u is not one of the tuner's candidates", b->tch,
                b->slice_target, b->shape);
  HIPCHK(hipStreamSynchronize(b->stream));
  for (void* q : b->allocs) (void)hipFree(q);
  b->allocs.clear();
  for (bn_problem p : b->members) {
    p->v.tch = std::min<uint32_t>(b->tch, p->v.tp);
    p->v.slice_target = b->slice_target;
  }
  const uint32_t K2 = b->colour_k * b->colour_k;
  auto dev_copy = [&](const void* src, size_t bytes, void** dst) -> bn_status {
    void* d = nullptr;
    if (hipMalloc(&d, std::max<size_t>(bytes, 4)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(BN_ENOMEM, "batch tables");
    }
    b->allocs.push_back(d);
    *dst = d;
    if (bytes) HIPCHK(hipMemcpy(d, src, bytes, hipMemcpyHostToDevice));
    return BN_OK;
  };
  // kind 0: whole-sweep counting views per set; kind 1: phase views per (set, class)
  auto upload = [&](BatchGroup& g, int kind, auto blocks_of, bool geo) -> bn_status {
    g.blocks = 0;
    g.views.clear();
    if (g.idx.empty()) return BN_OK;
    std::vector<uint32_t> pre(1, 0), gv;
    for (uint32_t i : g.idx) {
      const DevView& v = b->members[i]->v;
      if (geo) {
        uint32_t gx = 0, gy = 0, gz = 0, trl = 0;
        stage_geometry(v, b->shape, &gx, &gy, &gz, &trl);
        gv.push_back(gx);
        gv.push_back(gy);
        gv.push_back(trl);
        pre.push_back(pre.back() + gx * gy * gz);
      } else {
        pre.push_back(pre.back() + blocks_of(v));
      }
    }
    g.blocks = pre.back();
    bn_status st;
    if ((st = dev_copy(pre.data(), pre.size() * 4, (void**)&g.d_pre)) != BN_OK) return st;
    if ((st = dev_copy(gv.data(), gv.size() * 4, (void**)&g.d_geo)) != BN_OK) return st;
    const uint32_t ntab = kind == 0 ? 2 : 2 * K2;
    for (uint32_t tab = 0; tab < ntab; ++tab) {
      std::vector<DevView> views;
      for (uint32_t i : g.idx) {
        bn_problem p = b->members[i];
        views.push_back(kind == 0 ? sweep_view(p, (int)tab) : phase_view(p, (int)(tab / K2), tab % K2));
      }
      DevView* d = nullptr;
      if ((st = dev_copy(views.data(), views.size() * sizeof(DevView), (void**)&d)) != BN_OK) return st;
      g.views.push_back(d);
    }
    return BN_OK;
  };
  bn_status s;
  for (BatchGroup& g : b->count_groups)
    if ((s = upload(g, 0, [](const DevView& v) { return count_blocks(v, true); }, false)) != BN_OK) return s;
  for (BatchGroup& g : b->stage_groups)
    if ((s = upload(g, 1, [](const DevView&) { return 0u; }, true)) != BN_OK) return s;
  if ((s = upload(b->finish_all, 1, [](const DevView& v) { return (v.pc + 255) / 256; }, false)) != BN_OK) return s;
  if ((s = upload(b->commit_all, 1, [](const DevView& v) { return commit_blocks(v); }, false)) != BN_OK) return s;
  return BN_OK;
}

// Sweep-wide recount of every grouped member, `ahead` sweeps past its
// counter, into proposal set `set`, on stream st.
bn_status batch_recount(bn_batch b, int set, uint32_t ahead, hipStream_t st) {
  for (BatchGroup& g : b->count_groups)
    HIPCHK(launch_count_batch(g.kind, g.views[set], g.d_pre, (uint32_t)g.idx.size(), g.blocks, ahead, true, st));
  return BN_OK;
}

// Energy change and decision of colour class kappa for every grouped member,
// proposals from set `set` (no state change).
bn_status batch_evaluate(bn_batch b, int set, uint32_t kappa) {
  if (b->finish_all.idx.empty()) return BN_OK;   // no grouped members
  const uint32_t t = set * b->colour_k * b->colour_k + kappa;
  for (BatchGroup& g : b->stage_groups)
    HIPCHK(launch_stage_batch(g.radius, g.k, b->shape, g.views[t], g.d_pre, g.d_geo, (uint32_t)g.idx.size(), g.blocks,
                              kappa, b->stream));
  HIPCHK(launch_finish_batch(b->finish_all.views[t], b->finish_all.d_pre, (uint32_t)b->finish_all.idx.size(),
                             b->finish_all.blocks, b->stream));
  return BN_OK;
}

bn_status batch_phases(bn_batch b, int set) {
  bn_status s;
  for (uint32_t kappa = 0; kappa < b->colour_k * b->colour_k; ++kappa) {
    if ((s = batch_evaluate(b, set, kappa)) != BN_OK) return s;
    const uint32_t t = set * b->colour_k * b->colour_k + kappa;
    HIPCHK(launch_commit_batch(b->commit_all.views[t], b->commit_all.d_pre, (uint32_t)b->commit_all.idx.size(),
                               b->commit_all.blocks, kappa, b->stream));
  }
  return BN_OK;
}

bool batch_has_groups(bn_batch b) { return !b->commit_all.idx.empty(); }

// Proposals of every redraw member's current sweep into set 0 where they are
// not there yet (stream-ordered on the batch stream).
bn_status batch_prefetch(bn_batch b) {
  bn_status s;
  bool group_stale = false;
  for (uint32_t i : b->commit_all.idx) group_stale = group_stale || b->members[i]->prefetched != b->members[i]->sweep;
  if (group_stale && (s = batch_recount(b, 0, 0, b->stream)) != BN_OK) return s;
  for (uint32_t i : b->commit_all.idx) b->members[i]->prefetched = b->members[i]->sweep;
  for (uint32_t i : b->solo) {
    bn_problem p = b->members[i];
    if (p->cfg.move == BN_SWAP || p->prefetched == p->sweep) continue;
    if ((s = record_proposals(p, 0, 0, p->stream)) != BN_OK) return s;
    p->prefetched = p->sweep;
  }
  return BN_OK;
}

// Two sweeps of every member: the grouped members' overlapped halves
// [recount(s+1) -> set 1 || phases(s) from set 0], join, advance, then the
// same with the sets exchanged; each solo member's own overlapped pair (or two
// swap sweeps).  Set 0 holds every redraw member's current proposals before
// and after.
bn_status batch_record_pair(bn_batch b) {
  bn_status s;
  if (batch_has_groups(b)) {
    for (int half = 0; half < 2; ++half) {
      const int cur = half, nxt = 1 - half;
      HIPCHK(hipEventRecord(b->ev[2 * half], b->stream));
      HIPCHK(hipStreamWaitEvent(b->aux, b->ev[2 * half], 0));
      if ((s = batch_recount(b, nxt, 1, b->aux)) != BN_OK) return s;
      HIPCHK(hipEventRecord(b->ev[2 * half + 1], b->aux));
      if ((s = batch_phases(b, cur)) != BN_OK) return s;
      HIPCHK(hipStreamWaitEvent(b->stream, b->ev[2 * half + 1], 0));
      HIPCHK(launch_advance_batch(b->commit_all.views[0], (uint32_t)b->commit_all.idx.size(), b->stream));
    }
  }
  for (uint32_t i : b->solo) {
    bn_problem p = b->members[i];
    if (p->cfg.move == BN_SWAP) {
      if ((s = record_swap_sweep(p)) != BN_OK || (s = record_swap_sweep(p)) != BN_OK) return s;
    } else if ((s = record_pair(p)) != BN_OK) {
      return s;
    }
  }
  return BN_OK;
}

// One sweep of every member outside the pair graph, leaving the next sweep's
// proposals in set 0.
bn_status batch_single_sweep(bn_batch b) {
  bn_status s;
  if (batch_has_groups(b)) {
    if ((s = batch_phases(b, 0)) != BN_OK) return s;
    HIPCHK(launch_advance_batch(b->commit_all.views[0], (uint32_t)b->commit_all.idx.size(), b->stream));
    if ((s = batch_recount(b, 0, 0, b->stream)) != BN_OK) return s;
  }
  for (uint32_t i : b->solo) {
    bn_problem p = b->members[i];
    if (p->cfg.move == BN_SWAP) {
      if ((s = record_swap_sweep(p)) != BN_OK) return s;
    } else {
      if ((s = record_phases(p, 0)) != BN_OK) return s;
      HIPCHK(launch_advance(p->v, p->stream));
      if ((s = record_proposals(p, 0, 0, p->stream)) != BN_OK) return s;
    }
  }
  return BN_OK;
}

std::string batch_key(bn_batch b) {
  std::string key = "K" + std::to_string(b->colour_k);
  for (bn_problem p : b->members) {
    const DevView& v = p->v;
    key += ":n" + std::to_string(v.n) + "w" + std::to_string(v.w) + "h" + std::to_string(v.h) + "t" +
           std::to_string(v.t) + "r" + std::to_string(v.radius);
  }
  return key;
}

// Work the tuner times for one candidate: the grouped members' sweep-wide
// recount into set 1 (scratch until the next sweep writes it) and K^2
// evaluations of colour class 0 from set 0 (decisions only, no commit), so
// the optimisation state is untouched.
bn_status batch_tune_step(bn_batch b) {
  bn_status s = batch_recount(b, 1, 1, b->stream);
  for (uint32_t k = 0; k < b->colour_k * b->colour_k && s == BN_OK; ++k) s = batch_evaluate(b, 0, 0);
  return s;
}

// Launch-shape tuner: times batch_tune_step for every candidate (integrands
// per counting wave, workgroup target and block shape of the staged energy
// change) and keeps the fastest.  Results do not depend on the choice.
bn_status batch_tune(bn_batch b) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best = 1e30f;
  uint32_t bt = b->tch, bs = b->slice_target, bh = b->shape;
  bn_status s = BN_OK;
  for (uint32_t sh : kTuneShapes) {
    for (uint32_t tc : kTuneTch) {
      for (uint32_t sl : kTuneSlices) {
        b->tch = tc;
        b->slice_target = sl;
        b->shape = sh;
        if ((s = batch_upload(b)) != BN_OK) break;
        if ((s = batch_tune_step(b)) != BN_OK) break;   // warm-up
        if (hipEventRecord(e0, b->stream) != hipSuccess) { s = fail(BN_EHIP, "event record"); break; }
        if ((s = batch_tune_step(b)) != BN_OK) break;
        if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          s = fail(BN_EHIP, "event timing");
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
          best = ms;
          bt = tc;
          bs = sl;
          bh = sh;
        }
      }
      if (s != BN_OK) break;
    }
    if (s != BN_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != BN_OK) return s;
  b->tch = bt;
  b->slice_target = bs;
  b->shape = bh;
  return batch_upload(b);
}

}  // namespace

extern "C" {

const char* bn_status_string(bn_status s) {
  switch (s) {
    case BN_OK: return "ok";
    case BN_EINVAL: return "invalid argument";
    case BN_ENOMEM: return "out of memory";
    case BN_EHIP: return "HIP runtime error";
    case BN_ESTATE: return "call out of order";
    case BN_EUNSUPPORTED: return "unsupported";
    case BN_ENUMERIC: return "numeric error";
  }
  return "unknown status";
}

const char* bn_last_error(void) { return g_last_error.c_str(); }

bn_status bn_validate_config(const bn_config* cfg) { return validate(cfg); }

bn_status bn_window_classes(const bn_config* cfg, uint32_t* n_classes, uint32_t* class_d, double* class_w) {
  bn_status s = validate(cfg);
  if (s != BN_OK) return s;
  if (!n_classes) return fail(BN_EINVAL, "n_classes is NULL");
  std::vector<uint32_t> d;
  std::vector<double> w;
  window_classes(cfg->radius, cfg->sigma, d, w);
  if ((class_d || class_w) && *n_classes < d.size())
    return fail(BN_EINVAL, "arrays hold %u entries, %zu needed", *n_classes, d.size());
  *n_classes = (uint32_t)d.size();
  for (size_t i = 0; i < d.size(); ++i) {
    if (class_d) class_d[i] = d[i];
    if (class_w) class_w[i] = w[i];
  }
  return BN_OK;
}

bn_status bn_swap_permutation(const bn_config* cfg, uint32_t* out) {
  bn_status s = validate(cfg);
  if (s != BN_OK) return s;
  if (!out) return fail(BN_EINVAL, "out is NULL");
  if (!is_pow2(cfg->width * cfg->height)) return fail(BN_EINVAL, "W*H must be a power of two");
  const std::vector<uint32_t> perm = swap_permutation(*cfg);
  std::copy(perm.begin(), perm.end(), out);
  return BN_OK;
}

bn_status bn_heaviside_area(const bn_heaviside* h, double* out) {
  if (!h || !out) return fail(BN_EINVAL, "NULL argument");
  return heaviside_area_checked(*h, out);
}

bn_status bn_draw_heavisides(uint64_t seed, uint32_t problem_id, uint32_t t, bn_heaviside* out) {
  if (!out && t) return fail(BN_EINVAL, "out is NULL");
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (uint32_t i = 0; i < t; ++i) {
    uint32_t c[4] = {i, 0u, problem_id, S_INTEG};
    philox10(c, k0, k1);
    const double theta = 2.0 * M_PI * (double)c[0] * 0x1p-32;
    out[i].nx = (int16_t)std::nearbyint(16384.0 * std::cos(theta));
    out[i].ny = (int16_t)std::nearbyint(16384.0 * std::sin(theta));
    out[i].cx = (uint16_t)(c[1] >> 16);
    out[i].cy = (uint16_t)(c[2] >> 16);
  }
  return BN_OK;
}

bn_status bn_draw_gaussians(uint64_t seed, uint32_t problem_id, uint32_t t, bn_gaussian* out) {
  if (!out && t) return fail(BN_EINVAL, "out is NULL");
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (uint32_t i = 0; i < t; ++i) {
    uint32_t c[4] = {i, 1u, problem_id, S_INTEG};
    philox10(c, k0, k1);
    out[i].mx = (double)c[0] * 0x1p-32;
    out[i].my = (double)c[1] * 0x1p-32;
    out[i].s = 0.05 + 0.25 * ((double)c[2] * 0x1p-32);
  }
  return BN_OK;
}

bn_status bn_gaussian_integral(const bn_gaussian* g, double* out) {
  if (!g || !out) return fail(BN_EINVAL, "NULL argument");
  return gaussian_checked(*g, out);
}

bn_status bn_create_problem(const bn_config* cfg, const bn_heaviside* heavisides, const bn_gaussian* gaussians,
                            void* stream, bn_problem* out) {
  return bn_create_problem_ext(cfg, heavisides, gaussians, stream, nullptr, out);
}

bn_status bn_create_problem_ext(const bn_config* cfg, const bn_heaviside* heavisides, const bn_gaussian* gaussians,
                                void* stream, const bn_device_buffers* bufs, bn_problem* out) {
  bn_status s = validate(cfg);
  if (s != BN_OK) return s;
  if (!out) return fail(BN_EINVAL, "out is NULL");
  if ((s = supported(cfg)) != BN_OK) return s;
  *out = nullptr;
  if (bufs)
    for (const void* b : {bufs->offsets, bufs->counts, bufs->errors})
      if ((uintptr_t)b % 256) return fail(BN_EINVAL, "caller-owned device buffers must be 256-byte aligned");

  // Host tables first: every input is checked before the device is touched.
  std::vector<bn_heaviside> heav(cfg->t_heaviside);
  if (heavisides)
    std::copy(heavisides, heavisides + cfg->t_heaviside, heav.begin());
  else if ((s = bn_draw_heavisides(cfg->seed, cfg->problem_id, cfg->t_heaviside, heav.data())) != BN_OK)
    return s;
  std::vector<double> area(cfg->t_heaviside);
  for (uint32_t t = 0; t < cfg->t_heaviside; ++t)
    if ((s = heaviside_area_checked(heav[t], &area[t])) != BN_OK)
      return fail(s, "integrand %u: %s", t, g_last_error.c_str());
  std::vector<bn_gaussian> gauss(cfg->t_gauss);
  if (gaussians)
    std::copy(gaussians, gaussians + cfg->t_gauss, gauss.begin());
  else if ((s = bn_draw_gaussians(cfg->seed, cfg->problem_id, cfg->t_gauss, gauss.data())) != BN_OK)
    return s;
  std::vector<double> gint(cfg->t_gauss);
  for (uint32_t t = 0; t < cfg->t_gauss; ++t)
    if ((s = gaussian_checked(gauss[t], &gint[t])) != BN_OK)
      return fail(s, "Gaussian %u: %s", t, g_last_error.c_str());

  if ((s = check_device()) != BN_OK) return s;

  bn_problem p = new bn_problem_s();
  p->cfg = *cfg;
  if (hipGetDevice(&p->device) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return fail(BN_EHIP, "hipGetDevice failed");
  }
  p->heav = heav;
  p->area64 = area;
  p->gauss = gauss;
  p->gint64 = gint;
  window_classes(cfg->radius, cfg->sigma, p->cls_d, p->cls_w);
  if (stream) {
    p->stream = (hipStream_t)stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete p;
      return fail(BN_EHIP, "hipStreamCreateWithFlags: %s", hipGetErrorString(e));
    }
    p->own_stream = true;
  }

  DevView& v = p->v;
  v.n = cfg->n;
  v.log2n = 0;
  while ((1u << v.log2n) < cfg->n) ++v.log2n;
  v.w = cfg->width;
  v.h = cfg->height;
  v.t = cfg->t_heaviside;
  v.tp = round_up(v.t, T_ALIGN);
  v.k = cfg->colour_k;
  v.tch = 0;
  v.cw = cfg->width / cfg->colour_k;
  v.ch = cfg->height / cfg->colour_k;
  v.pc = v.cw * v.ch;
  v.problem = cfg->problem_id;
  v.seed_lo = (uint32_t)cfg->seed;
  v.seed_hi = (uint32_t)(cfg->seed >> 32);
  v.objective = cfg->objective;
  v.radius = cfg->radius;
  v.ncls = (uint32_t)p->cls_d.size();
  v.tch = std::min<uint32_t>(1024, v.tp);   // integrands per counting wave (fewer for small launches)
  v.slice_target = 512;
  // The colour phases share the CUs with the sweep-wide recount, which keeps
  // the vector ALU busy with two waves per SIMD. With the phase kernels at
  // raised wave priority, a cap of four workgroups per CU gave the fastest
  // event-timed sweeps at 256^2, N = 256, T = 1024 in both forms (FP32: 2.5 %
  // faster than two per CU; BF16: 6 % faster than one per CU).
  v.count_cap = 0;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      v.count_cap = 4u * (uint32_t)cus;
  }
  v.tg = cfg->t_gauss;
  v.tgp = round_up(v.tg, 64);
  v.tb = v.tp + v.tgp;
  // BF16 form: exact counts on the matrix cores where they are exact in BF16
  // (N <= 256, Heaviside rows only), else rounded error vectors
  v.mfma = cfg->precision != BN_BF16 ? 0u : (v.n <= 256 && v.tg == 0 ? 1u : 2u);
  v.xscale = v.mfma == 2 ? 0x1p-39 : 2.0 / ((double)v.n * (double)v.n);
  v.bf = nullptr;
  v.delta_bf = nullptr;
  const size_t P = (size_t)v.w * v.h;

  std::vector<uint32_t> lat(v.n);
  const uint32_t step = 65536u / v.n;
  for (uint32_t i = 0; i < v.n; ++i) {
    const uint32_t jx = (uint32_t)(((uint64_t)i * cfg->g[0]) % v.n);
    const uint32_t jy = (uint32_t)(((uint64_t)i * cfg->g[1]) % v.n);
    lat[i] = ((jx * step) & 0xFFFFu) | (((jy * step) & 0xFFFFu) << 16);
  }
  std::vector<int2> ihp(v.tp, make_int2(0, 0));
  std::vector<float> areaf(v.tp, 0.0f);
  for (uint32_t t = 0; t < v.t; ++t) {
    const bn_heaviside& h = heav[t];
    ihp[t].x = (int)(((uint32_t)(uint16_t)h.nx) | ((uint32_t)(uint16_t)h.ny << 16));
    ihp[t].y = (int)h.nx * ((int)h.cx - 32768) + (int)h.ny * ((int)h.cy - 32768);
    areaf[t] = (float)area[t];
  }

  uint32_t* lat_d;
  int2* ihp_d;
  float* area_d;
  double* wd_d;
  if ((s = p->alloc(&lat_d, v.n)) != BN_OK || (s = p->alloc(&ihp_d, v.tp)) != BN_OK ||
      (s = p->alloc(&area_d, v.tp)) != BN_OK || (s = p->alloc(&wd_d, v.ncls)) != BN_OK ||
      (s = p->adopt(&v.U, bufs ? bufs->offsets : nullptr, P)) != BN_OK ||
      (s = p->adopt(&v.cnt, bufs ? bufs->counts : nullptr, P * v.tp)) != BN_OK ||
      (s = p->adopt(&v.err, bufs ? bufs->errors : nullptr, P * v.tp)) != BN_OK || (s = p->alloc(&v.u_new, v.pc)) != BN_OK ||
      (s = p->alloc(&v.c_new, (size_t)v.pc * v.tp)) != BN_OK || (s = p->alloc(&v.delta, v.pc)) != BN_OK ||
      (s = p->alloc(&v.accept, v.pc)) != BN_OK || (s = p->alloc(&v.ctr, 4)) != BN_OK ||
      (s = p->alloc(&v.unsure, v.pc)) != BN_OK ||
      (s = p->alloc(&p->ysum, v.ncls)) != BN_OK || (s = p->alloc(&v.xpart, xpart_words(v))) != BN_OK) {
    delete p;
    return s;
  }
  v.lat = lat_d;
  v.ihp = ihp_d;
  v.area = area_d;
  v.wd = wd_d;
  // Gaussian t as exponent coefficients (base 2): with g = log2(e) / (2 s^2),
  // -g |x - mu|^2 = a |x|^2 + bx x + by y + c, a = -g, (bx, by) = 2 g mu,
  // c = -g |mu|^2.  Padding rows are all zero (estimate 1, integral 0).
  std::vector<double> gcoef((size_t)v.tgp * 4, 0.0), gintp(v.tgp, 0.0);
  for (uint32_t t = 0; t < v.tg; ++t) {
    const double g = M_LOG2E / (2.0 * gauss[t].s * gauss[t].s);
    gcoef[4 * t] = -g;
    gcoef[4 * t + 1] = 2.0 * g * gauss[t].mx;
    gcoef[4 * t + 2] = 2.0 * g * gauss[t].my;
    gcoef[4 * t + 3] = -g * (gauss[t].mx * gauss[t].mx + gauss[t].my * gauss[t].my);
    gintp[t] = gint[t];
  }
  if (v.tgp) {
    double *gcoef_d, *gint_d;
    if ((s = p->alloc(&gcoef_d, (size_t)v.tgp * 4)) != BN_OK || (s = p->alloc(&gint_d, v.tgp)) != BN_OK ||
        (s = p->alloc(&v.gest, P * v.tgp)) != BN_OK || (s = p->alloc(&v.gerr, P * v.tgp)) != BN_OK ||
        (s = p->alloc(&v.g_new, (size_t)v.pc * v.tgp)) != BN_OK || (s = p->alloc(&v.gdelta, v.pc)) != BN_OK ||
        (s = p->alloc(&p->gsum, v.ncls)) != BN_OK) {
      delete p;
      return s;
    }
    v.gcoef = gcoef_d;
    v.gint = gint_d;
    hipError_t ge = hipMemcpyAsync(gcoef_d, gcoef.data(), (size_t)v.tgp * 32, hipMemcpyHostToDevice, p->stream);
    if (ge == hipSuccess) ge = hipMemcpyAsync(gint_d, gintp.data(), v.tgp * 8, hipMemcpyHostToDevice, p->stream);
    if (ge != hipSuccess) {
      delete p;
      return fail(BN_EHIP, "uploading Gaussian tables: %s", hipGetErrorString(ge));
    }
  }
  v.pix_list = nullptr;
  const unsigned long long zero[4] = {0ull, 0ull, 0ull, 0ull};
  if (v.mfma && ((s = p->alloc(&v.bf, P * v.tb)) != BN_OK || (s = p->alloc(&v.delta_bf, v.pc)) != BN_OK)) {
    delete p;
    return s;
  }
  hipError_t e = v.mfma ? prepare_bf_kernels(v.radius, v.k) : hipSuccess;
  if (e == hipSuccess) e = hipMemcpyAsync(lat_d, lat.data(), v.n * 4, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(ihp_d, ihp.data(), v.tp * 8, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(area_d, areaf.data(), v.tp * 4, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(wd_d, p->cls_w.data(), v.ncls * 8, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(v.ctr, zero, sizeof zero, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(v.xpart, 0, (size_t)xpart_words(v) * 8, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(v.unsure, 0, (size_t)v.pc * 4, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) {
    delete p;
    return fail(BN_EHIP, "uploading tables: %s", hipGetErrorString(e));
  }
  if (cfg->move == BN_SWAP && (s = setup_swap(p)) != BN_OK) {
    delete p;
    return s;
  }
  log_msg("created problem %p: %ux%u, N=%u, T=%u+%u, r=%u, K=%u, %s, %s, %zu device buffers", (void*)p,
          cfg->width, cfg->height, cfg->n, cfg->t_heaviside, cfg->t_gauss, cfg->radius, cfg->colour_k,
          cfg->precision == BN_BF16 ? (v.mfma == 1 ? "BF16 (exact counts)" : "BF16 (rounded errors)") : "FP32",
          cfg->move == BN_SWAP ? "swap" : "redraw", p->allocs.size());
  *out = p;
  return BN_OK;
}

bn_status bn_destroy_problem(bn_problem p) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  log_msg("destroyed problem %p", (void*)p);
  delete p;
  return BN_OK;
}

bn_status bn_init_offsets(bn_problem p, const uint16_t* host_u) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  const size_t P = (size_t)p->v.w * p->v.h;
  if (host_u) {
    HIPCHK(hipMemcpyAsync(p->v.U, host_u, P * 4, hipMemcpyHostToDevice, p->stream));
    bn_status s = sync(p);  // the caller may reuse host_u as soon as we return
    if (s != BN_OK) return s;
  } else {
    HIPCHK(launch_init_offsets(p->v, p->stream));
  }
  p->have_offsets = true;
  p->have_counts = false;
  return BN_OK;
}

bn_status bn_compute_errors(bn_problem p) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  if (!p->have_offsets) return fail(BN_ESTATE, "offsets are not initialised");
  HIPCHK(launch_count(p->v, MODE_ALL, 0, p->v.w * p->v.h, p->stream));
  if (p->cfg.move == BN_SWAP) HIPCHK(launch_swap_rows(p->v, p->sv, p->stream));
  HIPCHK(launch_gauss_est(p->v, MODE_ALL, p->v.w * p->v.h, p->stream));
  HIPCHK(launch_gauss_errors(p->v, p->stream));
  HIPCHK(launch_bf_field(p->v, p->stream));
  p->have_counts = true;
  p->errors_valid = true;
  return BN_OK;
}

bn_status bn_sweep(bn_problem p, uint32_t k, bn_sweep_stats* stats) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  if (!p->have_counts) return fail(BN_ESTATE, "bn_compute_errors must run before bn_sweep");
  unsigned long long before[3] = {0, 0, 0}, after[3] = {0, 0, 0};
  if (stats) {
    HIPCHK(hipMemcpyAsync(before, p->v.ctr, sizeof before, hipMemcpyDeviceToHost, p->stream));
    bn_status s = sync(p);
    if (s != BN_OK) return s;
  }
  bn_status s = p->cfg.move == BN_SWAP ? swap_sweeps(p, k) : overlapped_sweeps(p, k);
  if (s != BN_OK) return s;
  p->sweep += k;
  if (k) p->errors_valid = false;
  if (stats) {
    HIPCHK(hipMemcpyAsync(after, p->v.ctr, sizeof after, hipMemcpyDeviceToHost, p->stream));
    if ((s = sync(p)) != BN_OK) return s;
    // redraw: one proposal per pixel; swap: one per couple
    stats->proposals = (uint64_t)k * p->v.w * p->v.h / (p->cfg.move == BN_SWAP ? 2 : 1);
    stats->accepts = after[1] - before[1];
    stats->bf16_vetoes = after[2] - before[2];
    stats->sweep_index = after[0];
  }
  return BN_OK;
}

bn_status bn_energy(bn_problem p, double* out) {
  if (!p || !out) return fail(BN_EINVAL, "NULL argument");
  if (!p->have_counts) return fail(BN_ESTATE, "bn_compute_errors must run first");
  HIPCHK(hipMemsetAsync(p->ysum, 0, p->v.ncls * sizeof(unsigned long long), p->stream));
  HIPCHK(launch_energy(p->v, p->ysum, p->stream));
  std::vector<unsigned long long> y(p->v.ncls);
  HIPCHK(hipMemcpyAsync(y.data(), p->ysum, y.size() * 8, hipMemcpyDeviceToHost, p->stream));
  bn_status s = sync(p);
  if (s != BN_OK) return s;
  // The kernel sums half of the window; the mirrored half has the same total.
  double acc = 0.0;
  for (uint32_t c = 0; c < p->v.ncls; ++c) acc = acc + p->cls_w[c] * (double)(long long)(2 * y[c]);
  *out = acc / ((double)p->v.n * (double)p->v.n);
  if (p->v.tgp) {
    std::vector<double> g(p->v.ncls);
    HIPCHK(hipMemsetAsync(p->gsum, 0, p->v.ncls * sizeof(double), p->stream));
    HIPCHK(launch_gauss_energy(p->v, p->gsum, p->stream));
    HIPCHK(hipMemcpyAsync(g.data(), p->gsum, g.size() * 8, hipMemcpyDeviceToHost, p->stream));
    if ((s = sync(p)) != BN_OK) return s;
    double ga = 0.0;
    for (uint32_t c = 0; c < p->v.ncls; ++c) ga = ga + p->cls_w[c] * (2.0 * g[c]);
    *out = *out + ga;
  }
  if (!std::isfinite(*out)) return fail(BN_ENUMERIC, "energy is not finite");
  return BN_OK;
}

bn_status bn_energy_bf16(bn_problem p, double* out) {
  if (!p || !out) return fail(BN_EINVAL, "NULL argument");
  if (!p->have_counts) return fail(BN_ESTATE, "bn_compute_errors must run first");
  if (!p->v.mfma) return fail(BN_ESTATE, "the problem is not in the BF16 form");
  double* acc = (double*)p->ysum;   // the energy's class-sum buffer, 8 bytes per class
  HIPCHK(hipMemsetAsync(acc, 0, p->v.ncls * sizeof(double), p->stream));
  HIPCHK(launch_energy_bf16(p->v, acc, p->stream));
  std::vector<double> y(p->v.ncls);
  HIPCHK(hipMemcpyAsync(y.data(), acc, y.size() * 8, hipMemcpyDeviceToHost, p->stream));
  bn_status s = sync(p);
  if (s != BN_OK) return s;
  // half window summed on the device; the mirrored half has the same total
  double e = 0.0;
  for (uint32_t c = 0; c < p->v.ncls; ++c) e = e + p->cls_w[c] * (2.0 * y[c]);
  if (p->v.mfma == 1) e = e / ((double)p->v.n * (double)p->v.n);
  *out = e;
  if (!std::isfinite(*out)) return fail(BN_ENUMERIC, "energy is not finite");
  return BN_OK;
}

bn_status bn_get_phase_bf16(bn_problem p, double* delta_bf16) {
  if (!p || !delta_bf16) return fail(BN_EINVAL, "NULL argument");
  if (!p->v.mfma) return fail(BN_ESTATE, "the problem is not in the BF16 form");
  if (p->cfg.move == BN_SWAP) return fail(BN_ESTATE, "swap passes have no BF16 form");
  HIPCHK(hipMemcpyAsync(delta_bf16, p->v.delta_bf, (size_t)p->v.pc * 8, hipMemcpyDeviceToHost, p->stream));
  return sync(p);
}

bn_status bn_quality_metric(bn_problem p, const double* sigmas, uint32_t n, double* out) {
  return bn_quality_metric_family(p, BN_ROWS_ALL, sigmas, n, out);
}

bn_status bn_quality_metric_family(bn_problem p, bn_rows rows, const double* sigmas, uint32_t n, double* out) {
  if (!p || (n && (!sigmas || !out))) return fail(BN_EINVAL, "NULL argument");
  if (rows != BN_ROWS_ALL && rows != BN_ROWS_HEAVISIDE && rows != BN_ROWS_GAUSSIAN)
    return fail(BN_EINVAL, "unknown row family");
  if (rows == BN_ROWS_GAUSSIAN && !p->v.tg) return fail(BN_EINVAL, "the problem has no Gaussian integrands");
  if (n > 64) return fail(BN_EINVAL, "at most 64 blur sizes");
  if (!p->have_counts) return fail(BN_ESTATE, "bn_compute_errors must run first");
  for (uint32_t i = 0; i < n; ++i)
    if (!(sigmas[i] > 0.0) || !std::isfinite(sigmas[i])) return fail(BN_EINVAL, "blur sizes must be > 0");
  {
    bn_status rs = refresh_errors(p);
    if (rs != BN_OK) return rs;
  }
  const size_t P = (size_t)p->v.w * p->v.h;
  const uint32_t pitch_max = std::max(p->v.tp, p->v.tgp);
  const uint32_t nparts = blur_partials(p->v, pitch_max);
  float *tmp = nullptr, *kx = nullptr, *ky = nullptr;
  int32_t *dx = nullptr, *dy = nullptr;
  double* part = nullptr;
  // Scratch for the blur lives for the duration of the call only.
  auto release = [&]() {
    for (void* q : {(void*)tmp, (void*)kx, (void*)ky, (void*)dx, (void*)dy, (void*)part})
      if (q) (void)hipFree(q);
  };
  hipError_t e = hipMalloc((void**)&tmp, P * pitch_max * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&kx, p->v.w * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&ky, p->v.h * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&dx, p->v.w * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&dy, p->v.h * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&part, (size_t)nparts * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(BN_ENOMEM, "quality metric scratch: %s", hipGetErrorString(e));
  }
  std::vector<double> hp(nparts);
  for (uint32_t i = 0; i < n; ++i) {
    std::vector<float> hkx, hky;
    std::vector<int32_t> hdx, hdy;
    blur_taps(p->v.w, sigmas[i], hkx, hdx);
    blur_taps(p->v.h, sigmas[i], hky, hdy);
    e = hipMemcpyAsync(kx, hkx.data(), hkx.size() * 4, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dx, hdx.data(), hdx.size() * 4, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ky, hky.data(), hky.size() * 4, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dy, hdy.data(), hdy.size() * 4, hipMemcpyHostToDevice, p->stream);
    double acc = 0.0;
    const float* fields[2] = {p->v.err, p->v.gerr};
    const uint32_t pitches[2] = {p->v.tp, p->v.tgp}, valids[2] = {p->v.t, p->v.tg};
    for (int f = 0; f < 2 && e == hipSuccess; ++f) {
      if (!pitches[f] || (rows == BN_ROWS_HEAVISIDE && f == 1) || (rows == BN_ROWS_GAUSSIAN && f == 0)) continue;
      uint32_t np = 0;
      e = launch_blur(p->v, fields[f], pitches[f], valids[f], kx, (uint32_t)hkx.size(), dx, ky,
                      (uint32_t)hky.size(), dy, tmp, part, &np, p->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), part, (size_t)np * 8, hipMemcpyDeviceToHost, p->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
      for (uint32_t b = 0; b < np && e == hipSuccess; ++b) acc += hp[b];
    }
    if (e != hipSuccess) {
      release();
      return fail(BN_EHIP, "quality metric: %s", hipGetErrorString(e));
    }
    const uint32_t count = rows == BN_ROWS_HEAVISIDE ? p->v.t : rows == BN_ROWS_GAUSSIAN ? p->v.tg : p->v.t + p->v.tg;
    out[i] = std::sqrt(acc / ((double)P * count));
  }
  release();
  return BN_OK;
}

bn_status bn_error_spectrum(bn_problem p, bn_rows rows, uint32_t nbins, double* out, uint32_t* counts) {
  if (!p || !nbins || !out) return fail(BN_EINVAL, "NULL argument or no bins");
  if (rows != BN_ROWS_ALL && rows != BN_ROWS_HEAVISIDE && rows != BN_ROWS_GAUSSIAN)
    return fail(BN_EINVAL, "unknown row family");
  if (rows == BN_ROWS_GAUSSIAN && !p->v.tg) return fail(BN_EINVAL, "the problem has no Gaussian integrands");
  if (!p->have_counts) return fail(BN_ESTATE, "bn_compute_errors must run first");
  bn_status rs = refresh_errors(p);
  if (rs != BN_OK) return rs;
  const uint32_t W = p->v.w, H = p->v.h;
  const size_t P = (size_t)W * H;
  std::vector<float2> twx(W), twy(H);
  for (uint32_t k = 0; k < W; ++k)
    twx[k] = make_float2((float)std::cos(2.0 * M_PI * k / W), (float)-std::sin(2.0 * M_PI * k / W));
  for (uint32_t k = 0; k < H; ++k)
    twy[k] = make_float2((float)std::cos(2.0 * M_PI * k / H), (float)-std::sin(2.0 * M_PI * k / H));
  float2 *d_rows = nullptr, *d_twx = nullptr, *d_twy = nullptr;
  double* d_pw = nullptr;
  auto release = [&]() {
    for (void* q : {(void*)d_rows, (void*)d_twx, (void*)d_twy, (void*)d_pw})
      if (q) (void)hipFree(q);
  };
  // scratch for the duration of the call only
  hipError_t e = hipMalloc((void**)&d_rows, spectrum_scratch_floats2(p->v) * sizeof(float2));
  if (e == hipSuccess) e = hipMalloc((void**)&d_twx, W * sizeof(float2));
  if (e == hipSuccess) e = hipMalloc((void**)&d_twy, H * sizeof(float2));
  if (e == hipSuccess) e = hipMalloc((void**)&d_pw, P * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(BN_ENOMEM, "spectrum scratch: %s", hipGetErrorString(e));
  }
  e = hipMemcpyAsync(d_twx, twx.data(), W * sizeof(float2), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_twy, twy.data(), H * sizeof(float2), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(d_pw, 0, P * sizeof(double), p->stream);
  const float* fields[2] = {p->v.err, p->v.gerr};
  const uint32_t pitches[2] = {p->v.tp, p->v.tgp}, valids[2] = {p->v.t, p->v.tg};
  uint32_t used = 0;
  for (int f = 0; f < 2 && e == hipSuccess; ++f) {
    if (!valids[f] || (rows == BN_ROWS_HEAVISIDE && f == 1) || (rows == BN_ROWS_GAUSSIAN && f == 0)) continue;
    used += valids[f];
    for (uint32_t t0 = 0; t0 < valids[f] && e == hipSuccess; t0 += spectrum_chunk())
      e = launch_spectrum_chunk(p->v, fields[f], pitches[f], valids[f], t0, d_twx, d_twy, d_rows, d_pw, p->stream);
  }
  std::vector<double> pw(P);
  if (e == hipSuccess) e = hipMemcpyAsync(pw.data(), d_pw, P * sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  release();
  if (e != hipSuccess) return fail(BN_EHIP, "error spectrum: %s", hipGetErrorString(e));
  // radial bins: the frequency in cycles per pixel, folded to [-1/2, 1/2),
  // in units of 1 / min(W, H), rounded
  std::vector<double> sum(nbins, 0.0);
  std::vector<uint32_t> cnt(nbins, 0);
  const double unit = (double)std::min(W, H);
  for (uint32_t v = 0; v < H; ++v)
    for (uint32_t u = 0; u < W; ++u) {
      const double fu = 2 * u < W ? (double)u / W : (double)u / W - 1.0;
      const double fv = 2 * v < H ? (double)v / H : (double)v / H - 1.0;
      const double b = std::nearbyint(std::sqrt(fu * fu + fv * fv) * unit);
      if (b < (double)nbins) {
        sum[(size_t)b] += pw[(size_t)v * W + u];
        cnt[(size_t)b] += 1;
      }
    }
  for (uint32_t b = 0; b < nbins; ++b) {
    out[b] = cnt[b] ? sum[b] / ((double)cnt[b] * (double)P * (double)used) : 0.0;
    if (counts) counts[b] = cnt[b];
  }
  return BN_OK;
}

bn_status bn_get_offsets(bn_problem p, uint16_t* host_u) {
  if (!p || !host_u) return fail(BN_EINVAL, "NULL argument");
  if (!p->have_offsets) return fail(BN_ESTATE, "offsets are not initialised");
  HIPCHK(hipMemcpyAsync(host_u, p->v.U, (size_t)p->v.w * p->v.h * 4, hipMemcpyDeviceToHost, p->stream));
  return sync(p);
}

bn_status bn_get_counts(bn_problem p, uint16_t* host) {
  if (!p || !host) return fail(BN_EINVAL, "NULL argument");
  if (!p->have_counts) return fail(BN_ESTATE, "bn_compute_errors must run first");
  return untile_counts(p, p->v.cnt, p->v.w * p->v.h, host);
}

bn_status bn_get_errors(bn_problem p, float* host) {
  if (!p || !host) return fail(BN_EINVAL, "NULL argument");
  if (!p->have_counts) return fail(BN_ESTATE, "bn_compute_errors must run first");
  bn_status rs = refresh_errors(p);
  if (rs != BN_OK) return rs;
  const size_t P = (size_t)p->v.w * p->v.h, row = (size_t)(p->v.t + p->v.tg) * 4;
  HIPCHK(hipMemcpy2DAsync(host, row, p->v.err, p->v.tp * 4, p->v.t * 4, P, hipMemcpyDeviceToHost, p->stream));
  if (p->v.tg)
    HIPCHK(hipMemcpy2DAsync(host + p->v.t, row, p->v.gerr, p->v.tgp * 4, p->v.tg * 4, P, hipMemcpyDeviceToHost,
                            p->stream));
  return sync(p);
}

bn_status bn_get_integrands(bn_problem p, bn_heaviside* heavisides, double* areas, bn_gaussian* gaussians,
                            double* gauss_integrals) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  if (heavisides) std::copy(p->heav.begin(), p->heav.end(), heavisides);
  if (areas) std::copy(p->area64.begin(), p->area64.end(), areas);
  if (gaussians) std::copy(p->gauss.begin(), p->gauss.end(), gaussians);
  if (gauss_integrals) std::copy(p->gint64.begin(), p->gint64.end(), gauss_integrals);
  return BN_OK;
}

bn_status bn_get_points(bn_problem p, uint32_t pixel, uint16_t* host) {
  if (!p || !host) return fail(BN_EINVAL, "NULL argument");
  if (!p->have_offsets) return fail(BN_ESTATE, "offsets are not initialised");
  if (pixel >= p->v.w * p->v.h) return fail(BN_EINVAL, "pixel %u out of range", pixel);
  // The list count buffer (m rows of Tp uint16) doubles as room for N uint32.
  bn_status s = ensure_list(p, std::max<uint32_t>(1, (2 * p->v.n + p->v.tp - 1) / p->v.tp));
  if (s != BN_OK) return s;
  uint32_t* buf = (uint32_t*)p->list_cnt;
  HIPCHK(launch_points(p->v, pixel, buf, p->stream));
  HIPCHK(hipMemcpyAsync(host, buf, (size_t)p->v.n * 4, hipMemcpyDeviceToHost, p->stream));
  return sync(p);
}

bn_status bn_delta_energy(bn_problem p, const uint32_t* pixels, const uint16_t* proposals, uint32_t m,
                          double* out_de, uint16_t* out_counts) {
  if (!p || (m && (!pixels || !proposals || !out_de))) return fail(BN_EINVAL, "NULL argument");
  if (!p->have_counts) return fail(BN_ESTATE, "bn_compute_errors must run first");
  const uint32_t P = p->v.w * p->v.h;
  if (m > P) return fail(BN_EINVAL, "m=%u exceeds the pixel count", m);
  for (uint32_t i = 0; i < m; ++i)
    if (pixels[i] >= P) return fail(BN_EINVAL, "pixel %u out of range", pixels[i]);
  if (m == 0) return BN_OK;
  bn_status s = ensure_list(p, m);
  if (s != BN_OK) return s;
  DevView lv = p->v;
  lv.c_new = p->list_cnt;
  lv.u_new = p->list_u;
  lv.pix_list = p->list_pix;
  lv.delta = p->list_delta;
  lv.accept = p->list_accept;
  lv.g_new = p->list_g;
  lv.gdelta = p->list_gdelta;
  HIPCHK(hipMemcpyAsync(p->list_pix, pixels, (size_t)m * 4, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemcpyAsync(p->list_u, proposals, (size_t)m * 4, hipMemcpyHostToDevice, p->stream));
  HIPCHK(launch_count(lv, MODE_LIST, 0, m, p->stream));
  HIPCHK(launch_gauss_est(lv, MODE_LIST, m, p->stream));
  HIPCHK(launch_gauss_delta(lv, MODE_LIST, 0, m, p->stream));
  HIPCHK(launch_delta(lv, MODE_LIST, 0, m, p->stream));
  HIPCHK(hipMemcpyAsync(out_de, p->list_delta, (size_t)m * 8, hipMemcpyDeviceToHost, p->stream));
  if (out_counts) return untile_counts(p, p->list_cnt, m, out_counts);
  return sync(p);
}

bn_status bn_delta_energy_noalloc(bn_problem p, const uint32_t* pixels, const uint16_t* proposals, uint32_t m,
                                  double* out_de, uint16_t* out_counts) {
  if (!p || (m && (!pixels || !proposals || !out_de))) return fail(BN_EINVAL, "NULL argument");
  if (!p->have_counts) return fail(BN_ESTATE, "bn_compute_errors must run first");
  const uint32_t P = p->v.w * p->v.h;
  if (m > P) return fail(BN_EINVAL, "m=%u exceeds the pixel count", m);
  for (uint32_t i = 0; i < m; ++i)
    if (pixels[i] >= P) return fail(BN_EINVAL, "pixel %u out of range", pixels[i]);
  if (m == 0) return BN_OK;
  uint16_t* rows = nullptr;
  Carve measure;
  (void)list_view_in(p, measure, m, out_counts != nullptr, &rows);
  if (measure.off > NOALLOC_SCRATCH_BYTES)
    return fail(BN_EINVAL, "%u pixels need %zu bytes of scratch; the allocation-free entry point holds %zu",
                m, measure.off, NOALLOC_SCRATCH_BYTES);
  void* base = nullptr;
  HIPCHK(noalloc_scratch(p->device, &base));
  Carve c;
  c.base = (char*)base;
  const DevView lv = list_view_in(p, c, m, out_counts != nullptr, &rows);
  HIPCHK(hipMemcpyAsync((void*)lv.pix_list, pixels, (size_t)m * 4, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemcpyAsync(lv.u_new, proposals, (size_t)m * 4, hipMemcpyHostToDevice, p->stream));
  HIPCHK(launch_count(lv, MODE_LIST, 0, m, p->stream));
  HIPCHK(launch_gauss_est(lv, MODE_LIST, m, p->stream));
  HIPCHK(launch_gauss_delta(lv, MODE_LIST, 0, m, p->stream));
  HIPCHK(launch_delta(lv, MODE_LIST, 0, m, p->stream));
  HIPCHK(hipMemcpyAsync(out_de, lv.delta, (size_t)m * 8, hipMemcpyDeviceToHost, p->stream));
  if (out_counts) {
    HIPCHK(launch_untile_counts(lv.c_new, m, p->v.t, rows, p->stream));
    HIPCHK(hipMemcpyAsync(out_counts, rows, (size_t)m * p->v.t * 2, hipMemcpyDeviceToHost, p->stream));
  }
  return sync(p);
}

bn_status bn_measure_peak(bn_peak kind, uint64_t bytes, uint32_t reps, double* out) {
  if (!out) return fail(BN_EINVAL, "out is NULL");
  if (kind != BN_PEAK_HBM_COPY && kind != BN_PEAK_VALU_DOT2 && kind != BN_PEAK_MFMA_BF16)
    return fail(BN_EINVAL, "unknown peak kind %d", (int)kind);
  if (reps < 1 || reps > 1000) return fail(BN_EINVAL, "reps must lie in [1, 1000]");
  if (kind == BN_PEAK_HBM_COPY && (bytes < (1u << 20) || bytes % 16))
    return fail(BN_EINVAL, "copy size must be a multiple of 16 bytes and at least 1 MiB");
  bn_status s = check_device();
  if (s != BN_OK) return s;
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const uint32_t blocks = 8u * (uint32_t)cus;   // eight workgroups of four waves per CU
  const uint32_t iters = kind == BN_PEAK_VALU_DOT2 ? 20000u : 4000u;
  const size_t nbuf = kind == BN_PEAK_HBM_COPY ? (size_t)bytes : (size_t)blocks * 256 * 4;
  void *a = nullptr, *b = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
  };
  hipError_t e = hipMalloc(&a, nbuf);
  if (e == hipSuccess && kind == BN_PEAK_HBM_COPY) e = hipMalloc(&b, nbuf);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(BN_ENOMEM, "peak buffers of %zu bytes: %s", nbuf, hipGetErrorString(e));
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemsetAsync(a, 1, nbuf, st);
  if (e == hipSuccess) e = peak_launch((int)kind, a, b, nbuf, iters, blocks, st);   // warm-up
  double best = 0.0;
  for (uint32_t r = 0; r < reps && e == hipSuccess; ++r) {
    // copies: odd repetitions time the runtime's own device-to-device copy,
    // even ones the library's copy kernel; the better rate is kept
    const bool rt_copy = kind == BN_PEAK_HBM_COPY && (r & 1);
    e = hipEventRecord(e0, st);
    if (e == hipSuccess)
      e = rt_copy ? hipMemcpyAsync(b, a, nbuf, hipMemcpyDeviceToDevice, st)
                  : peak_launch((int)kind, a, b, nbuf, iters, blocks, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess || ms <= 0.f) break;
    const double work = kind == BN_PEAK_HBM_COPY ? 2.0 * (double)nbuf
                        : kind == BN_PEAK_VALU_DOT2 ? (double)blocks * 256.0 * iters * 8.0
                                                    : (double)blocks * 4.0 * iters * 4.0 * 32768.0;
    best = std::max(best, work / (ms * 1e-3));
  }
  release();
  if (e != hipSuccess) return fail(BN_EHIP, "peak measurement: %s", hipGetErrorString(e));
  *out = best;
  return BN_OK;
}

bn_status bn_set_profiling(bn_problem p, int enable) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  bn_status s = sync(p);
  if (s != BN_OK) return s;
  if (p->aux) HIPCHK(hipStreamSynchronize(p->aux));
  for (auto* vec : {&p->prof_recount, &p->prof_eval, &p->prof_commit}) {
    for (hipEvent_t e : *vec) (void)hipEventDestroy(e);
    vec->clear();
  }
  p->profiling = enable != 0;
  return BN_OK;
}

bn_status bn_get_profile(bn_problem p, bn_profile_stats* out) {
  if (!p || !out) return fail(BN_EINVAL, "NULL argument");
  bn_status s = sync(p);
  if (s != BN_OK) return s;
  if (p->aux) HIPCHK(hipStreamSynchronize(p->aux));
  auto total = [](const std::vector<hipEvent_t>& v, double* ms) -> hipError_t {
    *ms = 0.0;
    for (size_t i = 0; i + 1 < v.size(); i += 2) {
      float t = 0.f;
      hipError_t e = hipEventElapsedTime(&t, v[i], v[i + 1]);
      if (e != hipSuccess) return e;
      *ms += t;
    }
    return hipSuccess;
  };
  HIPCHK(total(p->prof_recount, &out->recount_ms));
  HIPCHK(total(p->prof_eval, &out->evaluate_ms));
  HIPCHK(total(p->prof_commit, &out->commit_ms));
  out->recount_launches = p->prof_recount.size() / 2;
  out->phases = p->prof_eval.size() / 2;
  return BN_OK;
}

bn_status bn_set_recount_blocks(bn_problem p, uint32_t blocks) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  bn_status s = sync(p);
  if (s != BN_OK) return s;
  if (p->aux) HIPCHK(hipStreamSynchronize(p->aux));
  p->v.count_cap = blocks;
  // captured graphs hold the old launch shape
  if (p->pair_exec) (void)hipGraphExecDestroy(p->pair_exec);
  if (p->pair_graph) (void)hipGraphDestroy(p->pair_graph);
  p->pair_exec = nullptr;
  p->pair_graph = nullptr;
  p->pair_failed = false;
  return BN_OK;
}

bn_status bn_sample_device(const bn_problem* pairs, uint32_t npairs, const uint32_t* x, const uint32_t* y,
                           const uint32_t* k, uint32_t m, float* out, void* stream) {
  if (!pairs || !npairs) return fail(BN_EINVAL, "no dimension pairs");
  if (m && (!x || !y || !k || !out)) return fail(BN_EINVAL, "NULL query or output buffer");
  std::vector<SamplerPair> tab(npairs);
  for (uint32_t d = 0; d < npairs; ++d) {
    const bn_problem p = pairs[d];
    if (!p) return fail(BN_EINVAL, "pair %u is NULL", d);
    if (!p->have_offsets) return fail(BN_ESTATE, "pair %u has no offsets", d);
    tab[d] = SamplerPair{p->v.lat, p->v.U, p->v.w, p->v.h, p->v.n, p->v.log2n};
    // the pair's own work (sweeps) must be finished before its tile is read
    bn_status s = sync(p);
    if (s != BN_OK) return s;
    if (p->aux) HIPCHK(hipStreamSynchronize(p->aux));
  }
  if (!m) return BN_OK;
  hipStream_t st = stream ? (hipStream_t)stream : pairs[0]->stream;
  SamplerPair* dtab = nullptr;
  HIPCHK(hipMalloc((void**)&dtab, npairs * sizeof(SamplerPair)));
  hipError_t e = hipMemcpyAsync(dtab, tab.data(), npairs * sizeof(SamplerPair), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_sample(dtab, npairs, x, y, k, m, out, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dtab);
  if (e != hipSuccess) return fail(BN_EHIP, "sampler query: %s", hipGetErrorString(e));
  return BN_OK;
}

bn_status bn_sample(const bn_problem* pairs, uint32_t npairs, const uint32_t* x, const uint32_t* y,
                    const uint32_t* k, uint32_t m, float* out) {
  if (!pairs || !npairs) return fail(BN_EINVAL, "no dimension pairs");
  if (m && (!x || !y || !k || !out)) return fail(BN_EINVAL, "NULL query or output buffer");
  if (!m) return bn_sample_device(pairs, npairs, nullptr, nullptr, nullptr, 0, nullptr, nullptr);
  uint32_t* dq = nullptr;
  float* dout = nullptr;
  const size_t nout = (size_t)m * 2 * npairs;
  hipError_t e = hipMalloc((void**)&dq, (size_t)3 * m * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&dout, nout * 4);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (dq) (void)hipFree(dq);
    return fail(BN_ENOMEM, "sampler query buffers: %s", hipGetErrorString(e));
  }
  hipStream_t st = pairs[0] ? pairs[0]->stream : nullptr;
  e = hipMemcpyAsync(dq, x, (size_t)m * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dq + m, y, (size_t)m * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dq + 2 * (size_t)m, k, (size_t)m * 4, hipMemcpyHostToDevice, st);
  bn_status s = BN_OK;
  if (e != hipSuccess) s = fail(BN_EHIP, "sampler query upload: %s", hipGetErrorString(e));
  if (s == BN_OK) s = bn_sample_device(pairs, npairs, dq, dq + m, dq + 2 * (size_t)m, m, dout, st);
  if (s == BN_OK) {
    e = hipMemcpy(out, dout, nout * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) s = fail(BN_EHIP, "sampler query download: %s", hipGetErrorString(e));
  }
  (void)hipFree(dq);
  (void)hipFree(dout);
  return s;
}

bn_status bn_get_sweep_index(bn_problem p, uint64_t* out) {
  if (!p || !out) return fail(BN_EINVAL, "NULL argument");
  unsigned long long v = 0;
  HIPCHK(hipMemcpyAsync(&v, p->v.ctr, 8, hipMemcpyDeviceToHost, p->stream));
  bn_status s = sync(p);
  if (s != BN_OK) return s;
  p->sweep = v;
  *out = v;
  return BN_OK;
}

bn_status bn_set_sweep_index(bn_problem p, uint64_t sweep) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  const unsigned long long v = sweep;
  HIPCHK(hipMemcpyAsync(p->v.ctr, &v, 8, hipMemcpyHostToDevice, p->stream));
  bn_status s = sync(p);
  if (s != BN_OK) return s;
  p->sweep = sweep;
  return BN_OK;
}

bn_status bn_phase_propose(bn_problem p, uint32_t kappa) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  if (!p->have_counts) return fail(BN_ESTATE, "bn_compute_errors must run first");
  if (kappa >= p->v.k * p->v.k) return fail(BN_EINVAL, "class %u out of range", kappa);
  if (p->cfg.move == BN_SWAP) return BN_OK;   // couples are listed by the evaluation
  HIPCHK(launch_count(p->v, MODE_CLASS, kappa, p->v.pc, p->stream));
  HIPCHK(launch_gauss_est(p->v, MODE_CLASS, p->v.pc, p->stream));
  return BN_OK;
}

bn_status bn_phase_evaluate(bn_problem p, uint32_t kappa) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  if (!p->have_counts) return fail(BN_ESTATE, "bn_compute_errors must run first");
  if (kappa >= p->v.k * p->v.k) return fail(BN_EINVAL, "class %u out of range", kappa);
  if (p->cfg.move == BN_SWAP) return swap_evaluate(p, kappa);
  HIPCHK(launch_gauss_delta(p->v, MODE_CLASS, kappa, p->v.pc, p->stream));
  HIPCHK(launch_delta(p->v, MODE_CLASS, kappa, p->v.pc, p->stream));
  return BN_OK;
}

bn_status bn_phase_commit(bn_problem p, uint32_t kappa) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  if (!p->have_counts) return fail(BN_ESTATE, "bn_compute_errors must run first");
  if (kappa >= p->v.k * p->v.k) return fail(BN_EINVAL, "class %u out of range", kappa);
  if (p->cfg.move == BN_SWAP) {
    bn_status s = swap_commit(p);
    if (s != BN_OK) return s;
    p->errors_valid = false;
    return BN_OK;
  }
  HIPCHK(launch_commit(p->v, kappa, p->stream));
  HIPCHK(launch_gauss_commit(p->v, kappa, p->stream));
  p->errors_valid = false;
  return BN_OK;
}

bn_status bn_phase_advance(bn_problem p) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  HIPCHK(launch_advance(p->v, p->stream));
  p->sweep += 1;
  return BN_OK;
}

bn_status bn_get_swap_pass(bn_problem p, uint32_t* a, uint32_t* b, double* delta, uint8_t* accept) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  if (p->cfg.move != BN_SWAP) return fail(BN_ESTATE, "the problem does not use swap moves");
  const uint32_t half = p->sv.m / 2;
  if (a || b) {
    std::vector<uint32_t> ab((size_t)2 * half);
    HIPCHK(hipMemcpyAsync(ab.data(), p->v.u_new, ab.size() * 4, hipMemcpyDeviceToHost, p->stream));
    bn_status s = sync(p);
    if (s != BN_OK) return s;
    for (uint32_t i = 0; i < half; ++i) {
      if (a) a[i] = ab[2 * i];
      if (b) b[i] = ab[2 * i + 1];
    }
  }
  if (delta) HIPCHK(hipMemcpyAsync(delta, p->v.delta, (size_t)half * 8, hipMemcpyDeviceToHost, p->stream));
  if (accept) HIPCHK(hipMemcpyAsync(accept, p->v.accept, half, hipMemcpyDeviceToHost, p->stream));
  return sync(p);
}

bn_status bn_get_phase(bn_problem p, uint16_t* u_new, uint16_t* c_new, double* delta, uint8_t* accept) {
  if (!p) return fail(BN_EINVAL, "NULL problem");
  if (p->cfg.move == BN_SWAP) return fail(BN_ESTATE, "swap passes are read with bn_get_swap_pass");
  const uint32_t M = p->v.pc;
  if (u_new) HIPCHK(hipMemcpyAsync(u_new, p->v.u_new, (size_t)M * 4, hipMemcpyDeviceToHost, p->stream));
  if (c_new) {
    bn_status s = untile_counts(p, p->v.c_new, M, c_new);
    if (s != BN_OK) return s;
  }
  if (delta) HIPCHK(hipMemcpyAsync(delta, p->v.delta, (size_t)M * 8, hipMemcpyDeviceToHost, p->stream));
  if (accept) HIPCHK(hipMemcpyAsync(accept, p->v.accept, M, hipMemcpyDeviceToHost, p->stream));
  return sync(p);
}

bn_status bn_create_batch(const bn_problem* members, uint32_t m, const char* tune_cache, bn_batch* out) {
  if (!members || !out || m == 0) return fail(BN_EINVAL, "members and out must be non-NULL, m >= 1");
  *out = nullptr;
  for (uint32_t i = 0; i < m; ++i) {
    bn_problem p = members[i];
    if (!p) return fail(BN_EINVAL, "member %u is NULL", i);
    if (!p->have_counts) return fail(BN_ESTATE, "member %u: bn_compute_errors must run first", i);
    if (p->stream != members[0]->stream) return fail(BN_EINVAL, "members must share one stream");
    if (p->cfg.colour_k != members[0]->cfg.colour_k) return fail(BN_EINVAL, "members must share colour_k");
    if (p->profiling) return fail(BN_ESTATE, "member %u has kernel profiling on", i);
    for (uint32_t j = 0; j < i; ++j)
      if (members[j] == p) return fail(BN_EINVAL, "member %u appears twice", i);
  }
  const uint32_t K = members[0]->cfg.colour_k;
  if (K != 1 && K != 2 && K != 4) return fail(BN_EUNSUPPORTED, "batched sweeps need colour_k in {1, 2, 4}");
  bn_batch b = new bn_batch_s();
  b->members.assign(members, members + m);
  b->stream = members[0]->stream;
  b->colour_k = K;
  for (uint32_t i = 0; i < m; ++i) {
    const bn_problem mp = members[i];
    if (mp->cfg.precision != BN_FP32 || mp->cfg.move != BN_REDRAW || mp->cfg.t_gauss) {
      b->solo.push_back(i);
      continue;
    }
    const DevView& v = mp->v;
    const int kind = count_kind(v);
    auto cg = std::find_if(b->count_groups.begin(), b->count_groups.end(), [&](const BatchGroup& g) { return g.kind == kind; });
    if (cg == b->count_groups.end()) {
      b->count_groups.push_back(BatchGroup());
      b->count_groups.back().kind = kind;
      cg = b->count_groups.end() - 1;
    }
    cg->idx.push_back(i);
    auto sg = std::find_if(b->stage_groups.begin(), b->stage_groups.end(), [&](const BatchGroup& g) { return g.radius == v.radius; });
    if (sg == b->stage_groups.end()) {
      b->stage_groups.push_back(BatchGroup());
      b->stage_groups.back().radius = v.radius;
      b->stage_groups.back().k = K;
      sg = b->stage_groups.end() - 1;
    }
    sg->idx.push_back(i);
    b->finish_all.idx.push_back(i);
    b->commit_all.idx.push_back(i);
  }
  // The recount launches follow the members' order, except that the one of
  // the smallest N goes first: a long VALU-bound launch first meets the first
  // colour phases and was 8 % slower over the sweep.
  if (!b->count_groups.empty()) {
    auto first = std::min_element(b->count_groups.begin(), b->count_groups.end(),
                                  [](const BatchGroup& x, const BatchGroup& y) { return x.kind < y.kind; });
    std::rotate(b->count_groups.begin(), first, first + 1);
  }
  // proposal sets of every redraw member and the batch's auxiliary stream
  {
    bn_status s = BN_OK;
    for (uint32_t i = 0; i < m && s == BN_OK; ++i)
      if (members[i]->cfg.move == BN_REDRAW) s = ensure_sweep_sets(members[i]);
    hipError_t e = s == BN_OK ? hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking) : hipSuccess;
    for (hipEvent_t& ev : b->ev)
      if (e == hipSuccess && s == BN_OK) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (s == BN_OK && e != hipSuccess) s = fail(BN_EHIP, "batch stream and events: %s", hipGetErrorString(e));
    if (s != BN_OK) {
      delete b;
      return s;
    }
  }
  // launch choices: cached, else tuned on the device
  bool cached = false;
  const std::string key = batch_key(b);
  if (tune_cache) {
    if (FILE* f = std::fopen(tune_cache, "r")) {
      char line[8192];
      while (std::fgets(line, sizeof line, f)) {
        char k[4096];
        unsigned tc = 0, sl = 0, sh = 0;
        if (std::sscanf(line, "%4095s tch=%u slices=%u shape=%u", k, &tc, &sl, &sh) >= 3 && key == k) {
          // only the tuner's own candidates are trusted: a chunk that is not
          // a multiple of 64 integrands would make the counting waves' tiles
          // overlap
          if (!tune_choice_valid(tc, sl, sh)) continue;
          b->tch = tc;
          b->slice_target = sl;
          b->shape = sh;
          cached = true;
        }
      }
      std::fclose(f);
    }
  }
  bn_status s = batch_upload(b);
  if (s == BN_OK) s = batch_prefetch(b);
  if (s == BN_OK && !cached) s = batch_tune(b);
  if (s != BN_OK) {
    delete b;
    return s;
  }
  if (tune_cache && !cached) {
    if (FILE* f = std::fopen(tune_cache, "a")) {
      std::fprintf(f, "%s tch=%u slices=%u shape=%u\n", key.c_str(), b->tch, b->slice_target, b->shape);
      std::fclose(f);
    }
  }
  *out = b;
  return BN_OK;
}

bn_status bn_batch_sweep(bn_batch b, uint32_t k) {
  if (!b) return fail(BN_EINVAL, "NULL batch");
  if (!k) return BN_OK;
  bn_status s = batch_prefetch(b);
  if (s != BN_OK) return s;
  if (k >= 2 && !b->graph_exec) {
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    s = batch_record_pair(b);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (s != BN_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return fail(BN_EHIP, "batch graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      b->graph_exec = nullptr;
      return fail(BN_EHIP, "batch graph instantiate: %s", hipGetErrorString(e));
    }
    b->graph = g;
  }
  for (uint32_t i = 0; i + 1 < k; i += 2) HIPCHK(hipGraphLaunch(b->graph_exec, b->stream));
  if (k & 1) {
    if ((s = batch_single_sweep(b)) != BN_OK) return s;
  }
  for (bn_problem p : b->members) {
    p->sweep += k;
    p->errors_valid = false;
    if (p->cfg.move == BN_REDRAW) p->prefetched = p->sweep;
  }
  return BN_OK;
}

bn_status bn_batch_tuning(bn_batch b, uint32_t* tch, uint32_t* slice_target, uint32_t* stage_shape) {
  if (!b) return fail(BN_EINVAL, "NULL batch");
  if (tch) *tch = b->tch;
  if (slice_target) *slice_target = b->slice_target;
  if (stage_shape) *stage_shape = b->shape;
  return BN_OK;
}

bn_status bn_destroy_batch(bn_batch b) {
  if (!b) return fail(BN_EINVAL, "NULL batch");
  delete b;
  return BN_OK;
}

}  // extern "C"
