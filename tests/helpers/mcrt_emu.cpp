// CPU harness of the HIP library's per-lane code (test infrastructure).
//
// Runs the lane logic of the life-cycle, trace and peel-off kernels --
// mcrt_lane.hpp and mcrt_device.hpp, compiled here for the host -- in one
// emulated wavefront with the kernels' batching loop, on host buffers, with
// every memory access bounds-checked and every walk's length capped.  A
// violation aborts the call with a message instead of touching memory it
// should not.  Entry points mirror include/mcrt.h with host pointers and
// explicit buffer sizes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdexcept>
#include <string>
#include <vector>

#include "mcrt.h"
#include "mcrt_device.hpp"
#include "mcrt_host.hpp"
#include "mcrt_lane.hpp"

using namespace mcrt;

namespace {

thread_local std::string g_violation;

struct Violation : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define EMU_CHECK(cond, what, idx, lim)                                                                    \
  do {                                                                                                     \
    if (!(cond)) throw Violation(std::string(what) + " index " + std::to_string((long long)(idx)) +        \
                                 " outside [0, " + std::to_string((long long)(lim)) + ")");               \
  } while (0)

template <typename R>
struct HostLifeMem {
  const R* rho_;
  long long ncell;
  const host::Prepared& pr;
  double* images;
  long long n_images;
  double* absorbed;
  long long n_absorbed;
  const double* adj_;
  long long n_adj;
  double* grad;
  long long n_grad;
  unsigned long long next = 0;
  unsigned long long xs[7] = {0, 0, 0, 0, 0, 0, 0};

  R rho(int c) const {
    EMU_CHECK(c >= 0 && c < ncell, "density", c, ncell);
    return rho_[c];
  }
  const DetDev& det(int d) const {
    EMU_CHECK(d >= 0 && d < pr.P.n_det, "frame", d, pr.P.n_det);
    return pr.det[d];
  }
  const LamDev& lam(int l) const {
    EMU_CHECK(l >= 0 && l < pr.P.n_lambda, "wavelength", l, pr.P.n_lambda);
    return pr.lam[l];
  }
  const SrcDev& src(int s) const {
    EMU_CHECK(s >= 0 && s < pr.P.n_src, "source", s, pr.P.n_src);
    return pr.src[s];
  }
  double adj(long long i) const {
    EMU_CHECK(i >= 0 && i < n_adj, "adjoint image", i, n_adj);
    return adj_[i];
  }
  void add_image(long long i, double v) {
    EMU_CHECK(i >= 0 && i < n_images, "image", i, n_images);
    images[i] += v;
  }
  void add_absorbed(long long i, double v) {
    EMU_CHECK(i >= 0 && i < n_absorbed, "absorbed tally", i, n_absorbed);
    absorbed[i] += v;
  }
  void add_grad(int i, double v) {
    EMU_CHECK(i >= 0 && i < n_grad, "gradient", i, n_grad);
    grad[i] += v;
  }
  unsigned long long fetch() { return next++; }
  void flush_counts(unsigned a, unsigned b, unsigned c, unsigned d) {
    xs[0] += a;
    xs[1] += b;
    xs[2] += c;
    xs[6] += d;
  }
};

// The kernels' outer loop for one wavefront of `wave` lanes: events for
// every waiting lane, then lockstep crossings until `batch` lanes wait.
template <class LaneT, class Events, class Step, class Ncell>
void run_wave(std::vector<LaneT>& lanes, int batch, Events events, Step step, long long max_steps_per_ray,
              Ncell) {
  std::vector<long long> steps(lanes.size(), 0);
  for (long long outer = 0;; ++outer) {
    if (outer > (1ll << 40)) throw Violation("outer loop did not terminate");
    for (size_t i = 0; i < lanes.size(); ++i) {
      if (!lanes[i].ry.active) {
        events(lanes[i]);
        steps[i] = 0;
      }
    }
    int n_live = 0;
    for (auto& L : lanes) n_live += !L.done;
    if (n_live == 0) break;
    for (;;) {
      int n_act = 0;
      for (auto& L : lanes) n_act += L.ry.active;
      if (n_act == 0 || n_live - n_act >= batch) break;
      for (size_t i = 0; i < lanes.size(); ++i) {
        if (!lanes[i].ry.active) continue;
        step(lanes[i]);
        if (++steps[i] > max_steps_per_ray) throw Violation("a walk exceeded the grid's crossing bound");
      }
    }
  }
}

template <typename R, bool ADJ>
int emu_life(const mcrt_grid* grid, const void* rho, const mcrt_optics* optics, int n_src, const mcrt_source* sources,
             int n_det, const mcrt_detector* detectors, const mcrt_opts* opts, double* images, long long n_images,
             double* absorbed, long long n_absorbed, const double* adj, long long n_adj, double* grad, long long n_grad,
             mcrt_stats* stats, int wave) {
  host::Prepared pr;
  if (int e = host::prepare(grid, rho, optics, n_src, sources, n_det, detectors, opts, pr)) return e;
  RunParams P = pr.P;
  P.images = images;
  P.absorbed = ((opts->flags & MCRT_ABSORB) && !ADJ) ? absorbed : nullptr;
  P.adj = adj;
  P.grad = grad;
  if (!ADJ && n_images < pr.n_images && (opts->flags & 3) && n_det > 0)
    throw Violation("image buffer smaller than the layout needs");
  HostLifeMem<R> M{static_cast<const R*>(rho), (long long)P.G.ncell, pr, images, n_images, P.absorbed, n_absorbed,
                   adj, n_adj, grad, n_grad};
  if (images && !ADJ) std::fill(images, images + n_images, 0.0);
  if (P.absorbed) std::fill(absorbed, absorbed + n_absorbed, 0.0);
  if (grad) std::fill(grad, grad + n_grad, 0.0);
  std::vector<Lane<R>> lanes(wave);
  for (auto& L : lanes) lane_init(L);
  const long long cap = (long long)P.G.n[0] + P.G.n[1] + P.G.n[2] + 8;
  run_wave(
      lanes, P.batch, [&](Lane<R>& L) { lane_events<R, ADJ>(L, P, M); },
      [&](Lane<R>& L) { lane_step<R, ADJ>(L, P, M); }, cap, 0);
  if (stats) {
    double sa = 0, se = 0, st = 0;
    for (auto& L : lanes) {
      sa += L.s_abs;
      se += L.s_esc;
      st += L.s_trunc;
      M.xs[0] += L.x_path;
      M.xs[1] += L.x_loc;
      M.xs[2] += L.x_peel;
      M.xs[3] += L.n_ev;
      M.xs[4] += L.n_pk;
      M.xs[5] += L.n_pl;
      M.xs[6] += L.n_dep;
    }
    stats->emitted = pr.emitted;
    stats->absorbed = sa;
    stats->escaped = se;
    stats->truncated = st;
    stats->x_path = M.xs[0];
    stats->x_locate = M.xs[1];
    stats->x_peel = M.xs[2];
    stats->events = M.xs[3];
    stats->packages = M.xs[4];
    stats->peels = M.xs[5];
    stats->deposits = M.xs[6];
    stats->kernel_ms = 0.0;
  }
  return 0;
}

template <typename R>
struct HostTraceMem {
  const R* rho_;
  long long ncell;
  const TraceParams& P;
  long long cap_seg;  // entries of seg_cell / seg_len
  unsigned long long next = 0;
  R rho(int c) const {
    EMU_CHECK(c >= 0 && c < ncell, "density", c, ncell);
    return rho_[c];
  }
  unsigned long long fetch() { return next++; }
  void ray(long long q, double o[3], double k[3]) const {
    EMU_CHECK(q >= 0 && q < P.n_rays, "ray", q, P.n_rays);
    for (int a = 0; a < 3; ++a) {
      o[a] = P.origin[3 * q + a];
      k[a] = P.dir[3 * q + a];
    }
  }
  void set_tau(long long q, double t) const {
    EMU_CHECK(q >= 0 && q < P.n_rays, "tau", q, P.n_rays);
    P.tau[q] = t;
  }
  void set_nseg(long long q, int n) const {
    EMU_CHECK(q >= 0 && q < P.n_rays, "n_seg", q, P.n_rays);
    if (P.n_seg) P.n_seg[q] = n;
  }
  void store_seg(long long q, int j, int cell, double len) const {
    const long long i = q * P.max_seg + j;
    EMU_CHECK(j >= 0 && j < P.max_seg && i >= 0 && i < cap_seg, "segment", i, cap_seg);
    P.seg_cell[i] = cell;
    P.seg_len[i] = len;
  }
};

template <typename R>
int emu_trace(const mcrt_grid* grid, const void* rho, double kappa, int64_t n_rays, const double* origin,
              const double* dir, double* tau, int32_t max_seg, int32_t* seg_cell, double* seg_len, int32_t* n_seg,
              uint64_t* crossings, int wave) {
  const bool lists = seg_cell != nullptr;
  TraceParams P;
  std::memset(&P, 0, sizeof P);
  P.G = host::make_grid(*grid);
  P.rho = rho;
  P.kappa = kappa;
  P.n_rays = n_rays;
  P.origin = origin;
  P.dir = dir;
  P.tau = tau;
  P.max_seg = lists ? max_seg : 0;
  P.seg_cell = lists ? seg_cell : nullptr;
  P.seg_len = lists ? seg_len : nullptr;
  P.n_seg = n_seg;
  P.batch = 16;
  HostTraceMem<R> M{static_cast<const R*>(rho), (long long)P.G.ncell, P, lists ? (long long)max_seg * n_rays : 0};
  std::vector<TraceLane<R>> lanes(wave);
  for (auto& L : lanes) trace_init(L);
  const long long cap = (long long)P.G.n[0] + P.G.n[1] + P.G.n[2] + 8;
  run_wave(
      lanes, P.batch, [&](TraceLane<R>& L) { trace_events(L, P, M); }, [&](TraceLane<R>& L) { trace_step(L, P, M); },
      cap, 0);
  unsigned long long total = 0, over = 0;
  for (auto& L : lanes) {
    total += L.total;
    over += L.overflow;
  }
  if (crossings) *crossings = total;
  if (lists && over) return host::fail(MCRT_EOVERFLOW, "%llu rays had more than max_seg segments", over);
  return 0;
}

template <typename R>
struct HostPeelMem {
  const R* rho_;
  long long ncell;
  const PeelParams& P;
  const std::vector<DetDev>& dets;
  long long n_images;
  unsigned long long next = 0;
  R rho(int c) const {
    EMU_CHECK(c >= 0 && c < ncell, "density", c, ncell);
    return rho_[c];
  }
  unsigned long long fetch() { return next++; }
  const DetDev& det(int d) const {
    EMU_CHECK(d >= 0 && d < P.n_det, "frame", d, P.n_det);
    return dets[d];
  }
  void position(long long e, double r[3]) const {
    EMU_CHECK(e >= 0 && e < P.n_events, "event", e, P.n_events);
    for (int a = 0; a < 3; ++a) r[a] = P.pos[3 * e + a];
  }
  bool dir_in(long long e, double k[3]) const {
    if (!P.dir_in) return false;
    EMU_CHECK(e >= 0 && e < P.n_events, "event", e, P.n_events);
    for (int a = 0; a < 3; ++a) k[a] = P.dir_in[3 * e + a];
    return true;
  }
  double weight(long long e) const {
    EMU_CHECK(e >= 0 && e < P.n_events, "event", e, P.n_events);
    return P.w[e];
  }
  void add_image(long long i, double v) const {
    EMU_CHECK(i >= 0 && i < n_images, "image", i, n_images);
    P.images[i] += v;
  }
};

template <typename R>
int emu_peel(const mcrt_grid* grid, const void* rho, double kappa, double g, int64_t n_events, const double* pos,
             const double* dir_in, const double* w, int n_det, const mcrt_detector* detectors, double* images,
             int wave) {
  long long npix = 0;
  std::vector<DetDev> det = host::make_dets(n_det, detectors, &npix);
  PeelParams P;
  std::memset(&P, 0, sizeof P);
  P.G = host::make_grid(*grid);
  P.rho = rho;
  P.kappa = kappa;
  P.g = g;
  P.n_events = n_events;
  P.n_det = n_det;
  P.pos = pos;
  P.dir_in = dir_in;
  P.w = w;
  P.images = images;
  P.batch = 16;
  HostPeelMem<R> M{static_cast<const R*>(rho), (long long)P.G.ncell, P, det, npix};
  std::vector<PeelLane<R>> lanes(wave);
  for (auto& L : lanes) peel_init(L);
  const long long cap = (long long)P.G.n[0] + P.G.n[1] + P.G.n[2] + 8;
  run_wave(
      lanes, P.batch, [&](PeelLane<R>& L) { peel_events(L, P, M); }, [&](PeelLane<R>& L) { peel_step(L, P, M); },
      cap, 0);
  return 0;
}

int guard(const char* what, int (*f)(void*), void* arg) {
  try {
    g_violation.clear();
    return f(arg);
  } catch (const Violation& v) {
    g_violation = std::string(what) + ": " + v.what();
    return -100;
  }
}

}  // namespace

extern "C" {

const char* emu_violation(void) { return g_violation.c_str(); }
const char* emu_last_error(void) { return host::last_error().c_str(); }

int emu_run_photons(const mcrt_grid* grid, const void* rho, const mcrt_optics* optics, int n_src,
                    const mcrt_source* sources, int n_det, const mcrt_detector* detectors, const mcrt_opts* opts,
                    double* images, long long n_images, double* absorbed, long long n_absorbed, mcrt_stats* stats,
                    int wave) {
  try {
    g_violation.clear();
    host::last_error().clear();
    if (!opts) return host::fail(MCRT_EINVAL, "opts is NULL");
    return opts->precision == MCRT_PREC_FP32
               ? emu_life<float, false>(grid, rho, optics, n_src, sources, n_det, detectors, opts, images, n_images,
                                        absorbed, n_absorbed, nullptr, 0, nullptr, 0, stats, wave)
               : emu_life<double, false>(grid, rho, optics, n_src, sources, n_det, detectors, opts, images, n_images,
                                         absorbed, n_absorbed, nullptr, 0, nullptr, 0, stats, wave);
  } catch (const Violation& v) {
    g_violation = std::string("run_photons: ") + v.what();
    return -100;
  }
}

int emu_backward_density(const mcrt_grid* grid, const void* rho, const mcrt_optics* optics, int n_src,
                         const mcrt_source* sources, int n_det, const mcrt_detector* detectors, const mcrt_opts* opts,
                         const double* adj, long long n_adj, double* grad, long long n_grad, mcrt_stats* stats,
                         int wave) {
  try {
    g_violation.clear();
    host::last_error().clear();
    if (!opts) return host::fail(MCRT_EINVAL, "opts is NULL");
    mcrt_opts o = *opts;
    o.flags &= ~MCRT_ABSORB;
    return o.precision == MCRT_PREC_FP32
               ? emu_life<float, true>(grid, rho, optics, n_src, sources, n_det, detectors, &o, nullptr, 0, nullptr,
                                       0, adj, n_adj, grad, n_grad, stats, wave)
               : emu_life<double, true>(grid, rho, optics, n_src, sources, n_det, detectors, &o, nullptr, 0, nullptr,
                                        0, adj, n_adj, grad, n_grad, stats, wave);
  } catch (const Violation& v) {
    g_violation = std::string("backward_density: ") + v.what();
    return -100;
  }
}

int emu_trace_path(const mcrt_grid* grid, const void* rho, double kappa, int precision, int64_t n_rays,
                   const double* origin, const double* dir, double* tau, int32_t max_seg, int32_t* seg_cell,
                   double* seg_len, int32_t* n_seg, uint64_t* crossings, int wave) {
  try {
    g_violation.clear();
    host::last_error().clear();
    if (int e = host::check_trace(grid, rho, kappa, precision, n_rays, origin, dir, tau, max_seg, seg_cell, seg_len))
      return e;
    if (n_rays == 0) {
      if (crossings) *crossings = 0;
      return 0;
    }
    return precision == MCRT_PREC_FP32
               ? emu_trace<float>(grid, rho, kappa, n_rays, origin, dir, tau, max_seg, seg_cell, seg_len, n_seg,
                                  crossings, wave)
               : emu_trace<double>(grid, rho, kappa, n_rays, origin, dir, tau, max_seg, seg_cell, seg_len, n_seg,
                                   crossings, wave);
  } catch (const Violation& v) {
    g_violation = std::string("trace_path: ") + v.what();
    return -100;
  }
}

int emu_peel_off(const mcrt_grid* grid, const void* rho, double kappa, double g, int precision, int64_t n_events,
                 const double* pos, const double* dir_in, const double* w, int n_det, const mcrt_detector* detectors,
                 double* images, int wave) {
  try {
    g_violation.clear();
    host::last_error().clear();
    if (int e = host::check_peel(grid, rho, kappa, g, precision, n_events, pos, w, n_det, detectors, images))
      return e;
    if (n_events == 0) return 0;
    return precision == MCRT_PREC_FP32
               ? emu_peel<float>(grid, rho, kappa, g, n_events, pos, dir_in, w, n_det, detectors, images, wave)
               : emu_peel<double>(grid, rho, kappa, g, n_events, pos, dir_in, w, n_det, detectors, images, wave);
  } catch (const Violation& v) {
    g_violation = std::string("peel_off: ") + v.what();
    return -100;
  }
}

}  // extern "C"
