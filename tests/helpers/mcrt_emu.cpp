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
#include <cstddef>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "mcrt.h"
#include "mcrt_attached.hpp"
#include "mcrt_device.hpp"
#include "mcrt_host.hpp"
#include "mcrt_lane.hpp"

using namespace mcrt;

namespace {

thread_local std::string g_violation;
int g_events_kept = 32;  // adjoint event scratch per package, as the library keeps
int g_chunk_items = 0;   // > 0: smaller adjoint chunks than the library's (tests)

struct Violation : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define EMU_CHECK(cond, what, idx, lim)                                                                    \
  do {                                                                                                     \
    if (!(cond)) throw Violation(std::string(what) + " index " + std::to_string((long long)(idx)) +        \
                                 " outside [0, " + std::to_string((long long)(lim)) + ")");               \
  } while (0)

// Checks that c is the bricked address of a grid cell (not padding).
inline void check_cell(const GridDev& G, long long c, const char* what) {
  int i[3];
  EMU_CHECK(c >= 0 && c < G.ncell_pad, what, c, G.ncell_pad);
  EMU_CHECK(brick_cell(G, (int)c, i), (std::string(what) + " (padding cell)").c_str(), c, G.ncell_pad);
}

// Bricked copy of row-major densities, as the library makes on the device.
template <typename R>
std::vector<R> brick_copy(const GridDev& G, const R* rho) {
  std::vector<R> out((size_t)G.ncell_pad, R(0));
  for (int c = 0; c < G.ncell_pad; ++c) {
    int i[3];
    if (brick_cell(G, c, i)) out[c] = rho[i[0] + i[1] * G.stride[1] + i[2] * G.stride[2]];
  }
  return out;
}

// Library tally -> row-major [n][ncell]: the forward's absorbed tally
// [n][ntal] at tally_slot (slots), or a bricked array [n][ncell_pad].
inline void unbrick(const GridDev& G, const std::vector<double>& src, double* dst, int n, bool slots) {
  for (int l = 0; l < n; ++l)
    for (int m = 0; m < G.ncell; ++m) {
      int i[3] = {m % G.n[0], (m / G.n[0]) % G.n[1], m / G.n[0] / G.n[1]};
      const int c = brick_addr(G, i);
      dst[(long long)l * G.ncell + m] =
          slots ? src[(size_t)l * G.ntal + tally_slot(G, c)] : src[(size_t)l * G.ncell_pad + c];
    }
}

// Plane tables of a rectilinear grid for the harness: laid out by the
// library's own routine, checked against the caller's planes, then copied
// per axis between NaN guards (a read outside a table gives NaN crossing
// times, which end the walk and break the results the tests compare).
struct HostPlanes {
  std::vector<unsigned char> blob;
  std::vector<double> pa[3], qd[3];
  void attach(const mcrt_grid& g, GridDev& G) {
    if (G.kind == kGridRegular) return;
    blob.assign(host::plane_bytes(G, g), 0);
    host::put_planes(g, G, blob.data(), blob.data());
    if (G.kind == kGridTree) {  // the nodes as the library lays them out, checked
      for (int q = 0; q < g.tree_nodes; ++q) {
        EMU_CHECK(G.nodes[q].axis == g.tree_axis[q] && G.nodes[q].child == g.tree_child[q] &&
                      (G.nodes[q].axis < 0 || G.nodes[q].split == g.tree_split[q]),
                  "tree node table", q, g.tree_nodes);
      }
      return;
    }
    const double* P = g.planes;
    const double nan = std::nan("");
    for (int a = 0; a < 3; ++a) {
      const int n = G.n[a];
      for (int q = 0; q <= n; ++q) {
        EMU_CHECK(G.pa[a][q] == P[q], "plane table", q, n + 1);
        EMU_CHECK(G.qd[a][q] == P[q] - P[0], "relative plane table", q, n + 1);
      }
      pa[a].assign(n + 3, nan);
      qd[a].assign(n + 3, nan);
      for (int q = 0; q <= n; ++q) {
        pa[a][q + 1] = G.pa[a][q];
        qd[a][q + 1] = G.qd[a][q];
      }
      G.pa[a] = pa[a].data() + 1;
      G.qd[a] = qd[a].data() + 1;
      P += n + 1;
    }
  }
};

template <typename R, int GK, bool INST>
struct HostLifeMem {
  static constexpr int kGrid = GK;
  static constexpr bool kInst = INST;
  const R* rho_;
  const GridDev& G;
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
    check_cell(G, c, "density");
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
  const std::vector<double>* adj_abs_b = nullptr;  // bricked dL/dA [n_lambda][ncell_pad]
  double adj_abs(long long i) const {
    EMU_CHECK(adj_abs_b != nullptr, "absorbed adjoint without its buffer", i, 0);
    EMU_CHECK(i >= 0 && i < (long long)adj_abs_b->size(), "absorbed adjoint", i, (long long)adj_abs_b->size());
    check_cell(G, i % G.ncell_pad, "absorbed adjoint");
    return (*adj_abs_b)[i];
  }
  void add_image(long long i, double v) {
    EMU_CHECK(i >= 0 && i < n_images, "image", i, n_images);
    images[i] += v;
  }
  void add_absorbed(long long i, double v) {
    EMU_CHECK(i >= 0 && i < n_absorbed, "absorbed tally", i, n_absorbed);
    EMU_CHECK(i % G.ntal == tally_slot(G, (int)tally_cell(G, i % G.ntal)), "absorbed tally slot", i, n_absorbed);
    check_cell(G, tally_cell(G, i % G.ntal), "absorbed tally");
    absorbed[i] += v;
  }
  void add_grad(int i, double v) {
    EMU_CHECK(i >= 0 && i < n_grad, "gradient", i, n_grad);
    check_cell(G, i, "gradient");
    grad[i] += v;
  }
  template <bool ADJ>
  void walk_deposit(int d, long long i, double v) {
    EMU_CHECK(d >= 0 && d < kBlockWalk, "walk-block sub-step", d, kBlockWalk);
    if (ADJ)
      add_grad((int)i, v);
    else
      add_absorbed(i, v);
  }
  unsigned long long fetch() { return next++; }
  unsigned long long x_queue = 0, d_queue = 0;
  // adjoint peel-job queue
  std::vector<PeelJob>* jobs = nullptr;
  std::vector<unsigned short>* job_subs = nullptr;  // each ray's second sort key (the library's keys word)
  unsigned long long job_cap = 0, job_next = 0;
  long long n_keys = 0;
  unsigned long long job_slot() { return job_next++; }
  // adjoint event scratch [ev_max][ev_k][n_chunk], then [n_chunk]; T entries
  // (k = 0) must be written before they are read, q entries start at zero
  std::vector<double>* evs = nullptr;
  std::vector<double>* gpart = nullptr;  // pass B sums for the optics gradients [4][n_chunk]
  int ev_max = 0, ev_k = 0, n_chunk = 0;
  std::vector<unsigned char>* ev_set = nullptr;
  size_t ev_index(int slot, int e, int k) const {
    EMU_CHECK(slot >= 0 && slot < n_chunk, "event scratch package", slot, n_chunk);
    EMU_CHECK(e >= 0 && e < ev_max, "event scratch event", e, ev_max);
    EMU_CHECK(k >= 0 && k < ev_k, "event scratch entry", k, ev_k);
    return ((size_t)e * ev_k + k) * n_chunk + slot;
  }
  double ev_load(int slot, int e, int k) const {
    const size_t i = ev_index(slot, e, k);
    if (k == 0) EMU_CHECK((*ev_set)[i], "event scratch read before write", e, ev_max);
    return (*evs)[i];
  }
  void ev_store(int slot, int e, int k, double v) {
    const size_t i = ev_index(slot, e, k);
    (*evs)[i] = v;
    (*ev_set)[i] = 1;
  }
  void opt_store(int slot, double ga, double gg, double gl, int src) {
    EMU_CHECK(gpart != nullptr, "optics sums without their buffer", slot, n_chunk);
    EMU_CHECK(slot >= 0 && slot < n_chunk, "optics sums package", slot, n_chunk);
    EMU_CHECK(src >= 0 && src < pr.P.n_src, "optics sums source", src, pr.P.n_src);
    double* g = gpart->data();
    g[slot] = ga;
    g[n_chunk + slot] = gg;
    g[2 * n_chunk + slot] = gl;
    g[3 * n_chunk + slot] = (double)src;
  }
  double ev_load_beyond(int slot) const {
    EMU_CHECK(slot >= 0 && slot < n_chunk, "event scratch package", slot, n_chunk);
    return (*evs)[(size_t)ev_max * ev_k * n_chunk + slot];
  }
  void ev_add_beyond(int slot, double v) {
    EMU_CHECK(slot >= 0 && slot < n_chunk, "event scratch package", slot, n_chunk);
    (*evs)[(size_t)ev_max * ev_k * n_chunk + slot] += v;
  }
  void store_job(unsigned long long slot, const double r[3], double v, long long ii, unsigned key, unsigned sub,
                 unsigned item, int e, int d, unsigned lam) {
    EMU_CHECK(jobs != nullptr && slot < job_cap, "peel-job queue", slot, job_cap);
    EMU_CHECK(key < (unsigned long long)n_keys, "sort key", key, n_keys);
    EMU_CHECK(ii >= 0 && ii < (adj_ ? n_adj : n_images), "job image index", ii, adj_ ? n_adj : n_images);
    EMU_CHECK(item < (unsigned)n_chunk, "job package", item, n_chunk);
    EMU_CHECK(d >= 0 && d < pr.P.n_det, "job frame", d, pr.P.n_det);
    EMU_CHECK(lam < (unsigned)pr.P.n_lambda, "job wavelength", lam, pr.P.n_lambda);
    EMU_CHECK(e >= 0 && e <= kEventSat, "job event", e, kEventSat);
    EMU_CHECK(sub < (256u << kDepthBits), "second sort key", sub, 256 << kDepthBits);
    PeelJob& J = (*jobs)[slot];
    J.r[0] = r[0];
    J.r[1] = r[1];
    J.r[2] = r[2];
    J.v = v;
    J.ii = ii;
    J.key = key;
    J.slot = item;
    J.lam = lam;
    J.e = (unsigned short)e;
    J.d = (unsigned char)d;
    (*job_subs)[slot] = (unsigned short)sub;
  }
  // the forward run's tape (host memory here): every entry bounds-checked
  double* tape = nullptr;
  unsigned* tape_pix = nullptr;
  unsigned* tape_over = nullptr;
  int tape_ev = 0;
  unsigned long long tape_n = 0, item0 = 0;
  void tape_leg(int slot, int e, double T) {
    EMU_CHECK(tape != nullptr, "tape write without a tape", e, 0);
    EMU_CHECK(slot >= 0 && slot < n_chunk, "tape package", slot, n_chunk);
    if (e >= tape_ev) {
      *tape_over = 1u;
      return;
    }
    tape[(size_t)e * (1 + pr.P.n_det) * tape_n + item0 + slot] = T;
  }
  void tape_peel(int slot, int e, int d, double C, long long ii) {
    EMU_CHECK(tape != nullptr, "tape write without a tape", e, 0);
    EMU_CHECK(slot >= 0 && slot < n_chunk, "tape package", slot, n_chunk);
    EMU_CHECK(d >= 0 && d < pr.P.n_det, "tape frame", d, pr.P.n_det);
    EMU_CHECK(ii >= 0 && ii < n_images, "tape image index", ii, n_images);
    if (e >= tape_ev) {
      *tape_over = 1u;
      return;
    }
    const size_t item = item0 + slot;
    EMU_CHECK(item < tape_n, "tape item", item, tape_n);
    tape[((size_t)e * (1 + pr.P.n_det) + 1 + d) * tape_n + item] = C;
    tape_pix[((size_t)e * pr.P.n_det + d) * tape_n + item] = (unsigned)ii;
  }
  void flush_counts(unsigned a, unsigned b, unsigned c, unsigned d) {
    xs[0] += a;
    xs[1] += b;
    xs[2] += c;
    xs[6] += d;
  }
};

// The queued peel walk's accessor on regular grids: densities through the
// life-cycle accessor, cell addresses from the table of per-axis address
// terms that the peel-ray walk kernel keeps in LDS (lut_entry), every table
// index checked; brick_addr where the table would not fit, as the library
// then launches the kernel without it.
template <typename R, int GK, bool INST>
struct HostLutMem {
  static constexpr int kGrid = GK;
  static constexpr bool kLut = GK == kGridRegular;
  const HostLifeMem<R, GK, INST>& M;
  const GridDev& G;
  std::vector<int> lut;
  HostLutMem(const HostLifeMem<R, GK, INST>& m, const GridDev& g) : M(m), G(g) {
    if (kLut && lut_cells(G) <= kLutCells) {
      lut.resize(lut_cells(G));
      for (int t = 0; t < lut_cells(G); ++t) lut[t] = lut_entry(G, t);
    }
  }
  R rho(int c) const { return M.rho(c); }
  int lut_addr(const int i[3]) const {
    if (lut.empty()) return brick_addr(G, i);
    int c = 0;
    for (int a = 0; a < 3; ++a) {
      EMU_CHECK(i[a] >= -1 && i[a] <= G.n[a], "axis index for the address table", i[a], G.n[a] + 1);
      const int t = lut_first(G, a) + 1 + i[a];
      EMU_CHECK(t >= 0 && t < (int)lut.size(), "address table", t, lut.size());
      c += lut[t];
    }
    return c;
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

// Deposits of the bundled walk, straight into the bricked gradient.
template <int GK>
struct HostBundleMem {
  static constexpr int kGrid = GK;
  const GridDev& G;
  std::vector<double>& grad;
  void deposit(int cell, double v) {
    check_cell(G, cell, "bundle deposit");
    grad[cell] += v;
  }
};

// The library's counting sort of the chunk's queue by key, part by part as
// its workgroups run it (per-part key counts, exclusive scan of the
// key-major count matrix, per-part counters handing out positions), then
// each ray in sorted order: the optical-depth walk; forward, C into its
// pixel; adjoint, q = (dL/dI) C into the event scratch and, for q != 0, the
// deposit walk.  Returns the crossings; `deps` gets the deposits.
template <typename R, bool ADJ, int GK, bool INST>
unsigned long long emu_peel_jobs(HostLifeMem<R, GK, INST>& M, const RunParams& P, std::vector<PeelJob>& jobs,
                                 unsigned long long n_jobs, std::vector<double>& grad, unsigned long long& deps,
                                 long long cap_steps, bool direct = false) {
  const long long n_keys = M.n_keys;
  const int nb = host::kSortBlocks;
  const unsigned long long per = (n_jobs + nb - 1) / nb;
  std::vector<unsigned> counts((size_t)n_keys * nb, 0), starts((size_t)n_keys * nb + 1, 0);
  unsigned long long n_valid = 0;
  for (int b = 0; b < nb; ++b)
    for (unsigned long long j = b * per; j < std::min(n_jobs, (b + 1) * per); ++j) {
      EMU_CHECK(jobs[j].key < (unsigned long long)n_keys, "sort key", jobs[j].key, n_keys);
      ++counts[(size_t)jobs[j].key * nb + b];
      ++n_valid;
    }
  for (size_t i = 0; i < counts.size(); ++i) starts[i + 1] = starts[i] + counts[i];
  EMU_CHECK(starts.back() == n_valid, "sorted rays", starts.back(), n_valid);
  std::vector<unsigned> idx(n_valid, 0), perm(n_valid, 0);
  std::vector<unsigned short> subs(n_valid, 0);
  std::vector<unsigned char> filled(n_valid, 0);
  for (int b = 0; b < nb; ++b) {
    std::vector<unsigned> h(n_keys);
    for (long long k = 0; k < n_keys; ++k) h[k] = starts[(size_t)k * nb + b];
    for (unsigned long long j = b * per; j < std::min(n_jobs, (b + 1) * per); ++j) {
      const unsigned q = h[jobs[j].key]++;
      EMU_CHECK(q < n_valid && !filled[q], "sorted position", q, n_valid);
      filled[q] = 1;
      idx[q] = (unsigned)j;
      subs[q] = (*M.job_subs)[j];
    }
  }
  // second pass: each tile's run by the second key
  std::fill(filled.begin(), filled.end(), 0);
  for (long long k = 0; k < n_keys; ++k) {
    const unsigned lo = starts[(size_t)k * nb], hi = starts[(size_t)(k + 1) * nb];
    EMU_CHECK(lo <= hi && hi <= n_valid, "tile run", hi, n_valid);
    std::vector<unsigned> h(256 << kDepthBits, 0);
    for (unsigned i = lo; i < hi; ++i) ++h[subs[i]];
    unsigned run = lo;
    for (int c = 0; c < (256 << kDepthBits); ++c) {
      const unsigned t = h[c];
      h[c] = run;
      run += t;
    }
    for (unsigned i = lo; i < hi; ++i) {
      const unsigned q = h[subs[i]]++;
      EMU_CHECK(q >= lo && q < hi && !filled[q], "refined position", q, hi);
      filled[q] = 1;
      perm[q] = idx[i];
    }
  }
  HostBundleMem<GK> D{P.G, grad};
  HostLutMem<R, GK, INST> LM(M, P.G);
  unsigned long long nx = 0;
  deps = 0;
  for (unsigned long long qi = 0; qi < n_valid; ++qi) {
    const PeelJob& J = jobs[perm[qi]];
    if (qi > 0) {
      const PeelJob& Jp = jobs[perm[qi - 1]];
      const unsigned sp = (*M.job_subs)[perm[qi - 1]], sq = (*M.job_subs)[perm[qi]];
      EMU_CHECK(Jp.key < J.key || (Jp.key == J.key && sp <= sq), "sorted order", qi, n_valid);
    }
    int d = 0;
    while (d + 1 < P.n_det && (unsigned)M.det(d + 1).key_off <= J.key) ++d;
    EMU_CHECK(d == J.d, "job frame against its key", J.d, P.n_det);
    Ray<R> ry;
    long long steps = 0;
    double w = J.v;  // an adjoint from a tape: the ray's deposit weight, no optical-depth walk
    if (!direct) {
      {
        double kd[3], inv_d2, tmax;
        peel_geom<HostLifeMem<R, GK, INST>>(M.det(J.d), J.r, kd, inv_d2, tmax);
        ray_begin<R, GK>(ry, P.G, J.r, kd, tmax);
      }
      const R kap = (R)M.lam((int)J.lam).kappa;
      while (ry.active) {
        nx += tau_step<R, HostLutMem<R, GK, INST>, INST>(ry, P.G, kap, LM);
        if (++steps > cap_steps) throw Violation("a peel-job walk exceeded the grid's crossing bound");
      }
      const double C = J.v * exp(-(double)ry.tau);
      if (!ADJ) {
        M.add_image(J.ii, C);
        if (M.tape) M.tape_peel((int)J.slot, J.e, J.d, C, J.ii);
        continue;
      }
      const double q = M.adj(J.ii) * C;
      if (J.e < P.ev_max)
        M.ev_store((int)J.slot, J.e, 1 + J.d, q);
      else
        M.ev_add_beyond((int)J.slot, q);
      if (q == 0.0) continue;
      w = -q * M.lam((int)J.lam).kappa;
    } else {
      EMU_CHECK(ADJ && w != 0.0, "a deposit job from a tape without a weight", qi, n_valid);
    }
    {
      double kd[3], inv_d2, tmax;
      peel_geom<HostLifeMem<R, GK, INST>>(M.det(J.d), J.r, kd, inv_d2, tmax);
      ray_begin<R, GK>(ry, P.G, J.r, kd, tmax);
    }
    steps = 0;
    while (ry.active) {
      const unsigned n = bp_step<R, HostBundleMem<GK>, INST>(ry, P.G, w, D);
      nx += n;
      deps += n;
      if (++steps > cap_steps) throw Violation("a deposit walk exceeded the grid's crossing bound");
    }
  }
  return nx;
}

template <typename R, bool ADJ, int GK, bool INST>
int emu_life(const mcrt_grid* grid, const void* rho, const mcrt_optics* optics, int n_src, const mcrt_source* sources,
             int n_det, const mcrt_detector* detectors, const mcrt_opts* opts, double* images, long long n_images,
             double* absorbed, long long n_absorbed, const double* adj, long long n_adj, double* grad, long long n_grad,
             double* gopt, const double* adj_abs, mcrt_stats* stats, int wave) {
  host::Prepared pr;
  if (int e = host::prepare(grid, rho, optics, n_src, sources, n_det, detectors, opts, pr)) return e;
  HostPlanes planes;
  planes.attach(*grid, pr.P.G);
  // a cell source: per wavelength the prefix sums of its cells'
  // luminosities (host array here), NaN-fenced, and the totals
  std::vector<double> cum;
  if (pr.cell_src >= 0) {
    const int nl = pr.P.n_lambda, nc = pr.P.G.ncell;
    const double* x = sources[pr.cell_src].cell_lum;
    cum.assign((size_t)nl * (nc + 1) + 2, std::nan(""));
    std::vector<double> tot(nl);
    for (int l = 0; l < nl; ++l) {
      double acc = 0.0;
      for (int m = 0; m < nc; ++m) {
        const double v = x[(size_t)l * nc + m];
        if (!(v >= 0.0 && v < INFINITY)) return host::fail(MCRT_EINVAL, "cell_lum holds a negative or non-finite luminosity");
        cum[1 + (size_t)l * (nc + 1) + m] = acc;
        acc += v;
      }
      cum[1 + (size_t)l * (nc + 1) + nc] = acc;
      tot[l] = acc;
    }
    host::set_luminosities(pr, n_src, sources, tot.data(), opts->n_packages);
    pr.src[pr.cell_src].cum = cum.data() + 1;
  }
  RunParams P = pr.P;
  P.depth_drop = ADJ ? kDepthDropAdjoint : 0;  // as the library
  P.images = images;
  P.absorbed = ((opts->flags & MCRT_ABSORB) && !ADJ) ? absorbed : nullptr;
  P.adj = adj;
  P.grad = grad;
  if (!ADJ && n_images < pr.n_images && (opts->flags & 3) && n_det > 0)
    throw Violation("image buffer smaller than the layout needs");
  if (P.absorbed && n_absorbed < (long long)P.n_lambda * P.G.ncell) throw Violation("absorbed buffer too small");
  if (ADJ && grad && n_grad < P.G.ncell) throw Violation("gradient buffer too small");
  const std::vector<R> rho_b = brick_copy(P.G, static_cast<const R*>(rho));
  std::vector<double> abs_b(P.absorbed ? (size_t)P.n_lambda * P.G.ntal : 0, 0.0);
  std::vector<double> grad_b(ADJ && grad ? (size_t)P.G.ncell_pad : 0, 0.0);
  HostLifeMem<R, GK, INST> M{rho_b.data(), P.G, pr, images, n_images, P.absorbed ? abs_b.data() : nullptr,
                   (long long)abs_b.size(), adj, n_adj, grad_b.data(), (long long)grad_b.size()};
  P.absorbed = M.absorbed;
  if (images && !ADJ) std::fill(images, images + n_images, 0.0);
  const bool peel = (opts->flags & (MCRT_PEEL_EMIT | MCRT_PEEL_SCAT)) && n_det > 0;
  const long long cap = (long long)P.G.n[0] + P.G.n[1] + P.G.n[2] + 8;
  double sa = 0, se = 0, st = 0;
  // one launch of the life-cycle kernel: fresh lanes, then their statistics
  auto launch = [&](int split) {
    P.split = split;
    M.next = 0;
    std::vector<Lane<R>> lanes(wave);
    for (auto& L : lanes) lane_init(L);
    run_wave(
        lanes, P.batch, [&](Lane<R>& L) { lane_events<R, ADJ>(L, P, M); },
        [&](Lane<R>& L) { lane_step<R, ADJ>(L, P, M); },
        cap, 0);
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
  };
  // chunks of packages as the library runs them (the library sizes them by
  // its event-scratch and queue budgets; g_chunk_items overrides for tests)
  std::vector<double> aab;  // the absorbed tally's adjoint, bricked as the library does
  if (ADJ && adj_abs) {
    aab.assign((size_t)P.n_lambda * P.G.ncell_pad, 0.0);
    for (int l = 0; l < P.n_lambda; ++l) {
      const std::vector<double> row = brick_copy(P.G, adj_abs + (size_t)l * P.G.ncell);
      std::copy(row.begin(), row.end(), aab.begin() + (size_t)l * P.G.ncell_pad);
    }
    M.adj_abs_b = &aab;
    P.adj_abs = aab.data();  // only tested against null by the lanes; the loads go through M
  }
  // the adjoint tape: the forward run writes it (host memory here), an
  // adjoint with a usable one fills its scratch from it and replays once
  const uint64_t tape_need = peel ? host::tape_bytes(optics, n_det, opts) : 0;
  const int tape_ev = tape_need ? (int)host::tape_events(*optics, *opts) : 0;
  bool tape_adj = false;
  unsigned char* const tape_base = static_cast<unsigned char*>(opts->tape);
  const size_t tape_pix_off =
      host::kTapeHeader + ((sizeof(double) * (size_t)P.n_items * tape_ev * (1 + n_det) + 255) & ~size_t(255));
  if (opts->tape) {
    if (!tape_need) return host::fail(MCRT_EINVAL, "tape given, but this run cannot keep one (mcrt_tape_bytes is 0)");
    const uint64_t fp = host::tape_fingerprint(*grid, *optics, n_src, sources, n_det, detectors, *opts);
    if (!ADJ) {
      if (opts->tape_bytes < tape_need) return host::fail(MCRT_EINVAL, "tape_bytes too small");
      const host::TapeHeader hdr = host::tape_header(fp, P.n_items, tape_ev, n_det);
      std::memset(tape_base, 0, tape_need);
      std::memcpy(tape_base, &hdr, sizeof hdr);
      M.tape = reinterpret_cast<double*>(tape_base + host::kTapeHeader);
      M.tape_pix = reinterpret_cast<unsigned*>(tape_base + tape_pix_off);
      M.tape_over = reinterpret_cast<unsigned*>(tape_base + offsetof(host::TapeHeader, overflow));
      M.tape_ev = tape_ev;
      M.tape_n = P.n_items;
      P.tape = M.tape;  // only tested against null by the lanes; the writes go through M
    } else {
      host::TapeHeader hdr;
      std::memcpy(&hdr, tape_base, sizeof hdr);
      bool usable = false;
      if (int e = host::check_tape(hdr, fp, P.n_items, tape_ev, n_det, opts->tape_bytes, tape_need, &usable)) return e;
      tape_adj = usable && !adj_abs;
    }
  }
  if (ADJ) {
    P.ev_max = tape_adj ? tape_ev : g_events_kept;
    P.ev_k = 1 + P.n_det + (adj_abs ? 1 : 0);
    P.dep_jobs = tape_adj ? 1 : 0;
  }
  const size_t per_item = sizeof(double) * ((size_t)P.ev_max * P.ev_k + 1);
  unsigned long long chunk =
      ADJ ? std::min<unsigned long long>(P.n_items, std::max<size_t>(1 << 16, (size_t(1) << 30) / per_item))
          : P.n_items;
  if (g_chunk_items > 0) chunk = std::min<unsigned long long>(chunk, (unsigned long long)g_chunk_items);
  if (opts->max_chunk > 0) chunk = std::min<unsigned long long>(chunk, (unsigned long long)opts->max_chunk);
  std::vector<PeelJob> jobs;
  std::vector<unsigned short> job_subs;
  if (peel && opts->peel_queue != -1) {
    unsigned long long qcap =
        opts->peel_queue > 0 ? (unsigned long long)opts->peel_queue : chunk * (unsigned long long)P.n_det * 8ull;
    if (opts->peel_queue == 0) qcap = std::min(std::max(qcap, 1ull << 16), 1ull << 28);
    jobs.resize(qcap);
    job_subs.assign(qcap, 0);
    M.jobs = &jobs;
    M.job_subs = &job_subs;
    M.job_cap = qcap;
    M.n_keys = pr.n_keys;
    P.jobs = jobs.data();
    P.job_cap = qcap;
  }
  std::vector<double> evs, gpart;
  std::vector<unsigned char> ev_set;
  const int nl = P.n_lambda, ns = P.n_src;
  if (gopt) std::fill(gopt, gopt + (size_t)(2 + ns) * nl, 0.0);
  M.evs = &evs;
  M.ev_set = &ev_set;
  M.ev_max = P.ev_max;
  M.ev_k = P.ev_k;
  auto queue_phase = [&]() {
    unsigned long long deps = 0;
    const unsigned long long nx = emu_peel_jobs<R, ADJ, GK, INST>(M, P, jobs, std::min(M.job_next, M.job_cap),
                                                                  grad_b, deps, cap, tape_adj);
    M.x_queue += nx;
    M.d_queue += deps;
  };
  for (unsigned long long c0 = 0; c0 < P.n_items; c0 += chunk) {
    P.item0 = c0;
    P.n_chunk = std::min(chunk, P.n_items - c0);
    M.n_chunk = (int)P.n_chunk;
    M.item0 = c0;
    M.job_next = 0;
    if (!ADJ) {
      launch(0);
      if (P.jobs) queue_phase();
      continue;
    }
    evs.assign((size_t)P.n_chunk * ((size_t)P.ev_max * P.ev_k + 1), 0.0);
    ev_set.assign(evs.size(), 0);
    if (gopt) {
      gpart.assign(4 * (size_t)P.n_chunk, 0.0);
      M.gpart = &gpart;
      P.gpart = gpart.data();  // only tested against null by the lanes; the stores go through M
    }
    if (tape_adj) {  // the scratch from the tape (the library's k_tape_q), pass B, the deposit walks
      const double* tp = reinterpret_cast<const double*>(tape_base + host::kTapeHeader);
      const unsigned* px = reinterpret_cast<const unsigned*>(tape_base + tape_pix_off);
      const int nd = P.n_det;
      for (unsigned long long slot = 0; slot < P.n_chunk; ++slot) {
        const unsigned long long item = P.item0 + slot;
        for (int e = 0; e < P.ev_max; ++e) {
          const size_t b = (size_t)e * (1 + nd);
          M.ev_store((int)slot, e, 0, tp[b * P.n_items + item]);
          for (int d = 0; d < nd; ++d) {
            const double C = tp[(b + 1 + d) * P.n_items + item];
            M.ev_store((int)slot, e, 1 + d, C != 0.0 ? M.adj(px[((size_t)e * nd + d) * P.n_items + item]) * C : 0.0);
          }
        }
      }
      launch(2);  // pass B, queueing the deposit walks
      if (P.jobs) queue_phase();
    } else {
      launch(1);  // pass A
      if (P.jobs) queue_phase();
      launch(2);  // pass B
    }
    if (gopt) {  // per wavelength of the chunk: sums over its packages, then the gradients
      const unsigned long long nc = P.n_chunk;
      for (unsigned long long l = P.item0 / P.n_pkg; l <= (P.item0 + nc - 1) / P.n_pkg; ++l) {
        const unsigned long long b = std::max(l * P.n_pkg, P.item0), e = std::min((l + 1) * P.n_pkg, P.item0 + nc);
        double sa = 0.0, sg = 0.0, sl[MCRT_MAX_SOURCES] = {0};
        for (unsigned long long it = b; it < e; ++it) {
          const unsigned long long q = it - P.item0;
          sa += gpart[q];
          sg += gpart[nc + q];
          const int src = (int)gpart[3 * nc + q];
          EMU_CHECK(src >= 0 && src < ns, "optics sums source", src, ns);
          sl[src] += gpart[2 * nc + q];
        }
        optics_finish(sa, sg, sl, ns, pr.lam[l].albedo, pr.lums.data() + l, nl, gopt, gopt + nl, gopt + 2 * nl,
                      (int)l, nl);
      }
    }
  }
  M.xs[2] += M.x_queue;
  M.xs[6] += M.d_queue;
  if (P.absorbed) unbrick(P.G, abs_b, absorbed, P.n_lambda, true);
  if (ADJ && grad) unbrick(P.G, grad_b, grad, 1, false);
  if (stats) {
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
    stats->x_queue = M.x_queue;
    stats->life_ms = stats->queue_ms = 0.0;
    stats->d_queue = M.d_queue;
    stats->life_launches = (ADJ && !tape_adj ? 2 : 1) * ((P.n_items + chunk - 1) / chunk);
    stats->sort_ms = stats->peel_ms = stats->dep_ms = 0.0;
  }
  return 0;
}

template <typename R, int GK>
struct HostTraceMem {
  static constexpr int kGrid = GK;
  const R* rho_;
  const TraceParams& P;
  long long cap_seg;  // entries of seg_cell / seg_len
  unsigned long long next = 0;
  R rho(int c) const {
    check_cell(P.G, c, "density");
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
    check_cell(P.G, cell, "segment cell");
    P.seg_cell[i] = brick_to_linear(P.G, cell);
    P.seg_len[i] = len;
  }
};

template <typename R, int GK>
int emu_trace(const mcrt_grid* grid, const void* rho, double kappa, int64_t n_rays, const double* origin,
              const double* dir, double* tau, int32_t max_seg, int32_t* seg_cell, double* seg_len, int32_t* n_seg,
              uint64_t* crossings, int brick_shape, int wave) {
  const bool lists = seg_cell != nullptr;
  TraceParams P;
  std::memset(&P, 0, sizeof P);
  if (int e = host::make_grid(*grid, (int)sizeof(R), brick_shape, P.G)) return e;
  HostPlanes planes;
  planes.attach(*grid, P.G);
  const std::vector<R> rho_b = brick_copy(P.G, static_cast<const R*>(rho));
  P.rho = rho_b.data();
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
  HostTraceMem<R, GK> M{rho_b.data(), P, lists ? (long long)max_seg * n_rays : 0};
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

template <typename R, int GK>
struct HostPeelMem {
  static constexpr int kGrid = GK;
  const R* rho_;
  const PeelParams& P;
  const std::vector<DetDev>& dets;
  long long n_images;
  unsigned long long next = 0;
  R rho(int c) const {
    check_cell(P.G, c, "density");
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

template <typename R, int GK>
int emu_peel(const mcrt_grid* grid, const void* rho, double kappa, double g, int64_t n_events, const double* pos,
             const double* dir_in, const double* w, int n_det, const mcrt_detector* detectors, double* images,
             int brick_shape, int wave) {
  long long npix = 0;
  std::vector<DetDev> det = host::make_dets(n_det, detectors, &npix);
  PeelParams P;
  std::memset(&P, 0, sizeof P);
  if (int e = host::make_grid(*grid, (int)sizeof(R), brick_shape, P.G)) return e;
  HostPlanes planes;
  planes.attach(*grid, P.G);
  const std::vector<R> rho_b = brick_copy(P.G, static_cast<const R*>(rho));
  P.rho = rho_b.data();
  P.kappa = kappa;
  P.g = g;
  P.n_events = n_events;
  P.n_det = n_det;
  P.pos = pos;
  P.dir_in = dir_in;
  P.w = w;
  P.images = images;
  P.batch = 16;
  HostPeelMem<R, GK> M{rho_b.data(), P, det, npix};
  std::vector<PeelLane<R>> lanes(wave);
  for (auto& L : lanes) peel_init(L);
  const long long cap = (long long)P.G.n[0] + P.G.n[1] + P.G.n[2] + 8;
  run_wave(
      lanes, P.batch, [&](PeelLane<R>& L) { peel_events(L, P, M); }, [&](PeelLane<R>& L) { peel_step(L, P, M); },
      cap, 0);
  return 0;
}

// The attached gradient's per-item code (mcrt_attached.hpp) on host buffers:
// items one after another, in FP64 whatever the densities' storage (R), as
// the library runs it; every access checked, workspace reads checked to
// follow a write of the same item.
template <typename S, int GK>
struct HostAttMem {
  static constexpr int kGrid = GK;
  const S* rho_;  // as stored, read as FP64
  const GridDev& G;
  const host::Prepared& pr;
  const double* adj_;
  long long n_adj;
  std::vector<double>& grad;
  std::vector<double>& ws;
  std::vector<unsigned char>& ws_set;
  int ev_max;
  int n_chunk;
  bool over = false;
  double rho(int c) const {
    check_cell(G, c, "density");
    return (double)rho_[c];
  }
  const DetDev& det(int d) const {
    EMU_CHECK(d >= 0 && d < pr.P.n_det, "instrument", d, pr.P.n_det);
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
  void add_grad(int i, double v) {
    EMU_CHECK(i >= 0 && i < (long long)grad.size(), "gradient", i, (long long)grad.size());
    check_cell(G, i, "gradient");
    grad[i] += v;
  }
  size_t ws_index(int slot, int e, int f) const {
    EMU_CHECK(slot >= 0 && slot < n_chunk, "workspace item", slot, n_chunk);
    EMU_CHECK(e >= 0 && e < ev_max, "workspace event", e, ev_max);
    EMU_CHECK(f >= 0 && f < kAttF, "workspace field", f, kAttF);
    return ((size_t)e * kAttF + f) * n_chunk + slot;
  }
  double att_ld(int slot, int e, int f) const {
    const size_t i = ws_index(slot, e, f);
    EMU_CHECK(ws_set[i], "workspace read before write", e, ev_max);
    return ws[i];
  }
  void att_st(int slot, int e, int f, double v) {
    const size_t i = ws_index(slot, e, f);
    ws[i] = v;
    ws_set[i] = 1;
  }
  void att_over() { over = true; }
  // the library queues the peel rays' deposit walks for its peel-job kernels
  // when it can; the harness walks them in place (the same deposits, summed
  // in another order)
  bool queue_deposit(const DetDev&, int, const double*, int, double, long long, unsigned, int, unsigned) {
    return false;
  }
};

template <typename R, int GK>
int emu_attached(const mcrt_grid* grid, const void* rho, const mcrt_optics* optics, int n_src,
                 const mcrt_source* sources, int n_det, const mcrt_detector* detectors, const mcrt_opts* opts,
                 const double* adj, long long n_adj, double* grad, long long n_grad, mcrt_stats* stats) {
  host::Prepared pr;
  if (int e = host::prepare(grid, rho, optics, n_src, sources, n_det, detectors, opts, pr)) return e;
  int ev = 0;
  if (int e = host::attached_check(*optics, n_det, detectors, *opts, false, false, &ev)) return e;
  HostPlanes planes;
  planes.attach(*grid, pr.P.G);
  std::vector<double> cum;
  if (pr.cell_src >= 0) {  // as emu_life: the cell source's prefix sums, NaN-fenced
    const int nl = pr.P.n_lambda, nc = pr.P.G.ncell;
    const double* x = sources[pr.cell_src].cell_lum;
    cum.assign((size_t)nl * (nc + 1) + 2, std::nan(""));
    std::vector<double> tot(nl);
    for (int l = 0; l < nl; ++l) {
      double acc = 0.0;
      for (int m = 0; m < nc; ++m) {
        const double v = x[(size_t)l * nc + m];
        if (!(v >= 0.0 && v < INFINITY)) return host::fail(MCRT_EINVAL, "cell_lum holds a negative or non-finite luminosity");
        cum[1 + (size_t)l * (nc + 1) + m] = acc;
        acc += v;
      }
      cum[1 + (size_t)l * (nc + 1) + nc] = acc;
      tot[l] = acc;
    }
    host::set_luminosities(pr, n_src, sources, tot.data(), opts->n_packages);
    pr.src[pr.cell_src].cum = cum.data() + 1;
  }
  RunParams P = pr.P;
  if (n_grad < P.G.ncell) throw Violation("gradient buffer too small");
  const std::vector<R> rho_b = brick_copy(P.G, static_cast<const R*>(rho));
  std::vector<double> grad_b((size_t)P.G.ncell_pad, 0.0);
  const int chunk = g_chunk_items > 0 ? g_chunk_items : (int)std::min<unsigned long long>(P.n_items, 4096);
  std::vector<double> ws((size_t)ev * kAttF * chunk, std::nan(""));
  std::vector<unsigned char> ws_set(ws.size(), 0);
  HostAttMem<R, GK> M{rho_b.data(), P.G, pr, adj, n_adj, grad_b, ws, ws_set, ev, chunk};
  P.ev_max = ev;
  AttCounts c;
  unsigned long long launches = 0;
  for (unsigned long long c0 = 0; c0 < P.n_items; c0 += chunk) {
    const int n = (int)std::min<unsigned long long>(chunk, P.n_items - c0);
    M.n_chunk = n;
    std::fill(ws_set.begin(), ws_set.end(), 0);
    for (int k = 0; k < n; ++k) attached_item<double>(P, M, c0 + k, k, c);
    ++launches;
  }
  if (M.over) return host::fail(MCRT_EOVERFLOW, "MCRT_ATTACHED: a package had more events than %d", ev);
  unbrick(P.G, grad_b, grad, 1, false);
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    stats->emitted = pr.emitted;
    stats->absorbed = c.s_abs;
    stats->escaped = c.s_esc;
    stats->truncated = c.s_trunc;
    stats->x_path = c.x_path;
    stats->x_locate = c.x_loc;
    stats->x_peel = c.x_peel;
    stats->events = c.n_ev;
    stats->packages = c.n_pk;
    stats->peels = c.n_pl;
    stats->deposits = c.n_dep;
    stats->d_queue = c.x_dep;
    stats->life_launches = launches;
  }
  return 0;
}

// Precision and grid kind of a call, as the library dispatches its kernels.
inline int grid_kind(const mcrt_grid* g) {
  return !g ? kGridRegular : (g->tree_nodes > 0 ? kGridTree : (g->planes ? kGridRect : kGridRegular));
}

template <bool ADJ, typename R, bool INST, typename... A>
int life_kind(int kind, A... args) {
  if (kind == kGridRect) return emu_life<R, ADJ, kGridRect, INST>(args...);
  if (kind == kGridTree) return emu_life<R, ADJ, kGridTree, INST>(args...);
  return emu_life<R, ADJ, kGridRegular, INST>(args...);
}

// As the library: the full variant of the kernels (SED instruments,
// cameras, optics and absorbed-tally gradients) only when one is used.
template <bool ADJ, typename... A>
int life_dispatch(bool f32, int kind, int n_det, const mcrt_detector* dets, bool extras, A... args) {
  bool inst = extras;  // optics or absorbed-tally gradients take the full variant too
  for (int d = 0; d < n_det && dets; ++d) inst = inst || dets[d].kind != MCRT_DET_FRAME;
  if (inst) return f32 ? life_kind<ADJ, float, true>(kind, args...) : life_kind<ADJ, double, true>(kind, args...);
  return f32 ? life_kind<ADJ, float, false>(kind, args...) : life_kind<ADJ, double, false>(kind, args...);
}

template <typename R, typename... A>
int trace_kind(int kind, A... args) {
  if (kind == kGridRect) return emu_trace<R, kGridRect>(args...);
  if (kind == kGridTree) return emu_trace<R, kGridTree>(args...);
  return emu_trace<R, kGridRegular>(args...);
}

template <typename... A>
int trace_dispatch(bool f32, int kind, A... args) {
  return f32 ? trace_kind<float>(kind, args...) : trace_kind<double>(kind, args...);
}

template <typename R, typename... A>
int peel_kind(int kind, A... args) {
  if (kind == kGridRect) return emu_peel<R, kGridRect>(args...);
  if (kind == kGridTree) return emu_peel<R, kGridTree>(args...);
  return emu_peel<R, kGridRegular>(args...);
}

template <typename... A>
int peel_dispatch(bool f32, int kind, A... args) {
  return f32 ? peel_kind<float>(kind, args...) : peel_kind<double>(kind, args...);
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
void emu_set_events_kept(int n) { g_events_kept = n; }
void emu_set_chunk_items(int n) { g_chunk_items = n; }
const char* emu_last_error(void) { return host::last_error().c_str(); }

int emu_run_photons(const mcrt_grid* grid, const void* rho, const mcrt_optics* optics, int n_src,
                    const mcrt_source* sources, int n_det, const mcrt_detector* detectors, const mcrt_opts* opts,
                    double* images, long long n_images, double* absorbed, long long n_absorbed, mcrt_stats* stats,
                    int wave) {
  try {
    g_violation.clear();
    host::last_error().clear();
    if (!opts) return host::fail(MCRT_EINVAL, "opts is NULL");
    return life_dispatch<false>(opts->precision == MCRT_PREC_FP32, grid_kind(grid), n_det, detectors, false, grid,
                                rho, optics, n_src, sources, n_det, detectors, opts, images, n_images, absorbed,
                                n_absorbed,
                                (const double*)nullptr, 0ll, (double*)nullptr, 0ll, (double*)nullptr,
                                (const double*)nullptr, stats, wave);
  } catch (const Violation& v) {
    g_violation = std::string("run_photons: ") + v.what();
    return -100;
  }
}

int emu_backward_density(const mcrt_grid* grid, const void* rho, const mcrt_optics* optics, int n_src,
                         const mcrt_source* sources, int n_det, const mcrt_detector* detectors, const mcrt_opts* opts,
                         const double* adj, long long n_adj, double* grad, long long n_grad, double* gopt,
                         const double* adj_abs, mcrt_stats* stats, int wave) {
  try {
    g_violation.clear();
    host::last_error().clear();
    if (!opts) return host::fail(MCRT_EINVAL, "opts is NULL");
    mcrt_opts o = *opts;
    o.flags &= ~MCRT_ABSORB;
    if (o.flags & MCRT_ATTACHED) {
      if (gopt || adj_abs)
        return host::fail(MCRT_EINVAL, "MCRT_ATTACHED: the attached gradient is that of the densities only");
      const int kind = grid_kind(grid);
      const bool f32 = o.precision == MCRT_PREC_FP32;
      if (kind == kGridRect)
        return f32 ? emu_attached<float, kGridRect>(grid, rho, optics, n_src, sources, n_det, detectors, &o, adj, n_adj,
                                                    grad, n_grad, stats)
                   : emu_attached<double, kGridRect>(grid, rho, optics, n_src, sources, n_det, detectors, &o, adj,
                                                     n_adj, grad, n_grad, stats);
      if (kind == kGridTree)
        return f32 ? emu_attached<float, kGridTree>(grid, rho, optics, n_src, sources, n_det, detectors, &o, adj, n_adj,
                                                    grad, n_grad, stats)
                   : emu_attached<double, kGridTree>(grid, rho, optics, n_src, sources, n_det, detectors, &o, adj,
                                                     n_adj, grad, n_grad, stats);
      return f32 ? emu_attached<float, kGridRegular>(grid, rho, optics, n_src, sources, n_det, detectors, &o, adj,
                                                     n_adj, grad, n_grad, stats)
                 : emu_attached<double, kGridRegular>(grid, rho, optics, n_src, sources, n_det, detectors, &o, adj,
                                                      n_adj, grad, n_grad, stats);
    }
    return life_dispatch<true>(o.precision == MCRT_PREC_FP32, grid_kind(grid), n_det, detectors,
                               gopt != nullptr || adj_abs != nullptr, grid, rho, optics,
                               n_src, sources,
                               n_det, detectors, (const mcrt_opts*)&o, (double*)nullptr, 0ll, (double*)nullptr, 0ll,
                               adj, n_adj, grad, n_grad, gopt, adj_abs, stats, wave);
  } catch (const Violation& v) {
    g_violation = std::string("backward_density: ") + v.what();
    return -100;
  }
}

// Checks the library's absorbed-tally layout on grid (precision, brick
// shape as in a run): every bricked cell's slot lies in [0, ntal), no two
// cells share one, tally_cell inverts tally_slot, a cell keeps its place
// inside its unit, and the unit count is a power of two.  Returns ntal and
// the unit bits.
int emu_tally_layout(const mcrt_grid* grid, int precision, int brick_shape, int64_t* ntal, int* tb) {
  try {
    g_violation.clear();
    host::last_error().clear();
    GridDev G{};
    if (int e = host::make_grid(*grid, host::elem_bytes(precision), brick_shape, G)) return e;
    const long long unit = 1ll << G.tb, units = G.ntal / unit;
    EMU_CHECK(G.tb >= 3 && G.tb >= G.lb[0] + G.lb[1] + G.lb[2], "unit bits", G.tb, 32);
    EMU_CHECK(units * unit == G.ntal && (units & (units - 1)) == 0, "unit count", units, G.ntal);
    EMU_CHECK(G.ntal >= G.ncell_pad && G.ntal < 2 * ((long long)G.ncell_pad + unit), "tally slots", G.ntal,
              2 * ((long long)G.ncell_pad + unit));
    std::vector<unsigned char> seen((size_t)G.ntal, 0);
    for (int c = 0; c < G.ncell_pad; ++c) {
      const long long t = tally_slot(G, c);
      EMU_CHECK(t >= 0 && t < G.ntal, "tally slot", t, G.ntal);
      EMU_CHECK(!seen[(size_t)t], "tally slot taken twice", t, G.ntal);
      seen[(size_t)t] = 1;
      EMU_CHECK(tally_cell(G, t) == c, "tally_cell of the slot", c, G.ncell_pad);
      EMU_CHECK((t & (unit - 1)) == (c & (unit - 1)), "place inside the unit", c, unit);
    }
    *ntal = G.ntal;
    *tb = G.tb;
    return 0;
  } catch (const Violation& v) {
    g_violation = std::string("tally layout: ") + v.what();
    return -100;
  }
}

int emu_trace_path(const mcrt_grid* grid, const void* rho, double kappa, int precision, int64_t n_rays,
                   const double* origin, const double* dir, double* tau, int32_t max_seg, int32_t* seg_cell,
                   double* seg_len, int32_t* n_seg, uint64_t* crossings, int brick_shape, int wave) {
  try {
    g_violation.clear();
    host::last_error().clear();
    if (int e = host::check_trace(grid, rho, kappa, precision, n_rays, origin, dir, tau, max_seg, seg_cell, seg_len))
      return e;
    if (n_rays == 0) {
      if (crossings) *crossings = 0;
      return 0;
    }
    return trace_dispatch(precision == MCRT_PREC_FP32, grid_kind(grid), grid, rho, kappa, n_rays, origin, dir,
                          tau, max_seg, seg_cell, seg_len, n_seg, crossings, brick_shape, wave);
  } catch (const Violation& v) {
    g_violation = std::string("trace_path: ") + v.what();
    return -100;
  }
}

int emu_peel_off(const mcrt_grid* grid, const void* rho, double kappa, double g, int precision, int64_t n_events,
                 const double* pos, const double* dir_in, const double* w, int n_det, const mcrt_detector* detectors,
                 double* images, int brick_shape, int wave) {
  try {
    g_violation.clear();
    host::last_error().clear();
    if (int e = host::check_peel(grid, rho, kappa, g, precision, n_events, pos, w, n_det, detectors, images))
      return e;
    if (n_events == 0) return 0;
    return peel_dispatch(precision == MCRT_PREC_FP32, grid_kind(grid), grid, rho, kappa, g, n_events, pos,
                         dir_in, w, n_det, detectors, images, brick_shape, wave);
  } catch (const Violation& v) {
    g_violation = std::string("peel_off: ") + v.what();
    return -100;
  }
}

int emu_dust_emission(const mcrt_grid* grid, const void* rho, int precision, int n_abs, const double* absorbed,
                      int n_lambda, const double* lambda, const double* dlambda, const double* kappa_abs,
                      double emissivity, double* temperature, double* emission) {
  try {
    g_violation.clear();
    host::last_error().clear();
    if (int e = host::check_dust(grid, rho, precision, n_abs, absorbed, n_lambda, lambda, dlambda, kappa_abs,
                                 emissivity, emission))
      return e;
    DustParams P;
    std::memset(&P, 0, sizeof P);
    if (int e = host::make_grid(*grid, host::elem_bytes(precision), 0, P.G)) return e;
    HostPlanes planes;
    planes.attach(*grid, P.G);
    std::vector<double> a(n_lambda), b(n_lambda), lnP(kDustTable + 1);
    host::dust_constants(n_lambda, lambda, dlambda, kappa_abs, a.data(), b.data());
    P.D.nl = n_lambda;
    P.D.a = a.data();
    P.D.b = b.data();
    for (int k = 0; k <= kDustTable; ++k) lnP[k] = dust_table_entry(P.D, k);
    P.D.lnP = lnP.data();
    P.rho = rho;
    P.absorbed = absorbed;
    P.n_abs = n_abs;
    P.emissivity = emissivity;
    P.temperature = temperature;
    P.emission = emission;
    const bool f32 = precision == MCRT_PREC_FP32;
    for (int m = 0; m < P.G.ncell; ++m) {
      if (P.G.kind == kGridTree)
        f32 ? dust_cell<float, kGridTree>(P, m) : dust_cell<double, kGridTree>(P, m);
      else if (P.G.kind == kGridRect)
        f32 ? dust_cell<float, kGridRect>(P, m) : dust_cell<double, kGridRect>(P, m);
      else
        f32 ? dust_cell<float, kGridRegular>(P, m) : dust_cell<double, kGridRegular>(P, m);
    }
    return 0;
  } catch (const Violation& v) {
    g_violation = std::string("dust_emission: ") + v.what();
    return -100;
  }
}

}  // extern "C"
