// mcrt_lane.hpp -- per-lane logic of the life-cycle, trace and peel-off
// kernels: the package state machine and the walk step.
//
// Method: Camps & Baes (arXiv:1410.1629), Sect. 1 (photon packages; peel-off
// at emission and scattering, Yusef-Zadeh et al. 1984; continuous absorption,
// Lucy 1999, Niccolini et al. 2003; forced scattering, Cashwell & Everett
// 1959), Sect. 2.1 (multiple anisotropic scattering), Sect. 2.2 (cells of
// constant properties, geometries, parallel-projection frames, direct and
// scattered light recorded separately), Sect. 2.3 (kappa, albedo, g).
//
// A lane owns one package at a time.  Its state machine (lane_events) runs
// the events of the package -- emission, peel-off towards each frame, the
// pass-1 walk with continuous absorption, the pass-2 walk that locates the
// forced-scattering point, peel-off at the scattering, termination or HG
// turn -- and stops whenever the next event needs a walk through the grid,
// leaving a ray set up in `ry`.  lane_step advances that ray by one cell and
// does the per-crossing work of its mode.  The kernel interleaves the two
// across the lanes of a wavefront; the CPU test harness runs them lane by
// lane.  All memory goes through the accessor M:
//   M.rho(cell)  M.det(d)  M.lam(l)  M.src(s)  M.adj(i)
//   M.add_image(i, v)  M.add_absorbed(i, v)  M.add_grad(cell, v)
//   M.walk_deposit<ADJ>(d, i, v)   (sub-step d's deposit of a walk block)
//   M.fetch()  M.flush_counts(x_path, x_locate, x_peel, deposits)
//   M.job_slot()  M.store_job(slot, ...)   (peel-ray queue)
//   M.ev_load(slot, e, k)  M.ev_store(slot, e, k, v)   (adjoint event scratch)
//   M.opt_store(slot, ga, gg, gl, src)   (pass B sums for the optics gradients)
// Cells are bricked addresses (GridDev): densities, the gradient and dL/dA
// (wavelength-major, ncell_pad per wavelength) are in the bricked layout
// inside the library; the forward's absorbed tally is wavelength-major with
// ntal slots per wavelength, cell c at tally_slot(c).
//
// Adjoint (ADJ = true): the detached derivative of C, a peel-off contribution
// of event e, with respect to the density of cell m is
//   C [ sum_{i<=e} (delta(m, c_i)/rho_m - kappa l_m(leg_i)) - kappa l_m(peel) ]
// (c_i: cell of scattering i; leg_i: path from event i-1 to it).  With
// A = dL/dI at C's pixel, q = A C for one peel ray and G_e the sum of q over
// the frames for event e, the gradient collects, per package,
// R_i = sum_{e>=i} G_e on leg i and on c_i, and -q kappa l along each peel
// ray.  The adjoint runs on chunks of packages in two replays of each
// package, as two launches of the life-cycle kernel (P.split):
//   split 1 (pass A): the package's events; each peel ray goes to the queue
//     of peel jobs (or, with the queue full, is walked here: once for C,
//     and again to deposit -q kappa l); T of every leg and q of every walked
//     peel ray go to the event scratch;
//   the peel-job kernel walks the queued rays (sorted into bundles of
//     parallel neighbours) for C, writes q to the scratch, and walks each
//     ray with q != 0 again to deposit;
//   split 2 (pass B): the package again with R_1 = sum of its q and
//     R_i = R_1 - sum_{e<i} G_e, depositing along the locate walks; G_e and T
//     come from the scratch (events beyond it walk their peel rays and paths
//     again, without deposits).
#pragma once

#pragma once

#include "mcrt_device.hpp"

namespace mcrt {

constexpr int kFlagPeelEmit = 1, kFlagPeelScat = 2, kFlagAbsorb = 4, kFlagSplit = 8;

enum RayMode : int { M_PEEL = 0, M_PATH = 1, M_LOCATE = 2, M_PEEL_DEP = 3 };
enum Phase : int {
  PH_FETCH = 0,
  PH_EMIT,
  PH_PEEL_NEXT,
  PH_PEEL_END,
  PH_PEEL_DEP_END,
  PH_PATH_START,
  PH_PATH_END,
  PH_LOCATE_END,
  PH_TERM,
  PH_PKG_END
};

// A queued peel ray: from r towards frame d of event e (saturated at
// kEventSat) of chunk package `slot`, with v = W Phi / D^2 (so its
// contribution is C = v e^-tau), ii its index in the image block (the pixel
// it adds to, or the dL/dI it is weighted with) and lam its wavelength.
// key is its first sort key (tile_key); the device queue keeps both sort
// keys in RunParams::keys, the second one (sort_sub) outside the ray.
constexpr int kEventSat = 65535;
struct PeelJob {
  double r[3];
  double v;
  long long ii;
  unsigned key, slot, lam;
  unsigned short e;
  unsigned char d;
};

// Depth bits the adjoint's queued rays drop (RunParams::depth_drop).
// Measured with the tape (spiral, 1e7 packages): deposit walks 23.6 ms with 4
// depth bits, 26.0 with 6 and 26.0 with none; the forward's peel walks on
// the clumpy 512^3 disk (1e8 packages): 1063 ms with none, 716 / 645 / 611 ms
// with 4 / 5 / 6.
constexpr int kDepthDropAdjoint = 2;

struct RunParams {
  GridDev G;
  const void* rho;
  const LamDev* lam;
  const DetDev* det;
  const SrcDev* src;
  int n_lambda, n_src, n_det, comps;
  unsigned long long first, n_pkg, seed, n_items;
  double w_min;
  int max_scatter;
  unsigned flags;
  long long pix_lambda;
  double* images;
  double* absorbed;
  const double* adj;
  double* grad;
  unsigned long long* work;    // next work item (wavelength-major)
  double* dstats;              // absorbed, escaped, truncated
  unsigned long long* xstats;  // x_path, x_locate, x_peel, events, packages, peels, deposits
  int batch;
  // adjoint (ADJ): the launch's role and its chunk of work items
  int split;                   // 1: pass A, 2: pass B
  unsigned long long item0, n_chunk;  // work items [item0, item0 + n_chunk)
  PeelJob* jobs;               // forward run and pass A: queue of peel rays (NULL: walk every peel ray here)
  unsigned* keys;              // the device queue's sort keys, one word per ray: key | sub << 16
  unsigned long long job_cap;  // its capacity; rays beyond it are walked here
  int ev_max;                  // events kept per package in the event scratch
  int ev_k;                    // doubles per event: T of the leg after it, then q per frame
  double* evs;                 // event scratch [ev_max][ev_k][n_chunk], then q beyond ev_max [n_chunk]
  // pass B, when the optics and luminosity gradients are wanted: per package
  // of the chunk sum q n, sum q (score in g), sum q and its source index,
  // [4][n_chunk] (null: not wanted)
  double* gpart;
  // adjoint of a loss on the absorbed tally: dL/dA, bricked [n_lambda][ncell_pad]
  // (null: none); its path sums B sit in the event scratch's last entry
  const double* adj_abs;
  // forward run with an adjoint tape (null: none): T of the leg after event
  // e and C per frame, [tape_ev][1 + n_det][tape_n], and the image index of
  // each C, [tape_ev][n_det][tape_n], for the call's work items; tape_over
  // is set when a package has more events than the tape keeps
  double* tape;
  unsigned* tape_pix;
  unsigned* tape_over;
  int tape_ev;
  unsigned long long tape_n;
  // adjoint from a tape: pass B finds every q and T in the event scratch
  // (filled from the tape) and queues the deposit walks of the event's peel
  // rays with q != 0 (walked here when the queue is full)
  int dep_jobs;
  // low bits of the queued rays' depth keys cleared (sort_sub): 0 in the
  // forward run, 2 in the adjoint, whose deposit walks sum into LDS
  int depth_drop;
};

// The life-cycle walks keep their times in FP64 whatever R is (see Ray).
template <typename R>
struct Lane {
  Ray<R, double> ry;
  int phase;
  bool done;
  unsigned long long pkg;
  int lam, det, n, pix, mode;
  bool is_emit, found;
  double r[3], k[3];
  double W, w0, kap, alb, g, T, tau_s, wabs;
  R kapR, tau_sR, absf, trans, tau_prev, rho_hit;
  R tau_c;        // compensation of the walk's optical-depth sum (Kahan)
  double last_t;  // end of the last absorbing segment of a locate walk (ray time)
  unsigned uw1, uw2;
  int hit_cell, last_cell;
  long long lam_cell;  // the package's wavelength row of the absorbed tally: lam * ntal
  // adjoint replay
  int pass;
  int slot;  // the lane's index in the event scratch
  double Rtot, Gacc, Gabs, fac, Ge;
  bool t_kept;  // pass B: T of the next leg is in the scratch
  int src;      // source of the package
  double Sg, Ga, Gg, GL;  // pass B, optics gradients: score of the sampled directions; sums over q
  double Babs, Pabs;      // absorbed-tally adjoint: B of the current path, its running part P
  bool abs_dep;           // pass B: this path walk deposits the absorbed-tally terms
  // statistics
  double s_abs, s_esc, s_trunc;
  unsigned x_path, x_loc, x_peel, n_ev, n_pk, n_pl, n_dep;
};

template <typename R>
MCRT_HD void lane_init(Lane<R>& L) {
  L.ry.active = false;
  L.ry.tau = R(0);
  L.ry.t = R(0);
  L.ry.tin = 0.0;
  L.phase = PH_FETCH;
  L.done = false;
  L.pkg = 0;
  L.lam = L.det = L.n = L.pix = 0;
  L.mode = M_PEEL;
  L.is_emit = true;
  L.found = false;
  for (int a = 0; a < 3; ++a) L.r[a] = L.k[a] = 0.0;
  L.k[2] = 1.0;
  L.W = L.w0 = L.kap = L.alb = L.g = L.T = L.tau_s = L.wabs = 0.0;
  L.kapR = L.tau_sR = L.absf = L.tau_prev = L.rho_hit = R(0);
  L.last_t = 0.0;
  L.tau_c = R(0);
  L.trans = R(1);
  L.uw1 = L.uw2 = 0;
  L.hit_cell = L.last_cell = 0;
  L.lam_cell = 0;
  L.pass = 0;
  L.slot = 0;
  L.Rtot = L.Gacc = L.Gabs = L.fac = L.Ge = 0.0;
  L.t_kept = false;
  L.src = 0;
  L.Sg = L.Ga = L.Gg = L.GL = 0.0;
  L.Babs = L.Pabs = 0.0;
  L.abs_dep = false;
  L.s_abs = L.s_esc = L.s_trunc = 0.0;
  L.x_path = L.x_loc = L.x_peel = L.n_ev = L.n_pk = L.n_pl = L.n_dep = 0;
}

// Adjoint bookkeeping of one event (emission or scattering n = L.n): its
// peel-off contributions q sum to G_e.  Pass B takes the q the scratch holds
// for the event and skips its peel-offs; events beyond the scratch walk
// their peel rays again.  Called once the event's next phase is set: events
// without peel-off (the flags exclude it) have G_e = 0.
// Peel-off geometry for accessor Mem: the camera path only where the run
// has instruments other than frames (Mem::kInst), else the distant
// observer's.
template <class Mem>
MCRT_HD void peel_geom(const DetDev& D, const double r[3], double kd[3], double& inv_d2, double& tmax) {
  if constexpr (Mem::kInst) {
    peel_geometry(D, r, kd, inv_d2, tmax);
  } else {
    for (int a = 0; a < 3; ++a) kd[a] = D.kd[a];
    inv_d2 = D.inv_d2;
    tmax = INFINITY;
  }
}

// Pass B of a run with optics gradients: a peel-off contribution q of the
// current event towards frame d.  The event's scattering count n, its
// direction scores so far and its peel phase give q's factors: n (albedo),
// the score in g, and 1 (the source's luminosity).
template <typename R, class Mem>
MCRT_HD void optics_add(Lane<R>& L, Mem& M, int d, double q) {
  L.Ga += q * (double)L.n;
  L.GL += q;
  if (!L.is_emit) {
    double kd[3], inv_d2, tmax;
    peel_geom<Mem>(M.det(d), L.r, kd, inv_d2, tmax);
    L.Gg += q * (L.Sg + hg_dlng(L.g, L.k[0] * kd[0] + L.k[1] * kd[1] + L.k[2] * kd[2]));
  }
}

template <typename R, class Mem>
MCRT_HD void event_start(Lane<R>& L, const RunParams& P, Mem& M) {
  L.Ge = 0.0;
  if (L.pass == 1 && L.n < P.ev_max && L.phase == PH_PEEL_NEXT) {
    for (int d = 0; d < P.n_det; ++d) {
      const double q = M.ev_load(L.slot, L.n, 1 + d);
      L.Ge += q;
      if (Mem::kInst && P.gpart && q != 0.0) optics_add(L, M, d, q);
    }
    if (!P.dep_jobs) L.det = P.n_det;  // no peel-off walks: PEEL_NEXT goes straight on
  }
}

template <typename R, class Mem>
MCRT_HD void event_done(Lane<R>& L, const RunParams& P, Mem& M) {
  L.Gacc += L.Ge;
  L.Ge = 0.0;
}

// Pass A keeps q of a walked peel ray for pass B: per frame for the first
// ev_max events, summed beyond.
template <typename R, class Mem>
MCRT_HD void keep_q(Lane<R>& L, const RunParams& P, Mem& M, double q) {
  if (L.n < P.ev_max)
    M.ev_store(L.slot, L.n, 1 + L.det, q);
  else
    M.ev_add_beyond(L.slot, q);
}

// Runs the lane's events until its next walk is set up (ry.active) or no
// work is left (done).  Each pass goes once through the phase blocks in the
// order in which a package usually moves through them -- end of a peel-off
// walk, end of the pass-1 walk, end of the locate walk, next frame,
// termination or turn, next pass-1 walk, end of package, new package -- so
// a lane whose walk just ended normally reaches its next walk within one
// pass, and the lanes of a wavefront that are at different events share
// the pass instead of taking turns.  The walk itself is set up once, at the
// end of the pass, from the origin, direction and mode the blocks chose.
template <typename R, bool ADJ, class Mem>
MCRT_HD void lane_events(Lane<R>& L, const RunParams& P, Mem& M) {
  const GridDev& G = P.G;
  while (!L.ry.active && !L.done) {
    bool want = false;  // a walk is to be set up at the end of this pass
    bool to_det = false;  // towards frame L.det (else along the package direction)

    // -- end of a peel-off walk: the contribution, then the next frame
    if (L.phase == PH_PEEL_END) {
      const DetDev& D = M.det(L.det);
      double kd[3], inv_d2, tmax;
      peel_geom<Mem>(D, L.r, kd, inv_d2, tmax);
      const double ph = L.is_emit ? 1.0 / (4.0 * kPi)
                                  : hg_phase(L.g, L.k[0] * kd[0] + L.k[1] * kd[1] + L.k[2] * kd[2]);
      const double C = L.W * ph * exp(-(double)L.ry.tau) * inv_d2;
      const int comp = ((P.flags & kFlagSplit) && !L.is_emit) ? 1 : 0;
      const long long ii = ((long long)comp * P.n_lambda + L.lam) * P.pix_lambda + D.off + L.pix;
      if (L.pass == 0) ++L.n_pl;
      L.phase = PH_PEEL_NEXT;
      if (!ADJ) {
        M.add_image(ii, C);
        if (P.tape) M.tape_peel(L.slot, L.n, L.det, C, ii);
        ++L.det;
      } else {
        const double ac = M.adj(ii) * C;
        L.Ge += ac;
        if (L.pass == 0) keep_q(L, P, M, ac);
        if (Mem::kInst && L.pass == 1 && P.gpart && ac != 0.0) optics_add(L, M, L.det, ac);
        if (L.pass == 0 && ac != 0.0) {  // a second walk of the same ray deposits -A C kappa l
          L.fac = -ac * L.kap;
          want = to_det = true;
          L.mode = M_PEEL_DEP;
          L.phase = PH_PEEL_DEP_END;
        } else {
          ++L.det;
        }
      }
    }
    if (ADJ && L.phase == PH_PEEL_DEP_END && !want) {
      ++L.det;
      L.phase = PH_PEEL_NEXT;
    }

    // -- end of the pass-1 walk: escape and absorption, forced-scattering depth
    if (ADJ && Mem::kInst && L.phase == PH_PATH_END && P.adj_abs && !want) {
      if (L.pass == 0) {  // keep the path's B for pass B
        if (L.n < P.ev_max)
          M.ev_store(L.slot, L.n, P.ev_k - 1, L.Babs);
        else if (L.Babs != 0.0)
          M.ev_add_beyond(L.slot, L.Babs);
      } else if (!L.abs_dep && L.Babs != 0.0) {  // beyond the scratch: B known now, walk again to deposit
        L.abs_dep = true;
        L.Pabs = 0.0;
        L.absf = R(0);
        L.trans = R(1);
        want = true;
        L.mode = M_PATH;
      }
    }
    if (L.phase == PH_PATH_END && !want) {
      if (ADJ && L.pass == 1) L.Gacc += L.Babs;  // the path's B joins this event's contributions
      if (ADJ && L.t_kept) {
        L.T = M.ev_load(L.slot, L.n, 0);
        L.t_kept = false;
      } else {
        L.T = (double)L.ry.tau;
        if (ADJ && L.pass == 0 && L.n < P.ev_max) M.ev_store(L.slot, L.n, 0, L.T);
        if (!ADJ && P.tape) M.tape_leg(L.slot, L.n, L.T);
      }
      if (L.T == 0.0) {  // nothing to interact with: the package leaves
        if (L.pass == 0) L.s_esc += L.W;
        L.phase = PH_PKG_END;
      } else {
        if (L.pass == 0) {
          // the leg's absorbed fraction: the sum of its deposits, which
          // telescopes to 1 - e^-T, taken so when no tally is kept
          L.s_abs += L.wabs * ((!ADJ && !P.absorbed) ? -expm1(-L.T) : (double)L.absf);
          L.s_esc += L.W * exp(-L.T);
        }
        const U4 ws = draw_words(P.seed, L.pkg, (unsigned)L.lam, 2u + (unsigned)L.n);
        L.tau_s = -log1p(u01(ws.x) * expm1(-L.T));
        L.tau_sR = (R)L.tau_s;
        L.uw1 = ws.y;
        L.uw2 = ws.z;
        if (ADJ && L.pass == 1) L.fac = -(L.Rtot - L.Gacc) * L.kap;
        want = true;
        L.mode = M_LOCATE;
        L.found = false;
        L.phase = PH_LOCATE_END;
      }
    }

    // -- end of the locate walk: move to the interaction point, update the weight
    if (L.phase == PH_LOCATE_END && !want) {
      double s;
      if (L.found) {
        const double tp = ray_cell_entry64<R, Mem::kGrid>(L.ry, G, L.r, L.k);
        s = tp + (L.tau_s - (double)L.tau_prev) / (L.kap * (double)L.rho_hit);
        if (ADJ && L.pass == 1) {
          const double Ri = L.Rtot - L.Gacc;
          M.add_grad(L.hit_cell, Ri / (double)L.rho_hit - Ri * L.kap * (s - tp));
          ++L.n_dep;
        }
      } else {  // tau_s reached the total by rounding: end of the last absorbing segment
        s = L.ry.tin + L.last_t;
        if (ADJ && L.pass == 1) {
          M.add_grad(L.last_cell, (L.Rtot - L.Gacc) / (double)M.rho(L.last_cell));
          ++L.n_dep;
        }
      }
      L.r[0] += s * L.k[0];
      L.r[1] += s * L.k[1];
      L.r[2] += s * L.k[2];
      L.W *= L.alb * (-expm1(-L.T));
      ++L.n;
      if (L.pass == 0) ++L.n_ev;
      L.is_emit = false;
      L.det = 0;
      L.phase = (P.flags & kFlagPeelScat) ? PH_PEEL_NEXT : PH_TERM;
      if (ADJ) event_start(L, P, M);
    }

    // -- the next frame whose pixel the event projects into
    if (L.phase == PH_PEEL_NEXT && !want) {
      bool dep_inline = false;  // pass B from a tape: a deposit walk the full queue could not take
      while (L.det < P.n_det) {
        const DetDev& D = M.det(L.det);
        if (ADJ && P.dep_jobs && L.pass == 1 && L.n < P.ev_max) {  // the event's nonzero q: deposit walks
          const double q = M.ev_load(L.slot, L.n, 1 + L.det);
          if (q != 0.0) {
            L.pix = frame_pixel<Mem::kInst>(D, L.r);
            const unsigned long long slot = P.jobs ? M.job_slot() : P.job_cap;
            if (slot >= P.job_cap) {
              L.fac = -q * L.kap;
              dep_inline = true;
              break;
            }
            const int comp = ((P.flags & kFlagSplit) && !L.is_emit) ? 1 : 0;
            const long long ii = ((long long)comp * P.n_lambda + L.lam) * P.pix_lambda + D.off + L.pix;
            const int kp = key_pixel<Mem::kInst>(D, L.r, L.pix);
            M.store_job(slot, L.r, -q * L.kap, ii, tile_key(D, kp), sort_sub(D, kp, L.r, P.depth_drop), (unsigned)L.slot,
                        L.n < kEventSat ? L.n : kEventSat, L.det, (unsigned)L.lam);
          }
          ++L.det;
          continue;
        }
        L.pix = frame_pixel<Mem::kInst>(D, L.r);
        if (L.pix >= 0) {
          if (!P.jobs || L.pass != 0) break;
          const unsigned long long slot = M.job_slot();
          if (slot >= P.job_cap) break;  // queue full: walk it here
          // queued: C = v e^-tau is completed by the queue's walk kernel
          double kd[3], inv_d2, tmax;
          peel_geom<Mem>(D, L.r, kd, inv_d2, tmax);
          const double ph = L.is_emit ? 1.0 / (4.0 * kPi)
                                      : hg_phase(L.g, L.k[0] * kd[0] + L.k[1] * kd[1] + L.k[2] * kd[2]);
          const int comp = ((P.flags & kFlagSplit) && !L.is_emit) ? 1 : 0;
          const long long ii = ((long long)comp * P.n_lambda + L.lam) * P.pix_lambda + D.off + L.pix;
          const int kp = key_pixel<Mem::kInst>(D, L.r, L.pix);
          M.store_job(slot, L.r, L.W * ph * inv_d2, ii, tile_key(D, kp), sort_sub(D, kp, L.r, P.depth_drop), (unsigned)L.slot,
                      L.n < kEventSat ? L.n : kEventSat, L.det,
                      (unsigned)L.lam);
          ++L.n_pl;
        }
        ++L.det;
      }
      if (L.det < P.n_det) {
        want = to_det = true;
        L.mode = dep_inline ? M_PEEL_DEP : M_PEEL;
        L.phase = dep_inline ? PH_PEEL_DEP_END : PH_PEEL_END;
      } else {
        if (ADJ) event_done(L, P, M);
        L.phase = L.is_emit ? PH_PATH_START : PH_TERM;
      }
    }

    // -- termination, or a new direction from the HG phase function
    if (L.phase == PH_TERM && !want) {
      if (L.W < P.w_min * L.w0 || L.n >= P.max_scatter) {
        if (L.pass == 0) L.s_trunc += L.W;
        L.phase = PH_PKG_END;
      } else {
        const double mu = hg_sample_mu(L.g, u01(L.uw1));
        if (ADJ && Mem::kInst && L.pass == 1 && P.gpart) L.Sg += hg_dlng(L.g, mu);
        turn(L.k, mu, u01(L.uw2));
        L.phase = PH_PATH_START;
      }
    }

    // -- the pass-1 walk along the package direction
    if (L.phase == PH_PATH_START && !want) {
      L.absf = R(0);
      L.trans = R(1);
      L.wabs = L.W * (1.0 - L.alb);
      L.phase = PH_PATH_END;
      if (ADJ) {  // absorbed-tally adjoint: pass A sums B; pass B deposits with B known
        L.Babs = (Mem::kInst && P.adj_abs && L.pass == 1 && L.n < P.ev_max) ? M.ev_load(L.slot, L.n, P.ev_k - 1)
                                                                              : 0.0;
        L.Pabs = 0.0;
        L.abs_dep = L.Babs != 0.0;
      }
      if (ADJ && L.pass == 1 && L.n < P.ev_max) {
        L.t_kept = true;  // T of this leg is in the scratch: no walk unless it deposits
        if (!L.abs_dep) continue;
      }
      want = true;
      L.mode = M_PATH;
    }

    // -- end of the package: replay it for the adjoint, or take the next one
    if (L.phase == PH_PKG_END && !want) {
      if (ADJ && Mem::kInst && L.pass == 1 && P.gpart) {  // the package's sums for the optics gradients
        M.opt_store(L.slot, L.Ga, L.Gg, L.GL, L.src);
      }
      L.phase = PH_FETCH;
    }
    if (L.phase == PH_FETCH && !want) {
      if ((L.x_path | L.x_loc | L.x_peel | L.n_dep) & 0xC0000000u) {  // keep 32-bit counters from wrapping
        M.flush_counts(L.x_path, L.x_loc, L.x_peel, L.n_dep);
        L.x_path = L.x_loc = L.x_peel = L.n_dep = 0;
      }
      const unsigned long long k = M.fetch();
      if (k >= P.n_chunk) {
        L.done = true;
      } else {
        const unsigned long long item = P.item0 + k;
        L.slot = (int)k;
        L.lam = (int)(item / P.n_pkg);
        L.pkg = P.first + (item - (unsigned long long)L.lam * P.n_pkg);
        L.lam_cell = (long long)L.lam * G.ntal;
        const LamDev& LD = M.lam(L.lam);
        L.kap = LD.kappa;
        L.kapR = (R)L.kap;
        L.alb = LD.albedo;
        L.g = LD.g;
        L.w0 = LD.w0;
        L.pass = 0;
        L.Gacc = L.Gabs = 0.0;
        L.phase = PH_EMIT;
        if (ADJ && P.split == 2) {  // pass B: R_1 is the sum of the package's q; none, no replay
          double R1 = 0.0, Rabs = 0.0;
          for (int e = 0; e < P.ev_max; ++e)
            for (int d = 0; d < P.n_det; ++d) {
              const double q = M.ev_load(L.slot, e, 1 + d);
              R1 += q;
              Rabs += fabs(q);
            }
          if (Mem::kInst && P.adj_abs)
            for (int e = 0; e < P.ev_max; ++e) {
              const double q = M.ev_load(L.slot, e, P.ev_k - 1);
              R1 += q;
              Rabs += fabs(q);
            }
          const double qb = M.ev_load_beyond(L.slot);
          R1 += qb;
          Rabs += fabs(qb);
          L.pass = 1;
          L.Rtot = R1;
          if (Rabs == 0.0) {
            L.phase = PH_FETCH;
            continue;
          }
        }
        if (LD.ltot == 0.0) {  // nothing is emitted at this wavelength: the package ends unborn
          if (L.pass == 0) ++L.n_pk;
          L.phase = PH_FETCH;
          continue;
        }
      }
    }
    // -- emission (also the start of the adjoint replay)
    if (L.phase == PH_EMIT && !want && !L.done) {
      const LamDev& LD = M.lam(L.lam);
      const U4 wd = draw_words(P.seed, L.pkg, (unsigned)L.lam, 1u);
      int s = P.n_src - 1;
      const double target = u01(wd.z) * LD.ltot;
      for (int q = 0; q < P.n_src; ++q) {
        if (target < LD.cum[q]) {
          s = q;
          break;
        }
      }
      iso_direction(u01(wd.x), u01(wd.y), L.k);
      const SrcDev& S = M.src(s);
      L.src = s;
      if (ADJ) L.Sg = L.Ga = L.Gg = L.GL = 0.0;
      const U4 wp = draw_words(P.seed, L.pkg, (unsigned)L.lam, 0u);
      if (S.kind == 2)
        cell_source_position<Mem::kGrid>(S, G, L.lam, wp, L.r);
      else
        source_position(S, wp, L.r);
      L.W = L.w0;
      L.n = 0;
      if (L.pass == 0) ++L.n_pk;
      L.is_emit = true;
      L.det = 0;
      L.phase = (P.flags & kFlagPeelEmit) ? PH_PEEL_NEXT : PH_PATH_START;
      if (ADJ) event_start(L, P, M);
    }

    // -- set up the chosen walk (a walk that misses the grid ends at once and
    //    its end is handled in the next pass)
    if (want) {
      double kd[3], inv_d2, tmax = INFINITY;
      if (to_det) peel_geom<Mem>(M.det(L.det), L.r, kd, inv_d2, tmax);
      ray_begin<R, Mem::kGrid>(L.ry, G, L.r, to_det ? kd : L.k, tmax);
      L.tau_c = R(0);
      if (L.mode == M_LOCATE) {
        L.last_cell = ray_cell(L.ry, G);
        L.last_t = L.ry.t;
      }
    }
  }
}

// Walk block size: crossings per step of a lane, and density loads each
// lane keeps in flight.
constexpr int kBlockWalk = 4;

// A walk block's deposits -- forward: absorbed luminosity into the tally;
// adjoint: the walk's gradient terms (the locate leg's -R kappa l, an inline
// peel ray's -A C kappa l, the absorbed-tally terms) into the gradient -- go
// through M.walk_deposit<ADJ>(d, i, v), one per sub-step d at most.  The
// kernel stages them in LDS and issues them for the whole wavefront at once,
// transposed so that one walker's deposits -- neighbouring cells, often in
// one segment of the bricked array -- sit in adjacent lanes of one atomic
// instruction; the CPU harness applies them at once, in order.

// Up to kBlockWalk crossings of the lane's active ray, with the per-crossing
// work of its mode: pass-1 continuous absorption W (1 - albedo) e^-tau
// (1 - e^-dtau) into the cell; pass-2 search for the first segment whose
// optical depth passes tau_s (and, in the adjoint replay, -R kappa l deposits
// along the leg); peel rays accumulate tau (and, on the deposit walk,
// -A C kappa l).  Zero-length segments are skipped.  Returns whether the block
// made a deposit.
template <typename R, bool ADJ, class Mem>
MCRT_HD bool lane_step(Lane<R>& L, const RunParams& P, Mem& M) {
  auto& ry = L.ry;
  bool put = false;
  WalkBlock<kBlockWalk, R, double> b;
  ray_next_block(ry, b, P.G, M);
#pragma unroll
  for (int d = 0; d < kBlockWalk; ++d) {
    if (d >= b.n) break;
    const double tm = (Mem::kInst && b.tend[d] > ry.tmax) ? ry.tmax : b.tend[d];  // a peel walk to a camera stops there
    R seg = (R)(tm - ry.t);  // one rounding of an FP64 difference
    const bool pos = seg > R(0);
    seg = pos ? seg : R(0);
    const R rs = b.rho[d];
    const int cell = b.cell[d];
    const R dtau = L.kapR * rs * seg;
    if (L.mode == M_PATH) {
      L.x_path += pos;
      if (ADJ && Mem::kInst && P.adj_abs && dtau > R(0)) {
        // absorbed-tally adjoint: deposit dep = W (1 - albedo) e^-tau (1 - e^-dtau) weighted by b;
        // pass B also deposits -kappa l (B - P) + b W (1 - albedo) e^-tau e^-dtau kappa l
        const R em = expm1(-dtau);
        const double bj = M.adj_abs((long long)L.lam * P.G.ncell_pad + cell);
        const double da = L.wabs * (double)(-L.trans * em);
        if (L.abs_dep) {
          L.Pabs += bj * da;
          const double kl = L.kap * (double)seg;
          M.template walk_deposit<ADJ>(d, cell, -kl * (L.Babs - L.Pabs) + bj * L.wabs * (double)(L.trans * (R(1) + em)) * kl);
          put = true;
          ++L.n_dep;
        } else {
          L.Babs += bj * da;
        }
        L.trans += L.trans * em;
      }
      if (!ADJ && P.absorbed && dtau > R(0)) {
        // deposit e^-tau (1 - e^-dtau) with e^-tau carried along the walk
        // (without a tally nothing is summed: the leg's end takes 1 - e^-T)
        const R em = expm1(-dtau);
        const R f = -L.trans * em;
        L.trans += L.trans * em;
        L.absf += f;
        M.template walk_deposit<ADJ>(d, L.lam_cell + tally_slot(P.G, cell), L.wabs * (double)f);
        put = true;
        ++L.n_dep;
      }
    } else if (L.mode == M_LOCATE) {
      L.x_loc += pos;
      if (pos && ry.tau + dtau > L.tau_sR) {
        L.found = true;
        L.hit_cell = cell;
        L.tau_prev = ry.tau;
        L.rho_hit = rs;
        ray_rewind<kBlockWalk, R, Mem::kGrid>(ry, b, d, P.G);
        ry.active = false;
        return put;
      }
      if (dtau > R(0)) {
        L.last_cell = cell;
        L.last_t = tm;
      }
      if (ADJ && L.pass == 1 && pos) {
        M.template walk_deposit<ADJ>(d, cell, L.fac * (double)seg);
        put = true;
        ++L.n_dep;
      }
    } else {
      L.x_peel += pos;
      if (ADJ && L.mode == M_PEEL_DEP && pos) {
        M.template walk_deposit<ADJ>(d, cell, L.fac * (double)seg);
        put = true;
        ++L.n_dep;
      }
    }
    if constexpr (sizeof(R) == sizeof(float)) {  // FP32 sum compensated (Kahan): the leg's optical
      const R y = dtau - L.tau_c;                   // depth sets the forced-scattering point
      const R t = ry.tau + y;
      L.tau_c = (t - ry.tau) - y;
      ry.tau = t;
    } else {
      ry.tau += dtau;
    }
    if (pos) ry.t = tm;
  }
  if (b.out || (Mem::kInst && ry.t >= ry.tmax)) ry.active = false;
  return put;
}

// ---------------------------------------------------------------------------
// Queued peel rays (the peel-job kernels).  tau_step is the walk the inline
// M_PEEL mode makes -- same setup, segments and order of the optical-depth
// sum, without the inline mode's compensation of FP32 sums -- and bp_step
// the walk of the inline M_PEEL_DEP mode without density loads (its
// deposits w l do not depend on the densities); every deposit goes through
// M.deposit(cell, v).  Each advances the ray by one block and returns its
// positive-length crossings.  INST = false (frames only) compiles out the
// stop at a camera inside the grid.
//
// Crossings per step of the optical-depth walk: on regular grids eight
// (clumpy 512^3 disk, forward peel walks 510 -> 480 ms; spiral 32.3 -> 31.3),
// on rectilinear ones four (PowCub spiral 43.9 ms, 45.7 with eight).
template <int GK>
constexpr int kPeelBlock = GK == kGridRegular ? 8 : kBlockWalk;
template <typename R, class Mem, bool INST = true, typename T = R>
MCRT_HD unsigned tau_step(Ray<R, T>& ry, const GridDev& G, R kap, Mem& M) {
  constexpr int D = kPeelBlock<Mem::kGrid>;
  WalkBlock<D, R, T> b;
  ray_next_block(ry, b, G, M);
  unsigned n = 0;
  // Every sub-step is evaluated: with a branch per sub-step the compiler
  // moves each density load into its branch, and the block's loads then wait
  // for one another instead of being in flight together.  Sub-steps past b.n
  // repeat the last valid cell and end time, so their segments have no
  // positive length and add nothing.
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const T tm = (INST && b.tend[d] > ry.tmax) ? ry.tmax : b.tend[d];
    const R seg = (R)(tm - ry.t);
    const bool pos = seg > R(0);
    const R dtau = pos ? kap * b.rho[d] * seg : R(0);
    n += pos;
    ry.tau += dtau;
    if (pos) ry.t = tm;
  }
  if (b.out || (INST && ry.t >= ry.tmax)) ry.active = false;
  return n;
}

template <typename R, class Mem, bool INST = true, typename T = R>
MCRT_HD unsigned bp_step(Ray<R, T>& ry, const GridDev& G, double w, Mem& M) {
  WalkBlock<kBlockWalk, R, T> b;
  ray_next_block<kBlockWalk, R, Mem, false>(ry, b, G, M);
  unsigned n = 0;
#pragma unroll
  for (int d = 0; d < kBlockWalk; ++d) {
    if (d >= b.n) break;
    const T tm = (INST && b.tend[d] > ry.tmax) ? ry.tmax : b.tend[d];
    const R seg = (R)(tm - ry.t);
    if (seg > R(0)) {
      M.deposit(b.cell[d], w * (double)seg);
      ++n;
      ry.t = tm;
    }
  }
  if (b.out || (INST && ry.t >= ry.tmax)) ry.active = false;
  return n;
}

// ---------------------------------------------------------------------------
// trace_path and peel_off: one ray per work item.

struct TraceParams {
  GridDev G;
  const void* rho;
  double kappa;
  long long n_rays;
  const double* origin;
  const double* dir;
  double* tau;
  int max_seg;
  int* seg_cell;
  double* seg_len;
  int* n_seg;
  unsigned long long* work;
  unsigned long long* counters;  // [0] segments, [1] rays over max_seg
  int batch;
};

template <typename R>
struct TraceLane {
  Ray<R> ry;
  bool done, pending;
  long long q;
  int nseg;
  unsigned long long total, overflow;
};

template <typename R>
MCRT_HD void trace_init(TraceLane<R>& L) {
  L.ry.active = false;
  L.ry.tau = R(0);
  L.done = L.pending = false;
  L.q = 0;
  L.nseg = 0;
  L.total = L.overflow = 0;
}

// Finishes the lane's ray (if any) and sets up the next one.
template <typename R, class Mem>
MCRT_HD void trace_events(TraceLane<R>& L, const TraceParams& P, Mem& M) {
  while (!L.ry.active && !L.done) {
    if (L.pending) {
      M.set_tau(L.q, (double)L.ry.tau);
      M.set_nseg(L.q, L.nseg);
      L.total += (unsigned long long)L.nseg;
      L.overflow += (unsigned long long)(P.seg_cell != nullptr && L.nseg > P.max_seg);
      L.pending = false;
    }
    const unsigned long long item = M.fetch();
    if (item >= (unsigned long long)P.n_rays) {
      L.done = true;
      break;
    }
    L.q = (long long)item;
    double o[3], k[3];
    M.ray(L.q, o, k);
    L.nseg = 0;
    L.pending = true;
    ray_begin<R, Mem::kGrid>(L.ry, P.G, o, k);
  }
}

template <typename R, class Mem>
MCRT_HD void trace_step(TraceLane<R>& L, const TraceParams& P, Mem& M) {
  Ray<R>& ry = L.ry;
  WalkBlock<kBlockWalk, R> b;
  ray_next_block(ry, b, P.G, M);
  const R kap = (R)P.kappa;
#pragma unroll
  for (int d = 0; d < kBlockWalk; ++d) {
    if (d >= b.n) break;
    R seg = b.tend[d] - ry.t;
    const bool pos = seg > R(0);
    seg = pos ? seg : R(0);
    if (pos) {
      if (P.seg_cell != nullptr && L.nseg < P.max_seg) M.store_seg(L.q, L.nseg, b.cell[d], (double)seg);
      ++L.nseg;
      ry.t = b.tend[d];
    }
    ry.tau += kap * b.rho[d] * seg;
  }
  if (b.out) ry.active = false;
}

struct PeelParams {
  GridDev G;
  const void* rho;
  double kappa, g;
  long long n_events;
  int n_det;
  const DetDev* det;
  const double* pos;
  const double* dir_in;
  const double* w;
  double* images;
  unsigned long long* work;
  int batch;
};

template <typename R>
struct PeelLane {
  Ray<R> ry;
  bool done, pending;
  long long e;
  int d, pix;
};

template <typename R>
MCRT_HD void peel_init(PeelLane<R>& L) {
  L.ry.active = false;
  L.ry.tau = R(0);
  L.done = L.pending = false;
  L.e = 0;
  L.d = L.pix = 0;
}

template <typename R, class Mem>
MCRT_HD void peel_events(PeelLane<R>& L, const PeelParams& P, Mem& M) {
  const unsigned long long n_items = (unsigned long long)P.n_events * (unsigned long long)P.n_det;
  while (!L.ry.active && !L.done) {
    if (L.pending) {
      const DetDev& D = M.det(L.d);
      double r[3], kd[3], inv_d2, tmax, kin[3];
      M.position(L.e, r);
      peel_geometry(D, r, kd, inv_d2, tmax);
      double ph = 1.0 / (4.0 * kPi);
      if (M.dir_in(L.e, kin)) ph = hg_phase(P.g, kin[0] * kd[0] + kin[1] * kd[1] + kin[2] * kd[2]);
      M.add_image(D.off + L.pix, M.weight(L.e) * ph * exp(-(double)L.ry.tau) * inv_d2);
      L.pending = false;
    }
    const unsigned long long item = M.fetch();
    if (item >= n_items) {
      L.done = true;
      break;
    }
    L.e = (long long)(item / (unsigned long long)P.n_det);
    L.d = (int)(item - (unsigned long long)L.e * P.n_det);
    double r[3];
    M.position(L.e, r);
    L.pix = frame_pixel(M.det(L.d), r);
    if (L.pix < 0) continue;
    L.pending = true;
    double kd[3], inv_d2, tmax;
    peel_geometry(M.det(L.d), r, kd, inv_d2, tmax);
    ray_begin<R, Mem::kGrid>(L.ry, P.G, r, kd, tmax);
  }
}

template <typename R, class Mem>
MCRT_HD void peel_step(PeelLane<R>& L, const PeelParams& P, Mem& M) {
  Ray<R>& ry = L.ry;
  WalkBlock<kBlockWalk, R> b;
  ray_next_block(ry, b, P.G, M);
  const R kap = (R)P.kappa;
  // sub-steps past b.n masked, not skipped: the block's loads stay in flight together
#pragma unroll
  for (int d = 0; d < kBlockWalk; ++d) {
    const R tm = b.tend[d] > ry.tmax ? ry.tmax : b.tend[d];
    const R seg = tm - ry.t;
    const bool pos = d < b.n && seg > R(0);
    if (pos) ry.t = tm;
    ry.tau += pos ? kap * b.rho[d] * seg : R(0);
  }
  if (b.out || ry.t >= ry.tmax) ry.active = false;
}

}  // namespace mcrt
