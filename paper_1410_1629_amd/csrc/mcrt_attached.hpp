// mcrt_attached.hpp -- the attached (pathwise) density gradient: one work
// item (package x wavelength) per lane, a forward sweep that runs the
// package's life cycle and keeps its events, then a reverse sweep over them.
//
// Method: Camps & Baes (arXiv:1410.1629), Sect. 1 (peel-off at emission and
// scattering; forced scattering), Sect. 2.2 (cells of constant density),
// Sect. 2.3 (kappa, albedo, g).  The paper differentiates nothing; this is
// the derivative of the same estimator with its random numbers held fixed.
//
// The random numbers fix every direction (each one the previous one turned by
// drawn angles); the positions move with the densities through the
// forced-scattering step.  Event n sits at r_n with weight w_n; the leg after
// it runs along k_n with optical depth T_n to the boundary, draws
//   tau_s = -ln(1 - u (1 - e^-T_n)),
// and stops after the length s_n at which the optical depth from r_n reaches
// tau_s: r_{n+1} = r_n + s_n k_n, w_{n+1} = w_n albedo (1 - e^-T_n).  A
// peel-off contribution of event n is C = w_n Phi e^-tau_peel(r_n) / D^2, with
// the direction and distance of a frame's or SED instrument's distant
// observer (cameras are not supported: their geometry moves with r_n).  With
// q = (dL/dI) C and the loss the sum of q, the reverse sweep carries lbar
// (adjoint of ln w_n) and rbar (adjoint of r_n) from the last event back:
//   each q of event n:  lbar += q;  dL/drho -= q kappa l along the peel ray;
//                       rbar -= q dtau_peel/dr_n
//   the leg from event n-1 to event n:
//     sbar = rbar . k,  taubar = sbar / (kappa rho_s)   (rho_s: density at r_n)
//     Tbar = taubar e^(tau_s - T) (1 - e^-tau_s)/(1 - e^-T) + lbar e^-T/(1 - e^-T)
//     dL/drho += Tbar kappa l (the whole leg) - (sbar / rho_s) l (the leg up to s)
//     rbar += Tbar dT/dr - taubar dtau(r, k, s)/dr    (s fixed; lbar unchanged)
// The derivative of a ray's optical depth with respect to its origin comes
// from its crossings: moving the origin by dr moves the crossing of a plane
// normal to axis a by -dr_a / k_a, where the optical depth changes by
// kappa (rho_before - rho_after) (after the last cell: rho_after = 0).  Pixel
// choices, the escape test (T = 0) and the termination test stay fixed: the
// result is the derivative of the per-package estimator where it is smooth.
//
// The sweeps run in FP64 (R = double) whatever the densities' storage: the
// derivative amplifies the rounding of a point's position wherever a leg
// grazes a cell face (a term 1/k_a), and on rough media (neighbouring cells
// differing by factors of several) a package's derivative changes over
// density changes of 1e-9 relative -- FP32 walks, which move the points by
// 1e-7, would not follow it.  The forward sweep repeats the FP64 life
// cycle's arithmetic (the same draws, walks and locate test), so with FP64
// densities it follows the forward run's packages exactly.  It keeps, per
// event, [kAttF] doubles in the workspace [event][field][chunk item]; the
// host sizes the event dimension by the most events a package can have.
#pragma once

#include "mcrt_lane.hpp"

namespace mcrt {

enum AttField : int { AF_RX = 0, AF_RY, AF_RZ, AF_W, AF_KX, AF_KY, AF_KZ, AF_T, AF_TAUS, AF_S, AF_RHOS, kAttF };

// Crossings, walks and counts of one lane.
struct AttCounts {
  double s_abs = 0.0, s_esc = 0.0, s_trunc = 0.0;
  unsigned long long x_path = 0, x_loc = 0, x_peel = 0, n_ev = 0, n_pk = 0, n_pl = 0, n_dep = 0;
  unsigned long long x_dep = 0;  // crossings of the peel rays' deposit walks (part of x_peel; no density loads)
};

// Lowest axis in a 3-bit mask, or -1.
MCRT_HD int att_axis(unsigned m) { return (m & 1u) ? 0 : ((m & 2u) ? 1 : ((m & 4u) ? 2 : -1)); }

// One walk from o along k to the grid's boundary, with FP64 times, as the
// life-cycle walks; returns the optical depth.
// DEP: deposits dep_full l, plus dep_part l for the part of each segment
// before t_cut (a time from o), into the gradient.  GRAD: adds to g the
// derivative of the optical depth with respect to o, each crossing's term
// weighted by w_before (crossing before t_cut) or w_after.  A zero-length
// segment is skipped: the crossings on either side of it happen at once, and
// their plane is taken as the lowest axis among them.
template <typename R, bool GRAD, bool DEP, class Mem>
MCRT_HD R att_walk(const GridDev& G, Mem& M, const double o[3], const double k[3], double kap, double t_cut,
                   double dep_full, double dep_part, double w_before, double w_after, double g[3],
                   unsigned long long& nx) {
  Ray<R, double> ry;
  ray_begin<R, Mem::kGrid>(ry, G, o, k);
  const R kapR = (R)kap;
  const double tc = t_cut - ry.tin;  // in the walk's times (from the grid entry)
  unsigned pmask = 0;  // planes of the crossing at the end of the last segment
  R prho = R(0);
  double pt = 0.0;
  while (ry.active) {
    WalkBlock<kBlockWalk, R, double> b;
    ray_next_block(ry, b, G, M);
    // sub-steps past b.n (the last valid cell repeated) are masked rather
    // than skipped, so that the block's density loads stay in flight together
#pragma unroll
    for (int d = 0; d < kBlockWalk; ++d) {
      const unsigned m = (b.adv >> (3 * d)) & 7u;  // 0 past b.n
      const double tm = b.tend[d];
      const R s0 = (R)(tm - ry.t);
      const bool pos = d < b.n && s0 > R(0);
      const R seg = pos ? s0 : R(0);
      const R rs = b.rho[d];
      if (pos) {
        if (GRAD) {
          const int a = att_axis(pmask);
          if (a >= 0) g[a] -= (pt < tc ? w_before : w_after) * kap * ((double)prho - (double)rs) / k[a];
        }
        if (DEP) {
          double v = dep_full * (double)seg;
          if (ry.t < tc) v += dep_part * (fmin(tm, tc) - ry.t);
          M.add_grad(b.cell[d], v);
        }
        ++nx;
        prho = rs;
        pt = tm;
        pmask = m;
      } else {
        pmask |= m;
      }
      ry.tau += pos ? kapR * rs * seg : R(0);
      if (pos) ry.t = tm;
    }
    if (b.out) ry.active = false;
  }
  if (GRAD) {  // leaving the grid: the density after the last crossing is 0
    const int a = att_axis(pmask);
    if (a >= 0) g[a] -= (pt < tc ? w_before : w_after) * kap * (double)prho / k[a];
  }
  return ry.tau;
}

// The deposit walk of a peel ray: w l into every cell crossed (no density
// loads).
template <typename R, class Mem>
MCRT_HD void att_deposit(const GridDev& G, Mem& M, const double o[3], const double k[3], double w,
                         unsigned long long& nx) {
  Ray<R, double> ry;
  ray_begin<R, Mem::kGrid>(ry, G, o, k);
  while (ry.active) {
    WalkBlock<kBlockWalk, R, double> b;
    ray_next_block<kBlockWalk, R, Mem, false>(ry, b, G, M);
#pragma unroll
    for (int d = 0; d < kBlockWalk; ++d) {
      if (d >= b.n) break;
      const R seg = (R)(b.tend[d] - ry.t);
      if (seg > R(0)) {
        M.add_grad(b.cell[d], w * (double)seg);
        ++nx;
        ry.t = b.tend[d];
      }
    }
    if (b.out) ry.active = false;
  }
}

// The locate walk of the life cycle: the length s from o along k at which the
// optical depth reaches tau_s, and the density of that cell; when rounding
// leaves tau_s beyond the walk's total, the end of the last absorbing
// segment.
template <typename R, class Mem>
MCRT_HD void att_locate(const GridDev& G, Mem& M, const double o[3], const double k[3], double kap, double tau_s,
                        double& s, R& rho_s, unsigned long long& nx) {
  Ray<R, double> ry;
  ray_begin<R, Mem::kGrid>(ry, G, o, k);
  const R kapR = (R)kap, tau_sR = (R)tau_s;
  double last_t = ry.t;
  int last_cell = ry.active ? ray_cell(ry, G) : 0;
  while (ry.active) {
    WalkBlock<kBlockWalk, R, double> b;
    ray_next_block(ry, b, G, M);
    // every sub-step's depth first (past b.n: none) and whether the point
    // lies in this block, a test that needs all of the block's density loads,
    // so they are in flight together; a block without the point is taken
    // whole, the block with it step by step
    R dtau[kBlockWalk];
    bool pos[kBlockWalk];
    double t_run = ry.t;
    R run = ry.tau;
    bool hit = false;
#pragma unroll
    for (int d = 0; d < kBlockWalk; ++d) {
      const R s0 = (R)(b.tend[d] - t_run);
      pos[d] = d < b.n && s0 > R(0);
      dtau[d] = pos[d] ? kapR * b.rho[d] * s0 : R(0);
      hit = hit || (pos[d] && run + dtau[d] > tau_sR);
      run += dtau[d];
      if (pos[d]) t_run = b.tend[d];
    }
    if (!hit) {
#pragma unroll
      for (int d = 0; d < kBlockWalk; ++d) {
        nx += pos[d];
        if (dtau[d] > R(0)) {
          last_cell = b.cell[d];
          last_t = b.tend[d];
        }
      }
      ry.tau = run;
      ry.t = t_run;
    } else {
#pragma unroll
      for (int d = 0; d < kBlockWalk; ++d) {
        if (d >= b.n) break;
        const double tm = b.tend[d];
        const R rs = b.rho[d];
        nx += pos[d];
        if (pos[d] && ry.tau + dtau[d] > tau_sR) {
          ray_rewind<kBlockWalk, R, Mem::kGrid>(ry, b, d, G);
          const double tp = ray_cell_entry64<R, Mem::kGrid>(ry, G, o, k);
          s = tp + (tau_s - (double)ry.tau) / (kap * (double)rs);
          rho_s = rs;
          return;
        }
        if (dtau[d] > R(0)) {
          last_cell = b.cell[d];
          last_t = tm;
        }
        ry.tau += dtau[d];
        if (pos[d]) ry.t = tm;
      }
    }
    if (b.out) ry.active = false;
  }
  s = ry.tin + last_t;
  rho_s = M.rho(last_cell);
}

// The attached gradient of work item `item` (chunk slot `slot`).  Workspace
// accessors: M.att_st(slot, e, f, v), M.att_ld(slot, e, f); M.att_over() when
// a package has more events than the workspace keeps (the host's bound makes
// that impossible; the package's gradient is then skipped).
template <typename R, class Mem>
MCRT_HD void attached_item(const RunParams& P, Mem& M, unsigned long long item, int slot, AttCounts& cnt) {
  const GridDev& G = P.G;
  const int lam = (int)(item / P.n_pkg);
  const unsigned long long pkg = P.first + (item - (unsigned long long)lam * P.n_pkg);
  const LamDev& LD = M.lam(lam);
  ++cnt.n_pk;
  if (LD.ltot == 0.0) return;
  const double kap = LD.kappa, alb = LD.albedo, g = LD.g, w0 = LD.w0;

  // forward sweep: emission, then legs and scatterings as the life cycle
  double r[3], k[3];
  {
    const U4 wd = draw_words(P.seed, pkg, (unsigned)lam, 1u);
    int s = P.n_src - 1;
    const double target = u01(wd.z) * LD.ltot;
    for (int q = 0; q < P.n_src; ++q) {
      if (target < LD.cum[q]) {
        s = q;
        break;
      }
    }
    iso_direction(u01(wd.x), u01(wd.y), k);
    const SrcDev& S = M.src(s);
    const U4 wp = draw_words(P.seed, pkg, (unsigned)lam, 0u);
    if (S.kind == 2)
      cell_source_position<Mem::kGrid>(S, G, lam, wp, r);
    else
      source_position(S, wp, r);
  }
  double W = w0;
  int n = 0;
  M.att_st(slot, 0, AF_RX, r[0]);
  M.att_st(slot, 0, AF_RY, r[1]);
  M.att_st(slot, 0, AF_RZ, r[2]);
  M.att_st(slot, 0, AF_W, W);
  double none[3] = {0.0, 0.0, 0.0};
  for (;;) {
    const double T = (double)att_walk<R, false, false>(G, M, r, k, kap, 0.0, 0.0, 0.0, 0.0, 0.0, none, cnt.x_path);
    if (T == 0.0) {
      cnt.s_esc += W;
      break;
    }
    cnt.s_abs += W * (1.0 - alb) * (-expm1(-T));
    cnt.s_esc += W * exp(-T);
    const U4 ws = draw_words(P.seed, pkg, (unsigned)lam, 2u + (unsigned)n);
    const double tau_s = -log1p(u01(ws.x) * expm1(-T));
    double s;
    R rho_s;
    att_locate<R>(G, M, r, k, kap, tau_s, s, rho_s, cnt.x_loc);
    if (n + 1 >= P.ev_max) {  // beyond the workspace: the package's gradient is skipped
      M.att_over();
      return;
    }
    M.att_st(slot, n, AF_KX, k[0]);
    M.att_st(slot, n, AF_KY, k[1]);
    M.att_st(slot, n, AF_KZ, k[2]);
    M.att_st(slot, n, AF_T, T);
    M.att_st(slot, n, AF_TAUS, tau_s);
    M.att_st(slot, n, AF_S, s);
    M.att_st(slot, n, AF_RHOS, (double)rho_s);
    r[0] += s * k[0];
    r[1] += s * k[1];
    r[2] += s * k[2];
    W *= alb * (-expm1(-T));
    ++n;
    ++cnt.n_ev;
    M.att_st(slot, n, AF_RX, r[0]);
    M.att_st(slot, n, AF_RY, r[1]);
    M.att_st(slot, n, AF_RZ, r[2]);
    M.att_st(slot, n, AF_W, W);
    if (W < P.w_min * w0 || n >= P.max_scatter) {
      cnt.s_trunc += W;
      break;
    }
    turn(k, hg_sample_mu(g, u01(ws.y)), u01(ws.z));
  }

  // reverse sweep
  double lbar = 0.0, rb[3] = {0.0, 0.0, 0.0};
  for (int e = n; e >= 0; --e) {
    const double re[3] = {M.att_ld(slot, e, AF_RX), M.att_ld(slot, e, AF_RY), M.att_ld(slot, e, AF_RZ)};
    if (P.flags & (e == 0 ? kFlagPeelEmit : kFlagPeelScat)) {
      const double We = M.att_ld(slot, e, AF_W);
      double kin[3] = {0.0, 0.0, 0.0};
      if (e > 0) {
        kin[0] = M.att_ld(slot, e - 1, AF_KX);
        kin[1] = M.att_ld(slot, e - 1, AF_KY);
        kin[2] = M.att_ld(slot, e - 1, AF_KZ);
      }
      const int comp = ((P.flags & kFlagSplit) && e > 0) ? 1 : 0;
      for (int d = 0; d < P.n_det; ++d) {
        const DetDev& D = M.det(d);
        const int pix = frame_pixel<true>(D, re);
        if (pix < 0) continue;
        const long long ii = ((long long)comp * P.n_lambda + lam) * P.pix_lambda + D.off + pix;
        const double A = M.adj(ii);
        if (A == 0.0) continue;
        const double ph =
            e == 0 ? 1.0 / (4.0 * kPi) : hg_phase(g, kin[0] * D.kd[0] + kin[1] * D.kd[1] + kin[2] * D.kd[2]);
        double gp[3] = {0.0, 0.0, 0.0};
        const double tau = e > 0 ? (double)att_walk<R, true, false>(G, M, re, D.kd, kap, INFINITY, 0.0, 0.0, 1.0,
                                                                    1.0, gp, cnt.x_peel)
                                 : (double)att_walk<R, false, false>(G, M, re, D.kd, kap, INFINITY, 0.0, 0.0, 0.0,
                                                                     0.0, gp, cnt.x_peel);
        const double q = A * We * ph * exp(-tau) * D.inv_d2;
        ++cnt.n_pl;
        if (q == 0.0) continue;
        lbar += q;
        rb[0] -= q * gp[0];
        rb[1] -= q * gp[1];
        rb[2] -= q * gp[2];
        // the deposit walk: queued for the peel-job kernels (sorted, summed
        // on chip), or walked here when the queue is full or absent
        if (!M.queue_deposit(D, d, re, pix, -q * kap, ii, (unsigned)slot, e, (unsigned)lam)) {
          unsigned long long nd = 0;
          att_deposit<R>(G, M, re, D.kd, -q * kap, nd);
          cnt.x_peel += nd;
          cnt.x_dep += nd;
          cnt.n_dep += nd;
        }
      }
    }
    if (e == 0) break;
    // the leg from event e-1 to event e
    const int f = e - 1;
    const double kl[3] = {M.att_ld(slot, f, AF_KX), M.att_ld(slot, f, AF_KY), M.att_ld(slot, f, AF_KZ)};
    const double rp[3] = {M.att_ld(slot, f, AF_RX), M.att_ld(slot, f, AF_RY), M.att_ld(slot, f, AF_RZ)};
    const double T = M.att_ld(slot, f, AF_T), tau_s = M.att_ld(slot, f, AF_TAUS);
    const double s = M.att_ld(slot, f, AF_S), rho_s = M.att_ld(slot, f, AF_RHOS);
    const double sbar = rb[0] * kl[0] + rb[1] * kl[1] + rb[2] * kl[2];
    const double taubar = sbar / (kap * rho_s);
    const double Tbar = (taubar * exp(tau_s - T) * -expm1(-tau_s) + lbar * exp(-T)) / -expm1(-T);
    unsigned long long nd = 0;
    if (f > 0) {
      double gl[3] = {0.0, 0.0, 0.0};
      att_walk<R, true, true>(G, M, rp, kl, kap, s, Tbar * kap, -sbar / rho_s, Tbar - taubar, Tbar, gl, nd);
      rb[0] += gl[0];
      rb[1] += gl[1];
      rb[2] += gl[2];
    } else {  // the emission point does not move
      att_walk<R, false, true>(G, M, rp, kl, kap, s, Tbar * kap, -sbar / rho_s, 0.0, 0.0, none, nd);
    }
    cnt.x_path += nd;
    cnt.n_dep += nd;
  }
}

}  // namespace mcrt
