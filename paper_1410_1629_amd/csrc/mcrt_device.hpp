// mcrt_device.hpp -- lane-level primitives of the photon-package life cycle:
// counter-based random numbers, the grid walk, sources, the Henyey-Greenstein
// phase function and the frame projection.
//
// Method: Camps & Baes (arXiv:1410.1629).  Sect. 1 names the techniques
// (photon packages, peel-off, continuous absorption, forced scattering);
// Sect. 2.2 the grid of constant-property cells, the geometries and the
// frame instruments with parallel projection; Sect. 2.3 the optical
// properties and the asymmetry parameter g; Fig. 5 the seeded generator.
//
// Precision model.  Package state (position, direction, weight), event
// sampling and all tallies are FP64.  The walk through the cells -- the
// per-crossing work -- runs in the type R: double for the FP64 path, float
// for the FP32 path.  Crossing times are computed per plane from the first
// plane ahead (t = t0 + j * dt with an integer count j), never accumulated,
// and the interaction point of forced scattering is recomputed in FP64 from
// the entry plane of its cell, so FP32 error stays relative to one cell.
//
// Everything here is per lane and compiles for host and device (MCRT_HD):
// the kernels run it on gfx950, and the CPU test harness runs the same code
// with bounds-checked memory accessors.  Memory is reached only through an
// accessor object `M` (M.rho(cell) for densities).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <type_traits>

#define MCRT_HD __host__ __device__ __forceinline__

namespace mcrt {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxSrc = 8;
constexpr int kMaxDet = 8;
// Direction components below this magnitude are treated as parallel to the
// axis: the ray would need more than 1e20 lengths to reach the next plane,
// and FP32 crossing times stay finite for any grid up to 1e15 lengths.
constexpr double kParallel = 1e-20;

// Grid kinds (Table 1(d)): regular Cartesian cells (LinCub), rectilinear
// cells spaced by any rule per axis (PowCub and others), and the leaves of
// a binary space partition (k-d tree; an octree is three binary levels per
// octree level).  Each kernel is compiled once per kind.
constexpr int kGridRegular = 0, kGridRect = 1, kGridTree = 2;
// Deepest tree accepted (the host rejects deeper ones).
constexpr int kMaxTreeDepth = 64;

// A node of a tree grid: split along `axis` at `split` into children
// `child` (lower side) and `child + 1` (upper side), or a leaf (axis < 0)
// whose cell index is `child`.
struct TreeNode {
  double split;
  int axis;
  int child;
};

// Default event batches of the life-cycle kernel (how many of a wavefront's
// lanes wait before it runs their events, when the call leaves event_batch
// at 0).  A wavefront runs its event code for the waiting lanes only, so a
// larger batch runs more events per pass and leaves the walking lanes idle
// longer.  The adjoint's pass B keeps each path's optical depth from pass A
// and walks only the short locate legs, so events dominate it and it gains
// most from a large batch.  Measured on the spiral, PowCub and k-d tree
// workloads (1e7 packages): forward 32 (PowCub -7%, k-d tree -11%, spiral
// unchanged against 16); adjoint 32 / 48 (-19% to -28% against 16 / 16).
// A grid whose densities exceed the 256 MB MALL is walked from HBM, each
// step waits longer, and idle walkers cost more: there the forward takes
// 24 (clumpy 512^3 disk, 1e8 packages: life kernel 1436 ms against 1495 at
// 32, 1432 at 20, 1458 at 28).
constexpr int kBatchForward = 32, kBatchForwardHbm = 24, kBatchPassA = 32, kBatchPassB = 48;
constexpr long long kMallBytes = 256ll << 20;
// The ray kernels -- the peel-queue walks (optical depth, deposit walks) and
// the trace and peel-off entry points -- refill a lane with the next ray once
// this many of the wavefront's lanes have finished: measured on the spiral,
// 48 against 16 saves 4 ms of the forward's queue kernels, 6 ms of the
// adjoint's, and 6% of a trace over 4e6 random rays.  The optical-depth
// walk over a grid whose densities exceed the MALL takes 24 (clumpy 512^3
// disk: 423.5 ms at 16, 20 and 24 against 435.7 at 48; on the spiral 48
// stays best, 30.8 against 31.9 ms at 24).
constexpr int kBatchQueue = 48, kBatchQueueHbm = 24;

// ---------------------------------------------------------------------------
// Problem data, prepared by the host in FP64.

// Cells are stored internally in bricks: blocks of 2^lb[0] x 2^lb[1] x
// 2^lb[2] cells, x fastest inside a brick and bricks x fastest, so that one
// cache line holds a compact block of neighbouring cells and a walk in any
// direction reads several cells per line (row-major storage gives one cell
// per line for every step along y or z).  The caller's arrays stay in the
// row-major layout of the C ABI; the library converts at the boundary.
struct GridDev {
  double lo[3], hi[3], d[3], inv_d[3];
  int n[3];
  int stride[3];  // row-major strides 1, nx, nx*ny
  int ncell;      // nx*ny*nz
  int lb[3];      // log2 of the brick size along each axis
  int nb[3];      // bricks along each axis
  int bstride[3]; // brick strides in cells: 2^(lb0+lb1+lb2), nb0 of them, nb0*nb1 of them
  int ncell_pad;  // cells of the bricked arrays (whole bricks)
  // Grid kind (kGrid*).  Rectilinear grids: the cell-boundary planes of
  // each axis, n[a] + 1 of them, absolute (pa) and relative to the first
  // plane (qd), FP64; regular grids use lo + p d.  Tree grids: the nodes,
  // node 0 the box; the cells are the leaves, stored as a one-dimensional
  // array (n = {cells, 1, 1}, no bricks).
  int kind;
  const double* pa[3];
  const double* qd[3];
  const TreeNode* nodes;
  const double* leaf_box;  // tree grids: per cell lo x y z, hi x y z
  const int* ropes;        // tree grids: per cell and face (-x +x -y +y -z +z) the node across it, -1 outside
  // Layout of the forward's absorbed-luminosity tally (tally_slot): units of
  // 2^tb consecutive bricked cells, ntal cells per wavelength.
  int tb;
  long long ntal;
};

// Slot of bricked cell c in the forward's absorbed-luminosity tally.  The
// tally takes one FP64 atomic per cell crossing, which the memory side
// executes at the channel holding the address, so the busiest channel sets
// the rate.  In the bricked order the cells packages cross most (the dense
// middle of a disk) form short runs at a fixed stride, which can fall on few
// channels; how few depends on where the tally lands in physical memory
// (measured on the spiral: 93-115 ms for the forward life kernel over tally
// offsets of 0-4 MiB).  So units of 2^tb cells -- whole bricks, and at least
// one 64-byte segment -- are scattered over the array by a multiplicative
// permutation (an odd multiplier modulo the power-of-two unit count), which
// spreads any compact region over all channels (80-84 ms at every offset).
// A unit keeps its cells in order, so neighbouring cells still share a
// segment.
constexpr unsigned kTallyMul = 0x9E3779B1u, kTallyMulInv = 0x0E8B2F51u;  // inverses modulo 2^32

MCRT_HD long long tally_slot(const GridDev& G, int c) {
  const unsigned mask = (unsigned)((G.ntal >> G.tb) - 1);
  const unsigned u = ((unsigned)c >> G.tb) * kTallyMul & mask;
  return ((long long)u << G.tb) | (long long)(c & ((1 << G.tb) - 1));
}

// Bricked cell of tally slot t (0 <= t < ntal): the inverse of tally_slot.
MCRT_HD long long tally_cell(const GridDev& G, long long t) {
  const unsigned mask = (unsigned)((G.ntal >> G.tb) - 1);
  const unsigned u = (unsigned)(t >> G.tb) * kTallyMulInv & mask;
  return ((long long)u << G.tb) | (t & ((1ll << G.tb) - 1));
}

// Leaf below node q of a tree grid holding point (px, py, pz), for a ray
// with direction signs (sx, sy, sz): at each split a point on the plane goes
// to the side the ray moves to (the upper side when it moves parallel to
// the plane), the rule of the regular grid's walls.  Returns the leaf's cell
// (-1 for a path deeper than kMaxTreeDepth, which the host rejects).  The
// side is decided on all three axes and then picked by the node's axis, so
// nothing is indexed by a runtime axis.
MCRT_HD int tree_find(const GridDev& G, int q, double px, double py, double pz, int sx, int sy, int sz) {
  for (int depth = 0; depth <= kMaxTreeDepth; ++depth) {
    const TreeNode nd = G.nodes[q];
    if (nd.axis < 0) return nd.child;
    const double sp = nd.split;
    const bool u0 = px > sp || (px == sp && sx >= 0);
    const bool u1 = py > sp || (py == sp && sy >= 0);
    const bool u2 = pz > sp || (pz == sp && sz >= 0);
    const bool up = (nd.axis == 0 && u0) || (nd.axis == 1 && u1) || (nd.axis == 2 && u2);
    q = nd.child + (up ? 1 : 0);
  }
  return -1;
}

// Cell along one axis of a rectilinear grid: the largest c in [0, n - 1]
// with P[c] <= x (0 below the first plane).
MCRT_HD int rect_cell(const double* P, int n, double x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (P[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Bricked address of cell (i0, i1, i2).
MCRT_HD int brick_addr(const GridDev& G, const int i[3]) {
  const int m0 = (1 << G.lb[0]) - 1, m1 = (1 << G.lb[1]) - 1, m2 = (1 << G.lb[2]) - 1;
  return (i[0] >> G.lb[0]) * G.bstride[0] + (i[1] >> G.lb[1]) * G.bstride[1] + (i[2] >> G.lb[2]) * G.bstride[2] +
         ((i[0] & m0) | ((i[1] & m1) << G.lb[0]) | ((i[2] & m2) << (G.lb[0] + G.lb[1])));
}

// The bricked address is a sum of one term per axis (the fine parts occupy
// disjoint bits): term a of index i.  Walk kernels on regular grids keep the
// terms of every index in LDS and add three table entries per cell.
MCRT_HD int brick_axis_term(const GridDev& G, int a, int i) {
  const int sh = a == 0 ? 0 : (a == 1 ? G.lb[0] : G.lb[0] + G.lb[1]);
  return (i >> G.lb[a]) * G.bstride[a] + ((i & ((1 << G.lb[a]) - 1)) << sh);
}

// The terms of a regular grid's three axes in one table (kept in LDS by the
// peel-ray walk kernel): indices -1 .. n[0] of axis 0, then -1 .. n[1] of
// axis 1 and -1 .. n[2] of axis 2, the outer two of each clamped to the edge
// cells (a walk's indices leave their range by at most one, at its last
// crossing, whose address is not used).
constexpr int kLutCells = 4096;
MCRT_HD int lut_cells(const GridDev& G) { return G.n[0] + G.n[1] + G.n[2] + 6; }
MCRT_HD int lut_first(const GridDev& G, int a) { return a == 0 ? 0 : (a == 1 ? G.n[0] + 2 : G.n[0] + G.n[1] + 4); }
MCRT_HD int lut_entry(const GridDev& G, int t) {
  const int a = t < lut_first(G, 1) ? 0 : (t < lut_first(G, 2) ? 1 : 2);
  const int i = t - lut_first(G, a) - 1;
  return brick_axis_term(G, a, i < 0 ? 0 : (i >= G.n[a] ? G.n[a] - 1 : i));
}

// Cell indices of bricked address c; false for padding cells.
MCRT_HD bool brick_cell(const GridDev& G, int c, int i[3]) {
  const int cb = G.lb[0] + G.lb[1] + G.lb[2];
  const int b = c >> cb, off = c & ((1 << cb) - 1);
  const int b0 = b % G.nb[0], t = b / G.nb[0];
  const int b1 = t % G.nb[1], b2 = t / G.nb[1];
  i[0] = (b0 << G.lb[0]) | (off & ((1 << G.lb[0]) - 1));
  i[1] = (b1 << G.lb[1]) | ((off >> G.lb[0]) & ((1 << G.lb[1]) - 1));
  i[2] = (b2 << G.lb[2]) | (off >> (G.lb[0] + G.lb[1]));
  return c >= 0 && c < G.ncell_pad && i[0] < G.n[0] && i[1] < G.n[1] && i[2] < G.n[2];
}

// Row-major index of bricked address c (c must be a grid cell).
MCRT_HD int brick_to_linear(const GridDev& G, int c) {
  int i[3];
  brick_cell(G, c, i);
  return i[0] + i[1] * G.stride[1] + i[2] * G.stride[2];
}

// Instrument kinds.
constexpr int kDetFrame = 0, kDetSed = 1, kDetPerspective = 2;

struct DetDev {
  // frame and SED: kd towards the distant observer; perspective: kd the
  // view axis from the eye towards the target, and half_x, half_y the
  // tangents of the half field of view.  ex, ey: image axes.
  double kd[3], ex[3], ey[3];
  double inv_d2, half_x, half_y, inv_dpx, inv_dpy;  // pixels per unit length (per unit tangent)
  double eye[3];
  int kind;
  int nx, ny;
  long long off;  // offset of this frame inside one wavelength's image block
  // Sort keys of queued peel rays: the tile of 2^tshift x 2^tshift pixels
  // in Morton order, numbered from key_off, then the pixel's Morton index
  // inside its tile (shifted right by sub_shift to at most 8 bits).  Rays of
  // one frame whose keys are close land close together in the image, so
  // they are parallel rays a few cells apart that cross one narrow bundle of
  // cells.
  int tshift, key_off, sub_shift;
  // Width of the grid of sort-key pixels: the image's nx, or for an SED
  // instrument (one image pixel) a virtual kn x kn grid over the projection
  // of the model box (half_x, half_y and inv_dpx, inv_dpy describe it), so
  // that its rays spread over many keys.
  int kn;
  // Depth key of a queued ray: the projection of its origin on kd, from dlo
  // in buckets of 1/dscale over the model box's projection (depth_key).
  double dlo, dscale;
};

// Interleaves the low 16 bits of x (even bits) and y (odd bits).
MCRT_HD unsigned morton2(unsigned x, unsigned y) {
  unsigned v[2] = {x & 0xffffu, y & 0xffffu};
  for (int a = 0; a < 2; ++a) {
    unsigned t = v[a];
    t = (t | (t << 8)) & 0x00ff00ffu;
    t = (t | (t << 4)) & 0x0f0f0f0fu;
    t = (t | (t << 2)) & 0x33333333u;
    t = (t | (t << 1)) & 0x55555555u;
    v[a] = t;
  }
  return v[0] | (v[1] << 1);
}

// Sort key of key pixel `kp` of frame D (key_pixel).
MCRT_HD unsigned tile_key(const DetDev& D, int kp) {
  const int iy = kp / D.kn, ix = kp - iy * D.kn;
  return (unsigned)D.key_off + morton2((unsigned)ix >> D.tshift, (unsigned)iy >> D.tshift);
}

// Second sort key of key pixel `kp`: its place inside its tile.
MCRT_HD unsigned tile_sub(const DetDev& D, int kp) {
  const int iy = kp / D.kn, ix = kp - iy * D.kn;
  const unsigned m = (1u << D.tshift) - 1u;
  return morton2((unsigned)ix & m, (unsigned)iy & m) >> D.sub_shift;
}

// Depth of a peel ray's origin along kd, in 2^kDepthBits buckets over the
// model box: the low bits of its second sort key (sort_sub).  The rays of
// one pixel then run in order of where they start, so the lanes of a
// wavefront that walk one column of cells start a few cells apart and read
// the lines each other has just brought in; in any order they start anywhere
// along the column, and a line is gone from the cache before the next lane
// comes by.  `drop` coarsens the buckets (the low bits are cleared): the
// adjoint's deposit walks sum into an LDS table, where lanes that move in
// step would hit the same entry at once.
constexpr int kDepthBits = 6;
MCRT_HD unsigned depth_key(const DetDev& D, const double r[3], int drop = 0) {
  const double t = ((r[0] * D.kd[0] + r[1] * D.kd[1] + r[2] * D.kd[2]) - D.dlo) * D.dscale;
  return ((unsigned)fmin(fmax(floor(t), 0.0), (double)((1 << kDepthBits) - 1)) >> drop) << drop;
}

// Second sort key of a queued ray at r seen in key pixel kp: its place in
// its tile, then its depth.
MCRT_HD unsigned sort_sub(const DetDev& D, int kp, const double r[3], int drop = 0) {
  return (tile_sub(D, kp) << kDepthBits) | depth_key(D, r, drop);
}

struct SrcDev {
  int kind;  // 0 point, 1 exponential disk, 2 the grid's cells
  double c[3], hr, hz;
  // cells: per wavelength the exclusive prefix sums of the cells'
  // luminosities, ncell + 1 entries (the last one the total)
  const double* cum;
};

struct LamDev {
  double kappa, albedo, g, w0, ltot;
  double cum[kMaxSrc];  // cumulative luminosity over sources
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies and xors under a Weyl-incremented 64-bit key.

struct U4 {
  uint32_t x, y, z, w;
};

MCRT_HD U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = U4{(uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Words of draw number `c` of package p at wavelength index l.
MCRT_HD U4 draw_words(uint64_t seed, uint64_t p, uint32_t l, uint32_t c) {
  return philox4x32_10(U4{(uint32_t)p, (uint32_t)(p >> 32), l, c}, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Uniform deviate strictly inside (0,1): (w + 1/2) 2^-32, exact in FP64.
MCRT_HD double u01(uint32_t w) { return ((double)w + 0.5) * 2.3283064365386963e-10; }

// sin and cos of 2 pi u from one call (one argument reduction for both).
MCRT_HD void sincos2pi(double u, double* s, double* c) { sincos(2.0 * kPi * u, s, c); }

// ---------------------------------------------------------------------------
// Henyey-Greenstein phase function and sampling (g sets the phase function,
// Sect. 2.3), normalised to 1 over the sphere.

MCRT_HD double hg_phase(double g, double mu) {
  const double x = 1.0 + g * g - 2.0 * g * mu;
  return (1.0 - g * g) / (4.0 * kPi * x * sqrt(x));
}

MCRT_HD double hg_sample_mu(double g, double u) {
  if (fabs(g) < 1e-6) return 2.0 * u - 1.0;
  const double f = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
  const double mu = (1.0 + g * g - f * f) / (2.0 * g);
  return fmin(1.0, fmax(-1.0, mu));
}

// Direction at polar cosine mu and azimuth 2 pi u about k, in the
// branch-free orthonormal basis of Duff et al. (JCGT 2017), renormalised.
MCRT_HD void turn(double k[3], double mu, double u) {
  const double s = k[2] >= 0.0 ? 1.0 : -1.0;
  const double a = -1.0 / (s + k[2]);
  const double b = k[0] * k[1] * a;
  const double b1x = 1.0 + s * k[0] * k[0] * a, b1y = s * b, b1z = -s * k[0];
  const double b2x = b, b2y = s + k[1] * k[1] * a, b2z = -k[1];
  const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
  double sp, cp;
  sincos2pi(u, &sp, &cp);
  const double nx = st * (cp * b1x + sp * b2x) + mu * k[0];
  const double ny = st * (cp * b1y + sp * b2y) + mu * k[1];
  const double nz = st * (cp * b1z + sp * b2z) + mu * k[2];
  const double inv = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
  k[0] = nx * inv;
  k[1] = ny * inv;
  k[2] = nz * inv;
}

// ---------------------------------------------------------------------------
// Emission (Table 1(a)): isotropic direction; point or exponential-disk
// position (R ~ Gamma(2, h_R) from the area element, azimuth uniform, z
// Laplace with scale h_z).

MCRT_HD void iso_direction(double u0, double u1, double k[3]) {
  const double mu = 2.0 * u0 - 1.0;
  const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
  double sp, cp;
  sincos2pi(u1, &sp, &cp);
  k[0] = st * cp;
  k[1] = st * sp;
  k[2] = mu;
}

MCRT_HD void source_position(const SrcDev& S, const U4& w, double r[3]) {
  r[0] = S.c[0];
  r[1] = S.c[1];
  r[2] = S.c[2];
  if (S.kind == 1) {
    const double u0 = u01(w.x), u1 = u01(w.y), u2 = u01(w.z), u3 = u01(w.w);
    const double R = -S.hr * log(u0 * u1);
    double sp, cp;
    sincos2pi(u2, &sp, &cp);
    const double z = u3 < 0.5 ? S.hz * log(2.0 * u3) : -S.hz * log(2.0 * (1.0 - u3));
    r[0] += R * cp;
    r[1] += R * sp;
    r[2] += z;
  }
}

// Box of cell m (m = i + nx (j + ny k) on regular and rectilinear grids, the
// leaf's cell on tree grids).
template <int GK>
MCRT_HD void cell_box(const GridDev& G, int m, double lo[3], double hi[3]) {
  if constexpr (GK == kGridTree) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = G.leaf_box[6 * (long long)m + a];
      hi[a] = G.leaf_box[6 * (long long)m + 3 + a];
    }
  } else {
    const int i[3] = {m % G.n[0], (m / G.n[0]) % G.n[1], m / G.n[0] / G.n[1]};
    for (int a = 0; a < 3; ++a) {
      if constexpr (GK == kGridRect) {
        lo[a] = G.pa[a][i[a]];
        hi[a] = G.pa[a][i[a] + 1];
      } else {
        lo[a] = G.lo[a] + (double)i[a] * G.d[a];
        hi[a] = G.lo[a] + (double)(i[a] + 1) * G.d[a];
      }
    }
  }
}

// Emission point of the cell source at wavelength l: the cell c with
// cum[c] <= u0 * total < cum[c + 1] (binary search; cells of zero luminosity
// are never drawn), then the point lo + u (hi - lo) of its box.
template <int GK>
MCRT_HD void cell_source_position(const SrcDev& S, const GridDev& G, int l, const U4& w, double r[3]) {
  const double* cum = S.cum + (long long)l * (G.ncell + 1);
  const double target = u01(w.x) * cum[G.ncell];
  int lo = 0, hi = G.ncell - 1;  // the last c with cum[c] <= target
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cum[mid] <= target)
      lo = mid;
    else
      hi = mid - 1;
  }
  double bl[3], bh[3];
  cell_box<GK>(G, lo, bl, bh);
  const double u[3] = {u01(w.y), u01(w.z), u01(w.w)};
  for (int a = 0; a < 3; ++a) r[a] = bl[a] + u[a] * (bh[a] - bl[a]);
}

// ---------------------------------------------------------------------------
// Dust emission: grains as modified black bodies in radiative equilibrium.
// With a_i = kappa_abs_i dlambda_i lambda_i^-5 and b_i = c2 / lambda_i (c2
// the second radiation constant in um K), a cell of mass M at temperature T
// emits emissivity * M * P(T), P(T) = sum_i a_i / (exp(b_i / T) - 1); P
// rises strictly with T.  The temperature solves P(T) = y, y = L /
// (emissivity M), on [kDustTmin, kDustTmax]: Newton's method on
// ln P(e^x) = ln y, x = ln T, kept inside a bracket taken from a table of
// ln P at kDustTable + 1 equally spaced x (a step that leaves the bracket
// bisects it instead).

constexpr double kC2 = 14387.77;
constexpr double kDustTmin = 1.0, kDustTmax = 1e5;
constexpr int kDustTable = 512;

struct DustDev {
  int nl;
  const double* a;    // [nl]
  const double* b;    // [nl]
  const double* lnP;  // [kDustTable + 1]: ln P(exp(k h)), h = ln(kDustTmax) / kDustTable
};

MCRT_HD double dust_step() { return log(kDustTmax) / kDustTable; }

// P(T) and dP/dlnT.
MCRT_HD void dust_sum(const DustDev& D, double T, double& P, double& dP) {
  P = 0.0;
  dP = 0.0;
  for (int i = 0; i < D.nl; ++i) {
    const double u = D.b[i] / T, em = expm1(u), t = D.a[i] / em;
    P += t;
    dP += t * u * (1.0 + 1.0 / em);
  }
}

// Equilibrium temperature for y > 0 (kDustTmin or kDustTmax where the root
// lies outside).
MCRT_HD double dust_temperature(const DustDev& D, double y) {
  const double ly = log(y), h = dust_step();
  if (!(ly > D.lnP[0])) return kDustTmin;
  if (!(ly < D.lnP[kDustTable])) return kDustTmax;
  int k = 0, hi_k = kDustTable - 1;  // the last k with lnP[k] < ly
  while (k < hi_k) {
    const int mid = (k + hi_k + 1) >> 1;
    if (D.lnP[mid] < ly)
      k = mid;
    else
      hi_k = mid - 1;
  }
  double lo = k * h, hi = (k + 1) * h;
  const double p0 = D.lnP[k], p1 = D.lnP[k + 1];
  double x = std::isfinite(p0) ? lo + (ly - p0) / (p1 - p0) * h : 0.5 * (lo + hi);
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  for (int it = 0; it < 64; ++it) {
    double P, dP;
    dust_sum(D, exp(x), P, dP);
    const double f = log(P) - ly;
    if (f == 0.0) break;
    if (f < 0.0)
      lo = x;
    else
      hi = x;
    double xn = x - f * P / dP;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    const bool last = fabs(xn - x) <= 1e-15 * (1.0 + x) || hi - lo <= 1e-15 * (1.0 + hi);
    x = xn;
    if (last) break;
  }
  return exp(x);
}

MCRT_HD double dust_table_entry(const DustDev& D, int k) {
  double P, dP;
  dust_sum(D, exp(k * dust_step()), P, dP);
  return log(P);
}

struct DustParams {
  GridDev G;
  DustDev D;
  const void* rho;         // [ncell], R
  const double* absorbed;  // [n_abs][ncell]
  int n_abs;
  double emissivity;
  double* temperature;  // [ncell] or null
  double* emission;     // [nl][ncell]
};

// Cell m (row-major, as the caller's arrays): L = its absorbed luminosity,
// M = rho V; T solves emissivity M P(T) = L (T = 0 and no emission if L or
// M is 0), and wavelength i receives L a_i / (exp(b_i / T) - 1) / P(T).
template <typename R, int GK>
MCRT_HD void dust_cell(const DustParams& P, int m) {
  const int nc = P.G.ncell;
  double L = 0.0;
  for (int r = 0; r < P.n_abs; ++r) L += P.absorbed[(long long)r * nc + m];
  double lo[3], hi[3];
  cell_box<GK>(P.G, m, lo, hi);
  const double M = (double)static_cast<const R*>(P.rho)[m] * ((hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]));
  double T = 0.0, scale = 0.0;
  if (L > 0.0 && M > 0.0) {
    T = dust_temperature(P.D, L / (P.emissivity * M));
    double S, dS;
    dust_sum(P.D, T, S, dS);
    scale = S > 0.0 ? L / S : 0.0;
  }
  if (P.temperature) P.temperature[m] = T;
  for (int i = 0; i < P.D.nl; ++i)
    P.emission[(long long)i * nc + m] = scale > 0.0 ? scale * (P.D.a[i] / expm1(P.D.b[i] / T)) : 0.0;
}

// ---------------------------------------------------------------------------
// Instrument projection (Sect. 2.2): pixel index of r, or -1 -- parallel
// projection for frames, the single pixel of an SED instrument, central
// projection through a camera's eye.  INST = false (frames only) compiles
// out the other kinds: the life kernel's event code is sensitive to its size.
template <bool INST = true>
MCRT_HD int frame_pixel(const DetDev& D, const double r[3]) {
  if (INST && D.kind == kDetSed) return 0;  // the whole sky of the observer
  double xp, yp;
  if (INST && D.kind == kDetPerspective) {  // central projection through the eye
    const double d[3] = {r[0] - D.eye[0], r[1] - D.eye[1], r[2] - D.eye[2]};
    const double z = d[0] * D.kd[0] + d[1] * D.kd[1] + d[2] * D.kd[2];
    if (!(z > 0.0)) return -1;
    xp = (d[0] * D.ex[0] + d[1] * D.ex[1] + d[2] * D.ex[2]) / z;
    yp = (d[0] * D.ey[0] + d[1] * D.ey[1] + d[2] * D.ey[2]) / z;
  } else {
    xp = r[0] * D.ex[0] + r[1] * D.ex[1] + r[2] * D.ex[2];
    yp = r[0] * D.ey[0] + r[1] * D.ey[1] + r[2] * D.ey[2];
  }
  const double fx = floor((xp + D.half_x) * D.inv_dpx);
  const double fy = floor((yp + D.half_y) * D.inv_dpy);
  if (!(fx >= 0.0 && fx < (double)D.nx && fy >= 0.0 && fy < (double)D.ny)) return -1;
  return (int)fy * D.nx + (int)fx;
}

// d ln Phi / dg of the Henyey-Greenstein phase function at cosine mu (the
// score in g of a direction drawn from it).
MCRT_HD double hg_dlng(double g, double mu) {
  return -2.0 * g / (1.0 - g * g) - 3.0 * (g - mu) / (1.0 + g * g - 2.0 * g * mu);
}

// The optics and luminosity gradients of wavelength l from the pass-B sums
// of its packages (sum q n, sum q score, sum q per source): dL/dalbedo =
// sum q n / albedo, dL/dg = sum q score, dL/dL_s = sum_{source s} q / L_s
// (0 where albedo or L_s is 0).
MCRT_HD void optics_finish(double sa, double sg, const double* sl, int n_src, double albedo, const double* lum_l,
                           long long lum_stride, double* g_alb, double* g_g, double* g_lum, int l, int nl) {
  if (g_alb) g_alb[l] += albedo > 0.0 ? sa / albedo : 0.0;
  if (g_g) g_g[l] += sg;
  if (g_lum)
    for (int s = 0; s < n_src; ++s) {
      const double L = lum_l[s * lum_stride];
      g_lum[(long long)s * nl + l] += L > 0.0 ? sl[s] / L : 0.0;
    }
}

// Key pixel of an event at r seen in image pixel pix: pix itself, or for an
// SED instrument the virtual pixel of its parallel projection (clamped to
// the virtual grid).
template <bool INST = true>
MCRT_HD int key_pixel(const DetDev& D, const double r[3], int pix) {
  if (!INST || D.kind != kDetSed) return pix;
  const double xp = r[0] * D.ex[0] + r[1] * D.ex[1] + r[2] * D.ex[2];
  const double yp = r[0] * D.ey[0] + r[1] * D.ey[1] + r[2] * D.ey[2];
  const double last = (double)(D.kn - 1);
  const double fx = fmin(fmax(floor((xp + D.half_x) * D.inv_dpx), 0.0), last);
  const double fy = fmin(fmax(floor((yp + D.half_y) * D.inv_dpy), 0.0), last);
  return (int)fy * D.kn + (int)fx;
}

// Peel-off geometry of instrument D for an event at r: the direction of the
// peel ray, the 1/distance^2 factor and the length of the walk -- the
// distant instruments' direction and distance with a walk to the grid's
// boundary, or for a perspective camera the direction to the eye, its
// distance and a walk that stops at the eye.
MCRT_HD void peel_geometry(const DetDev& D, const double r[3], double kd[3], double& inv_d2, double& tmax) {
  if (D.kind == kDetPerspective) {
    const double v[3] = {D.eye[0] - r[0], D.eye[1] - r[1], D.eye[2] - r[2]};
    const double d2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double inv = 1.0 / sqrt(d2);
    for (int a = 0; a < 3; ++a) kd[a] = v[a] * inv;
    inv_d2 = inv * inv;
    tmax = d2 * inv;
  } else {
    for (int a = 0; a < 3; ++a) kd[a] = D.kd[a];
    inv_d2 = D.inv_d2;
    tmax = INFINITY;
  }
}

// ---------------------------------------------------------------------------
// Grid walk (Amanatides & Woo 1987): times in precision T, densities and
// optical depths in precision R.
//
// Times t of the walk are measured from the point where the ray enters the
// grid (its origin if that lies inside), so their FP32 rounding is relative
// to the chord, not to the distance from a far origin; `tin` is that entry
// time in the original parametrisation.  Along each non-parallel axis a,
// t0[a] is the crossing time of the first plane ahead of the entry point and
// dt[a] the time between planes, so after j[a] crossings along a the next
// plane is reached at t = t0[a] + j[a] * dt[a] -- one rounding of a product
// and a sum, no accumulation and no cancellation against a far anchor.
// i[a] is the current cell index along a and s[a] its step (+1, -1, or 0
// for an axis parallel to the ray, whose t0 is +inf and dt 0); the walk
// ends as soon as some i[a] leaves [0, n[a]).

//
// On a rectilinear grid the planes are not evenly spaced: there e[a] is the
// entry point's coordinate relative to the axis's first plane (FP64), dt[a]
// is 1 / k[a], and tp[a] = (Q[p] - e[a]) dt[a] is the crossing time of the
// next plane p ahead (Q the FP64 relative plane table), reloaded each time
// the walk crosses a plane along a.  The difference is taken in FP64 -- in
// precision R its rounding would scale with the box, not with t, and rays
// nearly parallel to an axis would magnify it -- so the FP32 walk's times
// carry a relative error of a few units of R, as on a regular grid.

//
// On a tree grid the walk carries, in FP64, the current point e (the start
// of the current segment), the direction k and the segment's start time tc
// (from the entry), and i[0] is the current cell; each crossing leaves that
// leaf through its nearest face, with the exit faces' coordinates set to
// the faces' planes exactly, and finds the neighbour through the face's rope
// (tree_cross).

//
// Times have their own type T, separate from the type R of densities and
// optical depths.  A segment's length is the difference of two crossing
// times, and in FP32 each time carries an absolute error of a few units of
// roundoff times t (the distance from the entry), so a short segment late in
// a long walk carries a relative error of eps t / length.  Where the walk
// is the package's path (its optical depth sets the forced-scattering point
// and every later event inherits that point's error), the life-cycle walks
// keep times in FP64 and round each segment length to R once; the peel-ray
// and trace walks, whose optical depths end in one exponential, keep T = R.
//
// FP32-time walks count planes in FP32 (the plane time fma(j, dt, t0) then
// needs no integer conversion per crossing; exact while j < 2^24, and the
// library rejects FP32 walks of grids with 2^24 or more cells along an axis)
// and, on regular grids, leave the grid by time: texit is the earliest
// boundary-plane time over the axes, the same fma at the axis's last plane.
// A walk first reaches that time at the crossing that leaves the grid (an
// index leaves its range there, or all later segments inside have zero
// length), so one comparison replaces three index tests.
template <typename T>
using PlaneCount = std::conditional_t<sizeof(T) == sizeof(float), float, int>;
template <int GK, typename T>
constexpr bool kExitByTime = GK == kGridRegular && sizeof(T) == sizeof(float);
template <typename R, typename T = R>
struct Ray {
  using Time = T;
  T t0[3], dt[3];
  T tp[3];       // rectilinear grids only
  double e[3];   // rectilinear and tree grids
  double k[3], tc;  // tree grids only
  PlaneCount<T> j[3];
  int i[3], s[3];
  T texit;  // kExitByTime walks only
  T t;
  R tau;
  T tmax;      // the walk stops here (time from the entry; +inf: at the boundary)
  double tin;  // FP64 entry time (0 for rays starting inside)
  bool active;
};

MCRT_HD float fmaR(float a, float b, float c) { return fmaf(a, b, c); }
MCRT_HD double fmaR(double a, double b, double c) { return fma(a, b, c); }

// Crossing time of the next plane ahead along axis a of a rectilinear grid
// (+inf for an axis parallel to the ray).  The plane index is clamped to the
// table: after the walk has left the grid the value is never used.
template <typename R, typename T>
MCRT_HD T rect_tplane(const Ray<R, T>& ry, const GridDev& G, int a) {
  if (ry.s[a] == 0) return T(INFINITY);
  int p = ry.i[a] + (ry.s[a] > 0 ? 1 : 0);
  p = p < 0 ? 0 : (p > G.n[a] ? G.n[a] : p);
  return (T)((G.qd[a][p] - ry.e[a]) * (double)ry.dt[a]);
}

// Sets up the walk of o + t k (0 <= t <= tmax): slab entry for origins
// outside the grid; cell indices by floor (regular grids) or by search in
// the plane table (rectilinear grids), with the lower cell for a coordinate
// on a wall while moving down; rays missing the grid (or with non-finite
// data, or ending before the grid) are left inactive with tau = 0.
template <typename R, int GK = kGridRegular, typename T = R>
MCRT_HD void ray_begin(Ray<R, T>& ry, const GridDev& G, const double o[3], const double k[3],
                       double tmax = INFINITY) {
  double tin = 0.0, tout = INFINITY;
  int entry = -1;
  bool miss = !(std::isfinite(o[0]) && std::isfinite(o[1]) && std::isfinite(o[2]) && std::isfinite(k[0]) &&
                std::isfinite(k[1]) && std::isfinite(k[2]));
  bool par[3];
  double inv[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    par[a] = !(fabs(k[a]) >= kParallel);
    inv[a] = par[a] ? 0.0 : 1.0 / k[a];
    if (par[a]) {
      if (!(o[a] >= G.lo[a] && o[a] < G.hi[a])) miss = true;
    } else {
      const double ta = (G.lo[a] - o[a]) * inv[a];
      const double tb = (G.hi[a] - o[a]) * inv[a];
      const double tn = fmin(ta, tb), tf = fmax(ta, tb);
      if (tn > tin) {
        tin = tn;
        entry = a;
      }
      tout = fmin(tout, tf);
    }
  }
  if (par[0] && par[1] && par[2]) miss = true;
  if (miss || !(tin < tout) || !(tin < tmax)) {
    ry.active = false;
    ry.tau = R(0);
    ry.t = T(0);
    ry.tin = 0.0;
    return;
  }
  ry.tmax = (T)(tmax - tin);
  if constexpr (GK == kGridTree) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ry.s[a] = par[a] ? 0 : (k[a] > 0.0 ? 1 : -1);
      ry.k[a] = par[a] ? 0.0 : k[a];
      ry.e[a] = a == entry ? (k[a] > 0.0 ? G.lo[a] : G.hi[a]) : o[a] + tin * k[a];
      ry.j[a] = 0;
      ry.i[a] = 0;
    }
    ry.i[0] = tree_find(G, 0, ry.e[0], ry.e[1], ry.e[2], ry.s[0], ry.s[1], ry.s[2]);
    ry.tc = 0.0;
    ry.t = T(0);
    ry.tin = tin;
    ry.tau = R(0);
    ry.active = ry.i[0] >= 0;
    return;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int i;
    if (a == entry) {
      i = k[a] > 0.0 ? 0 : G.n[a] - 1;
    } else if constexpr (GK == kGridRect) {
      const double x = o[a] + tin * k[a];
      i = rect_cell(G.pa[a], G.n[a], x);
      if (!par[a] && k[a] < 0.0 && x == G.pa[a][i]) i -= 1;
      i = i < 0 ? 0 : i;
    } else {
      const double p = o[a] + tin * k[a];
      const double x = (p - G.lo[a]) * G.inv_d[a];
      const double fx = floor(x);
      i = (int)fmin(fmax(fx, -1.0), (double)G.n[a]);
      if (!par[a] && k[a] < 0.0 && x == fx) i -= 1;
      i = i < 0 ? 0 : (i > G.n[a] - 1 ? G.n[a] - 1 : i);
    }
    ry.i[a] = i;
    ry.j[a] = 0;
    if constexpr (GK == kGridRect) {
      ry.s[a] = par[a] ? 0 : (k[a] > 0.0 ? 1 : -1);
      ry.e[a] = o[a] + tin * k[a] - G.pa[a][0];
      ry.t0[a] = T(0);
      ry.dt[a] = (T)inv[a];
      ry.tp[a] = rect_tplane(ry, G, a);
    } else if (par[a]) {
      ry.t0[a] = T(INFINITY);
      ry.dt[a] = T(0);
      ry.s[a] = 0;
    } else if (k[a] > 0.0) {
      ry.t0[a] = (T)((G.lo[a] + (double)(i + 1) * G.d[a] - o[a]) * inv[a] - tin);
      ry.dt[a] = (T)(G.d[a] * inv[a]);
      ry.s[a] = 1;
    } else {
      ry.t0[a] = (T)((G.lo[a] + (double)i * G.d[a] - o[a]) * inv[a] - tin);
      ry.dt[a] = (T)(-G.d[a] * inv[a]);
      ry.s[a] = -1;
    }
  }
  if constexpr (kExitByTime<GK, T>) {
    T te = T(INFINITY);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (ry.s[a] == 0) continue;
      const int last = ry.s[a] > 0 ? G.n[a] - 1 - ry.i[a] : ry.i[a];  // planes crossed before the boundary's
      te = fmin(te, fmaR((T)last, ry.dt[a], ry.t0[a]));
    }
    ry.texit = te;
  }
  ry.t = T(0);
  ry.tin = tin;
  ry.tau = R(0);
  ry.active = true;
}

// Bricked address of the ray's current cell.
template <typename R, typename T>
MCRT_HD int ray_cell(const Ray<R, T>& ry, const GridDev& G) {
  return brick_addr(G, ry.i);
}

// Crossing time of the next plane ahead along axis a.
template <typename R, int GK = kGridRegular, typename T = R>
MCRT_HD T ray_tplane(const Ray<R, T>& ry, int a) {
  if constexpr (GK == kGridRect)
    return ry.tp[a];
  else
    return fmaR((T)ry.j[a], ry.dt[a], ry.t0[a]);
}

// The next D cells of the walk, as a block: their bricked addresses, the end
// times of their segments and their densities.  The cell sequence of a walk
// does not depend on the densities, so the block first advances the walk D
// times (pure arithmetic: all axes whose plane is reached at the segment's
// end advance together) and then issues the D density loads back to back,
// which keeps D gathers in flight per lane instead of one.  The walk leaves
// the grid when some index leaves its range, or when no axis matched the end
// time (non-finite times); sub-steps after that repeat the last valid cell,
// so no load leaves the grid.  `adv` keeps the axes that advanced at each
// sub-step (3 bits each) so that a caller stopping inside the block can
// rewind the ray (ray_rewind), and that names the plane of each crossing
// (on a tree grid: the exit faces of each segment's leaf).
template <int D, typename R, typename T = R>
struct WalkBlock {
  int cell[D];
  T tend[D];  // in the ray's time type
  R rho[D];
  int n;         // valid entries (>= 1 for an active ray)
  unsigned adv;  // axes advanced at sub-step d: bits 3d .. 3d+2
  bool out;      // the walk has left the grid after entry n-1
  double tc0, tend64[D];  // tree grids: FP64 start of the block and segment ends
};

// One crossing of a tree grid: the current leaf (i[0], verified to hold the
// ray's point, else found from the root), its exit time (FP64, from the
// grid entry) and whether the exit face is the box's; moves the point to the
// exit -- the exit faces' coordinates set to the faces' planes exactly, the
// others advanced along k -- and finds the next leaf: across a single face,
// by descending from the face's rope (the deepest node covering the face),
// across an edge or corner, from the root.  A non-finite or negative exit
// time also ends the walk.  `axes` receives the axes of the exit faces (bit
// a for axis a), as a regular grid's walk block records the axes it
// advances.
template <typename R, typename T>
MCRT_HD void tree_cross(Ray<R, T>& ry, const GridDev& G, int& cell, double& tend, bool& out, unsigned& axes) {
  const double px = ry.e[0], py = ry.e[1], pz = ry.e[2];
  const int sx = ry.s[0], sy = ry.s[1], sz = ry.s[2];
  int c = ry.i[0];
  double l0 = 0, l1 = 0, l2 = 0, h0 = -1, h1 = -1, h2 = -1;
  if (c >= 0) {
    const double* bx = G.leaf_box + 6 * (long long)c;
    l0 = bx[0], l1 = bx[1], l2 = bx[2], h0 = bx[3], h1 = bx[4], h2 = bx[5];
  }
  if (!(px >= l0 && px <= h0 && py >= l1 && py <= h1 && pz >= l2 && pz <= h2)) {
    c = tree_find(G, 0, px, py, pz, sx, sy, sz);
    if (c >= 0) {
      const double* bx = G.leaf_box + 6 * (long long)c;
      l0 = bx[0], l1 = bx[1], l2 = bx[2], h0 = bx[3], h1 = bx[4], h2 = bx[5];
    }
  }
  cell = c;
  const double tx = sx > 0 ? (h0 - px) / ry.k[0] : (sx < 0 ? (l0 - px) / ry.k[0] : INFINITY);
  const double ty = sy > 0 ? (h1 - py) / ry.k[1] : (sy < 0 ? (l1 - py) / ry.k[1] : INFINITY);
  const double tz = sz > 0 ? (h2 - pz) / ry.k[2] : (sz < 0 ? (l2 - pz) / ry.k[2] : INFINITY);
  const double tm = fmin(tx, fmin(ty, tz));
  const bool valid = c >= 0 && tm >= 0.0 && tm < INFINITY;
  const bool ex = tx == tm, ey = ty == tm, ez = tz == tm;
  const double fx = sx > 0 ? h0 : l0, fy = sy > 0 ? h1 : l1, fz = sz > 0 ? h2 : l2;
  const bool boundary = (ex && fx == (sx > 0 ? G.hi[0] : G.lo[0])) || (ey && fy == (sy > 0 ? G.hi[1] : G.lo[1])) ||
                        (ez && fz == (sz > 0 ? G.hi[2] : G.lo[2]));
  const double nx = ex ? fx : px + tm * ry.k[0];
  const double ny = ey ? fy : py + tm * ry.k[1];
  const double nz = ez ? fz : pz + tm * ry.k[2];
  out = !valid || boundary;
  axes = valid ? ((unsigned)ex | ((unsigned)ey << 1) | ((unsigned)ez << 2)) : 0u;
  if (valid) {
    ry.e[0] = nx;
    ry.e[1] = ny;
    ry.e[2] = nz;
    ry.tc += tm;
  }
  tend = ry.tc;
  if (out) return;
  const int n_exit = (int)ex + (int)ey + (int)ez;
  const int face = ex ? (sx > 0 ? 1 : 0) : (ey ? (sy > 0 ? 3 : 2) : (sz > 0 ? 5 : 4));
  const int r = n_exit == 1 ? G.ropes[6 * (long long)c + face] : 0;
  ry.i[0] = tree_find(G, r < 0 ? 0 : r, nx, ny, nz, sx, sy, sz);
}

// Whether an accessor brings the per-axis address terms of a regular grid
// (Mem::kLut, with Mem::lut_addr(i): the bricked address of cell i).
template <class M, class = void>
struct HasLut : std::false_type {};
template <class M>
struct HasLut<M, std::void_t<decltype(M::kLut)>> : std::bool_constant<M::kLut> {};

// LOAD = false skips the density loads (walks whose work does not depend on
// the densities, such as the adjoint's peel-ray deposits).  The grid kind
// comes from the accessor (Mem::kGrid).
template <int D, typename R, class Mem, bool LOAD = true, typename T = R>
MCRT_HD void ray_next_block(Ray<R, T>& ry, WalkBlock<D, R, T>& b, const GridDev& G, Mem& M) {
  constexpr int GK = Mem::kGrid;
  b.n = 0;
  b.adv = 0;
  b.out = false;
  if constexpr (GK == kGridTree) {
    b.tc0 = ry.tc;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (!b.out) {
        int cell;
        double te;
        bool out;
        unsigned axes;
        tree_cross(ry, G, cell, te, out, axes);
        b.adv |= axes << (3 * d);
        b.cell[d] = cell < 0 ? 0 : cell;
        b.tend64[d] = te;
        b.tend[d] = (T)te;
        b.n += 1;
        b.out = out;
      } else {
        b.cell[d] = b.cell[d > 0 ? d - 1 : 0];
        b.tend64[d] = b.tend64[d > 0 ? d - 1 : 0];
        b.tend[d] = b.tend[d > 0 ? d - 1 : 0];
      }
    }
    if constexpr (LOAD) {
#pragma unroll
      for (int d = 0; d < D; ++d) b.rho[d] = M.rho(b.cell[d]);
    }
    return;
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const T tx = ray_tplane<R, GK>(ry, 0), ty = ray_tplane<R, GK>(ry, 1), tz = ray_tplane<R, GK>(ry, 2);
    const T tm = fmin(tx, fmin(ty, tz));
    const bool live = !b.out;
    const bool ax = live && tx == tm, ay = live && ty == tm, az = live && tz == tm;
    if constexpr (GK == kGridRegular && HasLut<Mem>::value) {
      const int c = M.lut_addr(ry.i);
      b.cell[d] = live ? c : b.cell[d > 0 ? d - 1 : 0];
    } else {
      b.cell[d] = live ? brick_addr(G, ry.i) : b.cell[d > 0 ? d - 1 : 0];
    }
    b.tend[d] = live ? tm : b.tend[d > 0 ? d - 1 : 0];
    ry.i[0] += ax ? ry.s[0] : 0;
    ry.i[1] += ay ? ry.s[1] : 0;
    ry.i[2] += az ? ry.s[2] : 0;
    ry.j[0] += (PlaneCount<T>)ax;
    ry.j[1] += (PlaneCount<T>)ay;
    ry.j[2] += (PlaneCount<T>)az;
    if constexpr (GK == kGridRect) {
      if (ax) ry.tp[0] = rect_tplane(ry, G, 0);
      if (ay) ry.tp[1] = rect_tplane(ry, G, 1);
      if (az) ry.tp[2] = rect_tplane(ry, G, 2);
    }
    b.adv |= ((unsigned)ax | ((unsigned)ay << 1) | ((unsigned)az << 2)) << (3 * d);
    b.n += live;
    bool outside;
    if constexpr (kExitByTime<GK, T>)
      outside = tm >= ry.texit;
    else
      outside = (unsigned)ry.i[0] >= (unsigned)G.n[0] || (unsigned)ry.i[1] >= (unsigned)G.n[1] ||
                (unsigned)ry.i[2] >= (unsigned)G.n[2];
    b.out = b.out || outside || !(ax || ay || az);
  }
  if constexpr (LOAD) {
#pragma unroll
    for (int d = 0; d < D; ++d) b.rho[d] = M.rho(b.cell[d]);
  }
}

// Undoes the plane crossings of sub-steps d .. D-1 of the last block, so the
// ray again describes the walk inside cell b.cell[d].
template <int D, typename R, int GK = kGridRegular, typename T = R>
MCRT_HD void ray_rewind(Ray<R, T>& ry, const WalkBlock<D, R, T>& b, int d, const GridDev& G) {
  if constexpr (GK == kGridTree) {  // back to the start of segment d (only its entry time is used)
    double tc = b.tc0;
    int cell = b.cell[0];
#pragma unroll
    for (int e = 1; e < D; ++e) {
      tc = e == d ? b.tend64[e - 1] : tc;
      cell = e == d ? b.cell[e] : cell;
    }
    ry.tc = tc;
    ry.i[0] = cell;
    return;
  }
  for (int e = d; e < D; ++e) {
    const unsigned m = b.adv >> (3 * e);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int x = (int)((m >> a) & 1u);
      ry.j[a] -= (PlaneCount<T>)x;
      ry.i[a] -= x * ry.s[a];
    }
  }
  if constexpr (GK == kGridRect) {
#pragma unroll
    for (int a = 0; a < 3; ++a) ry.tp[a] = rect_tplane(ry, G, a);
  }
}

// FP64 entry time of the current cell, in the original parametrisation of
// the ray: the latest plane already crossed, or the ray's entry time.  Moving
// up into cell i the last plane crossed is plane i; moving down, plane i + 1.
template <typename R, int GK = kGridRegular, typename T = R>
MCRT_HD double ray_cell_entry64(const Ray<R, T>& ry, const GridDev& G, const double o[3], const double k[3]) {
  if constexpr (GK == kGridTree) return ry.tin + ry.tc;
  double t = ry.tin;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (ry.s[a] == 0 || ry.j[a] == 0) continue;
    const int p = ry.s[a] > 0 ? ry.i[a] : ry.i[a] + 1;
    double plane;
    if constexpr (GK == kGridRect)
      plane = G.pa[a][p];
    else
      plane = G.lo[a] + (double)p * G.d[a];
    const double tl = (plane - o[a]) / k[a];
    t = fmax(t, tl);
  }
  return t;
}

}  // namespace mcrt
