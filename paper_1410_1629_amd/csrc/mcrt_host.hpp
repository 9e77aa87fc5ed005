// mcrt_host.hpp -- host-side argument checks and problem tables of the C ABI
// (include/mcrt.h): grid, frames (observer direction and image axes,
// Sect. 2.2 / Fig. 4-5), per-wavelength optics and source luminosities
// (Sect. 2.2-2.3).  No HIP runtime calls: the CPU test harness uses the same
// preparation as the library.
#pragma once

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "mcrt.h"
#include "mcrt_lane.hpp"

namespace mcrt {
namespace host {

inline std::string& last_error() {
  static thread_local std::string e;
  return e;
}

inline int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error() = buf;
  return code;
}

inline bool finite(double v) { return std::isfinite(v); }

// Tree grid checks: the nodes form a tree rooted at node 0 whose splits lie
// strictly inside their nodes, with the leaves numbering the cells once each.
inline int check_tree(const mcrt_grid& g) {
  const long long nn = g.tree_nodes, ncell = (long long)g.nx * g.ny * g.nz;
  if (nn < 1) return fail(MCRT_EINVAL, "tree_nodes = %lld must be >= 1", nn);
  if (!g.tree_axis || !g.tree_split || !g.tree_child) return fail(MCRT_EINVAL, "tree arrays are NULL");
  // a node's bounds are written (from its parent's) before they are read
  std::unique_ptr<double[]> lo(new double[3 * nn]), hi(new double[3 * nn]);
  std::vector<int> depth(nn, -1);
  std::vector<char> cell_used(ncell, 0);
  const double box[6] = {g.xmin, g.xmax, g.ymin, g.ymax, g.zmin, g.zmax};
  for (int a = 0; a < 3; ++a) {
    lo[a] = box[2 * a];
    hi[a] = box[2 * a + 1];
  }
  depth[0] = 0;
  long long leaves = 0;
  for (long long q = 0; q < nn; ++q) {  // children are numbered above their parent
    if (depth[q] < 0) return fail(MCRT_EINVAL, "tree node %lld is not reached from node 0", q);
    const int ax = g.tree_axis[q];
    const int c = g.tree_child[q];
    if (ax < 0) {
      if (ax != -1 || c < 0 || c >= ncell || cell_used[c])
        return fail(MCRT_EINVAL, "tree leaf %lld has cell %d (axis %d): cells must be 0..%lld, once each", q, c, ax,
                    ncell - 1);
      cell_used[c] = 1;
      ++leaves;
      continue;
    }
    const double sp = g.tree_split[q];
    if (ax > 2 || !finite(sp) || !(sp > lo[3 * q + ax] && sp < hi[3 * q + ax]))
      return fail(MCRT_EINVAL, "tree node %lld: axis %d, split %g not strictly inside the node", q, ax, sp);
    if (c <= q || (long long)c + 1 >= nn) return fail(MCRT_EINVAL, "tree node %lld: children %d, %d out of order", q, c,
                                                       c + 1);
    if (depth[q] + 1 > kMaxTreeDepth) return fail(MCRT_EINVAL, "tree deeper than %d levels", kMaxTreeDepth);
    for (int side = 0; side < 2; ++side) {
      const long long ch = c + side;
      if (depth[ch] >= 0) return fail(MCRT_EINVAL, "tree node %lld is reached twice", ch);
      depth[ch] = depth[q] + 1;
      for (int a = 0; a < 3; ++a) {
        lo[3 * ch + a] = lo[3 * q + a];
        hi[3 * ch + a] = hi[3 * q + a];
      }
      if (side == 0)
        hi[3 * ch + ax] = sp;
      else
        lo[3 * ch + ax] = sp;
    }
  }
  if (leaves != ncell) return fail(MCRT_EINVAL, "tree has %lld leaves for %lld cells", leaves, ncell);
  return 0;
}

inline int check_grid(const mcrt_grid* g) {
  if (!g) return fail(MCRT_EINVAL, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(MCRT_EINVAL, "grid cell counts must be >= 1");
  if ((long long)g->nx * g->ny * g->nz >= (1ll << 31))
    return fail(MCRT_EINVAL, "grid has %lld cells; at most 2^31 - 1 are supported",
                (long long)g->nx * g->ny * g->nz);
  const double b[6] = {g->xmin, g->xmax, g->ymin, g->ymax, g->zmin, g->zmax};
  for (int a = 0; a < 3; ++a)
    if (!finite(b[2 * a]) || !finite(b[2 * a + 1]) || !(b[2 * a + 1] > b[2 * a]))
      return fail(MCRT_EINVAL, "grid extent along axis %d must be finite and increasing", a);
  if (g->tree_nodes != 0) {
    if (g->planes) return fail(MCRT_EINVAL, "a grid has planes or a tree, not both");
    if (int e = check_tree(*g)) return e;
  }
  if (g->planes) {
    const int n[3] = {g->nx, g->ny, g->nz};
    const double* p = g->planes;
    for (int a = 0; a < 3; ++a) {
      if (p[0] != b[2 * a] || p[n[a]] != b[2 * a + 1])
        return fail(MCRT_EINVAL, "planes along axis %d must start at the box minimum and end at its maximum", a);
      for (int q = 0; q < n[a]; ++q)
        if (!finite(p[q + 1]) || !(p[q + 1] > p[q]))
          return fail(MCRT_EINVAL, "planes along axis %d must be finite and strictly increasing (plane %d)", a, q + 1);
      p += n[a] + 1;
    }
  }
  return 0;
}

// FP32 walks on regular and rectilinear grids count crossed planes in FP32,
// exact below 2^24 (FP32 plane times of farther planes would be inexact too).
inline int check_fp32_axes(const mcrt_grid& g, int precision) {
  if (precision != MCRT_PREC_FP32 || g.tree_nodes != 0) return 0;
  if (g.nx >= (1 << 24) || g.ny >= (1 << 24) || g.nz >= (1 << 24))
    return fail(MCRT_EINVAL, "FP32 precision: at most 2^24 - 1 cells along each axis (grid %d x %d x %d)", g.nx,
                g.ny, g.nz);
  return 0;
}

inline size_t align_up256(size_t x) { return (x + 255) & ~size_t(255); }

// Leaf tables of a tree grid (checked by check_tree): the box of each cell
// (lo x y z, hi x y z) and its ropes (Popov, Guenther, Seidel & Slusallek,
// "Stackless KD-tree traversal", Eurographics 2007): for each face (-x, +x,
// -y, +y, -z, +z) the deepest node whose region covers everything across
// that face, -1 on the box's faces.  Built top-down: a split gives each
// child its parent's ropes plus its sibling across the split plane, and
// every rope is pushed down while one child of the rope node still covers
// the whole face.  A node writes only its children's entries (a leaf its
// cell's), so the nodes of one depth are done in parallel, level after
// level, on up to kTreeThreads host threads: the rope descents are
// dependent loads, and a 967 656-leaf tree took 134 ms on one thread.
constexpr int kTreeThreads = 8;
inline void tree_leaf_tables(const mcrt_grid& g, double* box, int* ropes) {
  const size_t nn = (size_t)g.tree_nodes;
  // every entry is written (from its parent's) before it is read, the
  // root's here: no zero fill of some 140 MB for a million-leaf tree
  std::unique_ptr<double[]> lo(new double[3 * nn]), hi(new double[3 * nn]);
  std::unique_ptr<int[]> rp(new int[6 * nn]);
  const double b[6] = {g.xmin, g.xmax, g.ymin, g.ymax, g.zmin, g.zmax};
  for (int a = 0; a < 3; ++a) {
    lo[a] = b[2 * a];
    hi[a] = b[2 * a + 1];
  }
  for (int f = 0; f < 6; ++f) rp[f] = -1;
  // nodes by depth (children are numbered above their parent)
  std::vector<int> depth(nn, 0);
  int levels = 1;
  for (size_t q = 0; q < nn; ++q)
    if (g.tree_axis[q] >= 0) {
      depth[(size_t)g.tree_child[q]] = depth[(size_t)g.tree_child[q] + 1] = depth[q] + 1;
      levels = std::max(levels, depth[q] + 2);
    }
  std::vector<size_t> start(levels + 1, 0), order(nn);
  for (size_t q = 0; q < nn; ++q) ++start[depth[q] + 1];
  for (int d = 0; d < levels; ++d) start[d + 1] += start[d];
  {
    std::vector<size_t> fill(start.begin(), start.end() - 1);
    for (size_t q = 0; q < nn; ++q) order[fill[depth[q]]++] = q;
  }
  auto node = [&](size_t q) {
    const int ax = g.tree_axis[q];
    if (ax < 0) {
      const int c = g.tree_child[q];
      for (int a = 0; a < 3; ++a) {
        box[6 * (size_t)c + a] = lo[3 * q + a];
        box[6 * (size_t)c + 3 + a] = hi[3 * q + a];
      }
      for (int f = 0; f < 6; ++f) ropes[6 * (size_t)c + f] = rp[6 * q + f];
      return;
    }
    const size_t c0 = (size_t)g.tree_child[q];
    for (int side = 0; side < 2; ++side) {
      const size_t ch = c0 + side;
      for (int a = 0; a < 3; ++a) {
        lo[3 * ch + a] = lo[3 * q + a];
        hi[3 * ch + a] = hi[3 * q + a];
      }
      (side == 0 ? hi : lo)[3 * ch + ax] = g.tree_split[q];
      for (int f = 0; f < 6; ++f) rp[6 * ch + f] = rp[6 * q + f];
      rp[6 * ch + 2 * ax + (side == 0 ? 1 : 0)] = (int)(c0 + 1 - side);
      for (int f = 0; f < 6; ++f) {  // push the rope down
        int r = rp[6 * ch + f];
        const int fa = f / 2;
        const bool up = f % 2 == 1;
        while (r >= 0 && g.tree_axis[r] >= 0) {
          const int ra = g.tree_axis[r];
          const double rs = g.tree_split[r];
          if (ra == fa)
            r = g.tree_child[r] + (up ? 0 : 1);
          else if (hi[3 * ch + ra] <= rs)
            r = g.tree_child[r];
          else if (lo[3 * ch + ra] >= rs)
            r = g.tree_child[r] + 1;
          else
            break;
        }
        rp[6 * ch + f] = r;
      }
    }
  };
  const int hw = (int)std::thread::hardware_concurrency();
  const int nt = std::max(1, std::min(kTreeThreads, hw));
  for (int d = 0; d < levels; ++d) {
    const size_t a = start[d], n = start[d + 1] - a;
    if (nt == 1 || n < 4096) {
      for (size_t i = 0; i < n; ++i) node(order[a + i]);
      continue;
    }
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
      pool.emplace_back([&, t] {
        for (size_t i = n * t / nt; i < n * (t + 1) / nt; ++i) node(order[a + i]);
      });
    for (auto& th : pool) th.join();
  }
}

// Tables of a rectilinear grid (absolute planes, then relative to each
// axis's first plane, FP64, n + 1 per axis, 256-byte aligned) or of a tree
// grid (the nodes); 0 bytes for a regular grid.
inline size_t plane_bytes(const GridDev& G, const mcrt_grid& g) {
  if (G.kind == kGridTree)
    return align_up256(sizeof(TreeNode) * (size_t)g.tree_nodes) + align_up256(sizeof(double) * 6 * (size_t)G.ncell) +
           align_up256(sizeof(int) * 6 * (size_t)G.ncell);
  if (G.kind != kGridRect) return 0;
  const size_t n = (size_t)(G.n[0] + 1) + (G.n[1] + 1) + (G.n[2] + 1);
  return 2 * align_up256(n * sizeof(double));
}

// Writes the tables of g at `host` (plane_bytes bytes) and points G at their
// copy at `dev` (the same bytes in device memory, or `host` itself).
inline void put_planes(const mcrt_grid& g, GridDev& G, unsigned char* host, const unsigned char* dev) {
  if (G.kind == kGridTree) {
    const size_t nn = (size_t)g.tree_nodes, o_box = align_up256(sizeof(TreeNode) * nn),
                 o_rope = o_box + align_up256(sizeof(double) * 6 * (size_t)G.ncell);
    TreeNode* nodes = reinterpret_cast<TreeNode*>(host);
    for (size_t q = 0; q < nn; ++q) nodes[q] = TreeNode{g.tree_split[q], g.tree_axis[q], g.tree_child[q]};
    tree_leaf_tables(g, reinterpret_cast<double*>(host + o_box), reinterpret_cast<int*>(host + o_rope));
    G.nodes = reinterpret_cast<const TreeNode*>(dev);
    G.leaf_box = reinterpret_cast<const double*>(dev + o_box);
    G.ropes = reinterpret_cast<const int*>(dev + o_rope);
    return;
  }
  if (G.kind != kGridRect) return;
  const size_t n = (size_t)(G.n[0] + 1) + (G.n[1] + 1) + (G.n[2] + 1);
  const size_t o_qd = align_up256(n * sizeof(double));
  double* pa = reinterpret_cast<double*>(host);
  double* qd = reinterpret_cast<double*>(host + o_qd);
  size_t o = 0;
  for (int a = 0; a < 3; ++a) {
    const double* P = g.planes + o;
    for (int p = 0; p <= G.n[a]; ++p) {
      pa[o + p] = P[p];
      qd[o + p] = P[p] - P[0];
    }
    G.pa[a] = reinterpret_cast<const double*>(dev) + o;
    G.qd[a] = reinterpret_cast<const double*>(dev + o_qd) + o;
    o += G.n[a] + 1;
  }
}

inline int ilog2_ceil(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Brick of the internal layout.  By default: 2^cb cells (one 128-byte line
// of elements of `elem_bytes`), shaped to minimise the brick's surface per
// volume in physical units -- the rate at which a straight walk in a random
// direction leaves bricks -- with no side longer than the grid needs; ties
// go to the longest x, then y.  brick_shape (MCRT_BRICK) overrides.
inline void choose_brick(const GridDev& G, int elem_bytes, int brick_shape, int lb[3]) {
  if (brick_shape != 0) {
    lb[0] = brick_shape & 15;
    lb[1] = (brick_shape >> 4) & 15;
    lb[2] = (brick_shape >> 8) & 15;
    return;
  }
  int cb = 0;
  while ((1 << cb) * elem_bytes < 128) ++cb;
  const int cap[3] = {ilog2_ceil(G.n[0]), ilog2_ceil(G.n[1]), ilog2_ceil(G.n[2])};
  const int want = std::min(cb, cap[0] + cap[1] + cap[2]);
  double best = INFINITY;
  lb[0] = lb[1] = lb[2] = 0;
  for (int x = cap[0]; x >= 0; --x)
    for (int y = cap[1]; y >= 0; --y) {
      const int z = want - x - y;
      if (z < 0 || z > cap[2]) continue;
      const double score = 1.0 / ((1 << x) * G.d[0]) + 1.0 / ((1 << y) * G.d[1]) + 1.0 / ((1 << z) * G.d[2]);
      if (score < best * (1.0 - 1e-12)) {
        best = score;
        lb[0] = x;
        lb[1] = y;
        lb[2] = z;
      }
    }
}

inline int check_brick(int brick_shape) {
  if (brick_shape == 0) return 0;
  const int lx = brick_shape & 15, ly = (brick_shape >> 4) & 15, lz = (brick_shape >> 8) & 15;
  if ((brick_shape & ~0x1fff) || !(brick_shape & 0x1000) || lx > 7 || ly > 7 || lz > 7 || lx + ly + lz > 10)
    return fail(MCRT_EINVAL, "brick_shape 0x%x is not MCRT_BRICK(lx, ly, lz) with log2 sizes in [0, 7] and at most "
                "2^10 cells", brick_shape);
  return 0;
}

// Tally layout (tally_slot): units of whole bricks of at least 8 cells (one
// 64-byte segment of FP64 values), their count rounded up to a power of two.
inline void set_tally_layout(GridDev& G) {
  G.tb = std::max(G.lb[0] + G.lb[1] + G.lb[2], 3);
  long long units = 1;
  while ((units << G.tb) < (long long)G.ncell_pad) units <<= 1;
  G.ntal = units << G.tb;
}

// Device grid description: geometry, row-major strides and the bricked
// layout.  Fails if the bricked arrays would exceed 2^31 - 1 cells.
inline int make_grid(const mcrt_grid& g, int elem_bytes, int brick_shape, GridDev& G) {
  const double b[6] = {g.xmin, g.xmax, g.ymin, g.ymax, g.zmin, g.zmax};
  const int n[3] = {g.nx, g.ny, g.nz};
  for (int a = 0; a < 3; ++a) {
    G.lo[a] = b[2 * a];
    G.hi[a] = b[2 * a + 1];
    G.n[a] = n[a];
    G.d[a] = (G.hi[a] - G.lo[a]) / n[a];
    G.inv_d[a] = 1.0 / G.d[a];
  }
  G.kind = g.tree_nodes > 0 ? kGridTree : (g.planes ? kGridRect : kGridRegular);
  for (int a = 0; a < 3; ++a) G.pa[a] = G.qd[a] = nullptr;
  G.nodes = nullptr;
  if (G.kind == kGridTree) {  // the leaves as a one-dimensional array, no bricks
    const int nc = g.nx * g.ny * g.nz;
    for (int a = 0; a < 3; ++a) {
      G.n[a] = a == 0 ? nc : 1;
      G.lb[a] = 0;
      G.nb[a] = G.n[a];
    }
    G.stride[0] = 1;
    G.stride[1] = G.stride[2] = nc;
    G.ncell = nc;
    G.bstride[0] = 1;
    G.bstride[1] = G.bstride[2] = nc;
    G.ncell_pad = nc;
    set_tally_layout(G);
    return 0;
  }
  G.stride[0] = 1;
  G.stride[1] = g.nx;
  G.stride[2] = g.nx * g.ny;
  G.ncell = g.nx * g.ny * g.nz;
  if (int e = check_brick(brick_shape)) return e;
  choose_brick(G, elem_bytes, brick_shape, G.lb);
  long long pad = 1;
  for (int a = 0; a < 3; ++a) {
    G.nb[a] = (n[a] + (1 << G.lb[a]) - 1) >> G.lb[a];
    pad *= (long long)G.nb[a] << G.lb[a];
  }
  if (pad >= (1ll << 31))
    return fail(MCRT_EINVAL, "bricked grid has %lld cells; at most 2^31 - 1 are supported", pad);
  const int cpb = 1 << (G.lb[0] + G.lb[1] + G.lb[2]);
  G.bstride[0] = cpb;
  G.bstride[1] = G.nb[0] * cpb;
  G.bstride[2] = G.nb[0] * G.nb[1] * cpb;
  G.ncell_pad = (int)pad;
  set_tally_layout(G);
  return 0;
}

inline int elem_bytes(int precision) { return precision == MCRT_PREC_FP32 ? 4 : 8; }

// Perspective camera axes: w from the eye towards the target, e_y = up made
// perpendicular to w, e_x = w x e_y; false if they are degenerate.
inline bool camera_axes(const mcrt_detector& D, double w[3], double ex[3], double ey[3], double* dist) {
  double n2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    w[a] = D.target[a] - D.eye[a];
    n2 += w[a] * w[a];
  }
  if (!(n2 > 0.0) || !finite(n2)) return false;
  *dist = std::sqrt(n2);
  for (int a = 0; a < 3; ++a) w[a] /= *dist;
  const double uw = D.up[0] * w[0] + D.up[1] * w[1] + D.up[2] * w[2];
  double m2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    ey[a] = D.up[a] - uw * w[a];
    m2 += ey[a] * ey[a];
  }
  const double u2 = D.up[0] * D.up[0] + D.up[1] * D.up[1] + D.up[2] * D.up[2];
  if (!(m2 > 1e-20 * u2) || !finite(m2)) return false;  // up (nearly) along the view axis
  const double m = std::sqrt(m2);
  for (int a = 0; a < 3; ++a) ey[a] /= m;
  ex[0] = w[1] * ey[2] - w[2] * ey[1];
  ex[1] = w[2] * ey[0] - w[0] * ey[2];
  ex[2] = w[0] * ey[1] - w[1] * ey[0];
  return true;
}

inline int check_detectors(int n_det, const mcrt_detector* dets, bool allow_zero) {
  if (n_det < (allow_zero ? 0 : 1) || n_det > MCRT_MAX_DETECTORS)
    return fail(MCRT_EINVAL, "n_det = %d outside [%d, %d]", n_det, allow_zero ? 0 : 1, MCRT_MAX_DETECTORS);
  if (n_det > 0 && !dets) return fail(MCRT_EINVAL, "detectors is NULL");
  for (int d = 0; d < n_det; ++d) {
    const mcrt_detector& D = dets[d];
    if (D.kind != MCRT_DET_FRAME && D.kind != MCRT_DET_SED && D.kind != MCRT_DET_PERSPECTIVE)
      return fail(MCRT_EINVAL, "detector %d: unknown kind %d", d, D.kind);
    if (D.nx < 1 || D.ny < 1 || (long long)D.nx * D.ny > (1ll << 30))
      return fail(MCRT_EINVAL, "detector %d: pixel counts must be >= 1 (at most 2^30 pixels)", d);
    if (D.kind == MCRT_DET_PERSPECTIVE) {
      for (int a = 0; a < 3; ++a)
        if (!finite(D.eye[a]) || !finite(D.target[a]) || !finite(D.up[a]))
          return fail(MCRT_EINVAL, "detector %d: eye, target and up must be finite", d);
      double w[3], ex[3], ey[3], dist;
      if (!camera_axes(D, w, ex, ey, &dist))
        return fail(MCRT_EINVAL, "detector %d: target must differ from eye and up must not be parallel to the view", d);
    } else {
      if (!(D.distance > 0.0) || !finite(D.distance))
        return fail(MCRT_EINVAL, "detector %d: distance must be > 0", d);
      if (!finite(D.incl_deg) || !finite(D.azim_deg) || !finite(D.pa_deg))
        return fail(MCRT_EINVAL, "detector %d: angles must be finite", d);
    }
    if (D.kind == MCRT_DET_SED) {
      if (D.nx != 1 || D.ny != 1) return fail(MCRT_EINVAL, "detector %d: an SED instrument has 1 x 1 pixels", d);
    } else if (!(D.half_x > 0.0) || !(D.half_y > 0.0) || !finite(D.half_x) || !finite(D.half_y)) {
      return fail(MCRT_EINVAL, "detector %d: half-extents must be > 0", d);
    }
  }
  return 0;
}

// Observer direction k_d = (sin t cos p, sin t sin p, cos t), image axes
// e_x = (-sin p, cos p, 0), e_y = (-cos t cos p, -cos t sin p, sin t)
// rotated in the image plane by the position angle, pixel sizes.
inline DetDev make_det(const mcrt_detector& D, long long off) {
  DetDev R;
  const double th = D.incl_deg * (kPi / 180.0), ph = D.azim_deg * (kPi / 180.0), om = D.pa_deg * (kPi / 180.0);
  const double st = std::sin(th), ct = std::cos(th), sp = std::sin(ph), cp = std::cos(ph);
  const double so = std::sin(om), co = std::cos(om);
  const double kd[3] = {st * cp, st * sp, ct};
  const double ex[3] = {-sp, cp, 0.0};
  const double ey[3] = {-ct * cp, -ct * sp, st};
  for (int a = 0; a < 3; ++a) {
    R.kd[a] = kd[a];
    R.ex[a] = co * ex[a] + so * ey[a];
    R.ey[a] = -so * ex[a] + co * ey[a];
  }
  R.inv_d2 = 1.0 / (D.distance * D.distance);
  R.half_x = D.half_x;
  R.half_y = D.half_y;
  R.kind = D.kind;
  for (int a = 0; a < 3; ++a) R.eye[a] = 0.0;
  if (D.kind == MCRT_DET_PERSPECTIVE) {  // view axis, camera axes, tangents of the half field
    double w[3], ex[3], ey[3], dist = 1.0;
    camera_axes(D, w, ex, ey, &dist);
    for (int a = 0; a < 3; ++a) {
      R.kd[a] = w[a];
      R.ex[a] = ex[a];
      R.ey[a] = ey[a];
      R.eye[a] = D.eye[a];
    }
    R.inv_d2 = 0.0;
    R.half_x = D.half_x / dist;
    R.half_y = D.half_y / dist;
  }
  R.kn = D.nx;
  if (D.kind == MCRT_DET_SED) {  // sort keys only: set by sed_key_grid
    R.half_x = R.half_y = 1.0;
    R.kn = 1;
  }
  R.inv_dpx = R.kn / (2.0 * R.half_x);
  R.inv_dpy = (D.kind == MCRT_DET_SED ? 1 : D.ny) / (2.0 * R.half_y);
  R.nx = D.nx;
  R.ny = D.ny;
  R.off = off;
  R.tshift = 0;
  R.key_off = 0;
  R.sub_shift = 0;
  return R;
}

// Sort keys of the peel-ray queue, over all frames (the sort keeps one
// counter per key in LDS), and the parts the sort cuts the queue into.
constexpr long long kSortKeys = 1 << 14;
constexpr int kSortBlocks = 512;

// Virtual key grid of an SED instrument: kSedKeys x kSedKeys pixels over
// the parallel projection of the model box, so that its peel rays sort by
// where they start, as a frame's do.
constexpr int kSedKeys = 256;
inline void sed_key_grid(DetDev& D, const GridDev& G) {
  double hx = 0.0, hy = 0.0;
  for (int c = 0; c < 8; ++c) {
    const double p[3] = {(c & 1) ? G.hi[0] : G.lo[0], (c & 2) ? G.hi[1] : G.lo[1], (c & 4) ? G.hi[2] : G.lo[2]};
    hx = std::max(hx, std::fabs(p[0] * D.ex[0] + p[1] * D.ex[1] + p[2] * D.ex[2]));
    hy = std::max(hy, std::fabs(p[0] * D.ey[0] + p[1] * D.ey[1] + p[2] * D.ey[2]));
  }
  D.kn = kSedKeys;
  D.half_x = hx > 0.0 ? hx : 1.0;
  D.half_y = hy > 0.0 ? hy : 1.0;
  D.inv_dpx = kSedKeys / (2.0 * D.half_x);
  D.inv_dpy = kSedKeys / (2.0 * D.half_y);
}

// Depth buckets of an instrument's queued rays (depth_key): the projection
// of the model box's corners on kd, cut into 2^kDepthBits equal parts.
inline void depth_keys(DetDev& D, const GridDev& G) {
  double lo = INFINITY, hi = -INFINITY;
  for (int c = 0; c < 8; ++c) {
    const double p[3] = {(c & 1) ? G.hi[0] : G.lo[0], (c & 2) ? G.hi[1] : G.lo[1], (c & 4) ? G.hi[2] : G.lo[2]};
    const double t = p[0] * D.kd[0] + p[1] * D.kd[1] + p[2] * D.kd[2];
    lo = std::min(lo, t);
    hi = std::max(hi, t);
  }
  D.dlo = lo;
  D.dscale = hi > lo ? (double)(1 << kDepthBits) / (hi - lo) : 0.0;
}

// Sort-key ranges of the frames (tile_key): a Morton index over tiles of
// 2^tshift x 2^tshift pixels, the frames sharing kSortKeys keys (a power of
// 4 per frame).  Returns the total number of keys; *sub_bits gets the width
// of the second keys (sort_sub) over all frames.
inline long long tile_frames(std::vector<DetDev>& det, int n_det, int* sub_bits) {
  *sub_bits = 0;
  if (n_det <= 0) return 0;
  int bits = 0;  // key bits per frame: even, with n_det << bits <= kSortKeys
  while ((static_cast<long long>(n_det) << (bits + 2)) <= kSortKeys) bits += 2;
  long long keys = 0;
  for (int d = 0; d < n_det; ++d) {
    DetDev& D = det[d];
    int k = 0;
    while ((1 << k) < (D.kind == kDetSed ? D.kn : std::max(D.nx, D.ny))) ++k;
    int ts = 0;
    while (2 * (k - ts) > bits) ++ts;
    D.tshift = ts;
    D.sub_shift = std::max(0, 2 * ts - 8);
    *sub_bits = std::max(*sub_bits, 2 * ts - D.sub_shift + kDepthBits);
    D.key_off = (int)keys;
    keys += 1ll << (2 * (k - ts));
  }
  return keys;
}

// Checked run description of run_photons / backward_density.
struct Prepared {
  RunParams P;
  std::vector<LamDev> lam;
  std::vector<DetDev> det;
  std::vector<SrcDev> src;
  long long n_images = 0;  // comps * n_lambda * pixels of all frames
  double emitted = 0.0;    // sum over wavelengths of n_packages * w0
  long long n_keys = 0;    // image-plane tiles over all frames
  int sub_bits = 0;        // width of the second sort keys (sort_sub)
  int cell_src = -1;       // index of the cell source, -1 if none
  std::vector<double> lums;  // [n_src][n_lambda] luminosity of each source (a cell source: its total)
};

// Per wavelength: the sources' cumulative luminosities, the total and the
// package weight; the cell source (if any) with its totals cell_totals[l]
// (none yet: 0).
inline void set_luminosities(Prepared& out, int n_src, const mcrt_source* sources, const double* cell_totals,
                             unsigned long long n_packages) {
  out.emitted = 0.0;
  const size_t nl = out.lam.size();
  out.lums.assign((size_t)n_src * nl, 0.0);
  for (size_t l = 0; l < nl; ++l) {
    LamDev& L = out.lam[l];
    double cum = 0.0;
    for (int s = 0; s < n_src; ++s) {
      const double ls = s == out.cell_src ? (cell_totals ? cell_totals[l] : 0.0) : sources[s].lum[l];
      out.lums[(size_t)s * nl + l] = ls;
      cum += ls;
      L.cum[s] = cum;
    }
    L.ltot = cum;
    L.w0 = cum / (double)n_packages;
    out.emitted += L.w0 * (double)n_packages;
  }
}

inline int prepare(const mcrt_grid* grid, const void* rho_dev, const mcrt_optics* optics, int n_src,
                   const mcrt_source* sources, int n_det, const mcrt_detector* detectors, const mcrt_opts* opts,
                   Prepared& out) {
  if (int e = check_grid(grid)) return e;
  if (!rho_dev) return fail(MCRT_EINVAL, "rho_dev is NULL");
  if (!optics || !optics->kappa || !optics->albedo || !optics->g) return fail(MCRT_EINVAL, "optics incomplete");
  const int nl = optics->n_lambda;
  if (nl < 1 || nl > (1 << 20)) return fail(MCRT_EINVAL, "n_lambda = %d outside [1, 2^20]", nl);
  for (int l = 0; l < nl; ++l) {
    const double ka = optics->kappa[l], al = optics->albedo[l], gg = optics->g[l];
    if (!(ka >= 0.0) || !finite(ka)) return fail(MCRT_EINVAL, "kappa[%d] must be finite and >= 0", l);
    if (!(al >= 0.0 && al <= 1.0)) return fail(MCRT_EINVAL, "albedo[%d] must lie in [0, 1]", l);
    if (!(std::fabs(gg) < 1.0)) return fail(MCRT_EINVAL, "|g[%d]| must be < 1", l);
  }
  if (n_src < 1 || n_src > MCRT_MAX_SOURCES)
    return fail(MCRT_EINVAL, "n_src = %d outside [1, %d]", n_src, MCRT_MAX_SOURCES);
  if (!sources) return fail(MCRT_EINVAL, "sources is NULL");
  int cell_src = -1;
  for (int s = 0; s < n_src; ++s) {
    const mcrt_source& S = sources[s];
    if (S.kind == MCRT_SRC_CELLS) {
      if (cell_src >= 0) return fail(MCRT_EINVAL, "source %d: at most one cell source per call", s);
      if (!S.cell_lum) return fail(MCRT_EINVAL, "source %d: cell_lum is NULL", s);
      cell_src = s;
      continue;
    }
    if (S.kind != MCRT_SRC_POINT && S.kind != MCRT_SRC_EXPDISK)
      return fail(MCRT_EINVAL, "source %d: unknown kind %d", s, S.kind);
    if (!finite(S.x) || !finite(S.y) || !finite(S.z)) return fail(MCRT_EINVAL, "source %d: position must be finite", s);
    if (S.kind == MCRT_SRC_EXPDISK && (!(S.h_r > 0.0) || !(S.h_z > 0.0) || !finite(S.h_r) || !finite(S.h_z)))
      return fail(MCRT_EINVAL, "source %d: scale lengths must be > 0", s);
    if (!S.lum) return fail(MCRT_EINVAL, "source %d: lum is NULL", s);
    for (int l = 0; l < nl; ++l)
      if (!(S.lum[l] >= 0.0) || !finite(S.lum[l])) return fail(MCRT_EINVAL, "source %d: lum[%d] must be >= 0", s, l);
  }
  if (int e = check_detectors(n_det, detectors, true)) return e;
  if (!opts) return fail(MCRT_EINVAL, "opts is NULL");
  if (opts->n_packages < 1 || opts->n_packages > MCRT_MAX_PACKAGES)
    return fail(MCRT_EINVAL, "n_packages must lie in [1, 2e13]");
  if (opts->first_package > (1ull << 62)) return fail(MCRT_EINVAL, "first_package too large");
  if (opts->n_packages * (unsigned long long)nl > (1ull << 62)) return fail(MCRT_EINVAL, "too many work items");
  if (opts->precision != MCRT_PREC_FP64 && opts->precision != MCRT_PREC_FP32)
    return fail(MCRT_EINVAL, "unknown precision %d", opts->precision);
  if (int e = check_fp32_axes(*grid, opts->precision)) return e;
  if (!(opts->w_min >= 0.0) || !finite(opts->w_min)) return fail(MCRT_EINVAL, "w_min must be finite and >= 0");
  if (opts->max_scatter < 1 || opts->max_scatter > MCRT_MAX_SCATTER_LIMIT)
    return fail(MCRT_EINVAL, "max_scatter must lie in [1, %d]", MCRT_MAX_SCATTER_LIMIT);
  if (opts->flags & ~31u) return fail(MCRT_EINVAL, "unknown flag bits 0x%x", opts->flags);
  if (opts->launch_blocks < 0 || opts->launch_blocks > 64) return fail(MCRT_EINVAL, "launch_blocks outside [0, 64]");
  if (opts->event_batch < 0 || opts->event_batch > 64) return fail(MCRT_EINVAL, "event_batch outside [0, 64]");
  if (opts->peel_queue < -1 || opts->peel_queue > (1ll << 31))
    return fail(MCRT_EINVAL, "peel_queue outside [-1, 2^31]");
  if (opts->max_chunk < 0) return fail(MCRT_EINVAL, "max_chunk is negative");

  RunParams& P = out.P;
  std::memset(&P, 0, sizeof P);
  if (int e = make_grid(*grid, elem_bytes(opts->precision), opts->brick_shape, P.G)) return e;
  P.rho = rho_dev;
  P.n_lambda = nl;
  P.n_src = n_src;
  P.n_det = n_det;
  P.comps = (opts->flags & MCRT_SPLIT) ? 2 : 1;
  P.first = opts->first_package;
  P.n_pkg = opts->n_packages;
  P.seed = opts->seed;
  P.n_items = opts->n_packages * (unsigned long long)nl;
  P.w_min = opts->w_min;
  P.max_scatter = opts->max_scatter;
  P.flags = opts->flags;
  const long long rho_bytes = (long long)P.G.ncell_pad * elem_bytes(opts->precision);
  P.batch = opts->event_batch > 0 ? opts->event_batch : (rho_bytes > kMallBytes ? kBatchForwardHbm : kBatchForward);

  out.lam.assign(nl, LamDev{});
  for (int l = 0; l < nl; ++l) {
    LamDev& L = out.lam[l];
    std::memset(&L, 0, sizeof L);
    L.kappa = optics->kappa[l];
    L.albedo = optics->albedo[l];
    L.g = optics->g[l];
  }
  out.cell_src = cell_src;
  set_luminosities(out, n_src, sources, nullptr, opts->n_packages);
  out.det.assign(n_det > 0 ? n_det : 1, DetDev{});
  long long off = 0;
  for (int d = 0; d < n_det; ++d) {
    out.det[d] = make_det(detectors[d], off);
    off += (long long)detectors[d].nx * detectors[d].ny;
  }
  P.pix_lambda = off;
  out.n_images = (long long)P.comps * nl * off;
  for (int d = 0; d < n_det; ++d) {
    if (out.det[d].kind == kDetSed) sed_key_grid(out.det[d], P.G);
    depth_keys(out.det[d], P.G);
  }
  out.n_keys = tile_frames(out.det, n_det, &out.sub_bits);
  out.src.assign(n_src, SrcDev{});
  for (int s = 0; s < n_src; ++s) {
    out.src[s].kind = sources[s].kind;
    out.src[s].c[0] = sources[s].x;
    out.src[s].c[1] = sources[s].y;
    out.src[s].c[2] = sources[s].z;
    out.src[s].hr = sources[s].h_r;
    out.src[s].hz = sources[s].h_z;
  }
  return 0;
}

inline int check_trace(const mcrt_grid* grid, const void* rho_dev, double kappa, int precision, int64_t n_rays,
                       const double* origin_dev, const double* dir_dev, double* tau_dev, int32_t max_seg,
                       int32_t* seg_cell_dev, double* seg_len_dev) {
  if (int e = check_grid(grid)) return e;
  if (!rho_dev) return fail(MCRT_EINVAL, "rho_dev is NULL");
  if (!(kappa >= 0.0) || !std::isfinite(kappa)) return fail(MCRT_EINVAL, "kappa must be finite and >= 0");
  if (precision != MCRT_PREC_FP64 && precision != MCRT_PREC_FP32) return fail(MCRT_EINVAL, "unknown precision");
  if (int e = check_fp32_axes(*grid, precision)) return e;
  if (n_rays < 0) return fail(MCRT_EINVAL, "n_rays < 0");
  if (n_rays > 0 && (!origin_dev || !dir_dev || !tau_dev)) return fail(MCRT_EINVAL, "ray arrays are NULL");
  const bool lists = seg_cell_dev || seg_len_dev;
  if (lists && (!seg_cell_dev || !seg_len_dev)) return fail(MCRT_EINVAL, "seg_cell_dev and seg_len_dev go together");
  if (lists && max_seg < 1) return fail(MCRT_EINVAL, "max_seg must be >= 1 with segment lists");
  if (lists && (long long)max_seg * n_rays > (1ll << 40)) return fail(MCRT_EINVAL, "segment lists too large");
  return 0;
}

inline int check_peel(const mcrt_grid* grid, const void* rho_dev, double kappa, double g, int precision,
                      int64_t n_events, const double* pos_dev, const double* w_dev, int n_det,
                      const mcrt_detector* detectors, double* images_dev) {
  if (int e = check_grid(grid)) return e;
  if (!rho_dev) return fail(MCRT_EINVAL, "rho_dev is NULL");
  if (!(kappa >= 0.0) || !std::isfinite(kappa)) return fail(MCRT_EINVAL, "kappa must be finite and >= 0");
  if (!(std::fabs(g) < 1.0)) return fail(MCRT_EINVAL, "|g| must be < 1");
  if (precision != MCRT_PREC_FP64 && precision != MCRT_PREC_FP32) return fail(MCRT_EINVAL, "unknown precision");
  if (int e = check_fp32_axes(*grid, precision)) return e;
  if (n_events < 0) return fail(MCRT_EINVAL, "n_events < 0");
  if (int e = check_detectors(n_det, detectors, false)) return e;
  if (!images_dev) return fail(MCRT_EINVAL, "images_dev is NULL");
  if (n_events > 0 && (!pos_dev || !w_dev)) return fail(MCRT_EINVAL, "event arrays are NULL");
  return 0;
}

inline std::vector<DetDev> make_dets(int n_det, const mcrt_detector* detectors, long long* total_pixels) {
  std::vector<DetDev> det(n_det > 0 ? n_det : 1);
  long long off = 0;
  for (int d = 0; d < n_det; ++d) {
    det[d] = make_det(detectors[d], off);
    off += (long long)detectors[d].nx * detectors[d].ny;
  }
  if (total_pixels) *total_pixels = off;
  return det;
}

inline int check_dust(const mcrt_grid* grid, const void* rho_dev, int precision, int n_abs, const double* absorbed_dev,
                      int n_lambda, const double* lambda, const double* dlambda, const double* kappa_abs,
                      double emissivity, const double* emission_dev) {
  if (int e = check_grid(grid)) return e;
  if (!rho_dev) return fail(MCRT_EINVAL, "rho_dev is NULL");
  if (precision != MCRT_PREC_FP64 && precision != MCRT_PREC_FP32)
    return fail(MCRT_EINVAL, "unknown precision %d", precision);
  if (n_abs < 1 || n_abs > (1 << 20)) return fail(MCRT_EINVAL, "n_abs = %d outside [1, 2^20]", n_abs);
  if (!absorbed_dev) return fail(MCRT_EINVAL, "absorbed_dev is NULL");
  if (n_lambda < 1 || n_lambda > (1 << 20)) return fail(MCRT_EINVAL, "n_lambda = %d outside [1, 2^20]", n_lambda);
  if (!lambda || !dlambda || !kappa_abs) return fail(MCRT_EINVAL, "lambda, dlambda or kappa_abs is NULL");
  for (int i = 0; i < n_lambda; ++i)
    if (!(lambda[i] > 0.0) || !finite(lambda[i]) || !(dlambda[i] > 0.0) || !finite(dlambda[i]) ||
        !(kappa_abs[i] > 0.0) || !finite(kappa_abs[i]))
      return fail(MCRT_EINVAL, "lambda, dlambda and kappa_abs must be finite and > 0 (index %d)", i);
  if (!(emissivity > 0.0) || !finite(emissivity)) return fail(MCRT_EINVAL, "emissivity must be finite and > 0");
  if (!emission_dev) return fail(MCRT_EINVAL, "emission_dev is NULL");
  return 0;
}

// Per-wavelength constants of the dust emission: a_i = kappa_abs_i
// dlambda_i / lambda_i^5 and b_i = c2 / lambda_i.
inline void dust_constants(int n_lambda, const double* lambda, const double* dlambda, const double* kappa_abs,
                           double* a, double* b) {
  for (int i = 0; i < n_lambda; ++i) {
    const double l = lambda[i];
    a[i] = kappa_abs[i] * dlambda[i] / (l * l * l * l * l);
    b[i] = kC2 / l;
  }
}

// ---------------------------------------------------------------------------
// The adjoint tape (mcrt_opts.tape): a 256-byte header, then FP64
// [events][1 + n_det][items] (T of the leg after event e, then C per frame)
// and uint32 [events][n_det][items] (the image index of each C).

constexpr uint64_t kTapeMagic = 0x3145504154545243ull;  // "CRTTAPE1", little-endian
constexpr size_t kTapeHeader = 256;

struct TapeHeader {
  uint64_t magic, fingerprint, n_items;
  int32_t events, n_det;
  uint32_t overflow;  // set by the forward run's kernels: a package had more events than the tape keeps
  uint32_t pad;
};
static_assert(sizeof(TapeHeader) <= kTapeHeader, "tape header");

// The most events (emission and scatterings) a package can have: its weight
// after n scatterings is at most a^n of its initial weight (a the largest
// albedo; each scattering multiplies it by albedo (1 - e^-T) <= albedo),
// and a package with weight below w_min times its initial weight stops
// after that scattering's peel-off, so scattering n + 1 needs a^n >= w_min,
// n <= ln w_min / ln a; one more is allowed for rounding.  Scattering 1
// always happens (the first check follows it); max_scatter bounds the rest.
inline long long tape_events(const mcrt_optics& optics, const mcrt_opts& o) {
  double a = 0.0;
  for (int l = 0; l < optics.n_lambda; ++l) a = std::max(a, optics.albedo[l]);
  long long last = o.max_scatter;  // index of the last possible event
  if (a < 1.0 && o.w_min > 0.0) {
    const double r = a > 0.0 ? std::log(o.w_min) / std::log(a) : 0.0;
    if (r + 2.0 < (double)last) last = std::max(1ll, 2 + (long long)std::floor(r));
  }
  return last + 1;
}

// Checks a call of the attached gradient (MCRT_ATTACHED): frames and SED
// instruments, no absorbed-tally term, no optics gradients, a bound on a
// package's events within MCRT_ATTACHED_MAX_EVENTS (returned in *events).
inline int attached_check(const mcrt_optics& optics, int n_det, const mcrt_detector* detectors,
                          const mcrt_opts& o, bool absorbed_term, bool optics_grads, int* events) {
  if (absorbed_term) return fail(MCRT_EINVAL, "MCRT_ATTACHED: the attached gradient has no absorbed-tally term");
  if (optics_grads) return fail(MCRT_EINVAL, "MCRT_ATTACHED: the attached gradient is that of the densities only");
  for (int d = 0; d < n_det; ++d)
    if (detectors[d].kind == MCRT_DET_PERSPECTIVE)
      return fail(MCRT_EINVAL, "MCRT_ATTACHED: instrument %d is a perspective camera (frames and SED only)", d);
  const long long ev = tape_events(optics, o);
  if (ev > MCRT_ATTACHED_MAX_EVENTS)
    return fail(MCRT_EINVAL,
                "MCRT_ATTACHED: a package may have %lld events (at most %d): lower max_scatter, or raise w_min "
                "below an albedo of 1",
                ev, MCRT_ATTACHED_MAX_EVENTS);
  *events = (int)ev;
  return 0;
}

// Bytes of the tape, 0 when the run cannot have one.
inline uint64_t tape_bytes(const mcrt_optics* optics, int n_det, const mcrt_opts* o) {
  if (!optics || !o || !optics->albedo || optics->n_lambda < 1 || n_det < 1 || n_det > MCRT_MAX_DETECTORS) return 0;
  if (!(o->flags & (MCRT_PEEL_EMIT | MCRT_PEEL_SCAT)) || o->n_packages < 1 || o->max_scatter < 1) return 0;
  for (int l = 0; l < optics->n_lambda; ++l)
    if (!(optics->albedo[l] >= 0.0 && optics->albedo[l] <= 1.0)) return 0;
  if (!(o->w_min >= 0.0) || !finite(o->w_min)) return 0;
  const long long ev = tape_events(*optics, *o);
  if (ev > MCRT_TAPE_MAX_EVENTS) return 0;
  const uint64_t items = o->n_packages * (uint64_t)optics->n_lambda;
  const uint64_t doubles = items * (uint64_t)ev * (1 + n_det), words = items * (uint64_t)ev * n_det;
  return kTapeHeader + ((8 * doubles + 255) & ~uint64_t(255)) + 4 * words;
}

inline uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 0x100000001b3ull;
  return h;
}

template <typename T>
inline uint64_t fnv_value(uint64_t h, T v) {
  return fnv1a(h, &v, sizeof v);
}

// Fingerprint of everything the tape's contents depend on except the
// densities and a cell source's luminosities (device arrays): the grid and
// its planes or tree, the optics, the sources, the frames, the packages,
// key, precision, termination and peel-off flags.
inline uint64_t tape_fingerprint(const mcrt_grid& g, const mcrt_optics& op, int n_src, const mcrt_source* src,
                                 int n_det, const mcrt_detector* det, const mcrt_opts& o) {
  uint64_t h = 0xcbf29ce484222325ull;
  const double box[6] = {g.xmin, g.xmax, g.ymin, g.ymax, g.zmin, g.zmax};
  h = fnv1a(h, box, sizeof box);
  h = fnv_value(h, g.nx);
  h = fnv_value(h, g.ny);
  h = fnv_value(h, g.nz);
  if (g.planes) h = fnv1a(h, g.planes, sizeof(double) * ((size_t)g.nx + g.ny + g.nz + 3));
  h = fnv_value(h, g.tree_nodes);
  if (g.tree_nodes > 0 && g.tree_axis && g.tree_split && g.tree_child) {
    h = fnv1a(h, g.tree_axis, sizeof(int32_t) * g.tree_nodes);
    h = fnv1a(h, g.tree_split, sizeof(double) * g.tree_nodes);
    h = fnv1a(h, g.tree_child, sizeof(int32_t) * g.tree_nodes);
  }
  h = fnv_value(h, op.n_lambda);
  h = fnv1a(h, op.kappa, sizeof(double) * op.n_lambda);
  h = fnv1a(h, op.albedo, sizeof(double) * op.n_lambda);
  h = fnv1a(h, op.g, sizeof(double) * op.n_lambda);
  h = fnv_value(h, n_src);
  for (int s = 0; s < n_src; ++s) {
    const double v[5] = {src[s].x, src[s].y, src[s].z, src[s].h_r, src[s].h_z};
    h = fnv_value(h, src[s].kind);
    h = fnv1a(h, v, sizeof v);
    if (src[s].kind != MCRT_SRC_CELLS && src[s].lum) h = fnv1a(h, src[s].lum, sizeof(double) * op.n_lambda);
  }
  h = fnv_value(h, n_det);
  for (int d = 0; d < n_det; ++d) {
    const mcrt_detector& D = det[d];
    const double v[15] = {D.distance, D.incl_deg, D.azim_deg, D.pa_deg, D.half_x, D.half_y, D.eye[0], D.eye[1],
                          D.eye[2], D.target[0], D.target[1], D.target[2], D.up[0], D.up[1], D.up[2]};
    h = fnv1a(h, v, sizeof v);
    h = fnv_value(h, D.nx);
    h = fnv_value(h, D.ny);
    h = fnv_value(h, D.kind);
  }
  h = fnv_value(h, o.n_packages);
  h = fnv_value(h, o.first_package);
  h = fnv_value(h, o.seed);
  h = fnv_value(h, o.precision);
  h = fnv_value(h, o.w_min);
  h = fnv_value(h, o.max_scatter);
  h = fnv_value(h, o.flags & (MCRT_PEEL_EMIT | MCRT_PEEL_SCAT | MCRT_SPLIT));
  return h;
}

// The header a forward run writes, and the check an adjoint makes of a
// tape's header against its own arguments (0, or MCRT_EINVAL with a
// message; *usable = 0 when the forward run overflowed the tape).
inline TapeHeader tape_header(uint64_t fingerprint, uint64_t n_items, int events, int n_det) {
  TapeHeader t;
  std::memset(&t, 0, sizeof t);
  t.magic = kTapeMagic;
  t.fingerprint = fingerprint;
  t.n_items = n_items;
  t.events = events;
  t.n_det = n_det;
  return t;
}

inline int check_tape(const TapeHeader& t, uint64_t fingerprint, uint64_t n_items, int events, int n_det,
                      uint64_t have_bytes, uint64_t need_bytes, bool* usable) {
  *usable = false;
  if (t.magic != kTapeMagic) return fail(MCRT_EINVAL, "tape: not written by run_photons");
  if (t.fingerprint != fingerprint || t.n_items != n_items || t.events != events || t.n_det != n_det)
    return fail(MCRT_EINVAL, "tape: recorded by a run with other arguments");
  if (have_bytes < need_bytes) return fail(MCRT_EINVAL, "tape_bytes %llu < %llu", (unsigned long long)have_bytes,
                                           (unsigned long long)need_bytes);
  *usable = t.overflow == 0;
  return 0;
}

}  // namespace host
}  // namespace mcrt
