"""Seeded synthetic inputs for the photon-package life cycle.

This module only builds inputs: grids, densities, optical properties,
sources, frames and run options, as plain dicts that both the GPU library
binding and the CPU oracle accept.  It contains none of the transport
arithmetic and imports neither side.

Problem dict keys:
  name, box (xmin, xmax, ymin, ymax, zmin, zmax), n (nx, ny, nz),
  optional planes (x, y, z cell boundaries of a rectilinear grid),
  optional tree ({axis, split, child} per node of a tree grid; n = (cells, 1, 1)),
  rho (float64 array [nz, ny, nx]; for precision 1 its values are already
  float32-representable), kappa / albedo / g (one value per wavelength),
  sources [{kind, pos, h_r, h_z, lum[n_lambda]}] (kind "cells": the grid's
  cells emit cell_lum[n_lambda][ncell], e.g. dust emission),
  detectors [{distance, incl, azim, pa, nx, ny, half_x, half_y}] (frames;
  kind "sed": the distant observer's total flux, nx = ny = 1; kind
  "perspective": a camera with eye, target, up, nx, ny, half_x, half_y),
  n_packages, first_package, seed, w_min, max_scatter, flags,
  precision (0: FP64 path; 1: FP32 traversal with FP64 state and tallies).

The five workloads follow the configurations used to measure this path
(a uniform cube, an edge-on spiral, a multiwavelength disk, a clumpy disk
and an adjoint problem).  The spiral geometry is the one of the paper's
worked example (Sect. 2.5: stellar and dust exponential disks, frames at 10
Mpc); the dust mass is set through the face-on V-band optical depth, which
is one of the normalisations the paper lists (Sect. 2.2).
"""
import numpy as np

FLAG_PEEL_EMIT = 1
FLAG_PEEL_SCAT = 2
FLAG_ABSORB = 4
FLAG_SPLIT = 8
FLAGS_DEFAULT = FLAG_PEEL_EMIT | FLAG_PEEL_SCAT | FLAG_ABSORB

DEFAULT_SEED = 4357  # the paper's default random seed (Fig. 5)


def _centres(lo, hi, n):
    d = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * d


def cell_centres(box, n):
    """Cell-centre coordinates (x, y, z) as broadcastable [nz,ny,nx] arrays."""
    x = _centres(box[0], box[1], n[0])[None, None, :]
    y = _centres(box[2], box[3], n[1])[None, :, None]
    z = _centres(box[4], box[5], n[2])[:, None, None]
    return x, y, z


def exp_disk_density(box, n, rho0, h_r, h_z, planes=None):
    """rho0 * exp(-R/h_R - |z|/h_z) sampled at cell centres (float64 [nz,ny,nx]);
    planes: the (x, y, z) cell boundaries of a rectilinear grid, else regular cells."""
    if planes is None:
        x, y, z = cell_centres(box, n)
    else:
        x, y, z = plane_centres(planes)
    R = np.sqrt(x * x + y * y)
    return rho0 * np.exp(-R / h_r - np.abs(z) / h_z)


def power_law_planes(lo, hi, n, ratio):
    """Cell boundaries of a power-law mesh on [lo, hi] (the spacing of the
    PowCub grid, Table 1(d)): n cells whose widths are symmetric about the
    centre and grow geometrically outward, the outermost `ratio` times as
    wide as the innermost (ratio 1: regular cells).  Returns n + 1
    increasing coordinates, the first and last exactly lo and hi."""
    k = np.abs(np.arange(n) - (n - 1) / 2.0)
    k = k - k.min()
    w = np.power(float(ratio), k / k.max()) if n > 2 else np.ones(n)
    p = lo + (hi - lo) * np.concatenate([[0.0], np.cumsum(w) / w.sum()])
    p[0], p[-1] = lo, hi
    assert np.all(np.diff(p) > 0)
    return p


def plane_centres(planes):
    """Cell-centre coordinates of a rectilinear grid as broadcastable [nz,ny,nx] arrays."""
    c = [0.5 * (np.asarray(p[1:]) + np.asarray(p[:-1])) for p in planes]
    return c[0][None, None, :], c[1][:, None][None, :, :], c[2][:, None, None]


def as_f32_values(a):
    """Rounds to float32 and returns float64 holding exactly those values."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _point(pos=(0.0, 0.0, 0.0), lum=1.0):
    return {"kind": "point", "pos": tuple(float(v) for v in pos), "h_r": 0.0, "h_z": 0.0, "lum": lum}


def _expdisk(h_r, h_z, lum=1.0, pos=(0.0, 0.0, 0.0)):
    return {"kind": "expdisk", "pos": tuple(float(v) for v in pos), "h_r": float(h_r), "h_z": float(h_z), "lum": lum}


def _frame(distance, incl, nx, ny, half_x, half_y, azim=-90.0, pa=0.0):
    return {"distance": float(distance), "incl": float(incl), "azim": float(azim), "pa": float(pa),
            "nx": int(nx), "ny": int(ny), "half_x": float(half_x), "half_y": float(half_y)}


def _problem(name, box, n, rho, kappa, albedo, g, sources, detectors, n_packages, precision, seed=DEFAULT_SEED,
             flags=FLAGS_DEFAULT, w_min=1e-4, max_scatter=1000, first_package=0):
    kappa = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
    nl = kappa.size
    for s in sources:
        s["lum"] = np.broadcast_to(np.asarray(s["lum"], dtype=np.float64), (nl,)).copy()
    return {"name": name, "box": tuple(float(v) for v in box), "n": tuple(int(v) for v in n),
            "rho": np.ascontiguousarray(rho, dtype=np.float64), "kappa": kappa,
            "albedo": np.broadcast_to(np.asarray(albedo, dtype=np.float64), (nl,)).copy(),
            "g": np.broadcast_to(np.asarray(g, dtype=np.float64), (nl,)).copy(),
            "sources": sources, "detectors": detectors, "n_packages": int(n_packages),
            "first_package": int(first_package), "seed": int(seed), "w_min": float(w_min),
            "max_scatter": int(max_scatter), "flags": int(flags), "precision": int(precision)}


def n_pixels(prob):
    return int(sum(d["nx"] * d["ny"] for d in prob["detectors"]))


def split_frames(prob, images_lambda):
    """Splits one wavelength's flat image block into per-frame [ny, nx] arrays."""
    out, off = [], 0
    for d in prob["detectors"]:
        k = d["nx"] * d["ny"]
        out.append(np.asarray(images_lambda[off:off + k]).reshape(d["ny"], d["nx"]))
        off += k
    return out


# --------------------------------------------------------------------------
# The five measured workloads.

def cube(n_packages=100_000, precision=0, seed=DEFAULT_SEED, flags=FLAGS_DEFAULT):
    """Uniform cube: 32^3 cells over [-1,1]^3, kappa*rho = 1 (centre-to-edge
    tau = 1), albedo 0.6, g 0.5, unit point source at the origin, one 64x64
    frame face-on at distance 10 with half-extent 1."""
    box, n = (-1, 1, -1, 1, -1, 1), (32, 32, 32)
    rho = np.ones((32, 32, 32))
    return _problem("uniform_cube_32", box, n, rho, 1.0, 0.6, 0.5, [_point()],
                    [_frame(10.0, 0.0, 64, 64, 1.0, 1.0)], n_packages, precision, seed=seed, flags=flags)


def spiral(n_packages=10_000_000, precision=1, seed=DEFAULT_SEED, flags=FLAGS_DEFAULT):
    """Edge-on spiral: stellar exponential disk (h_R 4, h_z 0.4 kpc) and dust
    exponential disk (h_R 6, h_z 0.25 kpc, face-on V-band tau 1, i.e.
    kappa*rho0 = tau/(2 h_z) = 2 per kpc) on 256x256x64 cells over
    +-20 x +-20 x +-2 kpc; albedo 0.6, g 0.6; three 512x512 frames at
    10 Mpc (1e4 kpc), inclinations 0/60/90 degrees, half-extent 20 kpc."""
    box, n = (-20, 20, -20, 20, -2, 2), (256, 256, 64)
    rho = exp_disk_density(box, n, 2.0, 6.0, 0.25)
    if precision == 1:
        rho = as_f32_values(rho)
    dets = [_frame(1e4, inc, 512, 512, 20.0, 20.0) for inc in (0.0, 60.0, 90.0)]
    return _problem("edge_on_spiral_256x256x64", box, n, rho, 1.0, 0.6, 0.6, [_expdisk(4.0, 0.4)], dets,
                    n_packages, precision, seed=seed, flags=flags)


def powcub_spiral(n_packages=10_000_000, precision=1, seed=DEFAULT_SEED, flags=FLAGS_DEFAULT, ratio=(8.0, 8.0, 16.0)):
    """The edge-on spiral on a PowCub grid (Table 1(d)): the same box, cell
    counts, dust and stars, with cells graded geometrically so that they
    are finest at the disk centre and midplane -- outermost/innermost width
    8 in x and y, 16 in z -- and the dust sampled at the graded cells'
    centres."""
    box, n = (-20, 20, -20, 20, -2, 2), (256, 256, 64)
    planes = tuple(power_law_planes(box[2 * a], box[2 * a + 1], n[a], ratio[a]) for a in range(3))
    rho = exp_disk_density(box, n, 2.0, 6.0, 0.25, planes=planes)
    if precision == 1:
        rho = as_f32_values(rho)
    dets = [_frame(1e4, inc, 512, 512, 20.0, 20.0) for inc in (0.0, 60.0, 90.0)]
    prob = _problem("powcub_spiral_256x256x64", box, n, rho, 1.0, 0.6, 0.6, [_expdisk(4.0, 0.4)], dets,
                    n_packages, precision, seed=seed, flags=flags)
    prob["planes"] = planes
    return prob


class TreeGrid:
    """Node lists of a tree grid (Table 1(d)), built level by level: node 0
    is the box; a level's splits append their children in pairs at the end,
    so children are numbered above their parent.  axis[q] = -1 marks a leaf
    whose cell is child[q]; lo/hi hold each node's box."""

    def __init__(self, axis, split, child, lo, hi, n_cells):
        self.axis, self.split, self.child, self.lo, self.hi, self.n_cells = axis, split, child, lo, hi, n_cells

    def tree(self):
        return {"axis": self.axis.astype(np.int32), "split": self.split.astype(np.float64),
                "child": self.child.astype(np.int32)}

    def leaf_boxes(self):
        """Boxes (lo, hi) of the cells, indexed by cell."""
        leaf = self.axis < 0
        lo = np.zeros((self.n_cells, 3))
        hi = np.zeros((self.n_cells, 3))
        lo[self.child[leaf]] = self.lo[leaf]
        hi[self.child[leaf]] = self.hi[leaf]
        return lo, hi


def _grow(box, decide, cell_of=None):
    """Builds a tree level by level.  decide(lo, hi, state) gets the boxes
    and per-node state of a level and returns (axis, child_state): the split
    axis per node (-1: leaf) and the state of its children.  cell_of(lo, hi)
    numbers the leaves (default: in the order they are closed)."""
    b_lo, b_hi = np.array(box[0::2], dtype=np.float64), np.array(box[1::2], dtype=np.float64)
    axis, split, child = [np.array([-1])], [np.array([0.0])], [np.array([0])]
    los, his = [b_lo[None, :]], [b_hi[None, :]]
    ids, lo, hi, state = np.array([0]), b_lo[None, :], b_hi[None, :], np.zeros(1, dtype=np.int64)
    n_nodes, n_cells = 1, 0
    AX, SP, CH = {0: -1}, {0: 0.0}, {0: 0}
    ax_all, sp_all, ch_all = np.full(1, -1), np.zeros(1), np.zeros(1, dtype=np.int64)
    while ids.size:
        ax, cstate = decide(lo, hi, state)
        leaf = ax < 0
        nl = int(leaf.sum())
        cells = cell_of(lo[leaf], hi[leaf]) if cell_of else np.arange(n_cells, n_cells + nl)
        n_cells += nl
        sp_ids = ids[~leaf]
        a = ax[~leaf]
        lo_s, hi_s = lo[~leaf], hi[~leaf]
        k = np.arange(sp_ids.size)
        mid = 0.5 * (lo_s[k, a] + hi_s[k, a])
        first = n_nodes + 2 * k
        # grow the global arrays
        new_n = n_nodes + 2 * sp_ids.size
        ax_all = np.concatenate([ax_all, np.full(new_n - n_nodes, -1)])
        sp_all = np.concatenate([sp_all, np.zeros(new_n - n_nodes)])
        ch_all = np.concatenate([ch_all, np.zeros(new_n - n_nodes, dtype=np.int64)])
        ch_all[ids[leaf]] = cells
        ax_all[sp_ids] = a
        sp_all[sp_ids] = mid
        ch_all[sp_ids] = first
        lo_c = np.repeat(lo_s, 2, axis=0)
        hi_c = np.repeat(hi_s, 2, axis=0)
        kk = np.repeat(k, 2)
        side = np.tile([0, 1], sp_ids.size)
        aa = np.repeat(a, 2)
        hi_c[np.arange(kk.size)[side == 0], aa[side == 0]] = np.repeat(mid, 2)[side == 0]
        lo_c[np.arange(kk.size)[side == 1], aa[side == 1]] = np.repeat(mid, 2)[side == 1]
        los.append(lo_c)
        his.append(hi_c)
        ids = np.arange(n_nodes, new_n)
        lo, hi, state = lo_c, hi_c, np.repeat(cstate[~leaf], 2)
        n_nodes = new_n
    return TreeGrid(ax_all, sp_all, ch_all, np.concatenate(los), np.concatenate(his), n_cells)


def regular_tree(box, levels):
    """A k-d tree that halves the box levels[a] times along each axis (x, y,
    z in turn): the regular 2^lx x 2^ly x 2^lz grid as a tree, each leaf
    numbered with the regular grid's cell index i + nx (j + ny k)."""
    n = np.array([1 << L for L in levels])
    b_lo = np.array(box[0::2], dtype=np.float64)
    d = (np.array(box[1::2], dtype=np.float64) - b_lo) / n
    lv = np.array(levels)

    def decide(lo, hi, state):  # state: halvings done so far, x + 100 y + 10000 z
        done = np.stack([state % 100, (state // 100) % 100, state // 10000], axis=1)
        left = lv[None, :] - done
        ax = np.where(left.max(axis=1) > 0, np.argmax(left > 0, axis=1), -1)
        inc = np.where(ax == 0, 1, np.where(ax == 1, 100, 10000))
        return ax, state + inc

    def cell_of(lo, hi):
        ijk = np.floor((lo - b_lo) / d + 0.5).astype(np.int64)
        return ijk[:, 0] + n[0] * (ijk[:, 1] + n[1] * ijk[:, 2])

    return _grow(box, decide, cell_of)


def adaptive_tree(box, density, max_mass, max_depth, octree=False, samples=2):
    """A tree grid adapted to a density field: a node is divided while its
    mass (the density averaged over samples^3 points times the volume) is
    above max_mass and its depth (in binary levels) below max_depth.  k-d
    tree: halve the longest side; octree: halve x, then y, then z (one octree
    level, three binary levels)."""
    u = (np.arange(samples) + 0.5) / samples

    def mass(lo, hi):
        pts = [lo[:, a, None] + (hi - lo)[:, a, None] * u[None, :] for a in range(3)]
        x = pts[0][:, None, None, :]
        y = pts[1][:, None, :, None]
        z = pts[2][:, :, None, None]
        return density(x, y, z).reshape(lo.shape[0], -1).mean(axis=1) * np.prod(hi - lo, axis=1)

    def decide(lo, hi, state):  # state: depth * 4 + octree phase (0: an octree node)
        depth, phase = state // 4, state % 4
        if octree:
            refine = (phase != 0) | ((depth + 3 <= max_depth) & (mass(lo, hi) > max_mass))
            ax = np.where(refine, phase, -1)
            return ax, (depth + 1) * 4 + (phase + 1) % 3
        refine = (depth + 1 <= max_depth) & (mass(lo, hi) > max_mass)
        ax = np.where(refine, np.argmax(hi - lo, axis=1), -1)
        return ax, (depth + 1) * 4

    return _grow(box, decide)


def tree_problem(name, box, builder, density, kappa, albedo, g, sources, detectors, n_packages, precision,
                 seed=DEFAULT_SEED, flags=FLAGS_DEFAULT, **kw):
    """A problem on a tree grid: the density sampled at the leaves' centres."""
    lo, hi = builder.leaf_boxes()
    c = 0.5 * (lo + hi)
    rho = density(c[:, 0], c[:, 1], c[:, 2])
    if precision == 1:
        rho = as_f32_values(rho)
    n = (builder.n_cells, 1, 1)
    p = _problem(name, box, n, rho.reshape(1, 1, -1), kappa, albedo, g, sources, detectors, n_packages, precision,
                 seed=seed, flags=flags, **kw)
    p["tree"] = builder.tree()
    return p


def spiral_dust(x, y, z):
    """The spiral's dust: kappa*rho = 2 exp(-R/6 - |z|/0.25) per kpc."""
    return 2.0 * np.exp(-np.sqrt(x * x + y * y) / 6.0 - np.abs(z) / 0.25)


def kdtree_spiral(n_packages=10_000_000, precision=1, seed=DEFAULT_SEED, flags=FLAGS_DEFAULT, max_mass=3e-4,
                  max_depth=30):
    """The edge-on spiral on a k-d tree grid (Table 1(d), Sect. 2.4) adapted
    to the dust: a node is halved along its longest side while its dust mass
    exceeds max_mass (kappa-weighted, kpc^2 units), down to 30 levels; the
    dust is sampled at the leaves' centres.  Same box, stars and frames as
    the regular spiral."""
    box = (-20, 20, -20, 20, -2, 2)
    B = adaptive_tree(box, spiral_dust, max_mass, max_depth)
    dets = [_frame(1e4, inc, 512, 512, 20.0, 20.0) for inc in (0.0, 60.0, 90.0)]
    return tree_problem("kdtree_spiral_%d_cells" % B.n_cells, box, B, spiral_dust, 1.0, 0.6, 0.6,
                        [_expdisk(4.0, 0.4)], dets, n_packages, precision, seed=seed, flags=flags)


def multiwavelength(n_packages=1_000_000, precision=1, n_lambda=100, lambdas=None, seed=DEFAULT_SEED,
                    flags=FLAGS_DEFAULT):
    """Same disks on 128^3 cells; 100 wavelengths log-spaced 0.1-1000 micron;
    kappa(lambda) = kappa_V (max(lambda, 0.5)/0.55)^-1.5 (flat below 0.5
    micron), kappa_V rho0 = 2 per kpc; albedo = g = 0.7 (1 - i/99); unit
    luminosity per wavelength; one 256x256 edge-on frame.  `lambdas`
    selects a subset of the wavelength indices."""
    box, n = (-20, 20, -20, 20, -2, 2), (128, 128, 128)
    rho = exp_disk_density(box, n, 2.0, 6.0, 0.25)
    if precision == 1:
        rho = as_f32_values(rho)
    i = np.arange(n_lambda, dtype=np.float64)
    lam = 0.1 * 10.0 ** (4.0 * i / (n_lambda - 1))
    kappa = (np.maximum(lam, 0.5) / 0.55) ** -1.5
    alb = 0.7 * (1.0 - i / (n_lambda - 1))
    if lambdas is not None:
        sel = np.asarray(lambdas, dtype=np.int64)
        kappa, alb = kappa[sel], alb[sel]
    prob = _problem("multiwavelength_128", box, n, rho, kappa, alb, alb.copy(), [_expdisk(4.0, 0.4)],
                    [_frame(1e4, 90.0, 256, 256, 20.0, 20.0)], n_packages, precision, seed=seed, flags=flags)
    prob["lambda_um"] = lam if lambdas is None else lam[np.asarray(lambdas)]
    return prob


def clumpy(n_packages=100_000_000, precision=1, n=(512, 512, 512), n_clumps=20_000, seed=DEFAULT_SEED,
           flags=FLAG_PEEL_EMIT | FLAG_PEEL_SCAT, clump_seed=1):
    """Clumpy disk: the spiral's dust disk carrying half the mass plus
    n_clumps Gaussian clumps at uniform random positions in the box (sigma
    lognormal, median 0.1 kpc, sigma_ln 0.5; equal masses totalling the other
    half; each clump evaluated at cell centres within 4 sigma and scaled so
    its cell sum holds its mass); total mass that of the face-on tau 1 disk
    on this grid; two 1024x1024 frames at 0 and 90 degrees."""
    box = (-20.0, 20.0, -20.0, 20.0, -2.0, 2.0)
    smooth = exp_disk_density(box, n, 2.0, 6.0, 0.25)
    dv = np.prod([(box[2 * a + 1] - box[2 * a]) / n[a] for a in range(3)])
    mass = smooth.sum() * dv
    rho = 0.5 * smooth
    del smooth
    rng = np.random.default_rng(clump_seed)
    cen = rng.uniform([box[0], box[2], box[4]], [box[1], box[3], box[5]], size=(n_clumps, 3))
    sig = 0.1 * np.exp(0.5 * rng.standard_normal(n_clumps))
    m_clump = 0.5 * mass / n_clumps
    d = [(box[2 * a + 1] - box[2 * a]) / n[a] for a in range(3)]
    for c in range(n_clumps):
        lo_i, hi_i, ax = [], [], []
        for a in range(3):
            lo = int(np.floor((cen[c, a] - 4 * sig[c] - box[2 * a]) / d[a]))
            hi = int(np.floor((cen[c, a] + 4 * sig[c] - box[2 * a]) / d[a])) + 1
            lo, hi = max(lo, 0), min(hi, n[a])
            lo_i.append(lo)
            hi_i.append(hi)
            x = box[2 * a] + (np.arange(lo, hi) + 0.5) * d[a]
            ax.append(np.exp(-0.5 * ((x - cen[c, a]) / sig[c]) ** 2))
        if min(h - l for l, h in zip(lo_i, hi_i)) <= 0:
            continue
        blob = ax[2][:, None, None] * ax[1][None, :, None] * ax[0][None, None, :]
        s = blob.sum() * dv
        if s <= 0:
            continue
        rho[lo_i[2]:hi_i[2], lo_i[1]:hi_i[1], lo_i[0]:hi_i[0]] += blob * (m_clump / s)
    if precision == 1:
        rho = as_f32_values(rho)
    dets = [_frame(1e4, inc, 1024, 1024, 20.0, 20.0) for inc in (0.0, 90.0)]
    return _problem("clumpy_disk_%dx%dx%d" % tuple(n), box, n, rho, 1.0, 0.6, 0.6, [_expdisk(4.0, 0.4)], dets,
                    n_packages, precision, seed=seed, flags=flags)


def adjoint(n_packages=10_000_000, precision=1, seed=DEFAULT_SEED, n=64, flags=FLAG_PEEL_EMIT | FLAG_PEEL_SCAT):
    """Adjoint problem: 64^3 cells over [-1,1]^3, rho = exp(z - 1/2) with z
    i.i.d. standard normal (seed 2), kappa 1, albedo 0.6, g 0.5, unit point
    source at the origin, one 128x128 face-on frame at distance 10.  The
    target density is rho * exp(0.1 z') (z' from seed 3); the target image is
    rendered from it with Philox key 4358."""
    box, nn = (-1, 1, -1, 1, -1, 1), (n, n, n)
    z = np.random.default_rng(2).standard_normal((n, n, n))
    rho = np.exp(z - 0.5)
    zt = np.random.default_rng(3).standard_normal((n, n, n))
    rho_t = rho * np.exp(0.1 * zt)
    if precision == 1:
        rho, rho_t = as_f32_values(rho), as_f32_values(rho_t)
    prob = _problem("adjoint_lognormal_%d" % n, box, nn, rho, 1.0, 0.6, 0.5, [_point()],
                    [_frame(10.0, 0.0, 128, 128, 1.0, 1.0)], n_packages, precision, seed=seed, flags=flags)
    prob["rho_target"] = rho_t
    prob["target_seed"] = 4358
    prob["fd_cells"] = np.random.default_rng(4).choice(n * n * n, size=64, replace=False)
    return prob


CONFIGS = {"cube": cube, "spiral": spiral, "multiwavelength": multiwavelength, "clumpy": clumpy,
           "adjoint": adjoint}


# --------------------------------------------------------------------------
# Small test inputs.

def small_problem(name="small", n=(8, 8, 8), box=(-1, 1, -1, 1, -1, 1), rho=None, kappa=1.0, albedo=0.6, g=0.5,
                  sources=None, detectors=None, n_packages=1000, precision=0, seed=DEFAULT_SEED,
                  flags=FLAGS_DEFAULT, w_min=1e-4, max_scatter=1000, first_package=0):
    if rho is None:
        rho = np.ones((n[2], n[1], n[0]))
    if sources is None:
        sources = [_point()]
    if detectors is None:
        detectors = [_frame(10.0, 0.0, 16, 16, 1.0, 1.0)]
    return _problem(name, box, n, rho, kappa, albedo, g, sources, detectors, n_packages, precision, seed=seed,
                    flags=flags, w_min=w_min, max_scatter=max_scatter, first_package=first_package)


def lognormal_density(n, sigma_ln=1.0, seed=0, f32=False):
    z = np.random.default_rng(seed).standard_normal((n[2], n[1], n[0]))
    rho = np.exp(sigma_ln * z - 0.5 * sigma_ln * sigma_ln)
    return as_f32_values(rho) if f32 else rho


def point(pos=(0.0, 0.0, 0.0), lum=1.0):
    return _point(pos, lum)


def expdisk(h_r, h_z, lum=1.0, pos=(0.0, 0.0, 0.0)):
    return _expdisk(h_r, h_z, lum, pos)


def cells(cell_lum):
    """A cell source: the grid's cells emit cell_lum [n_lambda][ncell]
    (host array or device tensor), for instance dust emission."""
    return {"kind": "cells", "cell_lum": cell_lum, "lum": 0.0}


def log_bin_widths(lam):
    """Widths of wavelength bins around increasing centres lam: edges at the
    geometric means of neighbours, the end bins mirrored."""
    lam = np.asarray(lam, dtype=np.float64)
    if lam.size == 1:
        return np.array([0.1 * lam[0]])
    mid = np.sqrt(lam[1:] * lam[:-1])
    edges = np.concatenate([[lam[0] ** 2 / mid[0]], mid, [lam[-1] ** 2 / mid[-1]]])
    return np.diff(edges)


# Grain emission of the panchromatic workload: emissivity in the units of the
# multiwavelength disk (luminosity per unit density x kpc^3 and per unit of
# sum_i kappa_abs B dlambda) that puts its median dust near 20 K.
PANCHROMATIC_EMISSIVITY = 1.1e12


def panchromatic(n_packages=1_000_000, precision=1, n_lambda=100, seed=DEFAULT_SEED):
    """The multiwavelength disk (128^3 cells, 100 wavelengths 0.1-1000
    micron) as a panchromatic problem: the stellar run with the absorbed
    tally, then the dust's re-emission on the same wavelengths.  Returns
    (stellar problem, dust dict {lambda, dlambda, kappa_abs, emissivity});
    kappa_abs = kappa (1 - albedo)."""
    prob = multiwavelength(n_packages=n_packages, precision=precision, n_lambda=n_lambda, seed=seed,
                           flags=FLAGS_DEFAULT)
    prob["name"] = "panchromatic_128"
    lam = prob["lambda_um"]
    dust = {"lambda": lam, "dlambda": log_bin_widths(lam), "kappa_abs": prob["kappa"] * (1.0 - prob["albedo"]),
            "emissivity": PANCHROMATIC_EMISSIVITY}
    return prob, dust


def dust_problem(stellar, emission, n_packages=None, flags=FLAG_PEEL_EMIT | FLAG_PEEL_SCAT | FLAG_ABSORB):
    """The re-emission run of a panchromatic problem: the stellar problem's
    grid, optics and frames with the cells as the only source."""
    p = dict(stellar)
    p["sources"] = [cells(emission)]
    p["flags"] = int(flags)
    if n_packages is not None:
        p["n_packages"] = int(n_packages)
    p["name"] = stellar["name"] + "_dust"
    return p


def sed(distance, incl, azim=-90.0):
    """SED instrument: the total flux per wavelength seen by a distant
    observer in the direction (incl, azim)."""
    return {"kind": "sed", "distance": float(distance), "incl": float(incl), "azim": float(azim), "pa": 0.0,
            "nx": 1, "ny": 1, "half_x": 1.0, "half_y": 1.0}


def perspective(eye, target, up, nx, ny, half_x, half_y):
    """Perspective camera at `eye` looking at `target`, image y along `up`;
    nx x ny pixels over +-half_x x +-half_y of the plane through target."""
    return {"kind": "perspective", "eye": tuple(float(v) for v in eye), "target": tuple(float(v) for v in target),
            "up": tuple(float(v) for v in up), "nx": int(nx), "ny": int(ny), "half_x": float(half_x),
            "half_y": float(half_y)}


def frame(distance, incl, nx, ny, half_x, half_y, azim=-90.0, pa=0.0):
    return _frame(distance, incl, nx, ny, half_x, half_y, azim, pa)


def random_rays(n_rays, box, seed=0, outside_fraction=0.25, axis_fraction=0.1):
    """Ray origins and unit directions: most inside the box, some outside it
    (and aimed roughly at it), some exactly axis-parallel."""
    rng = np.random.default_rng(seed)
    lo = np.array([box[0], box[2], box[4]], dtype=np.float64)
    hi = np.array([box[1], box[3], box[5]], dtype=np.float64)
    o = rng.uniform(lo, hi, size=(n_rays, 3))
    mu = rng.uniform(-1, 1, n_rays)
    ph = rng.uniform(0, 2 * np.pi, n_rays)
    st = np.sqrt(1 - mu * mu)
    k = np.stack([st * np.cos(ph), st * np.sin(ph), mu], axis=1)
    n_out = int(outside_fraction * n_rays)
    if n_out:
        c = 0.5 * (lo + hi)
        span = hi - lo
        far = c + (rng.uniform(-1, 1, size=(n_out, 3)) * 1.5 * span)
        tgt = rng.uniform(lo, hi, size=(n_out, 3))
        dvec = tgt - far
        o[:n_out] = far
        k[:n_out] = dvec / np.linalg.norm(dvec, axis=1, keepdims=True)
    n_ax = int(axis_fraction * n_rays)
    if n_ax:
        sl = slice(n_out, n_out + n_ax)
        axis = rng.integers(0, 3, n_ax)
        sign = rng.choice([-1.0, 1.0], n_ax)
        kk = np.zeros((n_ax, 3))
        kk[np.arange(n_ax), axis] = sign
        k[sl] = kk
    return np.ascontiguousarray(o), np.ascontiguousarray(k)


def random_events(n_events, box, seed=0, isotropic=False):
    """Event positions inside the box, incoming unit directions (or None for
    isotropic emission) and positive weights."""
    rng = np.random.default_rng(seed)
    lo = np.array([box[0], box[2], box[4]], dtype=np.float64)
    hi = np.array([box[1], box[3], box[5]], dtype=np.float64)
    pos = rng.uniform(lo, hi, size=(n_events, 3))
    w = rng.uniform(0.1, 1.0, n_events)
    if isotropic:
        return np.ascontiguousarray(pos), None, w
    mu = rng.uniform(-1, 1, n_events)
    ph = rng.uniform(0, 2 * np.pi, n_events)
    st = np.sqrt(1 - mu * mu)
    k = np.stack([st * np.cos(ph), st * np.sin(ph), mu], axis=1)
    return np.ascontiguousarray(pos), np.ascontiguousarray(k), w
