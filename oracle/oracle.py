"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

A problem is a plain dict:
  box         (xmin, xmax, ymin, ymax, zmin, zmax)
  n           (nx, ny, nz)
  planes      optional (x, y, z) cell-boundary coordinates of a rectilinear grid
  tree        optional tree grid {axis, split, child} per node (n = (cells, 1, 1))
  rho         density, nz*ny*nx values, x fastest
  kappa, albedo, g         one value per wavelength
  sources     list of {kind: "point"|"expdisk", pos: (x, y, z), h_r, h_z, lum: [n_lambda]}, or
              {kind: "cells", cell_lum: [n_lambda][ncell]} (the grid's cells emit; at most one)
  detectors   list of {distance, incl, azim, pa (degrees), nx, ny, half_x, half_y}, optionally
              kind "frame" (default), "sed" (nx = ny = 1) or "perspective" (eye, target, up,
              nx, ny, half_x, half_y)
  n_packages, first_package, seed, w_min, max_scatter, flags

Images come back as an array [comps][n_lambda][sum of ny*nx over frames]
(comps = 2 with FLAG_SPLIT: direct, scattered).
"""
import ctypes as C
import os

import numpy as np

from .build_oracle import ensure_built

FLAG_PEEL_EMIT = 1
FLAG_PEEL_SCAT = 2
FLAG_ABSORB = 4
FLAG_SPLIT = 8
STAT_NAMES = ("emitted", "absorbed", "escaped", "truncated", "x_path", "x_locate", "x_peel", "events", "packages")

_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = C.CDLL(ensure_built())
        d, i, u32, u64, i64 = C.c_double, C.c_int, C.c_uint32, C.c_uint64, C.c_int64
        P = C.c_void_p
        _lib.oracle_philox.argtypes = [P, P, P]
        _lib.oracle_uniform.argtypes = [u32]
        _lib.oracle_uniform.restype = d
        _lib.oracle_hg_mu.argtypes = [d, d]
        _lib.oracle_hg_mu.restype = d
        _lib.oracle_hg_phase.argtypes = [d, d]
        _lib.oracle_hg_phase.restype = d
        _lib.oracle_forced_tau.argtypes = [d, d]
        _lib.oracle_forced_tau.restype = d
        _lib.oracle_rotate.argtypes = [P, d, d, P]
        _lib.oracle_emit_position.argtypes = [i, P, P, P]
        _lib.oracle_emit_direction.argtypes = [P, P]
        _lib.oracle_detector_basis.argtypes = [P, P]
        common = [P, P, P, i, P, P, P, i, P, P, P, i, P, P, u64, u64, u64, d, i, C.c_uint]
        _lib.oracle_run.argtypes = common + [P, P, P, i, P, P, P]
        _lib.oracle_run.restype = i
        _lib.oracle_grad.argtypes = common + [P, P, P, P, i, P, P, P, P, P]
        _lib.oracle_grad.restype = i
        _lib.oracle_grad_attached.argtypes = common + [P, P, P, P, i, P, P, P]
        _lib.oracle_grad_attached.restype = i
        _lib.oracle_reweight.argtypes = [P, P, P, P, i, P, P, P, i, P, P, P, i, P, P, u64, u64, u64, d, i,
                                         C.c_uint, P, P, i, P, P, P, P, P, P, P]
        _lib.oracle_reweight.restype = i
        _lib.oracle_trace.argtypes = [P, P, P, d, i64, P, P, P, i, P, P, P, P, P]
        _lib.oracle_trace.restype = i64
        _lib.oracle_peel.argtypes = [P, P, P, d, d, i64, P, P, P, i, P, P, P, P, P]
        _lib.oracle_peel.restype = i
        _lib.oracle_draw_words.argtypes = [u64, u64, i64, u32, u32, P]
        _lib.oracle_dust_emission.argtypes = [P, P, P, P, P, i, P, i, P, P, P, d, P, P]
        _lib.oracle_dust_emission.restype = i
        _lib.oracle_mbb_sum.argtypes = [i, P, P, P, d]
        _lib.oracle_mbb_sum.restype = d
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _i32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


def philox(counter, key):
    """Philox4x32-10 of one 128-bit counter under one 64-bit key."""
    c = np.asarray(counter, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    _load().oracle_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw_words(seed, p0, n, lam, c):
    """Philox words [n][4] of draw c for packages p0..p0+n-1 at wavelength index lam."""
    out = np.zeros((int(n), 4), dtype=np.uint32)
    _load().oracle_draw_words(int(seed), int(p0), int(n), int(lam), int(c), _ptr(out))
    return out


def uniform(w):
    return _load().oracle_uniform(int(w))


def hg_mu(g, u):
    return _load().oracle_hg_mu(float(g), float(u))


def hg_phase(g, mu):
    return _load().oracle_hg_phase(float(g), float(mu))


def forced_tau(T, u):
    return _load().oracle_forced_tau(float(T), float(u))


def rotate(k, mu, psi):
    k = _f64(k)
    out = np.zeros(3)
    _load().oracle_rotate(_ptr(k), float(mu), float(psi), _ptr(out))
    return out


def emit_position(kind, par, u):
    par, u = _f64(par), _f64(u)
    out = np.zeros(3)
    _load().oracle_emit_position(int(kind), _ptr(par), _ptr(u), _ptr(out))
    return out


def emit_direction(u):
    u = _f64(u)
    out = np.zeros(3)
    _load().oracle_emit_direction(_ptr(u), _ptr(out))
    return out


DET_KINDS = {"frame": 0, "sed": 1, "perspective": 2}


def _det_par(d):
    """The 16 instrument parameters of the oracle's entry points."""
    return ([d.get("distance", 1.0), d.get("incl", 0.0), d.get("azim", 0.0), d.get("pa", 0.0), d.get("half_x", 1.0),
             d.get("half_y", 1.0), DET_KINDS[d.get("kind", "frame")]] + list(d.get("eye", (0.0, 0.0, 0.0)))
            + list(d.get("target", (0.0, 0.0, 0.0))) + list(d.get("up", (0.0, 0.0, 0.0))))


def detector_basis(det):
    par = _f64(_det_par(det))
    out = np.zeros(9)
    _load().oracle_detector_basis(_ptr(par), _ptr(out))
    return out[0:3], out[3:6], out[6:9]


def _planes(planes, n):
    """Concatenated plane coordinates of a rectilinear grid (x, y, z; n + 1
    each), or None for a regular grid."""
    if planes is None:
        return None
    arr = _f64(np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in planes]))
    assert arr.size == sum(int(m) + 1 for m in n)
    return arr


def _tree(tree):
    """A tree grid {"axis", "split", "child"} packed as doubles (node count,
    then axis, split, child per node), or None."""
    if tree is None:
        return None
    ax = np.asarray(tree["axis"], dtype=np.float64)
    sp = np.asarray(tree["split"], dtype=np.float64)
    ch = np.asarray(tree["child"], dtype=np.float64)
    return _f64(np.concatenate([[ax.size], np.stack([ax, sp, ch], axis=1).reshape(-1)]))


def _marshal(prob):
    box = _f64(prob["box"])
    n = _i32(prob["n"])
    rho = _f64(prob["rho"]).reshape(-1)
    assert rho.size == int(n[0]) * int(n[1]) * int(n[2])
    kappa, albedo, g = _f64(prob["kappa"]), _f64(prob["albedo"]), _f64(prob["g"])
    nl = kappa.size
    srcs = prob["sources"]
    kind = _i32([{"point": 0, "expdisk": 1, "cells": 2}[s["kind"]] for s in srcs])
    spar = _f64([list(s.get("pos", (0.0, 0.0, 0.0))) + [s.get("h_r", 0.0), s.get("h_z", 0.0)] for s in srcs])
    cells = [s for s in srcs if s["kind"] == "cells"]
    cell_lum = None
    if cells:
        c = cells[0]["cell_lum"]
        c = c if isinstance(c, np.ndarray) else np.asarray(c.detach().cpu().numpy() if hasattr(c, "detach") else c)
        cell_lum = _f64(c).reshape(-1)
        assert cell_lum.size == nl * rho.size
    slum = _f64([np.broadcast_to(np.asarray(s["lum"], dtype=np.float64), (nl,)) for s in srcs])
    dets = prob["detectors"]
    dpar = _f64([_det_par(d) for d in dets] if dets else np.zeros((0, 16)))
    dpix = _i32([[d["nx"], d["ny"]] for d in dets] if dets else np.zeros((0, 2)))
    npix = int(sum(d["nx"] * d["ny"] for d in dets))
    planes = _planes(prob.get("planes"), n)
    tree = _tree(prob.get("tree"))
    keep = (box, n, rho, kappa, albedo, g, kind, spar, slum, dpar, dpix, planes, tree, cell_lum)
    args = [_ptr(box), _ptr(n), _ptr(rho), nl, _ptr(kappa), _ptr(albedo), _ptr(g), len(srcs), _ptr(kind),
            _ptr(spar), _ptr(slum), len(dets), _ptr(dpar), _ptr(dpix), int(prob["n_packages"]),
            int(prob.get("first_package", 0)), int(prob.get("seed", 4357)), float(prob.get("w_min", 1e-4)),
            int(prob.get("max_scatter", 1000)), int(prob.get("flags", 7))]
    return args, keep, nl, npix


def _comps(prob):
    return 2 if int(prob.get("flags", 7)) & FLAG_SPLIT else 1


def run(prob, threads=1):
    """Forward run: returns (images[comps][n_lambda][pixels], absorbed[n_lambda][ncell] or None, stats dict)."""
    args, keep, nl, npix = _marshal(prob)
    ncell = keep[2].size
    images = np.zeros((_comps(prob), nl, npix))
    absorbed = np.zeros((nl, ncell)) if int(prob.get("flags", 7)) & FLAG_ABSORB else None
    stats = np.zeros(len(STAT_NAMES))
    rc = _load().oracle_run(*args, _ptr(images), _ptr(absorbed), _ptr(stats), int(threads), _ptr(keep[11]),
                            _ptr(keep[12]), _ptr(keep[13]))
    if rc != 0:
        raise ValueError("oracle_run rejected its arguments")
    return images, absorbed, dict(zip(STAT_NAMES, stats.tolist()))


def grad(prob, adj, threads=1, optics=False, adj_absorbed=None):
    """Detached gradient dL/drho for dL/dI = adj (same layout as the images)
    and, if given, dL/dA = adj_absorbed [n_lambda][ncell] on the absorbed
    tally.  optics=True also returns {"albedo": [n_lambda], "g": [n_lambda],
    "lum": [n_src][n_lambda]} (of the image term) as a fourth value."""
    args, keep, nl, npix = _marshal(prob)
    ncell = keep[2].size
    adj = _f64(adj).reshape(_comps(prob), nl, npix)
    images = np.zeros((_comps(prob), nl, npix))
    g = np.zeros(ncell)
    stats = np.zeros(len(STAT_NAMES))
    n_src = len(prob["sources"])
    gopt = np.zeros((2 + n_src, nl)) if optics else None
    aa = None if adj_absorbed is None else _f64(adj_absorbed).reshape(nl, ncell)
    rc = _load().oracle_grad(*args, _ptr(adj), _ptr(images), _ptr(g), _ptr(stats), int(threads), _ptr(keep[11]),
                            _ptr(keep[12]), _ptr(keep[13]), _ptr(gopt), _ptr(aa))
    if rc != 0:
        raise ValueError("oracle_grad rejected its arguments")
    if optics:
        return g, images, dict(zip(STAT_NAMES, stats.tolist())), {"albedo": gopt[0], "g": gopt[1], "lum": gopt[2:]}
    return g, images, dict(zip(STAT_NAMES, stats.tolist()))


def grad_attached(prob, adj, threads=1):
    """Attached (pathwise) gradient dL/drho for dL/dI = adj: the random
    numbers held fixed, the scattering points moving with the densities.
    Frames and SED instruments only.  Returns (grad, images, stats)."""
    args, keep, nl, npix = _marshal(prob)
    ncell = keep[2].size
    adj = _f64(adj).reshape(_comps(prob), nl, npix)
    images = np.zeros((_comps(prob), nl, npix))
    g = np.zeros(ncell)
    stats = np.zeros(len(STAT_NAMES))
    rc = _load().oracle_grad_attached(*args, _ptr(adj), _ptr(images), _ptr(g), _ptr(stats), int(threads),
                                      _ptr(keep[11]), _ptr(keep[12]), _ptr(keep[13]))
    if rc != 0:
        raise ValueError("oracle_grad_attached rejected its arguments")
    return g, images, dict(zip(STAT_NAMES, stats.tolist()))


def reweight(prob, rho_eval, threads=1, albedo_eval=None, g_eval=None, lum_eval=None, absorbed=False):
    """Images of paths sampled at prob's parameters with weights evaluated at
    rho_eval (and at albedo_eval, g_eval [n_lambda], lum_eval [n_src][n_lambda]
    when given); absorbed=True returns (images, absorbed [n_lambda][ncell],
    stats)."""
    args, keep, nl, npix = _marshal(prob)
    rho_eval = _f64(rho_eval).reshape(-1)
    assert rho_eval.size == keep[2].size
    images = np.zeros((_comps(prob), nl, npix))
    stats = np.zeros(len(STAT_NAMES))
    a = args[:3] + [_ptr(rho_eval)] + args[3:]
    ae = None if albedo_eval is None else _f64(albedo_eval).reshape(nl)
    ge = None if g_eval is None else _f64(g_eval).reshape(nl)
    le = None if lum_eval is None else _f64(lum_eval).reshape(len(prob["sources"]), nl)
    ab = np.zeros((nl, keep[2].size)) if absorbed else None
    rc = _load().oracle_reweight(*a, _ptr(images), _ptr(stats), int(threads), _ptr(keep[11]),
                                 _ptr(keep[12]), _ptr(keep[13]), _ptr(ae), _ptr(ge), _ptr(le), _ptr(ab))
    if rc != 0:
        raise ValueError("oracle_reweight rejected its arguments")
    if absorbed:
        return images, ab, dict(zip(STAT_NAMES, stats.tolist()))
    return images, dict(zip(STAT_NAMES, stats.tolist()))


def trace(box, n, rho, kappa, origins, dirs, max_seg=0, planes=None, tree=None):
    """Optical depth along each ray to the grid boundary; with max_seg > 0 also
    the segment lists.  Returns (tau, total_segments, seg_cell, seg_len, n_seg).
    planes: (x, y, z) plane coordinates of a rectilinear grid, or None; tree:
    a tree grid {"axis", "split", "child"}, or None."""
    box, n, rho = _f64(box), _i32(n), _f64(rho).reshape(-1)
    pl, tr = _planes(planes, n), _tree(tree)
    o, k = _f64(origins).reshape(-1, 3), _f64(dirs).reshape(-1, 3)
    nr = o.shape[0]
    tau = np.zeros(nr)
    nseg = np.zeros(nr, dtype=np.int32)
    cell = np.zeros((nr, max(max_seg, 1)), dtype=np.int64) if max_seg > 0 else None
    length = np.zeros((nr, max(max_seg, 1))) if max_seg > 0 else None
    tot = _load().oracle_trace(_ptr(box), _ptr(n), _ptr(rho), float(kappa), nr, _ptr(o), _ptr(k), _ptr(tau),
                               int(max_seg), _ptr(cell), _ptr(length), _ptr(nseg), _ptr(pl), _ptr(tr))
    return tau, int(tot), cell, length, nseg


def peel(box, n, rho, kappa, g, pos, dir_in, w, detectors, planes=None, tree=None):
    """Peel-off of an event list into the frames of one wavelength (fresh zero images)."""
    box, n, rho = _f64(box), _i32(n), _f64(rho).reshape(-1)
    pl, tr = _planes(planes, n), _tree(tree)
    pos = _f64(pos).reshape(-1, 3)
    din = None if dir_in is None else _f64(dir_in).reshape(-1, 3)
    w = _f64(w).reshape(-1)
    dpar = _f64([_det_par(d) for d in detectors])
    dpix = _i32([[d["nx"], d["ny"]] for d in detectors])
    images = np.zeros(int(sum(d["nx"] * d["ny"] for d in detectors)))
    rc = _load().oracle_peel(_ptr(box), _ptr(n), _ptr(rho), float(kappa), float(g), pos.shape[0], _ptr(pos),
                             _ptr(din), _ptr(w), len(detectors), _ptr(dpar), _ptr(dpix), _ptr(images), _ptr(pl),
                             _ptr(tr))
    if rc != 0:
        raise ValueError("oracle_peel rejected its arguments")
    return images


def dust_emission(box, n, rho, absorbed, lam, dlam, kappa_abs, emissivity, planes=None, tree=None):
    """Equilibrium temperature [ncell] and emission spectrum [n_lambda][ncell]
    of every cell from its absorbed luminosity (absorbed: [n_abs][ncell],
    rows summed)."""
    box, n, rho = _f64(box), _i32(n), _f64(rho).reshape(-1)
    pl, tr = _planes(planes, n), _tree(tree)
    absorbed = _f64(absorbed).reshape(-1, rho.size)
    lam, dlam, ka = _f64(np.atleast_1d(lam)), _f64(np.atleast_1d(dlam)), _f64(np.atleast_1d(kappa_abs))
    T = np.zeros(rho.size)
    em = np.zeros((lam.size, rho.size))
    rc = _load().oracle_dust_emission(_ptr(box), _ptr(n), _ptr(pl), _ptr(tr), _ptr(rho), absorbed.shape[0],
                                      _ptr(absorbed), lam.size, _ptr(lam), _ptr(dlam), _ptr(ka), float(emissivity),
                                      _ptr(T), _ptr(em))
    if rc != 0:
        raise ValueError("oracle_dust_emission rejected its arguments")
    return T, em


def mbb_sum(lam, dlam, kappa_abs, T):
    """sum_i kappa_abs_i B(lambda_i, T) dlambda_i, B = lambda^-5 / (exp(c2 / (lambda T)) - 1)."""
    lam, dlam, ka = _f64(np.atleast_1d(lam)), _f64(np.atleast_1d(dlam)), _f64(np.atleast_1d(kappa_abs))
    return _load().oracle_mbb_sum(lam.size, _ptr(lam), _ptr(dlam), _ptr(ka), float(T))


def lib_path():
    return os.path.abspath(ensure_built())
