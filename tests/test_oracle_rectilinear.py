"""Pins of the oracle on rectilinear grids (cells spaced by any rule along
each axis, such as the power-law spacing of PowCub, Table 1(d)): closed
forms and brute force written independently of the oracle's plane lookups,
and the identity with the regular grid when the planes are evenly spaced."""
import numpy as np
import pytest

from test_oracle_traverse import slab

BOX = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)


def random_planes(lo, hi, n, rng):
    """n + 1 strictly increasing coordinates from lo to hi with random cell widths."""
    w = rng.uniform(0.2, 1.0, n)
    p = lo + (hi - lo) * np.concatenate([[0.0], np.cumsum(w) / w.sum()])
    p[0], p[-1] = lo, hi
    return p


def test_regular_planes_reproduce_the_regular_grid(orc, W):
    n = (7, 5, 3)
    rho = W.lognormal_density(n, 0.8, seed=3)
    planes = tuple(np.linspace(BOX[2 * a], BOX[2 * a + 1], n[a] + 1) for a in range(3))
    o, k = W.random_rays(3000, BOX, seed=2)
    t0, tot0, c0, l0, n0 = orc.trace(BOX, n, rho, 1.1, o, k, max_seg=64)
    t1, tot1, c1, l1, n1 = orc.trace(BOX, n, rho, 1.1, o, k, max_seg=64, planes=planes)
    np.testing.assert_allclose(t1, t0, rtol=1e-13, atol=1e-14)
    np.testing.assert_array_equal(n1, n0)
    np.testing.assert_array_equal(c1, c0)
    np.testing.assert_allclose(l1, l0, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("ratio", [1.0, 20.0])
def test_uniform_medium_tau_is_chord_length(orc, W, ratio):
    n = (9, 6, 11)
    planes = tuple(W.power_law_planes(BOX[2 * a], BOX[2 * a + 1], n[a], ratio) for a in range(3))
    o, k = W.random_rays(3000, BOX, seed=4)
    tau, *_ = orc.trace(BOX, n, np.ones(n[::-1]), 1.0, o, k, planes=planes)
    tin, tout, hit = slab(BOX, o, k)
    np.testing.assert_allclose(tau, tout - tin, rtol=1e-13, atol=1e-13)


def test_density_varying_along_x_only(orc, W):
    # power-law planes along x: tau = kappa * sum_i rho_i * (time the ray spends
    # between planes i and i + 1), the overlaps written out in numpy
    n = (12, 5, 7)
    rng = np.random.default_rng(5)
    xs = W.power_law_planes(-1.0, 1.0, n[0], 15.0)
    planes = (xs, random_planes(-1, 1, n[1], rng), random_planes(-1, 1, n[2], rng))
    col = rng.uniform(0.1, 3.0, n[0])
    rho = np.broadcast_to(col[None, None, :], (n[2], n[1], n[0])).copy()
    o, k = W.random_rays(3000, BOX, seed=7)
    tau, *_ = orc.trace(BOX, n, rho, 1.3, o, k, planes=planes)
    tin, tout, hit = slab(BOX, o, k)
    expect = np.zeros(len(o))
    for q in range(len(o)):
        if not hit[q]:
            continue
        if k[q, 0] == 0.0:
            i = min(np.searchsorted(xs, o[q, 0], side="right") - 1, n[0] - 1)
            expect[q] = col[i] * (tout[q] - tin[q])
            continue
        ta = (xs[:-1] - o[q, 0]) / k[q, 0]
        tb = (xs[1:] - o[q, 0]) / k[q, 0]
        a, b = np.minimum(ta, tb), np.maximum(ta, tb)
        ov = np.clip(np.minimum(b, tout[q]) - np.maximum(a, tin[q]), 0, None)
        expect[q] = (col * ov).sum()
    np.testing.assert_allclose(1.3 * expect, tau, rtol=1e-12, atol=1e-13)


def test_axis_parallel_rays_cross_the_plane_gaps(orc, W):
    n = (8, 6, 5)
    rng = np.random.default_rng(11)
    planes = tuple(random_planes(BOX[2 * a], BOX[2 * a + 1], n[a], rng) for a in range(3))
    xs, ys, zs = planes
    rho = np.ones(n[::-1])
    # from inside cell (2, 3, 1) along +x: the rest of cell 2, then whole gaps
    x0 = xs[2] + 0.3 * (xs[3] - xs[2])
    o = np.array([[x0, 0.5 * (ys[3] + ys[4]), 0.5 * (zs[1] + zs[2])]])
    tau, tot, cell, length, nseg = orc.trace(BOX, n, rho, 1.0, o, np.array([[1.0, 0.0, 0.0]]), max_seg=16,
                                             planes=planes)
    assert nseg[0] == 6
    np.testing.assert_array_equal(cell[0, :6], [i + 8 * (3 + 6 * 1) for i in range(2, 8)])
    np.testing.assert_allclose(length[0, :6], np.diff(np.concatenate([[x0], xs[3:]])), rtol=1e-14)
    # along -z from the same point: the part of cell 1 below the point, then cell 0
    tau, tot, cell, length, nseg = orc.trace(BOX, n, rho, 1.0, o, np.array([[0.0, 0.0, -1.0]]), max_seg=16,
                                             planes=planes)
    assert nseg[0] == 2
    np.testing.assert_array_equal(cell[0, :2], [2 + 8 * (3 + 6 * 1), 2 + 8 * 3])
    np.testing.assert_allclose(length[0, :2], [o[0, 2] - zs[1], zs[1] - zs[0]], rtol=1e-14)


def test_wall_conventions(orc, W):
    n = (5, 4, 4)
    xs = W.power_law_planes(-1.0, 1.0, n[0], 6.0)
    planes = (xs, np.linspace(-1, 1, 5), np.linspace(-1, 1, 5))
    rho = np.ones(n[::-1])
    # a point exactly on the interior plane xs[3] moving towards -x starts in cell 2
    o = np.array([[xs[3], 0.1, 0.1]])
    _, _, cell, length, nseg = orc.trace(BOX, n, rho, 1.0, o, np.array([[-1.0, 0.0, 0.0]]), max_seg=8,
                                         planes=planes)
    assert cell[0, 0] % 5 == 2 and nseg[0] == 3
    np.testing.assert_allclose(length[0, :3], [xs[3] - xs[2], xs[2] - xs[1], xs[1] - xs[0]], rtol=1e-14)
    # moving towards +x it starts in cell 3
    _, _, cell, length, nseg = orc.trace(BOX, n, rho, 1.0, o, np.array([[1.0, 0.0, 0.0]]), max_seg=8,
                                         planes=planes)
    assert cell[0, 0] % 5 == 3 and nseg[0] == 2


def test_brute_force_sampling_of_random_medium(orc, W):
    # midpoint sampling of kappa*rho along the ray, each sample located by
    # numpy's sorted search in the plane lists, against the segment sum
    n = (9, 6, 5)
    box = (-2.0, 1.0, 0.0, 3.0, -1.0, 0.5)
    rng = np.random.default_rng(17)
    planes = tuple(random_planes(box[2 * a], box[2 * a + 1], n[a], rng) for a in range(3))
    rho = W.lognormal_density(n, 1.0, seed=9)
    o, k = W.random_rays(40, box, seed=13)
    tau, *_ = orc.trace(box, n, rho, 0.7, o, k, planes=planes)
    tin, tout, hit = slab(box, o, k)
    m = 200_000
    for q in range(len(o)):
        if not hit[q]:
            assert tau[q] == 0.0
            continue
        t = tin[q] + (np.arange(m) + 0.5) * (tout[q] - tin[q]) / m
        p = o[q][None, :] + t[:, None] * k[q][None, :]
        idx = [np.clip(np.searchsorted(planes[a], p[:, a], side="right") - 1, 0, n[a] - 1) for a in range(3)]
        vals = rho[idx[2], idx[1], idx[0]]
        est = 0.7 * vals.sum() * (tout[q] - tin[q]) / m
        assert abs(est - tau[q]) <= 2e-4 * max(tau[q], 1e-3), (q, est, tau[q])


def test_direct_flux_is_exact_on_a_powcub_grid(orc, W):
    # a uniform medium: every package sees tau = kappa * 1 along +z from the
    # origin whatever the planes, so the direct pixel holds L e^-1/(4 pi D^2)
    n = (10, 10, 10)
    planes = tuple(W.power_law_planes(-1.0, 1.0, 10, 12.0) for _ in range(3))
    p = W.small_problem(n=n, rho=np.ones(n), kappa=1.0, albedo=0.6, g=0.5,
                        detectors=[W.frame(10.0, 0.0, 64, 64, 1.0, 1.0)], n_packages=2000,
                        flags=W.FLAGS_DEFAULT | W.FLAG_SPLIT)
    p["planes"] = planes
    img, ab, st = orc.run(p)
    direct = W.split_frames(p, img[0, 0])[0]
    expect = np.exp(-1.0) / (4 * np.pi * 100.0)
    assert abs(direct[32, 32] - expect) < 1e-13 * expect
    direct[32, 32] = 0
    assert np.all(direct == 0)
    closure = st["absorbed"] + st["escaped"] + st["truncated"] - st["emitted"]
    assert abs(closure) < 1e-12


def test_run_on_regular_planes_equals_the_regular_run(orc, W):
    n = (6, 7, 5)
    rho = W.lognormal_density(n, 0.6, seed=23)
    p = W.small_problem(n=n, rho=rho, kappa=1.4, albedo=0.7, g=0.4, n_packages=600,
                        detectors=[W.frame(10.0, 40.0, 12, 12, 1.2, 1.2, azim=15.0)])
    img0, ab0, st0 = orc.run(p)
    q = dict(p, planes=tuple(np.linspace(BOX[2 * a], BOX[2 * a + 1], n[a] + 1) for a in range(3)))
    img1, ab1, st1 = orc.run(q)
    np.testing.assert_allclose(img1, img0, rtol=1e-9, atol=1e-12 * np.abs(img0).max())
    np.testing.assert_allclose(ab1, ab0, rtol=1e-9, atol=1e-12 * np.abs(ab0).max())
    assert st1["events"] == st0["events"] and st1["x_path"] == st0["x_path"]


def test_non_scattering_gradient_closed_form(orc, W):
    # albedo 0, point source at the origin, face-on frame, power-law planes in
    # z: I = e^-tau / (4 pi D^2) with tau = kappa sum rho dz over the +z
    # column, and dL/drho_m = A (-kappa dz_m I) on that column only
    n = (8, 8, 8)
    zs = W.power_law_planes(-1.0, 1.0, 8, 9.0)
    planes = (np.linspace(-1, 1, 9), np.linspace(-1, 1, 9), zs)
    rho = W.lognormal_density(n, 1.0, seed=21)
    kappa, D = 1.7, 10.0
    p = W.small_problem(n=n, rho=rho, kappa=kappa, albedo=0.0, g=0.5, detectors=[W.frame(D, 0.0, 16, 16, 1.0, 1.0)],
                        n_packages=300, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    p["planes"] = planes
    adj = np.random.default_rng(3).standard_normal(256)
    g, img, st = orc.grad(p, adj)
    k0 = np.searchsorted(zs, 0.0, side="right") - 1  # the cell above the origin's plane (or holding it)
    dz = np.diff(zs)[k0:].copy()
    dz[0] = zs[k0 + 1] - 0.0
    col = rho[k0:, 4, 4]
    I = np.exp(-kappa * (col * dz).sum()) / (4 * np.pi * D * D)
    frame = img[0, 0].reshape(16, 16)
    assert abs(frame[8, 8] - I) < 1e-13 * I
    expect = np.zeros(n[::-1])
    expect[k0:, 4, 4] = adj[8 * 16 + 8] * (-kappa * dz * I)
    np.testing.assert_allclose(g.reshape(n[::-1]), expect, rtol=1e-12, atol=1e-20)


def test_gradient_matches_replay_finite_differences(orc, W):
    # on a PowCub grid: the gradient routine against central differences of
    # the reweighted estimator (paths frozen at rho0), h = 1e-4 rho_m
    n = (6, 6, 6)
    planes = tuple(W.power_law_planes(-1.0, 1.0, 6, r) for r in (5.0, 3.0, 8.0))
    rho = W.lognormal_density(n, 0.8, seed=31)
    p = W.small_problem(n=n, rho=rho, kappa=1.2, albedo=0.7, g=0.45, sources=[W.point((0.13, -0.21, 0.07))],
                        detectors=[W.frame(10.0, 30.0, 12, 12, 1.0, 1.0, azim=20.0)], n_packages=1000,
                        flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT, w_min=1e-3, max_scatter=50)
    p["planes"] = planes
    img, _, _ = orc.run(p)
    target = img * (1 + 0.3 * np.random.default_rng(5).standard_normal(img.shape))
    adj = 2 * (img - target)
    g, _, _ = orc.grad(p, adj)
    rho0 = p["rho"].reshape(-1)
    cells = np.argsort(-np.abs(g))[:10]

    def loss(r):
        im, _ = orc.reweight(p, r)
        return ((im - target) ** 2).sum()

    gmax = np.abs(g).max()
    for m in cells:
        h = 1e-4 * rho0[m]
        rp, rm = rho0.copy(), rho0.copy()
        rp[m] += h
        rm[m] -= h
        fd = (loss(rp) - loss(rm)) / (2 * h)
        assert abs(fd - g[m]) <= 1e-6 * abs(g[m]) + 1e-8 * gmax, (m, fd, g[m])
