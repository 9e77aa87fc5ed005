"""Pins of the oracle's attached (pathwise) gradient.

The attached derivative holds the random numbers fixed and lets the
scattering points move with the densities: it is the derivative of the
per-package estimator itself.  Where that estimator is a smooth function of
the densities -- SED instruments (no pixel edges) seen along directions
that no grid plane contains (a peel ray parallel to a plane switches to the
next column of cells when its origin crosses that plane), termination by
count (w_min = 0) -- a central difference of whole runs at rho (1 +- h v) with the
same seeds must reproduce it to the difference's own accuracy (h = 1e-8;
kinks, where a point or a ray crosses a cell edge within +-h, are O(h)
rare).  Held
against: that difference on every grid kind and with split images; the
detached gradient exactly, for a medium that does not scatter (nothing
moves); the detached gradient in expectation, and the full-resimulation
difference at h = 1e-2 within 3 sigma over 8 seeds (the statistical
reading of a central difference under common random numbers); linearity in
dL/dI and additivity over package ranges.
"""
import numpy as np
import pytest


def _problem(W, n_packages=400, seed=4357, **kw):
    n = (8, 7, 6)
    args = dict(n=n, rho=W.lognormal_density(n, 0.8, seed=31), kappa=[1.2, 0.7], albedo=[0.7, 0.5],
                g=[0.45, -0.1], sources=[W.point((0.13, -0.21, 0.07), [1.0, 0.6]), W.expdisk(0.4, 0.15, [0.5, 1.5])],
                detectors=[W.sed(10.0, 30.0, azim=20.0), W.sed(10.0, 95.0, azim=40.0)], n_packages=n_packages, seed=seed,
                flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT, w_min=0.0, max_scatter=6)
    args.update(kw)
    return W.small_problem(**args)


def _grid(W, prob, kind):
    if kind == "rect":
        from test_oracle_rectilinear import random_planes
        rng = np.random.default_rng(4)
        prob["planes"] = tuple(random_planes(prob["box"][2 * a], prob["box"][2 * a + 1], prob["n"][a], rng)
                               for a in range(3))
    elif kind == "tree":
        from test_oracle_tree import BOX, kd_tree
        T = kd_tree(W)
        prob = dict(prob, box=BOX, n=(T.n_cells, 1, 1), tree=T.tree(),
                    rho=np.random.default_rng(7).lognormal(0.0, 0.8, T.n_cells))
    return prob


def _loss(orc, prob, rho, adj):
    img, _, _ = orc.run(dict(prob, rho=rho), threads=4)
    return float((img * adj).sum())


@pytest.mark.parametrize("kind", ["regular", "rect", "tree", "split"])
def test_attached_equals_common_random_number_differences(orc, W, kind):
    prob = _grid(W, _problem(W), kind)
    if kind == "split":
        prob["flags"] |= W.FLAG_SPLIT
    img, _, _ = orc.run(prob)
    adj = np.random.default_rng(5).standard_normal(img.shape)
    g, img_a, _ = orc.grad_attached(prob, adj, threads=4)
    np.testing.assert_allclose(img_a, img, rtol=1e-13)  # the same run (thread sums in another order)
    rho = np.asarray(prob["rho"], dtype=np.float64)
    rng = np.random.default_rng(1)
    h = 1e-8
    fds, dirs = [], []
    for _ in range(8):
        v = rng.choice([-1.0, 1.0], size=rho.shape)
        fds.append((_loss(orc, prob, rho * (1 + h * v), adj) - _loss(orc, prob, rho * (1 - h * v), adj)) / (2 * h))
        dirs.append(float((g * (rho * v).reshape(-1)).sum()))
    fds, dirs = np.array(fds), np.array(dirs)
    scale = np.abs(fds).max()
    assert scale > 0
    # the rounding of L (about 1e-16 sum |a C| / h) and the rare kinks within
    # +-h (a ray passing within about h of a cell edge: the estimator is
    # continuous there, its slope is not)
    assert np.all(np.abs(fds - dirs) <= 1e-6 * scale), (fds, dirs)


def test_attached_equals_detached_without_scattering(orc, W):
    # albedo 0: every scattered weight is 0, nothing but the emission
    # peel-offs contributes and the emission points do not move
    prob = _problem(W, albedo=[0.0, 0.0], w_min=1e-3, max_scatter=50,
                    detectors=[W.frame(10.0, 30.0, 16, 16, 1.0, 1.0, azim=20.0), W.sed(10.0, 95.0)])
    img, _, _ = orc.run(prob)
    adj = np.random.default_rng(3).standard_normal(img.shape)
    ga, _, _ = orc.grad_attached(prob, adj)
    gd, _, _ = orc.grad(prob, adj)
    assert np.abs(gd).max() > 0
    np.testing.assert_allclose(ga, gd, rtol=1e-12, atol=1e-14 * np.abs(gd).max())


def test_attached_statistics_against_detached_and_full_resimulation(orc, W):
    # 8 seeds of 2000 packages: along 8 random +-1 directions v (relative,
    # rho_m v_m), the attached directional derivative agrees with the
    # detached one in expectation and with the full-resimulation central
    # difference at h = 1e-2 (common random numbers per seed), each within
    # 3 standard errors of the per-seed differences
    base = _problem(W, n_packages=2000)
    img, _, _ = orc.run(base)
    adj = np.random.default_rng(5).standard_normal(img.shape)
    rho = np.asarray(base["rho"], dtype=np.float64)
    rng = np.random.default_rng(1)
    V = [rng.choice([-1.0, 1.0], size=rho.shape) for _ in range(8)]
    h = 1e-2
    da, dd, fd = [], [], []
    for s in range(8):
        p = dict(base, seed=1000 + s)
        ga, _, _ = orc.grad_attached(p, adj, threads=4)
        gd, _, _ = orc.grad(p, adj, threads=4)
        da.append([float((ga * (rho * v).reshape(-1)).sum()) for v in V])
        dd.append([float((gd * (rho * v).reshape(-1)).sum()) for v in V])
        fd.append([(_loss(orc, p, rho * (1 + h * v), adj) - _loss(orc, p, rho * (1 - h * v), adj)) / (2 * h)
                   for v in V])
    da, dd, fd = np.array(da), np.array(dd), np.array(fd)
    for other in (dd, fd):
        diff = da - other
        se = diff.std(axis=0, ddof=1) / np.sqrt(len(diff))
        assert np.all(np.abs(diff.mean(axis=0)) <= 3 * se), (diff.mean(axis=0), se)


def test_attached_is_linear_in_adjoint_and_additive_over_shards(orc, W):
    p = _problem(W, n_packages=900, w_min=1e-3, max_scatter=50,
                 detectors=[W.frame(10.0, 30.0, 16, 16, 1.0, 1.0, azim=20.0), W.sed(10.0, 95.0)])
    img, _, _ = orc.run(p)
    rng = np.random.default_rng(9)
    a1, a2 = rng.standard_normal(img.shape), rng.standard_normal(img.shape)
    g1, _, _ = orc.grad_attached(p, a1)
    g2, _, _ = orc.grad_attached(p, a2)
    g12, _, _ = orc.grad_attached(p, 2 * a1 - 3 * a2)
    np.testing.assert_allclose(g12, 2 * g1 - 3 * g2, rtol=1e-9, atol=1e-12 * np.abs(g12).max())
    ga, _, _ = orc.grad_attached(dict(p, n_packages=400), a1)
    gb, _, _ = orc.grad_attached(dict(p, n_packages=500, first_package=400), a1)
    np.testing.assert_allclose(g1, (400 * ga + 500 * gb) / 900, rtol=1e-10, atol=1e-12 * np.abs(g1).max())
    gt, _, _ = orc.grad_attached(p, a1, threads=3)
    np.testing.assert_allclose(gt, g1, rtol=1e-12, atol=1e-14 * np.abs(g1).max())


def test_attached_rejects_a_perspective_instrument(orc, W):
    p = _problem(W, detectors=[W.perspective((0.3, -0.2, 0.1), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 8, 8, 1.0, 1.0)])
    with pytest.raises(ValueError):
        orc.grad_attached(p, np.zeros((1, 2, 64)))
