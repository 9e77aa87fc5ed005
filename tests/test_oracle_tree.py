"""Pins of the oracle on tree grids (k-d tree; an octree is three binary
levels per octree level; Table 1(d), Sect. 2.4): a tree that halves the box
into a regular grid reproduces the regular grid, and adaptive trees meet
closed forms and brute force written independently of the oracle's leaf
search."""
import numpy as np
import pytest

from test_oracle_traverse import slab

BOX = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)


def _blob(x, y, z):
    return 0.2 + 3.0 * np.exp(-4.0 * ((x - 0.2) ** 2 + (y + 0.1) ** 2 + (z - 0.3) ** 2))


def kd_tree(W, max_mass=0.02, depth=12):
    return W.adaptive_tree(BOX, _blob, max_mass, depth)


def octree(W, max_mass=0.05, depth=12):
    return W.adaptive_tree(BOX, _blob, max_mass, depth, octree=True)


def test_builders_are_trees_of_the_box(W):
    for B in (kd_tree(W), octree(W), W.regular_tree(BOX, (2, 1, 3))):
        lo, hi = B.leaf_boxes()
        assert abs(np.prod(hi - lo, axis=1).sum() - 8.0) < 1e-12  # the leaves tile the box
        leaf = B.axis < 0
        assert np.array_equal(np.sort(B.child[leaf]), np.arange(B.n_cells))
        inner = ~leaf
        assert np.all(B.child[inner] > np.nonzero(inner)[0])
    O = octree(W)
    assert (O.n_cells - 1) % 7 == 0 and (O.axis >= 0).sum() == O.n_cells - 1


def test_regular_tree_reproduces_the_regular_grid(orc, W):
    levels, n = (3, 2, 1), (8, 4, 2)
    T = W.regular_tree(BOX, levels)
    rho = W.lognormal_density(n, 0.8, seed=3)
    o, k = W.random_rays(3000, BOX, seed=2)
    t0, tot0, c0, l0, n0 = orc.trace(BOX, n, rho, 1.1, o, k, max_seg=40)
    t1, tot1, c1, l1, n1 = orc.trace(BOX, (T.n_cells, 1, 1), rho.reshape(-1), 1.1, o, k, max_seg=40, tree=T.tree())
    np.testing.assert_allclose(t1, t0, rtol=1e-13, atol=1e-14)
    np.testing.assert_array_equal(n1, n0)
    np.testing.assert_array_equal(c1, c0)
    np.testing.assert_allclose(l1, l0, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("kind", ["kd", "oct"])
def test_uniform_medium_tau_is_chord_length(orc, W, kind):
    T = kd_tree(W) if kind == "kd" else octree(W)
    o, k = W.random_rays(2000, BOX, seed=4)
    tau, *_ = orc.trace(BOX, (T.n_cells, 1, 1), np.ones(T.n_cells), 1.0, o, k, tree=T.tree())
    tin, tout, hit = slab(BOX, o, k)
    np.testing.assert_allclose(tau, tout - tin, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("kind", ["kd", "oct"])
def test_brute_force_sampling_of_random_medium(orc, W, kind):
    # midpoint sampling of kappa*rho along the ray, each sample located in
    # the leaf boxes by numpy, against the segment sum
    T = kd_tree(W) if kind == "kd" else octree(W)
    lo, hi = T.leaf_boxes()
    rho = np.random.default_rng(9).lognormal(0.0, 1.0, T.n_cells)
    o, k = W.random_rays(25, BOX, seed=13)
    tau, *_ = orc.trace(BOX, (T.n_cells, 1, 1), rho, 0.7, o, k, tree=T.tree())
    tin, tout, hit = slab(BOX, o, k)
    m = 20_000
    for q in range(len(o)):
        if not hit[q]:
            assert tau[q] == 0.0
            continue
        t = tin[q] + (np.arange(m) + 0.5) * (tout[q] - tin[q]) / m
        p = o[q][None, :] + t[:, None] * k[q][None, :]
        inside = np.all((p[:, None, :] >= lo[None, :, :]) & (p[:, None, :] < hi[None, :, :]), axis=2)
        assert np.all(inside.sum(axis=1) == 1)
        vals = rho[np.argmax(inside, axis=1)]
        est = 0.7 * vals.sum() * (tout[q] - tin[q]) / m
        assert abs(est - tau[q]) <= 3e-3 * max(tau[q], 1e-3), (q, est, tau[q])


def test_segments_are_leaf_chords(orc, W):
    # each segment lies in the leaf it names: its midpoint is inside that box,
    # and consecutive segments share their end points
    T = kd_tree(W)
    lo, hi = T.leaf_boxes()
    o, k = W.random_rays(300, BOX, seed=6)
    tau, tot, cell, length, nseg = orc.trace(BOX, (T.n_cells, 1, 1), np.ones(T.n_cells), 1.0, o, k,
                                             max_seg=T.n_cells, tree=T.tree())
    tin, tout, hit = slab(BOX, o, k)
    for q in np.nonzero(hit)[0]:
        m = nseg[q]
        ends = tin[q] + np.cumsum(length[q, :m])
        mids = ends - 0.5 * length[q, :m]
        p = o[q][None, :] + mids[:, None] * k[q][None, :]
        c = cell[q, :m]
        assert np.all((p >= lo[c] - 1e-12) & (p <= hi[c] + 1e-12))
        assert abs(ends[-1] - tout[q]) < 1e-12


def test_run_on_regular_tree_equals_the_regular_run(orc, W):
    levels, n = (2, 3, 2), (4, 8, 4)
    rho = W.lognormal_density(n, 0.6, seed=23)
    p = W.small_problem(n=n, rho=rho, kappa=1.4, albedo=0.7, g=0.4, n_packages=500,
                        detectors=[W.frame(10.0, 40.0, 12, 12, 1.2, 1.2, azim=15.0)])
    img0, ab0, st0 = orc.run(p)
    T = W.regular_tree(BOX, levels)
    q = dict(p, n=(T.n_cells, 1, 1), rho=rho.reshape(1, 1, -1), tree=T.tree())
    img1, ab1, st1 = orc.run(q)
    np.testing.assert_allclose(img1, img0, rtol=1e-9, atol=1e-12 * np.abs(img0).max())
    np.testing.assert_allclose(ab1.reshape(-1), ab0.reshape(-1), rtol=1e-9, atol=1e-12 * np.abs(ab0).max())
    assert st1["events"] == st0["events"] and st1["x_path"] == st0["x_path"]


def test_direct_flux_is_exact_on_an_octree(orc, W):
    # uniform medium: every package sees tau = kappa * 1 along +z from the origin
    T = octree(W)
    p = W.tree_problem("oct", BOX, T, lambda x, y, z: np.ones_like(x), 1.0, 0.6, 0.5, [W.point()],
                       [W.frame(10.0, 0.0, 64, 64, 1.0, 1.0)], 1500, 0, flags=W.FLAGS_DEFAULT | W.FLAG_SPLIT)
    img, ab, st = orc.run(p)
    direct = W.split_frames(p, img[0, 0])[0]
    expect = np.exp(-1.0) / (4 * np.pi * 100.0)
    assert abs(direct[32, 32] - expect) < 1e-13 * expect
    direct[32, 32] = 0
    assert np.all(direct == 0)
    closure = st["absorbed"] + st["escaped"] + st["truncated"] - st["emitted"]
    assert abs(closure) < 1e-12


def test_gradient_matches_replay_finite_differences(orc, W):
    T = kd_tree(W, max_mass=0.1, depth=8)
    p = W.tree_problem("kd", BOX, T, _blob, 1.2, 0.7, 0.45, [W.point((0.13, -0.21, 0.07))],
                       [W.frame(10.0, 30.0, 12, 12, 1.0, 1.0, azim=20.0)], 800, 0,
                       flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT, w_min=1e-3, max_scatter=50)
    img, _, _ = orc.run(p)
    target = img * (1 + 0.3 * np.random.default_rng(5).standard_normal(img.shape))
    adj = 2 * (img - target)
    g, _, _ = orc.grad(p, adj)
    rho0 = p["rho"].reshape(-1)

    def loss(r):
        im, _ = orc.reweight(p, r)
        return ((im - target) ** 2).sum()

    gmax = np.abs(g).max()
    for m in np.argsort(-np.abs(g))[:8]:
        h = 1e-4 * rho0[m]
        rp, rm = rho0.copy(), rho0.copy()
        rp[m] += h
        rm[m] -= h
        fd = (loss(rp) - loss(rm)) / (2 * h)
        assert abs(fd - g[m]) <= 1e-6 * abs(g[m]) + 1e-8 * gmax, (m, fd, g[m])
