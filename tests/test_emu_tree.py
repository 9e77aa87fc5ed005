"""The library's lane code on tree grids (k-d tree and octree; Table 1(d)),
run on the CPU by the bounds-checked harness against the FP64 oracle:
walks, peel-off, forward runs and the adjoint, in both precisions."""
import numpy as np
import pytest

from test_oracle_tree import BOX, _blob, kd_tree, octree


def rel_l1(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a).sum())


def _tree(W, kind):
    if kind == "kd":
        return kd_tree(W)
    if kind == "oct":
        return octree(W)
    return W.regular_tree(BOX, (3, 2, 2))


@pytest.mark.parametrize("kind", ["kd", "oct", "regular"])
@pytest.mark.parametrize("prec", [0, 1])
def test_trace(E, orc, W, kind, prec):
    T = _tree(W, kind)
    rho = np.random.default_rng(7).lognormal(0.0, 1.0, T.n_cells)
    if prec:
        rho = W.as_f32_values(rho)
    n = (T.n_cells, 1, 1)
    o, k = W.random_rays(2001, BOX, seed=19)
    max_seg = 256
    tau_o, tot_o, cell_o, len_o, nseg_o = orc.trace(BOX, n, rho, 0.9, o, k, max_seg=max_seg, tree=T.tree())
    rc, tau, tot, cell, length, nseg = E.trace(BOX, n, rho, 0.9, prec, o, k, max_seg=max_seg, tree=T.tree())
    assert rc == 0
    tol = 1e-12 if prec == 0 else 2e-6
    np.testing.assert_allclose(tau, tau_o, rtol=tol, atol=tol * max(1.0, tau_o.max()) * 1e-3)
    same = nseg == nseg_o
    assert same.mean() > (0.999 if prec == 0 else 0.99), same.mean()
    for q in np.nonzero(same)[0]:
        m = nseg[q]
        if not np.array_equal(cell[q, :m], cell_o[q, :m].astype(np.int32)):
            assert min(len_o[q, :m].min(), length[q, :m].min()) < 1e-6
            continue
        np.testing.assert_allclose(length[q, :m], len_o[q, :m], rtol=tol, atol=tol * 2.0)
    assert abs(tot - tot_o) <= 1e-3 * tot_o + 2


@pytest.mark.parametrize("prec", [0, 1])
def test_peel(E, orc, W, prec):
    T = kd_tree(W)
    rho = W.as_f32_values(_blob(*(0.5 * (np.add(*T.leaf_boxes()))).T)) if prec else _blob(
        *(0.5 * (np.add(*T.leaf_boxes()))).T)
    pos, din, w = W.random_events(2001, BOX, seed=5, isotropic=False)
    dets = [W.frame(10.0, inc, 17, 15, 1.1, 1.1) for inc in (0.0, 60.0, 90.0)]
    n = (T.n_cells, 1, 1)
    ref = orc.peel(BOX, n, rho, 1.1, 0.6, pos, din, w, dets, tree=T.tree())
    got = E.peel(BOX, n, rho, 1.1, 0.6, prec, pos, din, w, dets, tree=T.tree())
    assert rel_l1(got, ref) < (1e-12 if prec == 0 else 1e-6)


def _tree_problem(W, kind, prec, flags=None, n_packages=700):
    T = kd_tree(W, max_mass=0.05, depth=10) if kind == "kd" else octree(W)
    return W.tree_problem(kind, BOX, T, _blob, 1.3, 0.7, 0.4, [W.point((0.11, -0.07, 0.05))],
                          [W.frame(10.0, 0.0, 20, 20, 1.2, 1.2), W.frame(10.0, 70.0, 16, 24, 1.3, 1.1, azim=20.0)],
                          n_packages, prec, flags=flags if flags is not None else W.FLAGS_DEFAULT | W.FLAG_SPLIT)


@pytest.mark.parametrize("kind", ["kd", "oct"])
@pytest.mark.parametrize("prec", [0, 1])
def test_run(E, orc, W, kind, prec):
    p = _tree_problem(W, kind, prec)
    img_o, abs_o, st_o = orc.run(p)
    tol = 1e-10 if prec == 0 else 1e-5
    for queue in (-1, 0):
        images, absorbed, st = E.run(p, peel_queue=queue)
        assert rel_l1(images, img_o) < tol and rel_l1(absorbed, abs_o) < tol, queue
        assert st["packages"] == st_o["packages"]
        for key in ("events", "x_path", "x_locate", "x_peel"):
            assert abs(st[key] - st_o[key]) <= 1e-4 * st_o[key] + 2, (key, st[key], st_o[key])


@pytest.mark.parametrize("kind", ["kd", "oct"])
@pytest.mark.parametrize("prec", [0, 1])
def test_backward(E, orc, W, kind, prec):
    p = _tree_problem(W, kind, prec, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    img_o, _, _ = orc.run(p)
    adj = np.random.default_rng(8).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(p, adj)
    for queue in (-1, 0):
        g, st = E.grad(p, adj, peel_queue=queue)
        assert rel_l1(g, g_o) < (1e-9 if prec == 0 else 1e-5), (queue, rel_l1(g, g_o))
