"""The library's lane code on rectilinear grids (planes spaced by any rule
along each axis; PowCub's power-law spacing, Table 1(d)), run on the CPU by
the bounds-checked harness against the FP64 oracle: walks, peel-off,
forward runs and the adjoint, in both precisions.  The harness keeps each
plane table between NaN guards, so a read outside a table breaks the
results compared here."""
import numpy as np
import pytest

from test_oracle_rectilinear import random_planes


def rel_l1(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a).sum())


def _grids(W):
    rng = np.random.default_rng(29)
    box_r = (-2.0, 1.0, 0.0, 3.0, -1.0, 0.5)
    n_r = (9, 6, 5)
    return {
        "powcub": ((-1, 1, -1, 1, -1, 1), (16, 12, 10),
                   tuple(W.power_law_planes(-1.0, 1.0, m, r) for m, r in ((16, 20.0), (12, 5.0), (10, 30.0)))),
        "random_ragged": (box_r, n_r, tuple(random_planes(box_r[2 * a], box_r[2 * a + 1], n_r[a], rng)
                                            for a in range(3))),
        "one_cell": ((-1, 1, -1, 1, -1, 1), (1, 1, 1), tuple(np.array([-1.0, 1.0]) for _ in range(3))),
    }


@pytest.mark.parametrize("grid", ["powcub", "random_ragged", "one_cell"])
@pytest.mark.parametrize("prec", [0, 1])
def test_trace(E, orc, W, grid, prec):
    box, n, planes = _grids(W)[grid]
    rho = W.lognormal_density(n, 1.0, seed=7, f32=(prec == 1))
    o, k = W.random_rays(3001, box, seed=19)
    max_seg = int(sum(n)) + 4
    tau_o, tot_o, cell_o, len_o, nseg_o = orc.trace(box, n, rho, 0.9, o, k, max_seg=max_seg, planes=planes)
    rc, tau, tot, cell, length, nseg = E.trace(box, n, rho, 0.9, prec, o, k, max_seg=max_seg, planes=planes)
    assert rc == 0
    tol = 1e-12 if prec == 0 else 2e-6
    np.testing.assert_allclose(tau, tau_o, rtol=tol, atol=tol * max(1.0, tau_o.max()) * 1e-3)
    same = nseg == nseg_o
    assert same.mean() > (0.999 if prec == 0 else 0.99), same.mean()
    for q in np.nonzero(same)[0]:
        m = nseg[q]
        if not np.array_equal(cell[q, :m], cell_o[q, :m].astype(np.int32)):
            assert min(len_o[q, :m].min(), length[q, :m].min()) < 1e-6 * max(box[1] - box[0], 1.0)
            continue
        np.testing.assert_allclose(length[q, :m], len_o[q, :m], rtol=tol, atol=tol * max(box[1] - box[0], 1.0))
    assert abs(tot - tot_o) <= 1e-3 * tot_o + 2


def test_regular_planes_match_the_regular_grid(E, W):
    box, n = (-1, 1, -1, 1, -1, 1), (7, 5, 3)
    rho = W.lognormal_density(n, 0.8, seed=3)
    planes = tuple(np.linspace(box[2 * a], box[2 * a + 1], n[a] + 1) for a in range(3))
    o, k = W.random_rays(2000, box, seed=2)
    _, t0, _, c0, l0, n0 = E.trace(box, n, rho, 1.1, 0, o, k, max_seg=32)
    _, t1, _, c1, l1, n1 = E.trace(box, n, rho, 1.1, 0, o, k, max_seg=32, planes=planes)
    np.testing.assert_allclose(t1, t0, rtol=1e-13, atol=1e-14)
    np.testing.assert_array_equal(n1, n0)


@pytest.mark.parametrize("prec", [0, 1])
def test_peel(E, orc, W, prec):
    box, n = (-20, 20, -20, 20, -2, 2), (40, 36, 12)
    planes = tuple(W.power_law_planes(box[2 * a], box[2 * a + 1], n[a], r) for a, r in enumerate((8.0, 8.0, 16.0)))
    rho = W.exp_disk_density(box, n, 2.0, 6.0, 0.25, planes=planes)
    if prec:
        rho = W.as_f32_values(rho)
    pos, din, w = W.random_events(3001, box, seed=5, isotropic=False)
    dets = [W.frame(1e4, inc, 33, 31, 20.0, 20.0) for inc in (0.0, 60.0, 90.0)]
    ref = orc.peel(box, n, rho, 1.1, 0.6, pos, din, w, dets, planes=planes)
    got = E.peel(box, n, rho, 1.1, 0.6, prec, pos, din, w, dets, planes=planes)
    assert rel_l1(got, ref) < (1e-12 if prec == 0 else 1e-6)


def _powcub_problem(W, prec, flags=None, n_packages=800):
    n = (12, 10, 9)
    planes = tuple(W.power_law_planes(-1.0, 1.0, m, r) for m, r in zip(n, (10.0, 6.0, 14.0)))
    rho = W.lognormal_density(n, 0.8, seed=41, f32=(prec == 1))
    p = W.small_problem(n=n, rho=rho, kappa=1.3, albedo=0.7, g=0.4, sources=[W.point((0.11, -0.07, 0.05))],
                        detectors=[W.frame(10.0, 0.0, 20, 20, 1.2, 1.2), W.frame(10.0, 70.0, 16, 24, 1.3, 1.1,
                                                                                   azim=20.0)],
                        n_packages=n_packages, precision=prec,
                        flags=flags if flags is not None else W.FLAGS_DEFAULT | W.FLAG_SPLIT)
    p["planes"] = planes
    return p


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("queue", [-1, 0])
def test_run(E, orc, W, prec, queue):
    p = _powcub_problem(W, prec)
    images, absorbed, st = E.run(p, peel_queue=queue)
    img_o, abs_o, st_o = orc.run(p)
    tol = 1e-10 if prec == 0 else 1e-5
    assert rel_l1(images, img_o) < tol and rel_l1(absorbed, abs_o) < tol
    assert st["packages"] == st_o["packages"]
    for key in ("events", "x_path", "x_locate", "x_peel"):
        assert abs(st[key] - st_o[key]) <= 1e-4 * st_o[key] + 2, (key, st[key], st_o[key])


@pytest.mark.parametrize("prec", [0, 1])
def test_backward(E, orc, W, prec):
    p = _powcub_problem(W, prec, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    img_o, _, _ = orc.run(p)
    adj = np.random.default_rng(8).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(p, adj)
    for queue in (-1, 0):
        g, st = E.grad(p, adj, peel_queue=queue)
        assert rel_l1(g, g_o) < (1e-9 if prec == 0 else 1e-5), (queue, rel_l1(g, g_o))
