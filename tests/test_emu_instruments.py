"""The library's instruments (Sect. 2.2: SED and frame instruments of a
distant observer; perspective cameras anywhere, also inside the model) in
the bounds-checked CPU harness of its lane code, against the FP64 oracle:
forward runs with the peel rays queued and walked inline, the adjoint, and
the standalone peel-off, on regular, rectilinear and tree grids, in both
precisions."""
import numpy as np
import pytest

from test_oracle_tree import BOX, _blob, kd_tree


def rel_l1(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a).sum())


def instruments(W):
    return [W.frame(10.0, 30.0, 12, 10, 1.2, 1.1, azim=15.0),
            W.sed(10.0, 75.0, azim=-40.0),
            W.perspective((0.2, -0.1, 0.35), (0.8, 0.6, -0.5), (0.0, 0.0, 1.0), 11, 9, 1.5, 1.2),  # inside
            W.perspective((2.5, -3.0, 1.5), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 13, 13, 1.0, 1.0)]  # outside


def problem(W, grid, prec, n_packages=700, flags=None):
    n = (7, 6, 5)
    if grid == "tree":
        T = kd_tree(W, max_mass=0.05, depth=10)
        return W.tree_problem("tree", BOX, T, _blob, 1.3, 0.7, 0.4, [W.point((0.11, -0.07, 0.05))],
                              instruments(W), n_packages, prec,
                              flags=flags if flags is not None else W.FLAGS_DEFAULT | W.FLAG_SPLIT)
    rho = W.lognormal_density(n, 0.8, seed=41, f32=(prec == 1))
    p = W.small_problem(n=n, box=BOX, rho=rho, kappa=1.3, albedo=0.7, g=0.4, sources=[W.point((0.11, -0.07, 0.05))],
                        detectors=instruments(W), n_packages=n_packages, precision=prec,
                        flags=flags if flags is not None else W.FLAGS_DEFAULT | W.FLAG_SPLIT)
    if grid == "rect":
        p["planes"] = tuple(W.power_law_planes(-1.0, 1.0, m, r) for m, r in zip(n, (6.0, 3.0, 9.0)))
    return p


@pytest.mark.parametrize("grid", ["regular", "rect", "tree"])
@pytest.mark.parametrize("prec", [0, 1])
def test_run_matches_oracle(E, orc, W, grid, prec):
    p = problem(W, grid, prec)
    img_o, abs_o, st_o = orc.run(p)
    tol = 1e-10 if prec == 0 else 1e-5
    for queue in (-1, 0, 150):
        images, absorbed, st = E.run(p, peel_queue=queue)
        assert rel_l1(images, img_o) < tol and rel_l1(absorbed, abs_o) < tol, queue
        for key in ("events", "x_path", "x_locate", "x_peel"):
            assert abs(st[key] - st_o[key]) <= 1e-4 * st_o[key] + 2, (key, st[key], st_o[key])
    # every instrument saw light
    off = np.cumsum([0] + [d["nx"] * d["ny"] for d in p["detectors"]])
    for d in range(4):
        assert img_o[:, :, off[d]:off[d + 1]].sum() > 0, d


@pytest.mark.parametrize("grid", ["regular", "tree"])
def test_adjoint_matches_oracle(E, orc, W, grid):
    p = problem(W, grid, 0, n_packages=400, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    img_o, _, _ = orc.run(p)
    adj = np.random.default_rng(8).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(p, adj)
    for queue in (-1, 0):
        g, _ = E.grad(p, adj, peel_queue=queue)
        assert rel_l1(g, g_o) < 1e-9, queue


@pytest.mark.parametrize("prec", [0, 1])
def test_standalone_peel_matches_oracle(E, orc, W, prec):
    n = (7, 6, 5)
    rho = W.lognormal_density(n, 0.8, seed=3, f32=(prec == 1))
    pos, din, w = W.random_events(3001, BOX, seed=5, isotropic=False)
    ref = orc.peel(BOX, n, rho, 1.1, 0.6, pos, din, w, instruments(W))
    got = E.peel(BOX, n, rho, 1.1, 0.6, prec, pos, din, w, instruments(W))
    assert rel_l1(got, ref) < (1e-12 if prec == 0 else 1e-6)
