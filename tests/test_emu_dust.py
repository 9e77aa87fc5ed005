"""The library's dust emission and cell sources, run on the CPU by the
bounds-checked harness of its lane and per-cell code, against the FP64
oracle: equilibrium temperatures and spectra on regular, rectilinear and
tree grids (FP64 and FP32 densities), and forward and adjoint runs whose
only source is the cells (Sect. 1 and 2.1), in both precisions."""
import numpy as np
import pytest

from test_oracle_tree import BOX, _blob, kd_tree


def rel_l1(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a).sum())


def spectrum(n_lambda=30):
    lam = np.geomspace(1.0, 1000.0, n_lambda)
    i = np.arange(n_lambda)
    return lam, lam * (10 ** (1.5 / (n_lambda - 1)) - 10 ** (-1.5 / (n_lambda - 1))), \
        (np.maximum(lam, 0.5) / 0.55) ** -1.5 * (1.0 - 0.6 * (1.0 - i / (n_lambda - 1)))


def grids(W):
    planes = tuple(W.power_law_planes(-1.0, 1.0, m, r) for m, r in ((9, 8.0), (7, 3.0), (5, 12.0)))
    T = kd_tree(W, max_mass=0.05, depth=10)
    return {"regular": {"box": BOX, "n": (9, 7, 5)},
            "rect": {"box": BOX, "n": (9, 7, 5), "planes": planes},
            "tree": {"box": BOX, "n": (T.n_cells, 1, 1), "tree": T.tree()}}


def absorbed_field(ncell, seed, n_abs=2):
    rng = np.random.default_rng(seed)
    a = rng.lognormal(-8.0, 2.0, (n_abs, ncell))
    a[:, rng.choice(ncell, ncell // 10, replace=False)] = 0.0  # cells that absorbed nothing
    return a


@pytest.mark.parametrize("grid", ["regular", "rect", "tree"])
@pytest.mark.parametrize("prec", [0, 1])
def test_dust_emission_matches_oracle(E, orc, W, grid, prec):
    g = grids(W)[grid]
    ncell = int(np.prod(g["n"]))
    rng = np.random.default_rng(4)
    rho = rng.lognormal(0.0, 1.0, ncell)
    rho[rng.choice(ncell, 5, replace=False)] = 0.0  # dust-free cells
    if prec:
        rho = W.as_f32_values(rho)
    ab = absorbed_field(ncell, 8)
    lam, dlam, ka = spectrum()
    eps = 3e12
    T_o, em_o = orc.dust_emission(g["box"], g["n"], rho, ab, lam, dlam, ka, eps, planes=g.get("planes"),
                                  tree=g.get("tree"))
    T, em = E.dust_emission(g["box"], g["n"], rho, prec, ab, lam, dlam, ka, eps, planes=g.get("planes"),
                            tree=g.get("tree"))
    hot = T_o > 0
    assert np.array_equal(T > 0, hot)
    assert hot.sum() > ncell // 2 and T_o[hot].min() > 1.0 and T_o[hot].max() < 1e5
    np.testing.assert_allclose(T[hot], T_o[hot], rtol=1e-12)
    assert rel_l1(em, em_o) < 1e-12
    np.testing.assert_allclose(em.sum(axis=0)[hot], ab.sum(axis=0)[hot], rtol=1e-13, atol=0)
    assert np.all(em[:, ~hot] == 0.0)


def test_dust_emission_clamps_and_extremes(E, orc, W):
    # temperatures pinned at both ends of the range, and cells whose root
    # sits in the table's first and last intervals
    lam, dlam, ka = spectrum(12)
    n = (8, 1, 1)
    box = (0.0, 8.0, 0.0, 1.0, 0.0, 1.0)
    rho = np.ones(8)
    P = [orc.mbb_sum(lam, dlam, ka, T) for T in (0.5, 1.005, 2.0, 300.0, 9.9e4, 2e5)]
    L = np.array([P[0], P[1], P[2], P[3], P[4], P[5], 0.0, 1e-290])
    T_o, em_o = orc.dust_emission(box, n, rho, L[None, :], lam, dlam, ka, 1.0)
    T, em = E.dust_emission(box, n, rho, 0, L[None, :], lam, dlam, ka, 1.0)
    np.testing.assert_allclose(T, T_o, rtol=1e-12)
    np.testing.assert_allclose(em, em_o, rtol=1e-11, atol=1e-300)
    assert T[0] == 1.0 and T[5] == 1e5 and T[6] == 0.0 and T[7] == 1.0


def _cells_problem(W, grid, prec, n_packages=600, flags=None, n_lambda=3, dark=1):
    g = grids(W)[grid]
    ncell = int(np.prod(g["n"]))
    rng = np.random.default_rng(21)
    lum = rng.lognormal(0.0, 1.5, (n_lambda, ncell))
    lum[:, rng.choice(ncell, ncell // 4, replace=False)] = 0.0
    if dark is not None:
        lum[dark] = 0.0  # a wavelength at which nothing is emitted
    if grid == "tree":
        T = kd_tree(W, max_mass=0.05, depth=10)
        lo, hi = T.leaf_boxes()
        c = 0.5 * (lo + hi)
        rho = _blob(c[:, 0], c[:, 1], c[:, 2]).reshape(1, 1, -1)
    else:
        rho = W.lognormal_density(g["n"], 0.8, seed=41)
    if prec:
        rho = W.as_f32_values(rho)
    p = W.small_problem(n=g["n"], box=g["box"], rho=rho, kappa=np.linspace(1.5, 0.6, n_lambda),
                        albedo=np.linspace(0.7, 0.3, n_lambda), g=np.linspace(0.5, 0.1, n_lambda),
                        sources=[W.cells(lum), W.point((0.1, -0.2, 0.05), lum=0.3 * lum.sum(axis=1) / ncell)],
                        detectors=[W.frame(10.0, 0.0, 20, 20, 1.2, 1.2),
                                   W.frame(10.0, 70.0, 16, 24, 1.3, 1.1, azim=20.0)],
                        n_packages=n_packages, precision=prec,
                        flags=flags if flags is not None else W.FLAGS_DEFAULT | W.FLAG_SPLIT)
    for k in ("planes", "tree"):
        if k in g:
            p[k] = g[k]
    return p


@pytest.mark.parametrize("grid", ["regular", "rect", "tree"])
@pytest.mark.parametrize("prec", [0, 1])
def test_cell_source_run_matches_oracle(E, orc, W, grid, prec):
    p = _cells_problem(W, grid, prec)
    img_o, abs_o, st_o = orc.run(p)
    tol = 1e-10 if prec == 0 else 1e-5
    for queue in (-1, 0):
        images, absorbed, st = E.run(p, peel_queue=queue)
        assert rel_l1(images, img_o) < tol and rel_l1(absorbed, abs_o) < tol, queue
        assert st["packages"] == st_o["packages"] == 3 * p["n_packages"]
        assert abs(st["emitted"] - st_o["emitted"]) <= 1e-12 * st_o["emitted"]
        for key in ("events", "x_path", "x_locate", "x_peel"):
            assert abs(st[key] - st_o[key]) <= 1e-4 * st_o[key] + 2, (key, st[key], st_o[key])
    assert np.all(images[:, 1] == 0.0)


@pytest.mark.parametrize("grid", ["regular", "tree"])
def test_cell_source_adjoint_matches_oracle(E, orc, W, grid):
    p = _cells_problem(W, grid, 0, n_packages=400, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    img_o, _, _ = orc.run(p)
    adj = np.random.default_rng(8).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(p, adj)
    g, _ = E.grad(p, adj)
    assert rel_l1(g, g_o) < 1e-9


def test_bad_cell_luminosities_are_rejected(E, W):
    import paper_1410_1629_amd.binding as B
    for bad in (-1.0, np.nan, np.inf):
        p = _cells_problem(W, "regular", 0, n_packages=10)
        lum = np.array(p["sources"][0]["cell_lum"])
        lum[2, 5] = bad
        p["sources"][0]["cell_lum"] = lum
        with pytest.raises(B.McrtError, match="cell_lum"):
            E.run(p)
    p = _cells_problem(W, "regular", 0, n_packages=10)
    p["sources"] = [p["sources"][0], p["sources"][0]]
    with pytest.raises(B.McrtError, match="one cell source"):
        E.run(p)
