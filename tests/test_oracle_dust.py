"""Pins of the oracle's dust emission and cell sources (Sect. 1: the dust
absorbs and re-emits; Sect. 2.1: panchromatic simulations).

Dust emission: grains are modified black bodies in equilibrium; the
temperature of a cell is the one at which it emits what it absorbed.  The
pins do not retype the oracle's sum: one wavelength has a closed-form
temperature; grey and lambda^-2 opacities over a wide fine grid reduce the
sum to the integrals int lambda^-5-beta / (e^(c2/lambda T) - 1) dlambda =
(T/c2)^(4+beta) Gamma(4+beta) zeta(4+beta), with zeta(4) = pi^4/90 and
zeta(6) = pi^6/945; the spectrum peaks where Wien's displacement law puts
it; every cell re-emits its absorbed luminosity; cell volumes come from the
planes and the tree builder's own leaf boxes.

Cell sources: with no dust on the way the emission peel-off of each package
lands in the pixel of the cell it started in, so the images count the cells
drawn (multinomial in the cells' luminosities, never a dark cell) and the
positions inside a cell (uniform)."""
import math

import numpy as np
import pytest

C2 = 14387.77
WIEN_X = 4.965114231744276  # root of x = 5 (1 - e^-x)


def _one_cell(box=(0.0, 2.0, 0.0, 1.0, 0.0, 0.5)):
    return box, (1, 1, 1)


def _closed_form_T(a, b, y):
    # a / (exp(b / T) - 1) = y  <=>  T = b / ln(1 + a / y)
    return b / math.log1p(a / y)


@pytest.mark.parametrize("y_scale", [1e-3, 1.0, 1e3])
def test_single_wavelength_temperature_is_the_closed_form(orc, y_scale):
    lam, dlam, ka, eps = 100.0, 10.0, 2.0, 3.0
    a, b = ka * dlam / lam ** 5, C2 / lam
    box, n = _one_cell()
    V = 2.0 * 1.0 * 0.5
    for T_true in (3.0, 17.5, 60.0, 900.0):
        y = a / math.expm1(b / T_true) * y_scale
        rho = np.array([0.7])
        L = y * eps * rho[0] * V
        T, em = orc.dust_emission(box, n, rho, np.array([[L]]), [lam], [dlam], [ka], eps)
        want = _closed_form_T(a, b, y)
        want = min(max(want, 1.0), 1e5)
        assert abs(T[0] - want) <= 1e-13 * want, (T[0], want)
        assert abs(em[0, 0] - L) <= 1e-14 * L


def _log_grid(lo, hi, n):
    edges = np.geomspace(lo, hi, n + 1)
    return np.sqrt(edges[1:] * edges[:-1]), np.diff(edges)


@pytest.mark.parametrize("T_true", [15.0, 40.0, 150.0])
def test_grey_dust_follows_the_stefan_boltzmann_integral(orc, T_true):
    lam, dlam = _log_grid(0.5, 3e5, 60000)
    ka = np.full(lam.size, 0.3)
    box, n = _one_cell()
    eps, rho = 2.0, np.array([1.5])
    # sum_i ka B dlambda -> ka (T/c2)^4 pi^4 / 15
    y = 0.3 * (T_true / C2) ** 4 * math.pi ** 4 / 15.0
    L = y * eps * rho[0] * 1.0
    T, em = orc.dust_emission(box, n, rho, np.array([[L]]), lam, dlam, ka, eps)
    assert abs(T[0] / T_true - 1.0) < 2e-6, T[0]
    assert abs(em.sum() / L - 1.0) < 1e-13
    # Wien: the emission per unit wavelength peaks at lambda T = c2 / x
    peak = lam[np.argmax(em[:, 0] / dlam)]
    assert abs(peak * T[0] / (C2 / WIEN_X) - 1.0) < 3e-4


def test_lambda_minus_two_dust_follows_its_integral(orc):
    lam, dlam = _log_grid(0.5, 3e5, 60000)
    k0, l0, T_true = 0.8, 100.0, 25.0
    ka = k0 * (lam / l0) ** -2.0
    box, n = _one_cell()
    # sum_i ka B dlambda -> k0 l0^2 (T/c2)^6 Gamma(6) zeta(6)
    y = k0 * l0 ** 2 * (T_true / C2) ** 6 * 120.0 * math.pi ** 6 / 945.0
    rho = np.array([0.25])
    L = y * 1.0 * rho[0] * 1.0
    T, _ = orc.dust_emission(box, n, rho, np.array([[L]]), lam, dlam, ka, 1.0)
    assert abs(T[0] / T_true - 1.0) < 2e-6, T[0]
    assert abs(orc.mbb_sum(lam, dlam, ka, T_true) / y - 1.0) < 1e-5


def _spectrum():
    lam = np.geomspace(1.0, 2000.0, 40)
    return lam, np.diff(np.geomspace(0.9, 2200.0, 41)), 0.5 * (lam / 100.0) ** -1.5


def test_every_cell_reemits_what_it_absorbed(orc):
    lam, dlam, ka = _spectrum()
    rng = np.random.default_rng(3)
    box, n = (-1.0, 1.0, -2.0, 2.0, 0.0, 1.0), (5, 4, 3)
    rho = rng.lognormal(0.0, 1.0, 60)
    rows = rng.lognormal(-9.0, 1.5, (3, 60))
    T, em = orc.dust_emission(box, n, rho, rows, lam, dlam, ka, 1e13)
    L = rows.sum(axis=0)
    np.testing.assert_allclose(em.sum(axis=0), L, rtol=1e-13)
    assert np.all((T >= 1.0) & (T <= 1e5))
    # the rows only enter through their sum
    T1, em1 = orc.dust_emission(box, n, rho, L[None, :], lam, dlam, ka, 1e13)
    np.testing.assert_allclose(T1, T, rtol=1e-13)
    np.testing.assert_allclose(em1, em, rtol=1e-12)
    # hotter where the absorbed luminosity per unit mass is larger
    q = L / rho
    order = np.argsort(q)
    assert np.all(np.diff(T[order]) >= 0.0)


def test_degenerate_cells(orc):
    lam, dlam, ka = np.array([300.0, 1000.0]), np.array([30.0, 100.0]), np.array([1.0, 0.3])
    box, n = (0.0, 4.0, 0.0, 1.0, 0.0, 1.0), (4, 1, 1)
    rho = np.array([1.0, 0.0, 1.0, 1.0])
    L = np.array([0.0, 1.0, 1e-200, 1e30])
    T, em = orc.dust_emission(box, n, rho, L[None, :], lam, dlam, ka, 1.0)
    assert T[0] == 0.0 and np.all(em[:, 0] == 0.0)  # nothing absorbed
    assert T[1] == 0.0 and np.all(em[:, 1] == 0.0)  # no dust
    assert T[2] == 1.0  # colder than 1 K: held at 1 K, still re-emits L
    assert abs(em[:, 2].sum() / 1e-200 - 1.0) < 1e-13
    assert abs(T[3] / 1e5 - 1.0) < 1e-14  # hotter than 1e5 K: held at 1e5 K
    assert abs(em[:, 3].sum() / 1e30 - 1.0) < 1e-13


def test_cell_volumes_of_rectilinear_and_tree_grids(orc, W):
    lam, dlam, ka, eps = [200.0], [20.0], [1.3], 5.0
    a, b = 1.3 * 20.0 / 200.0 ** 5, C2 / 200.0
    box = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)
    planes = tuple(W.power_law_planes(-1.0, 1.0, m, r) for m, r in ((6, 8.0), (5, 3.0), (4, 12.0)))
    n = (6, 5, 4)
    V = np.einsum("k,j,i->kji", np.diff(planes[2]), np.diff(planes[1]), np.diff(planes[0])).reshape(-1)
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.5, 2.0, V.size)
    L = np.full(V.size, a / math.expm1(b / 30.0) * eps)  # a unit-mass cell would sit at 30 K
    T, _ = orc.dust_emission(box, n, rho, L[None, :], lam, dlam, ka, eps, planes=planes)
    want = np.array([_closed_form_T(a, b, L[m] / (eps * rho[m] * V[m])) for m in range(V.size)])
    np.testing.assert_allclose(T, want, rtol=1e-13)

    tree = W.adaptive_tree(box, lambda x, y, z: 0.3 + np.exp(-6.0 * (x * x + y * y + z * z)), 0.05, 10)
    lo, hi = tree.leaf_boxes()
    Vt = np.prod(hi - lo, axis=1)
    rho_t = rng.uniform(0.5, 2.0, tree.n_cells)
    Lt = np.full(tree.n_cells, L[0])
    T, _ = orc.dust_emission(box, (tree.n_cells, 1, 1), rho_t, Lt[None, :], lam, dlam, ka, eps, tree=tree.tree())
    want = np.array([_closed_form_T(a, b, Lt[m] / (eps * rho_t[m] * Vt[m])) for m in range(tree.n_cells)])
    np.testing.assert_allclose(T, want, rtol=1e-13)


# --------------------------------------------------------------------------
# Cell sources, with no dust: the emission peel-off of a package lands in
# its cell's pixel with weight w0 / (4 pi d^2).

def _cells_problem(W, n, box, cell_lum, n_packages, det, flags=1, seed=11):
    rho = np.zeros((n[2], n[1], n[0]))
    p = W.small_problem(n=n, box=box, rho=rho, kappa=1.0, albedo=0.5, g=0.3, sources=[W.cells(cell_lum)],
                        detectors=[det], n_packages=n_packages, flags=flags)
    p["seed"] = seed
    return p


def _pixel_of(orc, det, r):
    _, ex, ey = orc.detector_basis(det)
    x, y = float(np.dot(r, ex)), float(np.dot(r, ey))
    ix = int(math.floor((x + det["half_x"]) / (2 * det["half_x"]) * det["nx"]))
    iy = int(math.floor((y + det["half_y"]) / (2 * det["half_y"]) * det["ny"]))
    return ix + det["nx"] * iy


def test_cells_are_drawn_in_proportion_to_their_luminosity(orc, W):
    from scipy import stats
    n, box = (6, 5, 1), (-3.0, 3.0, -2.5, 2.5, -0.5, 0.5)
    rng = np.random.default_rng(2)
    lum = rng.uniform(0.0, 1.0, 30)
    lum[[0, 7, 29]] = 0.0  # dark cells, one at each end
    d = 100.0
    det = W.frame(d, 0.0, 6, 5, 3.0, 2.5)  # one pixel per cell footprint
    N = 60000
    img, _, st = orc.run(_cells_problem(W, n, box, lum[None, :], N, det), threads=8)
    w0 = lum.sum() / N
    counts = img[0, 0] * 4.0 * math.pi * d * d / w0
    assert np.allclose(counts, np.round(counts), atol=1e-6)
    counts = np.round(counts).astype(np.int64)
    assert counts.sum() == N and st["packages"] == N
    # map cells to pixels through the frame's own basis
    xs = np.linspace(-3.0, 3.0, 7)
    ys = np.linspace(-2.5, 2.5, 6)
    per_cell = np.zeros(30, dtype=np.int64)
    for m in range(30):
        i, j = m % 6, m // 6
        c = np.array([0.5 * (xs[i] + xs[i + 1]), 0.5 * (ys[j] + ys[j + 1]), 0.0])
        per_cell[m] = counts[_pixel_of(orc, det, c)]
    assert np.all(per_cell[lum == 0.0] == 0)
    live = lum > 0.0
    expect = N * lum[live] / lum.sum()
    chi2 = ((per_cell[live] - expect) ** 2 / expect).sum()
    assert stats.chi2.sf(chi2, live.sum() - 1) > 1e-4, chi2


def test_positions_are_uniform_inside_the_cell(orc, W):
    from scipy import stats
    n, box = (3, 3, 3), (-1.5, 1.5, -1.5, 1.5, -1.5, 1.5)
    lum = np.zeros(27)
    lum[13] = 2.0  # the centre cell [-0.5, 0.5]^3 only
    d = 50.0
    det = W.frame(d, 0.0, 8, 8, 0.5, 0.5)  # the centre cell's footprint, 8x8 pixels
    N = 32000
    img, _, _ = orc.run(_cells_problem(W, n, box, lum[None, :], N, det), threads=8)
    counts = img[0, 0] * 4.0 * math.pi * d * d / (2.0 / N)
    assert abs(counts.sum() - N) < 1e-6 * N  # every package in the footprint
    chi2 = ((counts - N / 64.0) ** 2 / (N / 64.0)).sum()
    assert stats.chi2.sf(chi2, 63) > 1e-4, chi2


def test_dark_wavelengths_launch_no_packages_and_energy_closes(orc, W):
    n, box = (4, 4, 4), (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)
    rng = np.random.default_rng(9)
    lum = np.stack([rng.uniform(0.0, 1.0, 64), np.zeros(64), rng.uniform(0.0, 3.0, 64)])
    rho = W.lognormal_density(n, 0.5, seed=4)
    p = W.small_problem(n=n, box=box, rho=rho, kappa=[1.0, 2.0, 0.5], albedo=[0.6, 0.5, 0.4], g=[0.3, 0.2, 0.1],
                        sources=[W.cells(lum)], detectors=[W.frame(10.0, 30.0, 8, 8, 1.5, 1.5)], n_packages=500,
                        flags=W.FLAGS_DEFAULT | W.FLAG_SPLIT)
    img, absorbed, st = orc.run(p)
    assert np.all(img[:, 1] == 0.0) and np.all(absorbed[1] == 0.0)
    assert st["packages"] == 1500
    assert abs(st["emitted"] - lum.sum()) < 1e-12 * lum.sum()
    closure = st["absorbed"] + st["escaped"] + st["truncated"] - st["emitted"]
    assert abs(closure) < 1e-12 * st["emitted"]
    # the dark wavelength alone: no events at all
    p1 = dict(p, kappa=p["kappa"][1:2], albedo=p["albedo"][1:2], g=p["g"][1:2],
              sources=[W.cells(lum[1:2])])
    _, _, s1 = orc.run(p1)
    assert s1["packages"] == 500 and s1["events"] == 0 and s1["x_path"] == 0 and s1["emitted"] == 0.0
