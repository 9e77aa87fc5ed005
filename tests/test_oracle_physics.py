"""Pins of the oracle's sampling steps and of whole runs against closed
forms, quadratures and exact identities."""
import os

import numpy as np
import pytest
from scipy import integrate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- sampling

@pytest.mark.parametrize("g", [0.0, 1e-7, 0.3, 0.5, 0.6, 0.9, -0.4])
def test_hg_phase_normalised_and_sampler_inverts_its_cdf(orc, g):
    total, _ = integrate.quad(lambda mu: 2 * np.pi * orc.hg_phase(g, mu), -1, 1, epsabs=1e-13, epsrel=1e-12)
    assert abs(total - 1.0) < 1e-10
    for u in (0.01, 0.2, 0.5, 0.77, 0.999):
        mu = orc.hg_mu(g, u)
        cdf, _ = integrate.quad(lambda m: 2 * np.pi * orc.hg_phase(g, m), -1, mu, epsabs=1e-13, epsrel=1e-12)
        assert abs(cdf - u) < 1e-6 if abs(g) >= 1e-6 else abs(cdf - u) < 1e-6


@pytest.mark.parametrize("g", [0.0, 0.5, 0.6, -0.3, 0.95])
def test_hg_sampler_moments(orc, g):
    # stratified deviates: the midpoint rule gives E[mu] = g and E[P2(mu)] = g^2
    n = 20000
    u = (np.arange(n) + 0.5) / n
    mu = np.array([orc.hg_mu(g, x) for x in u])
    assert abs(mu.mean() - g) < 2e-5
    assert abs((1.5 * mu * mu - 0.5).mean() - g * g) < 2e-4
    assert np.all(np.abs(mu) <= 1.0)


def test_rotation_preserves_angle_and_norm(orc):
    rng = np.random.default_rng(1)
    ks = rng.standard_normal((300, 3))
    ks /= np.linalg.norm(ks, axis=1, keepdims=True)
    ks = np.vstack([ks, [[0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0], [0, -1.0, 0]]])
    for k in ks:
        mu, psi = rng.uniform(-1, 1), rng.uniform(0, 2 * np.pi)
        out = orc.rotate(k, mu, psi)
        assert abs(np.linalg.norm(out) - 1) < 1e-15 * 4
        assert abs(out @ k - mu) < 1e-13
    # averaging over the azimuth leaves only mu * k
    k = ks[5]
    psis = (np.arange(64) + 0.5) * 2 * np.pi / 64
    mean = np.mean([orc.rotate(k, 0.3, p) for p in psis], axis=0)
    np.testing.assert_allclose(mean, 0.3 * k, atol=1e-13)


@pytest.mark.parametrize("T", [1e-6, 0.1, 1.0, 7.0, 40.0])
def test_forced_scattering_law(orc, T):
    n = 20000
    u = (np.arange(n) + 0.5) / n
    ts = np.array([orc.forced_tau(T, x) for x in u])
    assert np.all((ts >= 0) & (ts <= T))
    # the CDF of the truncated exponential maps tau_s back to u
    np.testing.assert_allclose(-np.expm1(-ts) / -np.expm1(-T), u, rtol=1e-12, atol=1e-15)
    mean = 1 - T * np.exp(-T) / -np.expm1(-T)
    assert abs(ts.mean() - mean) < 1e-4 * max(T, 1) * (1 if T > 1e-3 else T)


def test_exponential_disk_emission_moments(orc):
    h_r, h_z = 4.0, 0.4
    w = orc.draw_words(4357, 0, 200_000, 0, 0).astype(np.float64)
    u = (w + 0.5) / 2**32
    pos = np.array([orc.emit_position(1, [1.0, -2.0, 0.5, h_r, h_z], uu) for uu in u[:40000]])
    r = pos - np.array([1.0, -2.0, 0.5])
    R = np.hypot(r[:, 0], r[:, 1])
    n = len(R)
    # Gamma(2, h_R): mean 2 h_R, variance 2 h_R^2; Laplace(h_z): mean 0, E|z| = h_z
    assert abs(R.mean() - 2 * h_r) < 5 * np.sqrt(2 * h_r**2 / n)
    assert abs((R**2).mean() - 6 * h_r**2) < 5 * np.sqrt((120 - 36) * h_r**4 / n)
    assert abs(r[:, 2].mean()) < 5 * np.sqrt(2 * h_z**2 / n)
    assert abs(np.abs(r[:, 2]).mean() - h_z) < 5 * h_z / np.sqrt(n)
    phi = np.arctan2(r[:, 1], r[:, 0])
    assert abs(np.cos(phi).mean()) < 5 / np.sqrt(2 * n) and abs(np.sin(phi).mean()) < 5 / np.sqrt(2 * n)
    # point sources do not move
    np.testing.assert_array_equal(orc.emit_position(0, [1.0, 2.0, 3.0, 0, 0], u[0]), [1.0, 2.0, 3.0])


def test_isotropic_emission_direction(orc):
    w = orc.draw_words(4357, 0, 40000, 0, 1).astype(np.float64)
    u = (w + 0.5) / 2**32
    k = np.array([orc.emit_direction(uu) for uu in u])
    n = len(k)
    np.testing.assert_allclose(np.linalg.norm(k, axis=1), 1.0, atol=1e-15 * 4)
    assert np.all(np.abs(k.mean(axis=0)) < 5 / np.sqrt(3 * n))
    assert np.all(np.abs((k * k).mean(axis=0) - 1 / 3) < 5 * np.sqrt(4 / 45 / n))


def _xz_rows():
    rows = []
    with open(os.path.join(GOLDEN, "frame_xz_instrument.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, b, c = line.split("|")
            rows.append(([float(x) for x in a.split()], [float(x) for x in b.split()],
                         [float(x) for x in c.split()]))
    return rows


@pytest.mark.parametrize("angles,ex,ey", _xz_rows())
def test_frame_orientation_of_the_worked_example(orc, angles, ex, ey):
    det = {"distance": 1e4, "incl": angles[0], "azim": angles[1], "pa": angles[2], "half_x": 1.0, "half_y": 1.0}
    kd, gx, gy = orc.detector_basis(det)
    np.testing.assert_allclose(gx, ex, atol=1e-15)
    np.testing.assert_allclose(gy, ey, atol=1e-15)


def test_frame_basis_is_right_handed_and_position_angle_rotates(orc):
    rng = np.random.default_rng(2)
    for _ in range(50):
        t, p, w = rng.uniform(0, 180), rng.uniform(-180, 180), rng.uniform(-180, 180)
        kd, ex, ey = orc.detector_basis({"distance": 1, "incl": t, "azim": p, "pa": w, "half_x": 1, "half_y": 1})
        np.testing.assert_allclose(np.cross(ex, ey), kd, atol=1e-14)
        np.testing.assert_allclose([ex @ ex, ey @ ey, ex @ ey, ex @ kd], [1, 1, 0, 0], atol=1e-14)
        kd0, ex0, ey0 = orc.detector_basis({"distance": 1, "incl": t, "azim": p, "pa": 0, "half_x": 1, "half_y": 1})
        c, s = np.cos(np.radians(w)), np.sin(np.radians(w))
        np.testing.assert_allclose(ex, c * ex0 + s * ey0, atol=1e-14)
        np.testing.assert_allclose(kd, kd0, atol=1e-15)


# ---------------------------------------------------------------- whole runs

def test_direct_flux_through_uniform_cube_is_exact(orc, W):
    # every package sees the same e^-tau (tau = 1 along +z from the origin):
    # the direct pixel holds L e^-1 / (4 pi D^2) = 2.9275e-4 and nothing else
    p = W.cube(n_packages=5000, flags=W.FLAGS_DEFAULT | W.FLAG_SPLIT)
    img, ab, st = orc.run(p)
    direct = W.split_frames(p, img[0, 0])[0]
    expect = np.exp(-1.0) / (4 * np.pi * 100.0)
    assert abs(direct[32, 32] - expect) < 1e-13 * expect
    assert abs(expect - 2.9275e-4) < 5e-8
    direct[32, 32] = 0
    assert np.all(direct == 0)
    scat = W.split_frames(p, img[1, 0])[0]
    assert scat.sum() > 0


@pytest.mark.parametrize("case", ["cube", "disk", "two_sources_multi_lambda"])
def test_energy_closes_per_run(orc, W, case):
    if case == "cube":
        p = W.cube(n_packages=3000)
    elif case == "disk":
        p = W.small_problem(n=(24, 24, 8), box=(-20, 20, -20, 20, -2, 2), rho=W.exp_disk_density(
            (-20, 20, -20, 20, -2, 2), (24, 24, 8), 2.0, 6.0, 0.25), sources=[W.expdisk(4.0, 0.4)],
            detectors=[W.frame(1e4, i, 32, 32, 20, 20) for i in (0, 60, 90)], n_packages=3000, albedo=0.6, g=0.6)
    else:
        p = W.small_problem(n=(6, 7, 5), rho=W.lognormal_density((6, 7, 5), 1.0, seed=4), kappa=[0.5, 1.0, 2.0],
                            albedo=[0.9, 0.5, 0.0], g=[0.7, 0.0, -0.2],
                            sources=[W.point((0.2, 0.1, -0.3), [1.0, 2.0, 0.5]), W.expdisk(0.3, 0.1, [3.0, 1.0, 1.0])],
                            n_packages=2000)
    img, ab, st = orc.run(p)
    nl = len(p["kappa"])
    lum = sum(np.asarray(s["lum"]) for s in p["sources"]).sum()
    assert abs(st["emitted"] - lum) < 1e-12 * lum
    closure = st["absorbed"] + st["escaped"] + st["truncated"] - st["emitted"]
    assert abs(closure) < 1e-12 * st["emitted"]
    assert abs(ab.sum() - st["absorbed"]) < 1e-12 * st["emitted"]
    assert st["packages"] == nl * p["n_packages"]
    assert st["truncated"] < 1e-3 * st["emitted"]


def _mean_exp_over_sphere(a, n=800):
    """<exp(-a / max|k_i|)> over the unit sphere: Gauss-Legendre in mu times
    midpoint in psi, split at the kinks."""
    xm, wm = np.polynomial.legendre.leggauss(n)
    mu = xm  # over [-1, 1]
    psi = (np.arange(4 * n) + 0.5) * 2 * np.pi / (4 * n)
    st = np.sqrt(1 - mu * mu)[:, None]
    kx, ky, kz = st * np.cos(psi)[None, :], st * np.sin(psi)[None, :], np.broadcast_to(mu[:, None], st.shape * np.array([1, 4 * n]))
    m = np.maximum(np.maximum(np.abs(kx), np.abs(ky)), np.abs(kz))
    f = np.exp(-a / m)
    return (wm[:, None] * f).sum() / (2 * 4 * n)


def test_continuous_absorption_in_non_scattering_cube(orc, W):
    # albedo 0, unit source at the centre of the uniform cube (kappa rho = 1):
    # energy absorbed inside the central sub-cube [-a, a]^3 (a union of cells)
    # is 1 - <exp(-a / max|k|)>_sphere exactly in expectation.
    N = 40000
    p = W.cube(n_packages=N)
    p["albedo"][:] = 0.0
    img, ab, st = orc.run(p)
    A = ab[0].reshape(32, 32, 32)
    for cells in (4, 8, 12, 16):
        a = cells / 16.0
        inner = A[16 - cells:16 + cells, 16 - cells:16 + cells, 16 - cells:16 + cells].sum()
        expect = 1 - _mean_exp_over_sphere(a)
        # per-package variance of the estimator, from the direction distribution
        rng = np.random.default_rng(0)
        k = rng.standard_normal((200000, 3))
        k /= np.linalg.norm(k, axis=1, keepdims=True)
        sd = np.exp(-a / np.abs(k).max(axis=1)).std() / np.sqrt(N)
        assert abs(inner - expect) < 5 * sd + 1e-9, (cells, inner, expect, sd)
    assert abs(st["escaped"] - _mean_exp_over_sphere(1.0)) < 5 * 0.05 / np.sqrt(N)


def _single_scatter_quadrature(rho, albedo, g, D, n=300):
    """First-order scattered image of a unit point source at the common vertex
    of a 2x2x2 grid over [-1,1]^3, seen face-on with 2x2 pixels aligned with
    the cell columns.  From the origin a ray stays in one octant cell c up to
    t_e = 1/max|k_i|; the interaction density is kr e^{-kr s}; the peel ray
    goes up along +z through c (and, below the midplane, the whole upper cell
    of the column), so in both hemispheres the s-integrand is
    kr e^{-kr s (1 - k_z)} times a constant.  The s-integral is done in closed form, the angles by
    Gauss-Legendre in mu (per hemisphere) and midpoint in psi (per quadrant)."""
    def phase(mu):
        x = 1 + g * g - 2 * g * mu
        return (1 - g * g) / (4 * np.pi * x * np.sqrt(x))

    img = np.zeros((2, 2))
    xm, wm = np.polynomial.legendre.leggauss(n)
    npsi = 4 * n
    for iz, (m0, m1) in enumerate(((-1.0, 0.0), (0.0, 1.0))):
        mu = 0.5 * (m1 - m0) * xm + 0.5 * (m1 + m0)
        wmu = 0.5 * (m1 - m0) * wm
        for ix in range(2):
            for iy in range(2):
                # quadrant of psi with cos sign (ix) and sin sign (iy)
                q0 = {(1, 1): 0.0, (0, 1): 0.5 * np.pi, (0, 0): np.pi, (1, 0): 1.5 * np.pi}[(ix, iy)]
                psi = q0 + (np.arange(npsi) + 0.5) * (0.5 * np.pi) / npsi
                st = np.sqrt(1 - mu * mu)[:, None]
                kx, ky = st * np.cos(psi)[None, :], st * np.sin(psi)[None, :]
                kz = np.broadcast_to(mu[:, None], kx.shape)
                te = 1.0 / np.maximum(np.maximum(np.abs(kx), np.abs(ky)), np.abs(kz))
                kr = rho[iz, iy, ix]
                if iz == 1:
                    inner = np.exp(-kr) * -np.expm1(-kr * te * (1 - kz)) / (1 - kz)
                else:
                    # below the midplane the peel path inside c is s|k_z| = -s k_z
                    inner = np.exp(-rho[1, iy, ix]) * -np.expm1(-kr * te * (1 - kz)) / (1 - kz)
                f = phase(kz) * inner
                img[iy, ix] += albedo / (4 * np.pi * D * D) * (wmu[:, None] * f).sum() * (0.5 * np.pi / npsi)
    return img


def test_single_scattering_image_on_2x2x2_grid(orc, W):
    rho = np.array([0.3, 1.2, 0.7, 2.0, 0.5, 1.6, 0.9, 0.2]).reshape(2, 2, 2)
    alb, g, D = 0.7, 0.4, 10.0
    expect = _single_scatter_quadrature(rho, alb, g, D)
    K, N = 8, 25000
    runs = []
    for s in range(K):
        p = W.small_problem(n=(2, 2, 2), rho=rho, albedo=alb, g=g, detectors=[W.frame(D, 0.0, 2, 2, 1.0, 1.0)],
                            n_packages=N, seed=1000 + s, max_scatter=1, w_min=0.0,
                            flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT | W.FLAG_SPLIT)
        img, ab, st = orc.run(p)
        runs.append(img[1, 0].reshape(2, 2))
    runs = np.array(runs)
    mean, sem = runs.mean(axis=0), runs.std(axis=0, ddof=1) / np.sqrt(K)
    assert np.all(np.abs(mean - expect) < 5 * sem + 1e-12), (mean, expect, sem)
    assert np.all(sem < 0.01 * expect)


def test_dust_free_face_on_disk_image(orc, W):
    # rho = 0: the image is the projected surface brightness of the disk,
    # Sigma(R) = exp(-R/h)/(2 pi h^2), over 4 pi D^2 (pixel integrals by quadrature)
    h, D, npx = 0.3, 10.0, 8
    N = 100_000
    p = W.small_problem(n=(4, 4, 4), rho=np.zeros((4, 4, 4)), sources=[W.expdisk(h, 0.1)],
                        detectors=[W.frame(D, 0.0, npx, npx, 1.0, 1.0)], n_packages=N)
    img, ab, st = orc.run(p)
    frame = W.split_frames(p, img[0, 0])[0]
    counts = frame * 4 * np.pi * D * D * N
    edges = np.linspace(-1, 1, npx + 1)
    xg, wg = np.polynomial.legendre.leggauss(40)
    prob = np.zeros((npx, npx))
    for iy in range(npx):
        for ix in range(npx):
            xs = 0.5 * (edges[ix + 1] - edges[ix]) * xg + 0.5 * (edges[ix + 1] + edges[ix])
            ys = 0.5 * (edges[iy + 1] - edges[iy]) * xg + 0.5 * (edges[iy + 1] + edges[iy])
            R = np.hypot(xs[None, :], ys[:, None])
            f = np.exp(-R / h) / (2 * np.pi * h * h)
            prob[iy, ix] = (wg[:, None] * wg[None, :] * f).sum() * 0.25 * (edges[1] - edges[0]) ** 2
    sd = np.sqrt(N * prob * (1 - prob))
    assert np.all(np.abs(counts - N * prob) < 5 * sd + 1e-6)
    np.testing.assert_allclose(counts, np.round(counts), atol=1e-6)


def test_source_choice_follows_luminosity(orc, W):
    # two point sources of luminosity 1 and 3 in an empty grid, both inside
    # the frame: the direct image splits 1 : 3 up to multinomial noise
    N = 20000
    p = W.small_problem(n=(2, 2, 2), rho=np.zeros((2, 2, 2)),
                        sources=[W.point((-0.5, -0.5, 0.0), 1.0), W.point((0.5, 0.5, 0.0), 3.0)],
                        detectors=[W.frame(10.0, 0.0, 2, 2, 1.0, 1.0)], n_packages=N)
    img, ab, st = orc.run(p)
    fr = W.split_frames(p, img[0, 0])[0] * 4 * np.pi * 100
    assert abs(fr.sum() - 4.0) < 1e-12
    n1 = fr[0, 0] / 4.0 * N
    assert abs(n1 - N / 4) < 5 * np.sqrt(N * 0.25 * 0.75)


def test_sharding_and_threads_do_not_change_results(orc, W):
    N, M = 3000, 1100
    p = W.small_problem(n=(8, 8, 8), rho=W.lognormal_density((8, 8, 8), 1.0, seed=1), n_packages=N)
    img, ab, st = orc.run(p)
    pa = dict(p, n_packages=M)
    pb = dict(p, n_packages=N - M, first_package=M)
    ia, aa, sa = orc.run(pa)
    ib, ab_, sb = orc.run(pb)
    np.testing.assert_allclose(img, (M * ia + (N - M) * ib) / N, rtol=1e-11, atol=1e-18)
    np.testing.assert_allclose(ab, (M * aa + (N - M) * ab_) / N, rtol=1e-11, atol=1e-18)
    for key in ("x_path", "x_locate", "x_peel", "events"):
        assert st[key] == sa[key] + sb[key]
    it, at, stt = orc.run(p, threads=3)
    np.testing.assert_allclose(it, img, rtol=1e-12, atol=1e-20)
    np.testing.assert_allclose(at, ab, rtol=1e-12, atol=1e-20)
    assert stt["x_path"] == st["x_path"]


def _slab_single_scatter(rho_layers, dz, c, kappa, albedo, g, D):
    """First-order scattered flux of a unit point source on the wall between
    layers c-1 and c of a horizontally unbounded stack of layers, seen from
    +z.  Optical depths depend on the height only, so with mu the direction
    cosine, ds = dz/|mu|, and each layer's z-integral is in closed form; the
    mu-integral is done by adaptive quadrature per hemisphere."""
    kr = kappa * np.asarray(rho_layers) * dz
    nz = len(kr)

    def phase(mu):
        x = 1 + g * g - 2 * g * mu
        return (1 - g * g) / (4 * np.pi * x * np.sqrt(x))

    def up(mu):  # layers c..nz-1
        tot = 0.0
        for k in range(c, nz):
            A = kr[c:k].sum()
            B = kr[k:].sum()
            a = kr[k] * (1 / mu - 1)
            f = dz if a == 0 else -np.expm1(-a) / (a / dz)
            tot += (kr[k] / dz / mu) * np.exp(-A / mu - B) * f
        return phase(mu) * tot

    def down(nu):  # layers c-1..0, nu = |mu|
        tot = 0.0
        for k in range(c - 1, -1, -1):
            A = kr[k + 1:c].sum()
            Cabove = kr[k + 1:].sum()
            a = kr[k] * (1 / nu + 1)
            tot += (kr[k] / dz / nu) * np.exp(-A / nu - Cabove) * (-np.expm1(-a) / (a / dz))
        return phase(-nu) * tot

    su, _ = integrate.quad(up, 0, 1, limit=400, epsabs=0, epsrel=1e-10)
    sd, _ = integrate.quad(down, 0, 1, limit=400, epsabs=0, epsrel=1e-10)
    return albedo / (2 * D * D) * (su + sd)


def test_single_scattering_in_layered_slab(orc, W):
    # the interaction point is located several cells along the path: paths
    # cross up to 8 layers of different density before they scatter
    rho = np.array([0.4, 1.5, 0.2, 2.2, 0.9, 0.3, 1.8, 0.6])
    nz, H, D = 8, 1e5, 10.0
    alb, g, kappa = 0.8, 0.55, 1.3
    expect = _slab_single_scatter(rho, 2.0 / nz, nz // 2, kappa, alb, g, D)
    K, N = 8, 25000
    vals = []
    for s in range(K):
        p = W.small_problem(n=(1, 1, nz), box=(-H, H, -H, H, -1.0, 1.0), rho=rho.reshape(nz, 1, 1), kappa=kappa,
                            albedo=alb, g=g, detectors=[W.frame(D, 0.0, 1, 1, 10 * H, 10 * H)], n_packages=N,
                            seed=2000 + s, max_scatter=1, w_min=0.0,
                            flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT | W.FLAG_SPLIT)
        img, ab, st = orc.run(p)
        vals.append(img[1, 0].sum())
    vals = np.array(vals)
    mean, sem = vals.mean(), vals.std(ddof=1) / np.sqrt(K)
    assert abs(mean - expect) < 5 * sem + 1e-4 * expect, (mean, expect, sem)
    assert sem < 0.01 * expect
