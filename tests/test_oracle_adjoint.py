"""Pins of the oracle's detached density gradient (score-function /
path-replay form) and of the reweighted estimator it differentiates."""
import numpy as np
import pytest


def test_non_scattering_closed_form(orc, W):
    # albedo 0, unit point source at the origin, face-on frame: every package
    # gives I = e^-tau_axis / (4 pi D^2) in pixel (nx/2, ny/2), and
    # dL/drho_m = A (-kappa l_m I) for the cells of the +z column through
    # the origin (cells (4,4,k >= 4) by the wall convention), 0 elsewhere.
    n = (8, 8, 8)
    rho = W.lognormal_density(n, 1.0, seed=21)
    kappa, D = 1.7, 10.0
    p = W.small_problem(n=n, rho=rho, kappa=kappa, albedo=0.0, g=0.5, detectors=[W.frame(D, 0.0, 16, 16, 1.0, 1.0)],
                        n_packages=500, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    adj = np.random.default_rng(3).standard_normal(256)
    g, img, st = orc.grad(p, adj)
    dz = 0.25
    col = rho[4:, 4, 4]
    tau = kappa * col.sum() * dz
    I = np.exp(-tau) / (4 * np.pi * D * D)
    frame = img[0, 0].reshape(16, 16)
    assert abs(frame[8, 8] - I) < 1e-13 * I
    frame[8, 8] = 0
    assert np.all(frame == 0)
    expect = np.zeros(n[::-1])
    expect[4:, 4, 4] = adj[8 * 16 + 8] * (-kappa * dz * I)
    np.testing.assert_allclose(g.reshape(n[::-1]), expect, rtol=1e-12, atol=1e-20)


def _small_scattering_problem(W, N=1500, seed=4357, flags=None):
    n = (6, 6, 6)
    rho = W.lognormal_density(n, 0.8, seed=31)
    return W.small_problem(n=n, rho=rho, kappa=1.2, albedo=0.7, g=0.45, sources=[W.point((0.13, -0.21, 0.07))],
                           detectors=[W.frame(10.0, 30.0, 12, 12, 1.0, 1.0, azim=20.0),
                                      W.frame(10.0, 90.0, 8, 8, 1.2, 1.2)],
                           n_packages=N, seed=seed, flags=flags or (W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT),
                           w_min=1e-3, max_scatter=50)


def test_reweight_at_sampling_density_equals_forward(orc, W):
    p = _small_scattering_problem(W)
    img, ab, st = orc.run(p)
    rimg, rst = orc.reweight(p, p["rho"])
    np.testing.assert_allclose(rimg, img, rtol=1e-13, atol=1e-22)
    g, gimg, gst = orc.grad(p, np.zeros_like(img))
    np.testing.assert_allclose(gimg, img, rtol=0, atol=0)
    assert np.all(g == 0)


@pytest.mark.parametrize("split", [False, True])
def test_gradient_matches_replay_finite_differences(orc, W, split):
    # L = sum (I - T)^2 with T a perturbed image; dL/drho from the gradient
    # routine against the central difference of L over the reweighted
    # estimator (paths frozen at rho0), h = 1e-4 rho_m, on 24 cells
    flags = (W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT | (W.FLAG_SPLIT if split else 0))
    p = _small_scattering_problem(W, flags=flags)
    img, _, _ = orc.run(p)
    target = img * (1 + 0.3 * np.random.default_rng(5).standard_normal(img.shape))
    adj = 2 * (img - target)
    g, _, _ = orc.grad(p, adj)
    rho0 = p["rho"].reshape(-1)
    rng = np.random.default_rng(7)
    cells = np.concatenate([np.argsort(-np.abs(g))[:12], rng.choice(rho0.size, 12, replace=False)])

    def loss(r):
        im, _ = orc.reweight(p, r)
        return ((im - target) ** 2).sum()

    gmax = np.abs(g).max()
    assert gmax > 0
    for m in cells:
        h = 1e-4 * rho0[m]
        rp, rm = rho0.copy(), rho0.copy()
        rp[m] += h
        rm[m] -= h
        fd = (loss(rp) - loss(rm)) / (2 * h)
        assert abs(fd - g[m]) <= 1e-6 * abs(g[m]) + 1e-8 * gmax, (m, fd, g[m])


def test_gradient_is_linear_in_adjoint_and_additive_over_shards(orc, W):
    p = _small_scattering_problem(W, N=900)
    img, _, _ = orc.run(p)
    rng = np.random.default_rng(9)
    a1, a2 = rng.standard_normal(img.shape), rng.standard_normal(img.shape)
    g1, _, _ = orc.grad(p, a1)
    g2, _, _ = orc.grad(p, a2)
    g12, _, _ = orc.grad(p, 2 * a1 - 3 * a2)
    np.testing.assert_allclose(g12, 2 * g1 - 3 * g2, rtol=1e-10, atol=1e-12 * np.abs(g12).max())
    ga, _, _ = orc.grad(dict(p, n_packages=400), a1)
    gb, _, _ = orc.grad(dict(p, n_packages=500, first_package=400), a1)
    np.testing.assert_allclose(g1, (400 * ga + 500 * gb) / 900, rtol=1e-10, atol=1e-12 * np.abs(g1).max())


def test_reweighted_estimator_is_unbiased(orc, W):
    # paths sampled at rho0 and weighted for rho1 estimate the same expected
    # images as paths sampled at rho1 (strongly changed density): compare the
    # per-frame fluxes and the brightest pixels over independent seeds
    K = 10
    rho0 = _small_scattering_problem(W)["rho"]
    rho1 = rho0 * np.exp(0.6 * np.random.default_rng(8).standard_normal(rho0.shape))
    rw, fw = [], []
    for s in range(K):
        p0 = _small_scattering_problem(W, N=4000, seed=300 + s)
        p1 = dict(p0, rho=rho1, seed=600 + s)
        im_rw, _ = orc.reweight(p0, rho1)
        im_fw, _, _ = orc.run(p1)
        rw.append(im_rw[0, 0])
        fw.append(im_fw[0, 0])
    rw, fw = np.array(rw), np.array(fw)
    n0 = 144
    bright = np.argsort(-fw.mean(0))[:3]
    feats = lambda a: np.concatenate([a[:, :n0].sum(1, keepdims=True), a[:, n0:].sum(1, keepdims=True),
                                      a[:, bright]], axis=1)
    a, b = feats(rw), feats(fw)
    ma, mb = a.mean(0), b.mean(0)
    se = np.sqrt(a.var(0, ddof=1) / K + b.var(0, ddof=1) / K)
    assert np.all(np.abs(ma - mb) < 5 * se), (ma, mb, se)
    assert np.all(se[:2] < 0.02 * np.abs(mb[:2]))
