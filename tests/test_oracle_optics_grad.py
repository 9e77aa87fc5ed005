"""Pins of the oracle's gradients with respect to the albedo, the asymmetry
parameter g and the source luminosities (the detached derivative with paths
held fixed, the same reading as the density gradient):

- with one scattering at most, the scattered light is linear in the albedo:
  dL/dalbedo = sum(adj * scattered image) / albedo exactly;
- images are homogeneous of degree one in the luminosities:
  sum_s L_s dL/dL_s = sum(adj * image) for every sample (one source: the
  gradient is sum(adj * image) / L);
- central finite differences of the reweighted estimator (paths sampled at
  the nominal parameters, weights evaluated at the perturbed ones) in each
  parameter match the gradients -- the reweighting is written separately in
  the oracle (weight ratios), the gradients from per-contribution factors."""
import numpy as np
import pytest

BOX = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)


def _problem(W, n_packages=1500, flags=None, max_scatter=1000, two_sources=True, n_lambda=2):
    rho = W.lognormal_density((6, 5, 4), 0.7, seed=12)
    srcs = [W.point((0.1, -0.2, 0.05), lum=np.linspace(1.0, 0.6, n_lambda))]
    if two_sources:
        srcs.append(W.expdisk(0.4, 0.15, lum=np.linspace(0.5, 1.5, n_lambda)))
    return W.small_problem(n=(6, 5, 4), box=BOX, rho=rho, kappa=np.linspace(1.4, 0.9, n_lambda),
                           albedo=np.linspace(0.65, 0.45, n_lambda), g=np.linspace(0.55, -0.2, n_lambda),
                           sources=srcs,
                           detectors=[W.frame(10.0, 30.0, 9, 8, 1.3, 1.2, azim=20.0), W.sed(10.0, 80.0),
                                      W.perspective((0.3, 0.2, 0.4), (-0.5, 0.1, -0.3), (0, 0, 1), 7, 7, 1.5, 1.5)],
                           n_packages=n_packages, max_scatter=max_scatter,
                           flags=flags if flags is not None else W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT | W.FLAG_SPLIT)


def _adj(shape, seed=3):
    return np.random.default_rng(seed).standard_normal(shape)


def test_single_scattering_albedo_gradient_is_linear(orc, W):
    p = _problem(W, max_scatter=1)
    img, _, _ = orc.run(p)
    adj = _adj(img.shape)
    _, _, _, go = orc.grad(p, adj, optics=True)
    want = (adj[1] * img[1]).sum(axis=1) / p["albedo"]
    np.testing.assert_allclose(go["albedo"], want, rtol=1e-12)


def test_luminosity_gradients_are_homogeneous(orc, W):
    p = _problem(W)
    img, _, _ = orc.run(p)
    adj = _adj(img.shape)
    _, _, _, go = orc.grad(p, adj, optics=True)
    L = np.stack([s["lum"] for s in p["sources"]])
    np.testing.assert_allclose((L * go["lum"]).sum(axis=0), (adj * img).sum(axis=(0, 2)), rtol=1e-12)
    p1 = _problem(W, two_sources=False)  # same frames and wavelengths, one source
    img1, _, _ = orc.run(p1)
    _, _, _, g1 = orc.grad(p1, adj, optics=True)
    np.testing.assert_allclose(g1["lum"][0], (adj * img1).sum(axis=(0, 2)) / p1["sources"][0]["lum"], rtol=1e-12)


@pytest.mark.parametrize("param", ["albedo", "g", "lum"])
def test_gradient_matches_reweighted_finite_differences(orc, W, param):
    p = _problem(W)
    img, _, _ = orc.run(p)
    adj = _adj(img.shape)
    _, _, _, go = orc.grad(p, adj, optics=True)
    rho = np.asarray(p["rho"])
    nl = len(p["kappa"])
    for l in range(nl):
        if param == "lum":
            base = np.stack([s["lum"] for s in p["sources"]])
            for s in range(len(p["sources"])):
                h = 1e-4 * base[s, l]
                hi, lo = base.copy(), base.copy()
                hi[s, l] += h
                lo[s, l] -= h
                ih, _ = orc.reweight(p, rho, lum_eval=hi)
                il, _ = orc.reweight(p, rho, lum_eval=lo)
                fd = (adj * (ih - il)).sum() / (2 * h)
                assert abs(fd - go["lum"][s, l]) <= 1e-6 * abs(go["lum"][s, l]) + 1e-12, (s, l)
            continue
        base = np.asarray(p[param], dtype=np.float64)
        h = 1e-5
        hi, lo = base.copy(), base.copy()
        hi[l] += h
        lo[l] -= h
        kw = "albedo_eval" if param == "albedo" else "g_eval"
        ih, _ = orc.reweight(p, rho, **{kw: hi})
        il, _ = orc.reweight(p, rho, **{kw: lo})
        fd = (adj * (ih - il)).sum() / (2 * h)
        assert abs(fd - go[param][l]) <= 1e-6 * abs(go[param][l]) + 1e-10, (param, l, fd, go[param][l])
        assert go[param][l] != 0.0
