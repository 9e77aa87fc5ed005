"""Pins of the oracle's gradient of a loss on the absorbed-luminosity tally
(sum of b * A over wavelengths and cells, with or without an image term):

- central finite differences of the reweighted estimator's absorbed tally
  (paths sampled at rho, deposits and weights evaluated at rho +- h e_m) on
  every cell of a small grid;
- with no scattering (albedo 0) every deposit is W0 e^-tau_{j-1} (1 -
  e^-dtau_j) along one fixed path, and the gradient is the closed form
  written out per cell along each emission direction's ray (numpy, from the
  oracle's own segment lists of trace);
- the image and absorbed terms add: the gradient of the combined loss is the
  sum of the two separate gradients."""
import numpy as np
import pytest

BOX = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)


def _problem(W, albedo=0.6, n_packages=600, n=(5, 4, 3), n_lambda=2):
    rho = W.lognormal_density(n, 0.6, seed=17)
    return W.small_problem(n=n, box=BOX, rho=rho, kappa=np.linspace(1.2, 0.7, n_lambda),
                           albedo=np.full(n_lambda, albedo), g=np.linspace(0.4, -0.1, n_lambda),
                           sources=[W.point((0.12, -0.08, 0.03), lum=np.linspace(1.0, 0.5, n_lambda))],
                           detectors=[W.frame(10.0, 30.0, 7, 6, 1.3, 1.2)], n_packages=n_packages,
                           flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT | W.FLAG_ABSORB)


def test_absorbed_gradient_matches_reweighted_finite_differences(orc, W):
    p = _problem(W)
    img, A, _ = orc.run(p)
    b = np.random.default_rng(4).standard_normal(A.shape)
    g, _, _ = orc.grad(p, np.zeros_like(img), adj_absorbed=b)
    rho = np.asarray(p["rho"], dtype=np.float64).reshape(-1)
    for m in range(rho.size):
        h = 1e-5 * rho[m]
        hi, lo = rho.copy(), rho.copy()
        hi[m] += h
        lo[m] -= h
        _, ah, _ = orc.reweight(p, hi, absorbed=True)
        _, al, _ = orc.reweight(p, lo, absorbed=True)
        fd = (b * (ah - al)).sum() / (2 * h)
        assert abs(fd - g[m]) <= 1e-6 * np.abs(g).max(), (m, fd, g[m])


def test_non_scattering_absorbed_gradient_closed_form(orc, W):
    # albedo 0: each package deposits along one ray from the source; the
    # derivative of W0 e^-tau_{j-1} (1 - e^-dtau_j) in rho_k is written out
    p = _problem(W, albedo=0.0, n_packages=200, n_lambda=1)
    _, A, _ = orc.run(p)
    b = np.random.default_rng(6).standard_normal(A.shape)
    g, _, _ = orc.grad(p, np.zeros((1, 1, 42)), adj_absorbed=b)
    rho = np.asarray(p["rho"], dtype=np.float64).reshape(-1)
    kap = p["kappa"][0]
    src = np.array(p["sources"][0]["pos"])
    words = orc.draw_words(p["seed"], 0, p["n_packages"], 0, 1)
    w0 = p["sources"][0]["lum"][0] / p["n_packages"]
    want = np.zeros(rho.size)
    for q in range(p["n_packages"]):
        k = orc.emit_direction([orc.uniform(w) for w in words[q]])
        _, _, cell, length, nseg = orc.trace(BOX, p["n"], rho, kap, src[None], np.asarray(k)[None], max_seg=32)
        c, L = cell[0, :nseg[0]], length[0, :nseg[0]]
        dt = kap * rho[c] * L
        tau_before = np.concatenate([[0.0], np.cumsum(dt)[:-1]])
        dep = w0 * np.exp(-tau_before) * (-np.expm1(-dt))
        for j in range(len(c)):
            # d dep_j / d rho_k: -kappa L_k dep_j for k before j, own cell w0 e^-tau e^-dt kappa L_j
            for i in range(j):
                want[c[i]] += b[0, c[j]] * (-kap * L[i] * dep[j])
            want[c[j]] += b[0, c[j]] * w0 * np.exp(-tau_before[j]) * np.exp(-dt[j]) * kap * L[j]
    np.testing.assert_allclose(g, want, rtol=1e-10, atol=1e-12 * np.abs(want).max())


def test_image_and_absorbed_terms_add(orc, W):
    p = _problem(W)
    img, A, _ = orc.run(p)
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal(img.shape), rng.standard_normal(A.shape)
    g_i, _, _ = orc.grad(p, a)
    g_a, _, _ = orc.grad(p, np.zeros_like(img), adj_absorbed=b)
    g_t, _, _ = orc.grad(p, a, adj_absorbed=b)
    np.testing.assert_allclose(g_t, g_i + g_a, rtol=1e-11, atol=1e-13 * np.abs(g_t).max())
