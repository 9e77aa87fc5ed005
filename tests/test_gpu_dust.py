"""The HIP path's dust emission and cell sources (Sect. 1 and 2.1:
absorption, re-emission by the dust, panchromatic runs) through the C ABI,
against the FP64 oracle: equilibrium temperatures and spectra on regular
(ragged), rectilinear and tree grids; forward and adjoint runs whose source
is the cells; the cell CDF at 4.2 million cells; and the full panchromatic
disk (stellar run with the absorbed tally, dust emission, dust run)."""
import math
import time

import numpy as np
import pytest
from parity import check, rel_l1

from test_emu_dust import _cells_problem, absorbed_field, grids, spectrum

pytestmark = pytest.mark.gpu




@pytest.fixture(scope="module")
def B():
    import torch
    from paper_1410_1629_amd import binding
    binding.load()
    assert torch.cuda.is_available()
    return binding


def _dev(x, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype or torch.float64).cuda()


def _say(msg):
    print("[gpu] " + msg, flush=True)


def _gpu_dust(B, g, rho, prec, ab, lam, dlam, ka, eps):
    import torch
    ncell = rho.size
    T = torch.empty(ncell, dtype=torch.float64, device="cuda")
    em = torch.empty((len(lam), ncell), dtype=torch.float64, device="cuda")
    B.dust_emission(g, _dev(rho.reshape(-1), torch.float32 if prec else torch.float64), prec, _dev(ab), lam, dlam,
                    ka, eps, em, T)
    return T.cpu().numpy(), em.cpu().numpy()


@pytest.mark.parametrize("grid", ["ragged", "rect", "tree"])
@pytest.mark.parametrize("prec", [0, 1])
def test_dust_emission_matches_oracle(B, orc, W, grid, prec):
    _say("dust emission %s prec=%d" % (grid, prec))
    g = {"box": (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0), "n": (37, 29, 11)} if grid == "ragged" else grids(W)[grid]
    ncell = int(np.prod(g["n"]))
    rng = np.random.default_rng(6)
    rho = rng.lognormal(0.0, 1.0, ncell)
    rho[rng.choice(ncell, 7, replace=False)] = 0.0
    if prec:
        rho = W.as_f32_values(rho)
    ab = absorbed_field(ncell, 9, n_abs=3)
    lam, dlam, ka = spectrum(100)
    eps = 3e12
    T_o, em_o = orc.dust_emission(g["box"], g["n"], rho, ab, lam, dlam, ka, eps, planes=g.get("planes"),
                                  tree=g.get("tree"))
    T, em = _gpu_dust(B, g, rho, prec, ab, lam, dlam, ka, eps)
    hot = T_o > 0
    assert np.array_equal(T > 0, hot)
    np.testing.assert_allclose(T[hot], T_o[hot], rtol=1e-12)
    assert rel_l1(em, em_o) < 1e-12
    np.testing.assert_allclose(em.sum(axis=0)[hot], ab.sum(axis=0)[hot], rtol=1e-13)


def test_dust_emission_full_size(B, orc, W):
    # the multiwavelength disk's 128^3 cells and 100 wavelengths; every cell
    # re-emits what it absorbed, and 64 sampled cells match the oracle run
    # on the same cell alone
    import torch
    _say("dust emission at 128^3 cells x 100 wavelengths")
    prob, dust = W.panchromatic(n_packages=1)
    box, n = prob["box"], prob["n"]
    rho = np.asarray(prob["rho"]).reshape(-1)
    ncell = rho.size
    ab = torch.exp(torch.randn((2, ncell), generator=torch.Generator(device="cuda").manual_seed(2),
                               dtype=torch.float64, device="cuda") * 2.0 - 12.0)
    drho = _dev(rho, torch.float32)
    em = torch.empty((100, ncell), dtype=torch.float64, device="cuda")
    T = torch.empty(ncell, dtype=torch.float64, device="cuda")
    args = (prob, drho, 1, ab, dust["lambda"], dust["dlambda"], dust["kappa_abs"], dust["emissivity"], em, T)
    B.dust_emission(*args)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.dust_emission(*args)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    L = ab.sum(dim=0)
    live = drho.double() > 0
    err = ((em.sum(dim=0) - L).abs() / L)[live].max().item()
    assert err < 1e-12, err
    Tn = T.cpu().numpy()
    _say("  %.2f ms; T in [%.2f, %.2f] K, median %.2f K" % (ms, Tn[Tn > 0].min(), Tn.max(), np.median(Tn[Tn > 0])))
    idx = np.random.default_rng(1).choice(np.nonzero(rho > 0)[0], 64, replace=False)
    abh, emh = ab.cpu().numpy(), em.cpu().numpy()
    d = [(box[2 * a + 1] - box[2 * a]) / n[a] for a in range(3)]
    for m in idx:
        i = (m % n[0], (m // n[0]) % n[1], m // (n[0] * n[1]))
        cb = []
        for a in range(3):
            cb += [box[2 * a] + i[a] * d[a], box[2 * a] + (i[a] + 1) * d[a]]
        To, eo = orc.dust_emission(tuple(cb), (1, 1, 1), rho[m:m + 1], abh[:, m:m + 1], dust["lambda"],
                                   dust["dlambda"], dust["kappa_abs"], dust["emissivity"])
        assert abs(Tn[m] / To[0] - 1.0) < 1e-12, (m, Tn[m], To[0])
        assert rel_l1(emh[:, m], eo[:, 0]) < 1e-12


@pytest.mark.parametrize("grid", ["regular", "rect", "tree"])
@pytest.mark.parametrize("prec", [0, 1])
def test_cell_source_run_matches_oracle(B, orc, W, grid, prec):
    _say("cell source run %s prec=%d" % (grid, prec))
    p = _cells_problem(W, grid, prec, n_packages=3000)
    img_o, abs_o, st_o = orc.run(p, threads=8)
    tol = 1e-10 if prec == 0 else 1e-5
    for q in (-1, 0):
        images, absorbed, st = B.render(p, peel_queue=q)
        check(images.cpu().numpy(), img_o, tol, "queue %d: images" % q, _say)
        check(absorbed.cpu().numpy(), abs_o, tol, "queue %d: absorbed" % q, _say)
        assert st["packages"] == st_o["packages"]
        assert abs(st["emitted"] - st_o["emitted"]) <= 1e-12 * st_o["emitted"]
        for key in ("events", "x_path", "x_locate", "x_peel"):
            assert abs(st[key] - st_o[key]) <= 1e-4 * st_o[key] + 2, (key, st[key], st_o[key])


@pytest.mark.parametrize("prec", [0, 1])
def test_cell_source_adjoint_matches_oracle(B, orc, W, prec):
    import torch
    _say("cell source adjoint prec=%d" % prec)
    p = _cells_problem(W, "regular", prec, n_packages=2000, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    img_o, _, _ = orc.run(p, threads=8)
    adj = np.random.default_rng(8).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(p, adj, threads=8)
    rho = B.density_tensor(p)
    grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
    B.backward_density(p, rho, _dev(adj), grad)
    check(grad.cpu().numpy(), g_o, 1e-9 if prec == 0 else 1e-5, "grad", _say)


def test_cell_cdf_at_scale(B, orc, W):
    # 256 x 256 x 64 cells (2048 CDF tiles per wavelength, a ragged last
    # tile of the 4194304 + 1 entries), no dust: a package subset deep in
    # the run matches the oracle exactly, and 4e6 packages fill the face-on
    # frame's pixels (the columns of cells) in proportion to the columns'
    # luminosity
    import torch
    from scipy import stats
    _say("cell CDF at 4.2M cells")
    n, box = (256, 256, 64), (-20.0, 20.0, -20.0, 20.0, -2.0, 2.0)
    ncell = int(np.prod(n))
    rng = np.random.default_rng(12)
    lum = rng.lognormal(0.0, 1.0, (2, ncell))
    lum[:, rng.random(ncell) < 0.3] = 0.0
    d = 1000.0
    det = W.frame(d, 0.0, 256, 256, 20.0, 20.0)
    p = W.small_problem(n=n, box=box, rho=np.zeros((n[2], n[1], n[0])), kappa=[1.0, 0.5], albedo=[0.5, 0.5],
                        g=[0.3, 0.3], sources=[W.cells(lum)], detectors=[det], n_packages=1500, flags=1,
                        first_package=3_141_592)
    img_o, _, st_o = orc.run(p, threads=8)
    images, _, st = B.render(p)
    check(images.cpu().numpy(), img_o, 1e-12, "images", _say)
    p2 = dict(p, n_packages=4_000_000, first_package=0)
    images, _, st = B.render(p2)
    assert st["packages"] == 8_000_000
    for l in range(2):
        counts = images[0, l].cpu().numpy() * 4.0 * math.pi * d * d / (lum[l].sum() / 4e6)
        assert np.allclose(counts, np.round(counts), atol=1e-4)
        col = lum[l].reshape(n[2], n[1] * n[0]).sum(axis=0)
        # the frame's pixel of column (i, j): through the frame's own basis
        _, ex, ey = orc.detector_basis(det)
        xs = (np.arange(256) + 0.5) * (40.0 / 256) - 20.0
        X, Y = np.meshgrid(xs, xs)
        px = np.floor((X * ex[0] + Y * ex[1] + 20.0) / 40.0 * 256).astype(int)
        py = np.floor((X * ey[0] + Y * ey[1] + 20.0) / 40.0 * 256).astype(int)
        got = np.round(counts).astype(np.int64)[(px + 256 * py).reshape(-1)]
        assert got.sum() == 4_000_000
        assert np.all(got[col == 0.0] == 0)
        live = col > 0
        expect = 4e6 * col[live] / col.sum()
        chi2 = ((got[live] - expect) ** 2 / expect).sum()
        p_value = stats.chi2.sf(chi2, live.sum() - 1)
        _say("  wavelength %d: chi2 %.1f for %d columns, p = %.3g" % (l, chi2, live.sum(), p_value))
        assert p_value > 1e-4


def test_panchromatic_full_size(B, W):
    # stellar run (1e6 packages at each of 100 wavelengths) with the absorbed
    # tally, dust emission, then the dust run from the cells on the same
    # wavelengths: energy closes in each run and the dust re-emits exactly
    # what the stellar run deposited
    import torch
    _say("panchromatic disk: stellar run, dust emission, dust run")
    prob, dust = W.panchromatic(n_packages=1_000_000)
    rho = B.density_tensor(prob)
    ncell = rho.numel()
    images = torch.empty(B.image_shape(prob), dtype=torch.float64, device="cuda")
    absorbed = torch.empty((100, ncell), dtype=torch.float64, device="cuda")
    em = torch.empty((100, ncell), dtype=torch.float64, device="cuda")
    T = torch.empty(ncell, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s1 = B.run_photons(prob, rho, images, absorbed)
    t1 = time.perf_counter()
    B.dust_emission(prob, rho, 1, absorbed, dust["lambda"], dust["dlambda"], dust["kappa_abs"], dust["emissivity"],
                    em, T)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    dprob = W.dust_problem(prob, em)
    dimages = torch.empty(B.image_shape(dprob), dtype=torch.float64, device="cuda")
    dabs = torch.empty((100, ncell), dtype=torch.float64, device="cuda")
    s2 = B.run_photons(dprob, rho, dimages, dabs)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for s in (s1, s2):
        closure = (s["absorbed"] + s["escaped"] + s["truncated"] - s["emitted"]) / s["emitted"]
        assert abs(closure) < 1e-6 and s["packages"] == 100_000_000
    L = absorbed.sum().item()
    assert abs(em.sum().item() / L - 1.0) < 1e-12
    assert abs(s2["emitted"] / L - 1.0) < 1e-12
    Tn = T.cpu().numpy()
    _say("  stellar %.1f ms (kernel %.1f), dust emission %.1f ms, dust run %.1f ms (kernel %.1f); absorbed %.4f of "
         "%.1f; dust T median %.1f K, max %.1f K; dust run re-absorbs %.3g"
         % ((t1 - t0) * 1e3, s1["kernel_ms"], (t2 - t1) * 1e3, (t3 - t2) * 1e3, s2["kernel_ms"], L, s1["emitted"],
            np.median(Tn[Tn > 0]), Tn.max(), s2["absorbed"] / s2["emitted"]))
