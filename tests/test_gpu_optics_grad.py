"""The HIP path's gradients with respect to the albedo, g and the source
luminosities (with the densities, in one replay) through the C ABI, against
the FP64 oracle on mixed instruments and sources, tree grids and cell
sources, in both precisions and queue modes; then the adjoint workload at
full size: the optics gradients' cost beside the density-only replay, and
the single-source luminosity gradient against the image it scales."""
import time

import numpy as np
import pytest
from parity import check, rel_l1

from test_emu_optics_grad import problems

pytestmark = pytest.mark.gpu




@pytest.fixture(scope="module")
def B():
    import torch
    from paper_1410_1629_amd import binding
    binding.load()
    assert torch.cuda.is_available()
    return binding


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


def _say(msg):
    print("[gpu] " + msg, flush=True)


def _outputs(B, p, n_cells):
    import torch
    nl, ns = len(np.atleast_1d(p["kappa"])), len(p["sources"])
    z = lambda *s: torch.empty(s, dtype=torch.float64, device="cuda")  # noqa: E731
    return z(n_cells), z(nl), z(nl), z(ns, nl)


@pytest.mark.parametrize("name", ["mixed", "tree", "cells"])
@pytest.mark.parametrize("prec", [0, 1])
def test_optics_gradients_match_oracle(B, orc, W, name, prec):
    _say("optics gradients %s prec=%d" % (name, prec))
    p = problems(W, name, prec)
    p["n_packages"] = 3000
    img_o, _, _ = orc.run(p, threads=8)
    adj = np.random.default_rng(8).standard_normal(img_o.shape)
    g_o, _, _, go = orc.grad(p, adj, threads=8, optics=True)
    rho = B.density_tensor(p)
    tol = 1e-9 if prec == 0 else 1e-5
    for q in (-1, 0):
        gr, ga, gg, gl = _outputs(B, p, rho.numel())
        B.backward(p, rho, _dev(adj), gr, ga, gg, gl, peel_queue=q)
        check(gr.cpu().numpy(), g_o, tol, "queue %d: rho" % q, _say)
        for t, k in ((ga, "albedo"), (gg, "g"), (gl, "lum")):
            check(t.cpu().numpy(), go[k], tol, "queue %d: %s" % (q, k), _say)


def test_adjoint_workload_with_optics_gradients(B, W):
    import torch
    _say("adjoint workload, 1e7 packages: density-only replay vs all gradients")
    p = W.adjoint()
    rho = B.density_tensor(p)
    images = torch.empty(B.image_shape(p), dtype=torch.float64, device="cuda")
    B.run_photons(p, rho, images)
    adj = torch.randn(images.shape, generator=torch.Generator(device="cuda").manual_seed(3), dtype=torch.float64,
                      device="cuda")
    gr, ga, gg, gl = _outputs(B, p, rho.numel())
    gr2 = torch.empty_like(gr)
    B.backward_density(p, rho, adj, gr2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s1 = B.backward_density(p, rho, adj, gr2)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s2 = B.backward(p, rho, adj, gr, ga, gg, gl)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    assert torch.equal(gr, gr2) or rel_l1(gr.cpu().numpy(), gr2.cpu().numpy()) < 1e-12
    # one source: its luminosity gradient is sum(adj * image) / L exactly
    want = (adj * images).sum().item() / p["sources"][0]["lum"][0]
    assert abs(gl[0, 0].item() / want - 1.0) < 1e-9, (gl[0, 0].item(), want)
    _say("  density only %.1f ms (kernel %.1f); with albedo, g, luminosity %.1f ms (kernel %.1f); dL/dalbedo %.4e "
         "dL/dg %.4e dL/dL %.4e" % ((t1 - t0) * 1e3, s1["kernel_ms"], (t2 - t1) * 1e3, s2["kernel_ms"],
                                    ga[0].item(), gg[0].item(), gl[0, 0].item()))
    assert np.isfinite([ga[0].item(), gg[0].item()]).all()


def test_autograd_optics_matches_oracle(B, orc, W):
    import torch
    from paper_1410_1629_amd import autograd
    _say("autograd RTImageOptics")
    p = problems(W, "mixed", 0)
    p["n_packages"] = 2000
    img_o, _, _ = orc.run(p, threads=8)
    target = torch.as_tensor(img_o * 0.7).cuda()
    rho = B.density_tensor(p).requires_grad_(True)
    albedo = torch.as_tensor(p["albedo"], dtype=torch.float64).requires_grad_(True)
    g = torch.as_tensor(p["g"], dtype=torch.float64).requires_grad_(True)
    lum = torch.as_tensor(np.stack([s["lum"] for s in p["sources"]]), dtype=torch.float64).requires_grad_(True)
    images = autograd.render_optics(p, rho, albedo, g, lum)
    loss = ((images - target) ** 2).sum()
    loss.backward()
    adj = 2 * (img_o - img_o * 0.7)
    g_o, _, _, go = orc.grad(p, adj, threads=8, optics=True)
    check(images.detach().cpu().numpy(), img_o, 1e-10, "images", _say)
    check(rho.grad.cpu().numpy(), g_o, 1e-9, "rho", _say)
    check(albedo.grad.numpy(), go["albedo"], 1e-9, "albedo", _say)
    check(g.grad.numpy(), go["g"], 1e-9, "g", _say)
    check(lum.grad.numpy(), go["lum"], 1e-9, "lum", _say)
    # only some inputs requiring gradients
    albedo2 = albedo.detach().requires_grad_(True)
    img2 = autograd.render_optics(p, rho.detach(), albedo2, g.detach(), lum.detach())
    ((img2 - target) ** 2).sum().backward()
    check(albedo2.grad.numpy(), go["albedo"], 1e-9, "albedo", _say)
