"""The HIP path's gradient of a loss on the absorbed-luminosity tally (with
and without an image term) through the C ABI, against the FP64 oracle on
every grid kind, both precisions and queue modes; then the multiwavelength
disk at its full grid (128^3 cells, 100 wavelengths): a package subset
against the oracle and the full run's cost beside the image-only replay."""
import time

import numpy as np
import pytest
from parity import check, rel_l1

from test_emu_absorbed_grad import _setup

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


@pytest.mark.parametrize("grid", ["regular", "rect", "tree"])
@pytest.mark.parametrize("prec", [0, 1])
def test_absorbed_gradient_matches_oracle(B, orc, W, grid, prec):
    import torch
    _say("absorbed-tally gradient %s prec=%d" % (grid, prec))
    p, a, b = _setup(W, orc, grid, prec, n_packages=3000)
    g_o, _, _ = orc.grad(p, a, threads=8, adj_absorbed=b)
    rho = B.density_tensor(p)
    for q in (-1, 0):
        g = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
        B.backward(p, rho, _dev(a), g, adj_absorbed=_dev(b), peel_queue=q)
        check(g.cpu().numpy(), g_o, 1e-9 if prec == 0 else 1e-5, "queue %d: grad" % q, _say)


def test_multiwavelength_absorbed_gradient(B, orc, W):
    import torch
    _say("multiwavelength disk: absorbed-tally gradient, subset and full size")
    p = W.multiwavelength(n_packages=200, lambdas=[0, 30, 60])
    p["first_package"] = 777_777
    img, A, _ = orc.run(p, threads=8)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(A.shape) * 1e3
    a = np.zeros(img.shape)
    g_o, _, _ = orc.grad(p, a, threads=8, adj_absorbed=b)
    rho = B.density_tensor(p)
    g = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
    B.backward(p, rho, _dev(a), g, adj_absorbed=_dev(b))
    check(g.cpu().numpy(), g_o, 1e-5, "subset: grad", _say)
    full = W.multiwavelength(n_packages=1_000_000)
    rho = B.density_tensor(full)
    images = torch.empty(B.image_shape(full), dtype=torch.float64, device="cuda")
    absorbed = torch.empty((100, rho.numel()), dtype=torch.float64, device="cuda")
    B.run_photons(full, rho, images, absorbed)
    adj = torch.zeros_like(images)
    bb = torch.randn(absorbed.shape, generator=torch.Generator(device="cuda").manual_seed(4), dtype=torch.float64,
                     device="cuda")
    g = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s1 = B.backward(full, rho, adj, g)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s2 = B.backward(full, rho, adj, g, adj_absorbed=bb)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    assert torch.isfinite(g).all() and g.abs().max() > 0
    _say("  1e8 items: image-only replay %.1f ms (kernel %.1f), with the absorbed term %.1f ms (kernel %.1f)"
         % ((t1 - t0) * 1e3, s1["kernel_ms"], (t2 - t1) * 1e3, s2["kernel_ms"]))
