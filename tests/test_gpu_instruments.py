"""The HIP path's instruments (Sect. 2.2: SED and frame instruments of a
distant observer, perspective cameras anywhere, also inside the model)
through the C ABI against the FP64 oracle: forward runs with the peel rays
queued (and overflowing the queue) and walked inline, the adjoint and the
standalone peel-off on every grid kind in both precisions; then the edge-on
spiral at full size seen by an SED instrument and by a camera inside the
disk: a package subset deep in the run against the oracle, and 1e7
packages (closure, the SED against the face-on frame, throughput)."""
import time

import numpy as np
import pytest
from parity import check, rel_l1

from test_emu_instruments import BOX, instruments, problem

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


@pytest.mark.parametrize("grid", ["regular", "rect", "tree"])
@pytest.mark.parametrize("prec", [0, 1])
def test_run_matches_oracle(B, orc, W, grid, prec):
    _say("instruments run %s prec=%d" % (grid, prec))
    p = problem(W, grid, prec, n_packages=3000)
    img_o, abs_o, st_o = orc.run(p, threads=8)
    tol = 1e-10 if prec == 0 else 1e-5
    for q in (-1, 0, 500):
        images, absorbed, st = B.render(p, peel_queue=q)
        check(images.cpu().numpy(), img_o, tol, "queue %d: images" % q, _say)
        check(absorbed.cpu().numpy(), abs_o, tol, "queue %d: absorbed" % q, _say)
        for key in ("events", "x_path", "x_locate", "x_peel"):
            assert abs(st[key] - st_o[key]) <= 1e-4 * st_o[key] + 2, (key, st[key], st_o[key])


@pytest.mark.parametrize("grid", ["regular", "tree"])
@pytest.mark.parametrize("prec", [0, 1])
def test_adjoint_matches_oracle(B, orc, W, grid, prec):
    import torch
    _say("instruments adjoint %s prec=%d" % (grid, prec))
    p = problem(W, grid, prec, n_packages=2000, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    img_o, _, _ = orc.run(p, threads=8)
    adj = np.random.default_rng(8).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(p, adj, threads=8)
    rho = B.density_tensor(p)
    for q in (-1, 0):
        grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
        B.backward_density(p, rho, _dev(adj), grad, peel_queue=q)
        check(grad.cpu().numpy(), g_o, 1e-9 if prec == 0 else 1e-5, "queue %d: grad" % q, _say)


@pytest.mark.parametrize("prec", [0, 1])
def test_standalone_peel_matches_oracle(B, orc, W, prec):
    import torch
    _say("instruments peel_off prec=%d" % prec)
    n = (7, 6, 5)
    rho = W.lognormal_density(n, 0.8, seed=3, f32=(prec == 1))
    pos, din, w = W.random_events(20011, BOX, seed=5, isotropic=False)
    ref = orc.peel(BOX, n, rho, 1.1, 0.6, pos, din, w, instruments(W))
    img = torch.zeros(ref.size, dtype=torch.float64, device="cuda")
    B.peel_off({"box": BOX, "n": n}, _dev(rho.reshape(-1), torch.float32 if prec else torch.float64), 1.1, 0.6, prec,
               _dev(pos), _dev(din), _dev(w), instruments(W), img)
    check(img.cpu().numpy(), ref, 1e-12 if prec == 0 else 1e-6, "images", _say)


def _spiral_with_instruments(W, n_packages, precision=1):
    p = W.spiral(n_packages=n_packages, precision=precision)
    p["detectors"] = [p["detectors"][0], W.sed(1e4, 0.0),
                      W.perspective((8.0, 0.0, 0.02), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 512, 128, 12.0, 3.0)]
    return p


@pytest.mark.parametrize("prec", [0, 1])
def test_spiral_subset_with_camera_inside_matches_oracle(B, orc, W, prec):
    _say("spiral with SED and an inside camera, package subset, prec=%d" % prec)
    p = _spiral_with_instruments(W, 1500, precision=prec)
    p["first_package"] = 5_000_003
    img_o, abs_o, _ = orc.run(p, threads=8)
    images, absorbed, _ = B.render(p)
    check(images.cpu().numpy(), img_o, 1e-10 if prec == 0 else 1e-5, "images", _say)
    check(absorbed.cpu().numpy(), abs_o, 1e-10 if prec == 0 else 1e-5, "absorbed", _say)


def test_spiral_full_size_with_camera_inside(B, W):
    import torch
    _say("spiral, 1e7 packages: face-on frame, SED, camera inside the disk")
    out = {}
    for name, p in (("instruments", _spiral_with_instruments(W, 10_000_000)), ("frames", W.spiral())):
        rho = B.density_tensor(p)
        images = torch.empty(B.image_shape(p), dtype=torch.float64, device="cuda")
        absorbed = torch.empty((1, rho.numel()), dtype=torch.float64, device="cuda")
        B.run_photons(p, rho, images, absorbed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = B.run_photons(p, rho, images, absorbed)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        closure = (st["absorbed"] + st["escaped"] + st["truncated"] - st["emitted"]) / st["emitted"]
        assert st["packages"] == 10_000_000 and abs(closure) < 1e-6
        out[name] = (images, st, wall)
        _say("  %s: forward %.1f ms (life %.1f, queue %.1f; %.3g packages/s), %.3g peel rays, %.3g peel crossings"
             % (name, st["kernel_ms"], st["life_ms"], st["queue_ms"], 1e7 / wall, st["peels"], st["x_peel"]))
    images, st, _ = out["instruments"]
    img = images.cpu().numpy()
    frame, sed, cam = img[:, 0, :512 * 512].sum(), img[:, 0, 512 * 512].sum(), img[:, 0, 512 * 512 + 1:]
    _say("  SED %.6e, face-on frame total %.6e, camera total %.6e" % (sed, frame, cam.sum()))
    # the face-on frame misses the light from beyond its +-20 kpc square
    # (the untruncated stellar disk and its scattered light)
    assert frame <= sed * (1 + 1e-9) and frame > 0.95 * sed
    assert np.isfinite(cam).all() and cam.sum() > 0
