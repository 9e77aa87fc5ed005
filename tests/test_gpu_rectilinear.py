"""The HIP path on rectilinear grids (planes spaced by any rule along each
axis; PowCub's power-law spacing, Table 1(d)), through the C ABI, against
the FP64 oracle: walks, peel-off, forward runs (peel rays queued and
inline) and the adjoint in both precisions, a package subset of the PowCub
spiral at its full grid and frame sizes, then the full 1e7-package PowCub
spiral (closure, counts, throughput).  Tolerances as in test_gpu_parity."""
import time

import numpy as np
import pytest
from parity import check, rel_l1

from test_oracle_rectilinear import random_planes

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


def _grids(W):
    rng = np.random.default_rng(29)
    box_r, n_r = (-2.0, 1.0, 0.0, 3.0, -1.0, 0.5), (9, 6, 5)
    return {
        "powcub": ((-1, 1, -1, 1, -1, 1), (16, 12, 10),
                   tuple(W.power_law_planes(-1.0, 1.0, m, r) for m, r in ((16, 20.0), (12, 5.0), (10, 30.0)))),
        "random_ragged": (box_r, n_r, tuple(random_planes(box_r[2 * a], box_r[2 * a + 1], n_r[a], rng)
                                            for a in range(3))),
    }


@pytest.mark.parametrize("grid", ["powcub", "random_ragged"])
@pytest.mark.parametrize("prec", [0, 1])
def test_trace_matches_oracle(B, orc, W, grid, prec):
    import torch
    _say("rectilinear trace %s prec=%d" % (grid, prec))
    box, n, planes = _grids(W)[grid]
    rho = W.lognormal_density(n, 1.0, seed=7, f32=(prec == 1))
    o, k = W.random_rays(3001, box, seed=19)
    max_seg = int(sum(n)) + 4
    tau_o, tot_o, cell_o, len_o, nseg_o = orc.trace(box, n, rho, 0.9, o, k, max_seg=max_seg, planes=planes)
    drho = _dev(rho.reshape(-1), torch.float32 if prec else torch.float64)
    tau = torch.empty(len(o), dtype=torch.float64, device="cuda")
    cell = torch.empty((len(o), max_seg), dtype=torch.int32, device="cuda")
    length = torch.empty((len(o), max_seg), dtype=torch.float64, device="cuda")
    nseg = torch.empty(len(o), dtype=torch.int32, device="cuda")
    tot = B.trace_path({"box": box, "n": n, "planes": planes}, drho, 0.9, prec, _dev(o), _dev(k), tau, max_seg,
                       cell, length, nseg)
    tau, cell, length, nseg = tau.cpu().numpy(), cell.cpu().numpy(), length.cpu().numpy(), nseg.cpu().numpy()
    tol = 1e-12 if prec == 0 else 2e-6
    np.testing.assert_allclose(tau, tau_o, rtol=tol, atol=tol * max(1.0, tau_o.max()) * 1e-3)
    same = nseg == nseg_o
    assert same.mean() > (0.999 if prec == 0 else 0.99), same.mean()
    for q in np.nonzero(same)[0]:
        m = nseg[q]
        if not np.array_equal(cell[q, :m], cell_o[q, :m].astype(np.int32)):
            assert min(len_o[q, :m].min(), length[q, :m].min()) < 1e-6 * max(box[1] - box[0], 1.0)
            continue
        np.testing.assert_allclose(length[q, :m], len_o[q, :m], rtol=tol, atol=tol * max(box[1] - box[0], 1.0))
    assert abs(tot - tot_o) <= 1e-3 * tot_o + 2


@pytest.mark.parametrize("prec", [0, 1])
def test_peel_matches_oracle(B, orc, W, prec):
    import torch
    _say("rectilinear peel prec=%d" % prec)
    box, n = (-20, 20, -20, 20, -2, 2), (40, 36, 12)
    planes = tuple(W.power_law_planes(box[2 * a], box[2 * a + 1], n[a], r) for a, r in enumerate((8.0, 8.0, 16.0)))
    rho = W.exp_disk_density(box, n, 2.0, 6.0, 0.25, planes=planes)
    if prec:
        rho = W.as_f32_values(rho)
    pos, din, w = W.random_events(20011, box, seed=5, isotropic=False)
    dets = [W.frame(1e4, inc, 33, 31, 20.0, 20.0) for inc in (0.0, 60.0, 90.0)]
    ref = orc.peel(box, n, rho, 1.1, 0.6, pos, din, w, dets, planes=planes)
    img = torch.zeros(ref.size, dtype=torch.float64, device="cuda")
    B.peel_off({"box": box, "n": n, "planes": planes}, _dev(rho.reshape(-1), torch.float32 if prec else torch.float64),
               1.1, 0.6, prec, _dev(pos), _dev(din), _dev(w), dets, img)
    check(img.cpu().numpy(), ref, 1e-12 if prec == 0 else 1e-6, "images", _say)


def _powcub_problem(W, prec, flags=None, n_packages=3000):
    n = (12, 10, 9)
    planes = tuple(W.power_law_planes(-1.0, 1.0, m, r) for m, r in zip(n, (10.0, 6.0, 14.0)))
    rho = W.lognormal_density(n, 0.8, seed=41, f32=(prec == 1))
    p = W.small_problem(n=n, rho=rho, kappa=1.3, albedo=0.7, g=0.4, sources=[W.point((0.11, -0.07, 0.05))],
                        detectors=[W.frame(10.0, 0.0, 20, 20, 1.2, 1.2),
                                   W.frame(10.0, 70.0, 16, 24, 1.3, 1.1, azim=20.0)],
                        n_packages=n_packages, precision=prec,
                        flags=flags if flags is not None else W.FLAGS_DEFAULT | W.FLAG_SPLIT)
    p["planes"] = planes
    return p


@pytest.mark.parametrize("prec", [0, 1])
def test_run_matches_oracle(B, orc, W, prec):
    _say("rectilinear run prec=%d" % prec)
    p = _powcub_problem(W, prec)
    img_o, abs_o, st_o = orc.run(p)
    tol = 1e-10 if prec == 0 else 1e-5
    for q in (-1, 0):
        images, absorbed, st = B.render(p, peel_queue=q)
        check(images.cpu().numpy(), img_o, tol, "queue %d: images" % q, _say)
        check(absorbed.cpu().numpy(), abs_o, tol, "queue %d: absorbed" % q, _say)
        assert st["packages"] == st_o["packages"]
        for key in ("events", "x_path", "x_locate", "x_peel"):
            assert abs(st[key] - st_o[key]) <= 1e-4 * st_o[key] + 2, (key, st[key], st_o[key])


@pytest.mark.parametrize("prec", [0, 1])
def test_backward_matches_oracle(B, orc, W, prec):
    import torch
    _say("rectilinear backward prec=%d" % prec)
    p = _powcub_problem(W, prec, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    img_o, _, _ = orc.run(p)
    adj = np.random.default_rng(8).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(p, adj)
    rho = B.density_tensor(p)
    for q in (-1, 0):
        grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
        B.backward_density(p, rho, _dev(adj), grad, peel_queue=q)
        check(grad.cpu().numpy(), g_o, 1e-9 if prec == 0 else 1e-5, "queue %d: grad" % q, _say)


@pytest.mark.parametrize("prec", [0, 1])
def test_powcub_spiral_subset_matches_oracle(B, orc, W, prec):
    # the PowCub spiral's grid and three 512x512 frames, a package subset
    # from deep inside the run: forward and adjoint
    import torch
    _say("PowCub spiral subset prec=%d" % prec)
    p = W.powcub_spiral(n_packages=1500, precision=prec)
    p["first_package"] = 2_718_281
    img_o, abs_o, _ = orc.run(p)
    images, absorbed, st = B.render(p)
    tol = 1e-10 if prec == 0 else 1e-5
    check(images.cpu().numpy(), img_o, tol, "images", _say)
    check(absorbed.cpu().numpy(), abs_o, tol, "absorbed", _say)
    adj = np.random.default_rng(13).standard_normal(img_o.shape) * 1e9
    g_o, _, _ = orc.grad(p, adj)
    rho = B.density_tensor(p)
    grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
    B.backward_density(p, rho, _dev(adj), grad)
    check(grad.cpu().numpy(), g_o, 1e-9 if prec == 0 else 1e-5, "gradient", _say)


def test_powcub_spiral_full_size(B, W):
    # 1e7 packages, FP32 path: forward and adjoint, energy closure, every
    # package accounted for; throughput beside the regular spiral's
    import torch
    _say("PowCub spiral: 1e7 packages, forward + adjoint")
    out = {}
    for name, p in (("powcub", W.powcub_spiral(n_packages=10_000_000)), ("regular", W.spiral(n_packages=10_000_000))):
        rho = B.density_tensor(p)
        images = torch.empty(B.image_shape(p), dtype=torch.float64, device="cuda")
        absorbed = torch.empty((1, rho.numel()), dtype=torch.float64, device="cuda")
        grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sf = B.run_photons(p, rho, images, absorbed)
        adj = torch.randn(images.shape, generator=torch.Generator(device="cuda").manual_seed(3), dtype=torch.float64,
                          device="cuda")
        sb = B.backward_density(p, rho, adj, grad)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        closure = (sf["absorbed"] + sf["escaped"] + sf["truncated"] - sf["emitted"]) / sf["emitted"]
        assert sf["packages"] == 10_000_000 and abs(closure) < 1e-6
        assert abs(absorbed.sum().item() - sf["absorbed"]) < 1e-9 * sf["emitted"]
        g = grad.cpu().numpy()
        assert np.isfinite(g).all() and np.any(g != 0)
        x = sf["x_path"] + sf["x_locate"] + sf["x_peel"]
        out[name] = (sf["kernel_ms"], sb["kernel_ms"], x)
        _say("  %s: forward %.1f ms, adjoint %.1f ms, %.3g packages/s per step, %.3g forward crossings/s "
             "(%.2f s wall)" % (name, sf["kernel_ms"], sb["kernel_ms"],
                                1e7 / ((sf["kernel_ms"] + sb["kernel_ms"]) / 1e3), x / (sf["kernel_ms"] / 1e3), wall))
