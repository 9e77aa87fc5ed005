"""The HIP path on tree grids (k-d tree and octree; Table 1(d), Sect. 2.4),
through the C ABI, against the FP64 oracle: walks (a tree halving the box
into a regular grid, an adaptive k-d tree, an octree), peel-off, forward
runs with the queue on and off and the adjoint in both precisions, a package
subset of the k-d-tree spiral at full size, then the full 1e7-package k-d
tree spiral (closure, counts, throughput).  Tolerances as in
test_gpu_parity."""
import time

import numpy as np
import pytest
from parity import check, rel_l1

from test_oracle_tree import BOX, _blob, kd_tree, octree

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


def _tree(W, kind):
    return {"kd": kd_tree, "oct": octree}[kind](W) if kind != "regular" else W.regular_tree(BOX, (3, 2, 2))


@pytest.mark.parametrize("kind", ["kd", "oct", "regular"])
@pytest.mark.parametrize("prec", [0, 1])
def test_trace_matches_oracle(B, orc, W, kind, prec):
    import torch
    _say("tree trace %s prec=%d" % (kind, prec))
    T = _tree(W, kind)
    rho = np.random.default_rng(7).lognormal(0.0, 1.0, T.n_cells)
    if prec:
        rho = W.as_f32_values(rho)
    n = (T.n_cells, 1, 1)
    o, k = W.random_rays(3001, BOX, seed=19)
    max_seg = 256
    tau_o, tot_o, cell_o, len_o, nseg_o = orc.trace(BOX, n, rho, 0.9, o, k, max_seg=max_seg, tree=T.tree())
    drho = _dev(rho, torch.float32 if prec else torch.float64)
    tau = torch.empty(len(o), dtype=torch.float64, device="cuda")
    cell = torch.empty((len(o), max_seg), dtype=torch.int32, device="cuda")
    length = torch.empty((len(o), max_seg), dtype=torch.float64, device="cuda")
    nseg = torch.empty(len(o), dtype=torch.int32, device="cuda")
    tot = B.trace_path({"box": BOX, "n": n, "tree": T.tree()}, drho, 0.9, prec, _dev(o), _dev(k), tau, max_seg, cell,
                       length, nseg)
    tau, cell, length, nseg = tau.cpu().numpy(), cell.cpu().numpy(), length.cpu().numpy(), nseg.cpu().numpy()
    tol = 1e-12 if prec == 0 else 2e-6
    np.testing.assert_allclose(tau, tau_o, rtol=tol, atol=tol * max(1.0, tau_o.max()) * 1e-3)
    same = nseg == nseg_o
    assert same.mean() > (0.999 if prec == 0 else 0.99), same.mean()
    for q in np.nonzero(same)[0]:
        m = nseg[q]
        if not np.array_equal(cell[q, :m], cell_o[q, :m].astype(np.int32)):
            assert min(len_o[q, :m].min(), length[q, :m].min()) < 1e-6
            continue
        np.testing.assert_allclose(length[q, :m], len_o[q, :m], rtol=tol, atol=tol * 2.0)
    assert abs(tot - tot_o) <= 1e-3 * tot_o + 2


@pytest.mark.parametrize("prec", [0, 1])
def test_peel_matches_oracle(B, orc, W, prec):
    import torch
    _say("tree peel prec=%d" % prec)
    T = kd_tree(W)
    c = 0.5 * np.add(*T.leaf_boxes())
    rho = _blob(c[:, 0], c[:, 1], c[:, 2])
    if prec:
        rho = W.as_f32_values(rho)
    pos, din, w = W.random_events(20011, BOX, seed=5, isotropic=False)
    dets = [W.frame(10.0, inc, 17, 15, 1.1, 1.1) for inc in (0.0, 60.0, 90.0)]
    n = (T.n_cells, 1, 1)
    ref = orc.peel(BOX, n, rho, 1.1, 0.6, pos, din, w, dets, tree=T.tree())
    img = torch.zeros(ref.size, dtype=torch.float64, device="cuda")
    B.peel_off({"box": BOX, "n": n, "tree": T.tree()}, _dev(rho, torch.float32 if prec else torch.float64), 1.1, 0.6,
               prec, _dev(pos), _dev(din), _dev(w), dets, img)
    check(img.cpu().numpy(), ref, 1e-12 if prec == 0 else 1e-6, "images", _say)


def _tree_problem(W, kind, prec, flags=None, n_packages=3000):
    T = kd_tree(W, max_mass=0.05, depth=10) if kind == "kd" else octree(W)
    return W.tree_problem(kind, BOX, T, _blob, 1.3, 0.7, 0.4, [W.point((0.11, -0.07, 0.05))],
                          [W.frame(10.0, 0.0, 20, 20, 1.2, 1.2), W.frame(10.0, 70.0, 16, 24, 1.3, 1.1, azim=20.0)],
                          n_packages, prec, flags=flags if flags is not None else W.FLAGS_DEFAULT | W.FLAG_SPLIT)


@pytest.mark.parametrize("kind", ["kd", "oct"])
@pytest.mark.parametrize("prec", [0, 1])
def test_run_matches_oracle(B, orc, W, kind, prec):
    _say("tree run %s prec=%d" % (kind, prec))
    p = _tree_problem(W, kind, prec)
    img_o, abs_o, st_o = orc.run(p)
    tol = 1e-10 if prec == 0 else 1e-5
    for q in (-1, 0):
        images, absorbed, st = B.render(p, peel_queue=q)
        check(images.cpu().numpy(), img_o, tol, "queue %d: images" % q, _say)
        check(absorbed.cpu().numpy(), abs_o, tol, "queue %d: absorbed" % q, _say)
        assert st["packages"] == st_o["packages"]
        for key in ("events", "x_path", "x_locate", "x_peel"):
            assert abs(st[key] - st_o[key]) <= 1e-4 * st_o[key] + 2, (key, st[key], st_o[key])


@pytest.mark.parametrize("kind", ["kd", "oct"])
@pytest.mark.parametrize("prec", [0, 1])
def test_backward_matches_oracle(B, orc, W, kind, prec):
    import torch
    _say("tree backward %s prec=%d" % (kind, prec))
    p = _tree_problem(W, kind, prec, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    img_o, _, _ = orc.run(p)
    adj = np.random.default_rng(8).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(p, adj)
    rho = B.density_tensor(p)
    for q in (-1, 0):
        grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
        B.backward_density(p, rho, _dev(adj), grad, peel_queue=q)
        check(grad.cpu().numpy(), g_o, 1e-9 if prec == 0 else 1e-5, "queue %d: grad" % q, _say)


@pytest.mark.parametrize("prec", [0, 1])
def test_kdtree_spiral_subset_matches_oracle(B, orc, W, prec):
    # the k-d tree spiral (about 1e6 leaves) with its three 512x512 frames, a
    # package subset from deep inside the run: forward and adjoint (the
    # oracle's leaf search scans all leaves, so the subset is small)
    import torch
    _say("k-d tree spiral subset prec=%d" % prec)
    p = W.kdtree_spiral(n_packages=40, precision=prec, max_mass=3e-3)
    p["first_package"] = 1_234_567
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


def test_kdtree_spiral_full_size(B, W):
    # 1e7 packages, FP32 path: forward and adjoint, energy closure, every
    # package accounted for, throughput
    import torch
    p = W.kdtree_spiral(n_packages=10_000_000)
    _say("%s: 1e7 packages, forward + adjoint" % p["name"])
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
    _say("  forward %.1f ms, adjoint %.1f ms, %.3g packages/s per step, %.3g forward crossings/s (%.2f s wall)" % (
        sf["kernel_ms"], sb["kernel_ms"], 1e7 / ((sf["kernel_ms"] + sb["kernel_ms"]) / 1e3),
        x / (sf["kernel_ms"] / 1e3), wall))


@pytest.mark.parametrize("prec", [0, 1])
def test_kdtree_spiral_bench_tree_subset_matches_oracle(B, orc, W, prec):
    # the benchmark's own k-d tree (967 656 leaves, max_mass 3e-4) with its
    # three 512x512 frames: a few packages from deep inside the run, forward
    # and adjoint (the oracle's brute-force leaf search scans every leaf per
    # crossing, about 1 ms each)
    import os
    import torch
    _say("k-d tree spiral, the benchmark's tree, 16 packages, prec=%d" % prec)
    p = W.kdtree_spiral(n_packages=16, precision=prec)
    assert p["n"][0] > 900_000
    p["first_package"] = 7_777_777
    threads = len(os.sched_getaffinity(0))
    img_o, abs_o, st_o = orc.run(p, threads=threads)
    images, absorbed, st = B.render(p)
    tol = 1e-10 if prec == 0 else 1e-5
    check(images.cpu().numpy(), img_o, tol, "images", _say)
    check(absorbed.cpu().numpy(), abs_o, tol, "absorbed", _say)
    for key in ("events", "x_path", "x_locate", "x_peel"):
        assert abs(st[key] - st_o[key]) <= 1e-4 * st_o[key] + 2, (key, st[key], st_o[key])
    adj = np.random.default_rng(14).standard_normal(img_o.shape) * 1e9
    g_o, _, _ = orc.grad(p, adj, threads=threads)
    rho = B.density_tensor(p)
    grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
    B.backward_density(p, rho, _dev(adj), grad)
    check(grad.cpu().numpy(), g_o, 1e-9 if prec == 0 else 1e-5, "gradient", _say)
