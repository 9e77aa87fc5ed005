"""The attached (pathwise) density gradient (MCRT_ATTACHED) on the GPU
through the C ABI: against the oracle's attached gradient on every grid
kind, with split images, in chunks and in both precisions; on a package
subset of the edge-on spiral at full size (three 512x512 frames); against
the detached gradient in expectation on the 64^3 lognormal grid, with the
variance of the two estimators compared; and the time of the full-size
adjoint workload (1e7 packages) beside the detached adjoint."""
import time

import numpy as np
import pytest
from parity import check, rel_l1

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu] " + msg, flush=True)


def _dev(x, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype or torch.float64).cuda()


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_1410_1629_amd import binding
    binding.load()
    assert torch.cuda.is_available()
    return binding


def _problem(W, prec, n_packages=3000, **kw):
    n = (10, 9, 8)
    args = dict(n=n, rho=W.lognormal_density(n, 0.8, seed=31, f32=(prec == 1)), kappa=[1.2, 0.7],
                albedo=[0.7, 0.5], g=[0.45, -0.1],
                sources=[W.point((0.13, -0.21, 0.07), [1.0, 0.6]), W.expdisk(0.4, 0.15, [0.5, 1.5])],
                detectors=[W.frame(10.0, 30.0, 24, 24, 1.0, 1.0, azim=20.0), W.sed(10.0, 95.0, azim=40.0)],
                n_packages=n_packages, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT, w_min=1e-3, max_scatter=50,
                precision=prec)
    args.update(kw)
    return W.small_problem(**args)


def _grid(W, prob, kind, prec):
    if kind == "rect":
        from test_oracle_rectilinear import random_planes
        rng = np.random.default_rng(4)
        prob["planes"] = tuple(random_planes(prob["box"][2 * a], prob["box"][2 * a + 1], prob["n"][a], rng)
                               for a in range(3))
    elif kind == "tree":
        from test_oracle_tree import BOX, kd_tree
        T = kd_tree(W)
        rho = np.random.default_rng(7).lognormal(0.0, 0.8, T.n_cells)
        prob = dict(prob, box=BOX, n=(T.n_cells, 1, 1), tree=T.tree(),
                    rho=rho.astype(np.float32) if prec == 1 else rho)
    elif kind == "split":
        prob["flags"] |= W.FLAG_SPLIT
    return prob


def _attached(B, prob, rho, adj, **kw):
    import torch
    grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
    st = B.backward_density(prob, rho, adj, grad, attached=True, **kw)
    return grad, st


# The attached gradient runs in FP64 in both precisions (the FP32 path
# reads FP32 densities): its derivative amplifies the rounding of positions
# where a leg grazes a cell face, which FP32 walks do not follow (they gave
# 4e-6 on the regular grid, 8e-5 on the tree grid and 0.18 on the 64^3
# lognormal grid against the FP64 oracle).  Both precisions then meet the
# FP64 gate, the oracle taking the FP32 densities' values.
TOL32 = 1e-10


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind", ["regular", "rect", "tree", "split"])
def test_attached_matches_the_oracle(B, orc, W, kind, prec):
    _say("attached gradient: %s grid, precision %d" % (kind, prec))
    prob = _grid(W, _problem(W, prec), kind, prec)
    img, _, _ = orc.run(prob)
    adj = np.random.default_rng(5).standard_normal(img.shape)
    g_o, _, _ = orc.grad_attached(prob, adj)
    rho = B.density_tensor(prob)
    tol = 1e-10 if prec == 0 else TOL32
    for chunk in (0, 1700):
        grad, st = _attached(B, prob, rho, _dev(adj), max_chunk=chunk)
        check(grad.cpu().numpy(), g_o, tol, "%s, chunk %d: attached gradient" % (kind, chunk), _say)
        assert st["life_launches"] == (-(-2 * 3000 // chunk) if chunk else 1)
        assert st["packages"] == 2 * 3000


@pytest.mark.parametrize("prec", [0, 1])
def test_attached_deposit_walks_queued_inline_or_both(B, orc, W, prec):
    # the peel rays' deposit walks: all through the peel-job queue (the
    # default), all inline (no queue), or queued until a small queue is full
    _say("attached gradient: deposit walks by queue mode, precision %d" % prec)
    prob = _grid(W, _problem(W, prec), "regular", prec)
    img, _, _ = orc.run(prob)
    adj = np.random.default_rng(9).standard_normal(img.shape)
    g_o, _, _ = orc.grad_attached(prob, adj)
    rho = B.density_tensor(prob)
    tol = 1e-10 if prec == 0 else TOL32
    ref = None
    for q in (0, -1, 300):
        grad, st = _attached(B, prob, rho, _dev(adj), peel_queue=q)
        check(grad.cpu().numpy(), g_o, tol, "queue %d: attached gradient" % q, _say)
        if q == -1:
            assert st["x_queue"] == 0
        else:
            assert 0 < st["x_queue"] <= st["d_queue"]
        if q == 300:
            assert st["x_queue"] < st["d_queue"]  # the rest walked inline
        if ref is None:
            ref = st
        for key in ("x_path", "x_locate", "x_peel", "deposits", "d_queue", "events", "peels", "packages"):
            assert st[key] == ref[key], (q, key, st[key], ref[key])


def test_attached_rejects_what_it_cannot_differentiate(B, W):
    import torch
    prob = _problem(W, 0, n_packages=100)
    rho = B.density_tensor(prob)
    adj = torch.ones(B.image_shape(prob), dtype=torch.float64, device="cuda")
    cam = W.perspective((0.3, -0.2, 0.1), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 8, 8, 1.0, 1.0)
    p = dict(prob, detectors=[cam])
    with pytest.raises(B.McrtError):
        _attached(B, p, rho, torch.ones(B.image_shape(p), dtype=torch.float64, device="cuda"))
    with pytest.raises(B.McrtError):
        _attached(B, dict(prob, w_min=0.0, max_scatter=5000), rho, adj)
    ga = torch.empty(2, dtype=torch.float64, device="cuda")
    grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
    with pytest.raises(B.McrtError):
        B.backward(prob, rho, adj, grad_rho=grad, grad_albedo=ga, attached=True)


def test_attached_spiral_subset_matches_the_oracle(B, orc, W):
    _say("attached gradient: spiral, three 512x512 frames, 1500 packages deep in the run, FP32")
    prob = dict(W.spiral(n_packages=1500, precision=1), flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    prob["first_package"] = 3_141_592
    img_o, _, _ = orc.run(prob)
    adj = np.random.default_rng(13).standard_normal(img_o.shape) * 1e9
    g_o, _, _ = orc.grad_attached(prob, adj)
    rho = B.density_tensor(prob)
    grad, st = _attached(B, prob, rho, _dev(adj))
    check(grad.cpu().numpy(), g_o, TOL32, "spiral subset: attached gradient", _say)


def _sed_problem(W, n_packages, seed, precision=1):
    # the 64^3 lognormal grid of the adjoint workload, two SED instruments
    # seen along directions that no grid plane contains, termination by count:
    # the estimator is a smooth function of the densities, so both gradients
    # estimate the gradient of its expectation without bias
    base = W.adjoint(n_packages=n_packages, precision=precision)
    return dict(base, detectors=[W.sed(10.0, 30.0, azim=20.0), W.sed(10.0, 95.0, azim=40.0)], w_min=0.0,
                max_scatter=8, seed=seed)


def test_attached_at_full_grid_size_matches_the_oracle(B, orc, W):
    # the 64^3 grid of the adjoint workload, FP64 and FP32, 400 packages
    # deep in the run: the oracle's attached gradient element by element
    # (whole-run differences are no check at this size: with 64^3 i.i.d.
    # cells, a package whose leg grazes a cell face has a slope that holds
    # over a density change of 1e-9 only, so a difference at h = 1e-7
    # averages over kinks; per package the slopes agree at h = 1e-11).  The
    # same sensitivity makes FP64 rounding of the points (fused and unfused
    # products, the order of sums) show at 1e-9: gate 1e-8 in FP64.
    for prec in (0, 1):
        _say("attached gradient: 64^3 lognormal, two SED instruments, 400 packages, precision %d" % prec)
        prob = dict(_sed_problem(W, 400, 4357, precision=prec), first_package=2_718_281)
        img, _, _ = orc.run(prob)
        adj = np.random.default_rng(5).standard_normal(img.shape)
        g_o, _, _ = orc.grad_attached(prob, adj, threads=8)
        rho = B.density_tensor(prob)
        g, _ = _attached(B, prob, rho, _dev(adj))
        check(g.cpu().numpy(), g_o, 1e-8, "64^3 subset: attached gradient", _say)


def _spiral_sed(W, n_packages, seed):
    # the edge-on spiral's smooth disk (256 x 256 x 64 cells), seen by two
    # SED instruments along directions that no grid plane contains
    base = W.spiral(n_packages=n_packages, precision=1)
    return dict(base, detectors=[W.sed(1e4, 30.0, azim=20.0), W.sed(1e4, 95.0, azim=40.0)], w_min=0.0,
                max_scatter=8, seed=seed, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)


@pytest.mark.parametrize("medium", ["lognormal", "disk"])
def test_attached_and_detached_agree_in_expectation_and_compare_variances(B, W, medium):
    # Both gradients estimate the gradient of the expected loss (SED
    # instruments, termination by count); their means over 8 seeds agree
    # along 8 random directions within 3 standard errors, and their
    # variances are compared.  On the 64^3 i.i.d. lognormal grid the
    # attached estimator's crossing terms kappa (rho_before - rho_after)/k_a
    # are large and heavy-tailed (a leg that grazes a face); on the smooth
    # disk they are small.
    import torch
    K, N = 8, 500_000
    _say("attached vs detached: %s medium, two SED instruments, %d seeds x %d packages" % (medium, K, N))
    prob = _sed_problem(W, N, 1000) if medium == "lognormal" else _spiral_sed(W, N, 1000)
    rho = B.density_tensor(prob)
    rho_h = np.asarray(prob["rho"], dtype=np.float64).reshape(-1)
    adj = _dev(np.random.default_rng(5).standard_normal(B.image_shape(prob)))
    rng = np.random.default_rng(1)
    V = np.stack([rng.choice([-1.0, 1.0], size=rho_h.size) * rho_h for _ in range(8)])
    ga, gd = [], []
    for s in range(K):
        p = dict(prob, seed=1000 + s)
        g, _ = _attached(B, p, rho, adj)
        ga.append(g.cpu().numpy())
        g = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
        B.backward_density(p, rho, adj, g)
        gd.append(g.cpu().numpy())
    ga, gd = np.array(ga), np.array(gd)
    da, dd = ga @ V.T, gd @ V.T  # [seed][direction]
    diff = da - dd
    se = diff.std(axis=0, ddof=1) / np.sqrt(K)
    z = diff.mean(axis=0) / se
    _say("  directional derivatives (mean over seeds): attached %s" % np.array2string(da.mean(0), precision=3))
    _say("                                             detached %s" % np.array2string(dd.mean(0), precision=3))
    _say("  mean difference / standard error: %s" % np.array2string(z, precision=2))
    vr_dir = dd.var(axis=0, ddof=1) / da.var(axis=0, ddof=1)
    va, vd = ga.var(axis=0, ddof=1), gd.var(axis=0, ddof=1)
    live = (va > 0) & (vd > 0)
    ratio = vd[live] / va[live]
    _say("  variance detached / attached: directions %s" % np.array2string(vr_dir, precision=2))
    _say("  per cell: median %.2f, quartiles %.2f %.2f, summed over cells %.2f (%d cells)" % (
        np.median(ratio), np.quantile(ratio, 0.25), np.quantile(ratio, 0.75), vd.sum() / va.sum(), live.sum()))
    assert np.all(np.abs(z) <= 3.0)


def test_attached_full_size_adjoint_workload_time(B, W):
    # 1e7 packages of the adjoint workload (FP32): the attached gradient's
    # time beside the detached adjoint's (replay and tape).  Its face-on
    # frame looks along z, parallel to the x and y planes: there the
    # attached gradient omits the steps of the peel rays' columns (a
    # documented bias), so only its time and finiteness are checked here.
    import torch
    _say("adjoint workload, 1e7 packages: attached and detached adjoint times")
    prob = W.adjoint(n_packages=10_000_000, precision=1)
    rho = B.density_tensor(prob)
    images = torch.empty(B.image_shape(prob), dtype=torch.float64, device="cuda")
    tape = B.new_tape(prob)
    B.run_photons(prob, rho, images, None, tape=tape)
    adj = 2.0 * (images - 0.9 * images)
    out = {}
    for name, kw in (("attached", dict(attached=True)), ("detached, replay", {}), ("detached, tape", dict(tape=tape))):
        grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
        B.backward_density(prob, rho, adj, grad, **kw)  # untimed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = B.backward_density(prob, rho, adj, grad, **kw)
        torch.cuda.synchronize()
        out[name] = (grad.cpu().numpy(), st)
        _say("  %s: %.1f ms kernel (%d launches), %.2f s wall; crossings %.3e" % (
            name, st["kernel_ms"], st["life_launches"], time.perf_counter() - t0,
            st["x_path"] + st["x_locate"] + st["x_peel"]))
    g = out["attached"][0]
    assert np.isfinite(g).all() and np.abs(g).max() > 0
    _say("  rel_L1 attached vs detached: %.3e" % rel_l1(g, out["detached, replay"][0]))


def test_autograd_attached_estimator(B, W):
    # RTImage with adjoint_estimator = "attached": its backward pass is the
    # attached gradient of the C ABI (no tape), bit for bit up to atomic order
    import torch
    from paper_1410_1629_amd import autograd
    _say("autograd: RTImage with the attached estimator")
    prob = dict(_problem(W, 1, n_packages=2000), adjoint_estimator="attached")
    rho = B.density_tensor(prob).clone().requires_grad_(True)
    images = autograd.render(prob, rho)
    w = torch.as_tensor(np.random.default_rng(3).standard_normal(tuple(images.shape)), device="cuda")
    (images * w).sum().backward()
    g_ref, _ = _attached(B, prob, rho.detach(), w.contiguous())
    check(rho.grad.double().cpu().numpy(), g_ref.cpu().numpy(), 1e-6, "autograd vs C ABI: attached gradient", _say)
    with pytest.raises(ValueError):
        autograd.render(dict(prob, adjoint_estimator="pathwise"), rho)
    nl = len(prob["kappa"])
    with pytest.raises(ValueError):
        autograd.RTImageOptics.apply(rho, torch.tensor(prob["albedo"], device="cuda"),
                                     torch.tensor(prob["g"], device="cuda"),
                                     torch.ones((len(prob["sources"]), nl), dtype=torch.float64, device="cuda"), prob)
