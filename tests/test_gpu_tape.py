"""The adjoint tape (mcrt_opts.tape) on the GPU through the C ABI: the
forward run keeps T per leg and C per peel ray; the adjoint that reads them
replays each package once and skips the optical-depth walks of its peel
rays.  Against the oracle in every queue mode, with chunkings that differ
between forward and adjoint, with the optics gradients; a package subset of
the spiral at full size; tapes from other arguments rejected; an overflowed
tape replays without it; and the full-size adjoint workload (1e7 packages)
with and without the tape: the same gradient, the time saved printed."""
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


def _problem(W, prec, n_packages=3000):
    n = (10, 9, 8)
    return W.small_problem(n=n, rho=W.lognormal_density(n, 0.8, seed=31, f32=(prec == 1)), kappa=[1.2, 0.7],
                           albedo=[0.7, 0.5], g=[0.45, -0.1],
                           sources=[W.point((0.13, -0.21, 0.07), [1.0, 0.6]), W.expdisk(0.4, 0.15, [0.5, 1.5])],
                           detectors=[W.frame(10.0, 30.0, 24, 24, 1.0, 1.0, azim=20.0),
                                      W.frame(10.0, 90.0, 16, 16, 1.2, 1.2)],
                           n_packages=n_packages, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT, w_min=1e-3,
                           max_scatter=50, precision=prec)


def _grads(B, prob, rho, adj, tape, **kw):
    import torch
    nl, ns = len(prob["kappa"]), len(prob["sources"])
    out = [torch.empty(rho.numel(), dtype=torch.float64, device="cuda"),
           torch.empty(nl, dtype=torch.float64, device="cuda"), torch.empty(nl, dtype=torch.float64, device="cuda"),
           torch.empty(ns * nl, dtype=torch.float64, device="cuda")]
    st = B.backward(prob, rho, _dev(adj), *out, tape=tape, **kw)
    return [t.cpu().numpy() for t in out], st


@pytest.mark.parametrize("prec", [0, 1])
def test_tape_adjoint_matches_oracle(B, orc, W, prec):
    import torch
    _say("tape adjoint prec=%d" % prec)
    prob = _problem(W, prec)
    img_o, _, _ = orc.run(prob)
    adj = np.random.default_rng(5).standard_normal(img_o.shape)
    g_o, _, _, go = orc.grad(prob, adj, optics=True)
    rho = B.density_tensor(prob)
    tol = 1e-9 if prec == 0 else 1e-5
    for fq, fchunk in ((0, 0), (-1, 1700)):
        tape = B.new_tape(prob)
        images = torch.empty(B.image_shape(prob), dtype=torch.float64, device="cuda")
        B.run_photons(prob, rho, images, None, tape=tape, peel_queue=fq, max_chunk=fchunk)
        check(images.cpu().numpy(), img_o, 1e-10 if prec == 0 else 1e-5, "forward %d/%d: images" % (fq, fchunk), _say)
        for q in (-1, 0, 40):
            for chunk in (0, 1300):
                (gr, ga, gg, gl), st = _grads(B, prob, rho, adj, tape, peel_queue=q, max_chunk=chunk)
                what = "forward %d/%d, adjoint %d/%d" % (fq, fchunk, q, chunk)
                check(gr, g_o, tol, what + ": rho", _say)
                check(ga, go["albedo"], tol, what + ": albedo")
                check(gg, go["g"], tol, what + ": g")
                check(gl, np.asarray(go["lum"]).reshape(-1), tol, what + ": lum")
                assert st["life_launches"] == (-(-2 * 3000 // chunk) if chunk else 1)


def test_tape_spiral_subset_matches_oracle(B, orc, W):
    import torch
    _say("tape adjoint: spiral, three 512x512 frames, 1500 packages deep in the run")
    prob = dict(W.spiral(n_packages=1500, precision=1), flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    prob["first_package"] = 3_141_592
    img_o, _, _ = orc.run(prob)
    adj = np.random.default_rng(13).standard_normal(img_o.shape) * 1e9
    g_o, _, _ = orc.grad(prob, adj)
    rho = B.density_tensor(prob)
    tape = B.new_tape(prob)
    images = torch.empty(B.image_shape(prob), dtype=torch.float64, device="cuda")
    B.run_photons(prob, rho, images, None, tape=tape)
    grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
    st = B.backward_density(prob, rho, _dev(adj), grad, tape=tape)
    check(grad.cpu().numpy(), g_o, 1e-5, "gradient", _say)
    assert st["life_launches"] == 1


def test_tape_rejections_and_overflow_fallback(B, orc, W):
    import torch
    _say("tape: mismatched arguments, blank tape, overflowed tape")
    prob = _problem(W, 0, n_packages=800)
    rho = B.density_tensor(prob)
    tape = B.new_tape(prob)
    images = torch.empty(B.image_shape(prob), dtype=torch.float64, device="cuda")
    B.run_photons(prob, rho, images, None, tape=tape)
    adj = np.random.default_rng(2).standard_normal(B.image_shape(prob))
    grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
    for change in (dict(seed=99), dict(first_package=5), dict(albedo=[0.7, 0.51])):
        with pytest.raises(B.McrtError) as ei:
            B.backward_density(dict(prob, **change), rho, _dev(adj), grad, tape=tape)
        assert ei.value.code == B.EINVAL, change
    with pytest.raises(B.McrtError):
        B.backward_density(prob, rho, _dev(adj), grad, tape=torch.zeros_like(tape))
    g_o, _, _ = orc.grad(prob, adj)
    over = tape.clone()
    over[32] = 1  # the header's overflow word: the forward run had a package with more events than the tape keeps
    st = B.backward_density(prob, rho, _dev(adj), grad, tape=over)
    assert st["life_launches"] == 2  # replayed twice, without the tape
    check(grad.cpu().numpy(), g_o, 1e-9, "overflowed tape: gradient", _say)


def test_tape_full_size_adjoint_workload(B, W):
    # 1e7 packages of the adjoint workload, FP32 path: the gradient from the
    # tape equals the replay-only gradient (same dL/dI), and the time saved
    import torch
    _say("adjoint workload, 1e7 packages: adjoint with and without the tape")
    prob = W.adjoint(n_packages=10_000_000, precision=1)
    rho = B.density_tensor(prob)
    shape = B.image_shape(prob)
    images = torch.empty(shape, dtype=torch.float64, device="cuda")
    tape = B.new_tape(prob)
    sf = B.run_photons(prob, rho, images, None, tape=tape)
    adj = 2.0 * (images - 0.9 * images)
    out = {}
    for name, t in (("tape", tape), ("replay", None)):
        grad = torch.empty(rho.numel(), dtype=torch.float64, device="cuda")
        B.backward_density(prob, rho, adj, grad, tape=t)  # untimed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = B.backward_density(prob, rho, adj, grad, tape=t)
        torch.cuda.synchronize()
        out[name] = (grad.cpu().numpy(), time.perf_counter() - t0, st)
        _say("  %s: adjoint %.1f ms (life %.1f in %d launches, queue %.1f), %.2f s wall" % (
            name, st["kernel_ms"], st["life_ms"], st["life_launches"], st["queue_ms"], out[name][1]))
    _say("  forward with the tape %.1f ms; tape %.2f GB" % (sf["kernel_ms"], tape.numel() / 1e9))
    d = rel_l1(out["tape"][0], out["replay"][0])
    _say("  gradient rel_L1 tape vs replay %.3e" % d)
    assert d < 1e-9
    assert out["tape"][2]["kernel_ms"] < out["replay"][2]["kernel_ms"]
