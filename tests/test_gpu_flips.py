"""Pixel flips between the FP32 and the FP64 GPU paths, package by package.

An image is a sum of peel-off contributions, each added to the pixel that
its event's position projects into.  The FP32 traversal moves a package's
scattering points by rounding-sized amounts, so now and then an event lands
in the neighbouring pixel (or cell) in one precision and not the other: a
discrete difference that no tolerance on a continuous quantity describes.
This test measures that fraction directly.  Each package of a subset runs
alone (n_packages = 1, first_package = p) through the C ABI in both GPU
precisions; a package whose FP32 image has nonzero pixels the FP64 image
lacks, or the reverse, has a flipped contribution.  Reported: the fraction
of packages with a flip and the fraction of contributions that flipped.
Gated: the images summed over the flip-free packages (FP32 against FP64,
relative L1 and element-wise), and each frame's total over all packages,
at the FP32 tolerance of 1e-5.
"""
import numpy as np
import pytest
from parity import check, rel_l1

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu] " + msg, flush=True)


def _per_package(B, prob, prec, first, n):
    """Nonzero pixels (indices, values) of each package's own image."""
    import torch
    p = dict(prob, precision=prec, n_packages=1)
    rho = B.density_tensor(p)
    img = torch.empty(B.image_shape(p), dtype=torch.float64, device="cuda")
    out = []
    for i in range(n):
        B.run_photons(dict(p, first_package=first + i), rho, img, None, stats=False)
        flat = img.view(-1)
        idx = torch.nonzero(flat).view(-1)
        out.append((idx.cpu().numpy(), flat[idx].cpu().numpy()))
    return out


def _flips(B, prob, first, n, npix):
    a32 = _per_package(B, prob, 1, first, n)
    a64 = _per_package(B, prob, 0, first, n)
    flipped, contrib, one_sided = [], 0, 0
    sum32 = np.zeros(npix)
    sum64 = np.zeros(npix)
    clean32 = np.zeros(npix)
    clean64 = np.zeros(npix)
    for (i32, v32), (i64, v64) in zip(a32, a64):
        np.add.at(sum32, i32, v32)
        np.add.at(sum64, i64, v64)
        contrib += max(len(i64), len(i32))
        d = np.setxor1d(i32, i64)
        if len(d):
            flipped.append(len(d))
            one_sided += len(d)
        else:
            np.add.at(clean32, i32, v32)
            np.add.at(clean64, i64, v64)
    return {"packages": n, "flipped_packages": len(flipped), "pixels_touched": contrib,
            "one_sided_pixels": one_sided, "sum32": sum32 / n, "sum64": sum64 / n, "clean32": clean32 / n,
            "clean64": clean64 / n}


CASES = {
    "adjoint 64^3 lognormal": ("adjoint", 4000),
    "edge-on spiral, 3 x 512^2": ("spiral", 1000),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp32_pixel_flip_fraction(B, W, name):
    wl, n = CASES[name]
    prob = W.adjoint(n_packages=1, precision=1) if wl == "adjoint" else W.spiral(n_packages=1, precision=1)
    if wl == "spiral":
        prob = dict(prob, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    first = 1_000_003
    npix = int(np.prod(B.image_shape(prob)))
    _say("pixel flips FP32 vs FP64, %s, %d packages one by one" % (name, n))
    r = _flips(B, prob, first, n, npix)
    _say("  %d of %d packages have a flipped contribution (%.2e); %d one-sided pixels of %d touched (%.2e)" % (
        r["flipped_packages"], n, r["flipped_packages"] / n, r["one_sided_pixels"], r["pixels_touched"],
        r["one_sided_pixels"] / max(1, r["pixels_touched"])))
    _say("  all packages: images rel_L1 %.3e" % rel_l1(r["sum32"], r["sum64"]))
    check(r["clean32"], r["clean64"], 1e-5, "flip-free packages: images", _say)
    frames = [d["nx"] * d["ny"] for d in prob["detectors"]]
    off = 0
    for k, m in enumerate(frames):
        t32, t64 = r["sum32"][off:off + m].sum(), r["sum64"][off:off + m].sum()
        _say("  frame %d total: relative difference %.3e" % (k, abs(t32 - t64) / t64))
        assert abs(t32 - t64) < 1e-5 * t64
        off += m
    assert r["flipped_packages"] < 0.02 * n


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_1410_1629_amd import binding
    binding.load()
    assert torch.cuda.is_available()
    return binding
