"""Pins of the oracle's instruments (Sect. 2.2: SED and frame instruments for
a distant observer, and the perspective instrument that can be placed
anywhere, even inside the model).

- The SED instrument records exactly what a frame covering the whole model
  records in total, and the direct flux L e^-tau / (4 pi D^2) of a point
  source in a uniform cube.
- A perspective camera inside a uniform medium sees a point source with
  flux L e^(-kappa rho s) / (4 pi s^2), s its distance to the source; from
  outside, e^-tau counts the dust up to the boundary only.
- Points on one line of sight through the eye fall in one pixel whatever
  their depth; points behind the eye are not seen; a mirrored point falls
  in the mirrored pixel.
- Far away, a perspective camera looking back along a frame's observer
  direction with the frame's e_y as up reproduces the frame: same pixels,
  and flux within the O(size / distance) difference of the two projections.
- Inside a lognormal medium, the peel-off to the eye matches e^-tau with tau
  from brute-force midpoint sampling of the density along the segment."""
import math

import numpy as np
import pytest

BOX = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)


def _cube(W, detectors, n_packages=4000, flags=None, n=(8, 8, 8), rho=None, albedo=0.6, g=0.4):
    return W.small_problem(n=n, box=BOX, rho=rho, kappa=1.0, albedo=albedo, g=g, sources=[W.point()],
                           detectors=detectors, n_packages=n_packages,
                           flags=flags if flags is not None else W.FLAGS_DEFAULT | W.FLAG_SPLIT)


def test_sed_is_the_total_of_a_frame_covering_the_model(orc, W):
    dets = [W.frame(20.0, 35.0, 24, 24, 2.0, 2.0, azim=10.0), W.sed(20.0, 35.0, azim=10.0)]
    img, _, _ = orc.run(_cube(W, dets, rho=W.lognormal_density((8, 8, 8), 0.7, seed=3)))
    frame = img[:, :, :576].sum(axis=2)
    sed = img[:, :, 576]
    np.testing.assert_allclose(sed, frame, rtol=1e-13)
    assert sed[0, 0] > 0 and sed[1, 0] > 0


def test_sed_direct_flux_of_a_point_source(orc, W):
    # face-on observer: the direct light crosses half the cube, tau = kappa rho * 1
    img, _, _ = orc.run(_cube(W, [W.sed(10.0, 0.0)], n_packages=1000, flags=W.FLAG_PEEL_EMIT))
    assert abs(img[0, 0, 0] / (math.exp(-1.0) / (4 * math.pi * 100.0)) - 1.0) < 1e-13


@pytest.mark.parametrize("eye_z", [0.6, 0.35, 3.0])
def test_perspective_camera_sees_a_point_source_through_the_dust_in_front_of_it(orc, W, eye_z):
    cam = W.perspective((0.0, 0.0, eye_z), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 5, 5, 0.5, 0.5)
    img, _, _ = orc.run(_cube(W, [cam], n_packages=500, flags=W.FLAG_PEEL_EMIT))
    s = eye_z
    tau = min(s, 1.0)  # uniform kappa rho = 1; outside the cube from z = 1 on
    want = math.exp(-tau) / (4 * math.pi * s * s)
    assert abs(img[0, 0, 12] / want - 1.0) < 1e-13
    assert np.count_nonzero(img) == 1


def _events_on_rays(eye, dirs, depths):
    return np.array([np.asarray(eye) + t * d for d in dirs for t in depths])


def test_perspective_projection_geometry(orc, W):
    eye = np.array([0.3, -0.2, -4.0])
    target = np.array([0.1, 0.05, 0.2])
    up = np.array([0.2, 1.0, 0.1])
    cam = W.perspective(eye, target, up, 7, 5, 0.8, 0.6)
    rng = np.random.default_rng(1)
    dirs = rng.normal(size=(40, 3)) * 0.12 + (target - eye) / np.linalg.norm(target - eye)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    depths = [0.5, 1.7, 3.9, 6.0]
    pos = _events_on_rays(eye, dirs, depths)
    n = pos.shape[0]
    rho = np.zeros((4, 4, 4))  # no dust: the image is the weight / (4 pi distance^2)
    pix = []
    for i in range(n):
        img = orc.peel(BOX, (4, 4, 4), rho, 1.0, 0.0, pos[i:i + 1], None, np.ones(1), [cam])
        nz = np.nonzero(img)[0]
        pix.append(int(nz[0]) if nz.size else -1)
        if nz.size:
            d2 = float(np.sum((pos[i] - eye) ** 2))
            assert abs(img[nz[0]] * 4 * math.pi * d2 - 1.0) < 1e-13
    pix = np.array(pix).reshape(len(dirs), len(depths))
    assert np.all(pix == pix[:, :1])  # one line of sight, one pixel
    assert (pix[:, 0] >= 0).sum() >= 10
    behind = eye - 0.5 * (target - eye)
    img = orc.peel(BOX, (4, 4, 4), rho, 1.0, 0.0, behind[None, :], None, np.ones(1), [cam])
    assert not img.any()
    # mirror through the view axis in the image plane: (ix, iy) -> (nx-1-ix, ny-1-iy)
    w_ax = (target - eye) / np.linalg.norm(target - eye)
    for d in dirs[:10]:
        p = eye + 2.0 * d
        q = eye + 2.0 * (2.0 * np.dot(d, w_ax) * w_ax - d)  # d rotated by 180 deg about the axis
        ip = np.nonzero(orc.peel(BOX, (4, 4, 4), rho, 1.0, 0.0, p[None], None, np.ones(1), [cam]))[0]
        iq = np.nonzero(orc.peel(BOX, (4, 4, 4), rho, 1.0, 0.0, q[None], None, np.ones(1), [cam]))[0]
        if ip.size and iq.size:
            assert iq[0] == (5 - 1 - ip[0] // 7) * 7 + (7 - 1 - ip[0] % 7)


def test_far_perspective_camera_reproduces_the_frame(orc, W):
    D = 1e5
    frame = W.frame(D, 50.0, 16, 12, 1.2, 0.9, azim=25.0, pa=15.0)
    kd, ex, ey = orc.detector_basis(frame)
    cam = W.perspective(tuple(D * kd), (0.0, 0.0, 0.0), tuple(ey), 16, 12, 1.2, 0.9)
    _, cex, cey = orc.detector_basis(cam)
    np.testing.assert_allclose(cex, ex, atol=1e-14)
    np.testing.assert_allclose(cey, ey, atol=1e-14)
    rho = W.lognormal_density((6, 6, 6), 0.8, seed=2)
    p = W.small_problem(n=(6, 6, 6), box=BOX, rho=rho, kappa=1.2, albedo=0.7, g=0.5,
                        sources=[W.point((0.1, 0.2, 0.0))], detectors=[frame, cam], n_packages=3000,
                        flags=W.FLAGS_DEFAULT)
    img, _, _ = orc.run(p)
    f, c = img[0, 0, :192], img[0, 0, 192:]
    # pixels agree except where a point sits within O(size/D) of a pixel edge
    assert np.abs(c - f).sum() / f.sum() < 1e-3
    np.testing.assert_allclose(c.sum(), f.sum(), rtol=1e-4)


def test_peel_to_an_eye_inside_the_dust_matches_sampled_optical_depth(orc, W):
    n = (6, 5, 7)
    rho = W.lognormal_density(n, 1.0, seed=8)
    eye = np.array([0.13, -0.21, 0.07])
    cam = W.perspective(eye, (0.5, 0.3, -0.4), (0.0, 0.0, 1.0), 9, 9, 3.0, 3.0)
    rng = np.random.default_rng(4)
    pos = rng.uniform(-0.95, 0.95, (60, 3))
    kappa = 0.8
    got = []
    for q in range(pos.shape[0]):
        one = orc.peel(BOX, n, rho, kappa, 0.0, pos[q:q + 1], None, np.ones(1), [cam])
        got.append(one.sum())
    got = np.array(got)
    d = np.asarray(BOX)
    lo, hi = d[0::2], d[1::2]
    cell = (hi - lo) / np.array(n)
    seen = 0
    for q in range(pos.shape[0]):
        if got[q] == 0.0:
            continue
        seen += 1
        seg = eye - pos[q]
        L = np.linalg.norm(seg)
        t = (np.arange(20000) + 0.5) / 20000
        pts = pos[q][None, :] + t[:, None] * seg[None, :]
        ijk = np.floor((pts - lo) / cell).astype(int)
        ijk = np.clip(ijk, 0, np.array(n) - 1)
        tau = kappa * rho[ijk[:, 2], ijk[:, 1], ijk[:, 0]].mean() * L
        want = math.exp(-tau) / (4 * math.pi * L * L)
        assert abs(got[q] / want - 1.0) < 2e-3, (q, got[q], want)
    assert seen >= 10
