"""The HIP library's per-lane code, run on the CPU by the bounds-checked
harness (tests/helpers/mcrt_emu.cpp), against the FP64 oracle.

This checks the kernels' logic -- state machine, walk, tallies, adjoint
replay -- and that no access leaves its buffer, before any GPU run; the
GPU tests then check the same cases on the device.  Tolerances as for the
GPU: FP64 1e-10 relative L1, FP32 traversal 1e-5.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "helpers"))


def rel_l1(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a).sum())


def _same_counts(st, ref, keys, prec):
    """The life kernel's counts are identical in every queue mode; the
    peel-ray crossings too in FP64, and in FP32 up to the near-ties that the
    FP32 times of the queued walks merge or split."""
    for key in keys:
        assert st[key] == ref[key], key
    slack = 0 if prec == 0 else 1e-5 * ref["x_peel"] + 2
    assert abs(st["x_peel"] - ref["x_peel"]) <= slack, (st["x_peel"], ref["x_peel"])


TRACE_CASES = [
    ("uniform32", (-1, 1, -1, 1, -1, 1), (32, 32, 32), None, 1.0),
    ("lognormal_ragged", (-2.0, 1.0, 0.0, 3.0, -1.0, 0.5), (9, 6, 5), 9, 0.7),
    ("flat", (-20, 20, -20, 20, -2, 2), (64, 3, 17), 4, 1.3),
    ("one_cell", (-1, 1, -1, 1, -1, 1), (1, 1, 1), 5, 2.0),
]


@pytest.mark.parametrize("name,box,n,seed,kappa", TRACE_CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_trace(E, orc, W, name, box, n, seed, kappa, prec):
    rho = np.ones(n[::-1]) if seed is None else W.lognormal_density(n, 1.0, seed=seed, f32=(prec == 1))
    o, k = W.random_rays(3001, box, seed=17)
    max_seg = int(sum(n)) + 4
    tau_o, tot_o, cell_o, len_o, nseg_o = orc.trace(box, n, rho, kappa, o, k, max_seg=max_seg)
    rc, tau, tot, cell, length, nseg = E.trace(box, n, rho, kappa, prec, o, k, max_seg=max_seg)
    assert rc == 0
    tol = 1e-12 if prec == 0 else 2e-6
    np.testing.assert_allclose(tau, tau_o, rtol=tol, atol=tol * max(1.0, tau_o.max()) * 1e-3)
    same = nseg == nseg_o
    assert same.mean() > (0.999 if prec == 0 else 0.99), same.mean()
    for q in np.nonzero(same)[0]:
        m = nseg[q]
        if not np.array_equal(cell[q, :m], cell_o[q, :m].astype(np.int32)):
            assert min(len_o[q, :m].min(), length[q, :m].min()) < 1e-6 * max(box[1] - box[0], 1.0)
            continue
        # lengths are differences of crossing times: absolute rounding scales with the box
        np.testing.assert_allclose(length[q, :m], len_o[q, :m], rtol=tol, atol=tol * max(box[1] - box[0], 1.0))
    assert abs(tot - tot_o) <= 1e-3 * tot_o + 2


def test_trace_edge_cases(E, orc):
    box, n = (-1, 1, -1, 1, -1, 1), (4, 4, 4)
    o = np.array([[2.0, 0, 0], [1.0, 0, 0], [-1.0, 0.0, 0.1], [0.0, 0.1, 0.1], [0.0, 0.1, 0.1],
                  [0.0, 0.0, 0.0], [np.nan, 0, 0], [0.3, -0.2, 0.1]])
    k = np.array([[1.0, 0, 0], [1.0, 0, 0], [1.0, 0, 0], [-1.0, 0, 0], [1.0, 0, 0],
                  [1 / np.sqrt(3)] * 3, [1.0, 0, 0], [0.0, 1e-25, 1.0]])
    rc, tau, tot, cell, length, nseg = E.trace(box, n, np.ones(64), 1.0, 0, o, k, max_seg=2)
    assert rc == -2  # the wall-plane ray crosses 4 cells
    tau_o, _, cell_o, _, nseg_o = orc.trace(box, n, np.ones(64), 1.0, o[:6], k[:6], max_seg=4)
    np.testing.assert_allclose(tau[:6], tau_o, rtol=1e-14, atol=1e-15)
    np.testing.assert_array_equal(nseg[:6], nseg_o)
    assert tau[6] == 0.0 and nseg[6] == 0  # non-finite origin: no walk
    assert abs(tau[7] - 0.9) < 1e-14  # a component below 1e-20 counts as parallel
    rc, tau, tot, *_ = E.trace(box, n, np.ones(64), 1.0, 0, np.zeros((0, 3)), np.zeros((0, 3)))
    assert rc == 0 and tot == 0


def test_fp32_axis_limit(E):
    """FP32 walks count crossed planes in FP32, exact below 2^24: a grid
    with 2^24 cells along an axis is rejected in FP32 (before any walk) and
    accepted in FP64; 2^24 - 1 cells pass the check."""
    box = (-1, 1, -1, 1, -1, 1)
    o, k = np.zeros((0, 3)), np.zeros((0, 3))
    for n in ((1, 1, 1 << 24), (1 << 24, 1, 1), (1, 1 << 24, 1)):
        assert E.trace(box, n, np.ones(1), 1.0, 1, o, k)[0] == -1
        assert E.trace(box, n, np.ones(1), 1.0, 0, o, k)[0] == 0
    assert E.trace(box, (1, 1, (1 << 24) - 1), np.ones(1), 1.0, 1, o, k)[0] == 0


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("iso", [True, False])
def test_peel(E, orc, W, prec, iso):
    box, n = (-20, 20, -20, 20, -2, 2), (40, 36, 12)
    rho = W.exp_disk_density(box, n, 2.0, 6.0, 0.25)
    if prec:
        rho = W.as_f32_values(rho)
    pos, din, w = W.random_events(4011, box, seed=5, isotropic=iso)
    dets = [W.frame(1e4, inc, 33, 31, 20.0, 20.0) for inc in (0.0, 60.0, 90.0)] + [
        W.frame(1e4, 37.0, 16, 16, 10.0, 8.0, azim=25.0, pa=30.0)]
    ref = orc.peel(box, n, rho, 1.1, 0.6, pos, din, w, dets)
    got = E.peel(box, n, rho, 1.1, 0.6, prec, pos, din, w, dets)
    assert rel_l1(got, ref) < (1e-12 if prec == 0 else 1e-6)
    np.testing.assert_array_equal(got != 0, ref != 0)


def _compare(E, orc, prob, tol):
    images, absorbed, st = E.run(prob)
    img_o, abs_o, st_o = orc.run(prob)
    assert rel_l1(images, img_o) < tol, rel_l1(images, img_o)
    if absorbed is not None:
        assert rel_l1(absorbed, abs_o) < tol, rel_l1(absorbed, abs_o)
    for key in ("emitted", "absorbed", "escaped", "truncated"):
        assert abs(st[key] - st_o[key]) <= max(tol, 1e-12) * 10 * st_o["emitted"], (key, st[key], st_o[key])
    for key in ("packages",):
        assert st[key] == st_o[key]
    for key in ("events", "x_path", "x_locate", "x_peel"):
        assert abs(st[key] - st_o[key]) <= 1e-4 * st_o[key] + 2, (key, st[key], st_o[key])
    return images, absorbed, st


@pytest.mark.parametrize("prec", [0, 1])
def test_run_cube(E, orc, W, prec):
    prob = W.cube(n_packages=6000, precision=prec, flags=W.FLAGS_DEFAULT | W.FLAG_SPLIT)
    images, _, st = _compare(E, orc, prob, 1e-10 if prec == 0 else 1e-5)
    assert abs(images[0, 0].reshape(64, 64)[32, 32] - np.exp(-1) / (400 * np.pi)) < 1e-6 * 2.93e-4
    closure = st["absorbed"] + st["escaped"] + st["truncated"] - st["emitted"]
    assert abs(closure) < (1e-12 if prec == 0 else 1e-6) * st["emitted"]


def test_run_multiwavelength_two_sources(E, orc, W):
    prob = W.small_problem(n=(10, 7, 6), box=(-1.0, 1.5, -1.0, 1.0, -0.8, 0.8),
                           rho=W.lognormal_density((10, 7, 6), 1.0, seed=4), kappa=[0.5, 1.0, 2.5],
                           albedo=[0.9, 0.5, 0.0], g=[0.7, 0.0, -0.3],
                           sources=[W.point((0.2, 0.1, -0.3), [1.0, 2.0, 0.5]), W.expdisk(0.3, 0.1, [3.0, 1.0, 1.0])],
                           detectors=[W.frame(10.0, 30.0, 24, 20, 1.5, 1.2, azim=10.0),
                                      W.frame(10.0, 90.0, 17, 9, 1.5, 1.0, pa=20.0)],
                           n_packages=2003, flags=W.FLAGS_DEFAULT | W.FLAG_SPLIT)
    _compare(E, orc, prob, 1e-10)


@pytest.mark.parametrize("flags", [0, 1, 2, 3, 4, 7])
def test_run_flags(E, orc, W, flags):
    prob = W.small_problem(n=(8, 8, 8), rho=W.lognormal_density((8, 8, 8), 0.7, seed=6),
                           detectors=[W.frame(10.0, 45.0, 16, 16, 1.0, 1.0)], n_packages=1001, flags=flags)
    _compare(E, orc, prob, 1e-10)


def test_run_no_frames_and_empty_medium(E, orc, W):
    prob = W.small_problem(n=(5, 5, 5), detectors=[], n_packages=500)
    _compare(E, orc, prob, 1e-10)
    prob = W.small_problem(n=(5, 5, 5), rho=np.zeros((5, 5, 5)), n_packages=500, sources=[W.expdisk(0.5, 0.2)])
    images, absorbed, st = _compare(E, orc, prob, 1e-10)
    assert st["events"] == 0 and st["escaped"] == pytest.approx(st["emitted"], rel=1e-14)


def test_run_wave_sizes_and_batches_agree(E, W):
    prob = W.small_problem(n=(9, 9, 9), rho=W.lognormal_density((9, 9, 9), 1.0, seed=3), n_packages=1500)
    ref, ref_a, ref_s = E.run(prob)
    for wave, batch in ((1, 0), (7, 3), (64, 1), (64, 64)):
        im, ab, st = E.run(prob, wave=wave, event_batch=batch)
        assert rel_l1(im, ref) < 1e-12 and rel_l1(ab, ref_a) < 1e-12
        assert st["x_path"] == ref_s["x_path"] and st["events"] == ref_s["events"]


def test_run_spiral_full_grid_subset(E, orc, W):
    prob = W.spiral(n_packages=800, precision=1)
    prob["first_package"] = 7_654_321
    _compare(E, orc, prob, 1e-5)


@pytest.mark.parametrize("prec", [0, 1])
def test_backward(E, orc, W, prec):
    n = (10, 10, 10)
    prob = W.small_problem(n=n, rho=W.lognormal_density(n, 0.8, seed=31, f32=(prec == 1)), kappa=1.2, albedo=0.7,
                           g=0.45, sources=[W.point((0.13, -0.21, 0.07))],
                           detectors=[W.frame(10.0, 30.0, 24, 24, 1.0, 1.0, azim=20.0),
                                      W.frame(10.0, 90.0, 16, 16, 1.2, 1.2)],
                           n_packages=1200, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT, w_min=1e-3, max_scatter=50,
                           precision=prec)
    img_o, _, _ = orc.run(prob)
    target = img_o * (1 + 0.3 * np.random.default_rng(5).standard_normal(img_o.shape))
    adj = 2 * (img_o - target)
    g_o, _, st_o = orc.grad(prob, adj)
    g, st = E.grad(prob, adj)
    assert rel_l1(g, g_o) < (1e-9 if prec == 0 else 1e-5), rel_l1(g, g_o)
    assert st["packages"] == st_o["packages"]
    g0, _ = E.grad(prob, np.zeros_like(adj))
    assert np.all(g0 == 0)


def test_backward_split_and_multi_lambda(E, orc, W):
    prob = W.small_problem(n=(7, 6, 5), rho=W.lognormal_density((7, 6, 5), 0.6, seed=2), kappa=[0.8, 1.5],
                           albedo=[0.6, 0.3], g=[0.5, -0.2], detectors=[W.frame(10.0, 20.0, 12, 10, 1.0, 1.0)],
                           n_packages=700, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT | W.FLAG_SPLIT)
    img_o, _, _ = orc.run(prob)
    adj = np.random.default_rng(2).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(prob, adj)
    g, _ = E.grad(prob, adj)
    assert rel_l1(g, g_o) < 1e-9


# Internal cell layout: bricks of 2^lx x 2^ly x 2^lz cells.  The walk, its
# arithmetic and the order of every deposit do not depend on the brick, so
# every shape -- including ones that leave padding cells on ragged grids,
# which the harness refuses to read -- must give bit-identical results.
BRICKS = [None, (0, 0, 0), (5, 0, 0), (1, 1, 3), (2, 2, 2), (3, 0, 1), (0, 3, 2), (7, 0, 3)]


@pytest.mark.parametrize("prec", [0, 1])
def test_brick_shapes_trace_and_peel(E, W, prec):
    from paper_1410_1629_amd.binding import brick
    box, n = (-2.0, 1.0, 0.0, 3.0, -1.0, 0.5), (13, 6, 5)
    rho = W.lognormal_density(n, 1.0, seed=12, f32=(prec == 1))
    o, k = W.random_rays(1500, box, seed=19)
    pos, din, w = W.random_events(700, box, seed=8, isotropic=False)
    dets = [W.frame(1e3, 50.0, 20, 18, 3.0, 3.0, azim=15.0), W.frame(1e3, 90.0, 11, 7, 3.0, 2.0)]
    ref = None
    for b in BRICKS:
        shape = 0 if b is None else brick(*b)
        rc, tau, tot, cell, length, nseg = E.trace(box, n, rho, 0.9, prec, o, k, max_seg=40, brick_shape=shape)
        img = E.peel(box, n, rho, 0.9, 0.3, prec, pos, din, w, dets, brick_shape=shape)
        got = (tau, tot, cell, length, nseg, img)
        if ref is None:
            ref = got
            continue
        assert rc == 0 and tot == ref[1]
        for a, r in zip(got, ref):
            np.testing.assert_array_equal(a, r)


def test_brick_shapes_life_and_adjoint(E, W):
    from paper_1410_1629_amd.binding import brick
    n = (11, 7, 9)
    prob = W.small_problem(n=n, box=(-1.0, 1.5, -1.0, 1.0, -0.8, 0.8), rho=W.lognormal_density(n, 0.9, seed=21),
                           kappa=[0.9, 2.0], albedo=[0.7, 0.4], g=[0.5, -0.1],
                           detectors=[W.frame(10.0, 35.0, 16, 14, 1.5, 1.2)], n_packages=600,
                           flags=W.FLAGS_DEFAULT | W.FLAG_SPLIT)
    adj = np.random.default_rng(9).standard_normal((2, 2, 16 * 14))
    ref = None
    for b in BRICKS:
        shape = 0 if b is None else brick(*b)
        im, ab, st = E.run(prob, brick_shape=shape)
        g, _ = E.grad(prob, adj, brick_shape=shape)
        if ref is None:
            ref = (im, ab, st, g)
            continue
        np.testing.assert_array_equal(im, ref[0])
        np.testing.assert_array_equal(ab, ref[1])
        np.testing.assert_array_equal(g, ref[3])
        assert st == ref[2]


def test_brick_shape_rejected(E, W):
    from paper_1410_1629_amd.binding import McrtError, brick
    prob = W.small_problem(n=(4, 4, 4), n_packages=10)
    for bad in (brick(8, 0, 0), brick(4, 4, 3), 0x2000, 5):
        with pytest.raises(McrtError):
            E.run(prob, brick_shape=bad)


@pytest.mark.parametrize("prec", [0, 1])
def test_backward_peel_queue_modes(E, orc, W, prec):
    """Peel-ray deposits walked inline, all queued and bundled by tile, or
    queued until a tiny queue is full: same gradient and crossing counts."""
    n = (12, 10, 9)
    prob = W.small_problem(n=n, box=(-1.0, 1.2, -1.0, 1.0, -0.9, 0.9),
                           rho=W.lognormal_density(n, 0.8, seed=41, f32=(prec == 1)), kappa=1.1, albedo=0.65, g=0.4,
                           detectors=[W.frame(10.0, 0.0, 20, 20, 1.2, 1.2), W.frame(10.0, 90.0, 24, 16, 1.3, 1.0),
                                      W.frame(10.0, 55.0, 18, 18, 1.3, 1.3, azim=30.0, pa=15.0)],
                           n_packages=900, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT, precision=prec)
    img_o, _, _ = orc.run(prob)
    adj = np.random.default_rng(8).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(prob, adj)
    ref = None
    for q in (-1, 0, 7, 100000):
        g, st = E.grad(prob, adj, peel_queue=q)
        assert rel_l1(g, g_o) < (1e-9 if prec == 0 else 1e-5), (q, rel_l1(g, g_o))
        if q == -1:
            assert st["x_queue"] == 0 and st["d_queue"] == 0
        else:  # queued rays: an optical-depth walk each, a deposit walk when q != 0
            assert 0 < st["d_queue"] <= st["x_queue"] - st["d_queue"]
            assert st["d_queue"] <= st["deposits"]
        if ref is None:
            ref = (g, st)
            continue
        # FP32 path: inline peel walks keep their times in FP64 (the life
        # kernel's walk), queued ones in FP32, so the modes agree to FP32
        # rounding and a near-tie can merge or split a crossing
        assert rel_l1(g, ref[0]) < (1e-12 if prec == 0 else 1e-6)
        _same_counts(st, ref[1], ("x_path", "x_locate", "deposits", "events", "peels"), prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_forward_peel_queue_modes(E, orc, W, prec):
    """Forward peel rays walked inline, all queued (sorted, walked by the
    queue kernel, added to their pixels), queued until a tiny queue is full,
    and queued per chunk of 97 packages: the oracle's images and tallies and
    the same crossing counts in every mode."""
    n = (11, 9, 8)
    prob = W.small_problem(n=n, rho=W.lognormal_density(n, 0.8, seed=51, f32=(prec == 1)), kappa=1.2, albedo=0.7,
                           g=0.4, detectors=[W.frame(10.0, 0.0, 20, 20, 1.2, 1.2),
                                             W.frame(10.0, 70.0, 16, 24, 1.3, 1.1, azim=20.0)],
                           n_packages=800, precision=prec,
                           flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT | W.FLAG_ABSORB | W.FLAG_SPLIT)
    img_o, abs_o, _ = orc.run(prob)
    tol = 1e-10 if prec == 0 else 1e-5
    ref = None
    for q, chunk in ((-1, 0), (0, 0), (7, 0), (0, 97)):
        try:
            E.set_chunk_items(chunk)
            images, absorbed, st = E.run(prob, peel_queue=q)
        finally:
            E.set_chunk_items(0)
        assert rel_l1(images, img_o) < tol and rel_l1(absorbed, abs_o) < tol, (q, chunk)
        if q == -1:
            assert st["x_queue"] == 0
        else:
            assert 0 < st["x_queue"] <= st["x_peel"] and st["d_queue"] == 0
        assert st["life_launches"] == (1 if chunk == 0 else -(-800 // chunk))
        if ref is None:
            ref = (images, st)
            continue
        assert rel_l1(images, ref[0]) < (1e-12 if prec == 0 else 1e-6)
        _same_counts(st, ref[1], ("x_path", "x_locate", "deposits", "events", "peels", "packages"), prec)


def test_backward_events_beyond_the_job_event_field(E, orc, W):
    """Queued peel rays record their event number in 16 bits: the lane code
    saturates it (any event past the scratch's kept events is "beyond"), and
    the harness rejects a stored number past the saturation value.
    Packages with 70000 scatterings (pure scattering, no weight cut-off)
    with every ray queued give the oracle's gradient."""
    prob = W.small_problem(n=(3, 3, 3), kappa=4.0, albedo=1.0, g=0.3, w_min=0.0, max_scatter=70000, n_packages=2,
                           detectors=[W.frame(10.0, 30.0, 6, 6, 1.2, 1.2)],
                           flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    img_o, _, st_o = orc.run(prob)
    assert st_o["events"] == 2 * 70000
    adj = np.random.default_rng(9).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(prob, adj)
    for q in (-1, 150000):  # a queue that holds every ray
        g, st = E.grad(prob, adj, peel_queue=q)
        assert rel_l1(g, g_o) < 1e-9, (q, rel_l1(g, g_o))
        assert (st["x_queue"] == 0) == (q == -1)


@pytest.mark.parametrize("kept", [0, 1, 3, 32])
def test_backward_event_scratch_sizes(E, orc, W, kept):
    """Pass B reads G_e and T of the first `kept` events from the scratch and
    walks the rest again: the gradient does not depend on how many are kept,
    and no scratch entry is read before pass A wrote it."""
    n = (9, 8, 7)
    prob = W.small_problem(n=n, rho=W.lognormal_density(n, 0.9, seed=43), kappa=1.4, albedo=0.8, g=0.3,
                           detectors=[W.frame(10.0, 20.0, 16, 16, 1.1, 1.1), W.frame(10.0, 75.0, 12, 20, 1.2, 1.2)],
                           n_packages=700, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT, w_min=1e-5, max_scatter=40)
    img_o, _, _ = orc.run(prob)
    adj = np.random.default_rng(3).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(prob, adj)
    try:
        E.set_events_kept(kept)
        g, st = E.grad(prob, adj)
        g1, _ = E.grad(dict(prob, flags=W.FLAG_PEEL_SCAT), adj)  # no peel-off at emission
    finally:
        E.set_events_kept(32)
    g1_o, _, _ = orc.grad(dict(prob, flags=W.FLAG_PEEL_SCAT), adj)
    assert rel_l1(g, g_o) < 1e-9, rel_l1(g, g_o)
    assert rel_l1(g1, g1_o) < 1e-9, rel_l1(g1, g1_o)


@pytest.mark.parametrize("queue", [-1, 0, 50])
def test_backward_in_chunks(E, orc, W, queue):
    """The adjoint runs on chunks of packages (pass A, peel jobs, pass B per
    chunk): chunks of 97 packages, with and without the peel-job queue, give
    the unchunked gradient and the oracle's."""
    n = (9, 9, 8)
    prob = W.small_problem(n=n, rho=W.lognormal_density(n, 0.7, seed=47), kappa=1.2, albedo=0.7, g=0.5,
                           detectors=[W.frame(10.0, 25.0, 18, 18, 1.2, 1.2), W.frame(10.0, 80.0, 14, 16, 1.2, 1.2)],
                           n_packages=700, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT | W.FLAG_SPLIT)
    img_o, _, _ = orc.run(prob)
    adj = np.random.default_rng(4).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(prob, adj)
    g_full, st_full = E.grad(prob, adj, peel_queue=queue)
    try:
        E.set_chunk_items(97)
        g, st = E.grad(prob, adj, peel_queue=queue)
    finally:
        E.set_chunk_items(0)
    assert rel_l1(g, g_o) < 1e-9 and rel_l1(g_full, g_o) < 1e-9
    assert rel_l1(g, g_full) < 1e-12
    for key in ("x_path", "x_locate", "x_peel", "deposits", "events", "packages", "peels"):
        assert st[key] == st_full[key], key
    assert st_full["life_launches"] == 2 and st["life_launches"] == 2 * -(-700 // 97)


@pytest.mark.parametrize("queue", [-1, 0])
@pytest.mark.parametrize("prec", [0, 1])
def test_max_chunk_forward_and_adjoint(E, orc, W, prec, queue):
    """mcrt_opts.max_chunk: 2 wavelengths x 401 packages in chunks of at most
    150 items (some straddle the wavelengths) give the oracle's images,
    tallies and gradients (density, optics, luminosities, absorbed-tally
    term) and the single chunk's results and counts."""
    n = (8, 7, 6)
    prob = W.small_problem(n=n, rho=W.lognormal_density(n, 0.8, seed=61, f32=(prec == 1)), kappa=[0.9, 1.4],
                           albedo=[0.7, 0.55], g=[0.4, -0.2],
                           sources=[W.point((0.11, -0.07, 0.05), [1.0, 0.5]), W.expdisk(0.4, 0.15, [2.0, 1.0])],
                           detectors=[W.frame(10.0, 0.0, 12, 12, 1.2, 1.2), W.frame(10.0, 75.0, 10, 14, 1.3, 1.1,
                                                                                   azim=20.0)],
                           n_packages=401, precision=prec,
                           flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT | W.FLAG_ABSORB | W.FLAG_SPLIT)
    img_o, abs_o, _ = orc.run(prob)
    tol = 1e-10 if prec == 0 else 1e-5
    im, ab, st = E.run(prob, peel_queue=queue, max_chunk=150)
    assert st["life_launches"] == 6
    assert rel_l1(im, img_o) < tol and rel_l1(ab, abs_o) < tol
    im1, ab1, st1 = E.run(prob, peel_queue=queue)
    assert rel_l1(im, im1) < 1e-12 and rel_l1(ab, ab1) < 1e-12
    for key in ("x_path", "x_locate", "x_peel", "deposits", "events", "peels", "packages"):
        assert st[key] == st1[key], key
    rng = np.random.default_rng(21)
    adj = rng.standard_normal(img_o.shape)
    adj_abs = rng.standard_normal(abs_o.shape) * 10.0
    g_o, _, _, go = orc.grad(prob, adj, optics=True, adj_absorbed=adj_abs)
    g, st, gopt = E.grad(prob, adj, optics=True, adj_absorbed=adj_abs, peel_queue=queue, max_chunk=150)
    assert st["life_launches"] == 12
    tol_g = 1e-9 if prec == 0 else 1e-5
    assert rel_l1(g, g_o) < tol_g
    for k in ("albedo", "g", "lum"):
        assert rel_l1(gopt[k], go[k]) < tol_g, k
    g1, _, gopt1 = E.grad(prob, adj, optics=True, adj_absorbed=adj_abs, peel_queue=queue)
    assert rel_l1(g, g1) < 1e-12
    for k in ("albedo", "g", "lum"):
        assert rel_l1(gopt[k], gopt1[k]) < 1e-12, k
