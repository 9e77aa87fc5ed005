"""Pins of the oracle's grid traversal against closed forms and brute force."""
import numpy as np
import pytest

BOX = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)


def slab(box, o, k):
    """Entry and exit parameters of rays o + t k (t >= 0) in the box, by the
    slab method written out in numpy (t_in = t_out = 0 for a miss)."""
    lo = np.array(box[0::2])
    hi = np.array(box[1::2])
    with np.errstate(divide="ignore", invalid="ignore"):
        ta = (lo - o) / k
        tb = (hi - o) / k
    tn = np.where(k == 0, np.where((o >= lo) & (o < hi), -np.inf, np.inf), np.minimum(ta, tb))
    tf = np.where(k == 0, np.where((o >= lo) & (o < hi), np.inf, -np.inf), np.maximum(ta, tb))
    tin = np.maximum(tn.max(axis=1), 0.0)
    tout = tf.min(axis=1)
    hit = tin < tout
    return np.where(hit, tin, 0.0), np.where(hit, tout, 0.0), hit


@pytest.mark.parametrize("n", [(32, 32, 32), (7, 5, 3), (1, 1, 1), (64, 3, 17)])
def test_uniform_medium_tau_is_chord_length(orc, W, n):
    o, k = W.random_rays(4000, BOX, seed=1)
    rho = np.full(n[::-1], 1.0)
    tau, tot, cell, length, nseg = orc.trace(BOX, n, rho, 1.0, o, k, max_seg=256)
    tin, tout, hit = slab(BOX, o, k)
    np.testing.assert_allclose(tau, tout - tin, rtol=1e-13, atol=1e-13)
    # the segment lengths add up to the chord
    lsum = np.array([length[q, :nseg[q]].sum() for q in range(len(o))])
    np.testing.assert_allclose(lsum, tout - tin, rtol=1e-13, atol=1e-13)
    assert np.all(length[np.arange(256)[None, :] < nseg[:, None]] > 0)
    assert tot == nseg.sum()


def test_tau_from_centre_of_unit_cube(orc, W):
    # kappa*rho = 1 on [-1,1]^3: tau from the centre is 1 / max|k_i|; from an
    # interior point r it is min_i((k_i > 0 ? 1 - r_i : 1 + r_i) / |k_i|).
    rng = np.random.default_rng(3)
    k = rng.standard_normal((2000, 3))
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    n = (32, 32, 32)
    rho = np.ones(n)
    tau, *_ = orc.trace(BOX, n, rho, 1.0, np.zeros_like(k), k)
    np.testing.assert_allclose(tau, 1.0 / np.abs(k).max(axis=1), rtol=1e-14)
    r = rng.uniform(-1, 1, size=(2000, 3))
    tau, *_ = orc.trace(BOX, n, rho, 2.5, r, k)
    d = np.where(k > 0, 1 - r, 1 + r) / np.abs(k)
    np.testing.assert_allclose(tau, 2.5 * d.min(axis=1), rtol=1e-13)


def test_density_varying_along_x_only(orc, W):
    # rho depends on the x column only: tau = sum_i rho_i * (time spent in slab i)
    n = (12, 5, 7)
    rng = np.random.default_rng(5)
    col = rng.uniform(0.1, 3.0, n[0])
    rho = np.broadcast_to(col[None, None, :], (n[2], n[1], n[0])).copy()
    o, k = W.random_rays(3000, BOX, seed=7)
    tau, *_ = orc.trace(BOX, n, rho, 1.3, o, k)
    tin, tout, hit = slab(BOX, o, k)
    xs = np.linspace(-1, 1, n[0] + 1)
    expect = np.zeros(len(o))
    for q in range(len(o)):
        if not hit[q]:
            continue
        if k[q, 0] == 0.0:
            i = min(int(np.floor((o[q, 0] + 1) / (2 / n[0]))), n[0] - 1)
            expect[q] = col[i] * (tout[q] - tin[q])
            continue
        ta = (xs[:-1] - o[q, 0]) / k[q, 0]
        tb = (xs[1:] - o[q, 0]) / k[q, 0]
        a, b = np.minimum(ta, tb), np.maximum(ta, tb)
        ov = np.clip(np.minimum(b, tout[q]) - np.maximum(a, tin[q]), 0, None)
        expect[q] = (col * ov).sum()
    np.testing.assert_allclose(1.3 * expect, tau, rtol=1e-12, atol=1e-13)


def test_axis_parallel_rays_cross_whole_cells(orc):
    n = (8, 8, 8)
    rho = np.arange(512, dtype=np.float64).reshape(8, 8, 8) + 1
    d = 2.0 / 8
    # from the centre of cell (2,3,4) along +x: half a cell, then whole cells
    o = np.array([[-1 + 2.5 * d, -1 + 3.5 * d, -1 + 4.5 * d]])
    k = np.array([[1.0, 0.0, 0.0]])
    tau, tot, cell, length, nseg = orc.trace((-1, 1, -1, 1, -1, 1), n, rho, 1.0, o, k, max_seg=16)
    assert nseg[0] == 6
    np.testing.assert_array_equal(cell[0, :6], [2 + 8 * (3 + 8 * 4) + i for i in range(6)])
    np.testing.assert_allclose(length[0, :6], [d / 2] + [d] * 5, rtol=1e-14)
    # along -z from the same point
    tau, tot, cell, length, nseg = orc.trace((-1, 1, -1, 1, -1, 1), n, rho, 1.0, o, -k[:, [2, 1, 0]], max_seg=16)
    assert nseg[0] == 5
    np.testing.assert_array_equal(cell[0, :5], [2 + 8 * (3 + 8 * (4 - i)) for i in range(5)])


def test_wall_conventions(orc):
    n = (4, 4, 4)
    rho = np.ones(n)
    d = 0.5
    # a point exactly on the wall x = 0 moving towards -x starts in cell i = 1
    o = np.array([[0.0, 0.1, 0.1]])
    tau, tot, cell, length, nseg = orc.trace(BOX, n, rho, 1.0, o, np.array([[-1.0, 0.0, 0.0]]), max_seg=8)
    assert cell[0, 0] % 4 == 1 and nseg[0] == 2
    np.testing.assert_allclose(length[0, :2], [d, d])
    # moving towards +x it starts in cell i = 2
    tau, tot, cell, length, nseg = orc.trace(BOX, n, rho, 1.0, o, np.array([[1.0, 0.0, 0.0]]), max_seg=8)
    assert cell[0, 0] % 4 == 2 and nseg[0] == 2
    # a ray lying in the plane y = 0 belongs to the +y cells (j = 2)
    tau, tot, cell, length, nseg = orc.trace(BOX, n, rho, 1.0, np.array([[-1.0, 0.0, 0.1]]),
                                             np.array([[1.0, 0.0, 0.0]]), max_seg=8)
    assert nseg[0] == 4 and all((c // 4) % 4 == 2 for c in cell[0, :4])
    # a ray in the upper face plane y = 1 misses (half-open cells); y = -1 hits
    tau, *_ = orc.trace(BOX, n, rho, 1.0, np.array([[-2.0, 1.0, 0.1], [-2.0, -1.0, 0.1]]),
                        np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]]))
    np.testing.assert_allclose(tau, [0.0, 2.0])


def test_diagonal_ties_advance_together(orc):
    # a ray from a vertex along (1,1,1) crosses only the diagonal cells, each
    # with length sqrt(3) * cell size: tied axes advance together.
    n = (8, 8, 8)
    rho = np.ones(n)
    k = np.array([[1.0, 1.0, 1.0]]) / np.sqrt(3.0)
    tau, tot, cell, length, nseg = orc.trace(BOX, n, rho, 1.0, np.array([[-1.0, -1.0, -1.0]]), k, max_seg=32)
    assert nseg[0] == 8
    np.testing.assert_array_equal(cell[0, :8], [i * (1 + 8 + 64) for i in range(8)])
    np.testing.assert_allclose(length[0, :8], np.sqrt(3.0) * 0.25, rtol=1e-14)


def test_rays_missing_or_leaving(orc):
    n = (4, 4, 4)
    rho = np.ones(n)
    o = np.array([[2.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    k = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    tau, tot, cell, length, nseg = orc.trace(BOX, n, rho, 1.0, o, k, max_seg=8)
    np.testing.assert_allclose(tau, [0.0, 0.0, 1.0, 0.0])
    np.testing.assert_array_equal(nseg, [0, 0, 2, 0])


def test_brute_force_sampling_of_random_medium(orc, W):
    # midpoint sampling of kappa*rho along the ray agrees with the segment sum
    n = (9, 6, 5)
    box = (-2.0, 1.0, 0.0, 3.0, -1.0, 0.5)
    rho = W.lognormal_density(n, 1.0, seed=9)
    o, k = W.random_rays(40, box, seed=13)
    tau, *_ = orc.trace(box, n, rho, 0.7, o, k)
    tin, tout, hit = slab(box, o, k)
    lo = np.array(box[0::2])
    d = (np.array(box[1::2]) - lo) / np.array(n)
    m = 200_000
    for q in range(len(o)):
        if not hit[q]:
            assert tau[q] == 0.0
            continue
        t = tin[q] + (np.arange(m) + 0.5) * (tout[q] - tin[q]) / m
        p = o[q][None, :] + t[:, None] * k[q][None, :]
        idx = np.clip(np.floor((p - lo) / d).astype(int), 0, np.array(n) - 1)
        vals = rho[idx[:, 2], idx[:, 1], idx[:, 0]]
        est = 0.7 * vals.sum() * (tout[q] - tin[q]) / m
        assert abs(est - tau[q]) <= 2e-4 * max(tau[q], 1e-3), (q, est, tau[q])
