"""The adjoint tape (mcrt_opts.tape) on the CPU harness: a forward run keeps
T per leg and C per peel ray, and the adjoint that reads them -- one replay
per package, no optical-depth walks -- gives the oracle's gradients and the
replay-only adjoint's, in every queue mode, with chunkings that differ
between the forward run and the adjoint, with the optics and luminosity
gradients, for every grid kind and instrument kind; a tape recorded with
other arguments is rejected; runs that could exceed the tape's events keep
none; a forward run that overflowed its tape, and a loss on the absorbed
tally, make the adjoint replay without it."""
import numpy as np
import pytest

from paper_1410_1629_amd import binding as B


def rel_l1(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a).sum())


def _problem(W, prec, n_packages=1200, **kw):
    n = (9, 8, 7)
    args = dict(n=n, rho=W.lognormal_density(n, 0.8, seed=31, f32=(prec == 1)), kappa=[1.2, 0.7], albedo=[0.7, 0.5],
                g=[0.45, -0.1], sources=[W.point((0.13, -0.21, 0.07), [1.0, 0.6]), W.expdisk(0.4, 0.15, [0.5, 1.5])],
                detectors=[W.frame(10.0, 30.0, 18, 18, 1.0, 1.0, azim=20.0), W.frame(10.0, 90.0, 12, 12, 1.2, 1.2)],
                n_packages=n_packages, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT, w_min=1e-3, max_scatter=50,
                precision=prec)
    args.update(kw)
    return W.small_problem(**args)


def test_tape_size_follows_the_event_bound(W):
    prob = _problem(W, 0)
    # largest albedo 0.7, w_min 1e-3: ln(1e-3) / ln(0.7) = 19.4, so events 0 .. 21
    ev = 2 + int(np.floor(np.log(1e-3) / np.log(0.7))) + 1
    items = 2 * 1200
    doubles = items * ev * 3
    expect = 256 + ((8 * doubles + 255) // 256) * 256 + 4 * items * ev * 2
    assert B.tape_bytes(prob) == expect
    assert B.tape_bytes(dict(prob, max_scatter=5)) == 256 + ((8 * items * 6 * 3 + 255) // 256) * 256 + 4 * items * 6 * 2
    # albedo 1 or w_min 0: only max_scatter bounds the events (max_scatter + 1 of them, at most 64)
    assert B.tape_bytes(dict(prob, albedo=[1.0, 0.5], max_scatter=1000)) == 0
    assert B.tape_bytes(dict(prob, w_min=0.0, max_scatter=1000)) == 0
    assert B.tape_bytes(dict(prob, w_min=0.0, max_scatter=63)) > 0
    assert B.tape_bytes(dict(prob, w_min=0.0, max_scatter=64)) == 0
    # no peel-off, no frame: nothing to record
    assert B.tape_bytes(dict(prob, flags=W.FLAG_ABSORB)) == 0
    assert B.tape_bytes(dict(prob, detectors=[])) == 0


@pytest.mark.parametrize("prec", [0, 1])
def test_tape_adjoint_matches_the_oracle_in_every_mode(E, orc, W, prec):
    prob = _problem(W, prec)
    img_o, _, _ = orc.run(prob)
    adj = np.random.default_rng(5).standard_normal(img_o.shape)
    g_o, _, _, go = orc.grad(prob, adj, optics=True)
    tol = 1e-9 if prec == 0 else 1e-5
    for fq, fchunk in ((0, 0), (-1, 700)):
        tape = E.new_tape(prob)
        img, _, _ = E.run(prob, tape=tape, peel_queue=fq, max_chunk=fchunk)
        assert rel_l1(img, img_o) < (1e-10 if prec == 0 else 1e-5)
        for q in (-1, 0, 40):
            for chunk in (0, 500):
                g, st, gopt = E.grad(prob, adj, optics=True, tape=tape, peel_queue=q, max_chunk=chunk)
                assert rel_l1(g, g_o) < tol, (fq, fchunk, q, chunk, rel_l1(g, g_o))
                for k in ("albedo", "g", "lum"):
                    assert rel_l1(gopt[k], go[k]) < tol, k
                n_chunks = -(-2 * 1200 // chunk) if chunk else 1
                assert st["life_launches"] == n_chunks  # one replay per package
                g_r, st_r, _ = E.grad(prob, adj, optics=True, peel_queue=q, max_chunk=chunk)
                assert st_r["life_launches"] == 2 * n_chunks
                # the same gradient as the replay-only adjoint, without its optical-depth walks
                assert rel_l1(g, g_r) < (1e-12 if prec == 0 else 1e-6)
                assert st["x_locate"] == st_r["x_locate"] // 2


@pytest.mark.parametrize("kind", ["rect", "tree", "instruments"])
def test_tape_adjoint_on_other_grids_and_instruments(E, orc, W, kind):
    from test_oracle_rectilinear import random_planes
    from test_oracle_tree import BOX, kd_tree
    prob = _problem(W, 0, n_packages=800)
    if kind == "rect":
        rng = np.random.default_rng(4)
        prob["planes"] = tuple(random_planes(prob["box"][2 * a], prob["box"][2 * a + 1], prob["n"][a], rng)
                               for a in range(3))
    elif kind == "tree":
        T = kd_tree(W)
        prob = dict(prob, box=BOX, n=(T.n_cells, 1, 1), tree=T.tree(),
                    rho=np.random.default_rng(7).lognormal(0.0, 0.8, T.n_cells))
    else:
        prob["detectors"] = [prob["detectors"][0], W.sed(10.0, 45.0),
                             W.perspective((0.3, -0.2, 0.1), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 12, 10, 1.0, 0.8)]
    img_o, _, _ = orc.run(prob)
    adj = np.random.default_rng(6).standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(prob, adj)
    tape = E.new_tape(prob)
    E.run(prob, tape=tape)
    g, st = E.grad(prob, adj, tape=tape)
    assert rel_l1(g, g_o) < 1e-9
    assert st["life_launches"] == 1


def test_tape_from_other_arguments_is_rejected(E, W):
    prob = _problem(W, 0, n_packages=300)
    tape = E.new_tape(prob)
    E.run(prob, tape=tape)
    adj = np.ones(B.image_shape(prob))
    for change in (dict(seed=99), dict(n_packages=301), dict(first_package=5), dict(g=[0.45, -0.11]),
                   dict(detectors=[W.frame(10.0, 31.0, 18, 18, 1.0, 1.0, azim=20.0),
                                   W.frame(10.0, 90.0, 12, 12, 1.2, 1.2)])):
        other = dict(prob, **change)
        t = tape if B.tape_bytes(other) <= tape.size else np.zeros(B.tape_bytes(other), np.uint8)
        with pytest.raises(B.McrtError) as ei:
            E.grad(other, adj, tape=t)
        assert ei.value.code == B.EINVAL, change
    blank = np.zeros_like(tape)  # never written by a forward run
    with pytest.raises(B.McrtError):
        E.grad(prob, adj, tape=blank)
    with pytest.raises(B.McrtError):  # a run that cannot keep a tape
        E.run(dict(prob, albedo=[1.0, 0.5], max_scatter=1000), tape=tape)


def test_overflowed_tape_and_absorbed_loss_replay_without_it(E, orc, W):
    prob = _problem(W, 0, n_packages=400, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT | W.FLAG_ABSORB)
    img_o, abs_o, _ = orc.run(prob)
    rng = np.random.default_rng(9)
    adj = rng.standard_normal(img_o.shape)
    g_o, _, _ = orc.grad(prob, adj)
    tape = E.new_tape(prob)
    E.run(prob, tape=tape)
    over = tape.copy()
    over[32:36] = np.frombuffer(np.uint32(1).tobytes(), np.uint8)  # the header's overflow word
    g, st = E.grad(prob, adj, tape=over)
    assert rel_l1(g, g_o) < 1e-9 and st["life_launches"] == 2
    adj_abs = rng.standard_normal(abs_o.shape)
    g_oa, _, _ = orc.grad(prob, adj, adj_absorbed=adj_abs)
    g, st = E.grad(prob, adj, adj_absorbed=adj_abs, tape=tape)
    assert rel_l1(g, g_oa) < 1e-9 and st["life_launches"] == 2
