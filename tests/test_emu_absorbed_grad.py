"""The library's gradient of a loss on the absorbed tally (with and without
an image term) in the bounds-checked CPU harness of its lane code, against
the FP64 oracle: regular, rectilinear and tree grids, both precisions, the
peel rays queued and walked inline, and few events kept in the scratch (so
that pass B walks the later paths twice: once for their B, once to
deposit)."""
import numpy as np
import pytest

from test_emu_instruments import problem


def rel_l1(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a).sum())


def _setup(W, orc, grid, prec, n_packages=400, image_term=True):
    p = problem(W, grid, prec, n_packages=n_packages, flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT | W.FLAG_ABSORB)
    img, A, _ = orc.run(p)
    rng = np.random.default_rng(12)
    a = rng.standard_normal(img.shape) if image_term else np.zeros(img.shape)
    b = rng.standard_normal(A.shape)
    return p, a, b


@pytest.mark.parametrize("grid", ["regular", "rect", "tree"])
@pytest.mark.parametrize("prec", [0, 1])
def test_absorbed_gradient_matches_oracle(E, orc, W, grid, prec):
    p, a, b = _setup(W, orc, grid, prec)
    g_o, _, _ = orc.grad(p, a, adj_absorbed=b)
    tol = 1e-9 if prec == 0 else 1e-5
    for queue in (-1, 0):
        g, _ = E.grad(p, a, adj_absorbed=b, peel_queue=queue)
        assert rel_l1(g, g_o) < tol, queue


def test_absorbed_gradient_alone_and_with_few_kept_events(E, orc, W):
    p, a, b = _setup(W, orc, "regular", 0, image_term=False)
    g_o, _, _ = orc.grad(p, a, adj_absorbed=b)
    E.set_events_kept(2)
    E.set_chunk_items(150)
    try:
        g, _ = E.grad(p, a, adj_absorbed=b)
    finally:
        E.set_events_kept(32)
        E.set_chunk_items(0)
    assert rel_l1(g, g_o) < 1e-9
    assert np.abs(g_o).max() > 0
