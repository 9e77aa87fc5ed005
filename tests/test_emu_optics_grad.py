"""The library's gradients with respect to the albedo, g and the source
luminosities (and the densities in the same replay), run on the CPU by the
bounds-checked harness of its lane code, against the FP64 oracle: regular
and tree grids, frames, SED instruments and cameras, point, disk and cell
sources, with the peel rays queued and walked inline, and with few events
kept in the event scratch so that pass B walks the later events again."""
import numpy as np
import pytest

from test_oracle_optics_grad import _problem
from test_oracle_tree import _blob, kd_tree


def rel_l1(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a).sum())


def problems(W, name, prec=0):
    if name == "mixed":
        p = _problem(W, n_packages=500)
    elif name == "tree":
        T = kd_tree(W, max_mass=0.05, depth=10)
        p = W.tree_problem("tree", (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0), T, _blob, [1.3, 0.8], [0.7, 0.5], [0.4, 0.1],
                           [W.point((0.11, -0.07, 0.05), lum=[1.0, 0.5]), W.point((-0.3, 0.2, 0.1), lum=[0.2, 0.9])],
                           [W.frame(10.0, 0.0, 12, 12, 1.2, 1.2), W.sed(10.0, 60.0)], 500, prec,
                           flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    else:  # cells plus a point source
        n = (6, 5, 4)
        ncell = 120
        lum = np.random.default_rng(21).lognormal(0.0, 1.0, (2, ncell))
        p = W.small_problem(n=n, rho=W.lognormal_density(n, 0.6, seed=5), kappa=[1.1, 0.7], albedo=[0.6, 0.3],
                            g=[0.5, 0.2], sources=[W.cells(lum), W.point((0.2, 0.1, -0.1), lum=[3.0, 1.0])],
                            detectors=[W.frame(10.0, 40.0, 10, 10, 1.3, 1.3)], n_packages=500,
                            flags=W.FLAG_PEEL_EMIT | W.FLAG_PEEL_SCAT)
    p["precision"] = prec
    if prec and name != "tree":
        p["rho"] = W.as_f32_values(p["rho"])
    return p


@pytest.mark.parametrize("name", ["mixed", "tree", "cells"])
@pytest.mark.parametrize("prec", [0, 1])
def test_optics_gradients_match_oracle(E, orc, W, name, prec):
    p = problems(W, name, prec)
    img_o, _, _ = orc.run(p)
    adj = np.random.default_rng(8).standard_normal(img_o.shape)
    g_o, _, _, go = orc.grad(p, adj, optics=True)
    tol = 1e-9 if prec == 0 else 1e-5
    for queue in (-1, 0):
        g, _, ge = E.grad(p, adj, optics=True, peel_queue=queue)
        assert rel_l1(g, g_o) < tol, queue
        for key in ("albedo", "g", "lum"):
            assert rel_l1(ge[key], go[key]) < tol, (queue, key, ge[key], go[key])
    assert np.all(go["albedo"] != 0) and np.all(go["g"] != 0)


def test_optics_gradients_with_few_kept_events(E, orc, W):
    # pass B walks the peel rays of events past the scratch again
    p = problems(W, "mixed")
    img_o, _, _ = orc.run(p)
    adj = np.random.default_rng(9).standard_normal(img_o.shape)
    g_o, _, _, go = orc.grad(p, adj, optics=True)
    E.set_events_kept(2)
    E.set_chunk_items(300)
    try:
        g, _, ge = E.grad(p, adj, optics=True)
    finally:
        E.set_events_kept(32)
        E.set_chunk_items(0)
    assert rel_l1(g, g_o) < 1e-9
    for key in ("albedo", "g", "lum"):
        assert rel_l1(ge[key], go[key]) < 1e-9, key
