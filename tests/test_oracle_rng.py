"""Pins of the oracle's counter-based random numbers (Philox4x32-10) and of
the uniform deviates built from them."""
import os
import subprocess

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
HELPER = os.path.join(os.path.dirname(__file__), "helpers", "torch_philox.cpp")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat_rows())
def test_philox_known_answers(orc, ctr, key, out):
    assert orc.philox(ctr, key).tolist() == out


@pytest.fixture(scope="module")
def torch_philox(tmp_path_factory):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    exe = str(tmp_path_factory.mktemp("tp") / "torch_philox")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I" + inc, HELPER, "-o", exe], check=True)
    return exe


def test_philox_matches_pytorch_engine(orc, torch_philox):
    rng = np.random.default_rng(11)
    rows = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    rows[:50, 1] = 0       # small package indices as used in practice
    rows[50:100, 3] = 0xFFFFFFFF
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    res = subprocess.run([torch_philox], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(x) for x in line.split()] for line in res.stdout.strip().splitlines()], dtype=np.uint64)
    got = np.array([orc.philox(r[0:4], r[4:6]) for r in rows], dtype=np.uint64)
    np.testing.assert_array_equal(got, ref)


def test_draw_schedule_is_counter_layout(orc):
    # draw(p, l, c) is the block cipher of counter (p_lo, p_hi, l, c) under key (seed_lo, seed_hi)
    seed, p, lam, c = (1 << 40) + 4357, (3 << 32) + 17, 5, 9
    words = orc.draw_words(seed, p, 1, lam, c)[0]
    direct = orc.philox([p & 0xFFFFFFFF, p >> 32, lam, c], [seed & 0xFFFFFFFF, seed >> 32])
    np.testing.assert_array_equal(words, direct)


def test_uniform_open_interval_and_resolution(orc):
    assert orc.uniform(0) == 0.5 / 2**32
    assert orc.uniform(2**32 - 1) == 1.0 - 0.5 / 2**32
    assert 0.0 < orc.uniform(0) < orc.uniform(1) < orc.uniform(2**32 - 1) < 1.0


def test_uniform_words_are_uniform(orc):
    # chi-square over 256 bins per word position, and mean / variance of the
    # uniforms, on 2e5 packages; independence across word positions by the
    # correlation coefficient.
    w = orc.draw_words(4357, 0, 200_000, 0, 2).astype(np.float64)
    u = (w + 0.5) / 2**32
    n = u.shape[0]
    for j in range(4):
        h = np.bincount((w[:, j] // 2**24).astype(np.int64), minlength=256)
        chi2 = ((h - n / 256) ** 2 / (n / 256)).sum()
        assert 180 < chi2 < 340, chi2  # 255 dof, about 4.5 sigma
        assert abs(u[:, j].mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
        assert abs(u[:, j].var() - 1 / 12) < 5 * 0.075 / np.sqrt(n)
    c = np.corrcoef(u.T)
    assert np.all(np.abs(c - np.eye(4)) < 5 / np.sqrt(n))


def test_distinct_streams(orc):
    # different packages, wavelengths, draws and keys give different words
    a = orc.draw_words(4357, 0, 1000, 0, 0)
    b = orc.draw_words(4357, 0, 1000, 1, 0)
    c = orc.draw_words(4357, 0, 1000, 0, 1)
    d = orc.draw_words(4358, 0, 1000, 0, 0)
    for x in (b, c, d):
        assert np.mean(a == x) < 0.01
    assert len(np.unique(a[:, 0])) > 990
