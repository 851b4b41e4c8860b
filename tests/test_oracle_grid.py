"""Pins of the oracle's levels, temporal tree, restriction and prolongation.

The pins come from the paper (Sec. 3 Fig. 1, Sec. 4 Table 1 and the subset
sizes of the experiments, stored under tests/golden/) and from closed forms
and brute force.
"""

import os

import numpy as np
import pytest

from oracle import level_extents, temporal_sets, restrict, prolong

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def _ext(s):
    return tuple(int(v) for v in s.split("x"))


def test_table1_grid_progression():
    for row in _lines("table1_grids.txt"):
        finest, levels = _ext(row[1]), int(row[2])
        expected = [_ext(s) for s in row[3:]]
        assert level_extents(finest, levels) == expected


def test_fig1_temporal_tree():
    for row in _lines("fig1_temporal_tree.txt"):
        if row[0] == "size":
            n, nt, q, size = map(int, row[1:])
            assert len(temporal_sets(n, nt)[q]) == size
        else:
            n, nt, q = map(int, row[:3])
            frames = [int(v) - 1 for v in row[3:]]       # to 0-based
            assert temporal_sets(n, nt)[q] == frames


def test_temporal_tree_properties():
    for n in (2, 3, 8, 9, 17, 33, 64, 100, 129):
        for nt in (1, 2, 3, 4):
            K = temporal_sets(n, nt)
            assert K[-1] == list(range(n))
            for a, b in zip(K[:-1], K[1:]):
                assert set(a) <= set(b)
                assert a[0] == 0 and a[-1] == n - 1
    assert temporal_sets(8, 2)[0] == [0, 2, 4, 6, 7]
    assert [len(k) for k in temporal_sets(64, 3)] == [17, 33, 64]


def _restrict_brute(img):
    n = img.shape[0]
    fine = img.shape[1:]
    coarse = tuple((m + 1) // 2 for m in fine)
    out = np.zeros((n,) + coarse)
    for t in range(n):
        for I in np.ndindex(*coarse):
            vals = []
            for off in np.ndindex(*([2] * len(fine))):
                idx = tuple(2 * I[a] + off[a] for a in range(len(fine)))
                if all(idx[a] < fine[a] for a in range(len(fine))):
                    vals.append(img[(t,) + idx])
            out[(t,) + I] = sum(vals) / len(vals)
    return out


@pytest.mark.parametrize("shape", [(2, 5, 7), (1, 4, 6), (2, 3, 5, 4),
                                   (1, 1, 3), (1, 7, 1, 2)])
def test_restrict_brute_force(shape):
    rng = np.random.default_rng(1)
    img = rng.standard_normal(shape)
    np.testing.assert_allclose(restrict(img), _restrict_brute(img),
                               rtol=0, atol=1e-14)


def test_restrict_constants_and_mean():
    img = np.full((3, 6, 10), 0.7)
    np.testing.assert_array_equal(restrict(img), np.full((3, 3, 5), 0.7))
    rng = np.random.default_rng(2)
    img = rng.standard_normal((2, 8, 12, 6))
    c = restrict(img)
    np.testing.assert_allclose(c.mean(axis=(1, 2, 3)), img.mean(axis=(1, 2, 3)),
                               atol=1e-14)


def test_prolong_constants_and_linear():
    np.testing.assert_array_equal(prolong(np.full((2, 4, 5), 3.0), (8, 10)),
                                  np.full((2, 8, 10), 3.0))
    # a linear function of the coarse cell centres is reproduced at fine
    # centres that lie inside the coarse centre hull (no clamping)
    Mc = (6, 7)
    yc = (np.arange(Mc[0]) + 0.5) * 2.0
    xc = (np.arange(Mc[1]) + 0.5) * 2.0
    f = lambda y, x: 0.3 * y - 1.7 * x + 2.0
    coarse = f(yc[:, None], xc[None, :])
    fine_ext = (12, 14)
    fine = prolong(coarse, fine_ext)
    yf = np.arange(12) + 0.5
    xf = np.arange(14) + 0.5
    exact = f(yf[:, None], xf[None, :])
    np.testing.assert_allclose(fine[1:-1, 1:-1], exact[1:-1, 1:-1], atol=1e-12)


def test_prolong_weights_even():
    # a coarse delta at cell 2 spreads 3/4 to fine cells 4, 5 and 1/4 to 3, 6
    coarse = np.zeros(6)
    coarse[2] = 1.0
    fine = prolong(coarse, (12,))
    expect = np.zeros(12)
    expect[[4, 5]] = 0.75
    expect[[3, 6]] = 0.25
    np.testing.assert_allclose(fine, expect, atol=1e-15)


def test_prolong_odd_extent_clamps():
    coarse = np.arange(3, dtype=float)          # fine extent 5 -> 3 coarse
    fine = prolong(coarse, (5,))
    # fine i sits at coarse coordinate i/2 - 1/4, clamped to [0, 2]
    p = np.clip(np.arange(5) / 2 - 0.25, 0, 2)
    np.testing.assert_allclose(fine, p, atol=1e-15)
