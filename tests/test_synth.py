"""The synthetic input generator (host code shared by both sides)."""

import time

import numpy as np

from paper_2001_06613_amd import synth


def test_band_edges_small_heights_terminate_and_keep_min_thickness():
    # heights where rejection sampling would never (24) or hardly ever
    # (25..37) accept
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    for H in range(24, 80):
        for _ in range(20):
            b = synth.band_edges(rng, H)
            gaps = np.diff(np.concatenate([[0.0], b, [float(H)]]))
            assert gaps.min() >= 3 - 1e-9
            assert abs(gaps.sum() - H) < 1e-9
    assert time.perf_counter() - t0 < 20.0


def test_band_edges_direct_draw_has_the_conditioned_mean():
    # every gap of the conditioned uniform spacings has mean H / n_bands
    rng = np.random.default_rng(1)
    H = 30
    gaps = np.array([np.diff(np.concatenate([[0.0], synth.band_edges(rng, H),
                                             [float(H)]]))
                     for _ in range(4000)])
    np.testing.assert_allclose(gaps.mean(axis=0), H / 8, rtol=0.03)


def test_band_edges_infeasible_height_is_unconditioned():
    rng = np.random.default_rng(2)
    b = synth.band_edges(rng, 16)
    assert b.shape == (7,) and np.all(np.diff(b) >= 0)
    assert 0 <= b.min() and b.max() <= 16
