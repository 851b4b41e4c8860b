"""The synthetic input generator (host code shared by both sides)."""

import time

import numpy as np
import pytest

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


def test_affine_sequence_motion():
    # no motion reproduces the base image; a pure integer shift moves it by
    # whole pixels (interior); the largest displacement is max_disp
    rng = np.random.default_rng(0)
    B = synth.base_image(rng, (20, 16))
    M = np.zeros((2, 3))
    np.testing.assert_allclose(synth.affine_frame(B, M), B.astype(np.float32),
                               atol=1e-6)
    M[0, 2], M[1, 2] = 2.0, -1.0
    f = synth.affine_frame(B, M)
    np.testing.assert_allclose(f[4:-4, 4:-4], B[2:-6, 5:-3].astype(np.float32),
                               atol=1e-6)
    Ms = synth.affine_motion(9, 3, 4.0, (10, 8, 6), seed=3)
    corners = np.array(np.meshgrid(*[[-1.0, 1.0]] * 3, indexing="ij")) \
        .reshape(3, -1)
    disp = np.einsum("tae,ec->tac", Ms[:, :, :3], corners) + Ms[:, :, 3:]
    assert np.sqrt((disp ** 2).sum(axis=1)).max() == pytest.approx(4.0)
    fr, _ = synth.affine_sequence(3, (12, 10, 8), 2.0, seed=4)
    assert fr.shape == (3, 12, 10, 8) and fr.dtype == np.float32
