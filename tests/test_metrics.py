"""The paper's image metrics on images with known answers."""
import numpy as np
import pytest

from paper_1008_2042_amd import inputs, metrics


def test_rrms_known():
    f0 = np.ones((4, 4, 4))
    assert metrics.rrms(f0 * 1.1, f0) == pytest.approx(0.1, rel=1e-12)


def test_cnr_known_two_level_image():
    vol = np.zeros((1, 10, 10))
    roi = np.zeros(vol.shape, bool)
    roi[0, :5] = True
    bg = ~roi
    vol[roi] = np.where(np.arange(roi.sum()) % 2 == 0, 1.0, 3.0)  # mean 2, std 1
    vol[bg] = 0.0                                                  # mean 0, std 0
    assert metrics.cnr(vol, roi, bg) == pytest.approx(2 * 2 / 1.0)


def test_cnr_rois_on_voxelised_phantom():
    g = inputs.config("tiny")["geom"]
    ells = inputs.tiny_phantom(101)
    truth = inputs.voxelize(g, ells, ss=1)
    roi, bg = metrics.cnr_rois(g, ells, 0)
    assert roi.sum() > 0 and bg.sum() > 0 and not np.any(roi & bg)
    # noiseless piecewise-constant truth: background is exactly 0
    assert np.all(truth[bg] == 0.0)
