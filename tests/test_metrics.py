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


def test_mtf_of_a_point_is_flat():
    img = np.zeros((41, 41))
    img[20, 20] = 5.0
    f, m = metrics.mtf(img + 0.3, (20, 20), 0.5)
    assert f[0] == 0.0 and f[-1] == pytest.approx(10 / (21 * 0.5))
    np.testing.assert_allclose(m, 1.0, atol=0.02)
    assert metrics.mtf50(f, m) == f[-1]


def test_mtf_of_a_gaussian_psf():
    """A Gaussian PSF of sigma pixels has MTF exp(-2 pi^2 sigma^2 f^2) (f in
    cycles per pixel); the ring average of the discrete patch follows it
    while the PSF fits the patch, and the background level drops out."""
    s = 1.3
    y, x = np.mgrid[-30:31, -30:31].astype(float)
    img = np.exp(-(x * x + y * y) / (2 * s * s)) + 0.25
    f, m = metrics.mtf(img, (30, 30), 1.0)
    # the closed form at every FFT bin, averaged over the same rings
    fy, fx = np.meshgrid(np.arange(21) - 10, np.arange(21) - 10, indexing="ij")
    r = np.hypot(fy, fx)
    closed = np.exp(-2 * np.pi ** 2 * s * s * (r / 21.0) ** 2)
    want = np.array([closed[np.rint(r) == k].mean() for k in range(11)])
    np.testing.assert_allclose(m, want / want[0], atol=0.01)
    # the ring average sits a little below the radial profile itself
    f50 = np.sqrt(np.log(2) / (2 * np.pi ** 2 * s * s))
    assert metrics.mtf50(f, m) == pytest.approx(f50, rel=0.05)
