"""Image-quality metrics the paper reports, on host arrays.

* relative root-mean-square error e = ||f - f0|| / ||f0|| (section 3.1)
* contrast-to-noise ratio CNR = 2 |S - S_b| / (sigma + sigma_b), with S, S_b
  the mean values and sigma, sigma_b the standard deviations (ddof 0; the
  paper does not say) inside a region of interest and its background
  (section 3.2)
* the in-plane modulation transfer function from a point-like object
  (section 3.2): a 21 x 21 pixel patch of its slice centred on the object,
  background subtracted, 2-D FFT, amplitude averaged along the angular
  direction
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np


def rrms(f: np.ndarray, f0: np.ndarray) -> float:
    f = np.asarray(f, np.float64)
    f0 = np.asarray(f0, np.float64)
    return float(np.linalg.norm(f - f0) / np.linalg.norm(f0))


def cnr(vol: np.ndarray, roi: np.ndarray, background: np.ndarray) -> float:
    a = np.asarray(vol, np.float64)[roi]
    b = np.asarray(vol, np.float64)[background]
    return float(2.0 * abs(a.mean() - b.mean()) / (a.std() + b.std()))


def _inside(g, e, scale: float) -> np.ndarray:
    """Voxel centres inside ellipsoid e with its semi-axes scaled."""
    x = (np.arange(g.nx) - 0.5 * (g.nx - 1)) * g.dx - e.center[0]
    y = (np.arange(g.ny) - 0.5 * (g.ny - 1)) * g.dy - e.center[1]
    z = (np.arange(g.nz) - 0.5 * (g.nz - 1)) * g.dz - e.center[2]
    c, s = math.cos(e.phi), math.sin(e.phi)
    X, Y = x[None, None, :], y[None, :, None]
    xr = (X * c + Y * s) / (e.axes[0] * scale)
    yr = (-X * s + Y * c) / (e.axes[1] * scale)
    zr = (z / (e.axes[2] * scale))[:, None, None]
    return (xr * xr + yr * yr + zr * zr) <= 1.0


def cnr_rois(g, ellipsoids: Sequence, index: int):
    """ROI = ellipsoid `index` shrunk to 0.6x minus every other ellipsoid;
    background = outside every ellipsoid grown to 1.4x."""
    roi = _inside(g, ellipsoids[index], 0.6)
    for k, e in enumerate(ellipsoids):
        if k != index:
            roi &= ~_inside(g, e, 1.0)
    bg = np.ones(g.vol_shape, bool)
    for e in ellipsoids:
        bg &= ~_inside(g, e, 1.4)
    return roi, bg


def cnr_all(vol: np.ndarray, g, ellipsoids: List) -> List[float]:
    out = []
    for k in range(len(ellipsoids)):
        roi, bg = cnr_rois(g, ellipsoids, k)
        if roi.sum() >= 8 and bg.sum() >= 8:
            out.append(cnr(vol, roi, bg))
    return out


def mtf(slice2d: np.ndarray, center, pixel_mm: float, size: int = 21):
    """The in-plane MTF of section 3.2 from a point-like object.

    The size x size patch of `slice2d` centred on pixel `center` (row, col)
    is the point spread function after the background, read as the mean of
    the patch's outermost ring of pixels (the paper does not say how it is
    measured), is subtracted.  Its 2-D FFT amplitude is averaged over rings
    of equal radial frequency index k = 0 .. size // 2 (nearest integer
    radius of each frequency bin) and normalised by the zero-frequency
    value.  Returns (frequencies in cycles/mm, MTF values)."""
    a = np.asarray(slice2d, np.float64)
    r0, c0 = int(center[0]), int(center[1])
    h = size // 2
    patch = a[r0 - h:r0 + h + 1, c0 - h:c0 + h + 1].copy()
    if patch.shape != (size, size):
        raise ValueError("the patch leaves the slice")
    ring = np.ones((size, size), bool)
    ring[1:-1, 1:-1] = False
    patch -= patch[ring].mean()
    amp = np.abs(np.fft.fftshift(np.fft.fft2(patch)))
    fy, fx = np.meshgrid(np.arange(size) - h, np.arange(size) - h, indexing="ij")
    rad = np.rint(np.hypot(fy, fx)).astype(int)
    prof = np.array([amp[rad == k].mean() for k in range(h + 1)])
    freqs = np.arange(h + 1) / (size * pixel_mm)
    return freqs, prof / prof[0]


def mtf50(freqs: np.ndarray, m: np.ndarray) -> float:
    """The frequency where the MTF first falls to 0.5 (linear interpolation
    between samples), or the last frequency if it never does."""
    below = np.nonzero(m < 0.5)[0]
    if below.size == 0:
        return float(freqs[-1])
    k = int(below[0])
    if k == 0:
        return float(freqs[0])
    return float(freqs[k - 1] + (m[k - 1] - 0.5) / (m[k - 1] - m[k]) * (freqs[k] - freqs[k - 1]))
