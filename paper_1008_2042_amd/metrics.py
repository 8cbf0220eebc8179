"""Image-quality metrics the paper reports, on host arrays.

* relative root-mean-square error e = ||f - f0|| / ||f0|| (section 3.1)
* contrast-to-noise ratio CNR = 2 |S - S_b| / (sigma + sigma_b), with S, S_b
  the mean values and sigma, sigma_b the standard deviations (ddof 0; the
  paper does not say) inside a region of interest and its background
  (section 3.2)
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
