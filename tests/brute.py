"""Brute-force references for tiny grids, written independently of the
oracle's C code (different parametrisation, dense weights, numpy/scipy).

* ``joseph_matrix``: the projector of Eq. (1) discretised by Joseph's method,
  built one ray at a time: every sample point is formed in world coordinates
  as source + tau * (pixel - source) on the voxel-centre planes of the view's
  stepping axis, and its weight on EVERY voxel is the dense product of three
  hat functions (trilinear interpolation), times the path length between
  planes.
* ``framelet_matrix``: the 27-band analysis W assembled column by column from
  scipy.ndimage.convolve with mode='reflect' (half-sample symmetric).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.ndimage as ndi


def hat(t):
    return np.maximum(0.0, 1.0 - np.abs(t))


def view_angles(g):
    if getattr(g, "angles", None) is not None:
        return np.asarray(g.angles, np.float64)
    return 2.0 * math.pi * np.arange(g.n_views) / g.n_views


def joseph_matrix(g) -> np.ndarray:
    nx, ny, nz = g.nx, g.ny, g.nz
    ii, jj, kk = np.arange(nx), np.arange(ny), np.arange(nz)
    centres = [(ii - (nx - 1) / 2.0) * g.dx, (jj - (ny - 1) / 2.0) * g.dy]
    spacing = [g.dx, g.dy]
    rows = []
    for th in view_angles(g):
        ct, st = math.cos(th), math.sin(th)
        src = np.array([g.sad * ct, g.sad * st, 0.0])
        det_c = -(g.sdd - g.sad) * np.array([ct, st, 0.0])
        e_u = np.array([-st, ct, 0.0])
        e_v = np.array([0.0, 0.0, 1.0])
        ax = 0 if abs(ct) >= abs(st) - 1e-12 else 1
        for r in range(g.nv):
            for c in range(g.nu):
                pix = det_c + (c - (g.nu - 1) / 2.0) * g.du * e_u + (r - (g.nv - 1) / 2.0) * g.dv * e_v
                a = pix - src
                ell = spacing[ax] * np.linalg.norm(a) / abs(a[ax])
                row = np.zeros((nz, ny, nx))
                for coord in centres[ax]:
                    tau = (coord - src[ax]) / a[ax]
                    if not (0.0 < tau < 1.0):
                        continue
                    P = src + tau * a
                    fi = P[0] / g.dx + (nx - 1) / 2.0
                    fj = P[1] / g.dy + (ny - 1) / 2.0
                    fk = P[2] / g.dz + (nz - 1) / 2.0
                    if ax == 0:
                        fi = round(fi)  # exactly on the plane (removes 1e-16 noise)
                    else:
                        fj = round(fj)
                    row += ell * (hat(fk - kk)[:, None, None] * hat(fj - jj)[None, :, None]
                                  * hat(fi - ii)[None, None, :])
                rows.append(row.ravel())
    return np.array(rows)


# h[-1], h[0], h[+1] as printed in section 2.1
H = [np.array([1.0, 2.0, 1.0]) / 4.0,
     np.array([1.0, 0.0, -1.0]) * math.sqrt(2.0) / 4.0,
     np.array([-1.0, 2.0, -1.0]) / 4.0]


def kernel3d(l, m, n, dil=1):
    """Convolution kernel of band 9n+3m+l, array axes (z, y, x)."""
    def dil1(h):
        if dil == 1:
            return h
        out = np.zeros(2 * dil + 1)
        out[0], out[dil], out[-1] = h
        return out
    hx, hy, hz = dil1(H[l]), dil1(H[m]), dil1(H[n])
    return hz[:, None, None] * hy[None, :, None] * hx[None, None, :]


def analysis_scipy(f, dil=1):
    """W f by scipy: convolution with half-sample symmetric ('reflect') edges.
    scipy's kernel index c corresponds to tap offset c - centre, i.e. the
    printed order h[-1], h[0], h[+1]."""
    out = []
    for n in range(3):
        for m in range(3):
            for l in range(3):
                out.append(ndi.convolve(f, kernel3d(l, m, n, dil), mode="reflect"))
    return np.array(out)


def framelet_matrix(shape, dil=1) -> np.ndarray:
    n = int(np.prod(shape))
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(analysis_scipy(e.reshape(shape), dil).ravel())
    return np.array(cols).T  # (27 n, n)


def shrink_dense(coeff, lam):
    c = coeff.copy()
    nrm = np.sqrt((c[1:] ** 2).sum(axis=0))
    s = np.where(nrm <= lam, 0.0, 1.0 - lam / np.where(nrm > 0, nrm, 1.0))
    c[1:] *= s
    return c


def _view_frame(g, th):
    ct, st = math.cos(th), math.sin(th)
    src = np.array([g.sad * ct, g.sad * st, 0.0])
    det_c = -(g.sdd - g.sad) * np.array([ct, st, 0.0])
    e_u = np.array([-st, ct, 0.0])
    e_v = np.array([0.0, 0.0, 1.0])
    return src, det_c, e_u, e_v


def _voxel_boxes(g):
    """Lower and upper corners of every voxel box, each (nz, ny, nx, 3)."""
    ii = (np.arange(g.nx) - (g.nx - 1) / 2.0) * g.dx
    jj = (np.arange(g.ny) - (g.ny - 1) / 2.0) * g.dy
    kk = (np.arange(g.nz) - (g.nz - 1) / 2.0) * g.dz
    K, J, I = np.meshgrid(kk, jj, ii, indexing="ij")
    ctr = np.stack([I, J, K], axis=-1)
    half = 0.5 * np.array([g.dx, g.dy, g.dz])
    return ctr - half, ctr + half


def siddon_matrix(g) -> np.ndarray:
    """The radiological-path projector: entry (ray, voxel) is the length of
    the source-to-pixel segment inside the voxel's box, from the slab
    intersection of the segment with each box separately (no traversal).
    Boxes are half-open: a ray lying on a face plane counts in the box above."""
    lo, hi = _voxel_boxes(g)
    rows = []
    for th in view_angles(g):
        src, det_c, e_u, e_v = _view_frame(g, th)
        for r in range(g.nv):
            for c in range(g.nu):
                pix = det_c + (c - (g.nu - 1) / 2.0) * g.du * e_u + (r - (g.nv - 1) / 2.0) * g.dv * e_v
                a = pix - src
                t_in = np.zeros(lo.shape[:3])
                t_out = np.ones(lo.shape[:3])
                for ax in range(3):
                    if a[ax] == 0.0:
                        # half-open boxes: a ray on a face belongs to the box above it
                        inside = (src[ax] >= lo[..., ax]) & (src[ax] < hi[..., ax])
                        t_out = np.where(inside, t_out, -1.0)
                        continue
                    t0 = (lo[..., ax] - src[ax]) / a[ax]
                    t1 = (hi[..., ax] - src[ax]) / a[ax]
                    t_in = np.maximum(t_in, np.minimum(t0, t1))
                    t_out = np.minimum(t_out, np.maximum(t0, t1))
                rows.append((np.maximum(t_out - t_in, 0.0) * np.linalg.norm(a)).reshape(-1))
    return np.array(rows)


def detector_hit(g, th, pts):
    """Where the lines from the source through points pts (n, 3) meet the
    detector plane: (u*, v*, L, l) from the 3D line-plane intersection."""
    src, det_c, e_u, e_v = _view_frame(g, th)
    nrm = np.cross(e_u, e_v)  # detector normal
    d = pts - src
    t = ((det_c - src) @ nrm) / (d @ nrm)
    hit = src + t[:, None] * d
    rel = hit - det_c
    return rel @ e_u, rel @ e_v, np.linalg.norm(hit - src, axis=1), np.linalg.norm(d, axis=1)


def eq3_matrix(g) -> np.ndarray:
    """The Eq. (3) backprojection as a dense (voxel, ray) matrix: for every
    voxel centre and view, dx dy dz / (du dv) L^3 / (SDD l^2) times the
    bilinear weights (products of hats in pixel units) of the detector
    pixels around the hit point."""
    ii = (np.arange(g.nx) - (g.nx - 1) / 2.0) * g.dx
    jj = (np.arange(g.ny) - (g.ny - 1) / 2.0) * g.dy
    kk = (np.arange(g.nz) - (g.nz - 1) / 2.0) * g.dz
    K, J, I = np.meshgrid(kk, jj, ii, indexing="ij")
    pts = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    uc = (np.arange(g.nu) - (g.nu - 1) / 2.0) * g.du
    vr = (np.arange(g.nv) - (g.nv - 1) / 2.0) * g.dv
    pref = g.dx * g.dy * g.dz / (g.du * g.dv)
    blocks = []
    for th in view_angles(g):
        us, vs, L, l = detector_hit(g, th, pts)
        wu = hat((us[:, None] - uc[None, :]) / g.du)  # (voxels, nu)
        wv = hat((vs[:, None] - vr[None, :]) / g.dv)  # (voxels, nv)
        scale = pref * L ** 3 / (g.sdd * l ** 2)
        blocks.append((scale[:, None, None] * wv[:, :, None] * wu[:, None, :]).reshape(len(pts), -1))
    return np.concatenate(blocks, axis=1)
