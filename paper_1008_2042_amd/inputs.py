"""Seeded synthetic inputs: scanner geometries, ellipsoid phantoms, analytic
projections and Poisson noise.

This module is shared by the GPU path's tests/benchmark and by the oracle's
tests.  It holds none of the reconstruction method's arithmetic: no
discretised projector, no framelet, no solver.  Projection data are the exact
line integrals of Eq. (1) through additive ellipsoids (a closed form), so the
data never come from either implementation's projector.

Workload shapes follow the paper's cases (section 3: 512x512x70 volumes, a
512x384 flat panel, 40 views, SAD 1000 mm, SDD 1500 mm), with the paper's
NCAT/Catphan/patient data replaced by seeded ellipsoid phantoms.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Geometry:
    """Circular cone-beam orbit with a flat detector (units mm, radians)."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    nu: int
    nv: int
    du: float
    dv: float
    sad: float = 1000.0
    sdd: float = 1500.0
    n_views: int = 40
    angles: Optional[np.ndarray] = None  # None: 2 pi k / n_views

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def sino_shape(self):
        return (self.n_views, self.nv, self.nu)

    def view_angles(self) -> np.ndarray:
        if self.angles is not None:
            return np.asarray(self.angles, np.float64)
        return 2.0 * math.pi * np.arange(self.n_views, dtype=np.float64) / self.n_views


@dataclasses.dataclass
class Ellipsoid:
    center: Sequence[float]   # mm
    axes: Sequence[float]     # semi-axes (mm) before rotation
    phi: float                # rotation about z (rad)
    rho: float                # additive attenuation (1/mm)


# --------------------------------------------------------------------------
# Configurations (the reconstruction workloads)
# --------------------------------------------------------------------------
def config(name: str) -> dict:
    """Named workloads.  'tiny': 64x64x16; 'paper': the paper-scale
    512x512x70 case; 'precision': the tiny case at low dose; 'large':
    512x512x256 with 360 views."""
    if name == "tiny":
        g = Geometry(64, 64, 16, 1.0, 1.0, 1.0, 128, 64, 1.5, 1.5, n_views=30)
        return dict(name=name, geom=g, phantom=("tiny", 101), noise=None, lam=5e-4,
                    iters=[10], cgls_steps=3, framelet_levels=1)
    if name == "paper":
        g = Geometry(512, 512, 70, 0.5, 0.5, 2.5, 512, 384, 0.776, 0.776, n_views=40)
        return dict(name=name, geom=g, phantom=("body", 102, 4, 15), noise=(1e5, 202),
                    lam=5e-4, iters=[16, 24], cgls_steps=3, framelet_levels=1)
    if name.startswith("precision"):
        i0, seed = {"precision": (1e4, 301), "precision_5e4": (5e4, 302)}.get(name, (1e4, 301))
        g = Geometry(64, 64, 16, 1.0, 1.0, 1.0, 128, 64, 1.5, 1.5, n_views=30)
        return dict(name=name, geom=g, phantom=("tiny", 101), noise=(i0, seed), lam=5e-4,
                    iters=[10], cgls_steps=3, framelet_levels=1)
    if name == "large":
        g = Geometry(512, 512, 256, 0.5, 0.5, 0.5, 1024, 768, 0.388, 0.388, n_views=360)
        return dict(name=name, geom=g, phantom=("body", 105, 8, 31), noise=(5e4, 205),
                    lam=5e-4, iters=[5, 10, 15], cgls_steps=3, framelet_levels=2)
    raise KeyError(name)


def serving_geometry(nxy: int, nz: int, n_views: int) -> Geometry:
    """Serving-mix geometry: 256 mm in-plane FOV, 175 mm z-FOV for 70-slice
    volumes (z voxel 2.5 mm), detector nu = nx, nv = 3/4 nx at 0.776*512/nx mm."""
    dxy = 256.0 / nxy
    dz = 175.0 / nz
    pitch = 0.776 * 512.0 / nxy
    return Geometry(nxy, nxy, nz, dxy, dxy, dz, nxy, (3 * nxy) // 4, pitch, pitch,
                    n_views=n_views)


# --------------------------------------------------------------------------
# Phantoms
# --------------------------------------------------------------------------
def tiny_phantom(seed: int, n: int = 5) -> List[Ellipsoid]:
    """n random ellipsoids inside a 64x64x16 mm box: in-plane semi-axes
    U[4,14] mm, z semi-axis U[2,6] mm, rho ~ U[0.01, 0.03] /mm (additive)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        a, b = rng.uniform(4, 14, size=2)
        c = rng.uniform(2, 6)
        r = max(a, b)
        cx, cy = rng.uniform(-32 + r, 32 - r, size=2)
        cz = rng.uniform(-8 + c, 8 - c)
        out.append(Ellipsoid((cx, cy, cz), (a, b, c), rng.uniform(0, math.pi),
                             rng.uniform(0.01, 0.03)))
    return out


def body_phantom(seed: int, n_bone: int, n_soft: int, zhalf: float = 80.0) -> List[Ellipsoid]:
    """A body ellipsoid (115, 90, zhalf) mm at 0.02 /mm, bone inserts at an
    absolute 0.04 /mm (additive +0.02) and soft lesions with contrast
    U[-0.003, 0.003]; inserts lie inside the body and do not overlap
    (rejection sampling on bounding spheres)."""
    rng = np.random.default_rng(seed)
    body = Ellipsoid((0.0, 0.0, 0.0), (115.0, 90.0, zhalf), 0.0, 0.02)
    out = [body]
    placed = []  # (center, radius)
    specs = [("bone", n_bone), ("soft", n_soft)]
    for kind, count in specs:
        k = 0
        tries = 0
        while k < count:
            tries += 1
            if tries > 100000:
                raise RuntimeError("phantom placement failed")
            if kind == "bone":
                a, b = rng.uniform(6, 14, size=2)
                c = rng.uniform(10, 30)
                rho = 0.02
            else:
                a, b = rng.uniform(4, 12, size=2)
                c = rng.uniform(4, 15)
                rho = rng.uniform(-0.003, 0.003)
            r = max(a, b, c)
            ctr = rng.uniform(-1, 1, size=3) * np.array(body.axes)
            # inside the body with margin r on every axis
            q = ctr / (np.array(body.axes) - r)
            if np.any(np.array(body.axes) - r <= 0) or float(q @ q) > 1.0:
                continue
            if any(np.linalg.norm(ctr - pc) < r + pr for pc, pr in placed):
                continue
            placed.append((ctr, r))
            out.append(Ellipsoid(tuple(ctr), (a, b, c), rng.uniform(0, math.pi), rho))
            k += 1
    return out


def phantom_for(cfg: dict) -> List[Ellipsoid]:
    spec = cfg["phantom"]
    if spec[0] == "tiny":
        return tiny_phantom(spec[1])
    g = cfg["geom"]
    zhalf = min(80.0, 0.5 * g.nz * g.dz - 5.0) if g.nz * g.dz < 200 else 110.0
    return body_phantom(spec[1], spec[2], spec[3], zhalf=zhalf)


# --------------------------------------------------------------------------
# Exact line integrals through ellipsoids (Eq. (1) in closed form)
# --------------------------------------------------------------------------
def _scanner_rays(g: Geometry, view: int):
    """Source position and source-to-pixel vectors of one view.  The scanner
    model: source at SAD (cos t, sin t, 0); flat panel through
    -(SDD-SAD)(cos t, sin t, 0), u along (-sin t, cos t, 0), v along z; pixel
    centres (c-(nu-1)/2) du, (r-(nv-1)/2) dv."""
    t = g.view_angles()[view]
    ct, st = math.cos(t), math.sin(t)
    src = np.array([g.sad * ct, g.sad * st, 0.0])
    u = (np.arange(g.nu) - 0.5 * (g.nu - 1)) * g.du
    v = (np.arange(g.nv) - 0.5 * (g.nv - 1)) * g.dv
    det_c = -(g.sdd - g.sad) * np.array([ct, st, 0.0])
    px = det_c[0] - u[None, :] * st + 0.0 * v[:, None]
    py = det_c[1] + u[None, :] * ct + 0.0 * v[:, None]
    pz = np.broadcast_to(v[:, None], (g.nv, g.nu))
    a = np.stack([px - src[0], py - src[1], pz - src[2]], axis=-1)
    return src, a


def chord(src, a, e: Ellipsoid):
    """Length of the segment src + t a, t in [0, 1], inside ellipsoid e,
    times its density."""
    cphi, sphi = math.cos(e.phi), math.sin(e.phi)
    R = np.array([[cphi, -sphi, 0.0], [sphi, cphi, 0.0], [0.0, 0.0, 1.0]])
    ax = np.asarray(e.axes, np.float64)
    p = ((np.asarray(src, np.float64) - np.asarray(e.center, np.float64)) @ R) / ax
    q = (a @ R) / ax
    A = np.einsum("...i,...i->...", q, q)
    B = np.einsum("...i,...i->...", q, np.broadcast_to(p, q.shape))
    C = float(p @ p) - 1.0
    disc = B * B - A * C
    hit = disc > 0
    sq = np.sqrt(np.where(hit, disc, 0.0))
    t1 = np.clip((-B - sq) / A, 0.0, 1.0)
    t2 = np.clip((-B + sq) / A, 0.0, 1.0)
    alen = np.sqrt(np.einsum("...i,...i->...", a, a))
    return np.where(hit, (t2 - t1) * alen * e.rho, 0.0)


def analytic_projection(g: Geometry, ellipsoids: List[Ellipsoid]) -> np.ndarray:
    """Noiseless post-log data g[view][r][c] = sum of density x chord."""
    out = np.zeros(g.sino_shape, np.float64)
    for k in range(g.n_views):
        src, a = _scanner_rays(g, k)
        for e in ellipsoids:
            out[k] += chord(src, a, e)
    return out


def analytic_projection_torch(g: Geometry, ellipsoids: List[Ellipsoid], device,
                              views_per_chunk: int = 40):
    """The same exact chord integrals as analytic_projection, evaluated in
    FP64 with torch on `device` (fast generation of large serving mixes),
    a chunk of views at a time."""
    import torch
    out = torch.empty((g.n_views, g.nv, g.nu), dtype=torch.float64, device=device)
    ang = g.view_angles()
    for v0 in range(0, g.n_views, views_per_chunk):
        v1 = min(g.n_views, v0 + views_per_chunk)
        sub = dataclasses.replace(g, n_views=v1 - v0, angles=ang[v0:v1])
        out[v0:v1] = _chords_torch(sub, ellipsoids, device)
    return out


def _chords_torch(g: Geometry, ellipsoids: List[Ellipsoid], device):
    import torch
    f64 = torch.float64
    th = torch.tensor(g.view_angles(), dtype=f64, device=device)
    ct, st = torch.cos(th)[:, None, None], torch.sin(th)[:, None, None]
    u = ((torch.arange(g.nu, dtype=f64, device=device) - 0.5 * (g.nu - 1)) * g.du)[None, None, :]
    v = ((torch.arange(g.nv, dtype=f64, device=device) - 0.5 * (g.nv - 1)) * g.dv)[None, :, None]
    sx, sy = g.sad * ct, g.sad * st
    px = -(g.sdd - g.sad) * ct - u * st
    py = -(g.sdd - g.sad) * st + u * ct
    ax = (px - sx).expand(g.n_views, g.nv, g.nu)
    ay = (py - sy).expand(g.n_views, g.nv, g.nu)
    az = v.expand(g.n_views, g.nv, g.nu)
    alen = torch.sqrt(ax * ax + ay * ay + az * az)
    out = torch.zeros((g.n_views, g.nv, g.nu), dtype=f64, device=device)
    for e in ellipsoids:
        c, s = math.cos(e.phi), math.sin(e.phi)
        a0, a1, a2 = (float(x) for x in e.axes)
        ox, oy, oz = (sx - e.center[0]), (sy - e.center[1]), -float(e.center[2])
        # rotate into the ellipsoid frame (x R with R = [[c, -s], [s, c]]), scale by axes
        p0, p1, p2 = (ox * c + oy * s) / a0, (-ox * s + oy * c) / a1, oz / a2
        q0, q1, q2 = (ax * c + ay * s) / a0, (-ax * s + ay * c) / a1, az / a2
        A = q0 * q0 + q1 * q1 + q2 * q2
        B = q0 * p0 + q1 * p1 + q2 * p2
        C = p0 * p0 + p1 * p1 + p2 * p2 - 1.0
        disc = B * B - A * C
        hit = disc > 0
        sq = torch.sqrt(torch.where(hit, disc, torch.zeros_like(disc)))
        t1 = torch.clamp((-B - sq) / A, 0.0, 1.0)
        t2 = torch.clamp((-B + sq) / A, 0.0, 1.0)
        out += torch.where(hit, (t2 - t1) * alen * e.rho, torch.zeros_like(disc))
    return out


def poisson_log_torch(g_true, i0: float, seed: int):
    """-ln(max(I, 1) / I0) with I ~ Poisson(I0 exp(-g)), seeded torch generator
    on the tensor's device."""
    import torch
    gen = torch.Generator(device=g_true.device)
    gen.manual_seed(int(seed))
    counts = torch.poisson(i0 * torch.exp(-g_true), generator=gen)
    return -torch.log(torch.clamp(counts, min=1.0) / i0)


SERVING_SIZES = [(128, 128), (256, 48), (256, 96), (512, 70)]  # (nxy, nz)
SERVING_VIEWS = [20, 40, 60, 120]
SERVING_I0 = [1e4, 1e5]


def serving_mix(n: int = 64, seed: int = 404):
    """Seeded request mix: size, views and dose drawn uniformly from the
    serving sets; phantom seed 4000 + i (body + 4 bone + 15 soft inserts)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nxy, nz = SERVING_SIZES[int(rng.integers(len(SERVING_SIZES)))]
        views = SERVING_VIEWS[int(rng.integers(len(SERVING_VIEWS)))]
        i0 = SERVING_I0[int(rng.integers(len(SERVING_I0)))]
        out.append(dict(index=i, geom=serving_geometry(nxy, nz, views), i0=i0,
                        phantom_seed=4000 + i, noise_seed=5000 + i))
    return out


def poisson_log(g_true: np.ndarray, i0: float, seed: int) -> np.ndarray:
    """Counts I ~ Poisson(I0 exp(-g)); returns -ln(max(I, 1) / I0)."""
    rng = np.random.default_rng(seed)
    counts = rng.poisson(i0 * np.exp(-g_true))
    return -np.log(np.maximum(counts, 1) / i0)


def voxelize(g: Geometry, ellipsoids: List[Ellipsoid], ss: int = 4) -> np.ndarray:
    """Truth volume: mean density over an ss^3 sub-sample grid of each voxel
    (one voxel slice at a time, each ellipsoid within its bounding box)."""
    vol = np.zeros(g.vol_shape, np.float64)
    offs = (np.arange(ss) + 0.5) / ss - 0.5
    xs = ((np.arange(g.nx) - 0.5 * (g.nx - 1))[:, None] + offs[None, :]).ravel() * g.dx
    ys = ((np.arange(g.ny) - 0.5 * (g.ny - 1))[:, None] + offs[None, :]).ravel() * g.dy
    for k in range(g.nz):
        zs = ((k - 0.5 * (g.nz - 1)) + offs) * g.dz
        acc = np.zeros((ss, g.ny * ss, g.nx * ss), np.float64)
        for e in ellipsoids:
            r = max(e.axes[0], e.axes[1])
            zm = np.abs(zs - e.center[2]) <= e.axes[2]
            xm = np.nonzero(np.abs(xs - e.center[0]) <= r)[0]
            ym = np.nonzero(np.abs(ys - e.center[1]) <= r)[0]
            if not zm.any() or xm.size == 0 or ym.size == 0:
                continue
            cphi, sphi = math.cos(e.phi), math.sin(e.phi)
            X = xs[xm][None, None, :] - e.center[0]
            Y = ys[ym][None, :, None] - e.center[1]
            Z = zs[:, None, None] - e.center[2]
            xr = (X * cphi + Y * sphi) / e.axes[0]
            yr = (-X * sphi + Y * cphi) / e.axes[1]
            inside = (xr * xr + yr * yr + (Z / e.axes[2]) ** 2) <= 1.0
            acc[:, ym[0]:ym[-1] + 1, xm[0]:xm[-1] + 1] += inside * e.rho
        vol[k] = acc.reshape(ss, g.ny, ss, g.nx, ss).mean(axis=(0, 2, 4))
    return vol


def measured_data(cfg: dict) -> np.ndarray:
    """The post-log sinogram of a configuration (noiseless or Poisson)."""
    g = cfg["geom"]
    clean = analytic_projection(g, phantom_for(cfg))
    if cfg.get("noise"):
        i0, seed = cfg["noise"]
        return poisson_log(clean, i0, seed)
    return clean


# --------------------------------------------------------------------------
# Random operands for operator-level checks
# --------------------------------------------------------------------------
def random_volume(g: Geometry, seed: int, scale: float = 0.02) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, scale, size=g.vol_shape)


def random_sino(g: Geometry, seed: int, scale: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-scale, scale, size=g.sino_shape)


def random_field(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)
