"""FP64 CPU oracle of the tight-frame CBCT iteration (arXiv 1008.2042).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never does.  This binding imports
nothing from the GPU package; geometries are taken duck-typed (any object
with the fields of ``OrcGeom``).

The arithmetic lives in ``tf_oracle.c`` (plain C, double precision, OpenMP
over independent outputs).  Every function cites the passage it follows.
Pins (tests/test_oracle_*.py) tie each function to closed forms, library
routines, invariants and brute force; ``reconstruct`` composes pinned parts
and is itself pinned only by brute force on tiny grids (explicit matrices)
and the fixed-point invariant.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tf_oracle.c")
_LIB = os.path.join(_HERE, "libtf_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
             "-fno-fast-math", "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcGeom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("du", ctypes.c_double), ("dv", ctypes.c_double),
                ("sad", ctypes.c_double), ("sdd", ctypes.c_double),
                ("n_views", ctypes.c_int32), ("angles", ctypes.POINTER(ctypes.c_double))]


class OrcOpts(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("n_grids", ctypes.c_int32),
                ("iters", ctypes.c_int32 * 4), ("cgls_steps", ctypes.c_int32),
                ("framelet_levels", ctypes.c_int32), ("momentum", ctypes.c_int32),
                ("positivity", ctypes.c_int32), ("bin_coarse_detector", ctypes.c_int32),
                ("op_pair", ctypes.c_int32)]


class OrcTV(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("eps", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_steps", ctypes.c_int32)]


class OrcReport(ctypes.Structure):
    _fields_ = [("resid2_last", ctypes.c_double), ("cgls_breakdowns", ctypes.c_int32),
                ("iters_done", ctypes.c_int32 * 4)]


_lib = None
_P = np.ctypeslib.ndpointer
_D = _P(dtype=np.float64, flags="C_CONTIGUOUS")
_I = _P(dtype=np.int32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        G = ctypes.POINTER(OrcGeom)
        i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "orc_num_threads": ([], ctypes.c_int),
            "orc_project": ([G, _D, _D], None),
            "orc_project_rays": ([G, _D, i64, _I, _D], None),
            "orc_backproject": ([G, _D, _D], None),
            "orc_backproject_voxels": ([G, _D, i64, _I, _D], None),
            "orc_project_siddon": ([G, _D, _D], None),
            "orc_project_siddon_rays": ([G, _D, i64, _I, _D], None),
            "orc_backproject_eq3": ([G, _D, _D], None),
            "orc_backproject_eq3_voxels": ([G, _D, i64, _I, _D], None),
            "orc_framelet_analysis": ([i32, i32, i32, i32, _D, _D], None),
            "orc_framelet_synthesis": ([i32, i32, i32, i32, _D, _D], None),
            "orc_shrink": ([i64, dbl, _D], None),
            "orc_framelet_shrink": ([i32, i32, i32, i32, dbl, i32, _D, _D], None),
            "orc_cgls": ([G, _D, _D, i32, ctypes.POINTER(dbl), ctypes.c_void_p], ctypes.c_int),
            "orc_cgls_pair": ([G, i32, _D, _D, i32, ctypes.POINTER(dbl), ctypes.c_void_p],
                              ctypes.c_int),
            "orc_coarse_geom": ([G, i32, G], None),
            "orc_restrict_sino": ([G, _D, _D], None),
            "orc_prolong_vol": ([G, G, _D, _D], None),
            "orc_reconstruct": ([G, ctypes.POINTER(OrcOpts), _D, _D, ctypes.POINTER(OrcReport)],
                                ctypes.c_int),
            "orc_tf_iterations": ([G, ctypes.POINTER(OrcOpts), _D, i32, _D,
                                   ctypes.POINTER(OrcReport)], ctypes.c_int),
            "orc_ramlak": ([i32, dbl], dbl),
            "orc_fdk_filter": ([G, _D, _D], None),
            "orc_fdk_backproject": ([G, _D, _D], None),
            "orc_fdk": ([G, _D, _D], ctypes.c_int),
            "orc_tv_energy": ([i32, i32, i32, ctypes.POINTER(OrcTV), _D, _D], dbl),
            "orc_tv_gradient": ([i32, i32, i32, ctypes.POINTER(OrcTV), _D, _D, _D], None),
            "orc_rof": ([i32, i32, i32, ctypes.POINTER(OrcTV), _D, _D, ctypes.c_void_p],
                        ctypes.c_int),
            "orc_reconstruct_tv": ([G, ctypes.POINTER(OrcOpts), ctypes.POINTER(OrcTV), _D, _D,
                                    ctypes.POINTER(OrcReport), ctypes.POINTER(i32)],
                                   ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def _geom(g):
    """Marshal any object with the geometry fields into an OrcGeom.  The
    angle array (if any) is kept alive on the returned struct."""
    s = OrcGeom(int(g.nx), int(g.ny), int(g.nz), float(g.dx), float(g.dy), float(g.dz),
                int(g.nu), int(g.nv), float(g.du), float(g.dv), float(g.sad), float(g.sdd),
                int(g.n_views), None)
    ang = getattr(g, "angles", None)
    if ang is not None:
        a = np.ascontiguousarray(ang, dtype=np.float64)
        assert a.shape == (int(g.n_views),)
        s._keep = a
        s.angles = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return s


def _vol_shape(g):
    return (int(g.nz), int(g.ny), int(g.nx))


def _sino_shape(g):
    return (int(g.n_views), int(g.nv), int(g.nu))


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == tuple(shape), (a.shape, shape)
    return a


def project(g, f):
    """P f: Eq. (1) discretised by Joseph's method (section 2.1)."""
    f = _f64(f, _vol_shape(g))
    out = np.empty(_sino_shape(g), np.float64)
    _load().orc_project(ctypes.byref(_geom(g)), f, out)
    return out


def project_rays(g, f, vrc):
    """P f on the listed rays only; vrc is (n, 3) int (view, row, col)."""
    f = _f64(f, _vol_shape(g))
    vrc = np.ascontiguousarray(vrc, dtype=np.int32).reshape(-1, 3)
    out = np.empty(vrc.shape[0], np.float64)
    _load().orc_project_rays(ctypes.byref(_geom(g)), f, vrc.shape[0], vrc, out)
    return out


def backproject(g, proj):
    """P^T g: the exact transpose of ``project`` (Appendix 2, Eq. (A1))."""
    proj = _f64(proj, _sino_shape(g))
    out = np.empty(_vol_shape(g), np.float64)
    _load().orc_backproject(ctypes.byref(_geom(g)), proj, out)
    return out


def backproject_voxels(g, proj, kji):
    """P^T g at the listed voxels only; kji is (n, 3) int (k, j, i)."""
    proj = _f64(proj, _sino_shape(g))
    kji = np.ascontiguousarray(kji, dtype=np.int32).reshape(-1, 3)
    out = np.empty(kji.shape[0], np.float64)
    _load().orc_backproject_voxels(ctypes.byref(_geom(g)), proj, kji.shape[0], kji, out)
    return out


def project_siddon(g, f):
    """P f by Siddon's method (section 2.2.1): the exact length of each
    source-to-pixel segment inside each voxel box, times the voxel value."""
    f = _f64(f, _vol_shape(g))
    out = np.empty(_sino_shape(g), np.float64)
    _load().orc_project_siddon(ctypes.byref(_geom(g)), f, out)
    return out


def project_siddon_rays(g, f, vrc):
    """``project_siddon`` on the listed rays only; vrc is (n, 3) int (view, row, col)."""
    f = _f64(f, _vol_shape(g))
    vrc = np.ascontiguousarray(vrc, dtype=np.int32).reshape(-1, 3)
    out = np.empty(vrc.shape[0], np.float64)
    _load().orc_project_siddon_rays(ctypes.byref(_geom(g)), f, vrc.shape[0], vrc, out)
    return out


def backproject_eq3(g, proj):
    """The closed-form backprojection of Eq. (3) (section 2.2.2): per voxel
    and view, dx dy dz / (du dv) L^3 / (L0 l^2) times g bilinearly
    interpolated where the ray through the voxel centre meets the detector."""
    proj = _f64(proj, _sino_shape(g))
    out = np.empty(_vol_shape(g), np.float64)
    _load().orc_backproject_eq3(ctypes.byref(_geom(g)), proj, out)
    return out


def backproject_eq3_voxels(g, proj, kji):
    """``backproject_eq3`` at the listed voxels only; kji is (n, 3) int (k, j, i)."""
    proj = _f64(proj, _sino_shape(g))
    kji = np.ascontiguousarray(kji, dtype=np.int32).reshape(-1, 3)
    out = np.empty(kji.shape[0], np.float64)
    _load().orc_backproject_eq3_voxels(ctypes.byref(_geom(g)), proj, kji.shape[0], kji, out)
    return out


def framelet_analysis(f, dil=1):
    """W f: 27 bands (index 9n+3m+l) of the piecewise-linear tight frame (section 2.1)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx = f.shape
    out = np.empty((27, nz, ny, nx), np.float64)
    _load().orc_framelet_analysis(nx, ny, nz, dil, f, out)
    return out


def framelet_synthesis(coeff, dil=1):
    """W^T alpha: the exact adjoint of ``framelet_analysis``."""
    coeff = np.ascontiguousarray(coeff, dtype=np.float64)
    _, nz, ny, nx = coeff.shape
    out = np.empty((nz, ny, nx), np.float64)
    _load().orc_framelet_synthesis(nx, ny, nz, dil, coeff, out)
    return out


def shrink(coeff, lam):
    """T_mu of Eq. (2) on a (27, ...) coefficient array; returns a new array."""
    c = np.array(coeff, dtype=np.float64, order="C", copy=True)
    nvox = c.size // 27
    _load().orc_shrink(nvox, float(lam), c.reshape(-1))
    return c


def framelet_shrink(f, lam, levels=1, positivity=True):
    """H(W^T T_mu W f) (section 2.1, Algorithm A2 steps 3-4)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx = f.shape
    out = np.empty_like(f)
    _load().orc_framelet_shrink(nx, ny, nz, int(levels), float(lam), int(bool(positivity)), f, out)
    return out


def framelet_shrink_voxels(f, lam, kji, levels=1, positivity=True):
    """``framelet_shrink`` evaluated at the listed voxels (k, j, i) only.

    The operator is local: the output at a voxel depends on the coefficients
    within distance d (dilation) of it, and those on the input within 2d, so
    with one level it sees only the input within radius 2 (radius 6 with two
    levels: 2 + 2 * 2).  Each voxel is evaluated by the oracle on a crop of
    that radius whose faces are either faces of the volume (so the reflected
    extension is the same) or at least the radius away from the voxel."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    rad = 2 if levels == 1 else 6
    out = np.empty(len(kji), np.float64)
    for q, (k, j, i) in enumerate(np.asarray(kji, dtype=np.int64)):
        sl = []
        ctr = []
        for c, n in zip((k, j, i), f.shape):
            lo, hi = max(0, c - rad), min(n, c + rad + 1)
            sl.append(slice(lo, hi))
            ctr.append(c - lo)
        crop = np.ascontiguousarray(f[tuple(sl)])
        out[q] = framelet_shrink(crop, lam, levels, positivity)[tuple(ctr)]
    return out


def cgls(g, x0, proj, n, history=False, op_pair=0):
    """n CGLS steps warm-started from x0 (Appendix 1), with the Joseph pair
    (op_pair 0) or the paper's Siddon / Eq. (3) pair (op_pair 1).  Returns
    (x, broke, resid2[, resid_hist])."""
    x = np.array(x0, dtype=np.float64, order="C", copy=True)
    assert x.shape == _vol_shape(g)
    proj = _f64(proj, _sino_shape(g))
    r2 = ctypes.c_double(0.0)
    hist = np.zeros(n + 1, np.float64) if history else None
    broke = _load().orc_cgls_pair(ctypes.byref(_geom(g)), int(op_pair), x, proj, int(n),
                                  ctypes.byref(r2), hist.ctypes.data if history else None)
    if history:
        return x, bool(broke), r2.value, hist
    return x, bool(broke), r2.value


class _Coarse:
    pass


def coarse_geom(g, bin_detector=True):
    """The next-coarser grid of section 2.2.3 (all axes halved, voxel doubled)."""
    out = OrcGeom()
    src = _geom(g)
    _load().orc_coarse_geom(ctypes.byref(src), int(bool(bin_detector)), ctypes.byref(out))
    c = _Coarse()
    for name, _ in OrcGeom._fields_:
        if name != "angles":
            setattr(c, name, getattr(out, name))
    c.angles = getattr(g, "angles", None)
    return c


def restrict_sino(g_fine, proj):
    """2x2 detector binning (mean) of a fine sinogram."""
    proj = _f64(proj, _sino_shape(g_fine))
    out = np.empty((int(g_fine.n_views), (int(g_fine.nv) + 1) // 2, (int(g_fine.nu) + 1) // 2))
    _load().orc_restrict_sino(ctypes.byref(_geom(g_fine)), proj, out)
    return out


def prolong_vol(g_coarse, g_fine, vol):
    """Trilinear coarse-to-fine interpolation (section 2.2.3)."""
    vol = _f64(vol, _vol_shape(g_coarse))
    out = np.empty(_vol_shape(g_fine), np.float64)
    _load().orc_prolong_vol(ctypes.byref(_geom(g_coarse)), ctypes.byref(_geom(g_fine)), vol, out)
    return out


def _opts(lam, n_grids, iters, cgls_steps, framelet_levels, momentum, positivity, bin_detector,
          op_pair=0):
    it = list(iters) + [0] * (4 - len(iters))
    return OrcOpts(float(lam), int(n_grids), (ctypes.c_int32 * 4)(*it), int(cgls_steps),
                   int(framelet_levels), int(bool(momentum)), int(bool(positivity)),
                   int(bool(bin_detector)), int(op_pair))


def reconstruct(g, proj, lam, iters, cgls_steps=3, framelet_levels=1, momentum=True,
                positivity=True, bin_detector=True, op_pair=0):
    """Algorithm A2 (A1 if momentum is False) in the multigrid schedule of
    section 2.2.3; iters lists the outer iterations per grid, coarsest first;
    op_pair 1 takes the paper's Siddon / Eq. (3) operators.
    Returns (volume, report dict)."""
    proj = _f64(proj, _sino_shape(g))
    o = _opts(lam, len(iters), iters, cgls_steps, framelet_levels, momentum, positivity,
              bin_detector, op_pair)
    vol = np.empty(_vol_shape(g), np.float64)
    rep = OrcReport()
    rc = _load().orc_reconstruct(ctypes.byref(_geom(g)), ctypes.byref(o), proj, vol,
                                 ctypes.byref(rep))
    if rc != 0:
        raise ValueError("orc_reconstruct failed (%d)" % rc)
    return vol, {"resid2_last": rep.resid2_last, "cgls_breakdowns": rep.cgls_breakdowns,
                 "iters_done": list(rep.iters_done)}


def tf_iterations(g, proj, f0, n_iters, lam, cgls_steps=3, framelet_levels=1, momentum=True,
                  positivity=True, op_pair=0):
    """n_iters outer iterations of Algorithm A2 on one grid from f_cur = f_prev = f0."""
    proj = _f64(proj, _sino_shape(g))
    vol = np.array(f0, dtype=np.float64, order="C", copy=True)
    o = _opts(lam, 1, [n_iters], cgls_steps, framelet_levels, momentum, positivity, True,
              op_pair)
    rep = OrcReport()
    _load().orc_tf_iterations(ctypes.byref(_geom(g)), ctypes.byref(o), proj, int(n_iters), vol,
                              ctypes.byref(rep))
    return vol, {"resid2_last": rep.resid2_last, "cgls_breakdowns": rep.cgls_breakdowns}


# --------------------------------------------------------------------------
# The TV comparison method (section 2.3)
# --------------------------------------------------------------------------
TV_EPS = 1e-5       # smoothing of |d| (1/mm), about 0.05 % of soft tissue
TV_TOL = 1e-3       # the paper's 0.1 % stop
TV_MAX_STEPS = 100


def _tv(mu, eps=TV_EPS, tol=TV_TOL, max_steps=TV_MAX_STEPS):
    return OrcTV(float(mu), float(eps), float(tol), int(max_steps))


def tv_energy(x, f, mu, eps=TV_EPS):
    """||f - x||^2 + mu TV_eps(f) (the ROF energy of section 2.3)."""
    x = np.ascontiguousarray(x, np.float64)
    nz, ny, nx = x.shape
    return float(_load().orc_tv_energy(nx, ny, nz, ctypes.byref(_tv(mu, eps)), x,
                                       _f64(f, x.shape)))


def tv_gradient(x, f, mu, eps=TV_EPS):
    x = np.ascontiguousarray(x, np.float64)
    nz, ny, nx = x.shape
    out = np.empty_like(x)
    _load().orc_tv_gradient(nx, ny, nz, ctypes.byref(_tv(mu, eps)), x, _f64(f, x.shape), out)
    return out


def rof(x, mu, eps=TV_EPS, tol=TV_TOL, max_steps=TV_MAX_STEPS, history=False):
    """The ROF sub-problem by adaptive gradient descent from f = x.  Returns
    (f, accepted steps) or, with history, (f, steps, energies)."""
    x = np.ascontiguousarray(x, np.float64)
    nz, ny, nx = x.shape
    f = np.empty_like(x)
    hist = np.full(int(max_steps) + 1, np.nan)
    n = _load().orc_rof(nx, ny, nz, ctypes.byref(_tv(mu, eps, tol, max_steps)), x, f,
                        hist.ctypes.data_as(ctypes.c_void_p))
    if history:
        return f, int(n), hist[:n + 1]
    return f, int(n)


def reconstruct_tv(g, proj, mu, iters, cgls_steps=3, positivity=True, bin_detector=True,
                   eps=TV_EPS, tol=TV_TOL, max_steps=TV_MAX_STEPS):
    """The TV comparison method (x = CGLS(f), f = H(ROF(x))) in the multigrid
    schedule; returns (volume, report dict with the accepted ROF steps)."""
    proj = _f64(proj, _sino_shape(g))
    o = _opts(0.0, len(iters), iters, cgls_steps, 1, False, positivity, bin_detector)
    vol = np.empty(_vol_shape(g), np.float64)
    rep = OrcReport()
    steps = ctypes.c_int32(0)
    rc = _load().orc_reconstruct_tv(ctypes.byref(_geom(g)), ctypes.byref(o),
                                    ctypes.byref(_tv(mu, eps, tol, max_steps)), proj, vol,
                                    ctypes.byref(rep), ctypes.byref(steps))
    if rc != 0:
        raise ValueError("orc_reconstruct_tv failed (%d)" % rc)
    return vol, {"resid2_last": rep.resid2_last, "cgls_breakdowns": rep.cgls_breakdowns,
                 "iters_done": list(rep.iters_done), "rof_steps": int(steps.value)}


# --------------------------------------------------------------------------
# FDK, the comparison baseline (textbook Feldkamp-Davis-Kress)
# --------------------------------------------------------------------------
def ramlak(n, dp):
    """The Ram-Lak ramp kernel at integer lag n for spacing dp."""
    return float(_load().orc_ramlak(int(n), float(dp)))


def fdk_filter(g, proj):
    """Cosine-weighted, ramp-filtered projections (one row at a time)."""
    proj = _f64(proj, _sino_shape(g))
    out = np.empty_like(proj)
    _load().orc_fdk_filter(ctypes.byref(_geom(g)), proj, out)
    return out


def fdk_backproject(g, q):
    q = _f64(q, _sino_shape(g))
    vol = np.empty(_vol_shape(g), np.float64)
    _load().orc_fdk_backproject(ctypes.byref(_geom(g)), q, vol)
    return vol


def fdk(g, proj):
    """FDK reconstruction of an equally spaced full orbit."""
    if getattr(g, "angles", None) is not None:
        raise ValueError("FDK takes an equally spaced full orbit (angles None)")
    proj = _f64(proj, _sino_shape(g))
    vol = np.empty(_vol_shape(g), np.float64)
    if _load().orc_fdk(ctypes.byref(_geom(g)), proj, vol) != 0:
        raise ValueError("orc_fdk failed")
    return vol
