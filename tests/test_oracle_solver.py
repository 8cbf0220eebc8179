"""Pins of the oracle's CGLS (Appendix 1), Algorithm A2 (section 2.1) and the
multigrid transfer operators and schedule (section 2.2.3)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from brute import framelet_matrix, joseph_matrix, shrink_dense
from paper_1008_2042_amd.inputs import Geometry, random_field

TINY = Geometry(6, 5, 4, 1.0, 1.2, 0.9, 8, 6, 1.4, 1.3, sad=30.0, sdd=45.0, n_views=3,
                angles=np.array([0.1, 1.2, 2.0 * math.pi * 5 / 8]))

with open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")) as _fh:
    GOLD = json.load(_fh)


def _krylov_minimiser(P, x0, y, n):
    """argmin ||P x - y|| over x0 + K_n(P^T P, P^T r0), by an explicit basis
    and numpy's least squares."""
    r0 = y - P @ x0
    vecs = [P.T @ r0]
    for _ in range(n - 1):
        vecs.append(P.T @ (P @ vecs[-1]))
    B, _ = np.linalg.qr(np.array(vecs).T)
    coef, *_ = np.linalg.lstsq(P @ B, r0, rcond=None)
    return x0 + B @ coef


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_cgls_is_krylov_least_squares(n):
    P = joseph_matrix(TINY)
    x0 = random_field(TINY.vol_shape, 21, 0.0, 0.02)
    y = random_field(TINY.sino_shape, 22, 0.0, 1.0)
    x, broke, r2 = oracle.cgls(TINY, x0, y, n)
    want = _krylov_minimiser(P, x0.ravel(), y.ravel(), n)
    assert not broke
    np.testing.assert_allclose(x.ravel(), want, rtol=0, atol=1e-10 * np.abs(want).max())
    assert r2 == pytest.approx(float(np.sum((y.ravel() - P @ x.ravel()) ** 2)), rel=1e-10)


def test_cgls_residual_never_increases():
    y = random_field(TINY.sino_shape, 23, 0.0, 1.0)
    x0 = np.zeros(TINY.vol_shape)
    _, _, _, hist = oracle.cgls(TINY, x0, y, 8, history=True)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])
    assert hist[-1] < hist[0]


def test_cgls_square_full_rank_reaches_lstsq():
    g = Geometry(3, 3, 2, 1.0, 1.0, 1.0, 6, 4, 1.0, 1.0, sad=20.0, sdd=30.0, n_views=2,
                 angles=np.array([0.3, 1.9]))
    P = joseph_matrix(g)
    assert np.linalg.matrix_rank(P) == g.nx * g.ny * g.nz
    y = random_field(g.sino_shape, 24, 0.0, 1.0)
    want, *_ = np.linalg.lstsq(P, y.ravel(), rcond=None)
    # exact arithmetic needs N = 18 steps; in floating point the Krylov
    # vectors lose orthogonality, so allow 3N
    x, _, _ = oracle.cgls(g, np.zeros(g.vol_shape), y, 54)
    np.testing.assert_allclose(x.ravel(), want, rtol=0, atol=1e-10 * np.abs(want).max())


def test_cgls_breakdown_guard_on_consistent_start():
    f = random_field(TINY.vol_shape, 25, 0.0, 0.02)
    y = oracle.project(TINY, f)
    x, broke, r2 = oracle.cgls(TINY, f, y, 3)
    assert broke and r2 == 0.0
    np.testing.assert_array_equal(x, f)


# -------------------------------------------------------------- multigrid
def test_coarse_geometry():
    g = Geometry(512, 512, 70, 0.5, 0.5, 2.5, 512, 384, 0.776, 0.776, n_views=40)
    c = oracle.coarse_geom(g, True)
    assert (c.nx, c.ny, c.nz, c.nu, c.nv) == (256, 256, 35, 256, 192)
    assert (c.dx, c.dy, c.dz, c.du, c.dv) == (1.0, 1.0, 5.0, 1.552, 1.552)
    c2 = oracle.coarse_geom(c, False)
    assert (c2.nx, c2.nz, c2.nu, c2.du) == (128, 18, 256, 1.552)


def test_restrict_constant_and_linear():
    g = Geometry(8, 8, 4, 1.0, 1.0, 1.0, 10, 6, 0.7, 0.9, n_views=3)
    u = (np.arange(g.nu) - (g.nu - 1) / 2.0) * g.du
    v = (np.arange(g.nv) - (g.nv - 1) / 2.0) * g.dv
    lin = 0.3 + 0.05 * u[None, None, :] - 0.02 * v[None, :, None] + 0 * np.arange(3)[:, None, None]
    out = oracle.restrict_sino(g, lin)
    uc = (np.arange(5) - 2.0) * 2 * g.du
    vc = (np.arange(3) - 1.0) * 2 * g.dv
    want = 0.3 + 0.05 * uc[None, None, :] - 0.02 * vc[None, :, None] + 0 * np.arange(3)[:, None, None]
    np.testing.assert_allclose(out, want, atol=1e-14)
    np.testing.assert_allclose(oracle.restrict_sino(g, np.full(g.sino_shape, 1.7)), 1.7, atol=1e-15)
    # odd detector: last row / column average only the pixels that exist
    g2 = Geometry(8, 8, 4, 1.0, 1.0, 1.0, 5, 3, 0.7, 0.9, n_views=1)
    y = random_field(g2.sino_shape, 26)
    o2 = oracle.restrict_sino(g2, y)
    assert o2.shape == (1, 2, 3)
    assert o2[0, 1, 2] == y[0, 2, 4]
    assert o2[0, 0, 2] == pytest.approx((y[0, 0, 4] + y[0, 1, 4]) / 2, abs=1e-15)


@pytest.mark.parametrize("fine_shape", [(8, 10, 12), (7, 9, 5), (2, 3, 1)])
def test_prolong_is_clamped_trilinear(fine_shape):
    nz, ny, nx = fine_shape
    fine = Geometry(nx, ny, nz, 0.5, 0.6, 1.5, 8, 8, 1.0, 1.0)
    co = oracle.coarse_geom(fine, True)
    c = random_field((co.nz, co.ny, co.nx), 27)
    got = oracle.prolong_vol(co, fine, c)
    # scipy's order-1 map_coordinates at the clamped coarse fractional index
    def idx(n_f, d_f, n_c, d_c):
        p = (np.arange(n_f) - (n_f - 1) / 2.0) * d_f
        return np.clip(p / d_c + (n_c - 1) / 2.0, 0, n_c - 1)
    zi = idx(nz, fine.dz, co.nz, co.dz)
    yi = idx(ny, fine.dy, co.ny, co.dy)
    xi = idx(nx, fine.dx, co.nx, co.dx)
    Z, Y, X = np.meshgrid(zi, yi, xi, indexing="ij")
    want = ndi.map_coordinates(c, [Z, Y, X], order=1, mode="nearest")
    np.testing.assert_allclose(got, want, atol=1e-14)


def test_prolong_reproduces_linear_fields():
    fine = Geometry(12, 10, 8, 0.5, 0.5, 1.0, 8, 8, 1.0, 1.0)
    co = oracle.coarse_geom(fine, True)
    def field(nx, ny, nz, dx, dy, dz):
        x = (np.arange(nx) - (nx - 1) / 2.0) * dx
        y = (np.arange(ny) - (ny - 1) / 2.0) * dy
        z = (np.arange(nz) - (nz - 1) / 2.0) * dz
        return 0.1 + 0.01 * x[None, None, :] - 0.02 * y[None, :, None] + 0.03 * z[:, None, None]
    got = oracle.prolong_vol(co, fine, field(co.nx, co.ny, co.nz, co.dx, co.dy, co.dz))
    want = field(fine.nx, fine.ny, fine.nz, fine.dx, fine.dy, fine.dz)
    # interior (fine centres whose coarse index is not clamped)
    np.testing.assert_allclose(got[1:-1, 1:-1, 1:-1], want[1:-1, 1:-1, 1:-1], atol=1e-14)
    np.testing.assert_allclose(oracle.prolong_vol(co, fine, np.full((co.nz, co.ny, co.nx), 2.5)),
                               2.5, atol=1e-15)


# ------------------------------------------------------------ Algorithm A2
def _cgls_dense(P, x, y, n):
    """Textbook CGLS (Appendix 1) on an explicit matrix, n products q = P p."""
    r = y - P @ x
    s = P.T @ r
    p = s.copy()
    gamma = s @ s
    for l in range(n):
        q = P @ p
        delta = q @ q
        if gamma <= 1e-300 or delta <= 1e-300:
            break
        a = gamma / delta
        x = x + a * p
        r = r - a * q
        if l < n - 1:
            s = P.T @ r
            gnew = s @ s
            p = s + (gnew / gamma) * p
            gamma = gnew
    return x


def _a2_dense(P, W, shape, y, f0, iters, lam, n, momentum=True, positivity=True):
    coef = GOLD["a2_momentum"]["coefficient"]
    f_prev = f0.copy()
    f_cur = f0.copy()
    for k in range(iters):
        c = coef[k] if momentum else 0.0
        v = f_cur + c * (f_cur - f_prev)
        x = _cgls_dense(P, v, y, n)
        a = shrink_dense((W @ x).reshape((27,) + shape), lam)
        f_new = W.T @ a.ravel()
        if positivity:
            f_new = np.maximum(f_new, 0.0)
        f_prev, f_cur = f_cur, f_new
    return f_cur


@pytest.mark.parametrize("momentum", [True, False])
def test_a2_single_grid_brute_force(momentum):
    P = joseph_matrix(TINY)
    W = framelet_matrix(TINY.vol_shape)
    truth = random_field(TINY.vol_shape, 28, 0.0, 0.03)
    y = P @ truth.ravel() + random_field(TINY.sino_shape, 29, -1e-3, 1e-3).ravel()
    want = _a2_dense(P, W, TINY.vol_shape, y, np.zeros(truth.size), 5, 2e-3, 2, momentum)
    got, rep = oracle.reconstruct(TINY, y.reshape(TINY.sino_shape), 2e-3, [5], cgls_steps=2,
                                  momentum=momentum)
    np.testing.assert_allclose(got.ravel(), want, rtol=0, atol=1e-11 * np.abs(want).max())
    assert rep["iters_done"][0] == 5


def test_a2_two_grids_brute_force():
    fine = Geometry(8, 6, 4, 1.0, 1.0, 1.0, 10, 6, 1.5, 1.5, sad=40.0, sdd=60.0, n_views=4)
    coarse = Geometry(4, 3, 2, 2.0, 2.0, 2.0, 5, 3, 3.0, 3.0, sad=40.0, sdd=60.0, n_views=4)
    Pf, Pc = joseph_matrix(fine), joseph_matrix(coarse)
    Wf, Wc = framelet_matrix(fine.vol_shape), framelet_matrix(coarse.vol_shape)
    truth = random_field(fine.vol_shape, 30, 0.0, 0.03)
    y = (Pf @ truth.ravel()).reshape(fine.sino_shape)
    yc = y.reshape(4, 3, 2, 5, 2).mean(axis=(2, 4))  # 2x2 binning
    lam = 1e-3
    fc = _a2_dense(Pc, Wc, coarse.vol_shape, yc.ravel(), np.zeros(coarse.nx * coarse.ny * coarse.nz),
                   3, lam, 3)
    def idx(n_f, n_c):
        p = np.arange(n_f) - (n_f - 1) / 2.0
        return np.clip(p / 2.0 + (n_c - 1) / 2.0, 0, n_c - 1)
    Z, Y, X = np.meshgrid(idx(4, 2), idx(6, 3), idx(8, 4), indexing="ij")
    f0 = ndi.map_coordinates(fc.reshape(coarse.vol_shape), [Z, Y, X], order=1, mode="nearest")
    want = _a2_dense(Pf, Wf, fine.vol_shape, y.ravel(), f0.ravel(), 4, lam, 3)
    got, rep = oracle.reconstruct(fine, y, lam, [3, 4], cgls_steps=3)
    np.testing.assert_allclose(got.ravel(), want, rtol=0, atol=1e-11 * np.abs(want).max())
    assert rep["iters_done"][:2] == [3, 4]


def test_exact_nonnegative_solution_is_a_fixed_point():
    """lambda = 0: if P f* = g and f* >= 0, CGLS breaks down at once, W^T W = I
    and H keep f*, so A2 returns f* from f* (invariant)."""
    f = random_field(TINY.vol_shape, 31, 0.0, 0.02)
    y = oracle.project(TINY, f)
    got, rep = oracle.tf_iterations(TINY, y, f, 4, 0.0)
    np.testing.assert_allclose(got, f, rtol=0, atol=1e-15)
    # the first CGLS sees r = 0 exactly; later ones see W^T W rounding only
    assert rep["cgls_breakdowns"] >= 1


def test_golden_momentum_sequence_closed_form():
    """Every entry of the A2 table against Algorithm A2's recursion, and the
    recursion against its closed forms: t(1) = (1 + sqrt 5) / 2, and each
    t(k+1) is the positive root of t^2 - t = t(k)^2 (the quadratic the
    update solves), so t(k+1)^2 - t(k+1) - t(k)^2 = 0."""
    t = GOLD["a2_momentum"]["t"]
    c = GOLD["a2_momentum"]["coefficient"]
    assert len(t) == len(c) >= 6
    t_prev, t_cur = 1.0, 1.0
    for k in range(len(t)):
        assert t[k] == pytest.approx(t_cur, rel=1e-15, abs=0)
        assert c[k] == pytest.approx((t_prev - 1.0) / t_cur, rel=1e-15, abs=1e-300)
        t_prev, t_cur = t_cur, 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t_cur * t_cur))
    assert t[1] == pytest.approx((1 + math.sqrt(5)) / 2, abs=1e-15)
    for k in range(len(t) - 1):
        assert t[k + 1] ** 2 - t[k + 1] - t[k] ** 2 == pytest.approx(0.0, abs=1e-13)
    assert c[0] == 0.0 and c[1] == 0.0
    assert c[2] == pytest.approx(0.281753, abs=1e-6) and c[3] == pytest.approx(0.434043, abs=1e-6)
    assert c[4] == pytest.approx(0.531064, abs=1e-6)
