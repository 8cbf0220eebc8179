"""Pins of the oracle's TV comparison method (section 2.3): the smoothed TV
energy against closed forms, its gradient against finite differences, the
ROF descent against an independent minimiser and against the closed-form
solution of a piecewise-constant step, the descent and stop rules, and the
TV reconstruction schedule against explicit matrices."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.optimize as so

import oracle
from brute import joseph_matrix
from paper_1008_2042_amd.inputs import Geometry, random_field

TINY = Geometry(6, 5, 4, 1.0, 1.2, 0.9, 8, 6, 1.4, 1.3, sad=30.0, sdd=45.0, n_views=3,
                angles=np.array([0.1, 1.2, 2.0 * math.pi * 5 / 8]))


def _n_differences(shape):
    nz, ny, nx = shape
    return (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)


def test_energy_closed_forms():
    """Constant f = c against x = 0: V c^2 + mu eps (number of difference
    terms).  A ramp of slope a along x: the x terms are sqrt(a^2 + eps^2)
    each, the others eps.  Data term alone (mu = 0): ||f - x||^2."""
    shape = (3, 4, 5)
    mu, eps = 0.7, 1e-3
    x = np.zeros(shape)
    f = np.full(shape, 0.25)
    want = f.size * 0.0625 + mu * eps * _n_differences(shape)
    assert oracle.tv_energy(x, f, mu, eps) == pytest.approx(want, rel=1e-14)
    a = 0.3
    ramp = np.broadcast_to(a * np.arange(5.0), shape).copy()
    n_x = 4 * 4 * 3
    want = float(np.sum(ramp ** 2)) + mu * (n_x * math.sqrt(a * a + eps * eps)
                                            + eps * (_n_differences(shape) - n_x))
    assert oracle.tv_energy(x, ramp, mu, eps) == pytest.approx(want, rel=1e-14)
    r = random_field(shape, 1)
    s = random_field(shape, 2)
    assert oracle.tv_energy(r, s, 0.0, eps) == pytest.approx(float(np.sum((s - r) ** 2)),
                                                            rel=1e-14)


@pytest.mark.parametrize("shape", [(4, 5, 6), (1, 3, 7), (2, 1, 1)])
def test_gradient_matches_finite_differences(shape):
    x = random_field(shape, 3, 0.0, 0.05)
    f = random_field(shape, 4, 0.0, 0.05)
    mu, eps = 0.03, 0.02
    g = oracle.tv_gradient(x, f, mu, eps)
    h = 1e-6
    num = np.empty_like(f)
    for idx in np.ndindex(shape):
        fp, fm = f.copy(), f.copy()
        fp[idx] += h
        fm[idx] -= h
        num[idx] = (oracle.tv_energy(x, fp, mu, eps) - oracle.tv_energy(x, fm, mu, eps)) / (2 * h)
    np.testing.assert_allclose(g, num, rtol=0, atol=1e-7 * np.abs(num).max())


def test_rof_reaches_the_minimiser_of_an_independent_solver():
    """The smoothed ROF energy is strictly convex: its minimiser is unique.
    With a tight stop the descent reaches the one scipy's L-BFGS finds from
    the same energy and gradient."""
    shape = (4, 5, 6)
    x = random_field(shape, 5, 0.0, 0.05)
    mu, eps = 0.01, 2e-3
    f, n = oracle.rof(x, mu, eps, tol=1e-13, max_steps=20000)
    res = so.minimize(lambda v: oracle.tv_energy(x, v.reshape(shape), mu, eps), x.ravel(),
                      jac=lambda v: oracle.tv_gradient(x, v.reshape(shape), mu, eps).ravel(),
                      method="L-BFGS-B", options=dict(ftol=1e-16, gtol=1e-14, maxiter=20000))
    want = res.x.reshape(shape)
    assert np.linalg.norm(f - want) <= 1e-5 * np.linalg.norm(want)
    assert oracle.tv_energy(x, f, mu, eps) <= res.fun * (1 + 1e-10)


def test_rof_step_closed_form():
    """A step along x (constant in y and z), a on n1 voxels and b on n2.
    At the minimiser the gradient of each plateau sums to zero, and the TV
    terms inside a plateau telescope to the one across the jump J, so the
    plateau means move by exactly mu psi(J) / (2 n1) and mu psi(J) / (2 n2),
    psi(J) = J / sqrt(J^2 + eps^2), for any eps.  As eps -> 0 the plateaus
    turn flat at a + mu / (2 n1) and b - mu / (2 n2), the unsmoothed ROF
    solution of a two-level signal."""
    n1, n2, a, b, mu = 4, 6, 0.1, 1.1, 0.2
    x = np.zeros((2, 3, n1 + n2))
    x[..., :n1] = a
    x[..., n1:] = b
    flat = np.concatenate([np.full(n1, a + mu / (2 * n1)), np.full(n2, b - mu / (2 * n2))])
    dev = []
    for eps in (1e-2, 1e-3):
        f, n = oracle.rof(x, mu, eps, tol=1e-15, max_steps=20000)
        J = f[..., n1] - f[..., n1 - 1]
        psi = J / np.sqrt(J * J + eps * eps)
        np.testing.assert_allclose(f[..., :n1].mean(-1) - a, mu * psi / (2 * n1), rtol=1e-4)
        np.testing.assert_allclose(b - f[..., n1:].mean(-1), mu * psi / (2 * n2), rtol=1e-4)
        dev.append(float(np.abs(f - flat).max()))
    assert dev[1] <= 3e-3 and dev[1] <= 0.4 * dev[0], dev


def test_rof_descent_and_stop_rules():
    """Every accepted step lowers the energy; the descent ends at the first
    step whose relative decrease is under tol (0.1 %), or at the cap."""
    x = random_field((6, 8, 9), 6, 0.0, 0.04)
    f, n, e = oracle.rof(x, 0.004, 1e-5, history=True)
    assert n >= 2
    rel = -np.diff(e) / e[:-1]
    assert np.all(rel > 0)
    assert rel[-1] < 1e-3 and np.all(rel[:-1] >= 1e-3)
    assert oracle.tv_energy(x, f, 0.004, 1e-5) == pytest.approx(e[-1], rel=1e-14)
    f2, n2 = oracle.rof(x, 0.004, 1e-5, max_steps=1)
    assert n2 == 1
    # no regularisation: f = x already minimises, nothing moves
    f0, n0 = oracle.rof(x, 0.0)
    assert n0 == 0 and np.array_equal(f0, x)


def _cgls_dense(P, x, y, n):
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


def _tv_dense(P, shape, y, f0, iters, mu, n):
    """The TV outer iteration with an explicit P: x = CGLS(f); f = H(ROF(x))
    (the ROF sub-problem is the pinned oracle.rof)."""
    f = f0.copy()
    steps = 0
    for _ in range(iters):
        x = _cgls_dense(P, f, y, n)
        r, k = oracle.rof(x.reshape(shape), mu)
        steps += k
        f = np.maximum(r.ravel(), 0.0)
    return f, steps


# The two sides sum the CGLS products in different orders (dense matrix
# products here, loops in the oracle); the ROF descent with eps = 1e-5 then
# magnifies those 1e-16 differences about a thousandfold, hence 1e-8.
def test_tv_single_grid_brute_force():
    P = joseph_matrix(TINY)
    truth = random_field(TINY.vol_shape, 7, 0.0, 0.03)
    y = P @ truth.ravel() + random_field(TINY.sino_shape, 8, -1e-3, 1e-3).ravel()
    mu = 2e-3
    want, steps = _tv_dense(P, TINY.vol_shape, y, np.zeros(truth.size), 4, mu, 2)
    got, rep = oracle.reconstruct_tv(TINY, y.reshape(TINY.sino_shape), mu, [4], cgls_steps=2)
    np.testing.assert_allclose(got.ravel(), want, rtol=0, atol=1e-8 * np.abs(want).max())
    assert rep["rof_steps"] == steps and rep["iters_done"][0] == 4


def test_tv_two_grids_brute_force():
    fine = Geometry(8, 6, 4, 1.0, 1.0, 1.0, 10, 6, 1.5, 1.5, sad=40.0, sdd=60.0, n_views=4)
    coarse = Geometry(4, 3, 2, 2.0, 2.0, 2.0, 5, 3, 3.0, 3.0, sad=40.0, sdd=60.0, n_views=4)
    Pf, Pc = joseph_matrix(fine), joseph_matrix(coarse)
    truth = random_field(fine.vol_shape, 9, 0.0, 0.03)
    y = (Pf @ truth.ravel()).reshape(fine.sino_shape)
    yc = y.reshape(4, 3, 2, 5, 2).mean(axis=(2, 4))
    mu = 1e-3
    fc, s1 = _tv_dense(Pc, coarse.vol_shape, yc.ravel(), np.zeros(4 * 3 * 2), 2, mu, 3)

    def idx(n_f, n_c):
        p = np.arange(n_f) - (n_f - 1) / 2.0
        return np.clip(p / 2.0 + (n_c - 1) / 2.0, 0, n_c - 1)
    Z, Y, X = np.meshgrid(idx(4, 2), idx(6, 3), idx(8, 4), indexing="ij")
    f0 = ndi.map_coordinates(fc.reshape(coarse.vol_shape), [Z, Y, X], order=1, mode="nearest")
    want, s2 = _tv_dense(Pf, fine.vol_shape, y.ravel(), f0.ravel(), 3, mu, 3)
    got, rep = oracle.reconstruct_tv(fine, y, mu, [2, 3], cgls_steps=3)
    np.testing.assert_allclose(got.ravel(), want, rtol=0, atol=1e-8 * np.abs(want).max())
    assert rep["rof_steps"] == s1 + s2
