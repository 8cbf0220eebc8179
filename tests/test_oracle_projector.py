"""Pins of the oracle's projector P (Eq. (1), Joseph discretisation) and its
transpose P^T (Appendix 2, Eq. (A1); Eq. (3) as the continuous limit)."""
import math

import numpy as np
import pytest

import oracle
from brute import joseph_matrix
from paper_1008_2042_amd.inputs import Geometry, random_field

TINY = Geometry(6, 5, 4, 1.0, 1.2, 0.9, 8, 6, 1.4, 1.3, sad=30.0, sdd=45.0, n_views=3,
                angles=np.array([0.1, 1.2, 2.0 * math.pi * 5 / 8]))
TINY_EVEN = Geometry(4, 6, 3, 1.1, 0.9, 1.0, 7, 5, 1.6, 1.1, sad=25.0, sdd=40.0, n_views=4)


@pytest.mark.parametrize("g", [TINY, TINY_EVEN], ids=["odd-angles", "equispaced"])
def test_project_equals_brute_force_matrix(g):
    M = joseph_matrix(g)
    f = random_field(g.vol_shape, 1)
    got = oracle.project(g, f).ravel()
    np.testing.assert_allclose(got, M @ f.ravel(), rtol=0, atol=1e-12 * np.abs(M @ f.ravel()).max())
    assert np.count_nonzero(M) > 0


@pytest.mark.parametrize("g", [TINY, TINY_EVEN], ids=["odd-angles", "equispaced"])
def test_backproject_is_matrix_transpose(g):
    M = joseph_matrix(g)
    y = random_field(g.sino_shape, 2)
    got = oracle.backproject(g, y).ravel()
    ref = M.T @ y.ravel()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_adjoint_identity_c1_scale():
    g = Geometry(64, 64, 16, 1.0, 1.0, 1.0, 128, 64, 1.5, 1.5, n_views=30)
    f = random_field(g.vol_shape, 3, 0.0, 1.0)
    y = random_field(g.sino_shape, 4)
    lhs = float(np.vdot(oracle.project(g, f), y))
    rhs = float(np.vdot(f, oracle.backproject(g, y)))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + abs(rhs)) * 10


def test_constant_volume_closed_form():
    """f = 1 and rays that stay inside the grid: P f = N_step * d_step * |a| / |a_step|."""
    g = Geometry(33, 31, 33, 1.0, 1.1, 1.0, 5, 5, 0.3, 0.3, sad=500.0, sdd=750.0, n_views=5,
                 angles=np.array([0.0, 0.3, 1.0, 2.0, 4.0]))
    f = np.ones(g.vol_shape)
    got = oracle.project(g, f)
    for k, th in enumerate(g.angles):
        ct, st = math.cos(th), math.sin(th)
        step_x = abs(ct) >= abs(st) - 1e-12
        for r in range(g.nv):
            for c in range(g.nu):
                u = (c - 2) * g.du
                v = (r - 2) * g.dv
                a = np.array([-g.sdd * ct - u * st, -g.sdd * st + u * ct, v])
                if step_x:
                    want = g.nx * g.dx * np.linalg.norm(a) / abs(a[0])
                else:
                    want = g.ny * g.dy * np.linalg.norm(a) / abs(a[1])
                assert abs(got[k, r, c] - want) <= 1e-12 * want


@pytest.mark.parametrize("theta,axis", [(0.0, 0), (math.pi / 2, 1), (math.pi, 0)])
def test_axis_aligned_central_ray(theta, axis):
    """Odd grid, central pixel: the ray runs through voxel centres, so P f is
    the plain sum of one voxel row times the voxel size."""
    g = Geometry(9, 7, 5, 0.8, 1.3, 1.1, 5, 3, 1.0, 1.0, sad=100.0, sdd=150.0, n_views=1,
                 angles=np.array([theta]))
    f = random_field(g.vol_shape, 5, 0.0, 1.0)
    got = oracle.project(g, f)[0, 1, 2]
    if axis == 0:
        want = g.dx * f[2, 3, :].sum()
    else:
        want = g.dy * f[2, :, 4].sum()
    assert abs(got - want) <= 1e-12 * want


def _gaussian_case(sigma_vox):
    """Blob of fixed width sigma = 4 mm on a grid of voxel size sigma / sigma_vox."""
    sigma = 4.0
    h = sigma / sigma_vox
    n = int(math.ceil(5 * sigma_vox)) * 2 + 1
    g = Geometry(n, n, n, h, h, h, 9, 9, 2.0, 2.0, sad=400.0, sdd=600.0, n_views=3,
                 angles=np.array([0.2, 1.1, 2.6]))
    ctr = np.array([0.31, -0.17, 0.23])
    xs = (np.arange(n) - (n - 1) / 2.0) * h
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    f = np.exp(-((X - ctr[0]) ** 2 + (Y - ctr[1]) ** 2 + (Z - ctr[2]) ** 2) / (2 * sigma ** 2))
    got = oracle.project(g, f)
    err = []
    for k, th in enumerate(g.angles):
        ct, st = math.cos(th), math.sin(th)
        src = np.array([g.sad * ct, g.sad * st, 0.0])
        for r in range(g.nv):
            for c in range(g.nu):
                u = (c - (g.nu - 1) / 2.0) * g.du
                v = (r - (g.nv - 1) / 2.0) * g.dv
                a = np.array([-g.sdd * ct - u * st, -g.sdd * st + u * ct, v])
                d = np.linalg.norm(np.cross(ctr - src, a)) / np.linalg.norm(a)
                want = sigma * math.sqrt(2 * math.pi) * math.exp(-d * d / (2 * sigma ** 2))
                err.append((got[k, r, c] - want, want))
    e = np.array(err)
    return np.linalg.norm(e[:, 0]) / np.linalg.norm(e[:, 1])


def test_gaussian_blob_converges_second_order():
    """Line integrals of a Gaussian blob (closed form sigma sqrt(2 pi) exp(-d^2/2 sigma^2))."""
    e2 = _gaussian_case(2.0)   # sigma = 2 voxels: measured 2.6 %
    e4 = _gaussian_case(4.0)   # sigma = 4 voxels: measured 0.64 %
    assert e2 < 0.03 and e4 < 0.0075
    order = math.log(e2 / e4, 2)
    assert 1.8 < order < 2.2, (e2, e4, order)


def test_backproject_voxels_matches_full():
    g = Geometry(12, 10, 6, 1.0, 1.0, 1.5, 16, 8, 1.5, 1.5, sad=100.0, sdd=150.0, n_views=7)
    y = random_field(g.sino_shape, 6)
    full = oracle.backproject(g, y)
    kji = np.array([[0, 0, 0], [5, 9, 11], [2, 4, 6], [3, 7, 1], [1, 0, 11]])
    got = oracle.backproject_voxels(g, y, kji)
    want = full[kji[:, 0], kji[:, 1], kji[:, 2]]
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(full).max())


def test_project_rays_matches_full():
    g = Geometry(12, 10, 6, 1.0, 1.0, 1.5, 16, 8, 1.5, 1.5, sad=100.0, sdd=150.0, n_views=7)
    f = random_field(g.vol_shape, 7)
    full = oracle.project(g, f)
    vrc = np.array([[0, 0, 0], [6, 7, 15], [3, 4, 8], [5, 2, 9]])
    got = oracle.project_rays(g, f, vrc)
    np.testing.assert_array_equal(got, full[vrc[:, 0], vrc[:, 1], vrc[:, 2]])


def test_backprojection_continuous_limit_eq3():
    """On a smooth detector function the exact transpose approaches the
    closed form of Eq. (3): dx dy dz / (du dv) * L^3(u*) / (L0 l^2(x)) g(u*)."""
    g = Geometry(40, 40, 24, 0.5, 0.5, 0.5, 200, 160, 0.15, 0.15, sad=200.0, sdd=300.0,
                 n_views=1, angles=np.array([0.4]))
    uu = (np.arange(g.nu) - (g.nu - 1) / 2.0) * g.du
    vv = (np.arange(g.nv) - (g.nv - 1) / 2.0) * g.dv

    def gfun(u, v):
        return np.exp(-(u ** 2) / (2 * 6.0 ** 2) - (v - 1.0) ** 2 / (2 * 5.0 ** 2))

    y = gfun(uu[None, :], vv[:, None])[None]
    bp = oracle.backproject(g, y)
    th = g.angles[0]
    ct, st = math.cos(th), math.sin(th)
    src = np.array([g.sad * ct, g.sad * st, 0.0])
    rel = []
    for (k, j, i) in [(12, 20, 20), (8, 15, 25), (15, 27, 12), (11, 18, 23)]:
        x = np.array([(i - (g.nx - 1) / 2.0) * g.dx, (j - (g.ny - 1) / 2.0) * g.dy,
                      (k - (g.nz - 1) / 2.0) * g.dz])
        d = x - src
        n_det = -np.array([ct, st, 0.0])          # detector normal seen from the source
        t = g.sdd / float(d @ n_det)              # source + t d hits the detector plane
        hit = src + t * d
        det_c = -(g.sdd - g.sad) * np.array([ct, st, 0.0])
        u = float((hit - det_c) @ np.array([-st, ct, 0.0]))
        v = float(hit[2])
        L = np.linalg.norm(hit - src)
        l = np.linalg.norm(d)
        eq3 = g.dx * g.dy * g.dz / (g.du * g.dv) * L ** 3 / (g.sdd * l ** 2) * gfun(u, v)
        rel.append(abs(bp[k, j, i] - eq3) / eq3)
    assert max(rel) < 0.02, rel
