"""Pins of the oracle's FDK baseline (the comparison reconstruction of the
paper's section 3; textbook Feldkamp-Davis-Kress): the Ram-Lak kernel
against the integral that defines it, the ramp filter's zero response to a
constant, and whole reconstructions of analytic balls (density, position,
background) under exact chord data."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_1008_2042_amd import inputs
from paper_1008_2042_amd.inputs import Ellipsoid, Geometry


@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 10, 25])
def test_ramlak_is_the_band_limited_ramp(n):
    """h(n dp) = integral over |w| <= 1/(2 dp) of |w| exp(2 pi i w n dp) dw."""
    dp = 0.37
    W = 1.0 / (2.0 * dp)
    val, _ = integrate.quad(lambda w: 2.0 * w * math.cos(2.0 * math.pi * w * n * dp), 0.0, W,
                            limit=200, epsabs=1e-13, epsrel=1e-13)
    assert oracle.ramlak(n, dp) == pytest.approx(val, rel=1e-9, abs=1e-12 / dp ** 2)
    assert oracle.ramlak(-n, dp) == oracle.ramlak(n, dp)


def test_ramp_filter_removes_a_constant():
    """The ramp filter's DC response is zero: h(0) + 2 sum_{n odd} h(n) = 0, so
    a long constant row filters to nearly zero in its middle (the tail of
    the sum beyond the row, 2 sum_{odd n > N} 1/(pi n dp)^2, is all that is
    left).  A detector far from the source keeps the cosine weight at 1."""
    nu = 2001
    g = Geometry(2, 2, 1, 1.0, 1.0, 1.0, nu, 1, 1.0, 1.0, sad=1e7, sdd=2e7, n_views=1)
    q = oracle.fdk_filter(g, np.ones(g.sino_shape))
    dp = g.du * g.sad / g.sdd
    mid = q[0, 0, nu // 2]
    tail = sum(2.0 / (math.pi * n * dp) ** 2 for n in range(nu // 2 + 1, 400001, 2))
    assert mid * (1.0 / (4.0 * dp)) ** -1 < 2e-3  # against the kernel's own DC scale
    assert mid == pytest.approx(dp * tail, rel=2e-2)


def _ball_geometry():
    return Geometry(64, 64, 32, 1.0, 1.0, 1.0, 160, 96, 1.0, 1.0, sad=300.0, sdd=450.0,
                    n_views=240)


def test_fdk_reconstructs_a_centred_ball():
    """A uniform ball of radius 20 mm (density 0.02) at the isocentre, exact
    chord data: inside (r < 14 mm, central slices) FDK gives the density
    within 2 %, outside (r > 26 mm) under 3 % of it."""
    g = _ball_geometry()
    rho = 0.02
    y = inputs.analytic_projection(g, [Ellipsoid((0.0, 0.0, 0.0), (20.0, 20.0, 20.0), 0.0, rho)])
    f = oracle.fdk(g, y)
    z, yy, x = np.meshgrid(*[(np.arange(n) - 0.5 * (n - 1)) * d
                             for n, d in ((g.nz, g.dz), (g.ny, g.dy), (g.nx, g.dx))],
                           indexing="ij")
    r = np.sqrt(x * x + yy * yy + z * z)
    inner = (r < 14.0) & (np.abs(z) < 4.0)
    outer = (r > 26.0) & (np.abs(z) < 4.0) & (np.sqrt(x * x + yy * yy) < 30.0)
    assert abs(f[inner].mean() - rho) < 0.02 * rho
    assert np.abs(f[inner] - rho).max() < 0.05 * rho
    assert np.abs(f[outer]).max() < 0.03 * rho


def test_fdk_places_an_offset_ball():
    """A small ball off the axis reconstructs where it is: the density-weighted
    centroid of the reconstruction lies within 0.1 mm of the ball's centre
    (this fixes the orientation of the orbit and detector axes)."""
    g = _ball_geometry()
    c = (11.0, -7.0, 3.0)
    y = inputs.analytic_projection(g, [Ellipsoid(c, (5.0, 5.0, 5.0), 0.0, 0.02)])
    f = oracle.fdk(g, y)
    z, yy, x = np.meshgrid(*[(np.arange(n) - 0.5 * (n - 1)) * d
                             for n, d in ((g.nz, g.dz), (g.ny, g.dy), (g.nx, g.dx))],
                           indexing="ij")
    w = np.where(f > 0.3 * f.max(), f, 0.0)
    cen = [float((w * a).sum() / w.sum()) for a in (x, yy, z)]
    np.testing.assert_allclose(cen, c, atol=0.1)


def test_fdk_is_linear():
    g = Geometry(16, 12, 6, 1.0, 1.0, 1.0, 24, 10, 1.2, 1.2, sad=80.0, sdd=120.0, n_views=9)
    a = inputs.random_sino(g, 31)
    b = inputs.random_sino(g, 32)
    fa, fb = oracle.fdk(g, a), oracle.fdk(g, b)
    np.testing.assert_allclose(oracle.fdk(g, 2.0 * a - 3.0 * b), 2.0 * fa - 3.0 * fb,
                               rtol=0, atol=1e-12 * np.abs(fa).max())
    with pytest.raises(ValueError):
        g2 = Geometry(16, 12, 6, 1.0, 1.0, 1.0, 24, 10, 1.2, 1.2, sad=80.0, sdd=120.0,
                      n_views=9, angles=np.linspace(0, 3, 9))
        oracle.fdk(g2, a)
