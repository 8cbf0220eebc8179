"""The closed form the fused GPU framelet kernel evaluates, checked on the CPU
against the literal 27-band oracle (section 2.1 filters, Eq. (2) shrinkage).

The 3 x 3 filter matrix H[l][m] = h_l[m] of the piecewise-linear frame has
orthogonal columns, sum_l h_l[m] h_l[k] = c_m [m == k] with c = h0.  For the
tensor-product bank that gives, with K the separable h0 smoothing and s the
per-position shrink factor,
    W^T T W f = f K(s) + K(L - s alpha_0),   sum_b (W_b f)^2 = K(f^2),
and the high-band energy as a sum of weighted variances.  These tests pin
that reading: the Gram matrix from the printed filters, and the closed form
(written here in plain FP64 numpy, sharing nothing with the oracle) against
the oracle's analysis / shrink / synthesis on random and smooth fields."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1008_2042_amd.inputs import random_field

_SCALE = {"1/4": 0.25, "sqrt(2)/4": math.sqrt(2.0) / 4.0}


def _filters():
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")) as fh:
        h = json.load(fh)["framelet_filters"]
    return [np.array(h[n]["taps"], np.float64) * _SCALE[h[n]["scale"]] for n in ("h0", "h1", "h2")]


def test_filter_gram_matrix_is_h0_diagonal():
    H = np.stack(_filters())  # rows l, columns m = -1, 0, +1
    np.testing.assert_allclose(H.T @ H, np.diag(_filters()[0]), atol=1e-16)


def _smooth(a, axis, d):
    n = a.shape[axis]
    lo = np.take(a, range(0, n - 2 * d), axis=axis)
    mid = np.take(a, range(d, n - d), axis=axis)
    hi = np.take(a, range(2 * d, n), axis=axis)
    return 0.25 * (lo + hi) + 0.5 * mid


def _level(f, lam, d, low=None):
    """One level of W^T T W f in closed form (half-sample symmetric edges)."""
    fe = np.pad(f, 2 * d, mode="symmetric")
    b0 = _smooth(_smooth(fe, 2, d), 1, d)  # xy low band, margin d in x, y and 2d in z
    nz, ny, nx = b0.shape
    w = {-1: 0.25, 0: 0.5, 1: 0.25}
    e = np.zeros_like(b0)  # xy high-band energy = weighted variance around b0
    for my in (-1, 0, 1):
        for mx in (-1, 0, 1):
            fk = fe[:, d + my * d:d + my * d + ny, d + mx * d:d + mx * d + nx]
            e += w[my] * w[mx] * (fk - b0) ** 2
    bo, bm, bn = b0[:-2 * d], b0[d:-d], b0[2 * d:]
    a00 = 0.25 * (bo + bn) + 0.5 * bm
    a01 = math.sqrt(2.0) / 4.0 * (bn - bo)
    a02 = 0.5 * bm - 0.25 * (bo + bn)
    n2 = 0.25 * (e[:-2 * d] + e[2 * d:]) + 0.5 * e[d:-d] + a01 ** 2 + a02 ** 2
    nrm = np.sqrt(n2)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(nrm <= lam, 0.0, 1.0 - lam / nrm)
    L = a00 if low is None else np.pad(low, d, mode="symmetric")
    K = lambda g: _smooth(_smooth(_smooth(g, 0, d), 1, d), 2, d)
    return f * K(s) + K(L - s * a00)


def _closed_form(f, lam, levels, positivity):
    low = None
    if levels == 2:
        fe = np.pad(f, 1, mode="symmetric")
        low = _level(_smooth(_smooth(_smooth(fe, 0, 1), 1, 1), 2, 1), lam, 2)
    out = _level(f, lam, 1, low)
    return np.where(out < 0, 0.0, out) if positivity else out


@pytest.mark.parametrize("shape", [(9, 14, 15), (1, 5, 7), (2, 1, 3), (3, 17, 31)])
@pytest.mark.parametrize("levels", [1, 2])
def test_closed_form_equals_oracle(shape, levels):
    f = random_field(shape, 23, 0.0, 0.03)
    for lam in (0.0, 4e-3):
        for pos in (True, False):
            want = oracle.framelet_shrink(f, lam, levels, pos)
            got = _closed_form(f, lam, levels, pos)
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("levels", [1, 2])
def test_closed_form_smooth_field(levels):
    """Smooth data (tiny high-band energy next to a large mean): the variance
    form keeps its accuracy where K(f^2) - K(f)^2 would cancel."""
    z, y, x = np.meshgrid(np.arange(12), np.arange(20), np.arange(21), indexing="ij")
    f = 0.02 + 1e-4 * np.sin(x / 7.0) * np.cos(y / 5.0) + 1e-5 * z
    for lam in (1e-6, 1e-5):
        want = oracle.framelet_shrink(f, lam, levels, False)
        got = _closed_form(f, lam, levels, False)
        assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)
