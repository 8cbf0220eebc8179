"""Host-side arithmetic of the benchmark line: the plane-sample count that
prices the projector's roofline, and the per-kernel fractions."""
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1008_2042_amd import inputs  # noqa: E402
from paper_1008_2042_amd.inputs import Geometry  # noqa: E402


def _brute_samples(g):
    """Count (ray, plane) samples with at least one tap inside the grid by
    walking every ray's planes one at a time (the projector's own window
    rule: 0 < tau < 1, trans index in (-1, nt), z index in (-1, nz))."""
    th = g.view_angles()
    n = 0
    for k in range(g.n_views):
        cs, sn = math.cos(th[k]), math.sin(th[k])
        sx, sy = g.sad * cs, g.sad * sn
        step_x = abs(cs) >= abs(sn) - 1e-12
        for c in range(g.nu):
            u = (c - 0.5 * (g.nu - 1)) * g.du
            ax, ay = -g.sdd * cs - u * sn, -g.sdd * sn + u * cs
            if step_x:
                a_s, a_t, s_s, s_t, ns, nt, ds, dt = ax, ay, sx, sy, g.nx, g.ny, g.dx, g.dy
            else:
                a_s, a_t, s_s, s_t, ns, nt, ds, dt = ay, ax, sy, sx, g.ny, g.nx, g.dy, g.dx
            for r in range(g.nv):
                vz = (r - 0.5 * (g.nv - 1)) * g.dv / g.dz
                for p in range(ns):
                    tau = ((p - 0.5 * (ns - 1)) * ds - s_s) / a_s
                    t = (s_t + tau * a_t) / dt + 0.5 * (nt - 1)
                    z = tau * vz + 0.5 * (g.nz - 1)
                    if 0 < tau < 1 and -1 < t < nt and -1 < z < g.nz:
                        n += 1
    return n


def test_plane_samples_matches_brute_force():
    g = Geometry(12, 10, 6, 1.5, 1.7, 2.0, 20, 9, 1.6, 1.9, n_views=7)
    assert bench.plane_samples(g) == _brute_samples(g)


def test_kernel_fractions_arithmetic():
    g = inputs.config("paper")["geom"]
    samples = 3_000_000_000
    avg_ms = [1.5, 1.0, 0.1]
    copy = 5.0e12
    fr = bench.kernel_fractions(g, avg_ms, samples, copy)
    V = g.nx * g.ny * g.nz * 4.0
    S = g.n_views * g.nu * g.nv * 4.0
    p = fr[bench.KERNEL_NAMES[0]]
    assert p["compulsory_bytes"] == int(V + S)
    assert np.isclose(p["hbm_frac_compulsory"], (V + S) / 1.5e-3 / 8e12, atol=1e-4)
    assert np.isclose(p["hbm_frac_compulsory_vs_copy"], (V + S) / 1.5e-3 / copy, atol=1e-4)
    # 16 bytes of taps per sample against 64 B/clk/CU on 256 CUs at 2.4 GHz
    assert p["tap_bytes"] == 16 * samples
    assert np.isclose(p["vl1d_frac_tap_bytes"], 16.0 * samples / 1.5e-3 / (64 * 256 * 2.4e9),
                      atol=1e-4)
    w = fr[bench.KERNEL_NAMES[2]]
    assert w["compulsory_bytes"] == int(16 * g.nx * g.ny * g.nz)
    assert "tap_bytes" not in w
