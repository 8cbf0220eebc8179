"""Image-quality protocols of the paper's section 3.2 on synthetic analogues.

The paper measures on a Catphan phantom and patient scans, which are not
available; these protocols run the same measurements on the seeded
paper-scale body phantom (512x512x70 at 0.5 x 0.5 x 2.5 mm, 40 views of a
512x384 detector) with a point-like object added:

* MTF (section 3.2): a ball of 0.28 mm diameter (the Catphan bead's size)
  at a voxel centre of the central slice, whose 21 x 21 patch holds only
  body background; reconstructions by the TF method, the TV method and FDK
  at the paper-scale dose (I0 = 1e5), and by TF and TV at 0.3x and 0.1x that
  dose (the paper's 1.0 / 0.3 / 0.1 mAs per projection); the MTF50 of each.
* CNR against the threshold (section 3.2): TF reconstructions with lambda
  from 3e-5 to 3e-3 at 0.1x the paper-scale dose, the mean CNR of the four
  bone inserts against the surrounding body.
* Short scan: 40 views over 200 degrees (the Catphan scan's arc) against 40
  over 360, TF method, relative RMS error against the voxelised phantom
  inside the body.

Every reconstruction runs through the C-ABI library (tfcb); this module only
generates inputs and evaluates images on the host.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List

import numpy as np

from paper_1008_2042_amd import inputs, metrics, tfcb

POINT_RADIUS = 0.14   # mm: the 0.28 mm bead of section 3.2
POINT_RHO = 5.0       # 1/mm: the bead's added attenuation (a dense metal)
DOSES = (1e5, 3e4, 1e4)  # I0 for 1.0 / 0.3 / 0.1 of the paper-scale dose
LAMBDAS = (3e-5, 1e-4, 3e-4, 1e-3, 3e-3)
CNR_DOSE = 1e4        # the CNR sweep runs at 0.1x dose, where noise sets the optimum
TV_MU = 5e-4


def _centres(n: int, d: float) -> np.ndarray:
    return (np.arange(n) - 0.5 * (n - 1)) * d


def place_point(g, ells) -> tuple:
    """A voxel centre on the central slice whose 21 x 21 patch (plus a 2 mm
    margin) lies inside the body and clear of every insert: (k, j, i) and
    its position in mm."""
    k = g.nz // 2
    z = _centres(g.nz, g.dz)[k]
    xs, ys = _centres(g.nx, g.dx), _centres(g.ny, g.dy)
    half = 10.5 * max(g.dx, g.dy) + 2.0
    body = ells[0]
    for j in range(g.ny // 2, g.ny - 11):
        for i in list(range(g.nx // 2, g.nx - 11, 8)):
            x, y = xs[i], ys[j]
            corners = [(x + a, y + b) for a in (-half, half) for b in (-half, half)]
            if any((cx / body.axes[0]) ** 2 + (cy / body.axes[1]) ** 2 + (z / body.axes[2]) ** 2
                   > 1.0 for cx, cy in corners):
                continue
            clear = True
            for e in ells[1:]:
                r = max(e.axes[0], e.axes[1])
                if (abs(e.center[2] - z) < e.axes[2] + 1.0
                        and math.hypot(e.center[0] - x, e.center[1] - y) < r + half * 1.5):
                    clear = False
                    break
            if clear:
                return (k, j, i), (float(x), float(y), float(z))
    raise RuntimeError("no clear position for the point object")


def cnr_insert(vol: np.ndarray, g, ells, index: int) -> float:
    """CNR of insert `index` (its ellipsoid shrunk to 0.6x) against the body
    (inside the body ellipsoid shrunk to 0.9x, outside every insert grown to
    1.4x), over the slices the insert's ROI reaches."""
    roi = metrics._inside(g, ells[index], 0.6)
    bg = metrics._inside(g, ells[0], 0.9)
    for e in ells[1:]:
        bg &= ~metrics._inside(g, e, 1.4)
    zs = np.nonzero(roi.any(axis=(1, 2)))[0]
    sl = np.zeros(g.nz, bool)
    sl[zs] = True
    bg &= sl[:, None, None]
    return metrics.cnr(vol, roi, bg)


def _data(g, ells, i0, seed, dev):
    clean = inputs.analytic_projection_torch(g, ells, dev)
    return inputs.poisson_log_torch(clean, i0, seed).float().contiguous()


def run(device=None, cfg_name: str = "paper") -> Dict:
    import torch
    dev = device or torch.device("cuda:0")
    cfg = inputs.config(cfg_name)
    g = cfg["geom"]
    lam, iters = cfg["lam"], cfg["iters"]
    ells = inputs.phantom_for(cfg)
    (k, j, i), pos = place_point(g, ells)
    point = inputs.Ellipsoid(pos, (POINT_RADIUS,) * 3, 0.0, POINT_RHO)
    with_point = ells + [point]
    out: Dict = {"workload": "paper-scale body phantom + a 0.28 mm bead at (%.2f, %.2f, %.2f) mm"
                 % pos, "point_voxel": [k, j, i]}

    def recon(y, method, lam_=lam, geom=g):
        if method == "fdk":
            return tfcb.fdk(geom, y).cpu().numpy()
        vol, _ = tfcb.reconstruct(geom, y, lam_ if method == "tf" else TV_MU, iters,
                                  cfg["cgls_steps"], cfg["framelet_levels"],
                                  regulariser=1 if method == "tv" else 0)
        return vol.cpu().numpy()

    # MTF by method and dose
    mtf: Dict[str, Dict] = {}
    for d, i0 in enumerate(DOSES):
        y = _data(g, with_point, i0, 7000 + d, dev)
        for method in (("tf", "tv", "fdk") if d == 0 else ("tf", "tv")):
            v = recon(y, method)
            f, m = metrics.mtf(v[k], (j, i), g.dx)
            mtf["%s_dose%.1f" % (method, i0 / DOSES[0])] = {
                "mtf50_cycles_per_mm": round(metrics.mtf50(f, m), 4),
                "mtf": [round(float(x), 4) for x in m]}
        del y
    out["mtf"] = mtf
    out["mtf_frequencies_cycles_per_mm"] = [round(float(x), 4) for x in
                                            np.arange(11) / (21 * g.dx)]
    # CNR of the bone inserts against lambda (TF), at the low dose
    y = _data(g, ells, CNR_DOSE, 7100, dev)
    bones = [n for n, e in enumerate(ells) if n > 0 and e.rho > 0.01]
    sweep = []
    for lam_ in LAMBDAS:
        v = recon(y, "tf", lam_)
        sweep.append({"lambda": lam_, "cnr_bone_mean": round(float(np.mean(
            [cnr_insert(v, g, ells, n) for n in bones])), 3)})
    out["cnr_vs_lambda"] = sweep
    out["cnr_dose_i0"] = CNR_DOSE
    # short scan: 40 views over 200 degrees against the full orbit
    truth = inputs.voxelize(g, ells, ss=2)
    body = metrics._inside(g, ells[0], 1.0)
    rr = {}
    for name, ang in (("full_360", None),
                      ("short_200", np.linspace(0.0, math.radians(200.0), g.n_views))):
        gs = dataclasses.replace(g, angles=ang)
        ys = _data(gs, ells, DOSES[0], 7200, dev)
        v = recon(ys, "tf", geom=gs)
        rr[name] = round(metrics.rrms(v[body], truth[body]), 4)
    out["rrms_in_body_tf"] = rr
    out["note"] = ("MTF: 21x21 patch, background = the patch's outer ring, ring-averaged FFT "
                   "amplitude; CNR background = body minus inserts grown 1.4x; truth voxelised "
                   "with 2^3 sub-samples")
    return out


if __name__ == "__main__":
    import json
    print(json.dumps(run()))
