#!/usr/bin/env python3
"""Writes tests/golden/paper_recon_oracle.npz: sampled voxels of the FP64
oracle's reconstruction of the paper-scale workload.

The workload is the 512x512x70 case (0.5 x 0.5 x 2.5 mm voxels, 40 views of
a 512x384 detector at 0.776 mm, SAD 1000 / SDD 1500 mm, 20-ellipsoid body
phantom, Poisson I0 = 1e5) reconstructed by Algorithm A2 in the two-grid
schedule of section 2.2.3 with 16 + 24 outer iterations, 3 CGLS steps each,
a one-level framelet and lambda = 5e-4 /mm.  The data are the seeded
analytic projections of the input generator; the reconstruction is the
oracle's alone (this script imports nothing from the GPU package but the
input generator, which holds none of the method's arithmetic).

Stored (all indices [z][y][x]):
  slices_k      the z indices of the full slices kept
  slices        those slices, rounded to float32 (rounding 6e-8 relative,
                far below the 1e-3 parity tolerance)
  voxels_kji    4096 voxels drawn uniformly (seed 9102) with their exact
  voxels        FP64 values
  resid2_last   ||g - P x||^2 after the last CGLS update of the run
  meta          JSON: workload, schedule, threads, seconds, numpy version

Run:  python tests/golden/make_paper_golden.py   (about 45 min on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "paper_recon_oracle.npz")
SLICES = (10, 35, 60)
N_VOXELS = 4096
VOXEL_SEED = 9102


def main(out_path: str = OUT, full_volume_path: str | None = None) -> None:
    import oracle
    from paper_1008_2042_amd import inputs

    cfg = inputs.config("paper")
    g = cfg["geom"]
    t0 = time.time()
    y = inputs.measured_data(cfg)
    t_data = time.time() - t0
    print("data: %s in %.1f s" % (y.shape, t_data), flush=True)
    t0 = time.time()
    vol, rep = oracle.reconstruct(g, y, cfg["lam"], cfg["iters"], cfg["cgls_steps"],
                                  cfg["framelet_levels"])
    t_rec = time.time() - t0
    print("oracle reconstruction: %.1f s, resid2 %.6e" % (t_rec, rep["resid2_last"]), flush=True)
    rng = np.random.default_rng(VOXEL_SEED)
    kji = np.stack([rng.integers(0, g.nz, N_VOXELS), rng.integers(0, g.ny, N_VOXELS),
                    rng.integers(0, g.nx, N_VOXELS)], axis=1).astype(np.int32)
    meta = {"workload": "paper-scale 512x512x70, 40 views, 512x384 detector, Poisson I0=1e5",
            "iters": cfg["iters"], "cgls_steps": cfg["cgls_steps"],
            "framelet_levels": cfg["framelet_levels"], "lambda": cfg["lam"],
            "oracle_threads": oracle.num_threads(), "oracle_seconds": round(t_rec, 1),
            "numpy": np.__version__, "script": "tests/golden/make_paper_golden.py"}
    np.savez_compressed(out_path, slices_k=np.array(SLICES, np.int32),
                        slices=vol[list(SLICES)].astype(np.float32), voxels_kji=kji,
                        voxels=vol[kji[:, 0], kji[:, 1], kji[:, 2]],
                        resid2_last=np.float64(rep["resid2_last"]),
                        meta=np.array(json.dumps(meta)))
    print("wrote", out_path, flush=True)
    if full_volume_path:
        np.save(full_volume_path, vol)


if __name__ == "__main__":
    main(*(sys.argv[1:3]))
