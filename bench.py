#!/usr/bin/env python3
"""Benchmark of the TF-regularised CBCT reconstruction on one MI355X.

One step = one full reconstruction of the paper-scale workload through the
C-ABI: 512x512x70 volume (0.5 x 0.5 x 2.5 mm), 40 views over 360 degrees,
512x384 flat detector (0.776 mm), SAD 1000 / SDD 1500 mm, a 20-ellipsoid
seeded phantom with Poisson noise (I0 = 1e5), 2-grid multigrid with 16 + 24
outer iterations of Algorithm A2, 3 CGLS steps each, 1-level framelet,
lambda = 5e-4 /mm.  Projections are resident in HBM before timing starts;
the volume is written to HBM.

Prints ONE JSON line (rank 0) with the metric, the roofline of the dominant
kernel (event-timed live in the timed steps on the launching stream) and
the FP64 oracle's CPU baseline on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TF iterations/s + s/recon at 512²×70 (FP32 vs FP16-store); serving p99 latency"
PEAK_FP32_VECTOR_TFLOPS = 157.3  # MI355X: 256 CU x 2.4 GHz x 256 FP32 flop/clk/CU
FLOPS_PER_SAMPLE = 16.0          # algorithmic work of one (ray, plane) sample
VL1D_BYTES_PER_CLK_CU = 64.0     # vector L1 peak per CU and clock (the CDNA3 figure)
KERNEL_NAMES = ["P (k_project)", "P^T (k_backproject)", "framelet (k_framelet)"]
KERNEL_SOURCES = ["project.hip", "backproject.hip", "framelet.hip"]
TV_MU = 5e-4  # mu_TV of the TV comparison run (1/mm), tuned by hand as the paper does


def plane_samples(g) -> int:
    """Number of (ray, plane) samples of the Joseph projector with at least
    one tap inside the grid: per ray, the planes p of its stepping axis with
    0 < tau_p < 1, trans index in (-1, N_trans) and z index in (-1, N_z).
    This is the unit count of one P (and one P^T) application."""
    import numpy as np
    th = g.view_angles()
    cs, sn = np.cos(th), np.sin(th)
    step_x = np.abs(cs) >= np.abs(sn) - 1e-12
    u = (np.arange(g.nu) - 0.5 * (g.nu - 1)) * g.du
    vz = ((np.arange(g.nv) - 0.5 * (g.nv - 1)) * g.dv / g.dz)[None, :]

    def window(c0, c1, lo, hi, plo, phi):
        # p with lo < c0 + c1 p < hi (c1 != 0), intersected with (plo, phi)
        a, b = (lo - c0) / c1, (hi - c0) / c1
        return np.maximum(plo, np.minimum(a, b)), np.minimum(phi, np.maximum(a, b))

    total = 0
    for k in range(g.n_views):
        ax = -g.sdd * cs[k] - u * sn[k]
        ay = -g.sdd * sn[k] + u * cs[k]
        sx, sy = g.sad * cs[k], g.sad * sn[k]
        if step_x[k]:
            a_s, a_t, s_s, s_t, ns, nt, ds, dtr = ax, ay, sx, sy, g.nx, g.ny, g.dx, g.dy
        else:
            a_s, a_t, s_s, s_t, ns, nt, ds, dtr = ay, ax, sy, sx, g.ny, g.nx, g.dy, g.dx
        tau0 = (-0.5 * (ns - 1) * ds - s_s) / a_s                     # per column
        dtau = ds / a_s
        t0 = (s_t + tau0 * a_t) / dtr + 0.5 * (nt - 1)
        dt = dtau * a_t / dtr
        lo, hi = window(tau0, dtau, 0.0, 1.0, -1.0, float(ns))
        lo, hi = window(t0, dt, -1.0, float(nt), lo, hi)
        zc = 0.5 * (g.nz - 1)
        lo2, hi2 = window(tau0[:, None] * vz + zc, np.where(vz == 0, 1e-300, dtau[:, None] * vz),
                          -1.0, float(g.nz), lo[:, None], hi[:, None])
        n = np.ceil(hi2) - np.floor(lo2) - 1.0
        total += int(np.sum(np.maximum(n, 0.0)))
    return total


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1008_2042_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_idx: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current source of that kernel; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    ent = t.get(KERNEL_SOURCES[kernel_idx])
    if not ent or ent.get("source_hash") != source_hash([KERNEL_SOURCES[kernel_idx]]):
        return None
    return ent.get("bytes_per_launch")


def _host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _timed(fn, reps=1):
    """Median wall time of reps calls after one untimed warm-up call when
    reps > 1 (a single call is timed cold)."""
    if reps > 1:
        fn()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(sorted(ts)[len(ts) // 2])


def cpu_baseline(cfg, y):
    """The FP64 oracle, as it stands, on this host's cores.

    Measured on the paper-scale workload: one outer TF iteration (3 CGLS
    steps + framelet shrink) on its coarse grid (256x256x35, 40 views of
    256x192 binned data) and one on its fine grid (512x512x70, 40 x 512x384);
    the reconstruction time is 16 x coarse + 24 x fine from those two
    measured numbers (the prolongation and restriction are negligible).
    Also single applications of P, P^T and the framelet shrink on the fine
    grid, and on the 64x64x16 tiny workload the same operators (median of 3)
    and its whole 10-iteration reconstruction."""
    import numpy as np
    import oracle
    from paper_1008_2042_amd import inputs
    g = cfg["geom"]
    lam, n = cfg["lam"], cfg["cgls_steps"]
    gc = oracle.coarse_geom(g, True)
    yc = oracle.restrict_sino(g, y)
    t_c = _timed(lambda: oracle.tf_iterations(gc, yc, np.zeros((gc.nz, gc.ny, gc.nx)), 1, lam, n))
    t_f = _timed(lambda: oracle.tf_iterations(g, y, np.zeros(g.vol_shape), 1, lam, n))
    f = inputs.random_volume(g, 1)
    ops = {"P_s": _timed(lambda: oracle.project(g, f)),
           "PT_s": _timed(lambda: oracle.backproject(g, y)),
           "framelet_s": _timed(lambda: oracle.framelet_shrink(f, lam))}
    tiny = inputs.config("tiny")
    gt = tiny["geom"]
    yt = inputs.measured_data(tiny)
    ft = inputs.random_volume(gt, 2)
    tiny_ops = {"P_s": _timed(lambda: oracle.project(gt, ft), 3),
                "PT_s": _timed(lambda: oracle.backproject(gt, yt), 3),
                "framelet_s": _timed(lambda: oracle.framelet_shrink(ft, lam), 3),
                "recon_s": _timed(lambda: oracle.reconstruct(gt, yt, lam, tiny["iters"]), 3)}
    n_c, n_f = cfg["iters"]
    recon_s = n_c * t_c + n_f * t_f
    return {"value": round((n_c + n_f) / recon_s, 6), "unit": "TF iterations/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "one outer TF iteration of each grid of this workload, measured: coarse "
                      "256x256x35 %.2f s, fine 512x512x70 %.2f s; the 16+24 schedule is "
                      "16 x %.2f + 24 x %.2f = %.0f s per reconstruction"
                      % (t_c, t_f, t_c, t_f, recon_s),
            "s_per_recon": round(recon_s, 1),
            "coarse_iteration_s": round(t_c, 3), "fine_iteration_s": round(t_f, 3),
            "operators_512x512x70_s": {k: round(v, 3) for k, v in ops.items()},
            "tiny_64x64x16_s": {k: round(v, 4) for k, v in tiny_ops.items()},
            "host": {"cpu_model": _host_cpu_model(), "nproc": os.cpu_count(),
                     "omp_threads": oracle.num_threads()}}


LARGE_WORKLOAD = ("large single TF reconstruction: 512x512x256 volume at 0.5 mm, 360 views, "
                  "1024x768 detector at 0.388 mm, 3-grid multigrid 5+10+15 iterations, "
                  "3 CGLS steps, 2-level framelet, lambda 5e-4, 40-ellipsoid phantom, "
                  "Poisson I0=5e4")


def large_data(cfg, dev):
    """283 M rays: exact chords evaluated on the device in FP64, then Poisson
    noise, stored FP32."""
    from paper_1008_2042_amd import inputs
    clean = inputs.analytic_projection_torch(cfg["geom"], inputs.phantom_for(cfg), dev)
    yd = inputs.poisson_log_torch(clean, cfg["noise"][0], cfg["noise"][1]).float()
    del clean
    return yd


def load_counters(kernel_idx: int):
    """The committed counter figures of a kernel (traffic.json), if they were
    taken on its current source; else {}."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        t = json.load(fh)
    ent = t.get(KERNEL_SOURCES[kernel_idx])
    if not ent or ent.get("source_hash") != source_hash([KERNEL_SOURCES[kernel_idx]]):
        return {}
    return ent


def copy_bandwidth(dev, nbytes: int = 1 << 30) -> float:
    """Achieved rate of a plain device copy, read + write bytes per second:
    a 1 GiB device-to-device tensor copy, median of 5 after one untimed
    call.  The reference for the compulsory-byte fractions."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del src, dst
    return 2.0 * nbytes / sorted(ts)[2]


def kernel_fractions(g, avg_ms, samples, copy_Bps=None):
    """Per kernel of the fine grid: the HBM fraction of its compulsory bytes
    (P: volume + projections; P^T: the same; framelet: 16 B per voxel in
    FP32), against the 8 TB/s peak and against the measured rate of a plain
    device copy; for P and P^T the algorithmic tap bytes (4 taps of 4 bytes
    per sample, the gathers a matrix-free design must make) against the
    vector L1 peak of 64 B per clock per CU (256 CUs at 2.4 GHz; the kernels
    here take their taps from LDS, so this is the gather rate they stand in
    for); the HBM-side traffic rate from the committed counters, and the
    VALU instruction rate per CU and 2.4 GHz clock (SQ_INSTS_VALU per launch
    over 256 CUs x 2.4e9 x the launch's duration).  Non-packed FP32 code
    issues about one wave instruction per CU-clock, but the counter is a
    rate, not a bound: the 512x512x256 projector measures 1.13."""
    V, S = g.nx * g.ny * g.nz * 4.0, g.n_views * g.nu * g.nv * 4.0
    compulsory = [V + S, V + S, 16.0 * g.nx * g.ny * g.nz]
    vl1d_peak = VL1D_BYTES_PER_CLK_CU * 256 * 2.4e9
    out = {}
    for i, name in enumerate(KERNEL_NAMES):
        t = avg_ms[i] * 1e-3
        if t <= 0:
            continue
        ent = load_counters(i)
        d = {"compulsory_bytes": int(compulsory[i]),
             "hbm_frac_compulsory": round(compulsory[i] / t / 8e12, 4)}
        if copy_Bps:
            d["hbm_frac_compulsory_vs_copy"] = round(compulsory[i] / t / copy_Bps, 4)
        if i in (0, 1):
            d["tap_bytes"] = int(16 * samples)
            d["vl1d_frac_tap_bytes"] = round(16.0 * samples / t / vl1d_peak, 4)
        if ent.get("bytes_per_launch"):
            d["traffic_bytes"] = ent["bytes_per_launch"]
            d["traffic_GBps"] = round(ent["bytes_per_launch"] / t / 1e9, 1)
            d["traffic_frac_of_8TBps"] = round(ent["bytes_per_launch"] / t / 8e12, 4)
        if ent.get("valu_insts_per_launch"):
            d["valu_insts_per_launch"] = ent["valu_insts_per_launch"]
            d["valu_insts_per_cu_clock"] = round(ent["valu_insts_per_launch"] / t / (256 * 2.4e9), 4)
            if i == 0:
                d["lane_valu_per_sample"] = round(64.0 * ent["valu_insts_per_launch"] / samples, 2)
        out[name] = d
    return out


def with_transfers(g, yd, cfg, dev, reps: int = 3) -> dict:
    """Seconds per reconstruction when the projections start in pinned host
    memory and the volume ends there: the host-to-device copy, the
    reconstruction (FP32 storage) and the device-to-host copy, on one
    stream, median of reps after one untimed run."""
    import torch
    from paper_1008_2042_amd import tfcb
    h_proj = torch.empty(yd.shape, dtype=torch.float32, pin_memory=True)
    h_proj.copy_(yd.cpu())
    h_vol = torch.empty(g.vol_shape, dtype=torch.float32, pin_memory=True)
    d_proj = torch.empty_like(yd)
    d_vol = torch.empty(g.vol_shape, dtype=torch.float32, device=dev)
    opts = tfcb.options(cfg["lam"], cfg["iters"], cfg["cgls_steps"], cfg["framelet_levels"])
    ws = torch.empty(tfcb.workspace_size(g, opts), dtype=torch.uint8, device=dev)

    def once():
        d_proj.copy_(h_proj, non_blocking=True)
        tfcb.reconstruct(g, d_proj, cfg["lam"], cfg["iters"], cfg["cgls_steps"],
                         cfg["framelet_levels"], out=d_vol, ws=ws)
        h_vol.copy_(d_vol, non_blocking=True)
        torch.cuda.synchronize()

    once()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        once()
        ts.append(time.perf_counter() - t0)
    # the two copies alone, event-timed
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    d_proj.copy_(h_proj, non_blocking=True)
    e[1].record()
    h_vol.copy_(d_vol, non_blocking=True)
    e[2].record()
    torch.cuda.synchronize()
    out = {"s_per_recon": round(float(sorted(ts)[len(ts) // 2]), 4),
           "h2d_projections_ms": round(e[0].elapsed_time(e[1]), 3),
           "d2h_volume_ms": round(e[1].elapsed_time(e[2]), 3),
           "note": "projections from pinned host memory, volume back to pinned host memory, "
                   "median of %d" % reps}
    del ws, d_proj, d_vol
    return out


def oracle_samples_error(vol):
    """Relative L2 error of a paper-scale GPU volume against the FP64
    oracle's full-schedule reconstruction at its stored samples (three
    z-slices and 4096 random voxels, tests/golden/paper_recon_oracle.npz,
    written by tests/golden/make_paper_golden.py), or None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "paper_recon_oracle.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    v = vol.double().cpu().numpy()
    ks = [int(k) for k in z["slices_k"]]
    kji = z["voxels_kji"]
    got = np.concatenate([v[ks].ravel(), v[kji[:, 0], kji[:, 1], kji[:, 2]]])
    want = np.concatenate([z["slices"].astype(np.float64).ravel(), z["voxels"]])
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f16", action="store_true", help="skip the FP16/BF16-storage runs")
    ap.add_argument("--no-pair", action="store_true",
                    help="skip the run with the paper's own operators (Siddon P, Eq. (3) P^T)")
    ap.add_argument("--no-tv", action="store_true",
                    help="skip the TV comparison method (section 2.3) in the same schedule")
    ap.add_argument("--quality", type=int, default=1, choices=[0, 1],
                    help="run the image-quality protocols of section 3.2 (MTF, CNR against "
                         "lambda, short scan) on the paper workload")
    ap.add_argument("--serving", type=int, default=64, metavar="N",
                    help="requests in the serving measurement (0 = skip; 64 = the full mix)")
    ap.add_argument("--large", type=int, default=1, choices=[0, 1],
                    help="with the paper workload, also time the large workload once in FP32 "
                         "and FP16 storage (config.large)")
    ap.add_argument("--workload", default="paper", choices=["paper", "large"],
                    help="paper: 512x512x70, 40 views (default); large: 512x512x256, "
                         "360 views of 1024x768, 3 grids, 2-level framelet")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the reconstruction runs on a single MI355X; "
              "multi-GPU sharding is a design note, not a measured path (got --gpus %d, "
              "WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1008_2042_amd import inputs, tfcb

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    tfcb.load()
    cfg = inputs.config(args.workload)
    g = cfg["geom"]
    if args.workload == "paper":
        y = inputs.measured_data(cfg)
        yd = torch.tensor(y, dtype=torch.float32, device=dev)
        workload = ("paper-scale TF reconstruction: 512x512x70 volume at 0.5x0.5x2.5 mm, 40 "
                    "views, 512x384 detector at 0.776 mm, 2-grid multigrid 16+24 iterations, "
                    "3 CGLS steps, 1-level framelet, lambda 5e-4, 20-ellipsoid phantom, "
                    "Poisson I0=1e5")
    else:
        yd = large_data(cfg, dev)
        y = None
        args.no_cpu_baseline = True
        args.large = 0
        workload = LARGE_WORKLOAD
    n_iters = sum(cfg["iters"])

    def run(storage, steps, warmup, profile, op_pair=0, cfg=cfg, yd=yd, regulariser=0):
        g = cfg["geom"]
        lam = TV_MU if regulariser else cfg["lam"]
        opts = tfcb.options(lam, cfg["iters"], cfg["cgls_steps"], cfg["framelet_levels"],
                            storage=storage, profile=profile, op_pair=op_pair,
                            regulariser=regulariser)
        ws = torch.empty(tfcb.workspace_size(g, opts), dtype=torch.uint8, device=dev)
        out = torch.empty(g.vol_shape, dtype=torch.float32, device=dev)
        kw = dict(cgls_steps=cfg["cgls_steps"], framelet_levels=cfg["framelet_levels"],
                  storage=storage, out=out, ws=ws, op_pair=op_pair, regulariser=regulariser)
        for _ in range(warmup):
            tfcb.reconstruct(g, yd, lam, cfg["iters"], **kw)
        reps = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, rep = tfcb.reconstruct(g, yd, lam, cfg["iters"], profile=profile, **kw)
            reps.append(rep)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        del ws
        return out.clone(), dt, reps

    vol32, dt32, reps = run(tfcb.F32, args.steps, args.warmup, True)
    ms_per_step = dt32 / args.steps * 1e3
    value = n_iters * args.steps / dt32

    # per-kernel averages over the timed steps (finest grid launches)
    kms = np.sum([r["kernel_ms"] for r in reps], axis=0)
    kn = np.sum([r["kernel_launches"] for r in reps], axis=0)
    avg_ms = [float(kms[i] / kn[i]) if kn[i] else 0.0 for i in range(3)]
    dom = int(np.argmax(kms[:3]))
    samples = plane_samples(g)
    copy_Bps = copy_bandwidth(dev)
    roofline = None
    if dom in (0, 1):
        flops = samples * FLOPS_PER_SAMPLE
        achieved = flops / (avg_ms[dom] * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 3),
                    "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                    "traffic": load_traffic(dom), "kernel": KERNEL_NAMES[dom],
                    "avg_launch_ms": round(avg_ms[dom], 4),
                    "units_per_launch": samples, "flops_per_unit": FLOPS_PER_SAMPLE,
                    # the build emits no packed FP32 instructions, so the vector
                    # peak it can reach is half the published one
                    "frac_of_nonpacked_peak": round(achieved / (PEAK_FP32_VECTOR_TFLOPS / 2), 4)}
    else:
        nbytes = g.nx * g.ny * g.nz * 16.0
        achieved = nbytes / (avg_ms[dom] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0,
                    "unit": "GB/s", "frac": round(achieved / 8000.0, 4),
                    "traffic": load_traffic(dom), "kernel": KERNEL_NAMES[dom],
                    "avg_launch_ms": round(avg_ms[dom], 4)}

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "TF iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload,
                   "s_per_recon": round(ms_per_step / 1e3, 4),
                   "iterations_per_recon": n_iters,
                   "fine_grid_iters_per_s": round(cfg["iters"][-1] / np.mean(
                       [r["seconds_per_grid"][len(cfg["iters"]) - 1] for r in reps]), 3),
                   "coarse_grid_iters_per_s": round(cfg["iters"][0] / np.mean(
                       [r["seconds_per_grid"][0] for r in reps]), 3),
                   "kernel_avg_ms": {KERNEL_NAMES[i]: round(avg_ms[i], 4) for i in range(3)},
                   "copy_GBps": round(copy_Bps / 1e9, 1),
                   "kernel_fractions": kernel_fractions(g, avg_ms, samples, copy_Bps),
                   "kernel_share_fine_grid": {
                       n: round(float(kms[i] / max(np.sum(kms), 1e-30)), 3)
                       for i, n in enumerate(KERNEL_NAMES + ["other"])},
                   "paper_context": "about 5 min for 512x512x70 on a Tesla C1060 "
                                    "(different voxel size and 3-grid schedule; context only)"},
        "roofline": roofline,
    }
    if args.workload == "paper":
        line["config"]["rel_l2_vs_oracle_samples"] = oracle_samples_error(vol32)
        line["config"]["with_host_transfers"] = with_transfers(g, yd, cfg, dev)
    if not args.no_f16:
        for name, code in (("f16_storage", tfcb.F16), ("bf16_storage", tfcb.BF16)):
            volh, dth, _ = run(code, args.steps, 1, False)
            a = volh.double()
            b = vol32.double()
            line["config"][name] = {
                "value": round(n_iters * args.steps / dth, 3), "unit": "TF iterations/s",
                "ms_per_step": round(dth / args.steps * 1e3, 3),
                "rel_l2_vs_f32": float(torch.linalg.norm(a - b) / torch.linalg.norm(b))}
            if args.workload == "paper":
                line["config"][name]["rel_l2_vs_oracle_samples"] = oracle_samples_error(volh)
    if not args.no_pair:
        # the paper's own operators in the same schedule (section 2.2.1, Eq. (3))
        volp, dtp, repp = run(tfcb.F32, args.steps, 1, True, op_pair=1)
        kp = np.sum([r["kernel_ms"] for r in repp], axis=0)
        kpn = np.sum([r["kernel_launches"] for r in repp], axis=0)
        a = volp.double()
        b = vol32.double()
        line["config"]["paper_pair"] = {
            "value": round(n_iters * args.steps / dtp, 3), "unit": "TF iterations/s",
            "ms_per_step": round(dtp / args.steps * 1e3, 3),
            "kernel_avg_ms": {n: round(float(kp[i] / kpn[i]) if kpn[i] else 0.0, 4)
                              for i, n in enumerate(["P (k_project_siddon)",
                                                     "P^T (k_backproject_eq3)",
                                                     "framelet (k_framelet)"])},
            "rel_l2_vs_joseph_pair": float(torch.linalg.norm(a - b) / torch.linalg.norm(b))}
    if not args.no_tv:
        # the paper's comparison method (section 2.3) in the same schedule
        volt, dtt, rept = run(tfcb.F32, args.steps, 1, True, regulariser=1)
        kt = np.sum([r["kernel_ms"] for r in rept], axis=0)
        ktn = np.sum([r["kernel_launches"] for r in rept], axis=0)
        ng = len(cfg["iters"])
        line["config"]["tv"] = {
            "mu_tv": TV_MU, "value": round(n_iters * args.steps / dtt, 3),
            "unit": "TV iterations/s", "ms_per_step": round(dtt / args.steps * 1e3, 3),
            "s_per_iteration_by_grid_coarse_to_fine": [
                round(float(np.mean([r["seconds_per_grid"][i] for r in rept])) / cfg["iters"][i],
                      5) for i in range(ng)],
            "tf_s_per_iteration_by_grid_coarse_to_fine": [
                round(float(np.mean([r["seconds_per_grid"][i] for r in reps])) / cfg["iters"][i],
                      5) for i in range(ng)],
            "rof_steps_per_recon": float(np.mean([r["rof_steps"] for r in rept])),
            "rof_ms_per_iteration_fine_grid": round(float(kt[2] / max(ktn[2], 1)), 4),
            "note": "the paper reports TV/TF time per iteration 1.8/1.1, 5.1/4.1 and 17.7/15.2 s "
                    "on its three grids (C1060)"}
    if args.quality and args.workload == "paper":
        from paper_1008_2042_amd import quality
        line["config"]["image_quality"] = quality.run(dev)
    if args.serving > 0 and args.workload == "paper":
        from paper_1008_2042_amd import serve
        line["config"]["serving"] = serve.serving_benchmark(n=args.serving, device=dev)
        # the same mix with plain FP32 storage, for the latency against FP32
        sf = serve.serving_benchmark(n=args.serving, device=dev, storage=tfcb.F32)
        line["config"]["serving_f32_storage"] = {
            k: sf[k] for k in ("capacity_recons_per_min", "recons_per_min", "makespan_s",
                               "p50", "p95", "p99", "max_slots", "storage")}
    if args.large:
        # the large single reconstruction, FP32 and FP16 storage, in the same run
        lcfg = inputs.config("large")
        lyd = large_data(lcfg, dev)
        lg = lcfg["geom"]
        vl32, dtl32, lreps = run(tfcb.F32, 1, 1, True, cfg=lcfg, yd=lyd)
        del vl32
        vl16, dtl16, _ = run(tfcb.F16, 1, 1, False, cfg=lcfg, yd=lyd)
        del vl16, lyd
        lk = np.sum([r["kernel_ms"] for r in lreps], axis=0)
        lkn = np.sum([r["kernel_launches"] for r in lreps], axis=0)
        nl = sum(lcfg["iters"])
        line["config"]["large"] = {
            "workload": LARGE_WORKLOAD,
            "f32_s_per_recon": round(dtl32, 3), "f32_iters_per_s": round(nl / dtl32, 3),
            "f16_storage_s_per_recon": round(dtl16, 3),
            "f16_storage_iters_per_s": round(nl / dtl16, 3),
            "seconds_per_grid_f32": [round(x, 4) for x in lreps[0]["seconds_per_grid"]],
            "kernel_avg_ms_fine_grid_f32": {
                KERNEL_NAMES[i]: round(float(lk[i] / lkn[i]) if lkn[i] else 0.0, 3)
                for i in range(3)},
            "note": "one timed reconstruction each after one untimed one"}
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, y)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
