"""Operator micro-benchmark through the C-ABI (for timing and counter runs).

    python -m paper_1008_2042_amd.opbench --op project --config paper --reps 5

--op: project (P), backproject (P^T), framelet (fused W/T/W^T/H), rof (the
TV method's ROF sub-problem on a noisy piecewise-constant volume), fdk (the
FDK baseline), copy (a plain device copy of one volume's bytes, the
reference for HBM counters).
Inputs are seeded synthetic data of the named workload, resident on the
device before timing.  Prints one JSON line with the event-timed average.
"""
from __future__ import annotations

import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--op", required=True, choices=["project", "backproject", "framelet", "rof", "fdk",
                                                  "copy"])
    ap.add_argument("--config", default="paper")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    args = ap.parse_args()

    import torch

    from paper_1008_2042_amd import inputs, tfcb

    dev = torch.device("cuda:0")
    cfg = inputs.config(args.config)
    g = cfg["geom"]
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[args.dtype]
    vol = torch.tensor(inputs.random_volume(g, 1), device=dev).to(tdt)
    sino = torch.tensor(inputs.random_sino(g, 2), device=dev).to(tdt)
    out_s = torch.empty_like(sino)
    out_v = torch.empty_like(vol)
    ws = torch.empty(tfcb.operator_workspace_size(g, tfcb.dtype_code(tdt)), dtype=torch.uint8,
                     device=dev)

    # a CGLS-like iterate for the ROF: a body of 0.02 /mm with noise
    zz, yy, xx = torch.meshgrid(*[torch.linspace(-1, 1, n, device=dev) for n in g.vol_shape],
                                indexing="ij")
    gen = torch.Generator(device=dev)
    gen.manual_seed(3)
    rof_in = (0.02 * ((xx * xx + yy * yy) < 0.8).float()
              + 2e-3 * torch.randn(g.vol_shape, generator=gen, device=dev)).to(tdt)

    def once():
        if args.op == "project":
            tfcb.project(g, vol, out=out_s, ws=ws)
        elif args.op == "backproject":
            tfcb.backproject(g, sino, out=out_v, ws=ws)
        elif args.op == "framelet":
            tfcb.framelet_shrink(vol, cfg["lam"], cfg["framelet_levels"], True, out=out_v)
        elif args.op == "rof":
            tfcb.rof(rof_in, 5e-4, out=out_v)
        elif args.op == "fdk":
            tfcb.fdk(g, sino, out=out_v)
        else:
            out_v.copy_(vol)

    once()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.reps):
        once()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.reps
    nbytes = vol.numel() * vol.element_size()
    print(json.dumps({"op": args.op, "config": args.config, "dtype": args.dtype, "reps": args.reps,
                      "avg_ms_per_call": round(ms, 4), "volume_bytes": nbytes,
                      "sino_bytes": sino.numel() * sino.element_size()}), flush=True)


if __name__ == "__main__":
    main()
