"""Serving driver for the continuous-batching server.

Replays a seeded stream of reconstruction requests (mixed volume sizes, view
counts and doses) into tfcb.Server: a closed-loop run (everything submitted
at once) measures the capacity, then an open-loop run with exponential
inter-arrival times at a fraction of that capacity measures latency
(completion minus scheduled arrival, host monotonic clock) and reports
p50/p95/p99 (numpy 'linear' percentiles) and reconstructions per minute.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional

import numpy as np

from paper_1008_2042_amd import inputs, tfcb


def build_requests(mix, device, storage: int = tfcb.F16, lam: float = 5e-4,
                   iters=(16, 24)) -> List[Dict]:
    """Projection data on the device for every request of a mix."""
    import torch
    out = []
    for spec in mix:
        g = spec["geom"]
        ells = inputs.body_phantom(spec["phantom_seed"], 4, 15, zhalf=80.0)
        clean = inputs.analytic_projection_torch(g, ells, device)
        y = inputs.poisson_log_torch(clean, spec["i0"], spec["noise_seed"]).to(torch.float32)
        opts = tfcb.options(lam, list(iters), 3, 1, storage=storage)
        out.append(dict(spec=spec, geom=g, proj=y.contiguous(), opts=opts,
                        bytes=tfcb.Server.request_bytes(g, opts)))
    return out


def replay(requests: List[Dict], arrivals: np.ndarray, arena_bytes: int, max_slots: int,
           keep_results: bool = False, timeout_s: float = 600.0) -> Dict:
    """Submit request i at time arrivals[i] (seconds after start), drive the
    server until all finish, and return per-request latencies."""
    srv = tfcb.Server(arena_bytes, max_slots)
    order = np.argsort(arrivals, kind="stable")
    n = len(requests)
    ids: Dict[int, int] = {}
    t_sched = np.zeros(n)
    t_done = np.full(n, np.nan)
    status = [None] * n
    results: List[Optional[object]] = [None] * n
    nxt = 0
    t0 = time.monotonic()
    try:
        while True:
            now = time.monotonic() - t0
            while nxt < n and arrivals[order[nxt]] <= now:
                i = int(order[nxt])
                r = requests[i]
                ids[i] = srv.submit(r["geom"], r["proj"], r["opts"])
                t_sched[i] = t0 + arrivals[i]
                nxt += 1
            active, queued = srv.step()
            for i, rid in list(ids.items()):
                if status[i] is not None:
                    continue
                st, td, res = srv.poll(rid)
                if st in (tfcb.REQ_DONE, tfcb.REQ_FAILED, tfcb.REQ_CANCELLED):
                    status[i] = (st, res)
                    t_done[i] = td
                    if keep_results:
                        results[i] = srv.result(rid).clone()
                    srv.release(rid)
            if nxt == n and all(s is not None for s in status):
                break
            if time.monotonic() - t0 > timeout_s:
                raise TimeoutError("serving replay exceeded %.0f s" % timeout_s)
            if active == 0 and queued == 0 and nxt < n:
                time.sleep(max(0.0, min(0.002, arrivals[order[nxt]] - (time.monotonic() - t0))))
            else:
                time.sleep(0.0002)
        makespan = float(np.nanmax(t_done) - t0)
    finally:
        srv.close()
    lat = t_done - t_sched
    return dict(latency=lat, status=status, makespan=makespan, results=results)


def percentiles(lat: np.ndarray) -> Dict[str, float]:
    return {k: float(np.percentile(lat, q, method="linear"))
            for k, q in (("p50", 50), ("p95", 95), ("p99", 99))}


def serving_benchmark(n: int = 64, seed: int = 404, load: float = 0.8,
                      arena_gb: float = 8.0, max_slots: int = 3, device=None,
                      storage: int = tfcb.F16) -> Dict:
    import torch
    device = device or torch.device("cuda:0")
    mix = inputs.serving_mix(n, seed)
    reqs = build_requests(mix, device, storage)
    arena = int(arena_gb * (1 << 30))
    # closed loop: capacity in reconstructions per second
    sat = replay(reqs, np.zeros(n), arena, max_slots)
    capacity = n / sat["makespan"]
    rng = np.random.default_rng(seed)
    tau = 1.0 / (load * capacity)
    arrivals = np.cumsum(rng.exponential(tau, size=n))
    arrivals -= arrivals[0]
    run = replay(reqs, arrivals, arena, max_slots)
    ok = sum(1 for s in run["status"] if s[0] == tfcb.REQ_DONE)
    out = dict(n_requests=n, completed=ok, capacity_recons_per_min=round(60 * capacity, 2),
               mean_interarrival_s=round(tau, 4), load=load,
               recons_per_min=round(60 * n / run["makespan"], 2),
               makespan_s=round(run["makespan"], 3), arena_gb=arena_gb, max_slots=max_slots,
               storage={tfcb.F32: "f32", tfcb.F16: "f16", tfcb.BF16: "bf16"}[storage],
               percentile_note="numpy linear percentiles of %d samples; p99 lies between the "
                               "two largest order statistics" % n)
    out.update({k: round(v, 4) for k, v in percentiles(run["latency"]).items()})
    return out


def main():
    """Closed-loop capacity of a seeded mix (every request submitted at
    time 0), for kernel traces of the serving path:
        python -m paper_1008_2042_amd.serve --requests 64 --slots 3"""
    import argparse
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--slots", type=int, default=3)
    ap.add_argument("--arena-gb", type=float, default=8.0)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    reqs = build_requests(inputs.serving_mix(args.requests, 404), dev, tfcb.F16)
    torch.cuda.synchronize()
    sat = replay(reqs, np.zeros(args.requests), int(args.arena_gb * (1 << 30)), args.slots)
    print("closed loop: %d requests, %d slots, makespan %.3f s, %.1f reconstructions/min"
          % (args.requests, args.slots, sat["makespan"], 60 * args.requests / sat["makespan"]),
          flush=True)


if __name__ == "__main__":
    main()
