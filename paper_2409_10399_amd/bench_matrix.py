"""Throughput of the step over lattices, storage types and sizes on one GPU.

For each case: microseconds per step (HIP events around K steps on the
library's stream, after W warm-up steps), MLUPS, and the algorithmic HBM bytes
per node update over the step time against the 8 TB/s HBM3E peak.  Algorithmic
bytes per node: 4Q populations read and written, the (1 + D)-value
imposed-velocity record read and written, and the three lag values read when
n_gamma > 1 (as in bench.py).

python -m paper_2409_10399_amd.bench_matrix [--cases channel1024,column256] [--storages fp32,fp16,bf16]
python -m paper_2409_10399_amd.bench_matrix --sweep 512 [--sweep-steps 500]
Prints one JSON object per case (and a markdown table).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def bytes_per_node(D, Q, storage, lag):
    tb = {"fp64": 8, "fp32": 4, "fp32x": 4, "mixed": 3, "fp16": 2, "bf16": 2}[storage]
    cb = 8 if storage in ("fp64", "fp32x") else 4  # fp32x: FP32 populations, FP64 records
    return 2 * 4 * Q * tb + 2 * (1 + D) * cb + (3 * cb if lag else 0)


def make_case(name):
    import workloads
    if name.startswith("channel"):
        n = int(name[len("channel"):])
        return workloads.channel_2d(nx=n, ny=n)
    if name.startswith("column"):
        n = int(name[len("column"):])
        return workloads.column_3d(n=n, nblobs=max(1, round(256 * (n / 256) ** 3)))
    raise ValueError(name)


def time_case(cfg, fields, storage, steps, warmup):
    import torch
    from paper_2409_10399_amd import Lattice
    lat = Lattice(cfg, storage=storage)
    lat.init_fields(fields)
    lat.advance(warmup)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    lat.advance(steps)
    e1.record(st)
    torch.cuda.synchronize()
    ok = lat.diag()["nonfinite"] == 0
    del lat
    torch.cuda.empty_cache()
    return e0.elapsed_time(e1) * 1e3 / steps, ok


def batch_cases(count, steps, seed=0, tile=(64, 4), graph_steps=100, modes=("graph", "batched", "separate"),
                grid=0):
    """The channel sweep (count members, FP32) advanced three ways from its
    initial state: one batched launch per step replayed from HIP graphs of
    graph_steps steps, one batched launch per step, and every member launched
    on its own (steps / 20 steps).  tile None: the batch's autotuned tile.
    grid > 0: count channels of grid x grid nodes (the surrogate study's
    distribution) instead of the sweep's uneven sizes."""
    import torch
    import workloads
    from paper_2409_10399_amd import Batch, Lattice
    t0 = time.time()
    if grid:
        from paper_2409_10399_amd.surrogate_study import instances
        ws = [(cfg, f) for cfg, f, _ in instances(count, seed=seed + 1, n=grid)]
    else:
        ws = workloads.channel_sweep(count=count, seed=seed)
    nodes = sum(c["nx"] * c["ny"] for c, _ in ws)
    lats = []
    for cfg, f in ws:
        lat = Lattice(cfg, storage="fp32")
        lat.init_fields(f)
        if tile is not None:
            lat.set_launch(*tile)
        lats.append(lat)
    torch.cuda.synchronize()
    print(f"# sweep: {count} channels, {nodes} nodes, set up in {time.time() - t0:.1f} s", flush=True)
    st = torch.cuda.current_stream()
    rows = []

    def timed(fn, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        fn(n)
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / n

    for mode in modes:
        for lat, (cfg, f) in zip(lats, ws):  # every mode starts from the initial state
            lat.init_fields(f)
        if mode == "separate":
            n = max(10, steps // 20)
            us = timed(lambda k: [lat.advance(k) for lat in lats], n)
        else:
            b = Batch(lats, tile=tile, graph_steps=graph_steps if mode == "graph" else 0)
            b.advance(graph_steps if mode == "graph" else 2)  # capture / warm up
            us = timed(b.advance, steps)
            del b
        ok = all(lat.diag()["nonfinite"] == 0 for lat in lats)
        bpn = bytes_per_node(2, 9, "fp32", True)
        r = {"case": f"sweep{count}" + (f"x{grid}^2" if grid else ""), "mode": mode,
             "tile": "x".join(map(str, lats[0].get_launch()[:2])) + (" (auto)" if tile is None else ""),
             "nodes": nodes, "us_per_step": round(us, 2),
             "MLUPS": round(nodes / us, 1), "GB_s": round(bpn * nodes / us / 1e3, 1),
             "frac_hbm_peak": round(bpn * nodes / us / 1e3 / HBM_PEAK_GBS, 4), "finite": bool(ok)}
        rows.append(r)
        print(json.dumps(r), flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", default="channel1024,column256")
    ap.add_argument("--storages", default="fp32,fp16,bf16")
    ap.add_argument("--steps", type=int, default=0, help="0: about 0.5 s of steps per case")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sweep", type=int, default=0, help="members of the batched channel sweep (0: skip)")
    ap.add_argument("--sweep-steps", type=int, default=500)
    ap.add_argument("--sweep-tiles", default="64x4", help="tiles of the sweep batch, e.g. 64x4,128x2,auto")
    ap.add_argument("--sweep-modes", default="graph,batched,separate")
    ap.add_argument("--sweep-grid", type=int, default=0, help="square channels of this size (0: the sweep's sizes)")
    a = ap.parse_args()
    if a.sweep:
        for t in a.sweep_tiles.split(","):
            tile = None if t == "auto" else tuple(int(v) for v in t.split("x"))
            batch_cases(a.sweep, a.sweep_steps, tile=tile, modes=a.sweep_modes.split(","), grid=a.sweep_grid)
        return
    rows = []
    for case in a.cases.split(","):
        t0 = time.time()
        cfg, fields = make_case(case)
        nodes = cfg["nx"] * cfg["ny"] * cfg.get("nz", 1)
        D, Q = (2, 9) if cfg["lattice"] == "D2Q9" else (3, 19)
        print(f"# {case}: {nodes} nodes, inputs built in {time.time() - t0:.1f} s", flush=True)
        for storage in a.storages.split(","):
            steps = a.steps or max(20, int(0.5e6 / max(1.0, nodes * 7e-5)))
            us, ok = time_case(cfg, fields, storage, steps, a.warmup)
            bpn = bytes_per_node(D, Q, storage, cfg["n_gamma"] > 1)
            gbs = bpn * nodes / us / 1e3
            r = {"case": case, "lattice": cfg["lattice"], "storage": storage, "nodes": nodes, "steps": steps,
                 "us_per_step": round(us, 2), "MLUPS": round(nodes / us, 1), "bytes_per_node": bpn,
                 "GB_s": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4), "finite": bool(ok)}
            rows.append(r)
            print(json.dumps(r), flush=True)
    print("\n| case | storage | us/step | MLUPS | B/node | GB/s | frac of 8 TB/s |\n|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['case']} | {r['storage']} | {r['us_per_step']} | {r['MLUPS']} | {r['bytes_per_node']} | "
              f"{r['GB_s']} | {r['frac_hbm_peak']} |")


if __name__ == "__main__":
    main()
