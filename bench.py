"""Benchmark of the fused six-scheme LBM step on one MI355X.

Workload: D2Q9 1024x1024 bubble-column-like channel (R = 1000, Clift-Grace-
Weber drag for 3 mm bubbles, inlet gas fraction 0.05 with +-10 % seeded noise,
outlet at the top, no-slip side walls, gravity on), FP32 populations.  A step
is one launch of the fused kernel over the whole lattice; the timed region is
K steps with the inputs already resident in HBM.

Prints one JSON line: MLUPS, the roofline of the step kernel (algorithmic HBM
bytes per launch / measured launch time vs the 8 TB/s HBM3E peak), the FP64
oracle timed on a bounded sample of the same workload on the host cores, and
the learned surrogate's speedup over plain LBM within 2 % rel-L2, measured in
the same run from the saved network.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (6 coupled schemes) & % HBM peak; surrogate speedup at ≤2% rel L2"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2409_10399_amd", "csrc", "eelbm_kernels.hip")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_step_d2q9_fp32_channel1024_pmc.json")
SURROGATE_MODEL = os.path.join(ROOT, "paper_2409_10399_amd", "surrogate_weights", "cno_16_32_64_128")


def algorithmic_bytes_per_node(D, Q, tbytes, cbytes, lag):
    """State the method must carry from one node-update to the next: 4Q
    post-collision populations (f_g, f_l, f_ag, f_al) read and written, the
    1 + D imposed-velocity values (alpha_g, u_g - u_l) that stand in for the
    2Q source-scheme populations read and written, and the 3 lag values
    (S''_g, S''_l, Lambda') read; their write every n_gamma steps is not
    counted.  D2Q9 FP32: 288 + 24 + 12 = 324 B.  The kernel moves more than
    this minimum: its record (alpha_g, u_g, u_l, eps_g - 1: 2 + 2D values)
    also carries u_g, u_l and eps_g - 1 as the reference of the stored
    residuals (D2Q9 FP32: 348 B per node-update, 24 B records read and
    written); that overhead of the storage format counts against the
    kernel."""
    return 2 * 4 * Q * tbytes + 2 * (1 + D) * cbytes + (3 * cbytes if lag else 0)


def kernel_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def _cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(steps=20, procs=None):
    """The oracle as it stands on the host cores: a bounded sample of the same
    workload (the full 1024x1024 channel, `steps` steps), NumPy FP64, one
    thread per process.  Single core: one process.  All cores: `procs`
    processes each stepping its own copy at the same time (the oracle is not
    parallel itself; independent copies are how a CPU runs many such
    lattices); throughput = all node updates over the span from the first
    start to the last end of their stepping.  procs defaults to the host's
    cores, at most 16 (the CPU share of one GPU on these machines)."""
    model, ncpu = _cpu_info()
    procs = procs or max(1, min(16, ncpu))
    code = (
        "import sys, time, json; sys.path.insert(0, %r)\n"
        "import workloads\nfrom oracle import Oracle\n"
        "cfg, f = workloads.channel_2d()\n"
        "o = Oracle(cfg, f)\n"
        "t0 = time.time(); o.step(%d); t1 = time.time()\n"
        "print(json.dumps({'t0': t0, 't1': t1, 'nodes': cfg['nx'] * cfg['ny']}))\n" % (ROOT, steps))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")

    def run(n):
        ps = [subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                               text=True, env=env) for _ in range(n)]
        out = []
        for pr in ps:
            o, e = pr.communicate(timeout=900)
            if pr.returncode != 0:
                raise RuntimeError(e[-400:])
            out.append(json.loads(o.strip().splitlines()[-1]))
        span = max(d["t1"] for d in out) - min(d["t0"] for d in out)
        return sum(d["nodes"] for d in out) * steps / span / 1e6, span

    def one_core(body):
        """MLUPS of one process running `body` (sets `lats` = [(cfg, fields, steps)])"""
        src = ("import sys, time, json; sys.path.insert(0, %r)\n"
               "import workloads\nfrom oracle import Oracle\n" % ROOT + body +
               "os_ = [(Oracle(c, f), k) for c, f, k in lats]\n"
               "t0 = time.time()\nfor o, k in os_: o.step(k)\nt1 = time.time()\n"
               "n = sum(c['nx'] * c['ny'] * c.get('nz', 1) * k for c, f, k in lats)\n"
               "print(json.dumps({'t': t1 - t0, 'updates': n}))\n")
        pr = subprocess.run([sys.executable, "-c", src], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                            env=env, timeout=600)
        if pr.returncode != 0:
            raise RuntimeError(pr.stderr[-400:])
        d = json.loads(pr.stdout.strip().splitlines()[-1])
        return d["updates"] / d["t"] / 1e6

    try:
        one, dt1 = run(1)
        allc, dtn = run(procs)
        # for scale, on one core: the FP64 periodic box (D2Q9 64x64, R = 10,
        # 200 steps), the D3Q19 64^3 periodic column with the 256^3 column's
        # blob density (2 steps), and 8 members of the channel sweep (3 steps each)
        box_mlups = one_core("lats = [workloads.periodic_box_2d() + (200,)]\n")
        col_mlups = one_core("lats = [workloads.column_3d(n=64, nblobs=4) + (2,)]\n")
        swp_mlups = one_core("lats = [(c, f, 3) for c, f in workloads.channel_sweep(8, seed=0)]\n")
    except (RuntimeError, subprocess.TimeoutExpired) as e:
        return {"error": str(e)[-400:]}
    return {"value": allc, "unit": "MLUPS", "cores": procs, "kind": "oracle",
            "sample": f"D2Q9 1024x1024 channel, {steps} steps per copy, NumPy FP64, {procs} single-thread "
                      f"copies at once ({dtn:.1f} s span); one copy alone: {one:.3f} MLUPS ({dt1:.1f} s)",
            "single_core": one, "host_cpus": ncpu, "cpu_model": model,
            "periodic_box_64_single_core": box_mlups, "column_64_d3q19_single_core": col_mlups,
            "sweep_8_members_single_core": swp_mlups}


def surrogate_leg():
    """The surrogate half of the metric, measured now: the saved network
    (trained by surrogate_study.py, policy chosen on validation channels) is
    judged on its held-out test channels -- 8 D2Q9 256^2 channels of the sweep
    distribution, 50 jumps of 100 steps from t = 1000 -- against plain LBM
    (HIP-graph batched launches), both timed in this run."""
    if not os.path.exists(SURROGATE_MODEL + ".npz"):
        return {"error": "no saved surrogate model"}
    from paper_2409_10399_amd import surrogate_study as st
    res, meta = st.measure_saved(SURROGATE_MODEL, reps=3)
    ch, sp = res["chosen"], res["specified"]
    return {
        "speedup": round(ch["speedup"], 3), "rel_l2_alpha_g_max": round(ch["rel_l2_alpha_max"], 5),
        "within_2pct": bool(ch["rel_l2_alpha_max"] <= 0.02),
        "policy": {"defect_max": ch["defect_max"], "check_every": ch["check_every"], "chosen_on": "validation channels"},
        "jumps_reanchored": [ch["anchors"], ch["jumps"]],
        "ms_plain_lbm": round(ch["seconds_plain_lbm"] * 1e3, 2), "ms_rollout": round(ch["seconds_surrogate"] * 1e3, 2),
        "specified_policy_1e-3_every_5": {"speedup": round(sp["speedup"], 3),
                                          "rel_l2_alpha_g_max": round(sp["rel_l2_alpha_max"], 5)},
        "measured_by_this_run": True, "model": os.path.relpath(SURROGATE_MODEL, ROOT),
        "widths": meta["widths"], "test_channels": res["test_screened"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp64", "fp16", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the method's step is benchmarked on a single MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2409_10399_amd import Lattice

    cfg, fields = workloads.channel_2d()
    nodes = cfg["nx"] * cfg["ny"]
    lat = Lattice(cfg, storage=args.storage)
    lat.init_fields(fields)
    lat.advance(args.warmup)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    lat.advance(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    mlups = nodes * args.steps / (ms / 1e3) / 1e6

    tb = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}[args.storage]
    cb = 8 if args.storage == "fp64" else 4
    bpn = algorithmic_bytes_per_node(2, 9, tb, cb, cfg["n_gamma"] > 1)
    achieved = bpn * nodes / (ms_per_step / 1e3) / 1e9
    traffic = None
    if os.path.exists(PMC_SUMMARY):
        with open(PMC_SUMMARY) as fh:
            pmc = json.load(fh)
        if pmc.get("kernel_sha") == kernel_hash() and pmc.get("storage") == args.storage:
            traffic = pmc.get("bytes_per_launch")
    d = lat.diag()
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"fp64": "f64"}.get(args.storage, "f32"),
        "data": "synthetic",
        "config": {"workload": "D2Q9 1024x1024 bubble-column channel (R=1000, CGW 3 mm, inlet alpha 0.05 "
                               "+-10% noise, walls, outlet), 6 coupled schemes",
                   "lattice": "D2Q9", "nx": cfg["nx"], "ny": cfg["ny"], "storage": args.storage,
                   "n_gamma": cfg["n_gamma"], "bytes_per_node_update": bpn},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        "wall_s": round(wall, 3),
        "state_ok": bool(d["nonfinite"] == 0),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    if not args.no_surrogate:
        out["surrogate"] = surrogate_leg()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
