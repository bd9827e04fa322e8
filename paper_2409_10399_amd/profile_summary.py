"""Condense rocprofv3 CSV output into the short summaries kept under profiles/.

Two kinds of input, each from its own rocprofv3 run (``--output-format csv``):

* a ``--kernel-trace --stats`` run: ``*_kernel_stats.csv`` gives the average
  duration of every kernel;
* ``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` runs of the step and of the
  copy probe (paper_2409_10399_amd/probe.py) of known size:
  ``*_counter_collection.csv`` gives the counter per dispatch (KiB).

The copy probe calibrates the counters: factor = bytes the copy really
moves / bytes the counter reports for it.  The fetch factor comes from the
copy variant that loads like the step kernel (nontemporal loads), the write
factor from the one that stores like it (ordinary stores).

python -m paper_2409_10399_amd.profile_summary stats --csv DIR/x_kernel_stats.csv --cmd "..." --out profiles/a.txt
python -m paper_2409_10399_amd.profile_summary pmc --step-fetch CSV --step-write CSV --copy-fetch CSV \
    --copy-write CSV --copy-bytes N --kernel k_step --storage fp32 --cmd "..." --out profiles/b.json
"""
import argparse
import csv
import hashlib
import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(PKG, "csrc", "eelbm_kernels.hip")


def kernel_sha():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def read_stats(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def counter_per_dispatch(path, kernel_substr, counter):
    """Median of `counter` over the dispatches whose name contains
    kernel_substr; rows of one dispatch (one per XCD or SE instance) are
    summed first.  The median is the plain step: the last step of each
    advance, the same kernel, also writes the FP64 read-out fields.
    Returns (median, dispatches, kernel name)."""
    per = {}
    name = None
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            if kernel_substr not in r["Kernel_Name"] or r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no {counter} rows for {kernel_substr!r} in {path}")
    vals = sorted(per.values())
    m = len(vals) // 2
    med = vals[m] if len(vals) % 2 else 0.5 * (vals[m - 1] + vals[m])
    return med, len(vals), name


def cmd_stats(a):
    rows = read_stats(a.csv)
    lines = [f"# rocprofv3 kernel statistics ({a.title})", "", "command:", f"    {a.cmd}", "",
             "| kernel | calls | average us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows[: a.top]:
        lines.append(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    lines.append("")
    lines.append(f"kernel source sha256[:16] at profiling time: {kernel_sha()}")
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cmd_pmc(a):
    fs, nf, name = counter_per_dispatch(a.step_fetch, a.kernel, "FETCH_SIZE")
    ws, nw, _ = counter_per_dispatch(a.step_write, a.kernel, "WRITE_SIZE")
    cf, _, _ = counter_per_dispatch(a.copy_fetch, "k_copy", "FETCH_SIZE")
    cw, _, _ = counter_per_dispatch(a.copy_write, "k_copy", "WRITE_SIZE")
    half = a.copy_bytes / 2  # the copy reads and writes half each
    f_fetch = half / (cf * 1024.0)
    f_write = half / (cw * 1024.0)
    out = {
        "kernel": name, "kernel_sha": kernel_sha(), "storage": a.storage, "workload": a.workload,
        "fetch_kib_per_dispatch": fs, "write_kib_per_dispatch": ws, "dispatches": [nf, nw],
        "copy_bytes_per_launch": a.copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_factor": f_fetch, "write_factor": f_write,
        "bytes_per_launch": fs * 1024.0 * f_fetch + ws * 1024.0 * f_write,
        "commands": a.cmd,
    }
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--cmd", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--top", type=int, default=8)
    s.add_argument("--out", required=True)
    p = sub.add_parser("pmc")
    for k in ("step-fetch", "step-write", "copy-fetch", "copy-write"):
        p.add_argument("--" + k, required=True)
    p.add_argument("--copy-bytes", type=float, required=True)
    p.add_argument("--kernel", default="k_step")
    p.add_argument("--storage", default="fp32")
    p.add_argument("--workload", default="")
    p.add_argument("--cmd", nargs="+", required=True)
    p.add_argument("--out", required=True)
    a = ap.parse_args()
    (cmd_stats if a.what == "stats" else cmd_pmc)(a)


if __name__ == "__main__":
    main()
