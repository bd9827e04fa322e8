"""Build the HIP library ``_lib/libeelbm.so`` for gfx950 with hipcc.

Usage: ``python -m paper_2409_10399_amd.build`` (or ``build()`` from Python).
Always recompiles; the library lands in-tree next to this file.
"""
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_lib")
LIB = os.path.join(OUT_DIR, "libeelbm.so")
PROBE_LIB = os.path.join(OUT_DIR, "libeelbm_probe.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]
SOURCES = ["eelbm_kernels.hip", "eelbm_capi.cpp", "cno_kernels.hip"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("hipcc failed: " + " ".join(cmd))
    return r.stdout


def build(verbose=True):
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = []
    t0 = time.time()
    procs = []
    for src in SOURCES:
        obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    for cmd, pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            sys.stderr.write(out)
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    # copy-bandwidth probe (reference kernel for the roofline and counters)
    tmp = PROBE_LIB + ".tmp"
    _run([HIPCC] + FLAGS + ["-shared", "-o", tmp, os.path.join(CSRC, "probe_copy.hip")])
    os.replace(tmp, PROBE_LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f} s")
    return LIB


if __name__ == "__main__":
    build()
