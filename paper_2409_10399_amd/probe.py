"""Copy-bandwidth probe: times a plain device-to-device copy of known size
with HIP events (the HBM reference for the step kernel's roofline, and the
kernel whose FETCH_SIZE / WRITE_SIZE counters calibrate the traffic figure).

python -m paper_2409_10399_amd.probe [--mib 1024] [--reps 20]
"""
import argparse
import ctypes
import json
import os

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libeelbm_probe.so")


def copy_bandwidth(mib=1024, reps=20, blocks=None, variant=2):
    import torch
    if not os.path.exists(_LIB):
        raise RuntimeError(f"{_LIB} is missing (run python -m paper_2409_10399_amd.build)")
    L = ctypes.CDLL(_LIB)
    L.eelbm_probe_copy.restype = ctypes.c_int
    L.eelbm_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p]
    nbytes = mib * (1 << 20)
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    st = torch.cuda.current_stream()
    blocks = blocks or 256 * 32
    run = lambda: L.eelbm_probe_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                     nbytes, blocks, variant, ctypes.c_void_p(st.cuda_stream))
    for _ in range(3):
        assert run() == 0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        run()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes_per_launch": 2 * nbytes, "variant": variant, "blocks": blocks, "ms": ms,
            "GB_s": 2 * nbytes / (ms / 1e3) / 1e9}


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--variant", type=int, default=2)
    ap.add_argument("--blocks", type=int, default=0)
    a = ap.parse_args()
    print(json.dumps(copy_bandwidth(a.mib, a.reps, a.blocks or None, a.variant)))
