"""Storage-rounding floor of the 16-bit (and FP32) population storage,
computed by the FP64 oracle alone: the oracle's step with its stored
deviations (f_g, f_l from w_q; f_ag, f_al from w_q alpha_r, w_q (1 - alpha_r))
rounded to the storage type after every step (FP16 holding the deviations
x 2^15, BF16 unscaled, round to nearest even), against the plain oracle,
per field rel-L2.  Test infrastructure (calls only oracle/); the GPU errors
stated in test_gpu_precision.py are compared with these floors.

    python tests/storage_floor.py channel   # D2Q9 40x48 channel, 1000 steps (~30 s)
    python tests/storage_floor.py column    # D3Q19 32^3 column, 200 steps (~2.5 min)
"""
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import workloads  # noqa: E402
from oracle import Oracle  # noqa: E402


def to_bf16(x):
    """Round to BF16 (through FP32, as the GPU's FP32 values are), nearest even."""
    a = np.asarray(x, dtype=np.float32).view(np.uint32)
    r = ((a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)  # round to nearest even
    return r.view(np.float32).astype(np.float64)


def fp32_floor(cfg, f, steps):
    """rel-L2 per field of the oracle with its stored deviations rounded to
    FP32 after every step, against the plain oracle."""
    ref, em = Oracle(cfg, f), Oracle(cfg, f)
    w = ref.lat.w.reshape((-1,) + (1,) * (ref.f["g"].ndim - 1))
    ar = float(np.mean(f["alpha_g"]))
    bases = (("g", w), ("l", w), ("ag", w * ar), ("al", w * (1 - ar)))
    for _ in range(steps):
        ref.step(1)
        em.step(1)
        for s, base in bases:
            em.f[s] = base + (em.f[s] - base).astype(np.float32).astype(np.float64)
    ro, re = ref.read(), em.read()
    return {k: np.linalg.norm(re[k] - ro[k]) / np.linalg.norm(ro[k]) for k in ("alpha_g", "u_g", "u_l", "dp_k")}


def floors(cfg, f, steps, kinds):
    """Print the per-field rel-L2 floor of each storage kind after `steps`."""
    ref = Oracle(cfg, f)
    ems = {k: Oracle(cfg, f) for k in kinds}
    w = ref.lat.w.reshape((-1,) + (1,) * (ref.f["g"].ndim - 1))
    ar = float(np.mean(f["alpha_g"]))
    bases = (("g", w), ("l", w), ("ag", w * ar), ("al", w * (1 - ar)))
    t0 = time.time()
    for i in range(steps):
        ref.step(1)
        for k, em in ems.items():
            em.step(1)
            for s, base in bases:
                d = em.f[s] - base
                if k == "fp16":
                    d = (d * 32768.0).astype(np.float16).astype(np.float64) / 32768.0
                elif k == "bf16":
                    d = to_bf16(d)
                else:
                    d = d.astype(np.float32).astype(np.float64)
                em.f[s] = base + d
    ro = ref.read()
    for k, em in ems.items():
        re = em.read()
        err = {q: float(np.linalg.norm(re[q] - ro[q]) / np.linalg.norm(ro[q])) for q in ("alpha_g", "u_g", "u_l", "dp_k")}
        print(k, "storage floor", " ".join(f"{q}={v:.2e}" for q, v in err.items()), f"({time.time() - t0:.0f} s)", flush=True)

if __name__ == "__main__":
    case = sys.argv[1] if len(sys.argv) > 1 else "channel"
    if case == "channel":
        cfg, f = workloads.channel_2d(nx=40, ny=48, n_ramp=100.0)
        floors(cfg, f, 1000, ("fp32", "fp16", "bf16"))
    else:
        cfg, f = workloads.column_3d(n=32, nblobs=2)
        floors(cfg, f, 200, ("fp32", "fp16", "bf16"))
