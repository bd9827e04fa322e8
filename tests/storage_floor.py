"""Storage-rounding floor of the population storage, computed by the FP64
oracle alone: the oracle's step with its populations rounded to the stored
format after every step, against the plain oracle, per field rel-L2.  Test
infrastructure (calls only oracle/); the GPU errors stated in the GPU tests
are compared with these floors.

Two storage formats (periodic lattices: the sender of direction q at x is
x - v_q):

* "residual" -- the library's format: each population is stored as the
  residual f_q - E_q(r_s) against the equilibrium part of its sender's
  record r_s = (alpha_g - alpha_r, u_g, u_l, eps_g - 1), the record values
  themselves rounded to FP32:
      f_g:  w_q (de + 3 v.u_g)        f_l:  w_q 3 v.u_l
      f_ag: w_q (da + 3 a v.u_g)      f_al: w_q (-da + 3 (1 - a) v.u_l)
  (deviations from w_q, w_q alpha_r, w_q (1 - alpha_r); da = alpha_g -
  alpha_r from the record, a = alpha_r + da, de = eps_g - 1).  FP16 holds the
  residuals x 2^20 (the moving populations of f_l x 2^(20 + round(log2
  min(R, 64))), the rest population of f_l unscaled), BF16 unscaled.
* "deviation" -- the earlier format, for comparison: the deviations from
  w_q, w_q alpha_r, w_q (1 - alpha_r) themselves (FP16 x 2^15).

    python tests/storage_floor.py channel   # D2Q9 40x48 channel, 1000 steps
    python tests/storage_floor.py column    # D3Q19 32^3 column, 200 steps
"""
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import workloads  # noqa: E402
from oracle import Oracle  # noqa: E402

FIELDS = ("alpha_g", "u_g", "u_l", "dp_k")


def to_bf16(x):
    """Round to BF16 (through FP32, as the GPU's FP32 values are), nearest even."""
    a = np.asarray(x, dtype=np.float32).view(np.uint32)
    r = ((a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)  # round to nearest even
    return r.view(np.float32).astype(np.float64)


def r32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _round(d, kind, scale):
    if kind == "fp16":
        return (d * scale).astype(np.float16).astype(np.float64) / scale
    if kind == "bf16":
        return to_bf16(d)
    return r32(d)


def _sender(a, v):
    """Values of the sender x - v at x (periodic)."""
    D = len(v)
    return np.roll(a, shift=tuple(int(v[c]) for c in range(D)), axis=tuple(a.ndim - 1 - c for c in range(D)))


class Emulated:
    """The oracle with its populations rounded to a storage format after
    every step."""

    def __init__(self, cfg, f, kind, fmt):
        self.o = Oracle(cfg, f)
        self.kind, self.fmt = kind, fmt
        self.ar = float(np.mean(f["alpha_g"]))
        R = float(cfg["rho_l"]) / float(cfg["rho_g"])
        self.l_scale = 2.0 ** (20 + int(round(np.log2(min(max(R, 1.0), 64.0)))))

    def step(self):
        o = self.o
        lat = o.lat
        w = lat.w
        v = lat.v.astype(np.float64)
        m = o.moments() if self.fmt == "residual" else None
        o.step(1)
        ar = self.ar
        shape = (-1,) + (1,) * (o.f["g"].ndim - 1)
        if self.fmt == "deviation":
            bases = (("g", 1.0), ("l", 1.0), ("ag", ar), ("al", 1.0 - ar))
            for s, b in bases:
                base = w.reshape(shape) * b
                o.f[s] = base + _round(o.f[s] - base, self.kind, 32768.0)
            return
        da = r32(m["alpha_g"] - ar)
        a = ar + da
        ug, ul, de = r32(m["u_g"]), r32(m["u_l"]), r32(m["eps_g"] - 1.0)
        D = lat.D
        for q in range(lat.Q):
            vq = v[q]
            cug = sum(vq[c] * _sender(ug[c], vq) for c in range(D))
            cul = sum(vq[c] * _sender(ul[c], vq) for c in range(D))
            das, as_ = _sender(da, vq), _sender(a, vq)
            E = {"g": w[q] * (1.0 + _sender(de, vq) + 3.0 * cug),
                 "l": w[q] * (1.0 + 3.0 * cul),
                 "ag": w[q] * (ar + das + 3.0 * as_ * cug),
                 "al": w[q] * ((1.0 - ar) - das + 3.0 * (1.0 - as_) * cul)}
            for s in ("g", "l", "ag", "al"):
                scale = 2.0 ** 20
                if s == "l":
                    scale = 1.0 if q == 0 else self.l_scale
                o.f[s][q] = E[s] + _round(o.f[s][q] - E[s], self.kind, scale)


def storage_floor(cfg, f, steps, kinds=("fp32",), fmt="residual"):
    """rel-L2 per field, for each storage kind, of the oracle with its
    populations rounded to `fmt` after every step, against the plain oracle."""
    ref = Oracle(cfg, f)
    ems = {k: Emulated(cfg, f, k, fmt) for k in kinds}
    for _ in range(steps):
        ref.step(1)
        for em in ems.values():
            em.step()
    ro = ref.read()
    out = {}
    for k, em in ems.items():
        re = em.o.read()
        out[k] = {q: float(np.linalg.norm(re[q] - ro[q]) / np.linalg.norm(ro[q])) for q in FIELDS}
    return out


def fp32_floor(cfg, f, steps, fmt="residual"):
    """rel-L2 per field of FP32 storage in `fmt` after `steps`."""
    return storage_floor(cfg, f, steps, ("fp32",), fmt)["fp32"]


if __name__ == "__main__":
    case = sys.argv[1] if len(sys.argv) > 1 else "channel"
    if case == "channel":
        cfg, f, steps = *workloads.channel_2d(nx=40, ny=48, n_ramp=100.0), 1000
    else:
        cfg, f, steps = *workloads.column_3d(n=32, nblobs=2), 200
    t0 = time.time()
    for fmt in ("residual", "deviation"):
        for k, err in storage_floor(cfg, f, steps, ("fp32", "fp16", "bf16"), fmt).items():
            print(fmt, k, "storage floor", " ".join(f"{q}={v:.2e}" for q, v in err.items()),
                  f"({time.time() - t0:.0f} s)", flush=True)
