"""The paper's 1D tube tests (Sec. 3.6, TEST #1 - #4) on the GPU path, as
D2Q9 lattices of 200 x 1 nodes (the y-uniform D2Q9 step is the D1Q3 step,
pinned by test_oracle_scheme's projection tests).

* parity: TEST #1 (constant drag) and TEST #4 (Clift-Grace-Weber, R = 833,
  dashpot + lag) against the oracle for 1500 steps, FP64;
* the four tests to the paper's N_t = 6e6 steps in one batch: all stay
  finite (TEST #3 / #4 with the stabilisers of Sec. 3.2); at steady state
  the mixture flux alpha_g u_g + alpha_l u_l is uniform along the tube and
  equal to the inlet flux (TEST #1 - #3: 0.8 * 1e-2 + 0.2 * 1e-3 = 8.2e-3,
  printed 8.1999e-3; TEST #4: 0.1 * 0.0043 + 0.9 * 0.0011 = 1.42e-3); and the
  TEST #1 outlet values are compared with the printed ones (u_g and alpha_g
  within 0.1 %, u_l within 0.5 %) and with the outlet relation of Eq. (127)
  (within 0.5 %; the paper: 0.01 %).
"""
import json
import math
import os

import numpy as np
import pytest

import workloads
from parity import check, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "test1_outlet.json")
INLET_FLUX = {1: 8.2e-3, 2: 8.2e-3, 3: 8.2e-3, 4: 0.1 * 0.0043 + 0.9 * 0.0011}


@pytest.mark.parametrize("test", [1, 4])
def test_tube_parity(test):
    cfg, f = workloads.tube_1d(test)
    check(run_gpu(cfg, f, 1500, "fp64").read_all(), run_oracle(cfg, f, 1500).read(), "fp64", None,
          f"tube TEST #{test}")


def _outlet_relation(ag, ug, K_I, K_W, R, g):
    """u_l at the outlet predicted by Eqs. (124), (126), (127) from the
    outlet gas fraction and gas velocity."""
    al = 1.0 - ag
    ug0 = math.sqrt(ag * al * (R - 1.0) * g / K_I)                 # Eq. (124)
    r = K_W / K_I * ag                                              # text after Eq. (126)
    return (ug - math.sqrt(ug * ug - (1.0 - r) * (ug * ug - ug0 * ug0))) / (1.0 - r)   # Eq. (127)


@pytest.fixture(scope="module")
def tubes_6e6():
    import torch
    from paper_2409_10399_amd import Batch, Lattice
    out = {}
    lats = []
    for k in (1, 2, 3, 4):
        cfg, f = workloads.tube_1d(k)
        lat = Lattice(cfg, storage="fp64")
        lat.init_fields(f)
        lats.append((k, cfg, lat))
    batch = Batch([lat for _, _, lat in lats], tile=(256, 1), graph_steps=1000)
    for done in range(6):
        batch.advance(1_000_000)
        torch.cuda.synchronize()
        print(f"  tubes: {done + 1}e6 steps", flush=True)
    for k, cfg, lat in lats:
        out[k] = (cfg, lat.read_all(), lat.diag())
    return out


@pytest.mark.parametrize("test", [1, 2, 3, 4])
def test_tube_steady_state(tubes_6e6, test):
    cfg, r, d = tubes_6e6[test]
    ag, al, ug, ul = r["alpha_g"][0], r["alpha_l"][0], r["u_g"][0, 0], r["u_l"][0, 0]
    flux = ag * ug + al * ul
    print(f"  TEST #{test}: flux {flux.min():.6e}..{flux.max():.6e}; outlet u_g {ug[-1]:.5e} u_l {ul[-1]:.5e} "
          f"alpha_g {ag[-1]:.5f}", flush=True)
    assert d["nonfinite"] == 0
    assert np.all(np.isfinite(flux))
    assert np.max(np.abs(flux - INLET_FLUX[test])) / INLET_FLUX[test] < 2e-3


def test_tube1_outlet_against_the_paper(tubes_6e6):
    """TEST #1 at 6e6 steps: the outlet liquid velocity against Eq. (127)
    evaluated with our own outlet alpha_g and u_g (the paper: 0.01 %), and
    the outlet values against the printed ones."""
    cfg, r, _ = tubes_6e6[1]
    printed = json.load(open(GOLDEN))["printed"]
    ag, ug, ul = r["alpha_g"][0, -1], r["u_g"][0, 0, -1], r["u_l"][0, 0, -1]
    R = cfg["rho_l"] / cfg["rho_g"]
    ul_rel = _outlet_relation(ag, ug, cfg["K_I"], cfg["K_W"], R, cfg["g_hat"])
    mis = abs(ul - ul_rel) / ul_rel
    digits = json.load(open(GOLDEN))["outlet"]
    print(f"  TEST #1 outlet: u_g {ug:.6e} (printed {printed['ug']}), u_l {ul:.6e} (printed {printed['ul']}), "
          f"alpha_g {ag:.6f} (printed {printed['alpha_g']}); Eq. (127) gives u_l {ul_rel:.6e}, "
          f"mismatch {100 * mis:.3f} %", flush=True)
    assert abs(ug - digits["ug"]) / digits["ug"] < 1e-3
    assert abs(ag - digits["alpha_g"]) / digits["alpha_g"] < 1e-3
    assert abs(ul - digits["ul"]) / digits["ul"] < 5e-3
    assert mis < 5e-3
