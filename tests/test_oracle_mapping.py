"""Pins of the oracle's similarity mapping and 1D steady-state relations
against the numbers the paper prints (Sec. 3.6, TEST #1 and TEST #4)."""
import json
import math
import os

from oracle import mapping

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _sig(a, b, n):
    """a and b agree to n significant figures."""
    return abs(a - b) <= 0.5 * 10 ** (math.floor(math.log10(abs(b))) - n + 1) * 1.0001


def test_test4_similarity_numbers():
    g = json.load(open(os.path.join(GOLD, "test4_mapping.json")))
    i, pr = g["inputs"], g["printed"]
    assert abs(mapping.kappa_cgw(i["Cd"], i["d"]) - i["kappa_I"]) < 1e-12
    s = mapping.similarity(i["g"], i["g_hat"], i["kappa_I"], i["kappa_hat"])
    assert _sig(s["c_over_tau"], pr["c_over_tau"], 3)
    assert _sig(s["c_tau"], pr["c_tau"], 3)
    assert _sig(s["c"], pr["c"], 3)
    ug_hat = i["ug_max"] / s["c"]
    assert _sig(ug_hat, pr["ug_hat_max"], 2)
    assert _sig(ug_hat * i["ul_max_over_ug_max"], pr["ul_hat_max"], 2)
    R = i["rho_l"] / i["rho_g"]
    ul = i["ug_max"] * i["ul_max_over_ug_max"]
    mex = mapping.m_ex(i["kappa_I"], i["alpha_g_max"], R, i["ug_max"] - ul, i["g"])
    assert _sig(mex, pr["M_ex"], 3)
    # Eq. (142): the same ratio in lattice units is identical
    mex_hat = mapping.m_ex(i["kappa_hat"], i["alpha_g_max"], R, ug_hat * (1 - i["ul_max_over_ug_max"]), i["g_hat"])
    assert abs(mex_hat / mex - 1.0) < 1e-12


def test_test1_outlet_relations():
    g = json.load(open(os.path.join(GOLD, "test1_outlet.json")))
    p, o, d, pr = g["params"], g["outlet"], g["derived"], g["printed"]
    ag, al = o["alpha_g"], o["alpha_l"]
    # mixture flux at the outlet equals the inlet one (1D divergence-free mixture)
    flux = ag * o["ug"] + al * o["ul"]
    assert abs(flux - d["mixture_flux"]) < 1e-15
    inlet = p["alpha_g_in_max"] * p["ug_in_max"] + (1 - p["alpha_g_in_max"]) * p["ul_in_max"]
    assert abs(flux / inlet - 1.0) < 1e-4
    # Eq. (124) with the outlet volume fraction
    ug0 = mapping.slip_u0(p["K_I"], ag, p["R"], p["g_hat"])
    assert abs(ug0 - d["ug0"]) < 1e-15
    assert _sig(ug0, pr["ug0"], 5)
    r = p["K_W"] / p["K_I"] * ag
    assert abs(r - d["r"]) < 1e-15
    ul = mapping.steady_ul(o["ug"], ug0, r)                      # Eq. (127)
    assert abs(ul - d["ul_analytic"]) < 1e-15
    assert _sig(ul, pr["ul_analytic"], 5)
    assert abs(abs(ul / o["ul"] - 1) * 100 - pr["mismatch_analytic_percent"]) < 0.005
    ul1 = mapping.steady_ul_r1(o["ug"], ug0)
    assert abs(ul1 - d["ul_r1_approx"]) < 1e-15
    assert abs(round(abs(ul1 / o["ul"] - 1) * 100) - pr["mismatch_r1_percent"]) < 1e-12
    # Eq. (126) holds at the analytic liquid velocity
    assert abs(r * ul * ul - ((o["ug"] - ul) ** 2 - ug0 ** 2)) < 1e-18


def test_channel_workload_constants_follow_from_the_mapping():
    """The bubble-column constants of the workloads are the TEST #4 invariant
    c tau applied to 3 mm bubbles, (R-1) g_hat = 1e-6 and the Eq. (124) slip
    with the Clift-Grace-Weber factor at alpha_g = 0.05."""
    import workloads
    c_tau = 1.45e-4 / 247.5
    k3 = mapping.kappa_cgw(0.66, 0.003)
    assert abs(k3 * c_tau / workloads.KAPPA_HAT_3MM - 1) < 1e-3
    assert abs(999.0 * workloads.G_HAT_R1000 / 1e-6 - 1) < 1e-5
    K = workloads.KAPPA_HAT_3MM * mapping.cgw_lambda(0.05, 1000.0)
    slip = mapping.slip_u0(K, 0.05, 1000.0, workloads.G_HAT_R1000)
    assert abs(slip / workloads.UG_IN_R1000 - 1) < 5e-3


def test_sweep_inlet_slip_is_the_drift_flux_slip():
    """The channel sweep's inlet gas velocity (workloads.terminal_slip) is the
    uniform slip of Eq. (124) with the Clift-Grace-Weber coefficient
    K_I = kappa Lambda (Eqs. (135)-(136)), from the oracle's mapping helpers."""
    import workloads
    from oracle import mapping
    for R, kap, a in [(1000.0, workloads.KAPPA_HAT_3MM, 0.05), (2.0, 2.9e-4, 0.2), (37.0, 5.8e-5, 0.02)]:
        g = 1e-6 / (R - 1.0)
        K = kap * mapping.cgw_lambda(a, R)
        assert abs(workloads.terminal_slip(R, kap, a, g) - mapping.slip_u0(K, a, R, g)) < 1e-15
    assert abs(workloads.terminal_slip(1000.0, workloads.KAPPA_HAT_3MM, 0.05, workloads.G_HAT_R1000)
               - workloads.UG_IN_R1000) < 5e-6
