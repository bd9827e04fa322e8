"""Pins of the finite-difference reference (oracle/fd.py) and the
cross-check that ties the LBM oracle's coupled PDE content to it: under the
diffusive refinement of Sec. 2.1.2 the LBM solution must approach the FD
solution of the same two-fluid system at second order (the paper's claim at
the end of Secs. 2.1.2 and 2.2; its Sec. 3.6 compares the two engines in 1D).

FD pins (closed forms that do not retype the FD's formulas): exact periodic
budgets; the uniform drift-flux state of Eq. (124) as a fixed point; uniform
slip relaxation against its closed-form solution (and fourth order in the
time step); the Taylor-Green decay rate 2 nu k^2 approached at second order
in h; the mixture sound speed c_s sqrt(alpha_g + alpha_l / R) implied by
Eqs. (19), (23), (25), (32) (semi-discretely c sin(k)); a Gaussian carried by
a uniform flow; and, for the sigma . grad(alpha) / alpha term of Eqs. (24),
(26), the conservation of the alpha-weighted momentum of a shear layer that
the conservative form (1/alpha) div(alpha sigma) of Eqs. (16)-(17) implies."""
import math

import numpy as np
import pytest

import workloads
from oracle import CS2, Oracle
from oracle.fd import FD, FDParams


def _grid(N):
    x = (np.arange(N) + 0.5) / N
    return np.meshgrid(x, x)        # X varies along axis 1 (x), Y along axis 0 (y)


# ------------------------------------------------------------ FD pins


def test_fd_periodic_budgets():
    """Sum of dp and of alpha_g are invariants of the central-difference
    system on a periodic grid (the discrete divergence telescopes)."""
    N = 24
    X, Y = _grid(N)
    k = 2 * np.pi
    rng = np.random.default_rng(4)
    a = 0.3 + 0.1 * np.sin(k * X + 0.3) * np.cos(2 * k * Y) + 0.02 * rng.standard_normal((N, N))
    ug = 0.01 * np.stack([np.sin(k * Y), np.cos(k * X + 1.0)])
    ul = 0.01 * np.stack([np.cos(2 * k * Y), np.sin(k * X)])
    dp = 1e-4 * np.cos(k * X) * np.sin(k * Y)
    prm = FDParams(2, 10.0, 1.2, 0.8, psi_g=0.2, drag="cgw", kappa_I=0.05, K_W=0.01, g_hat=1e-5,
                   up_axis=1, rho_ref=5.0)
    fd = FD(prm, dict(alpha_g=a, u_g=ug, u_l=ul, dp_k=dp))
    s_dp, s_a = fd.dp.sum(), fd.alpha_g.sum()
    fd.step(0.5, 40)
    assert abs(fd.dp.sum() - s_dp) < 1e-15 * N * N
    assert abs(fd.alpha_g.sum() - s_a) < 1e-13 * abs(s_a)


@pytest.mark.parametrize("drag", ["const", "cgw"])
def test_fd_drift_flux_state_is_a_fixed_point(drag):
    """Eq. (124): at the slip |u_g - u_l|^2 = alpha_g alpha_l (R - 1) g / K_I
    (K_I = kappa_I Lambda for the Clift-Grace-Weber model, Eqs. (135)-(136))
    with the mixture-mean reference density, every time derivative vanishes."""
    R, g, ag = 10.0, 1e-5, 0.2
    al = 1.0 - ag
    if drag == "const":
        K, kw = 1e-2, dict(drag="const", K_I=1e-2)
    else:
        K, kw = 0.05 * ag * al * (ag + al * R), dict(drag="cgw", kappa_I=0.05)
    slip = math.sqrt(ag * al * (R - 1.0) * g / K)
    N = 6
    ug = np.zeros((2, N, N))
    ul = np.zeros((2, N, N))
    ul[0], ul[1] = 0.002, -0.001
    ug[0], ug[1] = 0.002, -0.001 + slip
    prm = FDParams(2, R, 1.0, 1.0, g_hat=g, up_axis=1, rho_ref=ag * 1.0 + al * R, **kw)
    fd = FD(prm, dict(alpha_g=np.full((N, N), ag), u_g=ug, u_l=ul, dp_k=np.zeros((N, N))))
    r = fd.rhs(fd.dp, fd.u_g, fd.u_l, fd.alpha_g)
    assert max(float(np.max(np.abs(x))) for x in r) < 1e-18
    # 1 % off the slip is not a fixed point
    ug[1] = -0.001 + 1.01 * slip
    r = FD(prm, dict(alpha_g=np.full((N, N), ag), u_g=ug, u_l=ul, dp_k=np.zeros((N, N)))).rhs(
        fd.dp, ug, ul, fd.alpha_g)
    assert float(np.max(np.abs(r[1]))) > 1e-9


def test_fd_uniform_slip_relaxation():
    """Gravity off, uniform state: d(du)/dt = -k |du| du with
    k = K_I (1/alpha_g + 1/(R alpha_l)) (Eqs. (24), (26)), solved by
    du(t) = du0 / (1 + k |du0| t); the mixture momentum alpha_g u_g +
    R alpha_l u_l is constant.  The integrator's error falls as dt^4."""
    R, K, ag = 4.0, 0.3, 0.3
    N = 4
    ug0, ul0 = np.array([0.01, 0.005]), np.array([-0.002, 0.001])
    k = K * (1.0 / ag + 1.0 / (R * (1.0 - ag)))
    T = 40.0
    errs = []
    for dt in (2.0, 1.0):
        ug = np.broadcast_to(ug0[:, None, None], (2, N, N)).copy()
        ul = np.broadcast_to(ul0[:, None, None], (2, N, N)).copy()
        fd = FD(FDParams(2, R, 1.0, 1.0, K_I=K, sigma_grad=False),
                dict(alpha_g=np.full((N, N), ag), u_g=ug, u_l=ul, dp_k=np.zeros((N, N))))
        fd.step(dt, int(T / dt))
        du0 = ul0 - ug0
        du = du0 / (1.0 + k * np.linalg.norm(du0) * T)
        errs.append(float(np.max(np.abs((fd.u_l - fd.u_g)[:, 0, 0] - du))))
        mom = ag * fd.u_g[:, 0, 0] + R * (1 - ag) * fd.u_l[:, 0, 0]
        assert np.max(np.abs(mom - (ag * ug0 + R * (1 - ag) * ul0))) < 1e-17
    assert errs[1] < 1e-11 and 12.0 < errs[0] / errs[1] < 20.0, errs


def test_fd_taylor_green_decay_rate_second_order():
    """Single-phase limit (R = 1, uniform alpha, u_g = u_l): the Taylor-Green
    vortex decays at 2 nu k^2; the FD's rate approaches it at second order."""
    nu_errs = []
    for N in (16, 32, 64):
        X, Y = _grid(N)
        k = 2 * np.pi / N                          # lattice wavenumber
        U = 1e-3
        xs, ys = X * N, Y * N
        u = U * np.stack([np.sin(k * xs) * np.cos(k * ys), -np.cos(k * xs) * np.sin(k * ys)])
        p = -(U * U / 4) * (np.cos(2 * k * xs) + np.cos(2 * k * ys))
        omega = 1.0
        nu = CS2 * (1.0 / omega - 0.5)
        fd = FD(FDParams(2, 1.0, omega, omega), dict(alpha_g=np.full((N, N), 0.5), u_g=u, u_l=u.copy(), dp_k=p))
        steps = N * N // 8
        fd.step(0.5, 2 * steps)
        ratio = np.sum(fd.u_g * u) / np.sum(u * u)
        rate = -math.log(ratio) / steps
        nu_errs.append(abs(rate / (2 * nu * k * k) - 1.0))
    assert nu_errs[0] / nu_errs[1] > 3.5 and nu_errs[1] / nu_errs[2] > 3.5, nu_errs
    assert nu_errs[2] < 2e-3


def test_fd_mixture_sound_speed():
    """Uniform alpha at rest, no viscosity (omega = 2), a small pressure
    wave: the linearised system gives d2p/dt2 = c_s^2 (alpha_g + alpha_l/R)
    lap p, so with central differences the mode cos(k x) oscillates at
    c sin(k), c = c_s sqrt(alpha_g + alpha_l / R)."""
    N, R, ag = 32, 5.0, 0.3
    k = 2 * np.pi / N
    x = np.arange(N)
    dp0 = 1e-9 * np.cos(k * x)
    fd = FD(FDParams(1, R, 2.0, 2.0), dict(alpha_g=np.full(N, ag), u_g=np.zeros((1, N)),
                                           u_l=np.zeros((1, N)), dp_k=dp0))
    c = math.sqrt(CS2 * (ag + (1 - ag) / R))
    w = c * math.sin(k)
    T = 200.0
    fd.step(0.25, int(T / 0.25))
    assert np.max(np.abs(fd.dp - dp0 * math.cos(w * T))) < 1e-4 * 1e-9
    # the wrong speed (no 1/R coupling, c_s sqrt(alpha_g + alpha_l)) is far off
    assert abs(math.cos(CS2 ** 0.5 * math.sin(k) * T) - math.cos(w * T)) > 0.1


def test_fd_gaussian_carried_by_uniform_flow():
    """alpha_g advected by a uniform flow with no slip (chi = 0): the exact
    solution is the translated profile; the FD error falls ~4x per halving
    of h at fixed physical time."""
    errs = []
    for N in (32, 64, 128):
        x = (np.arange(N) + 0.5) / N
        U = 0.2 / N                                  # lattice velocity, fixed physical speed
        a0 = 0.3 + 0.2 * np.exp(-((x - 0.5) ** 2) / (2 * 0.08 ** 2))
        fd = FD(FDParams(1, 3.0, 1.0, 1.0), dict(alpha_g=a0, u_g=np.full((1, N), U), u_l=np.full((1, N), U),
                                                 dp_k=np.zeros(N)))
        steps = N * N // 8
        fd.step(0.5, 2 * steps)
        shift = U * steps / N
        xe = (x - shift) % 1.0
        exact = 0.3 + 0.2 * np.exp(-((xe - 0.5) ** 2) / (2 * 0.08 ** 2))
        errs.append(np.linalg.norm(fd.alpha_g - exact) / np.linalg.norm(exact - 0.3))
        assert np.max(np.abs(fd.u_g - U)) < 1e-17
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_fd_sigma_grad_alpha_conserves_weighted_shear_momentum():
    """A shear layer u = (0, v(x)) over alpha_g(x), no gravity, drag or
    pressure gradient: the forces sigma . grad(alpha) / alpha of Eqs. (24),
    (26) come from (1/alpha) div(alpha sigma) of Eqs. (16)-(17), so
    sum(alpha_phi v_phi) is conserved by the PDE.  The FD keeps it to O(h^2);
    without the term it drifts at O(1)."""
    def drift(N, term):
        x = (np.arange(N) + 0.5) / N
        a = 0.4 + 0.3 * np.sin(2 * np.pi * x) + 0.1 * np.cos(4 * np.pi * x)
        v = 1e-3 * (np.cos(2 * np.pi * x + 0.4) + 0.5 * np.cos(4 * np.pi * x + 1.1)) / N
        z = np.zeros((N, N))
        ug = np.stack([z, np.broadcast_to(v, (N, N)).copy()])
        fd = FD(FDParams(2, 2.0, 1.0, 1.0, sigma_grad=term),
                dict(alpha_g=np.broadcast_to(a, (N, N)).copy(), u_g=ug, u_l=ug.copy(), dp_k=z.copy()))
        m0 = np.sum(fd.alpha_g * fd.u_g[1])
        fd.step(0.5, N * N // 10)
        return abs(np.sum(fd.alpha_g * fd.u_g[1]) - m0) / np.sum(np.abs(fd.alpha_g * ug[1]))
    d = [drift(N, True) for N in (16, 32, 64)]
    assert d[0] / d[1] > 3.5 and d[1] / d[2] > 3.5, d
    assert drift(32, False) > 20 * d[1]


# ------------------------------------------ LBM oracle against the FD


def _refinement_case(N, drag, psi, R):
    """Smooth periodic unit box at N nodes per side (epsilon = 1/N), in the
    diffusive scaling of Sec. 2.1.2: u = epsilon U, p_k - c_s^2 = epsilon^2 p,
    g_hat = epsilon^3 g, K_I = epsilon K (the drag of Eq. (6) scales like the
    other forces), T / epsilon^2 steps, omega fixed, and omega_alpha from
    Eq. (89) at a fixed physical diffusivity chi (so the LBM's alpha
    diffusivity epsilon^2 chi is one of its O(epsilon^2) errors; the FD
    carries none).  Initial state: a Taylor-Green flow shared by both phases
    (its own pressure, so no acoustic transient) over a smooth gas fraction;
    buoyancy and drag then build the slip."""
    eps = 1.0 / N
    X, Y = _grid(N)
    k = 2 * np.pi
    U, g, K, kappa, chi, omega = 0.5, 1.0, 10.0, 30.0, 1.0, 1.0
    a = 0.3 + 0.1 * np.sin(k * X) * np.cos(k * Y)
    u = np.stack([U * np.sin(k * X) * np.cos(k * Y), -U * np.cos(k * X) * np.sin(k * Y)])
    p = -(U * U / 4) * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    fields = dict(alpha_g=a, u_g=eps * u, u_l=eps * u.copy(), dp_k=eps * eps * p)
    rho_ref = float(np.mean(a)) + (1.0 - float(np.mean(a))) * R
    omega_a = 2.0 / (1.0 + 2.0 * eps * eps * chi / CS2)                 # Eq. (89)
    kw = dict(drag=drag, K_I=K * eps, kappa_I=kappa * eps, g_hat=g * eps ** 3)
    cfg = workloads._base("D2Q9", nx=N, ny=N, rho_g=1.0, rho_l=R, omega_g=omega, omega_l=omega,
                          psi_g=psi, psi_l=psi, omega_ag=omega_a, omega_al=omega_a, rho_ref=rho_ref,
                          up_axis=1, **kw)
    prm = FDParams(2, R, omega, omega, psi_g=psi, psi_l=psi, up_axis=1, rho_ref=rho_ref, **kw)
    return cfg, prm, fields


@pytest.mark.parametrize("drag,psi,R", [("const", 0.0, 10.0), ("cgw", 0.0, 10.0)])
def test_lbm_approaches_fd_at_second_order(drag, psi, R):
    """||LBM - FD|| / ||FD|| per field (alpha_g, u_g, u_l, p_k - c_s^2) at
    the physical time T = 1/4 on 16^2, 32^2 and 64^2 lattices: every field's
    error falls by a ratio in [3, 5] per halving of the lattice spacing.
    gamma = 0 and n_gamma = 1 (the stabilisers of Sec. 3.2 are not part of
    the FD system)."""
    T = 0.25
    prev = None
    for N in (16, 32, 64):
        cfg, prm, f = _refinement_case(N, drag, psi, R)
        steps = int(round(T * N * N))
        o = Oracle(cfg, f)
        o.step(steps)
        fd = FD(prm, f)
        fd.step(0.5, 2 * steps)
        ro, rf = o.read(), fd.read()
        err = {k: np.linalg.norm(ro[k] - rf[k]) / np.linalg.norm(rf[k]) for k in ("alpha_g", "u_g", "u_l", "dp_k")}
        print(f"  N={N} " + " ".join(f"{k}={v:.3e}" for k, v in err.items()), flush=True)
        if prev is not None:
            for k in err:
                r = prev[k] / err[k]
                assert 3.0 <= r <= 5.0, (N, k, r)
        prev = err
    assert max(prev.values()) < 0.02
