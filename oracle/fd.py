"""Finite-difference reference of the two-fluid artificially compressible
system (test infrastructure, see oracle/__init__.py).

Sec. 3.4 builds a finite-difference (FD) engine for the one-dimensional form
of the system the six LBM schemes approximate: central differences D_x and
D_x^2 (Eqs. (143)-(144)), the method of lines (Eqs. (145)-(148)) and an
explicit Runge-Kutta integrator.  This module is its periodic counterpart in
one, two or three dimensions, written in lattice units (hats dropped), for the
fields dp = p_k - c_s^2 (kinematic pressure deviation), u_g, u_l and alpha_g:

  d dp / dt   = c_s^2 (S_g - div u_g)                         Eqs. (19), (145)
  d u_g / dt  = -div(u_g u_g) - grad dp + div sigma_g + G_g     Eqs. (23), (146)
  d u_l / dt  = -div(u_l u_l) - (1/R) grad dp + div sigma_l + G_l   Eqs. (25), (147)
  d alpha_g/dt = -div(alpha_g u_g) + chi lap alpha_g            Eqs. (10), (148) (chi = 0: as written)

with S_g = div(alpha_l (u_g - u_l)), S_l = div(alpha_g (u_l - u_g))
(Eqs. (19)-(20)); the liquid feels (1/R) grad dp through its equation of
state (Eq. (32)); the stress that the momentum schemes recover (Eqs. (64),
(67)-(68)),

  sigma = nu (grad u + grad u^T + (div u) I) - (c_s^2 psi / omega) (div u) I,

nu = c_s^2 (1/omega - 1/2) (Eq. (65)), i.e. Eq. (7) with the bulk viscosity
of Eq. (66); and the forces of Eqs. (24), (26):

  G_g = S_g u_g + sigma_g . grad alpha_g / alpha_g + b_g e_up + (K_I/alpha_g) |du| du
  G_l = S_l u_l + sigma_l . grad alpha_l / alpha_l + b_l e_up - (K_I/(R alpha_l)) |du| du
        - (K_W/(R alpha_l)) |u_l| u_l,          du = u_l - u_g,

K_I constant or the Clift-Grace-Weber K_I = kappa_I alpha_g alpha_l (alpha_g +
alpha_l R) of Eq. (135) (no lag: the FD engine of the paper has none), the
buoyancy b_phi = (rho_ref / rho_phi - 1) g_hat along the up axis (reading R8
of the LBM oracle) and the 1/alpha factors floored at alpha_min (reading R13).

Discretisation: first derivatives are the central difference of Eq. (143)
along each axis; the Laplacian is the sum of the compact second differences of
Eq. (144); the mixed second derivatives d_i d_j (i != j) of div sigma are
products of central differences.  Time: the classical fourth-order
Runge-Kutta method (Kutta, 1901) with a fixed step -- the paper used the
adaptive Dormand-Prince pair of MATLAB's ode45; any integrator whose error is
far below the spatial one serves the comparison.  The paper also filters the
FD solution against checkerboard modes every ~100 steps; smooth periodic
cases over short times do not need it and none is applied.

Nothing here is shared with the LBM oracle (oracle/scheme.py) or with the HIP
path.  Pins: tests/test_oracle_fd.py.
"""
import numpy as np

CS2 = 1.0 / 3.0


class FDParams:
    """Physical parameters of the system in lattice units."""

    def __init__(self, D, R, omega_g, omega_l, psi_g=0.0, psi_l=0.0, drag="const", K_I=0.0, kappa_I=0.0,
                 K_W=0.0, g_hat=0.0, up_axis=None, rho_g=1.0, rho_ref=None, alpha_min=1e-6, chi=0.0,
                 sigma_grad=True):
        self.D = int(D)
        self.R = float(R)
        self.rho_g = float(rho_g)
        self.rho_l = self.R * self.rho_g
        self.nu_g = CS2 * (1.0 / omega_g - 0.5)          # Eq. (65)
        self.nu_l = CS2 * (1.0 / omega_l - 0.5)
        self.bulk_g = CS2 * psi_g / omega_g               # Eq. (68): (c_s^2 psi / omega) div u I
        self.bulk_l = CS2 * psi_l / omega_l
        self.drag = drag
        self.K_I, self.kappa_I, self.K_W = float(K_I), float(kappa_I), float(K_W)
        self.g_hat = float(g_hat)
        self.up = self.D - 1 if up_axis is None else int(up_axis)
        self.rho_ref = self.rho_l if rho_ref is None else float(rho_ref)
        self.alpha_min = float(alpha_min)
        self.chi = float(chi)
        self.sigma_grad = bool(sigma_grad)


# ------------------------------------------------------------- operators
# Arrays are (..., n_{D-1}, ..., n_0) with component c of space along array
# axis -1 - c (x fastest), periodic.

def _ax(c):
    return -1 - c


def d1(f, c):
    """Central difference along component c, Eq. (143): (f(i+1) - f(i-1)) / 2."""
    return 0.5 * (np.roll(f, -1, axis=_ax(c)) - np.roll(f, 1, axis=_ax(c)))


def d2(f, c):
    """Compact second difference along component c, Eq. (144)."""
    return np.roll(f, -1, axis=_ax(c)) - 2.0 * f + np.roll(f, 1, axis=_ax(c))


def div(v, D):
    return sum(d1(v[c], c) for c in range(D))


def grad(s, D):
    return np.stack([d1(s, c) for c in range(D)])


def lap(s, D):
    return sum(d2(s, c) for c in range(D))


def dd(f, i, j):
    """Second derivative d_i d_j: compact for i = j, product of central
    differences otherwise."""
    return d2(f, i) if i == j else d1(d1(f, i), j)


class FD:
    """Method-of-lines state (dp, u_g, u_l, alpha_g) on a periodic grid."""

    def __init__(self, prm, fields):
        self.p = prm
        D = prm.D
        self.dp = np.array(fields["dp_k"], dtype=np.float64)
        shape = self.dp.shape
        assert len(shape) == D
        self.u_g = np.array(fields["u_g"], dtype=np.float64).reshape((D,) + shape)
        self.u_l = np.array(fields["u_l"], dtype=np.float64).reshape((D,) + shape)
        self.alpha_g = np.array(fields["alpha_g"], dtype=np.float64).reshape(shape)
        self.t = 0.0

    # ---------------------------------------------------------------- terms
    def _stress_div(self, u, nu, bulk):
        """div sigma with sigma = nu (grad u + grad u^T + div u I) - bulk div u I:
        component i = nu lap u_i + (2 nu - bulk) d_i (div u)."""
        D = self.p.D
        out = []
        for i in range(D):
            gd = sum(dd(u[j], i, j) for j in range(D))     # d_i (div u)
            out.append(nu * lap(u[i], D) + (2.0 * nu - bulk) * gd)
        return np.stack(out)

    def _stress(self, u, nu, bulk):
        """sigma as a (D, D, ...) tensor from central differences."""
        D = self.p.D
        g = np.stack([np.stack([d1(u[i], j) for j in range(D)]) for i in range(D)])   # g[i, j] = d_j u_i
        dv = sum(g[k, k] for k in range(D))
        s = nu * (g + np.swapaxes(g, 0, 1))
        for k in range(D):
            s[k, k] = s[k, k] + (nu - bulk) * dv
        return s

    def _adv(self, u):
        """div(u u): component i = sum_j d_j (u_i u_j)."""
        D = self.p.D
        return np.stack([sum(d1(u[i] * u[j], j) for j in range(D)) for i in range(D)])

    def rhs(self, dp, u_g, u_l, a_g):
        p = self.p
        D = p.D
        a_l = 1.0 - a_g
        S_g = div(a_l * (u_g - u_l), D)                                   # Eq. (19)
        S_l = div(a_g * (u_l - u_g), D)                                   # Eq. (20)
        gp = grad(dp, D)
        ga_g = grad(a_g, D)
        ag_f = np.maximum(a_g, p.alpha_min)
        al_f = np.maximum(a_l, p.alpha_min)
        du = u_l - u_g
        dun = np.sqrt(np.sum(du * du, axis=0))
        K = p.kappa_I * a_g * a_l * (a_g + a_l * p.R) if p.drag == "cgw" else p.K_I   # Eq. (135)
        e_up = np.zeros((D,) + (1,) * D)
        e_up[p.up] = 1.0
        b_g = (p.rho_ref / p.rho_g - 1.0) * p.g_hat
        b_l = (p.rho_ref / p.rho_l - 1.0) * p.g_hat

        sig_g = self._stress(u_g, p.nu_g, p.bulk_g)
        sig_l = self._stress(u_l, p.nu_l, p.bulk_l)
        if p.sigma_grad:
            sga_g = np.einsum("ij...,j...->i...", sig_g, ga_g) / ag_f
            sga_l = np.einsum("ij...,j...->i...", sig_l, -ga_g) / al_f   # grad alpha_l = -grad alpha_g
        else:
            sga_g = sga_l = 0.0
        ul_n = np.sqrt(np.sum(u_l * u_l, axis=0))
        G_g = S_g * u_g + sga_g + b_g * e_up + (K / ag_f) * dun * du                        # Eq. (24)
        G_l = S_l * u_l + sga_l + b_l * e_up - (K / (p.R * al_f)) * dun * du \
            - (p.K_W / (p.R * al_f)) * ul_n * u_l                                          # Eq. (26)

        ddp = CS2 * (S_g - div(u_g, D))
        du_g = -self._adv(u_g) - gp + self._stress_div(u_g, p.nu_g, p.bulk_g) + G_g
        du_l = -self._adv(u_l) - gp / p.R + self._stress_div(u_l, p.nu_l, p.bulk_l) + G_l
        da_g = -div(a_g * u_g, D)
        if p.chi != 0.0:
            da_g = da_g + p.chi * lap(a_g, D)
        return ddp, du_g, du_l, da_g

    # ----------------------------------------------------------------- time
    def step(self, dt, n=1):
        """n steps of the classical fourth-order Runge-Kutta method."""
        for _ in range(int(n)):
            y = (self.dp, self.u_g, self.u_l, self.alpha_g)
            k1 = self.rhs(*y)
            k2 = self.rhs(*[a + 0.5 * dt * b for a, b in zip(y, k1)])
            k3 = self.rhs(*[a + 0.5 * dt * b for a, b in zip(y, k2)])
            k4 = self.rhs(*[a + dt * b for a, b in zip(y, k3)])
            self.dp, self.u_g, self.u_l, self.alpha_g = [
                a + (dt / 6.0) * (b1 + 2.0 * b2 + 2.0 * b3 + b4) for a, b1, b2, b3, b4 in zip(y, k1, k2, k3, k4)]
            self.t += dt

    def read(self):
        return {"alpha_g": self.alpha_g.copy(), "u_g": self.u_g.copy(), "u_l": self.u_l.copy(),
                "dp_k": self.dp.copy()}

