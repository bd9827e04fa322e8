"""Closed-form results the scheme must reproduce exactly (shared by the
oracle pins and the GPU tests)."""
import numpy as np

import workloads


def poiseuille_case(lattice, nx, omega_g, omega_l):
    """Plane Poiseuille flow of both phases: no-slip walls at x = -1/2 and
    x = nx - 1/2 (half-way bounce-back), periodic along the other axes, a
    uniform gas fraction 0.25 (so the volume-fraction gradient vanishes), no
    drag, buoyancy b_phi = (rho_ref / rho_phi - 1) g_hat along the flow axis
    (rho_ref between the phase densities: the gas is pushed one way, the
    liquid the other).  Returns (cfg, fields, exact) with exact(phase) the
    steady velocity profile along x."""
    rho_g, rho_l, rho_ref, g = 1.0, 2.0, 1.5, 1e-6
    if lattice == "D2Q9":
        shape, up, bc = (2, nx), 1, {"x-": "wall", "x+": "wall", "y-": "periodic", "y+": "periodic"}
        extra = {}
    else:
        shape, up = (2, 2, nx), 2
        bc = {"x-": "wall", "x+": "wall", "y-": "periodic", "y+": "periodic", "z-": "periodic", "z+": "periodic"}
        extra = {"nz": 2}
    D = len(shape)
    cfg = workloads._base(lattice, nx=nx, ny=2, rho_g=rho_g, rho_l=rho_l, omega_g=omega_g, omega_l=omega_l,
                          g_hat=g, rho_ref=rho_ref, up_axis=up, drag="const", K_I=0.0, bc=bc, **extra)
    fields = dict(alpha_g=np.full(shape, 0.25), u_g=np.zeros((D,) + shape), u_l=np.zeros((D,) + shape),
                  dp_k=np.zeros(shape))

    def exact(phase):
        # steady solution of the BGK scheme with half-way bounce-back walls
        # under a uniform body force b: the parabola with the walls half-way
        # between nodes plus a uniform slip (16 tau^2 - 20 tau + 3) / 12 in
        # units of b / (2 nu), tau = 1 / omega, nu = (tau - 1/2) / 3
        omega, rho = (omega_g, rho_g) if phase == "g" else (omega_l, rho_l)
        b = (rho_ref / rho - 1.0) * g
        tau = 1.0 / omega
        nu = (tau - 0.5) / 3.0
        x = np.arange(nx)
        return b / (2.0 * nu) * ((x + 0.5) * (nx - 0.5 - x) + (16.0 * tau * tau - 20.0 * tau + 3.0) / 12.0)

    return cfg, fields, up, exact
