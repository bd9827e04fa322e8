"""Equilibrium functions of the six schemes, written as the paper defines them
(test infrastructure, see oracle/__init__.py).

Array conventions: a scalar field has the grid shape, a vector field has a
leading component axis (D, *grid) ordered (x, y, z), and a population set has a
leading direction axis (Q, *grid).
"""
import numpy as np

from .lattice import CS2


def _cu(lat, u):
    """v_q . u for every direction: (Q, *grid)."""
    return np.einsum("qc,c...->q...", lat.v.astype(np.float64), u)


def _wq(lat, ndim):
    return lat.w.reshape((-1,) + (1,) * ndim)


def eta(lat, phi):
    """eta_q(phi), Eq. (38) with delta_q of Eq. (39); shape (Q, *phi.shape)."""
    phi = np.asarray(phi, dtype=np.float64)
    w0 = lat.w[0]
    out = np.empty((lat.Q,) + phi.shape)
    out[0] = 1.0 + (1.0 - w0) / w0 * (1.0 - phi)   # delta_q = 1
    out[1:] = phi                                   # delta_q = 0
    return out


def feq_I(lat, phi, eps, u):
    """Incompressible equilibrium f_I^eq(phi, eps, u), Eq. (37)."""
    eps = np.asarray(eps, dtype=np.float64)
    cu = _cu(lat, u)
    usq = np.sum(u * u, axis=0)
    w = _wq(lat, eps.ndim)
    return w * (eps * eta(lat, np.broadcast_to(phi, eps.shape))
                + cu / CS2 + (cu * cu - CS2 * usq) / (2.0 * CS2 * CS2))


def feq_S(lat, alpha, u):
    """Standard equilibrium f^eq(alpha, u), Eq. (72) (used for f_alpha and f_beta)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    cu = _cu(lat, u)
    usq = np.sum(u * u, axis=0)
    w = _wq(lat, alpha.ndim)
    return w * alpha * (1.0 + cu / CS2 + (cu * cu - CS2 * usq) / (2.0 * CS2 * CS2))


def feq_L(lat, psi, S, G):
    """Linearised equilibrium of the forcing operator f_L^eq(psi, S, G), Eq. (42)."""
    S = np.asarray(S, dtype=np.float64)
    cG = _cu(lat, G)
    w = _wq(lat, S.ndim)
    return w * (S * eta(lat, np.broadcast_to(psi, S.shape)) + cG / CS2)
