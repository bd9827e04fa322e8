"""Physical-to-lattice similarity mapping and the closed-form steady states of
the 1D tube (test infrastructure, see oracle/__init__.py)."""
import math


def similarity(g, g_hat, kappa, kappa_hat):
    """Sec. 3.3: c/tau = g / g_hat (Eq. (138)), c tau = kappa_hat / kappa
    (Eq. (139)), c = sqrt((c/tau)(c tau)) (Eq. (140))."""
    c_over_tau = g / g_hat
    c_tau = kappa_hat / kappa
    c = math.sqrt(c_over_tau * c_tau)
    return {"c_over_tau": c_over_tau, "c_tau": c_tau, "c": c, "tau": c / c_over_tau}


def kappa_cgw(Cd, d):
    """kappa_I = 3 C_d / (4 d), Sec. 3.3 (text before Eq. (135))."""
    return 3.0 * Cd / (4.0 * d)


def cgw_lambda(alpha_g, R):
    """Lambda(alpha_g) = alpha_g alpha_l (alpha_g + alpha_l R), Eq. (136)."""
    alpha_l = 1.0 - alpha_g
    return alpha_g * alpha_l * (alpha_g + alpha_l * R)


def m_ex(kappa, alpha_g, R, du, g):
    """Exchange-to-buoyancy force ratio, Eq. (141)."""
    return kappa * cgw_lambda(alpha_g, R) * du * du / alpha_g / ((R - 1.0) * g)


def slip_u0(K_I, alpha_g, R, g):
    """Eq. (124): (R-1) g = K_I / (alpha_g alpha_l) |u0| u0, solved for u0 > 0."""
    return math.sqrt(alpha_g * (1.0 - alpha_g) * (R - 1.0) * g / K_I)


def steady_ul(ug, ug0, r):
    """Eq. (127): liquid velocity of the uniform-gradient steady state."""
    return (ug - math.sqrt(ug * ug - (1.0 - r) * (ug * ug - ug0 * ug0))) / (1.0 - r)


def steady_ul_r1(ug, ug0):
    """The r -> 1 limit printed after Eq. (127)."""
    return (ug - ug0) * (1.0 + ug0 / ug) / 2.0
