"""Pins of the oracle's equilibria against what the paper fixes about them:
moment identities (Eqs. (50)-(51), (80)-(81), the right-hand side of
Eq. (49)) and the D1Q3 closed forms printed in Appendix A."""
import numpy as np
import pytest

from oracle import CS2, d1q3, d2q9, d3q19
from oracle import equilibria as eq

LATTICES = [d1q3, d2q9, d3q19]


def _rand(lat, rng, n=5):
    D = lat.D
    phi = 1.0 + 0.1 * rng.standard_normal(n)
    eps = 1.0 + 0.05 * rng.standard_normal(n)
    u = 0.05 * rng.standard_normal((D, n))
    return phi, eps, u


def _mom(lat, f):
    v = lat.v.astype(float)
    return (f.sum(0), np.einsum("qc,q...->c...", v, f), np.einsum("qc,qd,q...->cd...", v, v, f),
            np.einsum("qc,qd,qe,q...->cde...", v, v, v, f))


@pytest.mark.parametrize("mk", LATTICES)
def test_weights_isotropy(mk):
    lat = mk()
    v = lat.v.astype(float)
    D = lat.D
    assert abs(lat.w.sum() - 1.0) < 1e-15
    assert np.allclose(np.einsum("q,qc,qd->cd", lat.w, v, v), CS2 * np.eye(D), atol=1e-15)
    assert np.allclose(np.einsum("q,qc->c", lat.w, v), 0.0, atol=1e-16)
    if D > 1:
        # fourth-order isotropy needed by the quadratic equilibrium terms
        I = np.eye(D)
        iso = CS2 * CS2 * (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
                           + np.einsum("ad,bc->abcd", I, I))
        assert np.allclose(np.einsum("q,qa,qb,qc,qd->abcd", lat.w, v, v, v, v), iso, atol=1e-15)
    for q in range(lat.Q):
        assert np.all(lat.v[lat.opp[q]] == -lat.v[q])


@pytest.mark.parametrize("mk", LATTICES)
def test_incompressible_equilibrium_moments(mk):
    lat = mk()
    rng = np.random.default_rng(1)
    phi, eps, u = _rand(lat, rng)
    f = eq.feq_I(lat, phi, eps, u)
    m0, m1, m2, m3 = _mom(lat, f)
    D = lat.D
    I = np.eye(D)[:, :, None]
    assert np.allclose(m0, eps, rtol=0, atol=1e-14)                       # text before Eq. (38)
    assert np.allclose(m1, u, rtol=0, atol=1e-15)                         # incompressibility of f_I
    uu = np.einsum("cn,dn->cdn", u, u)
    assert np.allclose(m2, phi * CS2 * eps * I + uu, rtol=0, atol=1e-14)  # Eq. (50)
    if D > 1:
        ref3 = CS2 * (np.einsum("an,bc->abcn", u, np.eye(D)) + np.einsum("bn,ac->abcn", u, np.eye(D))
                      + np.einsum("cn,ab->abcn", u, np.eye(D)))
        assert np.allclose(m3, ref3, rtol=0, atol=1e-15)                  # Eq. (51)


@pytest.mark.parametrize("mk", LATTICES)
def test_standard_equilibrium_moments(mk):
    lat = mk()
    rng = np.random.default_rng(2)
    _, a, u = _rand(lat, rng)
    a = a - 0.7
    f = eq.feq_S(lat, a, u)
    m0, m1, m2, m3 = _mom(lat, f)
    D = lat.D
    I = np.eye(D)[:, :, None]
    assert np.allclose(m0, a, rtol=0, atol=1e-15)                         # Eq. (73) at equilibrium
    assert np.allclose(m1, a * u, rtol=0, atol=1e-15)
    uu = np.einsum("cn,dn->cdn", u, u)
    assert np.allclose(m2, CS2 * a * I + a * uu, rtol=0, atol=1e-15)      # Eq. (80)
    if D > 1:
        ref3 = CS2 * a * (np.einsum("an,bc->abcn", u, np.eye(D)) + np.einsum("bn,ac->abcn", u, np.eye(D))
                          + np.einsum("cn,ab->abcn", u, np.eye(D)))
        assert np.allclose(m3, ref3, rtol=0, atol=1e-15)                  # Eq. (81)


@pytest.mark.parametrize("mk", LATTICES)
def test_forcing_operator_moments(mk):
    lat = mk()
    rng = np.random.default_rng(3)
    psi, S, G = _rand(lat, rng)
    S = S - 1.0
    f = eq.feq_L(lat, psi, S, G)
    m0, m1, m2, _ = _mom(lat, f)
    I = np.eye(lat.D)[:, :, None]
    assert np.allclose(m0, S, rtol=0, atol=1e-15)          # source of Eq. (47)
    assert np.allclose(m1, G, rtol=0, atol=1e-15)          # force of Eq. (48)
    assert np.allclose(m2, psi * CS2 * S * I, rtol=0, atol=1e-15)   # psi c_s^2 S I of Eq. (49)


def test_d1q3_appendix_a_closed_forms():
    """Appendix A, Eqs. (A.2)-(A.4), typed from the paper's D1Q3 expressions
    and compared with the general-dimension functions at D1Q3 weights."""
    lat = d1q3()
    rng = np.random.default_rng(4)
    for _ in range(20):
        a, e, phi, psi, u, S, G = rng.uniform(-1.5, 1.5, 7)
        fS = eq.feq_S(lat, np.array(a), np.array([u]))
        fI = eq.feq_I(lat, np.array(phi), np.array(e), np.array([u]))
        fL = eq.feq_L(lat, np.array(psi), np.array(S), np.array([G]))
        ref_S = [a * (2 / 3 - u * u), a * (1 + 3 * u + 3 * u * u) / 6, a * (1 - 3 * u + 3 * u * u) / 6]
        ref_I = [e * (3 - phi) / 3 - u * u, (e * phi + 3 * u + 3 * u * u) / 6, (e * phi - 3 * u + 3 * u * u) / 6]
        ref_L = [S * (3 - psi) / 3, (S * psi + 3 * G) / 6, (S * psi - 3 * G) / 6]
        assert np.allclose(fS, ref_S, rtol=0, atol=1e-14)
        assert np.allclose(fI, ref_I, rtol=0, atol=1e-14)
        assert np.allclose(fL, ref_L, rtol=0, atol=1e-14)


def test_eta_reduces_to_standard_equilibrium_at_phi_one():
    """With phi = 1, eta_q = 1 (Eq. (38)) and f_I^eq(1, 1, u) equals the
    standard equilibrium f^eq(1, u) (Eq. (72)) on every lattice."""
    rng = np.random.default_rng(5)
    for mk in LATTICES:
        lat = mk()
        u = 0.05 * rng.standard_normal((lat.D, 7))
        one = np.ones(7)
        assert np.allclose(eq.feq_I(lat, one, one, u), eq.feq_S(lat, one, u), rtol=0, atol=1e-16)
        assert np.allclose(eq.eta(lat, one), 1.0)
