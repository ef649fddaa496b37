"""Pins of the oracle's softening laws and critical stretch (appendix A)
against the paper's printed bond-energy integral, numerical quadrature of the
fracture-energy integral and the laws' continuity conditions."""
import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import solver as S

K, ALPHA, GF, E = W.SOFT_K, W.SOFT_ALPHA, W.FRACTURE_ENERGY, W.E_MODULUS
S0 = W.S0_MEAN


def envelope_force(law, s, s0, sc, c):
    """Force along the monotone loading envelope, f = c (1 - D(s)) s."""
    return c * (1.0 - S.damage(law, s, s0, sc, K, ALPHA)) * s


def test_fracture_energy_geometry_factor():
    """The appendix-A 4-fold integral with w = xi * A (A the area under the
    force-stretch curve) equals A delta^5 pi / 5.  Integrate the geometric part
    numerically with delta = 1."""
    val, _ = integrate.nquad(
        lambda phi, xi, th, z: xi ** 3 * np.sin(phi),
        [lambda xi, th, z: (0.0, np.arccos(min(1.0, z / xi))),
         lambda th, z: (z, 1.0), (0.0, 2 * np.pi), (0.0, 1.0)],
        opts={"epsabs": 1e-11, "epsrel": 1e-11})
    assert val == pytest.approx(np.pi / 5, rel=1e-8)


@pytest.mark.parametrize("law", [S.LAW_EXPLIN, S.LAW_TRILINEAR])
@pytest.mark.parametrize("dx", [5e-3, 2.5e-3, 1.25e-3])
def test_critical_stretch_reproduces_fracture_energy(law, dx):
    delta = W.M_RATIO * dx
    c = S.micromodulus(E, delta)
    sc = S.critical_stretch(law, S0, c, GF, delta, K, ALPHA)
    assert sc > S0
    pts = [S0 + (sc - S0) * t for t in (0.05, 0.2, 0.5)]
    area, _ = integrate.quad(lambda s: envelope_force(law, s, S0, sc, c), S0, sc,
                             points=pts, limit=400, epsabs=0, epsrel=1e-12)
    assert area * delta ** 5 * np.pi / 5 == pytest.approx(GF, rel=1e-8)


def test_explin_bond_energy_closed_form():
    """Eq. exp_bond_energy: w = c s0 xi (s0 - sc) P / (2 k (e^k - 1)(1 + alpha))
    equals the quadrature of f xi over [s0, sc] with the oracle's damage law."""
    c, xi, sc = 3.0e18, 0.01, 7.5e-3
    ek = np.exp(K)
    P = 2 * K - 2 * ek + ALPHA * K - ALPHA * K * ek + 2
    w_paper = c * S0 * xi * (S0 - sc) * P / (2 * K * (ek - 1) * (1 + ALPHA))
    w_quad, _ = integrate.quad(lambda s: envelope_force(S.LAW_EXPLIN, s, S0, sc, c) * xi, S0, sc,
                               limit=400, epsabs=0, epsrel=1e-12,
                               points=[S0 + (sc - S0) * t for t in (0.01, 0.05, 0.2)])
    assert w_quad == pytest.approx(w_paper, rel=1e-9)


def test_printed_sc_rearrangement_differs_by_alpha_s0():
    """The printed 3D rearrangement (Eq. exp_sc) lacks the (1 + alpha) factor
    inside its bracket; it exceeds the consistent root of the energy relation
    by exactly alpha * s0."""
    delta = W.M_RATIO * 5e-3
    c = S.micromodulus(E, delta)
    ek = np.exp(K)
    P = 2 * K - 2 * ek + ALPHA * K - ALPHA * K * ek + 2
    printed = (10 * K * (1 - ek) * (1 + ALPHA)
               * (GF - np.pi * c * delta ** 5 * S0 ** 2 * P / (10 * K * (ek - 1)))
               / (c * delta ** 5 * S0 * np.pi * P))
    ours = S.critical_stretch(S.LAW_EXPLIN, S0, c, GF, delta, K, ALPHA)
    assert printed - ours == pytest.approx(ALPHA * S0, rel=1e-6)


@pytest.mark.parametrize("law", [S.LAW_EXPLIN, S.LAW_TRILINEAR])
def test_law_continuity_and_monotone_damage(law):
    c, sc = 1.0, 50 * S0
    # f(s0) = c s0 and f(sc) = 0, approached from inside
    assert envelope_force(law, S0 * (1 + 1e-12), S0, sc, c) == pytest.approx(c * S0, rel=1e-9)
    assert abs(envelope_force(law, sc * (1 - 1e-12), S0, sc, c)) < 1e-9 * c * S0
    assert S.damage(law, 0.5 * S0, S0, sc, K, ALPHA) == 0.0
    assert S.damage(law, -1.0, S0, sc, K, ALPHA) == 0.0
    assert S.damage(law, 2 * sc, S0, sc, K, ALPHA) == 1.0
    ks = np.linspace(0, 1.2 * sc, 4001)
    d = np.array([S.damage(law, x, S0, sc, K, ALPHA) for x in ks])
    assert np.all(np.diff(d) >= -1e-15) and d.min() >= 0 and d.max() <= 1
    if law == S.LAW_TRILINEAR:
        s1 = S0 + 0.2 * (sc - S0)
        assert envelope_force(law, s1, S0, sc, c) == pytest.approx(0.2 * c * S0, rel=1e-12)
