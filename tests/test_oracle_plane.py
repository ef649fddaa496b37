"""Pins of the oracle's plane-stress body (appendix A: Eq.
bond_stiffness_constant, plane-stress row; two-dimensional case, Eqs.
exp_fracture_energy_2D and exp_sc_2D; section 6.2: Specimen 3 and Table
discretisation).

A plane-stress body is the 3D lattice one node thick: only the 28 in-plane
offsets of the 122-point stencil find a neighbour, the nodal volume is
dx^2 t and c = 9E / (pi t delta^3).  The pins are continuum closed forms
(energy density and Navier operator of a plane-stress solid with Poisson's
ratio 1/3), the fracture-energy integral by quadrature, the paper's printed
2D critical stretch, brute-force neighbour counts and the paper's level
table."""
import dataclasses
import itertools
import os

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import geometry as G
from oracle import solver as S

HERE = os.path.dirname(os.path.abspath(__file__))
E, RHO, T = W.E_MODULUS, W.DENSITY, 50e-3
K, ALPHA, GF, S0 = W.SOFT_K, W.SOFT_ALPHA, W.FRACTURE_ENERGY, W.S0_MEAN


# (micromodulus, Poisson's ratio of the bond-based solid) per plane model
MODELS = {"stress": (S.micromodulus_plane_stress, 1.0 / 3.0), "strain": (S.micromodulus_plane_strain, 0.25)}


def plane_problem(shape, dx=1e-3, t=T, model="stress", **kw):
    bi, bj, v = G.unique_bonds(shape, W.M_RATIO)
    M = int(np.prod(shape))
    delta = W.M_RATIO * dx
    args = dict(shape=shape, dx=dx, bond_i=bi, bond_j=bj, xi=v * dx,
                support=np.zeros(0, dtype=np.int64), load=np.zeros(0, dtype=np.int64),
                s0=np.full(M, S0), c=np.full(M, MODELS[model][0](E, delta, t)), rho=RHO,
                damping=0.0, dt=1e-7, du=0.0, n_steps=0, law=S.LAW_TRILINEAR,
                k=K, alpha=ALPHA, GF=GF, delta=delta, thickness=t)
    args.update(kw)
    return S.Problem(**args)


def interior_2d(shape, layers=3):
    nx, ny, nz = shape
    assert ny == 1
    k, i = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    ok = (i >= layers) & (i < nx - layers) & (k >= layers) & (k < nz - layers)
    return np.nonzero(ok.ravel())[0]


def in_plane_offsets():
    return [(a, b) for a, b in itertools.product(range(-3, 4), repeat=2)
            if 0 < a * a + b * b <= W.M_RATIO ** 2]


# ---------------------------------------------------------------- lattice
def test_in_plane_stencil_has_28_offsets():
    st = G.stencil(W.M_RATIO)
    ip = st[st[:, 1] == 0]
    assert len(ip) == 28 == len(in_plane_offsets())
    assert sorted(map(tuple, ip[:, [0, 2]].tolist())) == sorted(in_plane_offsets())
    assert np.sum(1.0 / np.linalg.norm(ip, axis=1)) == pytest.approx(15.15368278, rel=1e-8)


@pytest.mark.parametrize("shape", [(9, 1, 7), (4, 1, 11), (35, 1, 10)])
def test_plane_bonds_match_brute_force(shape):
    nx, _, nz = shape
    pts = [(i, k) for k in range(nz) for i in range(nx)]
    want = {(p, q) for p in range(len(pts)) for q in range(p + 1, len(pts))
            if (pts[p][0] - pts[q][0]) ** 2 + (pts[p][1] - pts[q][1]) ** 2 <= W.M_RATIO ** 2}
    bi, bj, v = G.unique_bonds(shape, W.M_RATIO)
    assert np.all(v[:, 1] == 0)
    got = {(min(a, b), max(a, b)) for a, b in zip(bi.tolist(), bj.tolist())}
    assert got == want and len(got) == bi.size


def test_specimen3_levels_follow_the_paper_table():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "table_discretisation.txt"))
            if l.strip() and not l.startswith("#")]
    for lev, dx_mm, nodes in rows:
        lv = W.level2d(int(lev))
        assert lv.dx == pytest.approx(1e-3 * float(dx_mm), rel=1e-12)
        nx, ny, nz = lv.shape
        assert ny == 1 and nx * nz == int(nodes)
        # pads hold whole node columns at every level; the notch reaches half the depth
        sup, load = G.beam_pads(lv.shape, lv.dx, lv.beam)
        assert sup.size > 0 and load.size > 0
    assert W.SPECIMEN3.notch_depth == pytest.approx(0.5 * W.SPECIMEN3.depth)


# ---------------------------------------------------------------- micromodulus
@pytest.mark.parametrize("model", ["stress", "strain"])
def test_isotropic_strain_energy_density(model):
    """u = eps x in plane: every bond has stretch eps and the interior energy
    density (1/2) sum_j (c / 2) eps^2 |xi| V equals the lattice form of the
    continuum value, times sum_v |v| / (2 pi m^3 / 3): in plane stress
    (nu = 1/3) E eps^2 / (1 - nu) = 3 E eps^2 / 2; in plane strain (nu = 1/4)
    2 (lambda + mu) eps^2 = E eps^2 / ((1 + nu)(1 - 2 nu)) = 8 E eps^2 / 5."""
    shape, dx, eps = (13, 1, 13), 1e-3, 2e-5
    p = plane_problem(shape, dx, model=model)
    x = G.node_positions(shape, dx)
    u = eps * x
    u[:, 1] = 0.0
    s = p.stretch(u)
    assert np.max(np.abs(s - eps)) < 1e-9 * eps
    w_bond = 0.5 * p.c[0] * s ** 2 * np.linalg.norm(p.xi, axis=1) * p.volume
    W_node = np.zeros(p.n_nodes)
    np.add.at(W_node, p.bond_i, 0.5 * w_bond)
    np.add.at(W_node, p.bond_j, 0.5 * w_bond)
    lattice = sum(np.hypot(a, b) for a, b in in_plane_offsets()) / (2 * np.pi * W.M_RATIO ** 3 / 3)
    nu = MODELS[model][1]
    cont = (E / (1 - nu) if model == "stress" else E / ((1 + nu) * (1 - 2 * nu))) * eps ** 2
    assert cont == pytest.approx((1.5 if model == "stress" else 1.6) * E * eps ** 2, rel=1e-12)
    Wi = W_node[interior_2d(shape)]
    assert np.allclose(Wi, cont * lattice, rtol=1e-9, atol=0)
    assert lattice == pytest.approx(1.0, abs=0.1)
    # interior nodes carry no net force
    L = p.force(u)
    assert np.max(np.abs(L[interior_2d(shape)])) < 1e-8 * p.c[0] * eps * p.volume


@pytest.mark.parametrize("model", ["stress", "strain"])
def test_quadratic_field_navier_operator(model):
    """u_x = kappa x^2 / 2: the linearised interior force density is
    c V (kappa / 2) dx sum_v v_x^4 / |v|^3 over in-plane offsets, whose
    continuum limit is the Navier term (lambda + 2 mu) kappa: in plane stress
    E / (1 - nu^2) kappa = 9 E kappa / 8 (nu = 1/3), in plane strain
    E (1 - nu) / ((1 + nu)(1 - 2 nu)) kappa = 6 E kappa / 5 (nu = 1/4); no
    out-of-plane or vertical force."""
    shape, dx, kap = (13, 1, 13), 1e-3, 1e-4
    p = plane_problem(shape, dx, model=model)
    x = G.node_positions(shape, dx)
    u = np.zeros_like(x)
    u[:, 0] = 0.5 * kap * x[:, 0] ** 2
    L = p.force(u)
    lattice = sum(a ** 4 / np.hypot(a, b) ** 3 for a, b in in_plane_offsets())
    expect = p.c[0] * p.volume * 0.5 * kap * dx * lattice
    Li = L[interior_2d(shape)]
    assert np.allclose(Li[:, 0], expect, rtol=1e-5, atol=0)
    assert np.max(np.abs(Li[:, 1:])) < 1e-5 * expect
    nu = MODELS[model][1]
    cont = (E / (1 - nu * nu) if model == "stress" else E * (1 - nu) / ((1 + nu) * (1 - 2 * nu))) * kap
    assert cont == pytest.approx((9 / 8 if model == "stress" else 6 / 5) * E * kap, rel=1e-12)
    assert expect == pytest.approx(cont, rel=0.1)


def test_thickness_scales_only_the_reaction():
    """c V and c t do not depend on t, so displacements, damage and the peak
    step are unchanged by the thickness and the reaction scales with it."""
    lv = W.level2d(0, steps_scale=0.5)
    a = S.beam_problem(lv).run()
    lv2 = dataclasses.replace(lv, beam=dataclasses.replace(lv.beam, thickness=2 * lv.beam.thickness))
    b = S.beam_problem(lv2).run()
    assert b["nstar"] == a["nstar"]
    assert np.allclose(b["u"], a["u"], rtol=1e-12, atol=1e-20)
    assert np.allclose(b["R"], 2 * a["R"], rtol=1e-12, atol=1e-9)
    assert np.array_equal(b["kappa"] > 0, a["kappa"] > 0)


# ---------------------------------------------------------------- fracture energy
def test_2d_fracture_energy_geometry_factor():
    """Eq. exp_fracture_energy_2D with w = xi A: the geometric part
    2 int_0^delta int_z^delta int_0^{acos(z/xi)} xi^2 dphi dxi dz equals
    delta^4 / 2 (delta = 1 here)."""
    val, _ = integrate.nquad(lambda phi, xi, z: 2.0 * xi * xi,
                             [lambda xi, z: (0.0, np.arccos(min(1.0, z / xi))), lambda z: (z, 1.0), (0.0, 1.0)],
                             opts={"epsabs": 1e-12, "epsrel": 1e-12})
    assert val == pytest.approx(0.5, rel=1e-9)


def envelope_force(law, s, s0, sc, c):
    return c * (1.0 - S.damage(law, s, s0, sc, K, ALPHA)) * s


@pytest.mark.parametrize("law", [S.LAW_EXPLIN, S.LAW_TRILINEAR])
@pytest.mark.parametrize("dx", [10e-3, 2.5e-3, 0.625e-3])
def test_2d_critical_stretch_reproduces_fracture_energy(law, dx):
    delta = W.M_RATIO * dx
    c = S.micromodulus_plane_stress(E, delta, T)
    sc = S.critical_stretch_2d(law, S0, c, GF, delta, T, K, ALPHA)
    assert sc > S0
    pts = [S0 + (sc - S0) * f for f in (0.05, 0.2, 0.5)]
    area, _ = integrate.quad(lambda s: envelope_force(law, s, S0, sc, c), S0, sc,
                             points=pts, limit=400, epsabs=0, epsrel=1e-12)
    assert area * 0.5 * T * delta ** 4 == pytest.approx(GF, rel=1e-8)


def test_2d_critical_stretch_equals_printed_rearrangement():
    """Unlike the 3D one, the printed 2D rearrangement (Eq. exp_sc_2D) is the
    root of its own energy relation: it must agree with the oracle."""
    for dx in (10e-3, 1.25e-3):
        delta = W.M_RATIO * dx
        c = S.micromodulus_plane_stress(E, delta, T)
        ek = np.exp(K)
        P = 2 * K - 2 * ek + ALPHA * K - ALPHA * K * ek + 2
        h = T
        printed = (4 * K * (1 - ek) * (1 + ALPHA) * (GF - h * c * delta ** 4 * S0 ** 2 * P / (4 * K * (ek - 1) * (1 + ALPHA)))
                   / (h * c * delta ** 4 * S0 * P))
        assert S.critical_stretch_2d(S.LAW_EXPLIN, S0, c, GF, delta, T, K, ALPHA) == pytest.approx(printed, rel=1e-12)


def test_plane_beam_cracks_from_the_notch():
    """Specimen 3 at level 0: the peak comes mid-run, the reaction has
    softened well below it by the end and the most stretched bonds sit in
    the ligament just above the notch tip."""
    lv = W.level2d(0)
    p = S.beam_problem(lv)
    r = p.run()
    assert 0.2 * lv.n_steps < r["nstar"] < 0.8 * lv.n_steps
    assert r["R"][-1] < 0.6 * r["Q"]
    x = G.node_positions(lv.shape, lv.dx)
    mid = 0.5 * (x[p.bond_i] + x[p.bond_j])
    top = np.argsort(-r["kappa"])[:20]
    assert np.all(r["kappa"][top] > 10 * S0)
    assert np.all(np.abs(mid[top, 0] - 0.5 * lv.beam.length) < p.delta)
    assert np.all((mid[top, 2] >= lv.beam.notch_depth - 0.5 * lv.dx) & (mid[top, 2] < lv.beam.notch_depth + p.delta))


def test_unnotched_specimen_is_mirror_symmetric():
    """Case study 2's unnotched Specimen 3 (lambda = 0) is symmetric about
    mid-span in geometry, pads and loading, so the homogeneous solve is too:
    u_x(L - x) = -u_x(x) and u_z(L - x) = u_z(x), to rounding, through the
    first cracking steps."""
    lv = W.level2d(1, notched=False, steps_scale=0.3)
    p = S.beam_problem(lv)
    assert p.n_bonds == G.unique_bonds(lv.shape, W.M_RATIO)[0].size      # no bond is cut
    r = p.run()
    nx, ny, nz = lv.shape
    u = r["u"].reshape(nz, nx, 3)
    scale = np.max(np.abs(u))
    assert np.max(np.abs(u[:, ::-1, 0] + u[:, :, 0])) < 1e-9 * scale
    assert np.max(np.abs(u[:, ::-1, 2] - u[:, :, 2])) < 1e-9 * scale
    assert np.max(r["kappa"]) > S0                                           # damage has started
