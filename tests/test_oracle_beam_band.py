"""Small-strain elastic deflection of the three-point-bending beam: the
oracle's linearised force operator against Euler-Bernoulli bending plus
Timoshenko shear (a sanity band, not a parity bar: bond-based peridynamics
without a surface correction is softer than the continuum beam within a
horizon of every free face, and the pads indent the body locally)."""
from dataclasses import replace

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import solver as S


def bond_stiffness(p):
    """Small-displacement stiffness of the bond list, K = sum_b (c_b V^2 / |xi|)
    e e^T on the (i, i), (j, j), (i, j), (j, i) blocks (forces in N)."""
    M = p.n_nodes
    ln = np.linalg.norm(p.xi, axis=1)
    e = p.xi / ln[:, None]
    kb = 0.5 * (p.c[p.bond_i] + p.c[p.bond_j]) * p.volume ** 2 / ln
    rows, cols, vals = [], [], []
    for a in range(3):
        for b in range(3):
            kab = kb * e[:, a] * e[:, b]
            for I, J, sg in ((p.bond_i, p.bond_i, 1.0), (p.bond_j, p.bond_j, 1.0),
                             (p.bond_i, p.bond_j, -1.0), (p.bond_j, p.bond_i, -1.0)):
                rows.append(3 * I + a)
                cols.append(3 * J + b)
                vals.append(sg * kab)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(3 * M, 3 * M))


def timoshenko_stiffness(span, depth, thickness, E, nu=0.25):
    """Midspan load over deflection of a simply supported rectangular beam
    under a central point load: bending span^3 / (48 E I) plus shear
    span / (4 kappa G A), kappa = 5/6, G = E / (2 (1 + nu)); nu = 1/4 is the
    Poisson ratio of a bond-based body."""
    I = thickness * depth ** 3 / 12.0
    A = thickness * depth
    G = E / (2.0 * (1.0 + nu))
    return 1.0 / (span ** 3 / (48.0 * E * I) + span / (4.0 * (5.0 / 6.0) * G * A))


def pd_stiffness(ell):
    beam = replace(W.Beam(), notch_depth=0.0)
    p = S.beam_problem(replace(W.level(ell), beam=beam))
    M = p.n_nodes
    K = bond_stiffness(p)
    # the oracle's own force, linearised at rest, is this operator
    x = np.random.default_rng(ell).standard_normal(3 * M)
    h = 1e-12
    Lx = -p.force((h * x).reshape(M, 3)).ravel() / h * p.volume
    assert np.abs(K @ x - Lx).max() < 1e-5 * np.abs(Lx).max()
    # supports u_z = 0, load pad u_z = -U; rigid motions in x and y pinned
    fixed = np.zeros(3 * M, dtype=bool)
    fixed[3 * p.support + 2] = True
    fixed[3 * p.load + 2] = True
    fixed[3 * p.support[0]] = fixed[3 * p.support[0] + 1] = fixed[3 * p.support[-1] + 1] = True
    free = ~fixed
    U = 1e-6
    ubc = np.zeros(3 * M)
    ubc[3 * p.load + 2] = -U
    Kff = K[free][:, free].tocsr()
    rhs = -(K[free][:, fixed] @ ubc[fixed])
    y, info = spla.cg(Kff, rhs, rtol=1e-8, maxiter=20000)
    assert info == 0
    u = ubc.copy()
    u[free] = y
    # upward support reaction (K u is the external force that holds u) per
    # unit load-pad displacement
    R = (K @ u)[3 * p.support + 2].sum()
    assert R > 0
    return R / U, beam, 3.14 * p.dx


@pytest.mark.slow
def test_beam_stiffness_inside_the_surface_layer_band_and_converging():
    """Upper bound: the continuum beam (every node with its full horizon).
    Lower bound: the same beam with a layer delta/2 thick taken off every face
    (a node on a free face keeps at least half of its horizon, so the layer
    within delta of a face is at least half as stiff).  Both bounds are the
    Timoshenko beam of the respective cross-section.  Refinement thins the
    soft layer, so the stiffness ratio must grow toward 1."""
    ratios = []
    for ell in (0, 1):
        k_pd, beam, delta = pd_stiffness(ell)
        k_full = timoshenko_stiffness(beam.span, beam.depth, beam.thickness, W.E_MODULUS)
        k_layer = timoshenko_stiffness(beam.span, beam.depth - delta, beam.thickness - delta, W.E_MODULUS)
        assert k_layer < k_pd < k_full, (ell, k_pd, k_layer, k_full)
        ratios.append(k_pd / k_full)
    assert ratios[1] > ratios[0] + 0.1
