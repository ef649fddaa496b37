"""Pins of the oracle's version of the paper's material model (section 5,
section 6.2): exponential-covariance KL basis by Nystrom's method, the
Weibull marginal through the Gaussian copula, the fib relations, and the
per-node fracture energy in the solver.

* the Nystrom eigenvalues of the 1D exponential kernel converge to the
  closed-form values (roots of the transcendental equations);
* Mercer: the full spectrum reproduces the kernel on the reference points;
* the Nystrom extension reproduces the basis at the reference points;
* the canonical basis of a degenerate cluster does not depend on the basis
  the eigensolver returned (random rotations inside clusters);
* the copula transform has the Weibull median and CDF;
* a uniform per-node fracture energy reproduces the scalar one exactly."""
import numpy as np
import pytest
from scipy import special

import workloads as W
from oracle import material as OMAT
from oracle import solver as S


def test_1d_exponential_kernel_eigenvalues_converge_to_closed_form():
    a, lc = 0.1, 0.02
    exact = OMAT.exp_kernel_1d_eigenvalues(lc, a, 8)
    errs = []
    for n in (500, 1000, 2000):
        h = 2 * a / n
        x = -a + (np.arange(n) + 0.5) * h
        X = np.stack([x, np.zeros(n), np.zeros(n)], axis=1)
        b = OMAT.ExpBasis(X, h, lc, 8)
        errs.append(np.max(np.abs(b.lam / exact - 1)))
    assert errs[-1] < 2e-5
    assert 14 < errs[0] / errs[-1] < 18       # second order in h (4x finer: 16x smaller)


def _grid(nx, ny, nz, dx):
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([(i.ravel() + 0.5) * dx, (j.ravel() + 0.5) * dx, (k.ravel() + 0.5) * dx], axis=1)


def test_mercer_and_extension_identities():
    X = _grid(6, 4, 3, 5e-3)
    w = (5e-3) ** 3
    b = OMAT.ExpBasis(X, w, 20e-3, X.shape[0])
    K = OMAT.exp_kernel_exact(X, X, 20e-3)
    assert np.allclose((b.phi_ref * b.lam[None, :]) @ b.phi_ref.T, K, rtol=0, atol=1e-12)
    assert np.allclose(w * b.phi_ref.T @ b.phi_ref, np.eye(X.shape[0]), atol=1e-12)
    b50 = OMAT.ExpBasis(X, w, 20e-3, 20)
    assert np.allclose(b50.evaluate(X), b50.phi_ref, rtol=0, atol=1e-9 * np.max(np.abs(b50.phi_ref)))


def test_canonical_basis_is_independent_of_the_solvers_choice():
    X = _grid(5, 5, 5, 5e-3)                  # a cube: degenerate clusters by symmetry
    A = (5e-3) ** 3 * OMAT.exp_kernel_exact(X, X, 20e-3)
    lam, vec = np.linalg.eigh(A)
    lam, vec = lam[::-1][:40], vec[:, ::-1][:, :40]
    ref = OMAT.canonical_basis(lam, vec)
    sizes, k = [], 0
    while k < 40:
        e = k + 1
        while e < 40 and abs(lam[e] - lam[k]) <= OMAT.CLUSTER_RTOL * lam[k]:
            e += 1
        sizes.append(e - k)
        k = e
    assert max(sizes) >= 3                     # the cube has triply degenerate modes
    rng = np.random.default_rng(0)
    rot = vec.copy()
    k = 0
    for sz in sizes:
        Q, _ = np.linalg.qr(rng.standard_normal((sz, sz)))
        rot[:, k:k + sz] = vec[:, k:k + sz] @ Q
        k += sz
    assert np.allclose(OMAT.canonical_basis(lam, rot), ref, atol=1e-10)
    assert np.allclose(ref.T @ ref, np.eye(40), atol=1e-12)


def test_weibull_copula_marginal():
    fcm, m = 42.3e6, 3.0
    lam_w = fcm / special.gamma(1 + 1 / m)
    assert OMAT.weibull_from_gaussian(0.0, fcm, m) == pytest.approx(lam_w * np.log(2) ** (1 / m), rel=1e-14)
    g = np.random.default_rng(1).standard_normal(200000)
    fc = OMAT.weibull_from_gaussian(g, fcm, m)
    for x in (10e6, 30e6, 45e6, 70e6):
        emp = np.mean(fc <= x)
        assert emp == pytest.approx(1 - np.exp(-(x / lam_w) ** m), abs=5 * np.sqrt(0.25 / g.size))
    assert np.mean(fc) == pytest.approx(fcm, rel=5 * np.std(fc) / np.sqrt(g.size) / fcm)


def test_fib_relations_at_the_mean_strength():
    """At the paper's mean strength (section 6.2) the relations give the
    workload's tensile strength (limit stretch x E) and a fracture energy
    within 2.5% of its 140 N/m; all three grow with f_c."""
    E, ft, GF = OMAT.fib_properties(42.3e6)
    assert ft == pytest.approx(W.F_T, rel=1e-12)
    assert GF == pytest.approx(W.FRACTURE_ENERGY, rel=0.025)
    fc = np.linspace(5e6, 90e6, 50)
    for q in OMAT.fib_properties(fc):
        assert np.all(np.diff(q) >= 0)


def test_uniform_fracture_energy_field_equals_the_scalar():
    lv = W.level(0, fracture=True)
    rng = np.random.default_rng(2)
    s0 = W.S0_MEAN * np.exp(0.2 * rng.standard_normal(int(np.prod(lv.shape))))
    a = S.beam_problem(lv, s0=s0, n_steps=1200).run(want_state=False)
    b = S.beam_problem(lv, s0=s0, n_steps=1200, gf=np.full(s0.size, W.FRACTURE_ENERGY)).run(want_state=False)
    assert a["Q"] == b["Q"] and a["nstar"] == b["nstar"]
    # a doubled fracture energy everywhere is the scalar run with 2 G_F
    c = S.beam_problem(lv, s0=s0, n_steps=1200, GF=2 * W.FRACTURE_ENERGY).run(want_state=False)
    d = S.beam_problem(lv, s0=s0, n_steps=1200, gf=np.full(s0.size, 2 * W.FRACTURE_ENERGY)).run(want_state=False)
    assert c["Q"] == d["Q"] and c["Q"] != a["Q"]
