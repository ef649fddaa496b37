"""Pins of the oracle's KL random field and MLMC statistics: the integral
eigen-equation by adaptive quadrature, orthonormality, the trace identity,
Mercer's reconstruction, the ranking of separable modes against brute force,
lognormal moments, exact sums of integer sequences and the paper's tables."""
import os

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import kl, mlmc

HERE = os.path.dirname(os.path.abspath(__file__))
LC = W.FIELD_CORR_LEN


@pytest.fixture(scope="module")
def axis():
    return kl.Basis1D(0.175, LC, 256)


def test_eigenpairs_solve_the_integral_equation(axis):
    rng = np.random.default_rng(0)
    for m in range(0, 12):
        for x in rng.uniform(0, 0.175, size=3):
            lhs, _ = integrate.quad(
                lambda y: np.exp(-(x - y) ** 2 / (2 * LC * LC)) * axis.evaluate([y], [m])[0, 0],
                0, 0.175, epsabs=0, epsrel=1e-11, limit=200)
            assert lhs == pytest.approx(axis.lam[m] * axis.evaluate([x], [m])[0, 0], rel=1e-7, abs=1e-9)


def test_orthonormal_and_signed(axis):
    for a in range(6):
        for b in range(6):
            val, _ = integrate.quad(lambda y: axis.evaluate([y], [a])[0, 0] * axis.evaluate([y], [b])[0, 0],
                                    0, 0.175, epsabs=1e-12, limit=200)
            assert val == pytest.approx(1.0 if a == b else 0.0, abs=1e-8)
    left = axis.evaluate([0.0], np.arange(20))[0]
    assert np.all(left > 0)


def test_trace_and_mercer(axis):
    # sum of all eigenvalues = int k(x, x) dx = L
    assert np.sum(axis.lam) == pytest.approx(0.175, rel=1e-10)
    # Mercer: the full expansion reproduces the kernel off the quadrature nodes
    pts = np.array([0.013, 0.05, 0.0871, 0.16])
    n = 60
    Phi = axis.evaluate(pts, np.arange(n))
    K = (Phi * axis.lam[:n]) @ Phi.T
    assert np.allclose(K, kl.kernel(pts, pts, LC), atol=1e-9)


def test_quadrature_convergence():
    a = kl.Basis1D(0.05, LC, 128)
    b = kl.Basis1D(0.05, LC, 256)
    assert np.allclose(a.lam[:15], b.lam[:15], rtol=1e-10, atol=1e-14)


def test_mode_ranking_matches_brute_force():
    basis = kl.Basis3D((0.175, 0.05, 0.05), LC, 50, n_quad=128)
    lx, ly, lz = (ax.lam for ax in basis.axes)
    allp = sorted((lx[a] * ly[b] * lz[c] for a in range(30) for b in range(30) for c in range(30)),
                  reverse=True)
    assert np.allclose(sorted(basis.lam, reverse=True), allp[:50], rtol=1e-12)
    assert np.all(np.diff(basis.lam) <= 1e-12 * basis.lam[0])
    # equal products (the two 50 mm axes) come in lexicographic index order
    for i in range(49):
        if abs(basis.lam[i] - basis.lam[i + 1]) <= 1e-9 * basis.lam[i]:
            assert basis.modes[i][:3] < basis.modes[i + 1][:3]
    # captured variance of the unit-variance field over the beam
    frac = np.sum(basis.lam) / (0.175 * 0.05 * 0.05)
    assert 0.9 < frac < 1.0


def test_lognormal_marginal_moments():
    basis = kl.Basis3D((0.175, 0.05, 0.05), LC, 50, n_quad=128)
    pts = np.array([[0.0875, 0.025, 0.0025], [0.01, 0.04, 0.03]])
    xi = W.kl_coefficients(11, 20000)
    s0 = kl.lognormal_field(basis, pts, xi, W.S0_MEAN, W.FIELD_COV)
    mu, sigma = kl.lognormal_params(W.S0_MEAN, W.FIELD_COV)
    Phi = basis.eigenfunctions(pts)
    var_g = (Phi ** 2) @ basis.lam                     # pointwise variance of g
    logs = np.log(s0)
    for p in range(2):
        sd = sigma * np.sqrt(var_g[p])
        assert abs(logs[:, p].mean() - mu) < 4.5 * sd / np.sqrt(xi.shape[0])
        assert logs[:, p].std() == pytest.approx(sd, rel=0.03)
    # with the full variance the lognormal mean and CoV would be the targets
    assert np.exp(mu + 0.5 * sigma ** 2) == pytest.approx(W.S0_MEAN, rel=1e-12)
    assert np.sqrt(np.expm1(sigma ** 2)) == pytest.approx(W.FIELD_COV, rel=1e-12)


def test_level_moments_on_integer_sequences():
    for N in (2, 5, 17, 1000):
        n, s1, s2 = mlmc.level_sums(np.arange(1, N + 1))
        mean, var, unb = mlmc.level_moments(n, s1, s2)
        assert mean == (N + 1) / 2
        assert var == pytest.approx((N * N - 1) / 12, rel=1e-15)
        assert unb == pytest.approx(N * (N + 1) / 12, rel=1e-15)


def test_telescoping_sum():
    rng = np.random.default_rng(3)
    Q = [rng.normal(1000 + 10 * l, 5, size=64) for l in range(3)]
    levels = [mlmc.differences(Q[0])] + [mlmc.differences(Q[l], Q[l - 1]) for l in (1, 2)]
    est, _, _ = mlmc.mlmc_estimate(levels)
    assert est == pytest.approx(Q[2].mean(), rel=1e-13)


def _rows(name):
    return [l.split() for l in open(os.path.join(HERE, "golden", name))
            if l.strip() and not l.startswith("#")]


def test_paper_allocation_tables_scale_as_eps_minus_two_rounded_down():
    """Eq. sample_allocation and Eq. MC_num_samples scale as eps^-2; the
    paper's tables round down.  Feed per-level variances whose eps = 10 N
    allocation lands half-way into the printed counts and check the other
    two rows."""
    rows = _rows("mlmc_tables.txt")
    for case in ("type2", "type1"):
        r = {int(x[1]): x for x in rows if x[0] == case}
        N10 = np.array([int(v) for v in r[10][2:7]], dtype=float) + 0.5
        C = np.array([4.0 ** l for l in range(5)])            # gamma = 1, M_l = 4^l M_0
        # V_l = a N10_l^2 C_l makes the eps = 10 allocation a (sum N10 C) N10 / 100
        V = (100.0 / np.sum(N10 * C)) * N10 ** 2 * C
        real10, _ = mlmc.optimal_allocation(V, C, 10.0)
        assert np.allclose(real10, N10, rtol=1e-12)
        for eps in (50, 100):
            _, n = mlmc.optimal_allocation(V, C, float(eps))
            assert list(n) == [int(v) for v in r[eps][2:7]]
        Vmc = (int(r[10][7]) + 0.5) * 100.0
        for eps in (50, 100):
            assert mlmc.mc_samples(Vmc, float(eps))[1] == int(r[eps][7])


def test_paper_cost_exponents():
    for case, a, b, g, e_ml, e_mc in _rows("mlmc_rates.txt"):
        ml, mc = mlmc.cost_exponents(float(a), float(b), float(g))
        assert round(ml, 2) == float(e_ml)
        assert round(mc, 2) == float(e_mc)


def test_paper_cost_table_consistency():
    """Every standard-MC cost in the paper's tables is the same per-sample cost
    times N (about 13.9 min per finest-level sample), and the speed-up column
    is MC / MLMC to the printed precision."""
    rows = _rows("mlmc_tables.txt")
    per = [float(x[9]) / int(x[7]) for x in rows]
    assert max(per) / min(per) < 1.003      # costs are printed in whole minutes
    for x in rows:
        ratio = float(x[9]) / float(x[8])
        assert abs(ratio - float(x[10])) <= 0.5 if float(x[10]) >= 10 else abs(ratio - float(x[10])) < 0.05
