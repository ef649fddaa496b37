"""CPU checks of the MLMC decision logic (paper section 4.3).

* libpdmi's pd_mlmc_allocation / pd_mlmc_bias / pd_mlmc_fit_rate (host entry
  points, no GPU) against the paper's printed allocation tables and against
  the oracle on random inputs;
* pins of the oracle's adaptive driver (Algorithm 1) on deterministic level
  differences, where the finest level, the sample counts and the estimate
  have closed forms."""
import os

import numpy as np
import pytest

from oracle import mlmc as OM
from paper_2212_04415_amd import mlmc as PM
from paper_2212_04415_amd import pd

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows(name):
    return [l.split() for l in open(os.path.join(HERE, "golden", name))
            if l.strip() and not l.startswith("#")]


def test_allocation_reproduces_the_paper_tables():
    """Per-level variances whose eps = 10 allocation lands half-way into the
    printed counts (gamma = 1, M_l = 4^l M_0 in 2D) give the printed eps = 50
    and eps = 100 rows, rounded down (section 6.2 / 6.3 tables)."""
    rows = _rows("mlmc_tables.txt")
    for case in ("type2", "type1"):
        r = {int(x[1]): x for x in rows if x[0] == case}
        N10 = np.array([int(v) for v in r[10][2:7]], dtype=float) + 0.5
        Cs = np.array([4.0 ** l for l in range(5)])
        V = (100.0 / np.sum(N10 * Cs)) * N10 ** 2 * Cs
        real, _ = PM.allocation(V, Cs, 10.0)
        assert np.allclose(real, N10, rtol=1e-12)
        for eps in (50, 100):
            _, n = PM.allocation(V, Cs, float(eps))
            assert list(n) == [int(v) for v in r[eps][2:7]]


def test_allocation_bias_and_rates_match_the_oracle():
    rng = np.random.default_rng(17)
    for _ in range(50):
        L = int(rng.integers(1, 6))
        V = rng.uniform(1.0, 1e5, L)
        Cs = rng.uniform(1.0, 1e4, L)
        eps = float(rng.uniform(1.0, 100.0))
        real, n = PM.allocation(V, Cs, eps)
        oreal, on = OM.optimal_allocation(V, Cs, eps)
        assert np.allclose(real, oreal, rtol=1e-13)
        # the sampling error of the real allocation is exactly eps^2
        assert np.sum(V / real) == pytest.approx(eps ** 2, rel=1e-12)
        frac = oreal - np.floor(oreal)
        assert np.all(n[(frac > 1e-9) & (frac < 1 - 1e-9)] == on[(frac > 1e-9) & (frac < 1 - 1e-9)])
        y, a, m, r = float(rng.normal(0, 100)), float(rng.uniform(0.2, 2)), 8.0, float(rng.uniform(0.7, 1))
        assert PM.bias(y, a, m, r) == pytest.approx(OM.bias_bound(y, a, m, r), rel=1e-14)
        x = np.sort(rng.uniform(1.0, 1e6, 4))
        yy = rng.uniform(0.1, 10.0, 4) * np.where(rng.random(4) < 0.5, -1, 1)
        b, i = PM.fit_rate(x, yy)
        ob, oi = OM.fit_rate(x, yy)
        assert b == pytest.approx(ob, rel=1e-10, abs=1e-12) and i == pytest.approx(oi, rel=1e-10, abs=1e-12)


def test_rate_fit_recovers_exact_power_laws():
    x = np.array([3500.0, 28000.0, 224000.0, 1792000.0])
    for rate, c in ((-0.7, 3.0), (0.528, 0.01), (-1.0, -5.0)):
        y = c * x ** rate
        assert PM.fit_rate(x, y)[0] == pytest.approx(rate, abs=1e-12)
        assert OM.fit_rate(x, y)[0] == pytest.approx(rate, abs=1e-12)
        assert np.exp(PM.fit_rate(x, y)[1]) == pytest.approx(abs(c), rel=1e-10)


def test_host_entry_points_reject_bad_input():
    import ctypes as C
    out = C.c_double()
    assert pd.lib().pd_mlmc_bias(1.0, 0.0, 8.0, 1.0, C.byref(out)) == pd.PD_EINVAL     # 8^0 - 1 = 0
    V = np.array([1.0, -1.0]); Cs = np.array([1.0, 2.0]); n = np.zeros(2, dtype=np.int64)
    assert pd.lib().pd_mlmc_allocation(V.ctypes.data, Cs.ctypes.data, 2, 1.0, None, n.ctypes.data) == pd.PD_EINVAL
    V = np.array([1.0, 1.0])
    assert pd.lib().pd_mlmc_allocation(V.ctypes.data, Cs.ctypes.data, 2, 0.0, None, n.ctypes.data) == pd.PD_EINVAL
    x = np.array([2.0, 2.0]); y = np.array([1.0, 3.0]); b = C.c_double()
    assert pd.lib().pd_mlmc_fit_rate(x.ctypes.data, y.ctypes.data, 2, C.byref(b), None) == pd.PD_EINVAL


def test_oracle_adaptive_on_deterministic_differences():
    """With Y_l = c 8^(-a l) exactly (no variance) every level keeps its
    warm-up samples, the bias estimate of level L is c 8^(-a L) / (8^a - 1),
    and the algorithm stops at the first L where it is below eps / sqrt 2."""
    c, a = 400.0, 0.6
    sampler = lambda l, start, count: np.full(count, c * 8.0 ** (-a * l))
    costs = [8.0 ** l for l in range(6)]
    dofs = [1000.0 * 8 ** l for l in range(6)]
    for eps in (200.0, 50.0, 5.0):
        out = OM.adaptive(sampler, eps, costs, dofs, n_warm=7, alpha=a)
        L = next(l for l in range(1, 6) if c * 8.0 ** (-a * l) / (8.0 ** a - 1) < eps / np.sqrt(2))
        assert out["converged"] and out["L"] == L
        assert out["N"] == [7] * (L + 1)
        assert out["estimate"] == pytest.approx(sum(c * 8.0 ** (-a * l) for l in range(L + 1)), rel=1e-14)
        assert out["sampling_variance"] == pytest.approx(0.0, abs=1e-9)
    # fitted alpha: exact for a geometric sequence once two correction levels exist
    out = OM.adaptive(sampler, 5.0, costs, dofs, n_warm=3, alpha=None, alpha_default=0.3)
    assert out["history"][0]["alpha"] == 0.3 and out["history"][1]["alpha"] == 0.3
    assert all(h["alpha"] == pytest.approx(a, rel=1e-12) for h in out["history"][2:])
    # too few levels: stops at the last one, not converged
    out = OM.adaptive(sampler, 5.0, costs, dofs, n_warm=3, alpha=a, max_levels=2)
    assert out["L"] == 1 and not out["converged"]


def test_non_decaying_corrections_leave_the_bias_unbounded():
    """Eq. bias_error bounds the bias only for r m^alpha > 1.  Corrections
    that grow with the level fit a negative rate: the bias estimate is
    infinite and the algorithm refines to the last level without converging,
    in the oracle and in the GPU driver's own rule alike."""
    assert OM.bias_bound(50.0, -0.2, 4.0) == float("inf")
    assert OM.bias_bound(50.0, 0.0, 4.0) == float("inf")
    assert OM.bias_bound(50.0, 0.5, 4.0) == pytest.approx(50.0)
    c = 100.0
    sampler = lambda l, start, count: np.full(count, c * 2.0 ** l)      # |Y_l| grows
    costs = [4.0 ** l for l in range(4)]
    dofs = [350.0 * 4 ** l for l in range(4)]
    out = OM.adaptive(sampler, 100.0, costs, dofs, n_warm=3, alpha=None, alpha_default=0.5, refinement=4.0)
    assert out["L"] == 3 and not out["converged"]
    assert out["history"][-1]["alpha"] < 0 and out["history"][-1]["bias"] == float("inf")


def test_oracle_adaptive_allocation_meets_the_sampling_budget():
    """Gaussian level differences: after each iteration every level holds at
    least its allocation, the reported sampling variance is sum V_l / N_l of
    the samples taken, and each allocation's real-valued sampling error equals
    eps_s^2 for the variances it was computed from."""
    mu = [1000.0, 120.0, 40.0, 13.0]
    sig = [300.0, 60.0, 25.0, 10.0]
    pool = [np.random.default_rng(l).normal(mu[l], sig[l], 200000) for l in range(4)]
    sampler = lambda l, start, count: pool[l][start:start + count]
    costs = [1.0, 8.0, 64.0, 512.0]
    out = OM.adaptive(sampler, 10.0, costs, [8.0 ** l for l in range(4)], n_warm=20, alpha=0.5)
    assert out["L"] >= 2
    for h in out["history"]:
        assert all(n >= nh for n, nh in zip(h["N"], h["n_hat"]))
        real, _ = OM.optimal_allocation(h["V"], costs[:h["L"] + 1], out["eps_s"])
        assert np.sum(np.array(h["V"]) / real) == pytest.approx(out["eps_s"] ** 2, rel=1e-12)
    V = [OM.level_moments(*OM.level_sums(pool[l][:out["N"][l]]))[1] for l in range(out["L"] + 1)]
    assert out["sampling_variance"] == pytest.approx(sum(v / n for v, n in zip(V, out["N"])), rel=1e-12)
    assert out["estimate"] == pytest.approx(sum(pool[l][:out["N"][l]].mean() for l in range(out["L"] + 1)), rel=1e-13)


# ------------------------------------------------------------------ multilevel CDF (oracle pins)
def test_single_level_inverse_cdf_is_the_order_statistic():
    rng = np.random.default_rng(2)
    X = rng.normal(4000, 300, 37)
    N = X.size
    u = np.arange(1, N + 1) / N
    assert np.array_equal(OM.ml_inverse_cdf([X], [None], u), np.sort(X))
    # between grid points the next order statistic is taken (ceil)
    assert np.array_equal(OM.ml_inverse_cdf([X], [None], u - 0.5 / N), np.sort(X))
    # the CDF of the quantiles on the grid is the plain empirical CDF of the samples
    xq = np.concatenate([X, X + 1e-9, X - 1e-9, [X.min() - 1, X.max() + 1]])
    F = OM.ecdf(OM.ml_inverse_cdf([X], [None], u), xq)
    assert np.array_equal(F, np.array([np.mean(X <= x) for x in xq]))


def test_perfectly_coupled_hierarchy_telescopes_to_the_finest_level():
    """When each level's coarse partners are exactly the level below's fine
    samples (same count), the corrections cancel and F^-1 is the finest
    level's empirical quantile function."""
    rng = np.random.default_rng(3)
    levels = [rng.normal(4000 + 100 * l, 300, 64) for l in range(4)]
    u = rng.uniform(1e-6, 1.0, 200)
    got = OM.ml_inverse_cdf(levels, [None] + levels[:-1], u)
    assert np.allclose(got, OM.ml_inverse_cdf([levels[-1]], [None], u), rtol=0, atol=1e-9)


def test_inverse_cdf_of_uniform_samples_converges():
    """N = 20000 uniform samples: the empirical quantile stays within the
    Dvoretzky-Kiefer-Wolfowitz band (eps = sqrt(ln(2/0.001) / 2N)) of u."""
    rng = np.random.default_rng(4)
    X = rng.uniform(0.0, 1.0, 20000)
    u = np.linspace(0.001, 1.0, 999)
    band = np.sqrt(np.log(2 / 1e-3) / (2 * X.size))
    assert np.max(np.abs(OM.ml_inverse_cdf([X], [None], u) - u)) < band + 1.0 / X.size
