"""Oracle MC / MLMC estimators (paper section 4).

TEST INFRASTRUCTURE ONLY.  Plain NumPy in FP64.

* Y_l = Q_l - Q_{l-1} for l > 0 and Y_0 = Q_0, both evaluated on the same
  random input (section 4.2, telescoping sum);
* level mean Y_hat = (1/N) sum Y (Eq. MC_estimator);
* level variance s^2 = (1/N) sum Y^2 - Y_hat^2 (Eq. sample_variance), and the
  unbiased 1/(N-1) variant;
* MLMC estimate sum_l Y_hat_l (Eq. MLMC_estimator) and its sampling variance
  sum_l V_l / N_l (Eq. MLMC_error);
* optimal allocation N_l = eps^-2 (sum sqrt(V C)) sqrt(V_l / C_l)
  (Eq. sample_allocation), standard-MC count N = V / eps^2
  (Eq. MC_num_samples), both rounded down as in the paper's tables;
* cost growth exponents 2 + max(0, (gamma - beta)/alpha) for MLMC
  (Eq. MLMC_computational_cost) and 2 + gamma/alpha for standard MC;
* bias bound |Y_hat_L| / (r m^alpha - 1) (Eq. bias_error).
"""
from __future__ import annotations

import numpy as np


def level_sums(Y):
    Y = np.asarray(Y, dtype=np.float64)
    return Y.size, float(np.sum(Y)), float(np.sum(Y * Y))


def level_moments(n, s1, s2):
    """(mean, variance with 1/N, variance with 1/(N-1))."""
    mean = s1 / n
    var = s2 / n - mean * mean
    unbiased = var * n / (n - 1) if n > 1 else float("nan")
    return mean, var, unbiased


def differences(q_fine, q_coarse=None):
    """Y on a level from the coupled fine / coarse peak loads."""
    q_fine = np.asarray(q_fine, dtype=np.float64)
    if q_coarse is None:
        return q_fine.copy()
    return q_fine - np.asarray(q_coarse, dtype=np.float64)


def mlmc_estimate(levels):
    """levels: list of Y arrays, level 0 first.  Returns (estimate,
    sampling variance, per-level (N, mean, var))."""
    est, samp, per = 0.0, 0.0, []
    for Y in levels:
        n, s1, s2 = level_sums(Y)
        m, v, _ = level_moments(n, s1, s2)
        est += m
        samp += v / n
        per.append((n, m, v))
    return est, samp, per


def optimal_allocation(V, C, eps):
    V = np.asarray(V, dtype=np.float64); C = np.asarray(C, dtype=np.float64)
    real = eps ** -2 * np.sum(np.sqrt(V * C)) * np.sqrt(V / C)
    return real, np.floor(real).astype(np.int64)


def mc_samples(V, eps):
    real = V / eps ** 2
    return real, int(np.floor(real))


def cost_exponents(alpha, beta, gamma):
    return 2.0 + max(0.0, (gamma - beta) / alpha), 2.0 + gamma / alpha


def bias_bound(y_last, alpha, refinement, r=1.0):
    return abs(y_last) / (r * refinement ** alpha - 1.0)
